"""The C ABI used from C: tests/c/abi_host.c, compiled with gcc as C99
against include/fbn.h and linked to the built library, loads the hand-written
BIF network, looks names up, compiles a host-only tree, checks that a
device call on it is refused and that the per-slot option fields reach the
library as C lays out the struct (CPU only: no device call is made)."""
import os
import shutil
import subprocess

import pytest

from paper_2212_04241_amd import fbn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_header_compiles_as_c_and_the_host_calls_work(tmp_path):
    lib = fbn.LIB_PATH
    assert os.path.exists(lib)
    exe = str(tmp_path / "abi_host")
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "c", "abi_host.c"), "-o", exe, lib,
                           "-Wl,-rpath," + os.path.dirname(lib)])
    env = dict(os.environ, HIP_VISIBLE_DEVICES="")
    out = subprocess.run([exe, os.path.join(ROOT, "tests", "golden", "bif", "commute.bif")], capture_output=True,
                         text=True, timeout=120, env=env)
    assert out.returncode == 0, out.stderr
    words = out.stdout.split()
    kv = dict(zip(words[0::2], words[1::2]))
    assert kv["vars"] == "6" and kv["first"] == "weather" and kv["late"] == "5" and kv["yes"] == "1"
    assert kv["card"] == "2" and kv["parents"] == "2" and kv["cpt"] == "12"
    assert int(kv["cliques"]) >= 3 and int(kv["T"]) > 0
    assert int(kv["refused"]) == fbn.FBN_E_STATE
    # the options struct as C sees it: the per-slot knobs reach the library
    assert int(kv["knobs_ok"]) == fbn.FBN_OK
    assert int(kv["knobs_bad"]) == fbn.FBN_E_INVALID_ARG and kv["null"] == "1"
