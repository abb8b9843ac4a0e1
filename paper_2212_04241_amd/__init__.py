"""MI355X junction-tree exact inference on discrete Bayesian networks.

The potential-table work of junction-tree message passing (reduction,
marginalisation, extension; Jiang et al., PPoPP'23 poster, Section 2) runs in
hand-written HIP kernels for gfx950 behind the C ABI in include/fbn.h.  This
package is the thin Python binding (``fbn``) and the build helper.
"""
from . import fbn  # noqa: F401

__all__ = ["fbn"]
