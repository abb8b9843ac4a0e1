/* Host-side use of the C ABI from C (no GPU calls): load a network from BIF
 * text, look up names, compile a host-only junction tree and print its
 * statistics; every failing call reports its status string. */
#include <stdio.h>
#include <string.h>

#include "fbn.h"

static int check(fbn_status s, const char* what) {
    if (s != FBN_OK) {
        fprintf(stderr, "%s: %s (%s)\n", what, fbn_status_str(s), fbn_last_error());
        return 1;
    }
    return 0;
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    fbn_net* net = NULL;
    if (check(fbn_load_net(argv[1], &net), "fbn_load_net")) return 1;
    int32_t n = 0, v = -1, s = -1;
    if (check(fbn_net_n_vars(net, &n), "fbn_net_n_vars")) return 1;
    if (check(fbn_net_find_var(net, "late", &v), "fbn_net_find_var")) return 1;
    if (check(fbn_net_find_state(net, v, "yes", &s), "fbn_net_find_state")) return 1;
    char name[64];
    if (check(fbn_net_var_name(net, 0, name, sizeof name), "fbn_net_var_name")) return 1;
    int32_t card = 0, npar = 0, par[8];
    double cpt[64];
    size_t len = 0;
    if (check(fbn_net_cpt(net, v, &card, par, 8, &npar, cpt, 64, &len), "fbn_net_cpt")) return 1;
    fbn_jt_options opt;
    fbn_default_options(&opt);
    opt.host_only = 1;
    opt.precision = FBN_FP32_RESCALED;
    fbn_jt* jt = NULL;
    if (check(fbn_build_jt(net, &opt, &jt), "fbn_build_jt")) return 1;
    fbn_jt_stats_t st;
    if (check(fbn_jt_stats(jt, &st), "fbn_jt_stats")) return 1;
    /* a device call on a host-only tree is refused, not attempted */
    const int32_t zero = 0;
    const fbn_status refused = fbn_calibrate(jt, 1, &zero, NULL, NULL);
    /* the per-slot knobs: accepted values build, others are refused */
    fbn_jt* jt2 = NULL;
    opt.slots_per_block = 4;
    opt.fin_block = 1024;
    const fbn_status knobs_ok = fbn_build_jt(net, &opt, &jt2);
    fbn_free_jt(jt2);
    jt2 = NULL;
    opt.slots_per_block = 3;
    const fbn_status knobs_bad = fbn_build_jt(net, &opt, &jt2);
    printf("vars %d first %s late %d yes %d card %d parents %d cpt %zu cliques %d edges %d T %llu refused %d "
           "knobs_ok %d knobs_bad %d null %d\n",
           n, name, v, s, card, npar, len, st.n_cliques, st.n_edges, (unsigned long long)st.T, refused, knobs_ok,
           knobs_bad, jt2 == NULL);
    fbn_free_jt(jt);
    fbn_free_net(net);
    fbn_free_jt(NULL);
    fbn_free_net(NULL);
    return 0;
}
