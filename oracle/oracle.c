/*
 * FP64 junction-tree oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Written for a reader to check against the textbook by eye: adjacency
 * matrices, full recomputation of the min-fill key at every step, one
 * digit decomposition per table entry, Neumaier sums in ascending order.
 * Nothing here is blocked, fused or reordered for speed.
 */
#include "oracle.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* network                                                            */
/* ------------------------------------------------------------------ */

struct orc_net {
    int n;
    int* card;
    int* npar;
    int** par;
    double** cpt;      /* NULL entries: structure only */
    int64_t* cpt_len;
};

static void set_err(char* err, size_t errlen, const char* fmt, ...) {
    if (!err || errlen == 0) return;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(err, errlen, fmt, ap);
    va_end(ap);
}

void orc_net_free(orc_net* net) {
    if (!net) return;
    for (int v = 0; v < net->n; v++) {
        if (net->par) free(net->par[v]);
        if (net->cpt) free(net->cpt[v]);
    }
    free(net->card); free(net->npar); free(net->par); free(net->cpt); free(net->cpt_len);
    free(net);
}

static orc_net* net_alloc(int n) {
    orc_net* net = calloc(1, sizeof(orc_net));
    if (!net) return NULL;
    net->n = n;
    net->card = calloc((size_t)n, sizeof(int));
    net->npar = calloc((size_t)n, sizeof(int));
    net->par = calloc((size_t)n, sizeof(int*));
    net->cpt = calloc((size_t)n, sizeof(double*));
    net->cpt_len = calloc((size_t)n, sizeof(int64_t));
    if (!net->card || !net->npar || !net->par || !net->cpt || !net->cpt_len) { orc_net_free(net); return NULL; }
    return net;
}

/* Depth-first search for a directed cycle along parent arcs. */
static int has_cycle_from(const orc_net* net, int v, char* state) {
    state[v] = 1;
    for (int k = 0; k < net->npar[v]; k++) {
        int p = net->par[v][k];
        if (state[p] == 1) return 1;
        if (state[p] == 0 && has_cycle_from(net, p, state)) return 1;
    }
    state[v] = 2;
    return 0;
}

static int validate(orc_net* net, char* err, size_t errlen) {
    int n = net->n;
    for (int v = 0; v < n; v++) {
        if (net->card[v] < 2) { set_err(err, errlen, "variable %d: cardinality %d < 2", v, net->card[v]); return ORC_E_INVALID; }
        int64_t len = net->card[v];
        for (int k = 0; k < net->npar[v]; k++) {
            int p = net->par[v][k];
            if (p < 0 || p >= n || p == v) { set_err(err, errlen, "variable %d: bad parent %d", v, p); return ORC_E_INVALID; }
            for (int k2 = 0; k2 < k; k2++)
                if (net->par[v][k2] == p) { set_err(err, errlen, "variable %d: repeated parent %d", v, p); return ORC_E_INVALID; }
            len *= net->card[p];
        }
        net->cpt_len[v] = len;
    }
    char* state = calloc((size_t)n, 1);
    for (int v = 0; v < n; v++)
        if (state[v] == 0 && has_cycle_from(net, v, state)) { free(state); set_err(err, errlen, "directed cycle"); return ORC_E_INVALID; }
    free(state);
    for (int v = 0; v < n; v++) {
        if (!net->cpt[v]) continue;
        int r = net->card[v];
        for (int64_t row = 0; row < net->cpt_len[v] / r; row++) {
            double s = 0.0;
            for (int x = 0; x < r; x++) {
                double p = net->cpt[v][row * r + x];
                if (!(p >= 0.0) || !isfinite(p)) { set_err(err, errlen, "variable %d: CPT entry not finite/non-negative", v); return ORC_E_INVALID; }
                s += p;
            }
            if (fabs(s - 1.0) > 1e-9) { set_err(err, errlen, "variable %d: CPT row %lld sums to %.17g", v, (long long)row, s); return ORC_E_INVALID; }
        }
    }
    return ORC_OK;
}

int orc_net_from_arrays(int n, const int32_t* card, const int32_t* npar, const int32_t* parents,
                        const double* cpt, orc_net** out, char* err, size_t errlen) {
    *out = NULL;
    if (n <= 0 || !card || !npar) { set_err(err, errlen, "bad arguments"); return ORC_E_INVALID; }
    orc_net* net = net_alloc(n);
    if (!net) return ORC_E_NOMEM;
    int64_t po = 0, co = 0;
    for (int v = 0; v < n; v++) {
        net->card[v] = card[v];
        net->npar[v] = npar[v];
        if (npar[v] < 0) { orc_net_free(net); set_err(err, errlen, "negative parent count"); return ORC_E_INVALID; }
        net->par[v] = malloc(sizeof(int) * (size_t)(npar[v] > 0 ? npar[v] : 1));
        for (int k = 0; k < npar[v]; k++) net->par[v][k] = parents[po + k];
        po += npar[v];
    }
    /* lengths needed before copying CPT values */
    for (int v = 0; v < n; v++) {
        int64_t len = card[v];
        for (int k = 0; k < npar[v]; k++) {
            int p = net->par[v][k];
            if (p < 0 || p >= n) { orc_net_free(net); set_err(err, errlen, "bad parent"); return ORC_E_INVALID; }
            len *= card[p];
        }
        if (cpt) {
            net->cpt[v] = malloc(sizeof(double) * (size_t)len);
            if (!net->cpt[v]) { orc_net_free(net); return ORC_E_NOMEM; }
            memcpy(net->cpt[v], cpt + co, sizeof(double) * (size_t)len);
        }
        co += len;
    }
    int rc = validate(net, err, errlen);
    if (rc) { orc_net_free(net); return rc; }
    *out = net;
    return ORC_OK;
}

/* Tokeniser for the .fbn text form. */
typedef struct { const char* p; const char* end; } toks_t;

static int next_tok(toks_t* t, char* buf, size_t cap) {
    while (t->p < t->end && (*t->p == ' ' || *t->p == '\n' || *t->p == '\t' || *t->p == '\r')) t->p++;
    if (t->p >= t->end) return 0;
    size_t k = 0;
    while (t->p < t->end && !(*t->p == ' ' || *t->p == '\n' || *t->p == '\t' || *t->p == '\r')) {
        if (k + 1 < cap) buf[k++] = *t->p;
        t->p++;
    }
    buf[k] = 0;
    return 1;
}

static int tok_long(toks_t* t, long long* out) {
    char buf[64];
    if (!next_tok(t, buf, sizeof buf)) return 0;
    char* e;
    *out = strtoll(buf, &e, 10);
    return *e == 0;
}

int orc_net_from_text(const char* text, size_t len, orc_net** out, char* err, size_t errlen) {
    *out = NULL;
    toks_t t = { text, text + len };
    char buf[128];
    long long n, x;
    if (!next_tok(&t, buf, sizeof buf) || strcmp(buf, "fbn") || !tok_long(&t, &x) || x != 1) {
        set_err(err, errlen, "missing 'fbn 1' header"); return ORC_E_PARSE;
    }
    if (!next_tok(&t, buf, sizeof buf) || strcmp(buf, "vars") || !tok_long(&t, &n) || n <= 0 || n > 1000000) {
        set_err(err, errlen, "missing 'vars n'"); return ORC_E_PARSE;
    }
    orc_net* net = net_alloc((int)n);
    if (!net) return ORC_E_NOMEM;
    char* seen_var = calloc((size_t)n, 1);
    for (;;) {
        if (!next_tok(&t, buf, sizeof buf)) { set_err(err, errlen, "missing 'end'"); goto fail; }
        if (!strcmp(buf, "end")) break;
        if (!strcmp(buf, "var")) {
            long long v, r, k;
            if (!tok_long(&t, &v) || !tok_long(&t, &r) || !tok_long(&t, &k) || v < 0 || v >= n || k < 0 || k > n || seen_var[v]) {
                set_err(err, errlen, "bad 'var' line"); goto fail;
            }
            seen_var[v] = 1;
            net->card[v] = (int)r;
            net->npar[v] = (int)k;
            net->par[v] = malloc(sizeof(int) * (size_t)(k > 0 ? k : 1));
            for (long long i = 0; i < k; i++) {
                long long p;
                if (!tok_long(&t, &p)) { set_err(err, errlen, "bad parent list"); goto fail; }
                net->par[v][i] = (int)p;
            }
        } else if (!strcmp(buf, "cpt")) {
            long long v, m;
            if (!tok_long(&t, &v) || !tok_long(&t, &m) || v < 0 || v >= n || m <= 0 || net->cpt[v]) {
                set_err(err, errlen, "bad 'cpt' line"); goto fail;
            }
            net->cpt[v] = malloc(sizeof(double) * (size_t)m);
            net->cpt_len[v] = m;
            for (long long i = 0; i < m; i++) {
                char vb[64];
                if (!next_tok(&t, vb, sizeof vb)) { set_err(err, errlen, "truncated CPT"); goto fail; }
                char* e;
                net->cpt[v][i] = strtod(vb, &e);
                if (*e) { set_err(err, errlen, "bad number '%s'", vb); goto fail; }
            }
        } else {
            set_err(err, errlen, "unknown token '%s'", buf); goto fail;
        }
    }
    for (int v = 0; v < n; v++) {
        if (!seen_var[v]) { set_err(err, errlen, "variable %d not declared", v); goto fail; }
    }
    {
        /* check CPT lengths against declared cardinalities */
        for (int v = 0; v < n; v++) {
            int64_t want = net->card[v];
            for (int k = 0; k < net->npar[v]; k++) {
                int p = net->par[v][k];
                if (p < 0 || p >= n) { set_err(err, errlen, "bad parent"); goto fail; }
                want *= net->card[p];
            }
            if (!net->cpt[v] || net->cpt_len[v] != want) { set_err(err, errlen, "variable %d: CPT length", v); goto fail; }
        }
        int rc = validate(net, err, errlen);
        if (rc) { free(seen_var); orc_net_free(net); return rc; }
    }
    free(seen_var);
    *out = net;
    return ORC_OK;
fail:
    free(seen_var);
    orc_net_free(net);
    return ORC_E_PARSE;
}

/* ------------------------------------------------------------------ */
/* junction tree                                                      */
/* ------------------------------------------------------------------ */

struct orc_jt {
    int n;                 /* variables */
    int* card;
    int* elim_order;
    int nc;                /* cliques */
    int* cn;               /* variables per clique */
    int** cvars;           /* layout order */
    int64_t* csize;        /* table entries */
    int64_t** cstride;     /* stride of cvars[c][k] in clique c's layout */
    int root;
    int* parent;           /* parent clique, -1 at root */
    int* pedge;            /* edge id towards the parent, -1 at root */
    int* height;
    int* depth;
    int* nchild;
    int** child;           /* child cliques ascending */
    int ne;
    int* e_par;
    int* e_chi;
    int* e_n;
    int** e_sep;           /* separator variables ascending */
    int64_t* e_size;
    int64_t** map;         /* map[e][j] for j < csize[e_par[e]] */
    int* cpt_home;
    int* var_home;
    double** prior;        /* per clique, layout order */
};

void orc_jt_free(orc_jt* jt) {
    if (!jt) return;
    for (int c = 0; c < jt->nc; c++) {
        free(jt->cvars[c]); free(jt->cstride[c]); free(jt->child[c]); free(jt->prior[c]);
    }
    for (int e = 0; e < jt->ne; e++) { free(jt->e_sep[e]); free(jt->map[e]); }
    free(jt->card); free(jt->elim_order); free(jt->cn); free(jt->cvars); free(jt->csize); free(jt->cstride);
    free(jt->parent); free(jt->pedge); free(jt->height); free(jt->depth); free(jt->nchild); free(jt->child);
    free(jt->e_par); free(jt->e_chi); free(jt->e_n); free(jt->e_sep); free(jt->e_size); free(jt->map);
    free(jt->cpt_home); free(jt->var_home); free(jt->prior);
    free(jt);
}

static uint64_t sat_mul(uint64_t a, uint64_t b) {
    if (a != 0 && b > UINT64_MAX / a) return UINT64_MAX;
    return a * b;
}

static int int_cmp(const void* a, const void* b) {
    int x = *(const int*)a, y = *(const int*)b;
    return (x > y) - (x < y);
}

/* Is sorted list a (na) a subset of sorted list b (nb)? */
static int is_subset(const int* a, int na, const int* b, int nb) {
    int j = 0;
    for (int i = 0; i < na; i++) {
        while (j < nb && b[j] < a[i]) j++;
        if (j == nb || b[j] != a[i]) return 0;
        j++;
    }
    return 1;
}

static int contains(const int* a, int na, int x) {
    for (int i = 0; i < na; i++) if (a[i] == x) return 1;
    return 0;
}

typedef struct { int i, j, w; uint64_t prod; } pair_t;

static int pair_cmp(const void* pa, const void* pb) {
    const pair_t* a = pa; const pair_t* b = pb;
    /* ascending (-|sep|, product of sep cards, i, j) */
    if (a->w != b->w) return (a->w > b->w) ? -1 : 1;
    if (a->prod != b->prod) return (a->prod < b->prod) ? -1 : 1;
    if (a->i != b->i) return (a->i < b->i) ? -1 : 1;
    return (a->j < b->j) ? -1 : (a->j > b->j);
}

static int uf_find(int* uf, int x) {
    while (uf[x] != x) x = uf[x];
    return x;
}

/* Moral graph as an n x n 0/1 matrix: every arc made undirected and every
 * pair of parents of a common child joined. */
static unsigned char* moral_graph(const orc_net* net) {
    int n = net->n;
    unsigned char* adj = calloc((size_t)n * (size_t)n, 1);
    for (int v = 0; v < n; v++) {
        for (int k = 0; k < net->npar[v]; k++) {
            int p = net->par[v][k];
            adj[(size_t)v * n + p] = adj[(size_t)p * n + v] = 1;
            for (int k2 = 0; k2 < net->npar[v]; k2++) {
                int q = net->par[v][k2];
                if (q != p) adj[(size_t)p * n + q] = 1;
            }
        }
    }
    return adj;
}

/* Min-fill elimination on adj (modified in place).  At every step the
 * remaining vertex with the smallest (fill-in edge count, product of the
 * cardinalities of it and its neighbours, id) is eliminated: its clique
 * {v} u N(v) is recorded (ascending) and N(v) is completed.
 * Returns 1, and the offending clique in fail_cl/fail_n, when the selected
 * vertex's clique has more than max_entries entries (0 = no limit). */
static int minfill(const orc_net* net, unsigned char* adj, uint64_t max_entries, int* order,
                   int** elim_cl, int* elim_n, int32_t* fail_cl, int fail_cap, int* fail_n) {
    int n = net->n;
    char* gone = calloc((size_t)n, 1);
    int* nb = malloc(sizeof(int) * (size_t)n);
    int rc = 0;
    for (int step = 0; step < n; step++) {
        int best = -1;
        long long best_fill = 0;
        uint64_t best_w = 0;
        for (int v = 0; v < n; v++) {
            if (gone[v]) continue;
            int k = 0;
            for (int u = 0; u < n; u++) if (!gone[u] && u != v && adj[(size_t)v * n + u]) nb[k++] = u;
            long long fill = 0;
            for (int a = 0; a < k; a++)
                for (int b = a + 1; b < k; b++)
                    if (!adj[(size_t)nb[a] * n + nb[b]]) fill++;
            uint64_t w = (uint64_t)net->card[v];
            for (int a = 0; a < k; a++) w = sat_mul(w, (uint64_t)net->card[nb[a]]);
            if (best < 0 || fill < best_fill || (fill == best_fill && w < best_w)) {
                best = v; best_fill = fill; best_w = w;
            }
        }
        int v = best;
        int k = 0;
        for (int u = 0; u < n; u++) if (!gone[u] && u != v && adj[(size_t)v * n + u]) nb[k++] = u;
        if (max_entries && best_w > max_entries) {
            if (fail_cl && fail_n) {
                int m = 0;
                if (m < fail_cap) fail_cl[m++] = v;
                for (int a = 0; a < k && m < fail_cap; a++) fail_cl[m++] = nb[a];
                *fail_n = m;
            }
            rc = 1;
            break;
        }
        if (elim_cl) {
            elim_cl[step] = malloc(sizeof(int) * (size_t)(k + 1));
            elim_cl[step][0] = v;
            for (int a = 0; a < k; a++) elim_cl[step][a + 1] = nb[a];
            elim_n[step] = k + 1;
            qsort(elim_cl[step], (size_t)(k + 1), sizeof(int), int_cmp);
        }
        for (int a = 0; a < k; a++)
            for (int b = a + 1; b < k; b++) adj[(size_t)nb[a] * n + nb[b]] = adj[(size_t)nb[b] * n + nb[a]] = 1;
        gone[v] = 1;
        if (order) order[step] = v;
    }
    free(nb); free(gone);
    return rc;
}

int orc_probe_cap(const orc_net* net, uint64_t max_entries, int32_t* clique, int cap) {
    unsigned char* adj = moral_graph(net);
    int m = 0;
    int rc = minfill(net, adj, max_entries, NULL, NULL, NULL, clique, cap, &m);
    free(adj);
    return rc ? m : 0;
}

int orc_compile(const orc_net* net, uint64_t max_entries, orc_jt** out) {
    *out = NULL;
    int n = net->n;
    orc_jt* jt = calloc(1, sizeof(orc_jt));
    jt->n = n;
    jt->card = malloc(sizeof(int) * (size_t)n);
    memcpy(jt->card, net->card, sizeof(int) * (size_t)n);

    /* 1. moral graph: arcs made undirected, co-parents married */
    unsigned char* adj = moral_graph(net);

    /* 2. min-fill elimination, key (fill, weight, id) ascending */
    int* elim_n = calloc((size_t)n, sizeof(int));
    int** elim_cl = calloc((size_t)n, sizeof(int*));
    jt->elim_order = malloc(sizeof(int) * (size_t)n);
    if (minfill(net, adj, max_entries, jt->elim_order, elim_cl, elim_n, NULL, 0, NULL)) {
        for (int s = 0; s < n; s++) free(elim_cl[s]);
        free(elim_cl); free(elim_n); free(adj);
        orc_jt_free(jt);
        return ORC_E_TOO_LARGE;
    }
    free(adj);

    /* 3. maximal cliques in elimination order */
    char* keep = calloc((size_t)n, 1);
    int nc = 0;
    for (int s = 0; s < n; s++) {
        keep[s] = 1;
        for (int t = 0; t < n && keep[s]; t++)
            if (t != s && elim_n[s] <= elim_n[t] && is_subset(elim_cl[s], elim_n[s], elim_cl[t], elim_n[t])) keep[s] = 0;
        if (keep[s]) nc++;
    }
    jt->nc = nc;
    jt->cn = malloc(sizeof(int) * (size_t)nc);
    jt->cvars = calloc((size_t)nc, sizeof(int*));      /* ascending here; layout below */
    jt->csize = malloc(sizeof(int64_t) * (size_t)nc);
    jt->cstride = calloc((size_t)nc, sizeof(int64_t*));
    jt->child = calloc((size_t)nc, sizeof(int*));
    jt->prior = calloc((size_t)nc, sizeof(double*));
    {
        int c = 0;
        for (int s = 0; s < n; s++) {
            if (keep[s]) {
                jt->cn[c] = elim_n[s];
                jt->cvars[c] = malloc(sizeof(int) * (size_t)elim_n[s]);
                memcpy(jt->cvars[c], elim_cl[s], sizeof(int) * (size_t)elim_n[s]);
                c++;
            }
            free(elim_cl[s]);
        }
    }
    free(elim_cl); free(elim_n); free(keep);
    for (int c = 0; c < nc; c++) {
        uint64_t sz = 1;
        for (int k = 0; k < jt->cn[c]; k++) sz = sat_mul(sz, (uint64_t)net->card[jt->cvars[c][k]]);
        if ((max_entries && sz > max_entries) || sz > ((uint64_t)1 << 40)) { orc_jt_free(jt); return ORC_E_TOO_LARGE; }
        jt->csize[c] = (int64_t)sz;
    }

    /* 4. Kruskal over all clique pairs (empty separators join components) */
    int ne = nc - 1;
    jt->ne = ne;
    int* tree_i = malloc(sizeof(int) * (size_t)(ne > 0 ? ne : 1));
    int* tree_j = malloc(sizeof(int) * (size_t)(ne > 0 ? ne : 1));
    {
        size_t np = (size_t)nc * (size_t)(nc - 1) / 2;
        pair_t* pairs = malloc(sizeof(pair_t) * (np > 0 ? np : 1));
        size_t q = 0;
        for (int i = 0; i < nc; i++)
            for (int j = i + 1; j < nc; j++) {
                int w = 0;
                uint64_t prod = 1;
                for (int a = 0; a < jt->cn[i]; a++)
                    if (contains(jt->cvars[j], jt->cn[j], jt->cvars[i][a])) {
                        w++;
                        prod = sat_mul(prod, (uint64_t)net->card[jt->cvars[i][a]]);
                    }
                pairs[q].i = i; pairs[q].j = j; pairs[q].w = w; pairs[q].prod = prod;
                q++;
            }
        qsort(pairs, np, sizeof(pair_t), pair_cmp);
        int* uf = malloc(sizeof(int) * (size_t)nc);
        for (int c = 0; c < nc; c++) uf[c] = c;
        int got = 0;
        for (size_t p = 0; p < np && got < ne; p++) {
            int a = uf_find(uf, pairs[p].i), b = uf_find(uf, pairs[p].j);
            if (a == b) continue;
            uf[a] = b;
            tree_i[got] = pairs[p].i; tree_j[got] = pairs[p].j; got++;
        }
        free(uf); free(pairs);
    }

    /* 5. root = minimum eccentricity (ties: lowest id); depth, parent, height */
    int* deg = calloc((size_t)nc, sizeof(int));
    for (int t = 0; t < ne; t++) { deg[tree_i[t]]++; deg[tree_j[t]]++; }
    int** nbr = malloc(sizeof(int*) * (size_t)nc);
    for (int c = 0; c < nc; c++) { nbr[c] = malloc(sizeof(int) * (size_t)(deg[c] + 1)); deg[c] = 0; }
    for (int t = 0; t < ne; t++) {
        nbr[tree_i[t]][deg[tree_i[t]]++] = tree_j[t];
        nbr[tree_j[t]][deg[tree_j[t]]++] = tree_i[t];
    }
    int* dist = malloc(sizeof(int) * (size_t)nc);
    int* queue = malloc(sizeof(int) * (size_t)nc);
    int best_root = 0, best_ecc = -1;
    for (int s = 0; s < nc; s++) {
        for (int c = 0; c < nc; c++) dist[c] = -1;
        int h = 0, tl = 0, ecc = 0;
        dist[s] = 0; queue[tl++] = s;
        while (h < tl) {
            int c = queue[h++];
            if (dist[c] > ecc) ecc = dist[c];
            for (int a = 0; a < deg[c]; a++) {
                int d = nbr[c][a];
                if (dist[d] < 0) { dist[d] = dist[c] + 1; queue[tl++] = d; }
            }
        }
        if (best_ecc < 0 || ecc < best_ecc) { best_ecc = ecc; best_root = s; }
    }
    jt->root = best_root;
    jt->parent = malloc(sizeof(int) * (size_t)nc);
    jt->depth = malloc(sizeof(int) * (size_t)nc);
    jt->height = calloc((size_t)nc, sizeof(int));
    jt->nchild = calloc((size_t)nc, sizeof(int));
    for (int c = 0; c < nc; c++) { jt->depth[c] = -1; jt->parent[c] = -1; }
    {
        int h = 0, tl = 0;
        jt->depth[best_root] = 0; queue[tl++] = best_root;
        while (h < tl) {
            int c = queue[h++];
            for (int a = 0; a < deg[c]; a++) {
                int d = nbr[c][a];
                if (jt->depth[d] < 0) { jt->depth[d] = jt->depth[c] + 1; jt->parent[d] = c; queue[tl++] = d; }
            }
        }
        /* heights: visit in reverse BFS order so children precede parents */
        for (int q = tl - 1; q >= 0; q--) {
            int c = queue[q];
            if (jt->parent[c] >= 0 && jt->height[jt->parent[c]] < jt->height[c] + 1)
                jt->height[jt->parent[c]] = jt->height[c] + 1;
        }
    }
    for (int c = 0; c < nc; c++) if (jt->parent[c] >= 0) jt->nchild[jt->parent[c]]++;
    for (int c = 0; c < nc; c++) { jt->child[c] = malloc(sizeof(int) * (size_t)(jt->nchild[c] + 1)); jt->nchild[c] = 0; }
    for (int c = 0; c < nc; c++) if (jt->parent[c] >= 0) { int p = jt->parent[c]; jt->child[p][jt->nchild[p]++] = c; }
    /* children were appended in ascending id order already */
    for (int c = 0; c < nc; c++) free(nbr[c]);
    free(nbr); free(deg); free(dist); free(queue); free(tree_i); free(tree_j);

    /* 6. edges numbered by ascending child id; separator membership (the
     * order of a separator's variables is fixed with the layouts below) */
    jt->pedge = malloc(sizeof(int) * (size_t)nc);
    jt->e_par = malloc(sizeof(int) * (size_t)(ne > 0 ? ne : 1));
    jt->e_chi = malloc(sizeof(int) * (size_t)(ne > 0 ? ne : 1));
    jt->e_n = malloc(sizeof(int) * (size_t)(ne > 0 ? ne : 1));
    jt->e_sep = calloc((size_t)(ne > 0 ? ne : 1), sizeof(int*));
    jt->e_size = malloc(sizeof(int64_t) * (size_t)(ne > 0 ? ne : 1));
    jt->map = calloc((size_t)(ne > 0 ? ne : 1), sizeof(int64_t*));
    {
        int e = 0;
        for (int c = 0; c < nc; c++) {
            jt->pedge[c] = -1;
            if (c == jt->root) continue;
            int p = jt->parent[c];
            jt->pedge[c] = e;
            jt->e_par[e] = p; jt->e_chi[e] = c;
            jt->e_sep[e] = malloc(sizeof(int) * (size_t)jt->cn[c]);
            int k = 0;
            int64_t sz = 1;
            for (int a = 0; a < jt->cn[c]; a++)       /* cvars still ascending */
                if (contains(jt->cvars[p], jt->cn[p], jt->cvars[c][a])) {
                    jt->e_sep[e][k++] = jt->cvars[c][a];
                    sz *= net->card[jt->cvars[c][a]];
                }
            jt->e_n[e] = k; jt->e_size[e] = sz;
            e++;
        }
    }

    /* 7. layouts, from the root down: the root ascending; a separator's
     * variables in the order they take in its parent's layout; a non-root
     * clique [its parent separator, in that order] ++ [the rest ascending] */
    int maxd = 0;
    for (int c = 0; c < nc; c++) if (jt->depth[c] > maxd) maxd = jt->depth[c];
    for (int d = 0; d <= maxd; d++)
        for (int c = 0; c < nc; c++) {
            if (jt->depth[c] != d) continue;
            int m = jt->cn[c];
            int* lay = malloc(sizeof(int) * (size_t)m);
            int k = 0;
            if (c != jt->root) {
                int e = jt->pedge[c], p = jt->parent[c];
                int* ordered = malloc(sizeof(int) * (size_t)(jt->e_n[e] + 1));
                int q = 0;
                for (int b = 0; b < jt->cn[p]; b++)      /* parent layout is final */
                    if (contains(jt->e_sep[e], jt->e_n[e], jt->cvars[p][b])) ordered[q++] = jt->cvars[p][b];
                free(jt->e_sep[e]);
                jt->e_sep[e] = ordered;
                for (int a = 0; a < jt->e_n[e]; a++) lay[k++] = jt->e_sep[e][a];
                for (int a = 0; a < m; a++)
                    if (!contains(jt->e_sep[e], jt->e_n[e], jt->cvars[c][a])) lay[k++] = jt->cvars[c][a];
            } else {
                for (int a = 0; a < m; a++) lay[k++] = jt->cvars[c][a];
            }
            free(jt->cvars[c]);
            jt->cvars[c] = lay;
            jt->cstride[c] = malloc(sizeof(int64_t) * (size_t)m);
            int64_t s = 1;
            for (int a = m - 1; a >= 0; a--) { jt->cstride[c][a] = s; s *= net->card[lay[a]]; }
        }

    /* 8. index maps: map_e[j] = separator index of parent entry j */
    for (int e = 0; e < ne; e++) {
        int p = jt->e_par[e];
        int64_t* sep_stride = malloc(sizeof(int64_t) * (size_t)(jt->e_n[e] + 1));
        int64_t s = 1;
        for (int a = jt->e_n[e] - 1; a >= 0; a--) { sep_stride[a] = s; s *= net->card[jt->e_sep[e][a]]; }
        /* position of each separator variable inside the parent's layout */
        int* pos_in_p = malloc(sizeof(int) * (size_t)(jt->e_n[e] + 1));
        for (int a = 0; a < jt->e_n[e]; a++)
            for (int b = 0; b < jt->cn[p]; b++) if (jt->cvars[p][b] == jt->e_sep[e][a]) pos_in_p[a] = b;
        jt->map[e] = malloc(sizeof(int64_t) * (size_t)jt->csize[p]);
        for (int64_t j = 0; j < jt->csize[p]; j++) {
            int64_t idx = 0;
            for (int a = 0; a < jt->e_n[e]; a++) {
                int b = pos_in_p[a];
                int64_t digit = (j / jt->cstride[p][b]) % net->card[jt->cvars[p][b]];
                idx += digit * sep_stride[a];
            }
            jt->map[e][j] = idx;
        }
        free(sep_stride); free(pos_in_p);
    }

    /* 9. homes: CPT family -> smallest containing clique; variable likewise */
    jt->cpt_home = malloc(sizeof(int) * (size_t)n);
    jt->var_home = malloc(sizeof(int) * (size_t)n);
    for (int v = 0; v < n; v++) {
        int bc = -1, bv = -1;
        for (int c = 0; c < nc; c++) {
            int all = contains(jt->cvars[c], jt->cn[c], v);
            if (all && (bv < 0 || jt->csize[c] < jt->csize[bv])) bv = c;
            for (int k = 0; k < net->npar[v] && all; k++) all = contains(jt->cvars[c], jt->cn[c], net->par[v][k]);
            if (all && (bc < 0 || jt->csize[c] < jt->csize[bc])) bc = c;
        }
        jt->cpt_home[v] = bc;
        jt->var_home[v] = bv;
    }

    /* 10. prior potentials: product of the CPTs homed at each clique */
    int* digit = malloc(sizeof(int) * (size_t)n);
    for (int c = 0; c < nc; c++) {
        jt->prior[c] = malloc(sizeof(double) * (size_t)jt->csize[c]);
        for (int64_t i = 0; i < jt->csize[c]; i++) {
            for (int a = 0; a < jt->cn[c]; a++)
                digit[jt->cvars[c][a]] = (int)((i / jt->cstride[c][a]) % net->card[jt->cvars[c][a]]);
            double phi = 1.0;
            for (int v = 0; v < n; v++) {
                if (jt->cpt_home[v] != c) continue;
                int64_t idx = 0;
                for (int k = 0; k < net->npar[v]; k++) idx = idx * net->card[net->par[v][k]] + digit[net->par[v][k]];
                idx = idx * net->card[v] + digit[v];
                phi *= net->cpt[v] ? net->cpt[v][idx] : 1.0;
            }
            jt->prior[c][i] = phi;
        }
    }
    free(digit);
    *out = jt;
    return ORC_OK;
}

void orc_jt_stats(const orc_jt* jt, int64_t* st) {
    int64_t T = 0, K = 0, mx = 0;
    int D = 0;
    for (int c = 0; c < jt->nc; c++) {
        T += jt->csize[c];
        if (jt->csize[c] > mx) mx = jt->csize[c];
        if (jt->depth[c] > D) D = jt->depth[c];
    }
    for (int e = 0; e < jt->ne; e++) K += jt->csize[jt->e_par[e]];
    st[0] = jt->nc; st[1] = jt->ne; st[2] = jt->root; st[3] = jt->height[jt->root];
    st[4] = D; st[5] = T; st[6] = K; st[7] = mx;
}

int orc_jt_clique(const orc_jt* jt, int c, int32_t* vars, int cap, int32_t* height, int32_t* depth) {
    if (c < 0 || c >= jt->nc) return -1;
    for (int a = 0; a < jt->cn[c] && a < cap; a++) vars[a] = jt->cvars[c][a];
    if (height) *height = jt->height[c];
    if (depth) *depth = jt->depth[c];
    return jt->cn[c];
}

int orc_jt_edge(const orc_jt* jt, int e, int32_t* parent, int32_t* child, int32_t* sep, int cap) {
    if (e < 0 || e >= jt->ne) return -1;
    *parent = jt->e_par[e]; *child = jt->e_chi[e];
    for (int a = 0; a < jt->e_n[e] && a < cap; a++) sep[a] = jt->e_sep[e][a];
    return jt->e_n[e];
}

int orc_jt_map(const orc_jt* jt, int e, int64_t* out, size_t cap) {
    if (e < 0 || e >= jt->ne) return -1;
    int64_t m = jt->csize[jt->e_par[e]];
    if ((size_t)m > cap) return -1;
    memcpy(out, jt->map[e], sizeof(int64_t) * (size_t)m);
    return 0;
}

void orc_jt_elim_order(const orc_jt* jt, int32_t* order) {
    for (int v = 0; v < jt->n; v++) order[v] = jt->elim_order[v];
}

void orc_jt_homes(const orc_jt* jt, int32_t* cpt_home, int32_t* var_home) {
    for (int v = 0; v < jt->n; v++) { cpt_home[v] = jt->cpt_home[v]; var_home[v] = jt->var_home[v]; }
}

int orc_jt_prior(const orc_jt* jt, double* out, size_t cap) {
    size_t o = 0;
    for (int c = 0; c < jt->nc; c++) {
        if (o + (size_t)jt->csize[c] > cap) return -1;
        memcpy(out + o, jt->prior[c], sizeof(double) * (size_t)jt->csize[c]);
        o += (size_t)jt->csize[c];
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* propagation                                                        */
/* ------------------------------------------------------------------ */

/* Neumaier (1974) compensated sum. */
typedef struct { double s, c; } nsum_t;

static void nsum_add(nsum_t* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

static double nsum_get(const nsum_t* a) { return a->s + a->c; }

/* Hugin ratio with 0/0 taken as 0 (a zero old entry implies a zero new one). */
static double ratio(double num, double den) { return den == 0.0 ? 0.0 : num / den; }

typedef struct { int key, id; } ord_t;
static int ord_cmp(const void* a, const void* b) {
    const ord_t* x = a; const ord_t* y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

int orc_query(const orc_jt* jt, int n_obs, const int32_t* vars, const int32_t* states,
              double* log_pe, double* post, double* tables_out, double* seps_out) {
    int nc = jt->nc, ne = jt->ne, n = jt->n;
    /* validate evidence: distinct variables, states in range */
    int* obs = malloc(sizeof(int) * (size_t)n);
    for (int v = 0; v < n; v++) obs[v] = -1;
    for (int k = 0; k < n_obs; k++) {
        int v = vars[k];
        if (v < 0 || v >= n || obs[v] >= 0 || states[k] < 0 || states[k] >= jt->card[v]) { free(obs); return ORC_E_INVALID; }
        obs[v] = states[k];
    }
    double** phi = malloc(sizeof(double*) * (size_t)nc);
    for (int c = 0; c < nc; c++) {
        phi[c] = malloc(sizeof(double) * (size_t)jt->csize[c]);
        if (!phi[c]) { for (int d = 0; d < c; d++) free(phi[d]); free(phi); free(obs); return ORC_E_NOMEM; }
        memcpy(phi[c], jt->prior[c], sizeof(double) * (size_t)jt->csize[c]);
    }
    double** sep = malloc(sizeof(double*) * (size_t)(ne > 0 ? ne : 1));
    for (int e = 0; e < ne; e++) {
        sep[e] = malloc(sizeof(double) * (size_t)jt->e_size[e]);
        for (int64_t m = 0; m < jt->e_size[e]; m++) sep[e][m] = 1.0;
    }

    /* reduction: in every clique containing an observed variable, zero the
     * entries that disagree with the observed state */
    for (int c = 0; c < nc; c++)
        for (int a = 0; a < jt->cn[c]; a++) {
            int v = jt->cvars[c][a];
            if (obs[v] < 0) continue;
            for (int64_t i = 0; i < jt->csize[c]; i++)
                if ((i / jt->cstride[c][a]) % jt->card[v] != obs[v]) phi[c][i] = 0.0;
        }

    ord_t* ord = malloc(sizeof(ord_t) * (size_t)nc);

    /* collect: ascending (height, id); each non-root clique sends to its parent */
    for (int c = 0; c < nc; c++) { ord[c].key = jt->height[c]; ord[c].id = c; }
    qsort(ord, (size_t)nc, sizeof(ord_t), ord_cmp);
    for (int q = 0; q < nc; q++) {
        int c = ord[q].id;
        if (c == jt->root) continue;
        int e = jt->pedge[c], p = jt->parent[c];
        int64_t ns = jt->e_size[e], seg = jt->csize[c] / ns;
        nsum_t* acc = calloc((size_t)ns, sizeof(nsum_t));
        for (int64_t i = 0; i < jt->csize[c]; i++) nsum_add(&acc[i / seg], phi[c][i]);
        double* snew = malloc(sizeof(double) * (size_t)ns);
        for (int64_t m = 0; m < ns; m++) snew[m] = nsum_get(&acc[m]);
        for (int64_t j = 0; j < jt->csize[p]; j++) {
            int64_t m = jt->map[e][j];
            phi[p][j] *= ratio(snew[m], sep[e][m]);
        }
        free(sep[e]);
        sep[e] = snew;
        free(acc);
    }

    /* P(e) = sum of the root table */
    nsum_t z = { 0, 0 };
    for (int64_t i = 0; i < jt->csize[jt->root]; i++) nsum_add(&z, phi[jt->root][i]);
    double pe = nsum_get(&z);
    int rc = ORC_OK;
    if (!(pe > 0.0)) {
        rc = ORC_E_ZERO_EVIDENCE;
        if (log_pe) *log_pe = -INFINITY;
        goto done;
    }
    if (log_pe) *log_pe = log(pe);

    /* distribute: ascending (depth, id); each clique sends to its children */
    for (int c = 0; c < nc; c++) { ord[c].key = jt->depth[c]; ord[c].id = c; }
    qsort(ord, (size_t)nc, sizeof(ord_t), ord_cmp);
    for (int q = 0; q < nc; q++) {
        int p = ord[q].id;
        for (int k = 0; k < jt->nchild[p]; k++) {
            int c = jt->child[p][k];
            int e = jt->pedge[c];
            int64_t ns = jt->e_size[e], seg = jt->csize[c] / ns;
            nsum_t* acc = calloc((size_t)ns, sizeof(nsum_t));
            for (int64_t j = 0; j < jt->csize[p]; j++) nsum_add(&acc[jt->map[e][j]], phi[p][j]);
            double* snew = malloc(sizeof(double) * (size_t)ns);
            for (int64_t m = 0; m < ns; m++) snew[m] = nsum_get(&acc[m]);
            for (int64_t i = 0; i < jt->csize[c]; i++)
                phi[c][i] *= ratio(snew[i / seg], sep[e][i / seg]);
            free(sep[e]);
            sep[e] = snew;
            free(acc);
        }
    }

    /* posteriors: marginal of each variable at its home clique, normalised */
    if (post) {
        size_t o = 0;
        for (int v = 0; v < n; v++) {
            int c = jt->var_home[v];
            int a = 0;
            while (jt->cvars[c][a] != v) a++;
            int r = jt->card[v];
            nsum_t* acc = calloc((size_t)r, sizeof(nsum_t));
            for (int64_t i = 0; i < jt->csize[c]; i++) nsum_add(&acc[(i / jt->cstride[c][a]) % r], phi[c][i]);
            nsum_t tot = { 0, 0 };
            for (int x = 0; x < r; x++) nsum_add(&tot, nsum_get(&acc[x]));
            double zt = nsum_get(&tot);
            for (int x = 0; x < r; x++) post[o + (size_t)x] = nsum_get(&acc[x]) / zt;
            o += (size_t)r;
            free(acc);
        }
    }
    if (tables_out) {
        size_t o = 0;
        for (int c = 0; c < nc; c++) {
            memcpy(tables_out + o, phi[c], sizeof(double) * (size_t)jt->csize[c]);
            o += (size_t)jt->csize[c];
        }
    }
    if (seps_out) {
        size_t o = 0;
        for (int e = 0; e < ne; e++) {
            memcpy(seps_out + o, sep[e], sizeof(double) * (size_t)jt->e_size[e]);
            o += (size_t)jt->e_size[e];
        }
    }
done:
    for (int c = 0; c < nc; c++) free(phi[c]);
    for (int e = 0; e < ne; e++) free(sep[e]);
    free(phi); free(sep); free(ord); free(obs);
    return rc;
}

/* ------------------------------------------------------------------ */
/* joint posterior of several query variables                          */
/* ------------------------------------------------------------------ */

/* The problem statement asks for the conditional probability of the query
 * variables (plural) given the evidence.  For query variables that lie
 * together in one clique this is read from that clique's calibrated table,
 * which holds P(X_C, e): sum it over the clique's other variables and
 * normalise.  The clique is the smallest one holding every query variable
 * (lowest id on ties).  out has prod card[q] entries, q[0] slowest and
 * q[nq-1] fastest. */
int orc_query_joint(const orc_jt* jt, int n_obs, const int32_t* vars, const int32_t* states,
                    int nq, const int32_t* q, double* out) {
    if (nq <= 0) return ORC_E_INVALID;
    for (int a = 0; a < nq; a++) {
        if (q[a] < 0 || q[a] >= jt->n) return ORC_E_INVALID;
        for (int b = 0; b < a; b++) if (q[b] == q[a]) return ORC_E_INVALID;
    }
    int home = -1;
    for (int c = 0; c < jt->nc; c++) {
        int all = 1;
        for (int a = 0; a < nq && all; a++) all = contains(jt->cvars[c], jt->cn[c], q[a]);
        if (all && (home < 0 || jt->csize[c] < jt->csize[home])) home = c;
    }
    if (home < 0) return ORC_E_INVALID;
    int64_t total = 0;
    for (int c = 0; c < jt->nc; c++) total += jt->csize[c];
    double* tables = malloc(sizeof(double) * (size_t)total);
    if (!tables) return ORC_E_NOMEM;
    int rc = orc_query(jt, n_obs, vars, states, NULL, NULL, tables, NULL);
    if (rc) { free(tables); return rc; }
    int64_t off = 0;
    for (int c = 0; c < home; c++) off += jt->csize[c];
    const double* phi = tables + off;
    /* position of each query variable in the clique layout, and its stride
     * in the output (last listed fastest) */
    int64_t* cs = malloc(sizeof(int64_t) * (size_t)nq);
    int64_t* os = malloc(sizeof(int64_t) * (size_t)nq);
    int64_t nout = 1;
    for (int a = nq - 1; a >= 0; a--) {
        int k = 0;
        while (jt->cvars[home][k] != q[a]) k++;
        cs[a] = jt->cstride[home][k];
        os[a] = nout;
        nout *= jt->card[q[a]];
    }
    nsum_t* acc = calloc((size_t)nout, sizeof(nsum_t));
    for (int64_t i = 0; i < jt->csize[home]; i++) {
        int64_t o = 0;
        for (int a = 0; a < nq; a++) o += ((i / cs[a]) % jt->card[q[a]]) * os[a];
        nsum_add(&acc[o], phi[i]);
    }
    nsum_t z = { 0, 0 };
    for (int64_t o = 0; o < nout; o++) nsum_add(&z, nsum_get(&acc[o]));
    const double zt = nsum_get(&z);
    for (int64_t o = 0; o < nout; o++) out[o] = nsum_get(&acc[o]) / zt;
    free(acc); free(cs); free(os); free(tables);
    return ORC_OK;
}
