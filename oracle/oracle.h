/*
 * FP64 junction-tree oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded-per-query CPU implementation of exact
 * inference on a discrete Bayesian network by the junction tree (Hugin)
 * method.  It exists to check the GPU library; it shares no code, header,
 * table or helper with it.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark may load it.
 *
 * What it computes (paper, Section 1 and Section 2):
 *   - the query P(X_v | e) for every variable v given hard evidence e;
 *   - by compiling the network into a junction tree (cliques joined by
 *     separators, each holding a potential table) and passing messages
 *     along it so every table is updated (Section 1);
 *   - with the three table operations the paper names (Section 2):
 *     reduction (entering evidence), marginalisation onto a separator and
 *     extension by the new/old separator ratio.
 * The paper gives no formulas; every step below follows the textbook
 * construction, with these fixed tie-breaks:
 *   moralise -> min-fill elimination (key: fill, table weight, id)
 *   -> maximal elimination cliques (id = elimination rank)
 *   -> Kruskal maximum-weight spanning tree over all clique pairs
 *      (key: -|sep|, product of sep cardinalities, i, j)
 *   -> root = minimum eccentricity (ties: lowest id), BFS depth, height
 *   -> layouts: root ascending; a separator's variables in the order
 *      they take in its parent's layout; other cliques [parent separator]
 *      ++ [rest ascending]; last variable fastest
 *   -> one index map per edge (parent entry -> separator entry)
 *   -> priors: product of CPTs homed at the smallest containing clique
 *   -> evidence, collect (ascending height,id), P(e), distribute
 *      (ascending depth,id), posteriors at each variable's smallest clique.
 * Every sum is Neumaier-compensated in ascending source-index order.
 */
#ifndef FBN_ORACLE_H
#define FBN_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_E_INVALID = 1, ORC_E_PARSE = 2, ORC_E_TOO_LARGE = 3,
       ORC_E_ZERO_EVIDENCE = 4, ORC_E_NOMEM = 5 };

typedef struct orc_net orc_net;
typedef struct orc_jt orc_jt;

/* .fbn text; err receives a message on failure. */
int  orc_net_from_text(const char* text, size_t len, orc_net** out, char* err, size_t errlen);
/* Arrays: card[n]; npar[n]; parents concatenated; cpt concatenated per
 * variable (parents in listed order, variable fastest).  cpt may be NULL:
 * structure only, every CPT entry taken as 1. */
int  orc_net_from_arrays(int n, const int32_t* card, const int32_t* npar, const int32_t* parents,
                         const double* cpt, orc_net** out, char* err, size_t errlen);
void orc_net_free(orc_net* net);

/* Compile.  max_entries: fail with ORC_E_TOO_LARGE when an elimination
 * clique exceeds it (0 = no limit). */
int  orc_compile(const orc_net* net, uint64_t max_entries, orc_jt** out);
void orc_jt_free(orc_jt* jt);
/* Moralise and run min-fill only.  Returns 0 when every elimination clique
 * has at most max_entries entries, else the size of the first one that does
 * not, written (unsorted, eliminated variable first) to clique[0..cap). */
int  orc_probe_cap(const orc_net* net, uint64_t max_entries, int32_t* clique, int cap);

/* stats[0..7] = n_cliques, n_edges, root, H (root height), D (max depth),
 *               T (sum of clique entries), K (sum of map entries), max clique */
void orc_jt_stats(const orc_jt* jt, int64_t* stats);
/* vars in layout order; returns count */
int  orc_jt_clique(const orc_jt* jt, int c, int32_t* vars, int cap, int32_t* height, int32_t* depth);
/* edge e (edges numbered by ascending child id); sep vars in the separator's
 * layout order (their order in the parent's layout); returns count */
int  orc_jt_edge(const orc_jt* jt, int e, int32_t* parent, int32_t* child, int32_t* sep, int cap);
/* map_e[j] for j < |parent table| */
int  orc_jt_map(const orc_jt* jt, int e, int64_t* out, size_t cap);
void orc_jt_elim_order(const orc_jt* jt, int32_t* order);
/* cpt_home[v], var_home[v] */
void orc_jt_homes(const orc_jt* jt, int32_t* cpt_home, int32_t* var_home);
/* prior tables concatenated by clique id, in layout order */
int  orc_jt_prior(const orc_jt* jt, double* out, size_t cap);

/* One query.  post: concat over v of card[v] probabilities (may be NULL).
 * tables_out: calibrated clique tables (T entries, may be NULL).
 * seps_out: calibrated separator tables by edge id (may be NULL).
 * Returns ORC_E_ZERO_EVIDENCE when P(e) = 0 (log_pe = -inf, no posteriors). */
int  orc_query(const orc_jt* jt, int n_obs, const int32_t* vars, const int32_t* states,
               double* log_pe, double* post, double* tables_out, double* seps_out);

/* Joint posterior P(q | e) of nq distinct query variables that lie together
 * in one clique: the calibrated table of the smallest such clique (lowest id
 * on ties) summed onto them and normalised.  out: prod card[q] entries, q[0]
 * slowest, q[nq-1] fastest.  ORC_E_INVALID when q is empty, repeats a
 * variable or shares no clique; ORC_E_ZERO_EVIDENCE as orc_query. */
int  orc_query_joint(const orc_jt* jt, int n_obs, const int32_t* vars, const int32_t* states,
                     int nq, const int32_t* q, double* out);

#ifdef __cplusplus
}
#endif
#endif
