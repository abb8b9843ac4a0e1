/*
 * fbn.h -- C ABI of the MI355X junction-tree inference library.
 *
 * The calls follow the problem statement of Jiang, Wen, Mansoor and Mian,
 * "Fast Parallel Exact Inference on Bayesian Networks" (PPoPP'23 poster):
 *   - a Bayesian network is a DAG over discrete variables with conditional
 *     probability tables (Section 1)                      -> fbn_load_net*
 *   - it is compiled into a junction tree whose cliques and separators
 *     each hold a potential table (Section 1), with every clique and
 *     separator marked by its layer and the root chosen for the fewest
 *     layers (Section 2)                                  -> fbn_build_jt
 *   - evidence fixes the values of some variables (Section 1); entering it
 *     is the "reduction" table operation (Section 2)     -> fbn_set_evidence
 *   - messages pass along the tree and update every table, using the
 *     marginalisation and extension operations on index mappings between
 *     tables (Sections 1 and 2), one launch per layer   -> fbn_calibrate
 *   - the answer is the conditional probability of query variables given
 *     the evidence (Section 1)                           -> fbn_query_marginals
 *
 * Conventions
 *   Ownership: handles are opaque, created by the library and released by
 *   the caller (fbn_free_*; NULL is accepted).  Input arrays are borrowed for
 *   the duration of the call only.  Output arrays are caller-allocated host
 *   memory with the sizes stated.  A jt copies everything it needs from the
 *   net, which may be freed right after fbn_build_jt.
 *   Errors: every call returns an fbn_status; FBN_OK is 0.  No C++ exception
 *   crosses the ABI.  fbn_last_error() gives a thread-local detail string.
 *   A failing call leaves the handle in its previous valid state.
 *   Device and streams: a jt lives on the HIP device that was current when
 *   it was built; all of its work is enqueued on its stream (options.stream,
 *   or the legacy default stream when NULL).  fbn_calibrate is asynchronous
 *   unless it is asked for log_pe / per_slot; the query calls synchronise
 *   the stream.  One jt must be driven by one host thread at a time;
 *   separate jts may run concurrently on separate streams.
 *   Precision: results at the boundary are always float64.
 */
#ifndef FBN_H
#define FBN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fbn_net fbn_net;   /* host-only network (DAG + float64 CPTs) */
typedef struct fbn_jt fbn_jt;     /* compiled junction tree + device state  */
typedef int32_t fbn_status;

enum {
    FBN_OK = 0,
    FBN_E_INVALID_ARG = 1,    /* bad pointer, index, size or evidence         */
    FBN_E_PARSE = 2,          /* malformed .fbn text                          */
    FBN_E_IO = 3,             /* file could not be read                       */
    FBN_E_NOMEM_HOST = 4,
    FBN_E_NOMEM_DEVICE = 5,   /* the allocator returned NULL                  */
    FBN_E_TOO_LARGE = 6,      /* a clique exceeds max_clique_entries          */
    FBN_E_ZERO_EVIDENCE = 7,  /* P(e) = 0 for that slot                       */
    FBN_E_STATE = 8,          /* call not valid in this state (e.g. host_only) */
    FBN_E_DEVICE = 9,         /* a HIP runtime call failed                    */
    FBN_E_UNDERFLOW = 10      /* FP32 message vanished; rerun the case in FP64 */
};

enum { FBN_FP64 = 0, FBN_FP32_RESCALED = 1 };

/* Device layout of the per-slot tables.  PER_SLOT keeps each slot's tables
 * contiguous and spreads one slot's table entries over the lanes of a wave:
 * long sums run across lanes.  INTERLEAVED stores entry x of slot s at
 * x * max_slots + s and gives each lane one slot, with every index
 * computation shared by the wave: gathers onto large separators are cheaper,
 * but every long sum runs within one lane.  INTERLEAVED also keeps no
 * working table for a clique with at most six children (the distribute
 * rebuilds it from the prior, the evidence and the child messages, to the
 * same bits), so its slots take far less device memory.  AUTO is PER_SLOT;
 * the Python autotuner measures both.  Results are the same to rounding. */
enum { FBN_LAYOUT_AUTO = 0, FBN_LAYOUT_PER_SLOT = 1, FBN_LAYOUT_INTERLEAVED = 2 };

/* Device memory comes from the caller when alloc is set (e.g. PyTorch's
 * caching allocator); otherwise hipMalloc / hipFree are used. */
typedef struct {
    void* (*alloc)(void* ctx, size_t bytes, void* stream);  /* NULL on failure */
    void (*free)(void* ctx, void* ptr, void* stream);
    void* ctx;
} fbn_allocator;

typedef struct {
    int32_t precision;            /* FBN_FP64 or FBN_FP32_RESCALED            */
    int32_t max_slots;            /* evidence cases resident at once (>= 1)   */
    uint64_t max_clique_entries;  /* build fails with FBN_E_TOO_LARGE above   */
    int32_t host_only;            /* 1: compile the tree, no device state     */
    int32_t tile_entries;         /* table entries per workgroup; 0 = default */
    fbn_allocator allocator;
    void* stream;                 /* hipStream_t                              */
    int32_t layout;               /* FBN_LAYOUT_*                             */
    int32_t shrink_evidence;      /* PER_SLOT layout, the reduction of
                                   * Section 2 shrinking what is streamed:
                                   * 1 reads and writes, per slot, only the
                                   * table entries that agree with its
                                   * evidence; 0 (default) streams every
                                   * entry, the zeroed ones included.
                                   * Results are bitwise the same.            */
    int32_t fp64_rerun;           /* FP32 trees: 1 recomputes a slot whose
                                   * FP32 messages vanished (FBN_E_UNDERFLOW)
                                   * on a one-slot FP64 tree of the same
                                   * network, built on first need, inside
                                   * fbn_calibrate (when it reports results),
                                   * fbn_query_all / _marginals and
                                   * fbn_query_joint; that slot's results are
                                   * then the FP64 ones and its status is the
                                   * FP64 status.  fbn_fetch_async still
                                   * reports the raw flags.  0: no rerun.     */
    int32_t slots_per_block;      /* PER_SLOT layout: most evidence slots one
                                   * layer workgroup carries, sharing its index
                                   * arithmetic: 1, 2, 4 or 8.  0 (default):
                                   * as many as the layer's LDS stage fits in
                                   * 32 KB, fewer while the layer's grid would
                                   * not give every compute unit a workgroup.
                                   * Results are bitwise the same.            */
    int32_t fin_block;            /* PER_SLOT layout: separator entries per
                                   * block when a large separator is finalised
                                   * in blocks, 64 to 4096; 0 (default) 4096.
                                   * Only the order of the posterior sums'
                                   * additions changes.  Other values:
                                   * FBN_E_INVALID_ARG.                       */
} fbn_jt_options;

typedef struct {
    int32_t n_vars, n_cliques, n_edges, root, H, D; /* root: first root; H: max height, D: max depth */
    uint64_t T;            /* sum of clique table entries                         */
    uint64_t K;            /* sum over edges of the parent table size (map length) */
    uint64_t max_clique;   /* largest clique table                                */
    uint64_t sep_total;    /* sum of separator table entries                      */
    uint64_t device_bytes; /* device memory held by the jt (host_only: the bytes a */
    uint64_t slot_bytes;   /* device build would hold); of which per evidence slot */
    int32_t n_trees;       /* networks (roots) in the jt: 1 unless built as a forest */
    int32_t interleaved;   /* 1 when the jt uses FBN_LAYOUT_INTERLEAVED              */
} fbn_jt_stats_t;

/* Fill opt with defaults: FP64, 1 slot, 2^31-1 max entries, device build. */
void fbn_default_options(fbn_jt_options* opt);

/* --- networks (Section 1) -------------------------------------------------
 * Two text formats, told apart by the first word:
 *  .fbn: "fbn 1", "vars n", then per variable "var v r k p1..pk", then per
 *    variable "cpt v m x1..xm" (parents in listed order, v fastest; values as
 *    C99 hexadecimal or decimal floats), then "end".
 *  BIF (Bayesian Interchange Format, the format of the public networks the
 *    paper evaluates on, Section 3 and Table 1): "network", "variable NAME {
 *    type discrete [r] { states }; }" and "probability ( NAME | PARENTS ) {
 *    (parent states) p..; default p..; }" blocks ("table p..;" for a variable
 *    without parents); comments and property lines are skipped.  Variables
 *    are numbered in declaration order, parents kept in the listed order.  A
 *    conditional distribution given as one flat table is refused as
 *    ambiguous (FBN_E_PARSE); a row summing to within 1e-3 of one is divided
 *    by its sum (rounded decimals), larger deviations are FBN_E_PARSE.
 * Validation (both): acyclic, 2 <= r <= 65535, entries finite and >= 0,
 * each row summing to 1 within 1e-9.  Errors: FBN_E_IO (file), FBN_E_PARSE
 * (syntax, names, missing rows; fbn_last_error() gives the line),
 * FBN_E_INVALID_ARG (a parsed network that fails validation). */
fbn_status fbn_load_net(const char* path, fbn_net** out);
fbn_status fbn_load_net_mem(const char* text, size_t len, fbn_net** out);
/* Names and tables of a loaded network.  A BIF network keeps its declared
 * variable and state names; an .fbn one is named by decimal ids ("0", "1",
 * ...).  Name buffers are caller-owned, NUL-terminated (FBN_E_INVALID_ARG if
 * cap is too small).  fbn_net_cpt gives v's cardinality, its parents (at
 * most par_cap written) and its CPT in the layout above (at most cpt_cap
 * doubles); any output pointer may be NULL. */
fbn_status fbn_net_n_vars(const fbn_net* net, int32_t* n);
fbn_status fbn_net_var_name(const fbn_net* net, int32_t v, char* buf, size_t cap);
fbn_status fbn_net_state_name(const fbn_net* net, int32_t v, int32_t s, char* buf, size_t cap);
fbn_status fbn_net_find_var(const fbn_net* net, const char* name, int32_t* v);
fbn_status fbn_net_find_state(const fbn_net* net, int32_t v, const char* name, int32_t* s);
fbn_status fbn_net_cpt(const fbn_net* net, int32_t v, int32_t* card, int32_t* parents, int32_t par_cap,
                       int32_t* n_parents, double* cpt, size_t cpt_cap, size_t* cpt_len);
/* The same network from arrays: card[n], n_parents[n], parents concatenated,
 * cpt concatenated per variable in the layout above. */
fbn_status fbn_net_from_arrays(int32_t n_vars, const int32_t* card, const int32_t* n_parents,
                               const int32_t* parents, const double* cpt, fbn_net** out);
void fbn_free_net(fbn_net* net);

/* --- junction tree (Sections 1, 2) ----------------------------------------
 * Moralise, min-fill triangulation, maximum-weight spanning junction tree,
 * root of minimum eccentricity (fewest layers), per-edge index maps, prior
 * potentials, device upload.  opt may be NULL (defaults). */
fbn_status fbn_build_jt(const fbn_net* net, const fbn_jt_options* opt, fbn_jt** out);
/* Several independent networks in one jt: each is compiled exactly as by
 * fbn_build_jt (its own tree and root), and the trees form one forest whose
 * layers are aligned by height in the collect sweep and by depth in the
 * distribute sweep, so one launch per layer serves every network (the
 * paper's layer-wise parallelism of Section 2 taken across networks).
 * Variables, cliques and edges of network k follow those of networks
 * 0..k-1 (ids offset by their counts); one slot carries evidence for all
 * networks at once, and its log P(e) is the sum over the networks.
 * nets[n_nets] are borrowed for the call.  A network that fails to compile
 * fails the whole call (its index is named in fbn_last_error()). */
fbn_status fbn_build_forest(const fbn_net* const* nets, int32_t n_nets, const fbn_jt_options* opt, fbn_jt** out);
void fbn_free_jt(fbn_jt* jt);  /* synchronises its stream first */
/* Replace the stream used by later calls (drops captured graphs). */
fbn_status fbn_set_stream(fbn_jt* jt, void* stream);
/* Graph mode (Section 2's one task per layer, with the whole sequence of
 * layer launches of one calibration captured once as a HIP graph per batch
 * size and replayed): on = 1 enables it, 0 returns to eager launches.
 * Needs a non-NULL stream (FBN_E_STATE otherwise).  Results are bitwise
 * identical to eager launches.  Kernel timing (below) disables replay. */
fbn_status fbn_set_graph_mode(fbn_jt* jt, int32_t on);

/* --- evidence: the reduction operation (Section 2) -------------------------
 * Hard evidence for one slot: distinct variables, 0 <= state < card.  n_obs = 0
 * clears the slot.  Staged on the host; uploaded by the next fbn_calibrate. */
fbn_status fbn_set_evidence(fbn_jt* jt, int32_t slot, int32_t n_obs, const int32_t* vars,
                            const int32_t* states);
/* Several slots at once: case i uses vars/states[offsets[i] .. offsets[i+1]). */
fbn_status fbn_set_evidence_batch(fbn_jt* jt, int32_t n_slots, const int32_t* slots,
                                  const int32_t* offsets, const int32_t* vars, const int32_t* states);

/* --- propagation: marginalisation and extension, layer by layer (Section 2)
 * Collect then distribute for the listed slots, all slots in the same
 * launches.  log_pe (n_slots doubles) and per_slot (n_slots statuses) may be
 * NULL; if either is given the call waits for the device and fills them. */
fbn_status fbn_calibrate(fbn_jt* jt, int32_t n_slots, const int32_t* slots, double* log_pe,
                         fbn_status* per_slot);

/* --- queries (Section 1) ---------------------------------------------------
 * Posterior P(v | e) of each listed variable, concatenated (card[v] doubles
 * each) into out[0 .. out_len).  Synchronises. */
fbn_status fbn_query_marginals(fbn_jt* jt, int32_t slot, int32_t n_vars, const int32_t* vars,
                               double* out, size_t out_len);
/* All posteriors of several slots: out holds n_slots * sum(card) doubles,
 * slot-major; log_pe and per_slot as in fbn_calibrate (may be NULL). */
fbn_status fbn_query_all(fbn_jt* jt, int32_t n_slots, const int32_t* slots, double* out,
                         size_t out_len, double* log_pe, fbn_status* per_slot);
/* Asynchronous form of fbn_query_all: enqueues the copies on the jt's stream
 * into caller-owned host memory (pinned for true overlap); the caller must
 * synchronise that stream before reading.  per_slot receives raw flags: 0 ok,
 * bit 0 zero evidence, bit 1 FP32 underflow, bit 2 results recomputed in FP64
 * (fp64_rerun). */
fbn_status fbn_fetch_async(fbn_jt* jt, int32_t n_slots, const int32_t* slots, double* post_out,
                           double* log_pe_out, int32_t* flags_out);

/* Joint posterior P(Q | e) of n_q distinct query variables that lie together
 * in one clique (Section 1: the conditional probability of the query
 * variables -- plural -- given the evidence).  Reads what the slot's last
 * fbn_calibrate left on the device: the calibrated table of the smallest
 * clique holding every query variable (lowest id on ties) is rebuilt entry
 * by entry (prior, evidence, child messages, parent ratio), summed onto Q in
 * float64 in a fixed order and normalised.  out (host memory, out_len >=
 * prod card[q] doubles) receives the joint with q_vars[0] slowest and
 * q_vars[n_q-1] fastest.  Errors: FBN_E_INVALID_ARG for an empty, repeated
 * or out-of-range Q, Q spanning no single clique, or out_len too small;
 * FBN_E_NOMEM_DEVICE if its scratch (about prod card[q] doubles plus one
 * per 16 clique entries when Q is small) cannot be allocated; the slot's
 * FBN_E_ZERO_EVIDENCE / FBN_E_UNDERFLOW as in fbn_query_marginals (out then
 * unspecified).  Allocates device scratch per call (the jt's allocator
 * when set) and synchronises the jt's stream. */
fbn_status fbn_query_joint(fbn_jt* jt, int32_t slot, int32_t n_q, const int32_t* q_vars, double* out,
                           size_t out_len);
/* fbn_query_joint for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, hosts that forbid allocation): the same
 * read-out, bitwise the same result, with its scratch in a static device
 * array of 2^22 doubles (32 MiB) that each GPU the library runs on holds
 * until the process ends.  Calls no allocator.  A read-out needing more
 * scratch than that (about n_out + n_out / 256 doubles, plus n_out * chunks
 * when each joint assignment covers more than 16 * 64 clique entries) fails
 * with FBN_E_TOO_LARGE and changes nothing.  All calls on one GPU share that
 * GPU's array: calls that overlap in time on one GPU (other host threads,
 * other jts' streams) race and must be serialised by the caller.  Other
 * errors as fbn_query_joint. */
fbn_status fbn_query_joint_noalloc(fbn_jt* jt, int32_t slot, int32_t n_q, const int32_t* q_vars, double* out,
                                   size_t out_len);

/* --- kernel timing ----------------------------------------------------------
 * When enabled, every kernel launch of fbn_calibrate is bracketed by HIP
 * events on the jt's stream.  fbn_jt_profile_read waits for the stream and
 * returns, per kernel kind (0 collect layer, 1 collect separator finalise,
 * 2 distribute layer, 3 distribute separator finalise, 4 posteriors), the
 * summed milliseconds, launch count and algorithmic bytes (table entries
 * each layer must read or write, times the entry width, times slots), then
 * resets the counters.  Arrays have FBN_PROFILE_KINDS entries. */
enum { FBN_PROFILE_KINDS = 5 };
fbn_status fbn_jt_profile_enable(fbn_jt* jt, int32_t on);
/* Which kinds are timed while profiling is on: bit k for kind k (default all,
 * 0x1f).  Launches of other kinds get no events, so a run timing one kind
 * pays for one event pair per launch of that kind only. */
fbn_status fbn_jt_profile_kinds(fbn_jt* jt, uint32_t mask);
fbn_status fbn_jt_profile_read(fbn_jt* jt, double* ms, int64_t* launches, double* bytes);

const char* fbn_status_str(fbn_status s);
const char* fbn_last_error(void);

/* --- introspection for structure parity tests ------------------------------ */
fbn_status fbn_jt_stats(const fbn_jt* jt, fbn_jt_stats_t* out);
/* Variables of clique c in table layout order (at most cap written; *n gets
 * the count), with its height (collect layer) and depth (distribute layer). */
fbn_status fbn_jt_clique(const fbn_jt* jt, int32_t c, int32_t* vars, int32_t cap, int32_t* n,
                         int32_t* height, int32_t* depth);
/* Edge e (numbered by ascending child clique id): parent, child, separator
 * variables in the separator's table layout, which is the order they take in
 * the parent clique's layout. */
fbn_status fbn_jt_edge(const fbn_jt* jt, int32_t e, int32_t* parent, int32_t* child,
                       int32_t* sep_vars, int32_t cap, int32_t* n);
/* The index map of edge e: out[j] = separator entry of parent entry j, for
 * j < |parent table| (cap must be at least that).  Expanded on the host from
 * the factored tables the kernels read. */
fbn_status fbn_jt_index_map(const fbn_jt* jt, int32_t e, int32_t* out, size_t cap);
/* The same map expanded by a kernel from the device copy of those tables. */
fbn_status fbn_jt_device_index_map(fbn_jt* jt, int32_t e, int32_t* out, size_t cap);
/* Elimination order (n_vars), CPT home clique and posterior home clique per variable. */
fbn_status fbn_jt_elim_order(const fbn_jt* jt, int32_t* order);
fbn_status fbn_jt_homes(const fbn_jt* jt, int32_t* cpt_home, int32_t* var_home);

#ifdef __cplusplus
}
#endif
#endif
