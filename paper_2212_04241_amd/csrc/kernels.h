// Launch interface of the layer kernels (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include "fbn_internal.h"

namespace fbn {

// Device pointers and per-slot strides for one junction tree.  Per-slot
// arrays are slot-major: slot s starts at base + s * stride.
struct Ctx {
    const DClique* cl;
    const DChild* ch;
    const DTarget* tg;
    const DMargVar* mv;
    const DWTarget* wt;
    const DPiece* pc;
    const DHomeVar* hv;
    const uint64_t* dig;
    const uint32_t* map;
    const void* prior;     // T
    void* psi;             // T, working tables (psi_stride)
    void* sepc;            // T, collect messages, rescaled (sep_stride)
    void* sepd;            // T, distribute ratios, rescaled (sep_stride)
    void* acc;             // new separator sums (sep_stride), table precision: every sum is
                           // accumulated in float64 and rounded once when stored
    void* part;            // partial sums (part_stride), table precision, likewise
    double* rsum;          // per slot: each root's sum (its tree's share of P(e)), float64, unrounded
                           // (nroots per slot; interleaved: root r of slot s at r * S + s)
    int32_t* kexp;         // collect rescale exponents (kexp_stride)
    double* marg;          // float64 marginal accumulators (marg_stride)
    double* post;          // float64 posteriors (marg_stride)
    double* logpe;         // per slot
    int32_t* flags;        // per slot: bit 0 zero evidence, bit 1 FP32 underflow
    const DEvidence* ev;   // ev_stride per slot
    double* bmax;          // per slot: maximum of each large-separator block (bmax_stride)
    double* bmarg;         // per slot: partial posterior sums of those blocks (bmarg_stride)
    uint64_t psi_stride;
    uint32_t sep_stride, part_stride, kexp_stride, marg_stride, ev_stride, bmax_stride, bmarg_stride;
    int32_t nvars, ne, kappa_total, fp32;
    uint32_t sep_total, nroots;  // the roots' one-entry separators follow sep_total
    uint32_t S;            // slot-interleaved layout: entry x of slot s at x * S + s (0: per-slot layout)
    uint32_t tile;         // LDS entries reserved per slot in a workgroup
    int32_t dense;         // per-slot layout: 1 streams every table entry; 0 skips, per slot, the
                           // entries its evidence zeroes (never read, psi never written there):
                           // the shrink_evidence option
    int32_t bcap;          // per-slot layout: most slots per layer workgroup (0: no cap)
};

// Bytes of LDS one slot's tile may take: plans keep every collect group and
// distribute work item of the per-slot layout within it.
constexpr int kSlotStageBytes = 16384;
// Bytes of LDS a layer workgroup stages at most; slots per workgroup times
// the layer's stage times the entry width must fit.  Twice one slot's bound,
// so that the largest tiles still share a workgroup between slots.
constexpr int kStageBytes = 32768;
// Workgroups (one per compute unit) below which a layer launch trades shared
// index arithmetic for parallel slots: fewer slots per workgroup, more
// workgroups.
constexpr uint64_t kFillGrid = 256;
// Slots one workgroup carries for a stage of `tile` entries of width w, over
// `items` work items and `nslots` slots;
// `cap` (0: none) bounds the result.
inline int slots_per_block(uint32_t tile, int w, uint64_t items, int nslots, int cap) {
    if (nslots < 4) return 1;
    int b = kStageBytes / (int)(tile * (uint32_t)w);
    if (cap > 0 && b > cap) b = cap;
    b = b >= 8 && nslots >= 8 ? 8 : (b >= 4 ? 4 : (b >= 2 ? 2 : 1));
    while (b > 1 && items * (uint64_t)((nslots + b - 1) / b) < kFillGrid) b /= 2;
    return b;
}

// prec: 0 = float64 tables, 1 = float32 tables
// stage: LDS entries per slot of the layer's largest group (collect) or work
// item (distribute); the launch sizes its LDS and slots per workgroup from it.
hipError_t launch_collect(const Ctx& c, int prec, const DGroup* groups, uint32_t ngroups, uint32_t stage,
                          const int32_t* slots, int nslots, hipStream_t s);
// A layer's finalisers, first launch: the nsmall small separators `sfins`
// (the first nbig of them a workgroup each, the rest a wave each) and the
// first phase of the large separators' blocks `blks` (nblks; `fins` is the
// whole finaliser array).
hipError_t launch_fin_collect(const Ctx& c, int prec, const DSepFin* sfins, uint32_t nsmall, uint32_t nbig,
                              const DSepFin* fins, const DFinBlk* blks, uint32_t nblks, const int32_t* slots,
                              int nslots, hipStream_t s);
// Second phase of the large separators' blocks, for the collect
// (distribute = false) or distribute sweep.
hipError_t launch_fin_blocks(const Ctx& c, int prec, bool distribute, const DSepFin* fins, const DFinBlk* blks,
                             uint32_t nblks, const int32_t* slots, int nslots, hipStream_t s);
hipError_t launch_distribute(const Ctx& c, int prec, const DWork* works, uint32_t nworks, uint32_t stage,
                             const int32_t* slots, int nslots, hipStream_t s);
hipError_t launch_fin_distribute(const Ctx& c, int prec, const DSepFin* sfins, uint32_t nsmall, uint32_t nbig,
                                 const DSepFin* fins, const DFinBlk* blks, uint32_t nblks, const int32_t* slots,
                                 int nslots, hipStream_t s);
hipError_t launch_marginals(const Ctx& c, const int32_t* slots, int nslots, hipStream_t s);
hipError_t launch_gather(const Ctx& c, const int32_t* slots, int nslots, double* post_out,
                         double* logpe_out, int32_t* flags_out, hipStream_t s);
hipError_t launch_begin(const Ctx& c, const int32_t* slots, int nslots, hipStream_t s);
hipError_t launch_expand_map(const uint32_t* map, uint32_t mh, uint32_t ml, uint32_t L, uint32_t Lmul,
                             uint32_t Lsh, uint32_t n, int32_t* out, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// Slot-interleaved layout (kernels_interleaved.hip): one wave per work item,
// lanes over the batch.  `items` is the layer's DGroup / DWork / DFinBlk
// array by kind; `fins` is the whole finaliser array (block kinds).
enum : int { kIlCollect, kIlDistribute, kIlFinCollectB, kIlFinDistributeB };
hipError_t launch_interleaved(const Ctx& c, int prec, int kind, const void* items, uint32_t nitems,
                              const DSepFin* fins, const int32_t* slots, int nslots, hipStream_t s);
// A layer's small separators (`small`, nsmall of them) and the first phase of
// its large separators' blocks (`blks`, nblks) in one launch.
hipError_t launch_fin_interleaved(const Ctx& c, int prec, bool dist, const DSepFin* small, uint32_t nsmall,
                                  const DFinBlk* blks, uint32_t nblks, const DSepFin* fins, const int32_t* slots,
                                  int nslots, hipStream_t s);
hipError_t launch_marginals_interleaved(const Ctx& c, const int32_t* slots, int nslots, hipStream_t s);

// Joint posterior read-out (kernels_query.hip).  A clique variable as the
// read-out enumerates it: its cardinality (with the multiply-high constants
// of a division by it) and its stride in the clique table.
constexpr int kJointMaxVars = 32;
struct JointVar {
    uint32_t card, cmul, csh, stride;
};
struct JointArgs {
    uint32_t clique;     // the clique read (its evidence record)
    int32_t slot;
    uint32_t n_out;      // joint assignments of the query variables
    uint32_t n_r;        // clique entries per assignment: |C| / n_out
    uint32_t nchunk;     // chunks per assignment
    uint32_t chunk;      // entries per chunk
    uint32_t tpo;        // lanes per chunk (a power of two, at most 64)
    uint32_t nq, no;     // query variables, other variables of the clique
    JointVar qv[kJointMaxVars];  // query variables, the last listed (fastest) first
    JointVar ov[kJointMaxVars];  // the clique's other variables, fastest first
};
// Device doubles the read-out needs: the outputs, one sum per block of 256
// outputs and, when an output has several chunks, the chunk sums.
size_t joint_scratch_doubles(const JointArgs& a);
// Normalised P(Q | e) of slot a.slot into scratch[0 .. a.n_out), from the
// calibrated tables of clique q; scratch holds joint_scratch_doubles(a).
hipError_t launch_joint(const Ctx& c, int prec, const DClique& q, const JointArgs& a, double* scratch,
                        hipStream_t s);
// The allocation-free read-out's scratch: a device array of
// kJointScratchDoubles doubles (32 MiB) per GPU, held until the process
// ends.  *ptr receives its address on the current device, looked up once per
// device.
constexpr size_t kJointScratchDoubles = size_t(1) << 22;
hipError_t joint_static_scratch(double** ptr);

}  // namespace fbn
