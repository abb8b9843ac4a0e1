// Layer kernels of junction-tree propagation for gfx950 (CDNA4, wave64).
//
// The paper identifies three potential-table operations as the dominant
// cost of exact inference -- reduction (entering evidence), marginalisation
// onto a separator and extension by a separator ratio -- and runs all the
// table entries of one tree layer as one parallel task (Section 2).  Here a
// layer is one launch over packed workgroup tiles x evidence slots:
//
//   collect layer (cliques of height h, leaves first)
//     psi[i] = prior[i] * [evidence agrees at i] * prod_children R_f[map_f(i)]
//     (reduction + extension by the children's messages), psi is stored,
//     and its contiguous parent-separator segments are summed
//     (marginalisation; the parent separator's variables lead the layout).
//   collect finalise: message max -> exact power-of-two rescale; exponent
//     kept for log P(e).
//   distribute layer (cliques of depth d, root first)
//     phi*[i] = psi[i] * Rd_parent[pmap(i)]  (extension by new/old ratio),
//     gathered onto every child separator (marginalisation onto a
//     non-contiguous index set): whole rows of the clique are staged in LDS
//     and each separator entry is summed by fixed lanes in a fixed order.
//   distribute finalise: posterior marginals from the calibrated separator;
//     Rd = S_new / S_old (0/0 = 0), rescaled.
//
// A workgroup carries B evidence slots (cases) of the same tile: index
// maps, packed digits and prior values are computed once per entry and
// reused for every slot, and the per-slot gathers are independent loads in
// flight together.  Tables stream through HBM in coalesced runs of
// consecutive entries; index maps come from small factored tables
// (H[hi] + L[lo]) that stay in cache; separator sums are accumulated in
// float64 and stored in table precision, scale factors are exact powers of
// two.  No atomics on data, so a case gives bitwise the same result
// alone or in any batch.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace fbn {
namespace {

constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;
constexpr int kMaxKids = 8;  // child maps held in registers; more use a loop
// loads kept in flight per thread: collect entries x slots x children, the
// distribute stage's entries, and the summed entries per lane of an output
constexpr int kCollectLoads = 32;
constexpr int kCollectMaxU = 4;
constexpr uint32_t kStageEntries = 8;
constexpr uint32_t kOutEntries = 4;

__device__ __forceinline__ uint32_t mdiv(uint32_t n, uint32_t mul, uint32_t sh) {
    return (uint32_t)(((uint64_t)__umulhi(n, mul) + n) >> sh);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// XCD-aware placement of a layer's workgroups.  The hardware hands
// consecutive workgroup ids to the chip's eight XCDs in turn, and each XCD
// has its own L2.  A layer launch is (work item x slot group) flattened to
// one dimension; workgroup w runs on XCD w % 8 as that XCD's (w / 8)-th, and
// is given the pair at position start(XCD) + w / 8 of the slot-group-major
// order, so that each XCD walks a contiguous range of slot groups and the
// workgroups resident on one XCD gather from the separators of only a few
// slots at a time.
constexpr uint32_t kXcds = 8;

struct Cell {
    uint32_t item, group;  // work item, slot group
};

__device__ __forceinline__ Cell xcd_cell(uint32_t nitems, uint32_t ngroups) {
    const uint32_t total = nitems * ngroups;
    const uint32_t w = blockIdx.x;
    const uint32_t x = w % kXcds, k = w / kXcds;
    const uint32_t base = total / kXcds, extra = total % kXcds;
    const uint32_t idx = x * base + min(x, extra) + k;
    return Cell{idx % nitems, idx / nitems};
}

// Block-wide sum; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) scratch[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kWaves; k++) s += scratch[k];
    return s;
}

// ------------------------------------------------------------------ collect

// What a collect workgroup needs about one of its runs, copied to LDS once.
struct RunC {
    uint64_t off;        // arena offset of the run's clique
    uint32_t begin, count, gofs;
    uint32_t L, Lmul, Lsh, hdig, ldig;
    uint32_t seg, out0;  // segment length; separator entry of the run's first segment
    uint32_t nchild, child0;
    uint32_t seg0;       // segments of the tile before this run
    uint32_t psi;        // the clique's working-table offset
};

struct KidC {
    uint32_t sep, mh, ml;
};

// One table entry of a collect tile for every slot of the workgroup, with
// NC child messages whose loads are issued together (NC == kMaxKids:
// further children, if any, read one by one).
template <typename T, int B>
struct EntryC {
    uint32_t hi, lo;
    T prior;
    uint64_t dig, toff;
    uint32_t gi, child0, nchild;
    uint32_t need;  // bit b: slot b reads and writes this entry
};

// Slots of the workgroup that must touch an entry with packed digits d:
// every slot in the batch when tables are streamed whole (SKIP false), else
// only those whose evidence agrees at d (an entry the evidence zeroes is
// neither read nor written: it contributes an exact zero to every sum).
template <int B, bool SKIP>
__device__ __forceinline__ uint32_t need_mask(uint64_t d, const DEvidence (&ev)[B], uint32_t valid) {
    if (!SKIP) return valid;
    uint32_t m = 0;
#pragma unroll
    for (int b = 0; b < B; b++) m |= ((d ^ ev[b].want) & ev[b].mask) ? 0u : (1u << b);
    return m & valid;
}

template <typename T, int B, int NC, int U, bool SKIP>
__device__ __forceinline__ void collect_entries(const Ctx& c, const EntryC<T, B> (&e)[U], uint32_t nvalid,
                                                const DEvidence (&ev)[B], const int (&sl)[B],
                                                const uint32_t (&ksep)[kMaxKids], const uint32_t (&kmh)[kMaxKids],
                                                const uint32_t (&kml)[kMaxKids], T* const (&psi_b)[B],
                                                const T* const (&sepc_b)[B], T* vals) {
    constexpr int NW = NC > 0 ? NC : 1;
    const uint32_t* __restrict__ map = c.map;
    uint32_t jk[U][NW];
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
        for (int k = 0; k < NC; k++) jk[u][k] = ksep[k] + map[kmh[k] + e[u].hi] + map[kml[k] + e[u].lo];
    T w[U][B][NW];
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
        for (int b = 0; b < B; b++)
#pragma unroll
            for (int k = 0; k < NC; k++) {
                if (!SKIP || ((e[u].need >> b) & 1u)) w[u][b][k] = sepc_b[b][jk[u][k]];
                else w[u][b][k] = T(0);
            }
#pragma unroll
    for (int u = 0; u < U; u++) {
        if ((uint32_t)u >= nvalid) break;
#pragma unroll
        for (int b = 0; b < B; b++) {
            if (sl[b] < 0) continue;
            T v = T(0);
            if (!SKIP || ((e[u].need >> b) & 1u)) {
                v = ((e[u].dig ^ ev[b].want) & ev[b].mask) ? T(0) : e[u].prior;
#pragma unroll
                for (int k = 0; k < NC; k++) v *= w[u][b][k];
                if (NC == kMaxKids) {
                    for (uint32_t k = kMaxKids; k < e[u].nchild; k++) {
                        const DChild ch = c.ch[e[u].child0 + k];
                        v *= sepc_b[b][ch.sep + map[ch.mh + e[u].hi] + map[ch.ml + e[u].lo]];
                    }
                }
                psi_b[b][e[u].toff] = v;
            }
            vals[b * c.tile + e[u].gi] = v;
        }
    }
}

// A group that is one run of one clique: U entries per thread at a time
// (as many as keep U x B x children loads in registers), their lookups and
// loads issued together.
template <typename T, int B, int NC, bool SKIP>
__device__ __forceinline__ void collect_run(const Ctx& c, uint32_t total, uint32_t r_base, uint32_t L, uint32_t Lmul,
                                            uint32_t Lsh, uint32_t hdig, uint32_t ldig, bool anyev, uint32_t valid,
                                            const T* r_prior, uint32_t psi0, uint32_t child0, uint32_t nk,
                                            const DEvidence (&ev)[B], const int (&sl)[B],
                                            const uint32_t (&ksep)[kMaxKids], const uint32_t (&kmh)[kMaxKids],
                                            const uint32_t (&kml)[kMaxKids], T* const (&psi_b)[B],
                                            const T* const (&sepc_b)[B], T* vals) {
    constexpr int NW = NC > 0 ? NC : 1;
    constexpr int U0 = kCollectLoads / (B * NW);
    constexpr int U = U0 >= kCollectMaxU ? kCollectMaxU : (U0 >= 2 ? 2 : 1);
    for (uint32_t g0 = threadIdx.x; g0 < total; g0 += U * kBlock) {
        EntryC<T, B> e[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint32_t gi = min(g0 + (uint32_t)u * kBlock, total - 1);
            const uint32_t i = gi + r_base;
            e[u].hi = mdiv(i, Lmul, Lsh);
            e[u].lo = i - e[u].hi * L;
            e[u].dig = anyev ? (c.dig[hdig + e[u].hi] | c.dig[ldig + e[u].lo]) : 0;
            e[u].need = need_mask<B, SKIP>(e[u].dig, ev, valid);
            e[u].prior = r_prior[i];
            e[u].toff = (uint64_t)psi0 + i;
            e[u].gi = gi;
            e[u].child0 = child0;
            e[u].nchild = nk;
        }
        const uint32_t nvalid = min((uint32_t)U, (total - g0 + kBlock - 1) / kBlock);
        collect_entries<T, B, NC, U, SKIP>(c, e, nvalid, ev, sl, ksep, kmh, kml, psi_b, sepc_b, vals);
    }
}

template <typename T, int B, bool SKIP>
__global__ __launch_bounds__(kBlock) void k_collect(Ctx c, const DGroup* __restrict__ groups, uint32_t ngroups,
                                                    const int32_t* __restrict__ slots, int nslots) {
    extern __shared__ __align__(16) unsigned char stage[];  // B * c.tile entries, sized at launch
    __shared__ RunC runs[kMaxPieces];
    __shared__ KidC kids[kMaxPieces][kMaxKids];
    __shared__ DEvidence evs[kMaxPieces][B];
    __shared__ uint32_t nseg_total;
    __shared__ double red[kWaves];
    T* vals = reinterpret_cast<T*>(stage);
    const Cell cell = xcd_cell(ngroups, ((uint32_t)nslots + B - 1) / B);
    const DGroup g = groups[cell.item];
    int sl[B];
    uint32_t valid = 0;
#pragma unroll
    for (int b = 0; b < B; b++) {
        const int k = (int)cell.group * B + b;
        sl[b] = k < nslots ? slots[k] : -1;
        valid |= (sl[b] >= 0 ? 1u : 0u) << b;
    }
    // ---- run metadata into LDS
    if (threadIdx.x < g.npiece) {
        const DPiece pc = c.pc[g.piece0 + threadIdx.x];
        const DClique q = c.cl[pc.clique];
        RunC r;
        r.off = q.off;
        r.begin = pc.begin;
        r.count = pc.count;
        r.gofs = pc.gofs;
        r.L = q.L;
        r.Lmul = q.Lmul;
        r.Lsh = q.Lsh;
        r.hdig = q.hdig;
        r.ldig = q.ldig;
        r.seg = q.seg;
        r.out0 = q.psep + pc.begin / q.seg;
        r.nchild = q.nchild;
        r.child0 = q.child0;
        r.seg0 = 0;
        r.psi = q.psi;
        runs[threadIdx.x] = r;
#pragma unroll
        for (int b = 0; b < B; b++)
            evs[threadIdx.x][b] = sl[b] >= 0 ? c.ev[(uint64_t)sl[b] * c.ev_stride + pc.clique] : DEvidence{0, 0};
        for (uint32_t k = 0; k < q.nchild && k < (uint32_t)kMaxKids; k++) {
            const DChild ch = c.ch[q.child0 + k];
            kids[threadIdx.x][k] = KidC{ch.sep, ch.mh, ch.ml};
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (uint32_t r = 0; r < g.npiece; r++) {
            runs[r].seg0 = s;
            s += runs[r].count / runs[r].seg;
        }
        nseg_total = s;
    }

    // ---- psi = prior x evidence x children's messages, per slot
    const T* __restrict__ prior = static_cast<const T*>(c.prior);
    const uint32_t* __restrict__ map = c.map;
    T* psi_b[B];
    const T* sepc_b[B];
#pragma unroll
    for (int b = 0; b < B; b++) {
        const uint64_t s = sl[b] >= 0 ? (uint64_t)sl[b] : 0;
        psi_b[b] = static_cast<T*>(c.psi) + s * c.psi_stride;
        sepc_b[b] = static_cast<const T*>(c.sepc) + s * c.sep_stride;
    }
    // the current run's fields, reloaded from LDS only when the run changes
    uint32_t p = 0, r_end = 0, r_base = 0, r_L = 1, r_Lmul = 0, r_Lsh = 0, r_hdig = 0, r_ldig = 0, nk = 0;
    const T* r_prior = prior;
    uint32_t kmh[kMaxKids], kml[kMaxKids], ksep[kMaxKids];
    DEvidence ev[B];
    uint64_t anyev = 0;
    bool first = true;
    if (g.npiece == 1) {
        // one run: its fields once, several entries per thread at a time
        const RunC& r = runs[0];
#pragma unroll
        for (int k = 0; k < kMaxKids; k++)
            if (k < (int)r.nchild) {
                ksep[k] = kids[0][k].sep;
                kmh[k] = kids[0][k].mh;
                kml[k] = kids[0][k].ml;
            }
#pragma unroll
        for (int b = 0; b < B; b++) {
            ev[b] = evs[0][b];
            anyev |= ev[b].mask;
        }
        const uint32_t rb = r.begin - r.gofs;
        const T* rp = prior + r.off;
        switch (r.nchild) {
#define FBN_RUN(NC)                                                                                                   \
    collect_run<T, B, NC, SKIP>(c, g.total, rb, r.L, r.Lmul, r.Lsh, r.hdig, r.ldig, anyev != 0, valid, rp, r.psi, r.child0, \
                          r.nchild, ev, sl, ksep, kmh, kml, psi_b, sepc_b, vals)
        case 0: FBN_RUN(0); break;
        case 1: FBN_RUN(1); break;
        case 2: FBN_RUN(2); break;
        case 3: FBN_RUN(3); break;
        case 4: FBN_RUN(4); break;
        case 5: FBN_RUN(5); break;
        case 6: FBN_RUN(6); break;
        case 7: FBN_RUN(7); break;
        default: FBN_RUN(kMaxKids); break;
#undef FBN_RUN
        }
    } else {
        for (uint32_t gi = threadIdx.x; gi < g.total; gi += kBlock) {
            if (first || gi >= r_end) {
                if (!first) p++;
                while (gi >= runs[p].gofs + runs[p].count) p++;
                first = false;
                const RunC& r = runs[p];
                r_end = r.gofs + r.count;
                r_base = r.begin - r.gofs;     // entry = gi + r_base
                r_L = r.L;
                r_Lmul = r.Lmul;
                r_Lsh = r.Lsh;
                r_hdig = r.hdig;
                r_ldig = r.ldig;
                nk = r.nchild;
                r_prior = prior + r.off;
    #pragma unroll
                for (int k = 0; k < kMaxKids; k++)
                    if (k < (int)nk) {
                        ksep[k] = kids[p][k].sep;
                        kmh[k] = kids[p][k].mh;
                        kml[k] = kids[p][k].ml;
                    }
                anyev = 0;
    #pragma unroll
                for (int b = 0; b < B; b++) {
                    ev[b] = evs[p][b];
                    anyev |= ev[b].mask;
                }
            }
            const uint32_t i = gi + r_base;
            const uint32_t hi = mdiv(i, r_Lmul, r_Lsh);
            const uint32_t lo = i - hi * r_L;
            const uint64_t d = anyev ? (c.dig[r_hdig + hi] | c.dig[r_ldig + lo]) : 0;
            const uint32_t need = need_mask<B, SKIP>(d, ev, valid);
            const T pv = r_prior[i];
            const uint64_t toff = (uint64_t)runs[p].psi + i;
            const EntryC<T, B> e[1] = {{hi, lo, pv, d, toff, gi, runs[p].child0, nk, need}};
            switch (nk) {
            case 0: collect_entries<T, B, 0, 1, SKIP>(c, e, 1u, ev, sl, ksep, kmh, kml, psi_b, sepc_b, vals); break;
            case 1: collect_entries<T, B, 1, 1, SKIP>(c, e, 1u, ev, sl, ksep, kmh, kml, psi_b, sepc_b, vals); break;
            case 2: collect_entries<T, B, 2, 1, SKIP>(c, e, 1u, ev, sl, ksep, kmh, kml, psi_b, sepc_b, vals); break;
            case 3: collect_entries<T, B, 3, 1, SKIP>(c, e, 1u, ev, sl, ksep, kmh, kml, psi_b, sepc_b, vals); break;
            case 4: collect_entries<T, B, 4, 1, SKIP>(c, e, 1u, ev, sl, ksep, kmh, kml, psi_b, sepc_b, vals); break;
            case 5: collect_entries<T, B, 5, 1, SKIP>(c, e, 1u, ev, sl, ksep, kmh, kml, psi_b, sepc_b, vals); break;
            case 6: collect_entries<T, B, 6, 1, SKIP>(c, e, 1u, ev, sl, ksep, kmh, kml, psi_b, sepc_b, vals); break;
            case 7: collect_entries<T, B, 7, 1, SKIP>(c, e, 1u, ev, sl, ksep, kmh, kml, psi_b, sepc_b, vals); break;
            default: collect_entries<T, B, kMaxKids, 1, SKIP>(c, e, 1u, ev, sl, ksep, kmh, kml, psi_b, sepc_b, vals); break;
            }
        }
    }
    __syncthreads();

    // ---- marginalise onto the parent separators: every segment of the tile
    // at once, tps lanes per segment, all slots together
    if (g.part >= 0) {
#pragma unroll
        for (int b = 0; b < B; b++) {
            if (sl[b] < 0) continue;
            double s = 0.0;
            for (uint32_t k = threadIdx.x; k < g.total; k += kBlock) s += (double)vals[b * c.tile + k];
            s = block_sum(s, red);
            if (threadIdx.x == 0) static_cast<T*>(c.part)[(uint64_t)sl[b] * c.part_stride + (uint32_t)g.part] = (T)s;
        }
        return;
    }
    const uint32_t ns = nseg_total;
    uint32_t tps = 1;
    while (tps < 64 && tps * 2 * ns <= (uint32_t)kBlock) tps *= 2;
    const uint32_t sub = threadIdx.x & (tps - 1);
    uint32_t q = 0;
    for (uint32_t base = 0; base < ns * tps; base += kBlock) {
        const uint32_t sidx = (base + threadIdx.x) / tps;
        double a[B];
#pragma unroll
        for (int b = 0; b < B; b++) a[b] = 0.0;
        uint32_t out = 0;
        if (sidx < ns) {
            while (q + 1 < g.npiece && sidx >= runs[q + 1].seg0) q++;
            const uint32_t seg = runs[q].seg;
            const uint32_t s = sidx - runs[q].seg0;
            const uint32_t e0 = runs[q].gofs + s * seg;
            out = runs[q].out0 + s;
            for (uint32_t k = sub; k < seg; k += tps) {
#pragma unroll
                for (int b = 0; b < B; b++) a[b] += (double)vals[b * c.tile + e0 + k];
            }
        }
#pragma unroll
        for (int b = 0; b < B; b++)
            for (uint32_t o = tps / 2; o > 0; o >>= 1) a[b] += __shfl_xor(a[b], (int)o, kWave);
        if (sidx < ns && sub == 0) {
#pragma unroll
            for (int b = 0; b < B; b++)
                if (sl[b] >= 0) {
                    static_cast<T*>(c.acc)[(uint64_t)sl[b] * c.sep_stride + out] = (T)a[b];
                    // a root's sum (its tree's share of P(e)) also kept unrounded
                    if (out >= c.sep_total) c.rsum[(uint64_t)sl[b] * c.nroots + (out - c.sep_total)] = a[b];
                }
        }
    }
}

// A separator finaliser runs as a team: a whole workgroup for a large
// separator (the first nbig of a layer), one wave for a small one.
struct Team {
    uint32_t lane, size;
    bool block;
    double* red;
    __device__ double sum(double v) const { return block ? block_sum(v, red) : wave_sum(v); }
    __device__ double max(double v) const { return block ? block_max(v) : wave_max(v); }
    __device__ double block_max(double v) const {
        v = wave_max(v);
        const int l = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
        __syncthreads();
        if (l == 0) red[w] = v;
        __syncthreads();
        double s = red[0];
        for (int k = 1; k < kWaves; k++) s = fmax(s, red[k]);
        return s;
    }
    // make this team's global writes visible to the whole team
    __device__ void sync() const {
        if (block) __syncthreads();
        else __threadfence_block();
    }
};

__device__ __forceinline__ bool team_of(uint32_t bx, uint32_t nbig, uint32_t nfins, double* red, Team& t,
                                        uint32_t& fi) {
    if (bx < nbig) {
        fi = bx;
        t = Team{threadIdx.x, (uint32_t)kBlock, true, red};
        return true;
    }
    fi = nbig + (bx - nbig) * kWaves + threadIdx.x / kWave;
    t = Team{threadIdx.x & (kWave - 1), (uint32_t)kWave, false, red};
    return fi < nfins;
}

// Finish the entries [b, e) of separator f (acc and part offset to the
// separator; partials chunk-major, chunk k of entry m at k * size + m): an
// entry whose sum was split over chunks gets its partials added by tpe lanes
// of one wave (a power of two, about four partials per lane), combined by a
// fixed xor-shuffle tree, and stored; fn(m, v) is then
// called once per entry, v its finished value.  t is the thread's index in
// its team of nt threads (a wave or a workgroup); every thread of the team
// must make the call.
template <typename T, typename F>
__device__ __forceinline__ void finish_range(const DSepFin& f, T* acc, const T* part, uint32_t b, uint32_t e,
                                             uint32_t t, uint32_t nt, F fn) {
    if (!f.nchunk) {
        // four entries per thread at a time, their loads issued together
        for (uint32_t m0 = b + t; m0 < e; m0 += 4 * nt) {
            T x[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; u++) x[u] = acc[min(m0 + u * nt, e - 1)];
#pragma unroll
            for (uint32_t u = 0; u < 4; u++)
                if (m0 + u * nt < e) fn(m0 + u * nt, (double)x[u]);
        }
        return;
    }
    // partials are chunk-major (chunk k of entry m at k * size + m): a wave
    // takes epw consecutive entries with an entry's tpe lanes epw apart, so
    // every load reads runs of epw consecutive partials.  tpe gives each lane
    // about four partials, more when the separator has fewer than 64 / tpe
    // entries; the split depends on the separator alone, so an entry's sum
    // has one order however the separator is cut into blocks
    uint32_t tpe = 1;
    while (tpe < (uint32_t)kWave && tpe * 4 < f.nchunk) tpe *= 2;
    uint32_t epw = (uint32_t)kWave / tpe;
    while (epw > 1 && epw / 2 >= f.size) epw /= 2;
    tpe = (uint32_t)kWave / epw;
    const uint32_t lane = t & (kWave - 1), wv = t / kWave, nw = nt / kWave;
    const uint32_t sub = lane / epw, eo = lane & (epw - 1);
    for (uint32_t m0 = b + wv * epw; m0 < e; m0 += nw * epw) {
        const uint32_t m = m0 + eo;
        double v = 0.0;
        if (m < e) {
#pragma unroll 4
            for (uint32_t k = sub; k < f.nchunk; k += tpe) v += part[(uint64_t)k * f.size + m];
        }
        for (uint32_t o = tpe / 2; o > 0; o >>= 1) v += __shfl_xor(v, (int)(o * epw), kWave);
        if (m < e && sub == 0) {
            acc[m] = (T)v;
            fn(m, v);
        }
    }
}

// Entries m < n of a separator whose digit of a variable (stride, card) is x:
// whole periods of stride * card entries hold stride each.
__device__ __forceinline__ uint32_t digit_below(uint32_t n, uint32_t stride, uint32_t card, uint32_t x) {
    const uint32_t span = stride * card;
    const uint32_t r = n % span;
    const uint32_t lo = x * stride;
    return (n / span) * stride + (r > lo ? min(r - lo, stride) : 0u);
}

// Posterior shares of the entries [b, e) of separator f: for every state x
// of every variable it carries (mw pairs in all, taken in variable order),
// the sum of get(m) over the entries m with digit x.  Each pair gets tpp
// lanes of one wave (a power of two, as many as the team allows), whose
// sums are combined by a fixed xor-shuffle tree; put(pair, variable, x,
// sum) is called once per pair.  t is the thread's index in its team of nt
// threads; every thread of the team must make the call.
template <typename Get, typename Put>
__device__ __forceinline__ void shares_grouped(const DSepFin& f, const Ctx& c, uint32_t b, uint32_t e, uint32_t mw,
                                               uint32_t t, uint32_t nt, Get get, Put put) {
    uint32_t tpp = 1;
    while (tpp < (uint32_t)kWave && tpp * 2 * mw <= nt) tpp *= 2;
    const uint32_t sub = t & (tpp - 1);
    for (uint32_t base = 0; base < mw * tpp; base += nt) {
        const uint32_t pidx = (base + t) / tpp;
        double s = 0.0;
        DMargVar mv{};
        uint32_t x = 0;
        if (pidx < mw) {
            uint32_t vo = 0, a = 0;
            mv = c.mv[f.mv0];
            while (pidx >= vo + mv.card) {
                vo += mv.card;
                mv = c.mv[f.mv0 + ++a];
            }
            x = pidx - vo;
            const uint32_t e0 = digit_below(b, mv.stride, mv.card, x);
            const uint32_t e1 = digit_below(e, mv.stride, mv.card, x);
            for (uint32_t k = e0 + sub; k < e1; k += tpp) {
                const uint32_t o = mdiv(k, mv.smul, mv.ssh);
                s += get((o * mv.card + x) * mv.stride + (k - o * mv.stride));
            }
        }
        for (uint32_t o2 = tpp / 2; o2 > 0; o2 >>= 1) s += __shfl_xor(s, (int)o2, kWave);
        if (pidx < mw && sub == 0) put(pidx, mv, x, s);
    }
}

// After a collect layer, per separator: finish the message (sum partial
// sums where a segment spanned several tiles), rescale it by an exact power
// of two so its largest entry lies in [0.5, 1), store it in table precision
// and record the exponent.  A root's one-entry virtual separator holds its
// tree's share of P(e); zero there means the evidence is impossible.
template <typename T>
__device__ __forceinline__ void fin_collect_team(const Ctx& c, const DSepFin* __restrict__ fins, uint32_t nfins,
                                                 uint32_t nbig, const int32_t* __restrict__ slots, uint32_t bx) {
    __shared__ double red[kWaves];
    Team tm;
    uint32_t fi;
    if (!team_of(bx, nbig, nfins, red, tm, fi)) return;
    const uint32_t lane = tm.lane;
    const DSepFin f = fins[fi];
    const int slot = slots[blockIdx.y];
    T* __restrict__ acc = static_cast<T*>(c.acc) + (uint64_t)slot * c.sep_stride;
    const T* __restrict__ part = static_cast<const T*>(c.part) + (uint64_t)slot * c.part_stride;
    int32_t* kexp = c.kexp + (uint64_t)slot * c.kexp_stride;

    double mx = 0.0;
    finish_range(f, acc + f.sep, part + f.part0, 0u, f.size, lane, tm.size, [&](uint32_t, double v) {
        mx = fmax(mx, v);
        if (f.edge < 0) c.rsum[(uint64_t)slot * c.nroots + (f.sep - c.sep_total)] = v;
    });
    if (f.nchunk) tm.sync();  // other lanes rescale these sums below
    mx = tm.max(mx);

    if (f.edge < 0) {
        if (lane == 0 && !(acc[f.sep] > 0.0)) atomicOr(&c.flags[slot], c.fp32 ? 2 : 1);
        return;
    }
    int k = 0;
    if (mx > 0.0) frexp(mx, &k);
    else if (lane == 0) atomicOr(&c.flags[slot], c.fp32 ? 2 : 1);
    const double scale = ldexp(1.0, -k);
    T* __restrict__ sepc = static_cast<T*>(c.sepc) + (uint64_t)slot * c.sep_stride;
#pragma unroll 4
    for (uint32_t m = lane; m < f.size; m += tm.size) sepc[f.sep + m] = (T)(acc[f.sep + m] * scale);
    if (lane == 0) kexp[f.edge] = k;
}

// --------------------------------------------------------------- distribute

// One workgroup marginalises clique entries onto target separators, for B
// slots at once.
//   Large clique: ng groups x nk rows of one target (each row L consecutive
//   entries, read coalesced and extended by the parent's distribute ratio
//   on the way in) are staged in LDS; every separator entry of the block is
//   summed by a fixed set of lanes in a fixed order.
//   Packed small cliques: each whole clique is staged once, and all of its
//   targets are summed from LDS.
// What a packed distribute workgroup needs about one of its runs (a whole
// small clique) and about each of its targets, copied to LDS once.
struct RunD {
    uint64_t off;
    uint32_t count, gofs;
    uint32_t L, Lmul, Lsh;
    int32_t pedge;
    uint32_t psep, segmul, segsh, psi;  // parent separator entry = psep + entry / seg; psi: working-table offset
    uint32_t hdig, ldig;           // packed-digit tables (evidence test)
};

struct TgtD {
    DTarget t;
    uint32_t out0, gofs, L, pad;
};

template <typename T, int B, bool SKIP>
__global__ __launch_bounds__(kBlock) void k_dist_gather(Ctx c, const DWork* __restrict__ works, uint32_t nworks,
                                                        const int32_t* __restrict__ slots, int nslots) {
    extern __shared__ __align__(16) unsigned char stage[];  // B * c.tile entries, sized at launch
    __shared__ RunD runs[kMaxPieces];
    __shared__ TgtD tgts[kMaxPieces];
    __shared__ DEvidence evs[SKIP ? kMaxPieces : 1][B];
    T* vals = reinterpret_cast<T*>(stage);
    const Cell cell = xcd_cell(nworks, ((uint32_t)nslots + B - 1) / B);
    const DWork w = works[cell.item];
    int sl[B];
    uint32_t valid = 0;
#pragma unroll
    for (int b = 0; b < B; b++) {
        const int k = (int)cell.group * B + b;
        sl[b] = k < nslots ? slots[k] : -1;
        valid |= (sl[b] >= 0 ? 1u : 0u) << b;
    }
    const uint32_t* __restrict__ map = c.map;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const bool packed = w.npiece > 0;

    // ---- stage: phi* = psi * parent ratio, for every slot
    DTarget tg{};
    DClique q{};
    uint32_t n;
    if (packed) {
        if (threadIdx.x < w.npiece) {
            const DPiece pc = c.pc[w.piece0 + threadIdx.x];
            const DClique cq = c.cl[pc.clique];
            runs[threadIdx.x] = RunD{cq.off, pc.count, pc.gofs, cq.L, cq.Lmul, cq.Lsh, cq.pedge, cq.psep, cq.segmul,
                                     cq.segsh, cq.psi, cq.hdig, cq.ldig};
            if (SKIP) {
#pragma unroll
                for (int b = 0; b < B; b++)
                    evs[threadIdx.x][b] = sl[b] >= 0 ? c.ev[(uint64_t)sl[b] * c.ev_stride + pc.clique]
                                                     : DEvidence{0, 0};
            }
        }
        if (threadIdx.x >= 64 && threadIdx.x - 64 < w.nwt) {
            const uint32_t k = threadIdx.x - 64;
            const DWTarget wt = c.wt[w.wt0 + k];
            const DPiece pc = c.pc[w.piece0 + wt.piece];
            tgts[k] = TgtD{c.tg[wt.target], wt.out0, pc.gofs, c.cl[pc.clique].L, 0u};
        }
        __syncthreads();
        n = w.total;
    } else {
        tg = c.tg[w.target];
        q = c.cl[tg.clique];
        n = w.ng * w.nk * q.L;
    }
    const T* psi_b[B];
    const T* sepd_b[B];
#pragma unroll
    for (int b = 0; b < B; b++) {
        const uint64_t s = sl[b] >= 0 ? (uint64_t)sl[b] : 0;
        psi_b[b] = static_cast<const T*>(c.psi) + s * c.psi_stride;
        sepd_b[b] = static_cast<const T*>(c.sepd) + s * c.sep_stride;
    }
    if (!packed) {
        // four entries per thread at a time, their map lookups and every
        // slot's psi and ratio loads issued together; a slot whose evidence
        // zeroes an entry reads nothing for it (its psi there was never
        // written), unless tables are streamed whole
        constexpr uint32_t U = kStageEntries;
        const bool ratio = q.pedge >= 0;
        DEvidence ev[B];
        uint64_t anyev = 0;
#pragma unroll
        for (int b = 0; b < B; b++) {
            ev[b] = SKIP && sl[b] >= 0 ? c.ev[(uint64_t)sl[b] * c.ev_stride + tg.clique] : DEvidence{0, 0};
            anyev |= ev[b].mask;
        }
        const bool test = SKIP && anyev;
        for (uint32_t g0 = threadIdx.x; g0 < n; g0 += U * kBlock) {
            uint32_t ent[U], row[U], lo[U], pr[U];
#pragma unroll
            for (uint32_t u = 0; u < U; u++) {
                const uint32_t gi = min(g0 + u * kBlock, n - 1);
                const uint32_t ri = mdiv(gi, q.Lmul, q.Lsh);
                lo[u] = gi - ri * q.L;
                const uint32_t gg = mdiv(ri, w.nkmul, w.nksh);
                const uint32_t k = ri - gg * w.nk;
                row[u] = map[tg.rg + w.g0 + gg] + map[tg.rq + w.k0 + k];
                ent[u] = row[u] * q.L + lo[u];
                pr[u] = 0u;
            }
            if (ratio) {
#pragma unroll
                for (uint32_t u = 0; u < U; u++) pr[u] = q.psep + mdiv(ent[u], q.segmul, q.segsh);
            }
            uint32_t nd[U];
#pragma unroll
            for (uint32_t u = 0; u < U; u++)
                nd[u] = need_mask<B, SKIP>(test ? (c.dig[q.hdig + row[u]] | c.dig[q.ldig + lo[u]]) : 0, ev, valid);
            T v[U][B], r[U][B];
#pragma unroll
            for (uint32_t u = 0; u < U; u++)
#pragma unroll
                for (int b = 0; b < B; b++) {
                    if (!SKIP || ((nd[u] >> b) & 1u)) {
                        v[u][b] = psi_b[b][(uint64_t)q.psi + ent[u]];
                        r[u][b] = sepd_b[b][pr[u]];
                    } else {
                        v[u][b] = T(0);
                        r[u][b] = T(0);
                    }
                }
#pragma unroll
            for (uint32_t u = 0; u < U; u++) {
                const uint32_t gi = g0 + u * kBlock;
                if (gi >= n) continue;
#pragma unroll
                for (int b = 0; b < B; b++)
                    if (sl[b] >= 0) vals[b * c.tile + gi] = ratio ? v[u][b] * r[u][b] : v[u][b];
            }
        }
    } else {
        // packed: the current run's fields, reloaded only when the run changes
        uint32_t p = 0, r_end = 0, r_gofs = 0, r_L = 1, r_Lmul = 0, r_Lsh = 0, r_psep = 0, r_segmul = 0, r_segsh = 0;
        uint32_t r_psi = 0, r_hdig = 0, r_ldig = 0;
        int32_t r_pedge = -1;
        bool first = true, test = false;
        DEvidence ev[B];
        for (uint32_t gi = threadIdx.x; gi < n; gi += kBlock) {
            if (first || gi >= r_end) {
                if (!first) p++;
                while (gi >= runs[p].gofs + runs[p].count) p++;
                first = false;
                const RunD& rr = runs[p];
                r_end = rr.gofs + rr.count;
                r_gofs = rr.gofs;
                r_L = rr.L;
                r_Lmul = rr.Lmul;
                r_Lsh = rr.Lsh;
                r_pedge = rr.pedge;
                r_psep = rr.psep;
                r_segmul = rr.segmul;
                r_segsh = rr.segsh;
                r_psi = rr.psi;
                r_hdig = rr.hdig;
                r_ldig = rr.ldig;
                uint64_t anyev = 0;
#pragma unroll
                for (int b = 0; b < B; b++) {
                    ev[b] = SKIP ? evs[p][b] : DEvidence{0, 0};
                    anyev |= ev[b].mask;
                }
                test = SKIP && anyev;
            }
            const uint32_t ent = gi - r_gofs;
            const uint32_t row = mdiv(ent, r_Lmul, r_Lsh);
            const uint32_t l = ent - row * r_L;
            const uint32_t pr = r_pedge >= 0 ? r_psep + mdiv(ent, r_segmul, r_segsh) : 0u;
            const uint32_t nd = need_mask<B, SKIP>(test ? (c.dig[r_hdig + row] | c.dig[r_ldig + l]) : 0, ev, valid);
            // every needed slot's loads issued together (a root clique reads
            // ratio entry 0, unused)
            T v[B], r[B];
#pragma unroll
            for (int b = 0; b < B; b++) {
                if (!SKIP || ((nd >> b) & 1u)) {
                    v[b] = psi_b[b][(uint64_t)r_psi + ent];
                    r[b] = sepd_b[b][pr];
                } else {
                    v[b] = T(0);
                    r[b] = T(0);
                }
            }
#pragma unroll
            for (int b = 0; b < B; b++)
                if (sl[b] >= 0) vals[b * c.tile + gi] = r_pedge >= 0 ? v[b] * r[b] : v[b];
        }
    }
    __syncthreads();

    // ---- outputs: tpo lanes per separator entry, B sums each
    const uint32_t nout = packed ? w.nout : w.ng * tg.nPL;
    uint32_t tpo = 1;
    while (tpo < 64 && tpo * 2 * nout <= (uint32_t)kBlock) tpo *= 2;
    const uint32_t sub = lane & (tpo - 1);
    uint32_t a = 0;
    for (uint32_t base = 0; base < nout * tpo; base += kBlock) {
        const uint32_t o = (base + threadIdx.x) / tpo;
        double s[B];
#pragma unroll
        for (int b = 0; b < B; b++) s[b] = 0.0;
        uint32_t m = 0, sep = 0, gofs = 0;
        int32_t part0 = -1;
        uint32_t tsz = 0;  // target size: chunk-major partials
        if (o < nout) {
            DTarget t2 = tg;
            uint32_t L = q.L, g, t, nk, rowbase;
            if (packed) {
                while (a + 1 < w.nwt && o >= tgts[a + 1].out0) a++;
                t2 = tgts[a].t;
                L = tgts[a].L;
                gofs = tgts[a].gofs;
                const uint32_t oo = o - tgts[a].out0;
                g = oo / t2.nPL;
                t = oo - g * t2.nPL;
                nk = t2.NQ;
                rowbase = 0;
                m = map[t2.tb + g] + map[t2.tv + t];
            } else {
                g = o / t2.nPL;
                t = o - g * t2.nPL;
                nk = w.nk;
                rowbase = g * w.nk;
                m = map[t2.tb + w.g0 + g] + map[t2.tv + t];
            }
            const uint32_t lp = map[t2.lp + t];
            const uint32_t nQL = t2.nQL;
            // The output's entries are rows k < nk by low offsets u < nQL.  With
            // at least tpo offsets, lane sub takes offsets sub, sub + tpo, ...
            // over every row; with fewer, lane sub takes offset sub % nQL and
            // rows sub / nQL, + q, ... (q = tpo / nQL; lanes past q * nQL idle).
            // Each offset's index is loaded once and the rows are stepped by
            // adding L, kOutEntries rows at a time.
            uint32_t u0 = sub, ustep = tpo, k0 = 0, kstep = 1;
            if (nQL < tpo) {
                const uint32_t qq = tpo / nQL;
                u0 = sub % nQL;
                ustep = nQL;
                k0 = sub < qq * nQL ? sub / nQL : nk;
                kstep = qq;
            }
            const uint32_t rg = packed ? map[t2.rg + g] : 0u;
            for (uint32_t u = u0; u < nQL; u += ustep) {
                const uint32_t off = gofs + lp + map[t2.lq + u];
                if (packed) {
                    for (uint32_t k = k0; k < nk; k += kstep) {
                        const uint32_t idx = off + (rg + map[t2.rq + k]) * L;
#pragma unroll
                        for (int b = 0; b < B; b++) s[b] += (double)vals[b * c.tile + idx];
                    }
                } else {
                    const uint32_t step = kstep * L;
                    uint32_t idx = off + (rowbase + k0) * L;
                    uint32_t k = k0;
                    for (; k + (kOutEntries - 1) * kstep < nk; k += kOutEntries * kstep) {
                        T x[kOutEntries][B];
#pragma unroll
                        for (uint32_t y = 0; y < kOutEntries; y++)
#pragma unroll
                            for (int b = 0; b < B; b++) x[y][b] = vals[b * c.tile + idx + y * step];
#pragma unroll
                        for (uint32_t y = 0; y < kOutEntries; y++)
#pragma unroll
                            for (int b = 0; b < B; b++) s[b] += (double)x[y][b];
                        idx += kOutEntries * step;
                    }
                    for (; k < nk; k += kstep, idx += step) {
#pragma unroll
                        for (int b = 0; b < B; b++) s[b] += (double)vals[b * c.tile + idx];
                    }
                }
            }
            sep = t2.sep;
            part0 = t2.part0;
            tsz = t2.G * t2.nPL;
        }
#pragma unroll
        for (int b = 0; b < B; b++)
            for (uint32_t o2 = tpo / 2; o2 > 0; o2 >>= 1) s[b] += __shfl_xor(s[b], (int)o2, kWave);
        if (o < nout && sub == 0) {
#pragma unroll
            for (int b = 0; b < B; b++) {
                if (sl[b] < 0) continue;
                if (part0 < 0) static_cast<T*>(c.acc)[(uint64_t)sl[b] * c.sep_stride + sep + m] = (T)s[b];
                else static_cast<T*>(c.part)[(uint64_t)sl[b] * c.part_stride + (uint32_t)part0 + w.chunk * tsz + m] = (T)s[b];
            }
        }
    }
}

// After a distribute layer, per separator (real or one-variable virtual):
// finish the new separator table S* (summing partials), read the posterior
// marginals of the variables assigned to it, and for a real separator form
// the new/old ratio S*/S (0/0 = 0) rescaled by an exact power of two.
template <typename T>
__device__ __forceinline__ void fin_distribute_team(const Ctx& c, const DSepFin* __restrict__ fins, uint32_t nfins,
                                                    uint32_t nbig, const int32_t* __restrict__ slots, uint32_t bx) {
    __shared__ double red[kWaves];
    Team tm;
    uint32_t fi;
    if (!team_of(bx, nbig, nfins, red, tm, fi)) return;
    const uint32_t lane = tm.lane;
    const DSepFin f = fins[fi];
    const int slot = slots[blockIdx.y];
    T* __restrict__ acc = static_cast<T*>(c.acc) + (uint64_t)slot * c.sep_stride;
    const T* __restrict__ part = static_cast<const T*>(c.part) + (uint64_t)slot * c.part_stride;
    if (f.nchunk) {
        finish_range(f, acc + f.sep, part + f.part0, 0u, f.size, lane, tm.size, [](uint32_t, double) {});
        tm.sync();  // other lanes of the team read these sums below
    }
    // posteriors: each state of each assigned variable is a team-wide sum
    // over the separator entries carrying that state
    double* __restrict__ marg = c.marg + (uint64_t)slot * c.marg_stride;
    uint32_t mw = 0;
    for (uint32_t a = 0; a < f.nmv; a++) mw += c.mv[f.mv0 + a].card;
    shares_grouped(f, c, 0u, f.size, mw, lane, tm.size, [&](uint32_t m) { return (double)acc[f.sep + m]; },
                   [&](uint32_t, const DMargVar& mv, uint32_t x, double s) { marg[mv.out + x] = s; });
    if (f.edge < 0) return;
    const T* __restrict__ sepc = static_cast<const T*>(c.sepc) + (uint64_t)slot * c.sep_stride;
    T* __restrict__ sepd = static_cast<T*>(c.sepd) + (uint64_t)slot * c.sep_stride;
    double mx = 0.0;
#pragma unroll 4
    for (uint32_t m = lane; m < f.size; m += tm.size) {
        const double den = (double)sepc[f.sep + m];
        mx = fmax(mx, den == 0.0 ? 0.0 : acc[f.sep + m] / den);
    }
    mx = tm.max(mx);
    int k = 0;
    if (mx > 0.0) frexp(mx, &k);
    const double scale = ldexp(1.0, -k);
#pragma unroll 4
    for (uint32_t m = lane; m < f.size; m += tm.size) {
        const double den = (double)sepc[f.sep + m];
        sepd[f.sep + m] = (T)((den == 0.0 ? 0.0 : acc[f.sep + m] / den) * scale);
    }
}

// ------------------------------------------------- large separator finalisers

// A separator larger than one workgroup's share is finalised in blocks of at
// most kFinBlock entries, in two launches.  Phase one finishes each block's
// entries (partial sums), records the block's maximum and, in the
// distribute sweep, the block's partial posterior sums.  Phase two takes the
// separator's maximum over its blocks and writes the rescaled message
// (collect) or ratio (distribute); the separator's first block also adds the
// posterior sums of all blocks (strided lane sums and a shuffle tree).
// Every sum has a fixed order, as in the one-team finalisers.

__device__ __forceinline__ double block_max_all(double v, double* scratch) {
    v = wave_max(v);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) scratch[w] = v;
    __syncthreads();
    double s = scratch[0];
#pragma unroll
    for (int k = 1; k < kWaves; k++) s = fmax(s, scratch[k]);
    return s;
}

// Separator maximum over the blocks of b's separator.
__device__ __forceinline__ double fin_max(const Ctx& c, const DFinBlk& b, int slot, double* red) {
    const double* bm = c.bmax + (uint64_t)slot * c.bmax_stride + b.blk0;
    double mx = 0.0;
    for (uint32_t k = threadIdx.x; k < b.nblk; k += kBlock) mx = fmax(mx, bm[k]);
    return block_max_all(mx, red);
}

template <typename T>
__device__ __forceinline__ void fin_collect_a(const Ctx& c, const DSepFin* __restrict__ fins,
                                              const DFinBlk* __restrict__ blks, const int32_t* __restrict__ slots,
                                              uint32_t bx) {
    __shared__ double red[kWaves];
    const DFinBlk b = blks[bx];
    const DSepFin f = fins[b.fin];
    const int slot = slots[blockIdx.y];
    T* __restrict__ acc = static_cast<T*>(c.acc) + (uint64_t)slot * c.sep_stride + f.sep;
    const T* __restrict__ part = static_cast<const T*>(c.part) + (uint64_t)slot * c.part_stride + f.part0;
    double mx = 0.0;
    finish_range(f, acc, part, b.begin, b.begin + b.count, threadIdx.x, (uint32_t)kBlock,
                 [&](uint32_t, double v) { mx = fmax(mx, v); });
    mx = block_max_all(mx, red);
    if (threadIdx.x == 0) c.bmax[(uint64_t)slot * c.bmax_stride + b.id] = mx;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fin_collect_b(Ctx c, const DSepFin* __restrict__ fins,
                                                          const DFinBlk* __restrict__ blks,
                                                          const int32_t* __restrict__ slots) {
    __shared__ double red[kWaves];
    const DFinBlk b = blks[blockIdx.x];
    const DSepFin f = fins[b.fin];
    const int slot = slots[blockIdx.y];
    const double mx = fin_max(c, b, slot, red);
    int k = 0;
    if (mx > 0.0) frexp(mx, &k);
    else if (b.begin == 0 && threadIdx.x == 0) atomicOr(&c.flags[slot], c.fp32 ? 2 : 1);
    const double scale = ldexp(1.0, -k);
    const T* __restrict__ acc = static_cast<const T*>(c.acc) + (uint64_t)slot * c.sep_stride + f.sep;
    T* __restrict__ sepc = static_cast<T*>(c.sepc) + (uint64_t)slot * c.sep_stride + f.sep;
#pragma unroll 4
    for (uint32_t m = b.begin + threadIdx.x; m < b.begin + b.count; m += kBlock) sepc[m] = (T)(acc[m] * scale);
    if (b.begin == 0 && threadIdx.x == 0) c.kexp[(uint64_t)slot * c.kexp_stride + f.edge] = k;
}

template <typename T>
__device__ __forceinline__ void fin_distribute_a(const Ctx& c, const DSepFin* __restrict__ fins,
                                                 const DFinBlk* __restrict__ blks, const int32_t* __restrict__ slots,
                                                 uint32_t bx) {
    __shared__ double red[kWaves];
    const DFinBlk b = blks[bx];
    const DSepFin f = fins[b.fin];
    const int slot = slots[blockIdx.y];
    T* __restrict__ acc = static_cast<T*>(c.acc) + (uint64_t)slot * c.sep_stride + f.sep;
    const T* __restrict__ part = static_cast<const T*>(c.part) + (uint64_t)slot * c.part_stride + f.part0;
    const T* __restrict__ sepc = static_cast<const T*>(c.sepc) + (uint64_t)slot * c.sep_stride + f.sep;
    const uint32_t end = b.begin + b.count;
    // the block's new values are read back as stored (other lanes wrote them)
    if (f.nchunk) {
        finish_range(f, acc, part, b.begin, end, threadIdx.x, (uint32_t)kBlock, [](uint32_t, double) {});
        __syncthreads();
    }
    double mx = 0.0;
    for (uint32_t m0 = b.begin + threadIdx.x; m0 < end; m0 += 4 * kBlock) {
        T d[4], v[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; u++) {
            const uint32_t m = min(m0 + u * kBlock, end - 1);
            d[u] = sepc[m];
            v[u] = acc[m];
        }
#pragma unroll
        for (uint32_t u = 0; u < 4; u++)
            if (m0 + u * kBlock < end) mx = fmax(mx, d[u] == T(0) ? 0.0 : (double)v[u] / (double)d[u]);
    }
    mx = block_max_all(mx, red);
    if (threadIdx.x == 0) c.bmax[(uint64_t)slot * c.bmax_stride + b.id] = mx;
    // this block's share of each posterior sum: the entries with digit x
    // are m = (o * card + x) * stride + r, enumerated by e = o * stride + r
    double* __restrict__ bm = c.bmarg + (uint64_t)slot * c.bmarg_stride + b.mbase + (b.id - b.blk0) * b.mw;
    shares_grouped(f, c, b.begin, b.begin + b.count, b.mw, threadIdx.x, (uint32_t)kBlock,
                   [&](uint32_t m) { return (double)acc[m]; },
                   [&](uint32_t k, const DMargVar&, uint32_t, double s) { bm[k] = s; });
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fin_distribute_b(Ctx c, const DSepFin* __restrict__ fins,
                                                             const DFinBlk* __restrict__ blks,
                                                             const int32_t* __restrict__ slots) {
    __shared__ double red[kWaves];
    const DFinBlk b = blks[blockIdx.x];
    const DSepFin f = fins[b.fin];
    const int slot = slots[blockIdx.y];
    const double mx = fin_max(c, b, slot, red);
    int k = 0;
    if (mx > 0.0) frexp(mx, &k);
    const double scale = ldexp(1.0, -k);
    const T* __restrict__ acc = static_cast<const T*>(c.acc) + (uint64_t)slot * c.sep_stride + f.sep;
    const T* __restrict__ sepc = static_cast<const T*>(c.sepc) + (uint64_t)slot * c.sep_stride + f.sep;
    T* __restrict__ sepd = static_cast<T*>(c.sepd) + (uint64_t)slot * c.sep_stride + f.sep;
#pragma unroll 4
    for (uint32_t m = b.begin + threadIdx.x; m < b.begin + b.count; m += kBlock) {
        const double den = (double)sepc[m];
        sepd[m] = (T)((den == 0.0 ? 0.0 : acc[m] / den) * scale);
    }
    if (b.begin != 0) return;
    // the separator's first block adds every pair's shares over the blocks:
    // tpp lanes of one wave per pair, combined by a fixed xor-shuffle tree
    const double* __restrict__ bm = c.bmarg + (uint64_t)slot * c.bmarg_stride + b.mbase;
    double* __restrict__ marg = c.marg + (uint64_t)slot * c.marg_stride;
    const uint32_t mw = b.mw;
    uint32_t tpp = 1;
    while (tpp < (uint32_t)kWave && tpp * 2 * mw <= (uint32_t)kBlock) tpp *= 2;
    const uint32_t sub = threadIdx.x & (tpp - 1);
    for (uint32_t base = 0; base < mw * tpp; base += kBlock) {
        const uint32_t pidx = (base + threadIdx.x) / tpp;
        double s = 0.0;
        if (pidx < mw)
            for (uint32_t j = sub; j < b.nblk; j += tpp) s += bm[(uint64_t)j * mw + pidx];
        for (uint32_t o2 = tpp / 2; o2 > 0; o2 >>= 1) s += __shfl_xor(s, (int)o2, kWave);
        if (pidx < mw && sub == 0) {
            uint32_t vo = 0, a = 0;
            DMargVar mv = c.mv[f.mv0];
            while (pidx >= vo + mv.card) {
                vo += mv.card;
                mv = c.mv[f.mv0 + ++a];
            }
            marg[mv.out + pidx - vo] = s;
        }
    }
}

// Posteriors: normalise each variable's marginal.  log P(e): the log of the
// product of the roots' sums (one per tree of the forest) plus the
// rescaling exponents of the priors and of every collect message.
__global__ __launch_bounds__(kBlock) void k_marginals(Ctx c, const int32_t* __restrict__ slots) {
    __shared__ double s_log[kBlock];
    __shared__ long long s_exp[kBlock];
    const int slot = slots[blockIdx.x];
    const double* marg = c.marg + (uint64_t)slot * c.marg_stride;
    double* post = c.post + (uint64_t)slot * c.marg_stride;
    {
        const int32_t* kexp = c.kexp + (uint64_t)slot * c.kexp_stride;
        double lg = 0.0;
        long long ks = 0;
        for (uint32_t r = threadIdx.x; r < c.nroots; r += kBlock) {
            const double z = c.rsum[(uint64_t)slot * c.nroots + r];
            lg += z > 0.0 ? log(z) : -INFINITY;
        }
        for (int e = threadIdx.x; e < c.ne; e += kBlock) ks += kexp[e];
        s_log[threadIdx.x] = lg;
        s_exp[threadIdx.x] = ks;
        __syncthreads();
        for (int h = kBlock / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) {
                s_log[threadIdx.x] += s_log[threadIdx.x + h];
                s_exp[threadIdx.x] += s_exp[threadIdx.x + h];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double l = s_log[0];
            c.logpe[slot] = l > -INFINITY ? l + 0.69314718055994530942 * (double)(s_exp[0] + c.kappa_total) : -INFINITY;
        }
    }
    bool empty = false;
    for (int v = threadIdx.x; v < c.nvars; v += kBlock) {
        const DHomeVar h = c.hv[v];
        double s = 0.0;
        for (uint32_t x = 0; x < h.card; x++) s += marg[h.out + x];
        for (uint32_t x = 0; x < h.card; x++) post[h.out + x] = s > 0.0 ? marg[h.out + x] / s : 0.0;
        if (!(s > 0.0)) empty = true;
    }
    if (empty) atomicOr(&c.flags[slot], c.fp32 ? 2 : 1);
}

__global__ void k_gather(Ctx c, const int32_t* __restrict__ slots, double* __restrict__ post_out,
                         double* __restrict__ logpe_out, int32_t* __restrict__ flags_out) {
    const int b = blockIdx.x;
    const int slot = slots[b];
    const double* post = c.post + (uint64_t)slot * c.marg_stride;
    const uint32_t total = c.marg_stride;
    if (post_out)
        for (uint32_t k = threadIdx.x; k < total; k += blockDim.x) post_out[(uint64_t)b * total + k] = post[k];
    if (threadIdx.x == 0) {
        if (logpe_out) logpe_out[b] = c.logpe[slot];
        if (flags_out) flags_out[b] = c.flags[slot];
    }
}

// Start of a calibration: clear the batch's flags (and, with interleaved
// tables, its running sum of collect exponents, kept after the edges' own).
__global__ void k_begin(Ctx c, const int32_t* __restrict__ slots, int n) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n) {
        c.flags[slots[b]] = 0;
        if (c.S) c.kexp[(uint64_t)c.ne * c.S + (uint32_t)slots[b]] = 0;
    }
}

__global__ void k_expand_map(const uint32_t* __restrict__ map, uint32_t mh, uint32_t ml, uint32_t L,
                             uint32_t Lmul, uint32_t Lsh, uint32_t n, int32_t* __restrict__ out) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t hi = mdiv(j, Lmul, Lsh), lo = j - hi * L;
    out[j] = (int32_t)(map[mh + hi] + map[ml + lo]);
}

__global__ void k_zero(uint32_t* __restrict__ p, size_t words) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < words; k += (size_t)gridDim.x * blockDim.x)
        p[k] = 0u;
}

// The per-slot layer kernels stage B slots of c.tile entries each in LDS
// allocated at launch; c.tile is the layer's stage.
template <typename T, int B>
void launch_collect_b(const Ctx& c, const DGroup* groups, uint32_t ngroups, const int32_t* slots, int nslots,
                      hipStream_t s) {
    const uint64_t total = (uint64_t)ngroups * (uint64_t)((nslots + B - 1) / B);
    const size_t lds = (size_t)B * c.tile * sizeof(T);
    if (c.dense)
        hipLaunchKernelGGL((k_collect<T, B, false>), dim3((unsigned)total), dim3(kBlock), lds, s, c, groups, ngroups,
                           slots, nslots);
    else
        hipLaunchKernelGGL((k_collect<T, B, true>), dim3((unsigned)total), dim3(kBlock), lds, s, c, groups, ngroups,
                           slots, nslots);
}

template <typename T, int B>
void launch_gather_b(const Ctx& c, const DWork* works, uint32_t nworks, const int32_t* slots, int nslots,
                     hipStream_t s) {
    const uint64_t total = (uint64_t)nworks * (uint64_t)((nslots + B - 1) / B);
    const size_t lds = (size_t)B * c.tile * sizeof(T);
    if (c.dense)
        hipLaunchKernelGGL((k_dist_gather<T, B, false>), dim3((unsigned)total), dim3(kBlock), lds, s, c, works,
                           nworks, slots, nslots);
    else
        hipLaunchKernelGGL((k_dist_gather<T, B, true>), dim3((unsigned)total), dim3(kBlock), lds, s, c, works,
                           nworks, slots, nslots);
}

template <typename T>
void launch_collect_t(const Ctx& c, const DGroup* groups, uint32_t ngroups, const int32_t* slots, int nslots,
                      hipStream_t s) {
    const int B = slots_per_block(c.tile, sizeof(T), ngroups, nslots, c.bcap);
    if (B == 8) launch_collect_b<T, 8>(c, groups, ngroups, slots, nslots, s);
    else if (B == 4) launch_collect_b<T, 4>(c, groups, ngroups, slots, nslots, s);
    else if (B == 2) launch_collect_b<T, 2>(c, groups, ngroups, slots, nslots, s);
    else launch_collect_b<T, 1>(c, groups, ngroups, slots, nslots, s);
}

template <typename T>
void launch_gather_t(const Ctx& c, const DWork* works, uint32_t nworks, const int32_t* slots, int nslots,
                     hipStream_t s) {
    const int B = slots_per_block(c.tile, sizeof(T), nworks, nslots, c.bcap);
    if (B == 8) launch_gather_b<T, 8>(c, works, nworks, slots, nslots, s);
    else if (B == 4) launch_gather_b<T, 4>(c, works, nworks, slots, nslots, s);
    else if (B == 2) launch_gather_b<T, 2>(c, works, nworks, slots, nslots, s);
    else launch_gather_b<T, 1>(c, works, nworks, slots, nslots, s);
}

// A layer's finalisers in one launch: the first nteam workgroups finish the
// small separators (team per separator, as above), the next ones run the
// first phase of the large separators' blocks, one workgroup per block.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fin_collect(Ctx c, const DSepFin* __restrict__ sfins, uint32_t nsmall,
                                                        uint32_t nbig, uint32_t nteam, const DSepFin* __restrict__ fins,
                                                        const DFinBlk* __restrict__ blks,
                                                        const int32_t* __restrict__ slots) {
    if (blockIdx.x < nteam) fin_collect_team<T>(c, sfins, nsmall, nbig, slots, blockIdx.x);
    else fin_collect_a<T>(c, fins, blks, slots, blockIdx.x - nteam);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fin_distribute(Ctx c, const DSepFin* __restrict__ sfins, uint32_t nsmall,
                                                           uint32_t nbig, uint32_t nteam,
                                                           const DSepFin* __restrict__ fins,
                                                           const DFinBlk* __restrict__ blks,
                                                           const int32_t* __restrict__ slots) {
    if (blockIdx.x < nteam) fin_distribute_team<T>(c, sfins, nsmall, nbig, slots, blockIdx.x);
    else fin_distribute_a<T>(c, fins, blks, slots, blockIdx.x - nteam);
}

}  // namespace

hipError_t launch_collect(const Ctx& c, int prec, const DGroup* groups, uint32_t ngroups, uint32_t stage,
                          const int32_t* slots, int nslots, hipStream_t s) {
    if (!ngroups || !nslots) return hipSuccess;
    if (stage == 0 || stage * (prec ? 4u : 8u) > (uint32_t)kSlotStageBytes) return hipErrorInvalidValue;
    Ctx cl = c;
    cl.tile = stage;
    if (prec) launch_collect_t<float>(cl, groups, ngroups, slots, nslots, s);
    else launch_collect_t<double>(cl, groups, ngroups, slots, nslots, s);
    return hipGetLastError();
}

hipError_t launch_fin_collect(const Ctx& c, int prec, const DSepFin* sfins, uint32_t nsmall, uint32_t nbig,
                              const DSepFin* fins, const DFinBlk* blks, uint32_t nblks, const int32_t* slots,
                              int nslots, hipStream_t s) {
    const uint32_t nteam = nsmall ? nbig + (nsmall - nbig + kWaves - 1) / kWaves : 0;
    if (!(nteam + nblks) || !nslots) return hipSuccess;
    dim3 grid(nteam + nblks, (unsigned)nslots);
    if (prec)
        hipLaunchKernelGGL(k_fin_collect<float>, grid, dim3(kBlock), 0, s, c, sfins, nsmall, nbig, nteam, fins, blks,
                           slots);
    else
        hipLaunchKernelGGL(k_fin_collect<double>, grid, dim3(kBlock), 0, s, c, sfins, nsmall, nbig, nteam, fins, blks,
                           slots);
    return hipGetLastError();
}

hipError_t launch_fin_blocks(const Ctx& c, int prec, bool distribute, const DSepFin* fins, const DFinBlk* blks,
                             uint32_t nblks, const int32_t* slots, int nslots, hipStream_t s) {
    if (!nblks || !nslots) return hipSuccess;
    const dim3 grid(nblks, (unsigned)nslots), block(kBlock);
    if (!distribute) {
        if (prec) hipLaunchKernelGGL(k_fin_collect_b<float>, grid, block, 0, s, c, fins, blks, slots);
        else hipLaunchKernelGGL(k_fin_collect_b<double>, grid, block, 0, s, c, fins, blks, slots);
    } else {
        if (prec) hipLaunchKernelGGL(k_fin_distribute_b<float>, grid, block, 0, s, c, fins, blks, slots);
        else hipLaunchKernelGGL(k_fin_distribute_b<double>, grid, block, 0, s, c, fins, blks, slots);
    }
    return hipGetLastError();
}

hipError_t launch_distribute(const Ctx& c, int prec, const DWork* works, uint32_t nworks, uint32_t stage,
                             const int32_t* slots, int nslots, hipStream_t s) {
    if (!nworks || !nslots) return hipSuccess;
    if (stage == 0 || stage * (prec ? 4u : 8u) > (uint32_t)kSlotStageBytes) return hipErrorInvalidValue;
    Ctx cl = c;
    cl.tile = stage;
    if (prec) launch_gather_t<float>(cl, works, nworks, slots, nslots, s);
    else launch_gather_t<double>(cl, works, nworks, slots, nslots, s);
    return hipGetLastError();
}

hipError_t launch_fin_distribute(const Ctx& c, int prec, const DSepFin* sfins, uint32_t nsmall, uint32_t nbig,
                                 const DSepFin* fins, const DFinBlk* blks, uint32_t nblks, const int32_t* slots,
                                 int nslots, hipStream_t s) {
    const uint32_t nteam = nsmall ? nbig + (nsmall - nbig + kWaves - 1) / kWaves : 0;
    if (!(nteam + nblks) || !nslots) return hipSuccess;
    dim3 grid(nteam + nblks, (unsigned)nslots);
    if (prec)
        hipLaunchKernelGGL(k_fin_distribute<float>, grid, dim3(kBlock), 0, s, c, sfins, nsmall, nbig, nteam, fins,
                           blks, slots);
    else
        hipLaunchKernelGGL(k_fin_distribute<double>, grid, dim3(kBlock), 0, s, c, sfins, nsmall, nbig, nteam, fins,
                           blks, slots);
    return hipGetLastError();
}

hipError_t launch_marginals(const Ctx& c, const int32_t* slots, int nslots, hipStream_t s) {
    if (!nslots) return hipSuccess;
    hipLaunchKernelGGL(k_marginals, dim3((unsigned)nslots), dim3(kBlock), 0, s, c, slots);
    return hipGetLastError();
}

hipError_t launch_gather(const Ctx& c, const int32_t* slots, int nslots, double* post_out, double* logpe_out,
                         int32_t* flags_out, hipStream_t s) {
    if (!nslots) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)nslots), dim3(kBlock), 0, s, c, slots, post_out, logpe_out, flags_out);
    return hipGetLastError();
}

hipError_t launch_begin(const Ctx& c, const int32_t* slots, int nslots, hipStream_t s) {
    if (!nslots) return hipSuccess;
    hipLaunchKernelGGL(k_begin, dim3((unsigned)((nslots + 255) / 256)), dim3(256), 0, s, c, slots, nslots);
    return hipGetLastError();
}

hipError_t launch_expand_map(const uint32_t* map, uint32_t mh, uint32_t ml, uint32_t L, uint32_t Lmul, uint32_t Lsh,
                             uint32_t n, int32_t* out, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_expand_map, dim3((n + 255) / 256), dim3(256), 0, s, map, mh, ml, L, Lmul, Lsh, n, out);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    const size_t words = bytes / 4;
    if (!words) return hipSuccess;
    size_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint32_t*>(p), words);
    return hipGetLastError();
}

}  // namespace fbn
