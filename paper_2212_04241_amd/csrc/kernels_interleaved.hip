// Layer kernels for slot-interleaved tables (gfx950, wave64).
//
// Same operations as kernels.hip -- reduction, extension and
// marginalisation over the layers of the tree (the paper, Section 2) -- for
// trees that run large batches of evidence slots.  Every per-slot array is
// stored entry-major with the slots interleaved: entry x of slot s lives at
// x * S + s, S being the tree's slot capacity.  A wave takes one work item
// (a collect tile, a block of one distribute target, a separator or a
// finaliser block) for 64 batch positions, one per lane:
//   * everything that depends only on the table entry -- index maps, packed
//     digits, prior values, loop bounds -- is the same for the whole wave and
//     is computed once, in scalar registers;
//   * each lane does only its own slot's arithmetic, and every table load or
//     store of the wave touches one contiguous run of slots;
//   * every sum runs in a fixed order within its lane, so a slot's result
//     does not depend on which other slots share the launch: no
//     floating-point atomics and no cross-lane reductions (the only atomics
//     are an integer max on the bit pattern of a non-negative double and an
//     integer sum of exponents, both exact).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace fbn {
namespace {

constexpr int kLanes = 64;
constexpr int kWavesPerBlock = kBlock / kLanes;
constexpr uint32_t kUnroll = 8;  // collect: entries whose loads are issued together
constexpr uint32_t kDistBatch = 16;  // distribute: (output, entry) pairs whose loads are issued together

__device__ __forceinline__ uint32_t mdiv_i(uint32_t n, uint32_t mul, uint32_t sh) {
    return (uint32_t)(((uint64_t)__umulhi(n, mul) + n) >> sh);
}

// New separator sums and partial sums, stored in table precision.
template <typename T>
__device__ __forceinline__ T* accp(const Ctx& c) {
    return static_cast<T*>(c.acc);
}
template <typename T>
__device__ __forceinline__ T* partp(const Ctx& c) {
    return static_cast<T*>(c.part);
}

// Wave-uniform value in a scalar register.
__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// The wave's work item and slot group on a one-dimensional grid.  Workgroup
// w (four waves: four consecutive items of one slot group) is dispatched to
// XCD w % 8; each XCD takes one contiguous range of the (slot group, item
// quad) cells, so the waves that read one clique's tables and messages
// share that XCD's L2.
constexpr uint32_t kXcds = 8;
struct WaveCell {
    uint32_t item, group;
};
__device__ __forceinline__ WaveCell wave_cell(uint32_t nitems, int nslots) {
    const uint32_t nq = (nitems + kWavesPerBlock - 1) / kWavesPerBlock;
    const uint32_t ng = ((uint32_t)nslots + kLanes - 1) / kLanes;
    const uint32_t total = nq * ng;
    const uint32_t w = blockIdx.x, x = w % kXcds, k = w / kXcds;
    const uint32_t base = total / kXcds, extra = total % kXcds;
    const uint32_t idx = x * base + min(x, extra) + k;
    return WaveCell{uniform((idx % nq) * kWavesPerBlock + threadIdx.x / kLanes), uniform(idx / nq)};
}
// Workgroups of a launch over nitems items and nslots slots.
inline uint32_t cell_blocks(uint32_t nitems, int nslots) {
    return ((nitems + kWavesPerBlock - 1) / kWavesPerBlock) * (((uint32_t)nslots + kLanes - 1) / kLanes);
}
// The lane's slot in slot group g, or -1 past the batch.
__device__ __forceinline__ int lane_slot(const int32_t* slots, int nslots, uint32_t g) {
    const int b = (int)g * kLanes + (int)(threadIdx.x & (kLanes - 1));
    return b < nslots ? slots[b] : -1;
}

// Broadcast lane u's value of v (u uniform) to the whole wave.
__device__ __forceinline__ uint32_t bcast(uint32_t v, uint32_t u) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)u);
}
__device__ __forceinline__ uint64_t bcast(uint64_t v, uint32_t u) {
    return ((uint64_t)bcast((uint32_t)(v >> 32), u) << 32) | bcast((uint32_t)v, u);
}
__device__ __forceinline__ float bcast(float v, uint32_t u) { return __uint_as_float(bcast(__float_as_uint(v), u)); }
__device__ __forceinline__ double bcast(double v, uint32_t u) {
    return __longlong_as_double((long long)bcast((uint64_t)__double_as_longlong(v), u));
}

constexpr int kKids = 6;  // child indices held per lane; more children are read per entry

// ------------------------------------------------------------------ collect

// One piece of a collect group with NC children handled with loads issued
// together (NC == kKids: further children, if any, read per entry).  The
// entries are taken 64 at a time: lane j first works out entry j's digits,
// prior value and child separator indices (one coalesced read of each
// table), then the wave walks the 64 entries in order with those values
// broadcast from lane j, each lane applying them to its own slot.
template <typename T, int NC>
__device__ __forceinline__ void collect_piece_i(const Ctx& c, const DPiece& pc, const DClique& q,
                                                const DEvidence& ev, uint32_t lane, bool act, uint64_t S,
                                                uint64_t s, bool partial, double& part) {
    constexpr uint32_t U = NC <= 2 ? kUnroll : kUnroll / 2;  // entries per batch of loads
    constexpr int NW = NC > 0 ? NC : 1;
    const T* __restrict__ prior = static_cast<const T*>(c.prior);
    const T* __restrict__ sepc = static_cast<const T*>(c.sepc);
    T* __restrict__ psi = static_cast<T*>(c.psi);
    const uint32_t* __restrict__ map = c.map;
    const uint32_t nch = q.nchild;
    const uint32_t end = pc.begin + pc.count;
    uint32_t seg_left = q.seg - pc.begin % q.seg;
    uint32_t out = q.psep + pc.begin / q.seg;
    double acc = 0.0;
    for (uint32_t i0 = pc.begin; i0 < end; i0 += kLanes) {
        const uint32_t cnt = min((uint32_t)kLanes, end - i0);
        // lane j: entry i0 + j
        const uint32_t ej = i0 + min(lane, cnt - 1);
        const uint32_t rj = mdiv_i(ej, q.Lmul, q.Lsh);
        const uint32_t lj = ej - rj * q.L;
        const uint64_t dj = c.dig[q.hdig + rj] | c.dig[q.ldig + lj];
        const T pj = prior[q.off + ej];
        uint32_t xj[NW];
#pragma unroll
        for (int k = 0; k < NC; k++) {
            const DChild ch = c.ch[q.child0 + k];
            xj[k] = ch.sep + map[ch.mh + rj] + map[ch.ml + lj];
        }
        for (uint32_t u0 = 0; u0 < cnt; u0 += U) {
            T w[U][NW];
#pragma unroll
            for (uint32_t x = 0; x < U; x++) {
                const uint32_t u = min(u0 + x, cnt - 1);
#pragma unroll
                for (int k = 0; k < NC; k++) w[x][k] = sepc[(uint64_t)bcast(xj[k], u) * S + s];
            }
            T v[U];
#pragma unroll
            for (uint32_t x = 0; x < U; x++) {
                const uint32_t u = min(u0 + x, cnt - 1);
                const uint64_t d = bcast(dj, u);
                v[x] = ((d ^ ev.want) & ev.mask) ? T(0) : bcast(pj, u);
#pragma unroll
                for (int k = 0; k < NC; k++) v[x] *= w[x][k];
            }
            if (NC == kKids) {
                for (uint32_t k = kKids; k < nch; k++) {
                    const DChild ch = c.ch[q.child0 + k];
#pragma unroll
                    for (uint32_t x = 0; x < U; x++) {
                        const uint32_t u = min(u0 + x, cnt - 1);
                        const uint32_t idx = ch.sep + map[ch.mh + bcast(rj, u)] + map[ch.ml + bcast(lj, u)];
                        v[x] *= sepc[(uint64_t)idx * S + s];
                    }
                }
            }
#pragma unroll
            for (uint32_t x = 0; x < U; x++) {
                if (u0 + x < cnt) {
                    if (q.psi != kNoPsi && act) psi[((uint64_t)q.psi + i0 + u0 + x) * S + s] = v[x];
                    acc += (double)v[x];
                    if (--seg_left == 0) {
                        if (partial) part += acc;
                        else if (act) {
                            accp<T>(c)[(uint64_t)out * S + s] = acc;
                            // a root's sum (its tree's share of P(e)) also kept unrounded
                            if (out >= c.sep_total) c.rsum[(uint64_t)(out - c.sep_total) * S + s] = acc;
                        }
                        acc = 0.0;
                        out++;
                        seg_left = q.seg;
                    }
                }
            }
        }
    }
    if (partial) part += acc;
}

// psi[i] = prior[i] * [evidence agrees at i] * prod_children sepc[map(i)],
// stored; contiguous parent-separator segments summed in float64.  One wave
// per group of pieces, a lane per slot.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_collect_i(Ctx c, const DGroup* __restrict__ groups, uint32_t ngroups,
                                                      const int32_t* __restrict__ slots, int nslots) {
    const WaveCell wc = wave_cell(ngroups, nslots);
    const uint32_t gi = wc.item;
    if (gi >= ngroups) return;
    const uint32_t lane = threadIdx.x & (kLanes - 1);
    const int sl = lane_slot(slots, nslots, wc.group);
    const bool act = sl >= 0;                  // lanes past the batch still help with metadata
    const uint64_t S = c.S;
    const uint64_t s = act ? (uint64_t)sl : 0;
    const DGroup g = groups[gi];
    const bool partial = g.part >= 0;
    double part = 0.0;  // a partial group's single chunk sum
    for (uint32_t p = 0; p < g.npiece; p++) {
        const DPiece pc = c.pc[g.piece0 + p];
        const DClique q = c.cl[pc.clique];
        const DEvidence ev = c.ev[s * c.ev_stride + pc.clique];
        switch (q.nchild) {
        case 0: collect_piece_i<T, 0>(c, pc, q, ev, lane, act, S, s, partial, part); break;
        case 1: collect_piece_i<T, 1>(c, pc, q, ev, lane, act, S, s, partial, part); break;
        case 2: collect_piece_i<T, 2>(c, pc, q, ev, lane, act, S, s, partial, part); break;
        case 3: collect_piece_i<T, 3>(c, pc, q, ev, lane, act, S, s, partial, part); break;
        case 4: collect_piece_i<T, 4>(c, pc, q, ev, lane, act, S, s, partial, part); break;
        case 5: collect_piece_i<T, 5>(c, pc, q, ev, lane, act, S, s, partial, part); break;
        default: collect_piece_i<T, kKids>(c, pc, q, ev, lane, act, S, s, partial, part); break;
        }
    }
    if (partial && act) partp<T>(c)[(uint64_t)(uint32_t)g.part * S + s] = part;
}

// ---------------------------------------------------------------- distribute

// One work item of a target separator: outputs (g, t), g in [g0, g0+ng),
// each the sum over rows k in [k0, k0+nk) and lo offsets u of phi* at entry
// (RG[g] + RQ[k]) * L + LP[t] + LQ[u], phi* = psi * (parent ratio there).
// The work's (output, entry) pairs are walked in order, 64 at a time: lane j
// works out pair j's table entry, ratio entry and output index, and the
// wave then sums with those broadcast, writing each output when its last
// entry is in.
// The pairs of one work item, for a clique with NC children (NC == kKids:
// further children read per pair).  phi* at an entry is rebuilt exactly as
// the collect formed psi there -- prior, evidence mask, then the child
// messages in child order -- times the parent ratio, so it is bitwise the
// value the collect computed; the collect stores no psi.
template <typename T, int NC>
__device__ __forceinline__ void dist_pairs_i(const Ctx& c, const DWork& w, const DTarget& tg, const DClique& q,
                                             const DEvidence& ev, uint32_t lane, bool act, uint64_t S,
                                             uint64_t s) {
    constexpr int NW = NC > 0 ? NC : 1;
    constexpr uint32_t U = NC <= 1 ? kDistBatch : (NC <= 3 ? kDistBatch / 2 : kDistBatch / 4);
    const T* __restrict__ prior = static_cast<const T*>(c.prior);
    const T* __restrict__ sepc = static_cast<const T*>(c.sepc);
    const T* __restrict__ sepd = static_cast<const T*>(c.sepd);
    const uint32_t* __restrict__ map = c.map;
    const bool ratio = q.pedge >= 0;
    const uint32_t per = w.nk * tg.nQL;  // entries summed per output
    const uint32_t total = w.ng * tg.nPL * per;
    double acc = 0.0;
    uint32_t left = per;
    for (uint32_t f0 = 0; f0 < total; f0 += kLanes) {
        const uint32_t cnt = min((uint32_t)kLanes, total - f0);
        // lane j: pair f0 + j -- its entry's digits, prior, child message
        // indices, ratio index and output
        const uint32_t f = f0 + min(lane, cnt - 1);
        const uint32_t o = f / per, j = f - o * per;
        const uint32_t gg = o / tg.nPL, t = o - gg * tg.nPL;
        const uint32_t k = j / tg.nQL, u = j - k * tg.nQL;
        const uint32_t row = map[tg.rg + w.g0 + gg] + map[tg.rq + w.k0 + k];
        const uint32_t l = map[tg.lp + t] + map[tg.lq + u];
        const uint64_t dj = c.dig[q.hdig + row] | c.dig[q.ldig + l];
        const T pj = prior[q.off + row * q.L + l];
        uint32_t xj[NW];
#pragma unroll
        for (int ch = 0; ch < NC; ch++) {
            const DChild cd = c.ch[q.child0 + ch];
            xj[ch] = cd.sep + map[cd.mh + row] + map[cd.ml + l];
        }
        // the parent separator leads the clique's layout: entry / seg
        const uint32_t rj = ratio ? q.psep + mdiv_i(row * q.L + l, q.segmul, q.segsh) : 0u;
        const uint32_t mj = map[tg.tb + w.g0 + gg] + map[tg.tv + t];
        for (uint32_t x0 = 0; x0 < cnt; x0 += U) {
            T m[U][NW], r[U];
#pragma unroll
            for (uint32_t x = 0; x < U; x++) {
                const uint32_t b = min(x0 + x, cnt - 1);
#pragma unroll
                for (int ch = 0; ch < NC; ch++) m[x][ch] = sepc[(uint64_t)bcast(xj[ch], b) * S + s];
                r[x] = ratio ? sepd[(uint64_t)bcast(rj, b) * S + s] : T(1);
            }
            T v[U];
#pragma unroll
            for (uint32_t x = 0; x < U; x++) {
                const uint32_t b = min(x0 + x, cnt - 1);
                v[x] = ((bcast(dj, b) ^ ev.want) & ev.mask) ? T(0) : bcast(pj, b);
#pragma unroll
                for (int ch = 0; ch < NC; ch++) v[x] *= m[x][ch];
            }
            if (NC == kKids) {
                for (uint32_t ch = kKids; ch < q.nchild; ch++) {
                    const DChild cd = c.ch[q.child0 + ch];
#pragma unroll
                    for (uint32_t x = 0; x < U; x++) {
                        const uint32_t b = min(x0 + x, cnt - 1);
                        const uint32_t idx = cd.sep + map[cd.mh + bcast(row, b)] + map[cd.ml + bcast(l, b)];
                        v[x] *= sepc[(uint64_t)idx * S + s];
                    }
                }
            }
#pragma unroll
            for (uint32_t x = 0; x < U; x++) {
                if (x0 + x < cnt) {
                    acc += (double)(ratio ? v[x] * r[x] : v[x]);
                    if (--left == 0) {
                        const uint32_t mo = bcast(mj, x0 + x);
                        if (act) {
                            if (tg.part0 < 0) accp<T>(c)[(uint64_t)(tg.sep + mo) * S + s] = acc;
                            else partp<T>(c)[(uint64_t)((uint32_t)tg.part0 + mo * tg.nchunk + w.chunk) * S + s] = acc;
                        }
                        acc = 0.0;
                        left = per;
                    }
                }
            }
        }
    }
}

// The pairs of one work item of a clique whose psi the collect stored (one
// with more than kRebuildKidsInterleaved children, in the compact arena):
// phi* = stored psi times the parent ratio.
template <typename T>
__device__ __forceinline__ void dist_pairs_psi_i(const Ctx& c, const DWork& w, const DTarget& tg, const DClique& q,
                                                 uint32_t lane, bool act, uint64_t S, uint64_t s) {
    const T* __restrict__ psi = static_cast<const T*>(c.psi);
    const T* __restrict__ sepd = static_cast<const T*>(c.sepd);
    const uint32_t* __restrict__ map = c.map;
    const bool ratio = q.pedge >= 0;
    const uint32_t per = w.nk * tg.nQL;  // entries summed per output
    const uint32_t total = w.ng * tg.nPL * per;
    double acc = 0.0;
    uint32_t left = per;
    for (uint32_t f0 = 0; f0 < total; f0 += kLanes) {
        const uint32_t cnt = min((uint32_t)kLanes, total - f0);
        // lane j: pair f0 + j
        const uint32_t f = f0 + min(lane, cnt - 1);
        const uint32_t o = f / per, j = f - o * per;
        const uint32_t gg = o / tg.nPL, t = o - gg * tg.nPL;
        const uint32_t k = j / tg.nQL, u = j - k * tg.nQL;
        const uint32_t row = map[tg.rg + w.g0 + gg] + map[tg.rq + w.k0 + k];
        const uint32_t l = map[tg.lp + t] + map[tg.lq + u];
        const uint32_t ej = row * q.L + l;  // within the clique
        const uint32_t rj = ratio ? q.psep + mdiv_i(ej, q.segmul, q.segsh) : 0u;
        const uint32_t mj = map[tg.tb + w.g0 + gg] + map[tg.tv + t];
        for (uint32_t x0 = 0; x0 < cnt; x0 += kDistBatch) {
            T v[kDistBatch], r[kDistBatch];
#pragma unroll
            for (uint32_t x = 0; x < kDistBatch; x++) {
                const uint32_t b = min(x0 + x, cnt - 1);
                v[x] = psi[((uint64_t)q.psi + bcast(ej, b)) * S + s];
                r[x] = ratio ? sepd[(uint64_t)bcast(rj, b) * S + s] : T(1);
            }
#pragma unroll
            for (uint32_t x = 0; x < kDistBatch; x++) {
                if (x0 + x < cnt) {
                    acc += (double)(ratio ? v[x] * r[x] : v[x]);
                    if (--left == 0) {
                        const uint32_t mo = bcast(mj, x0 + x);
                        if (act) {
                            if (tg.part0 < 0) accp<T>(c)[(uint64_t)(tg.sep + mo) * S + s] = acc;
                            else partp<T>(c)[(uint64_t)((uint32_t)tg.part0 + mo * tg.nchunk + w.chunk) * S + s] = acc;
                        }
                        acc = 0.0;
                        left = per;
                    }
                }
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dist_i(Ctx c, const DWork* __restrict__ works, uint32_t nworks,
                                                   const int32_t* __restrict__ slots, int nslots) {
    const WaveCell wc = wave_cell(nworks, nslots);
    const uint32_t wi = wc.item;
    if (wi >= nworks) return;
    const uint32_t lane = threadIdx.x & (kLanes - 1);
    const int sl = lane_slot(slots, nslots, wc.group);
    const bool act = sl >= 0;
    const uint64_t S = c.S;
    const uint64_t s = act ? (uint64_t)sl : 0;
    const DWork w = works[wi];
    const DTarget tg = c.tg[w.target];
    const DClique q = c.cl[tg.clique];
    const DEvidence ev = c.ev[s * c.ev_stride + tg.clique];
    if (q.psi != kNoPsi) {
        dist_pairs_psi_i<T>(c, w, tg, q, lane, act, S, s);
        return;
    }
    switch (q.nchild) {
    case 0: dist_pairs_i<T, 0>(c, w, tg, q, ev, lane, act, S, s); break;
    case 1: dist_pairs_i<T, 1>(c, w, tg, q, ev, lane, act, S, s); break;
    case 2: dist_pairs_i<T, 2>(c, w, tg, q, ev, lane, act, S, s); break;
    case 3: dist_pairs_i<T, 3>(c, w, tg, q, ev, lane, act, S, s); break;
    case 4: dist_pairs_i<T, 4>(c, w, tg, q, ev, lane, act, S, s); break;
    case 5: dist_pairs_i<T, 5>(c, w, tg, q, ev, lane, act, S, s); break;
    default: dist_pairs_i<T, kKids>(c, w, tg, q, ev, lane, act, S, s); break;
    }
}

// --------------------------------------------------------------- finalisers

// Finish the entries [b, e) of separator f: with partial sums, an entry's
// value is the sum of its chunks in order.  The partials of consecutive
// entries are contiguous, so the whole range is read as one run, sixteen
// loads in flight, each entry's sum closed and stored as its last chunk
// comes in.  fn(m, v) is called once per entry in entry order.
template <typename T, typename F>
__device__ __forceinline__ void finish_range_i(const DSepFin& f, const Ctx& c, uint64_t S, uint64_t s, uint32_t b,
                                               uint32_t e, F fn) {
    T* __restrict__ acc = accp<T>(c);
    if (!f.nchunk) {
#pragma unroll 8
        for (uint32_t m = b; m < e; m++) fn(m, (double)acc[(uint64_t)(f.sep + m) * S + s]);
        return;
    }
    const T* __restrict__ part = partp<T>(c);
    const uint64_t q0 = (uint64_t)f.part0 + (uint64_t)b * f.nchunk;
    const uint64_t q1 = (uint64_t)f.part0 + (uint64_t)e * f.nchunk;
    double v = 0.0;
    uint32_t m = b, left = f.nchunk;
    for (uint64_t q = q0; q < q1; q += 16) {
        double x[16];
#pragma unroll
        for (uint32_t y = 0; y < 16; y++) x[y] = part[min(q + y, q1 - 1) * S + s];
#pragma unroll
        for (uint32_t y = 0; y < 16; y++) {
            if (q + y < q1) {
                v += x[y];
                if (--left == 0) {
                    acc[(uint64_t)(f.sep + m) * S + s] = (T)v;
                    fn(m, v);
                    v = 0.0;
                    left = f.nchunk;
                    m++;
                }
            }
        }
    }
}

// New values of n (1 <= n <= N) consecutive entries m0, m0 + 1, ... of a
// separator: fn(m, value) for each, then v[j] = entry m0 + j as stored in
// table precision (the rest of v zero).  An entry with chunks is the sum of
// its chunk partials in chunk order, stored into the accumulator.  A block
// at least half full walks the chunks with one load per entry each (N loads
// in flight, straight-line code); a sparser one walks the (entry, chunk)
// pairs flat and reads v back.
template <typename T, uint32_t N, typename F>
__device__ __forceinline__ void finish_block_i(const DSepFin& f, const Ctx& c, uint64_t S, uint64_t s, uint32_t m0,
                                               uint32_t n, double (&v)[N], F fn) {
    T* __restrict__ acc = accp<T>(c);
    if (f.nchunk && 2 * n >= N) {
        const T* __restrict__ part = partp<T>(c);
        const uint64_t p0 = (uint64_t)f.part0 + (uint64_t)m0 * f.nchunk;
#pragma unroll
        for (uint32_t j = 0; j < N; j++) v[j] = 0.0;
#pragma unroll 1
        for (uint32_t k = 0; k < f.nchunk; k++) {
            T x[N];
#pragma unroll
            for (uint32_t j = 0; j < N; j++) x[j] = part[(p0 + (uint64_t)min(j, n - 1) * f.nchunk + k) * S + s];
#pragma unroll
            for (uint32_t j = 0; j < N; j++) v[j] += (double)x[j];
        }
#pragma unroll
        for (uint32_t j = 0; j < N; j++) {
            if (j < n) {
                fn(m0 + j, v[j]);
                const T t = (T)v[j];
                acc[(uint64_t)(f.sep + m0 + j) * S + s] = t;
                v[j] = (double)t;
            } else {
                v[j] = 0.0;
            }
        }
        return;
    }
    if (f.nchunk) finish_range_i<T>(f, c, S, s, m0, m0 + n, fn);
    T x[N];
#pragma unroll
    for (uint32_t j = 0; j < N; j++) x[j] = acc[(uint64_t)(f.sep + m0 + min(j, n - 1)) * S + s];
#pragma unroll
    for (uint32_t j = 0; j < N; j++) {
        v[j] = j < n ? (double)x[j] : 0.0;
        if (!f.nchunk && j < n) fn(m0 + j, v[j]);
    }
}

// Posterior shares of n (>= 1) consecutive entries m0, m0 + 1, ... of a
// separator whose values are v[0..n) (the rest of v is zero): for each
// variable the separator carries and each state x, the sum of the values
// whose digit of that variable is x, in entry order, passed to
// put(variable, x, k, sum) with k the running (variable, state) index.
template <uint32_t N, typename Put>
__device__ __forceinline__ void shares_i(const DSepFin& f, const Ctx& c, uint32_t m0, uint32_t n,
                                         const double (&v)[N], Put put) {
    uint32_t k = 0;
    for (uint32_t a = 0; a < f.nmv; a++) {
        const DMargVar mv = c.mv[f.mv0 + a];
        uint32_t dg[N];
#pragma unroll
        for (uint32_t j = 0; j < N; j++) {
            const uint32_t t = mdiv_i(m0 + min(j, n - 1), mv.smul, mv.ssh);
            dg[j] = t - mdiv_i(t, mv.cmul, mv.csh) * mv.card;
        }
        for (uint32_t x = 0; x < mv.card; x++) {
            double sum = 0.0;
#pragma unroll
            for (uint32_t j = 0; j < N; j++) sum += dg[j] == x ? v[j] : 0.0;
            put(mv, x, k++, sum);
        }
    }
}

// After a collect layer: finish, rescale to a max in [0.5, 1), store, and
// keep the exponent; a root's entry flags impossible evidence.
template <typename T>
__device__ __forceinline__ void fin_collect_small_i(const Ctx& c, const DSepFin* __restrict__ fins, uint32_t fi,
                                                    int sl) {
    if (sl < 0) return;
    const uint64_t S = c.S, s = (uint64_t)sl;
    const DSepFin f = fins[fi];
    // the whole separator (at most kBigSeparatorInterleaved entries) in registers
    double v[kBigSeparatorInterleaved];
    double mx = 0.0;
    finish_block_i<T>(f, c, S, s, 0u, f.size, v, [&](uint32_t, double w) {
        mx = fmax(mx, w);
        if (f.edge < 0 && f.nchunk) c.rsum[(uint64_t)(f.sep - c.sep_total) * S + s] = w;
    });
    if (f.edge < 0) {
        if (!(v[0] > 0.0)) atomicOr(&c.flags[s], c.fp32 ? 2 : 1);
        return;
    }
    int k = 0;
    if (mx > 0.0) frexp(mx, &k);
    else atomicOr(&c.flags[s], c.fp32 ? 2 : 1);
    const double scale = ldexp(1.0, -k);
    T* __restrict__ sepc = static_cast<T*>(c.sepc);
#pragma unroll
    for (uint32_t j = 0; j < kBigSeparatorInterleaved; j++)
        if (j < f.size) sepc[(uint64_t)(f.sep + j) * S + s] = (T)(v[j] * scale);
    c.kexp[(uint64_t)f.edge * S + s] = k;
    atomicAdd(&c.kexp[(uint64_t)c.ne * S + s], k);  // exact: integer sum
}

// After a distribute layer: finish the new separator, its posterior sums,
// and for a real separator the ratio new/old (0/0 = 0) rescaled.
template <typename T>
__device__ __forceinline__ void fin_distribute_small_i(const Ctx& c, const DSepFin* __restrict__ fins, uint32_t fi,
                                                       int sl) {
    if (sl < 0) return;
    const uint64_t S = c.S, s = (uint64_t)sl;
    const DSepFin f = fins[fi];
    if (f.size <= kBigSeparatorInterleaved) {
        // the whole separator in registers: new values, posterior sums
        // straight to the marginal accumulators, then the ratio
        double v[kBigSeparatorInterleaved];
        T den[kBigSeparatorInterleaved];
        const T* __restrict__ sepc = static_cast<const T*>(c.sepc);
        if (f.edge >= 0) {
#pragma unroll
            for (uint32_t j = 0; j < kBigSeparatorInterleaved; j++)
                den[j] = sepc[(uint64_t)(f.sep + min(j, f.size - 1)) * S + s];
        }
        finish_block_i<T>(f, c, S, s, 0u, f.size, v, [](uint32_t, double) {});
        double mx = 0.0;
#pragma unroll
        for (uint32_t j = 0; j < kBigSeparatorInterleaved; j++)
            if (f.edge >= 0 && j < f.size) mx = fmax(mx, den[j] == T(0) ? 0.0 : v[j] / (double)den[j]);
        shares_i(f, c, 0, f.size, v, [&](const DMargVar& mv, uint32_t x, uint32_t, double sum) {
            c.marg[(uint64_t)(mv.out + x) * S + s] = sum;
        });
        if (f.edge < 0) return;
        int k = 0;
        if (mx > 0.0) frexp(mx, &k);
        const double scale = ldexp(1.0, -k);
        T* __restrict__ sepd = static_cast<T*>(c.sepd);
#pragma unroll
        for (uint32_t j = 0; j < kBigSeparatorInterleaved; j++)
            if (j < f.size)
                sepd[(uint64_t)(f.sep + j) * S + s] = (T)((den[j] == T(0) ? 0.0 : v[j] / (double)den[j]) * scale);
        return;
    }
    if (f.nchunk) finish_range_i<T>(f, c, S, s, 0u, f.size, [](uint32_t, double) {});
    // the posterior sums go straight to the marginal accumulators
    for (uint32_t a = 0; a < f.nmv; a++) {
        const DMargVar mv = c.mv[f.mv0 + a];
        const uint32_t span = mv.stride * mv.card;
        for (uint32_t x = 0; x < mv.card; x++) {
            double acc = 0.0;
            for (uint32_t m = x * mv.stride; m < f.size; m += span) {
#pragma unroll 8
                for (uint32_t y = m; y < m + mv.stride; y++) acc += accp<T>(c)[(uint64_t)(f.sep + y) * S + s];
            }
            c.marg[(uint64_t)(mv.out + x) * S + s] = acc;
        }
    }
    if (f.edge < 0) return;
    const T* __restrict__ sepc = static_cast<const T*>(c.sepc);
    T* __restrict__ sepd = static_cast<T*>(c.sepd);
    double mx = 0.0;
#pragma unroll 8
    for (uint32_t m = 0; m < f.size; m++) {
        const double den = (double)sepc[(uint64_t)(f.sep + m) * S + s];
        mx = fmax(mx, den == 0.0 ? 0.0 : accp<T>(c)[(uint64_t)(f.sep + m) * S + s] / den);
    }
    int k = 0;
    if (mx > 0.0) frexp(mx, &k);
    const double scale = ldexp(1.0, -k);
#pragma unroll 8
    for (uint32_t m = 0; m < f.size; m++) {
        const uint64_t x = (uint64_t)(f.sep + m) * S + s;
        const double den = (double)sepc[x];
        sepd[x] = (T)((den == 0.0 ? 0.0 : accp<T>(c)[x] / den) * scale);
    }
}

// Large separators in blocks of at most kFinBlockInterleaved entries, one
// wave per block.  Phase a finishes the block's entries and folds its
// maximum into the separator's maximum with an integer atomic max on the
// bit pattern (exact and order-independent for non-negative doubles; the
// separator's slot, its index among the large separators, is cleared before
// every calibration); in the
// distribute sweep it also writes the block's share of every posterior sum.
// Phase b rescales with the separator's maximum; the separator's blocks
// split its posterior sums between them, each adding one sum's block
// shares in block order.
__device__ __forceinline__ void fold_max(const Ctx& c, const DFinBlk& b, uint64_t S, uint64_t s, double mx) {
    atomicMax(reinterpret_cast<unsigned long long*>(c.bmax) + (uint64_t)b.mx * S + s,
              (unsigned long long)__double_as_longlong(mx));
}
__device__ __forceinline__ double fin_max_i(const Ctx& c, const DFinBlk& b, uint64_t S, uint64_t s) {
    return c.bmax[(uint64_t)b.mx * S + s];
}

template <typename T>
__device__ __forceinline__ void fin_collect_a_i(const Ctx& c, const DSepFin* __restrict__ fins,
                                                const DFinBlk* __restrict__ blks, uint32_t bi,
                                                int sl) {
    if (sl < 0) return;
    const uint64_t S = c.S, s = (uint64_t)sl;
    const DFinBlk b = blks[bi];
    const DSepFin f = fins[b.fin];
    double mx = 0.0, v[kFinBlockInterleaved];
    finish_block_i<T>(f, c, S, s, b.begin, b.count, v, [&](uint32_t, double w) { mx = fmax(mx, w); });
    fold_max(c, b, S, s, mx);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fin_collect_ib(Ctx c, const DSepFin* __restrict__ fins,
                                                           const DFinBlk* __restrict__ blks, uint32_t nblks,
                                                           const int32_t* __restrict__ slots, int nslots) {
    const WaveCell wc = wave_cell(nblks, nslots);
    const uint32_t bi = wc.item;
    if (bi >= nblks) return;
    const int sl = lane_slot(slots, nslots, wc.group);
    if (sl < 0) return;
    const uint64_t S = c.S, s = (uint64_t)sl;
    const DFinBlk b = blks[bi];
    const DSepFin f = fins[b.fin];
    const double mx = fin_max_i(c, b, S, s);
    int k = 0;
    if (mx > 0.0) frexp(mx, &k);
    else if (b.begin == 0) atomicOr(&c.flags[s], c.fp32 ? 2 : 1);
    const double scale = ldexp(1.0, -k);
    T* __restrict__ sepc = static_cast<T*>(c.sepc);
    T a[kFinBlockInterleaved];
#pragma unroll
    for (uint32_t j = 0; j < kFinBlockInterleaved; j++)
        a[j] = accp<T>(c)[(uint64_t)(f.sep + b.begin + min(j, b.count - 1)) * S + s];
#pragma unroll
    for (uint32_t j = 0; j < kFinBlockInterleaved; j++)
        if (j < b.count) sepc[(uint64_t)(f.sep + b.begin + j) * S + s] = (T)((double)a[j] * scale);
    if (b.begin == 0) {
        c.kexp[(uint64_t)f.edge * S + s] = k;
        atomicAdd(&c.kexp[(uint64_t)c.ne * S + s], k);  // exact: integer sum
    }
}

template <typename T>
__device__ __forceinline__ void fin_distribute_a_i(const Ctx& c, const DSepFin* __restrict__ fins,
                                                   const DFinBlk* __restrict__ blks, uint32_t bi,
                                                   int sl) {
    if (sl < 0) return;
    const uint64_t S = c.S, s = (uint64_t)sl;
    const DFinBlk b = blks[bi];
    const DSepFin f = fins[b.fin];
    const T* __restrict__ sepc = static_cast<const T*>(c.sepc);
    // the block's new separator values, as stored, stay in registers for
    // the ratio maximum and the posterior shares
    T den[kFinBlockInterleaved];
#pragma unroll
    for (uint32_t j = 0; j < kFinBlockInterleaved; j++)
        den[j] = sepc[(uint64_t)(f.sep + b.begin + min(j, b.count - 1)) * S + s];
    double v[kFinBlockInterleaved];
    finish_block_i<T>(f, c, S, s, b.begin, b.count, v, [](uint32_t, double) {});
    double mx = 0.0;
#pragma unroll
    for (uint32_t j = 0; j < kFinBlockInterleaved; j++)
        if (j < b.count) mx = fmax(mx, den[j] == T(0) ? 0.0 : v[j] / (double)den[j]);
    fold_max(c, b, S, s, mx);
    // this block's share of each posterior sum
    double* __restrict__ bm = c.bmarg;
    const uint64_t o0 = (uint64_t)b.mbase + (uint64_t)(b.id - b.blk0) * b.mw;
    shares_i(f, c, b.begin, b.count, v,
             [&](const DMargVar&, uint32_t, uint32_t k, double sum) { bm[(o0 + k) * S + s] = sum; });
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fin_distribute_ib(Ctx c, const DSepFin* __restrict__ fins,
                                                              const DFinBlk* __restrict__ blks, uint32_t nblks,
                                                              const int32_t* __restrict__ slots, int nslots) {
    const WaveCell wc = wave_cell(nblks, nslots);
    const uint32_t bi = wc.item;
    if (bi >= nblks) return;
    const int sl = lane_slot(slots, nslots, wc.group);
    if (sl < 0) return;
    const uint64_t S = c.S, s = (uint64_t)sl;
    const DFinBlk b = blks[bi];
    const DSepFin f = fins[b.fin];
    const double mx = fin_max_i(c, b, S, s);
    int k = 0;
    if (mx > 0.0) frexp(mx, &k);
    const double scale = ldexp(1.0, -k);
    const T* __restrict__ sepc = static_cast<const T*>(c.sepc);
    T* __restrict__ sepd = static_cast<T*>(c.sepd);
    T a[kFinBlockInterleaved], den[kFinBlockInterleaved];
#pragma unroll
    for (uint32_t j = 0; j < kFinBlockInterleaved; j++) {
        const uint64_t x = (uint64_t)(f.sep + b.begin + min(j, b.count - 1)) * S + s;
        a[j] = accp<T>(c)[x];
        den[j] = sepc[x];
    }
#pragma unroll
    for (uint32_t j = 0; j < kFinBlockInterleaved; j++)
        if (j < b.count)
            sepd[(uint64_t)(f.sep + b.begin + j) * S + s] =
                (T)((den[j] == T(0) ? 0.0 : (double)a[j] / (double)den[j]) * scale);
    // posterior sums: block j of the separator adds sums j, j + nblk, ...
    const uint32_t j = b.id - b.blk0;
    for (uint32_t pidx = j; pidx < b.mw; pidx += b.nblk) {
        uint32_t vo = 0, a = 0;
        DMargVar mv = c.mv[f.mv0];
        while (pidx >= vo + mv.card) {
            vo += mv.card;
            mv = c.mv[f.mv0 + ++a];
        }
        double acc = 0.0;
#pragma unroll 8
        for (uint32_t jj = 0; jj < b.nblk; jj++) acc += c.bmarg[((uint64_t)b.mbase + (uint64_t)jj * b.mw + pidx) * S + s];
        c.marg[(uint64_t)(mv.out + pidx - vo) * S + s] = acc;
    }
}

// A layer's finalisers in one launch: the first nsmall waves take the small
// separators whole, the next nblks the first phase of the large separators'
// blocks (their second phase is a launch of its own).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fin_collect_i(Ctx c, const DSepFin* __restrict__ sfins, uint32_t nsmall,
                                                          const DFinBlk* __restrict__ blks, uint32_t nblks,
                                                          const DSepFin* __restrict__ fins,
                                                          const int32_t* __restrict__ slots, int nslots) {
    const WaveCell wc = wave_cell(nsmall + nblks, nslots);
    const uint32_t wi = wc.item;
    if (wi >= nsmall + nblks) return;
    const int sl = lane_slot(slots, nslots, wc.group);
    if (wi < nsmall) fin_collect_small_i<T>(c, sfins, wi, sl);
    else fin_collect_a_i<T>(c, fins, blks, wi - nsmall, sl);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fin_distribute_i(Ctx c, const DSepFin* __restrict__ sfins,
                                                             uint32_t nsmall, const DFinBlk* __restrict__ blks,
                                                             uint32_t nblks, const DSepFin* __restrict__ fins,
                                                             const int32_t* __restrict__ slots, int nslots) {
    const WaveCell wc = wave_cell(nsmall + nblks, nslots);
    const uint32_t wi = wc.item;
    if (wi >= nsmall + nblks) return;
    const int sl = lane_slot(slots, nslots, wc.group);
    if (wi < nsmall) fin_distribute_small_i<T>(c, sfins, wi, sl);
    else fin_distribute_a_i<T>(c, fins, blks, wi - nsmall, sl);
}

// ---------------------------------------------------------------- posteriors

// Per slot: normalise every variable's marginal into the slot-major
// posterior array read by the gather, and form log P(e) from the roots'
// sums and the exponents (fixed order per lane).
__global__ __launch_bounds__(kBlock) void k_marginals_i(Ctx c, const int32_t* __restrict__ slots, int nslots,
                                                        uint32_t vars_per_wave) {
    const uint32_t wi = uniform(blockIdx.x * kWavesPerBlock + threadIdx.x / kLanes);
    const int sl = lane_slot(slots, nslots, blockIdx.y);
    if (sl < 0) return;
    const uint64_t S = c.S, s = (uint64_t)sl;
    const uint32_t v0 = wi * vars_per_wave;
    const uint32_t v1 = min((uint32_t)c.nvars, v0 + vars_per_wave);
    double* __restrict__ post = c.post + s * c.marg_stride;
    bool empty = false;
    for (uint32_t v = v0; v < v1; v++) {
        const DHomeVar h = c.hv[v];
        double sum = 0.0;
        for (uint32_t x = 0; x < h.card; x++) sum += c.marg[(uint64_t)(h.out + x) * S + s];
        for (uint32_t x = 0; x < h.card; x++)
            post[h.out + x] = sum > 0.0 ? c.marg[(uint64_t)(h.out + x) * S + s] / sum : 0.0;
        if (!(sum > 0.0)) empty = true;
    }
    if (empty) atomicOr(&c.flags[s], c.fp32 ? 2 : 1);
    if (wi != 0) return;
    double lg = 0.0;
    for (uint32_t r = 0; r < c.nroots; r++) {
        const double z = c.rsum[(uint64_t)r * S + s];
        lg += z > 0.0 ? log(z) : -INFINITY;
    }
    const long long ks = c.kexp[(uint64_t)c.ne * S + s];  // summed by the collect finalisers
    c.logpe[s] = lg > -INFINITY ? lg + 0.69314718055994530942 * (double)(ks + c.kappa_total) : -INFINITY;
}

}  // namespace

hipError_t launch_interleaved(const Ctx& c, int prec, int kind, const void* items, uint32_t nitems,
                              const DSepFin* fins, const int32_t* slots, int nslots, hipStream_t st) {
    if (!nitems || !nslots) return hipSuccess;
    const dim3 grid(cell_blocks(nitems, nslots));
    const dim3 block(kBlock);
    const auto* groups = static_cast<const DGroup*>(items);
    const auto* works = static_cast<const DWork*>(items);
    const auto* blks = static_cast<const DFinBlk*>(items);
    switch (kind) {
    case kIlCollect:
        if (prec) hipLaunchKernelGGL(k_collect_i<float>, grid, block, 0, st, c, groups, nitems, slots, nslots);
        else hipLaunchKernelGGL(k_collect_i<double>, grid, block, 0, st, c, groups, nitems, slots, nslots);
        break;
    case kIlDistribute:
        if (prec) hipLaunchKernelGGL(k_dist_i<float>, grid, block, 0, st, c, works, nitems, slots, nslots);
        else hipLaunchKernelGGL(k_dist_i<double>, grid, block, 0, st, c, works, nitems, slots, nslots);
        break;
    case kIlFinCollectB:
        if (prec) hipLaunchKernelGGL(k_fin_collect_ib<float>, grid, block, 0, st, c, fins, blks, nitems, slots, nslots);
        else hipLaunchKernelGGL(k_fin_collect_ib<double>, grid, block, 0, st, c, fins, blks, nitems, slots, nslots);
        break;
    case kIlFinDistributeB:
        if (prec)
            hipLaunchKernelGGL(k_fin_distribute_ib<float>, grid, block, 0, st, c, fins, blks, nitems, slots, nslots);
        else
            hipLaunchKernelGGL(k_fin_distribute_ib<double>, grid, block, 0, st, c, fins, blks, nitems, slots, nslots);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fin_interleaved(const Ctx& c, int prec, bool dist, const DSepFin* small, uint32_t nsmall,
                                  const DFinBlk* blks, uint32_t nblks, const DSepFin* fins, const int32_t* slots,
                                  int nslots, hipStream_t st) {
    const uint32_t n = nsmall + nblks;
    if (!n || !nslots) return hipSuccess;
    const dim3 grid(cell_blocks(n, nslots));
    const dim3 block(kBlock);
    if (dist) {
        if (prec)
            hipLaunchKernelGGL(k_fin_distribute_i<float>, grid, block, 0, st, c, small, nsmall, blks, nblks, fins,
                               slots, nslots);
        else
            hipLaunchKernelGGL(k_fin_distribute_i<double>, grid, block, 0, st, c, small, nsmall, blks, nblks, fins,
                               slots, nslots);
    } else {
        if (prec)
            hipLaunchKernelGGL(k_fin_collect_i<float>, grid, block, 0, st, c, small, nsmall, blks, nblks, fins,
                               slots, nslots);
        else
            hipLaunchKernelGGL(k_fin_collect_i<double>, grid, block, 0, st, c, small, nsmall, blks, nblks, fins,
                               slots, nslots);
    }
    return hipGetLastError();
}

hipError_t launch_marginals_interleaved(const Ctx& c, const int32_t* slots, int nslots, hipStream_t st) {
    if (!nslots) return hipSuccess;
    const uint32_t per = 16;  // variables per wave
    const uint32_t waves = ((uint32_t)c.nvars + per - 1) / per;
    const dim3 grid(std::max<uint32_t>(1u, (waves + kWavesPerBlock - 1) / kWavesPerBlock),
                    (unsigned)((nslots + kLanes - 1) / kLanes));
    hipLaunchKernelGGL(k_marginals_i, grid, dim3(kBlock), 0, st, c, slots, nslots, per);
    return hipGetLastError();
}

}  // namespace fbn
