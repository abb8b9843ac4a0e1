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
// (H[hi] + L[lo]) that stay in cache; separator sums and scale factors are
// float64.  No atomics on data, so a case gives bitwise the same result
// alone or in any batch.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace fbn {
namespace {

constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;
constexpr int kMaxKids = 8;  // child maps held in registers; more use a loop

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

template <typename T, int B>
__global__ __launch_bounds__(kBlock) void k_collect(Ctx c, const DGroup* __restrict__ groups,
                                                    const int32_t* __restrict__ slots, int nslots) {
    __shared__ __align__(16) unsigned char stage[kStageBytes];
    __shared__ DPiece pcs[kMaxPieces];
    __shared__ double red[kWaves];
    T* vals = reinterpret_cast<T*>(stage);
    const DGroup g = groups[blockIdx.x];
    int sl[B];
#pragma unroll
    for (int b = 0; b < B; b++) {
        const int k = (int)blockIdx.y * B + b;
        sl[b] = k < nslots ? slots[k] : -1;
    }
    for (uint32_t k = threadIdx.x; k < g.npiece; k += kBlock) pcs[k] = c.pc[g.piece0 + k];
    __syncthreads();

    const T* __restrict__ prior = static_cast<const T*>(c.prior);
    const uint32_t* __restrict__ map = c.map;
    uint32_t p = 0;
    int cur = -1;
    DClique q{};
    DEvidence e[B];
    uint64_t anyev = 0;
    for (uint32_t gi = threadIdx.x; gi < g.total; gi += kBlock) {
        while (gi >= pcs[p].gofs + pcs[p].count) p++;
        if ((int)p != cur) {
            cur = (int)p;
            q = c.cl[pcs[p].clique];
            anyev = 0;
#pragma unroll
            for (int b = 0; b < B; b++) {
                e[b] = sl[b] >= 0 ? c.ev[(uint64_t)sl[b] * c.ev_stride + pcs[p].clique] : DEvidence{0, 0};
                anyev |= e[b].mask;
            }
        }
        const uint32_t i = pcs[p].begin + (gi - pcs[p].gofs);
        const uint32_t hi = mdiv(i, q.Lmul, q.Lsh);
        const uint32_t lo = i - hi * q.L;
        const T pv = prior[q.off + i];
        const uint64_t d = anyev ? (c.dig[q.hdig + hi] | c.dig[q.ldig + lo]) : 0;
        uint32_t jk[kMaxKids];
#pragma unroll
        for (int k = 0; k < kMaxKids; k++)
            if (k < (int)q.nchild) {
                const DChild ch = c.ch[q.child0 + k];
                jk[k] = ch.sep + map[ch.mh + hi] + map[ch.ml + lo];
            }
#pragma unroll
        for (int b = 0; b < B; b++) {
            if (sl[b] < 0) continue;
            const T* __restrict__ sepc = static_cast<const T*>(c.sepc) + (uint64_t)sl[b] * c.sep_stride;
            T v = ((d ^ e[b].want) & e[b].mask) ? T(0) : pv;
#pragma unroll
            for (int k = 0; k < kMaxKids; k++)
                if (k < (int)q.nchild) v *= sepc[jk[k]];
            for (uint32_t k = kMaxKids; k < q.nchild; k++) {
                const DChild ch = c.ch[q.child0 + k];
                v *= sepc[ch.sep + map[ch.mh + hi] + map[ch.ml + lo]];
            }
            static_cast<T*>(c.psi)[(uint64_t)sl[b] * c.psi_stride + q.off + i] = v;
            vals[b * c.tile + gi] = v;
        }
    }
    __syncthreads();

    // marginalise onto the parent separator: contiguous segments of q.seg
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int b = 0; b < B; b++) {
        if (sl[b] < 0) continue;
        const T* v = vals + b * c.tile;
        double* __restrict__ acc = c.acc + (uint64_t)sl[b] * c.sep_stride;
        if (g.part >= 0) {
            double s = 0.0;
            for (uint32_t k = threadIdx.x; k < g.total; k += kBlock) s += (double)v[k];
            s = block_sum(s, red);
            if (threadIdx.x == 0) c.part[(uint64_t)sl[b] * c.part_stride + (uint32_t)g.part] = s;
            continue;
        }
        for (uint32_t r = 0; r < g.npiece; r++) {
            const DPiece pc = pcs[r];
            const DClique qq = c.cl[pc.clique];
            const uint32_t seg = qq.seg;
            const uint32_t nseg = pc.count / seg;
            const uint32_t out0 = qq.psep + pc.begin / seg;
            if (seg >= 32) {
                for (uint32_t s = (uint32_t)wid; s < nseg; s += kWaves) {
                    double a = 0.0;
                    for (uint32_t k = (uint32_t)lane; k < seg; k += kWave) a += (double)v[pc.gofs + s * seg + k];
                    a = wave_sum(a);
                    if (lane == 0) acc[out0 + s] = a;
                }
            } else {
                for (uint32_t s = threadIdx.x; s < nseg; s += kBlock) {
                    double a = 0.0;
                    for (uint32_t k = 0; k < seg; k++) a += (double)v[pc.gofs + s * seg + k];
                    acc[out0 + s] = a;
                }
            }
        }
    }
}

// After a collect layer, one wave per separator: finish the message (sum
// partial sums where a segment spanned several tiles), rescale it by an
// exact power of two so its largest entry lies in [0.5, 1), store it in
// table precision and record the exponent.  The root's one-entry virtual
// separator yields log P(e).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fin_collect(Ctx c, const DSepFin* __restrict__ fins, uint32_t nfins,
                                                        const int32_t* __restrict__ slots) {
    const uint32_t fi = blockIdx.x * kWaves + threadIdx.x / kWave;
    if (fi >= nfins) return;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const DSepFin f = fins[fi];
    const int slot = slots[blockIdx.y];
    double* __restrict__ acc = c.acc + (uint64_t)slot * c.sep_stride;
    const double* __restrict__ part = c.part + (uint64_t)slot * c.part_stride;
    int32_t* kexp = c.kexp + (uint64_t)slot * c.kexp_stride;

    double mx = 0.0;
    for (uint32_t m = lane; m < f.size; m += kWave) {
        double v;
        if (f.nchunk) {
            v = 0.0;
            const double* pp = part + f.part0 + (uint64_t)m * f.nchunk;
            for (uint32_t k = 0; k < f.nchunk; k++) v += pp[k];
            acc[f.sep + m] = v;
        } else {
            v = acc[f.sep + m];
        }
        mx = fmax(mx, v);
    }
    mx = wave_max(mx);

    if (f.edge < 0) {
        if (lane == 0) {
            const double z = acc[f.sep];
            long long ks = c.kappa_total;
            for (int e = 0; e < c.ne; e++) ks += kexp[e];
            if (z > 0.0) {
                c.logpe[slot] = log(z) + 0.69314718055994530942 * (double)ks;
            } else {
                c.logpe[slot] = -INFINITY;
                atomicOr(&c.flags[slot], c.fp32 ? 2 : 1);
            }
        }
        return;
    }
    int k = 0;
    if (mx > 0.0) frexp(mx, &k);
    else if (lane == 0) atomicOr(&c.flags[slot], c.fp32 ? 2 : 1);
    const double scale = ldexp(1.0, -k);
    T* __restrict__ sepc = static_cast<T*>(c.sepc) + (uint64_t)slot * c.sep_stride;
    for (uint32_t m = lane; m < f.size; m += kWave) sepc[f.sep + m] = (T)(acc[f.sep + m] * scale);
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
template <typename T, int B>
__global__ __launch_bounds__(kBlock) void k_dist_gather(Ctx c, const DWork* __restrict__ works,
                                                        const int32_t* __restrict__ slots, int nslots) {
    __shared__ __align__(16) unsigned char stage[kStageBytes];
    __shared__ DPiece pcs[kMaxPieces];
    __shared__ DWTarget wts[kMaxPieces];
    T* vals = reinterpret_cast<T*>(stage);
    const DWork w = works[blockIdx.x];
    int sl[B];
#pragma unroll
    for (int b = 0; b < B; b++) {
        const int k = (int)blockIdx.y * B + b;
        sl[b] = k < nslots ? slots[k] : -1;
    }
    const uint32_t* __restrict__ map = c.map;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const bool packed = w.npiece > 0;

    // ---- stage: phi* = psi * parent ratio, for every slot
    DTarget tg{};
    DClique q{};
    uint32_t n;
    if (packed) {
        for (uint32_t k = threadIdx.x; k < w.npiece; k += kBlock) pcs[k] = c.pc[w.piece0 + k];
        for (uint32_t k = threadIdx.x; k < w.nwt; k += kBlock) wts[k] = c.wt[w.wt0 + k];
        __syncthreads();
        n = w.total;
    } else {
        tg = c.tg[w.target];
        q = c.cl[tg.clique];
        n = w.ng * w.nk * q.L;
    }
    uint32_t p = 0;
    int cur = -1;
    for (uint32_t gi = threadIdx.x; gi < n; gi += kBlock) {
        uint64_t ent;   // entry index within the clique
        uint32_t row, l;
        if (packed) {
            while (gi >= pcs[p].gofs + pcs[p].count) p++;
            if ((int)p != cur) {
                cur = (int)p;
                q = c.cl[pcs[p].clique];
            }
            ent = gi - pcs[p].gofs;
            row = mdiv((uint32_t)ent, q.Lmul, q.Lsh);
            l = (uint32_t)ent - row * q.L;
        } else {
            const uint32_t ri = mdiv(gi, q.Lmul, q.Lsh);
            l = gi - ri * q.L;
            const uint32_t gg = mdiv(ri, w.nkmul, w.nksh);
            const uint32_t k = ri - gg * w.nk;
            row = map[tg.rg + w.g0 + gg] + map[tg.rq + w.k0 + k];
            ent = (uint64_t)row * q.L + l;
        }
        const uint32_t pr = q.pedge >= 0 ? q.psep + map[q.pmh + row] + map[q.pml + l] : 0u;
#pragma unroll
        for (int b = 0; b < B; b++) {
            if (sl[b] < 0) continue;
            T v = static_cast<const T*>(c.psi)[(uint64_t)sl[b] * c.psi_stride + q.off + ent];
            if (q.pedge >= 0) v *= static_cast<const T*>(c.sepd)[(uint64_t)sl[b] * c.sep_stride + pr];
            vals[b * c.tile + gi] = v;
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
        uint32_t nchunk = 0;
        if (o < nout) {
            DTarget t2 = tg;
            uint32_t L = q.L, g, t, nk, rowbase;
            if (packed) {
                while (a + 1 < w.nwt && o >= wts[a + 1].out0) a++;
                const DWTarget wt = wts[a];
                t2 = c.tg[wt.target];
                const DPiece pc = pcs[wt.piece];
                L = c.cl[pc.clique].L;
                gofs = pc.gofs;
                const uint32_t oo = o - wt.out0;
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
            const uint32_t per = nk * t2.nQL;
            for (uint32_t j = sub; j < per; j += tpo) {
                const uint32_t k = j / t2.nQL;
                const uint32_t u = j - k * t2.nQL;
                const uint32_t row = packed ? map[t2.rg + g] + map[t2.rq + k] : rowbase + k;
                const uint32_t idx = gofs + row * L + lp + map[t2.lq + u];
#pragma unroll
                for (int b = 0; b < B; b++) s[b] += (double)vals[b * c.tile + idx];
            }
            sep = t2.sep;
            part0 = t2.part0;
            nchunk = t2.nchunk;
        }
#pragma unroll
        for (int b = 0; b < B; b++)
            for (uint32_t o2 = tpo / 2; o2 > 0; o2 >>= 1) s[b] += __shfl_xor(s[b], (int)o2, kWave);
        if (o < nout && sub == 0) {
#pragma unroll
            for (int b = 0; b < B; b++) {
                if (sl[b] < 0) continue;
                if (part0 < 0) c.acc[(uint64_t)sl[b] * c.sep_stride + sep + m] = s[b];
                else c.part[(uint64_t)sl[b] * c.part_stride + (uint32_t)part0 + m * nchunk + w.chunk] = s[b];
            }
        }
    }
}

// After a distribute layer, one wave per separator (real or one-variable
// virtual): finish the new separator table S* (summing partials), read the
// posterior marginals of the variables assigned to it, and for a real
// separator form the new/old ratio S*/S (0/0 = 0) rescaled by an exact
// power of two.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fin_distribute(Ctx c, const DSepFin* __restrict__ fins, uint32_t nfins,
                                                           const int32_t* __restrict__ slots) {
    const uint32_t fi = blockIdx.x * kWaves + threadIdx.x / kWave;
    if (fi >= nfins) return;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const DSepFin f = fins[fi];
    const int slot = slots[blockIdx.y];
    double* __restrict__ acc = c.acc + (uint64_t)slot * c.sep_stride;
    const double* __restrict__ part = c.part + (uint64_t)slot * c.part_stride;
    if (f.nchunk) {
        for (uint32_t m = lane; m < f.size; m += kWave) {
            double v = 0.0;
            const double* pp = part + f.part0 + (uint64_t)m * f.nchunk;
            for (uint32_t k = 0; k < f.nchunk; k++) v += pp[k];
            acc[f.sep + m] = v;
        }
        // other lanes of this wave read these sums below
        __threadfence_block();
    }
    // posteriors: each state of each assigned variable is a wave-wide sum
    // over the separator entries carrying that state
    double* __restrict__ marg = c.marg + (uint64_t)slot * c.marg_stride;
    for (uint32_t a = 0; a < f.nmv; a++) {
        const DMargVar mv = c.mv[f.mv0 + a];
        const uint32_t per = f.size / mv.card;
        for (uint32_t x = 0; x < mv.card; x++) {
            double s = 0.0;
            for (uint32_t e = lane; e < per; e += kWave) {
                const uint32_t o = e / mv.stride;
                s += acc[f.sep + (o * mv.card + x) * mv.stride + (e - o * mv.stride)];
            }
            s = wave_sum(s);
            if (lane == 0) marg[mv.out + x] = s;
        }
    }
    if (f.edge < 0) return;
    const T* __restrict__ sepc = static_cast<const T*>(c.sepc) + (uint64_t)slot * c.sep_stride;
    T* __restrict__ sepd = static_cast<T*>(c.sepd) + (uint64_t)slot * c.sep_stride;
    double mx = 0.0;
    for (uint32_t m = lane; m < f.size; m += kWave) {
        const double den = (double)sepc[f.sep + m];
        mx = fmax(mx, den == 0.0 ? 0.0 : acc[f.sep + m] / den);
    }
    mx = wave_max(mx);
    int k = 0;
    if (mx > 0.0) frexp(mx, &k);
    const double scale = ldexp(1.0, -k);
    for (uint32_t m = lane; m < f.size; m += kWave) {
        const double den = (double)sepc[f.sep + m];
        sepd[f.sep + m] = (T)((den == 0.0 ? 0.0 : acc[f.sep + m] / den) * scale);
    }
}

// Posteriors: normalise each variable's marginal.
__global__ __launch_bounds__(kBlock) void k_marginals(Ctx c, const int32_t* __restrict__ slots) {
    const int slot = slots[blockIdx.x];
    const double* marg = c.marg + (uint64_t)slot * c.marg_stride;
    double* post = c.post + (uint64_t)slot * c.marg_stride;
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

__global__ void k_begin(Ctx c, const int32_t* __restrict__ slots, int n) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n) c.flags[slots[b]] = 0;
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

template <typename T, int B>
void launch_collect_b(const Ctx& c, const DGroup* groups, uint32_t ngroups, const int32_t* slots, int nslots,
                      hipStream_t s) {
    dim3 grid(ngroups, (unsigned)((nslots + B - 1) / B));
    hipLaunchKernelGGL((k_collect<T, B>), grid, dim3(kBlock), 0, s, c, groups, slots, nslots);
}

template <typename T, int B>
void launch_gather_b(const Ctx& c, const DWork* works, uint32_t nworks, const int32_t* slots, int nslots,
                     hipStream_t s) {
    dim3 grid(nworks, (unsigned)((nslots + B - 1) / B));
    hipLaunchKernelGGL((k_dist_gather<T, B>), grid, dim3(kBlock), 0, s, c, works, slots, nslots);
}

template <typename T>
void launch_collect_t(const Ctx& c, const DGroup* groups, uint32_t ngroups, const int32_t* slots, int nslots,
                      hipStream_t s) {
    const int B = nslots >= 4 ? slots_per_block(c.tile, sizeof(T)) : 1;
    if (B >= 4) launch_collect_b<T, 4>(c, groups, ngroups, slots, nslots, s);
    else if (B == 2) launch_collect_b<T, 2>(c, groups, ngroups, slots, nslots, s);
    else launch_collect_b<T, 1>(c, groups, ngroups, slots, nslots, s);
}

template <typename T>
void launch_gather_t(const Ctx& c, const DWork* works, uint32_t nworks, const int32_t* slots, int nslots,
                     hipStream_t s) {
    const int B = nslots >= 4 ? slots_per_block(c.tile, sizeof(T)) : 1;
    if (B >= 4) launch_gather_b<T, 4>(c, works, nworks, slots, nslots, s);
    else if (B == 2) launch_gather_b<T, 2>(c, works, nworks, slots, nslots, s);
    else launch_gather_b<T, 1>(c, works, nworks, slots, nslots, s);
}

}  // namespace

hipError_t launch_collect(const Ctx& c, int prec, const DGroup* groups, uint32_t ngroups, const int32_t* slots,
                          int nslots, hipStream_t s) {
    if (!ngroups || !nslots) return hipSuccess;
    if (prec) launch_collect_t<float>(c, groups, ngroups, slots, nslots, s);
    else launch_collect_t<double>(c, groups, ngroups, slots, nslots, s);
    return hipGetLastError();
}

hipError_t launch_fin_collect(const Ctx& c, int prec, const DSepFin* fins, uint32_t nfins, const int32_t* slots,
                              int nslots, hipStream_t s) {
    if (!nfins || !nslots) return hipSuccess;
    dim3 grid((nfins + kWaves - 1) / kWaves, (unsigned)nslots);
    if (prec) hipLaunchKernelGGL(k_fin_collect<float>, grid, dim3(kBlock), 0, s, c, fins, nfins, slots);
    else hipLaunchKernelGGL(k_fin_collect<double>, grid, dim3(kBlock), 0, s, c, fins, nfins, slots);
    return hipGetLastError();
}

hipError_t launch_distribute(const Ctx& c, int prec, const DWork* works, uint32_t nworks, const int32_t* slots,
                             int nslots, hipStream_t s) {
    if (!nworks || !nslots) return hipSuccess;
    if (prec) launch_gather_t<float>(c, works, nworks, slots, nslots, s);
    else launch_gather_t<double>(c, works, nworks, slots, nslots, s);
    return hipGetLastError();
}

hipError_t launch_fin_distribute(const Ctx& c, int prec, const DSepFin* fins, uint32_t nfins, const int32_t* slots,
                                 int nslots, hipStream_t s) {
    if (!nfins || !nslots) return hipSuccess;
    dim3 grid((nfins + kWaves - 1) / kWaves, (unsigned)nslots);
    if (prec) hipLaunchKernelGGL(k_fin_distribute<float>, grid, dim3(kBlock), 0, s, c, fins, nfins, slots);
    else hipLaunchKernelGGL(k_fin_distribute<double>, grid, dim3(kBlock), 0, s, c, fins, nfins, slots);
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
