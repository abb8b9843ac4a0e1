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
//     scattered into every child separator and every home variable's
//     marginal (marginalisation onto non-contiguous index sets).
//   distribute finalise: Rd = S_new / S_old (0/0 = 0), rescaled.
//
// The tables stream through HBM once per layer pass (coalesced runs of
// consecutive entries); index maps come from small factored tables
// (H[hi] + L[lo]) that stay in cache; all arithmetic on the separator
// sums and the scale factors is float64.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace fbn {
namespace {

constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;

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

// Block-wide reductions; every thread gets the result.
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

__device__ __forceinline__ double block_max(double v, double* scratch) {
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

// ------------------------------------------------------------------ collect

template <typename T>
__global__ __launch_bounds__(kBlock) void k_collect(Ctx c, const DGroup* __restrict__ groups,
                                                    const int32_t* __restrict__ slots) {
    __shared__ T vals[kTileMax];
    __shared__ DPiece pcs[kMaxPieces];
    __shared__ double red[kWaves];
    const DGroup g = groups[blockIdx.x];
    const int slot = slots[blockIdx.y];
    for (uint32_t k = threadIdx.x; k < g.npiece; k += kBlock) pcs[k] = c.pc[g.piece0 + k];
    __syncthreads();

    const T* __restrict__ prior = static_cast<const T*>(c.prior);
    T* __restrict__ psi = static_cast<T*>(c.psi) + (uint64_t)slot * c.psi_stride;
    const T* __restrict__ sepc = static_cast<const T*>(c.sepc) + (uint64_t)slot * c.sep_stride;
    const DEvidence* __restrict__ ev = c.ev + (uint64_t)slot * c.ev_stride;

    uint32_t p = 0;
    int cur = -1;
    DClique q{};
    DEvidence e{};
    for (uint32_t gi = threadIdx.x; gi < g.total; gi += kBlock) {
        while (gi >= pcs[p].gofs + pcs[p].count) p++;
        if ((int)p != cur) {
            cur = (int)p;
            q = c.cl[pcs[p].clique];
            e = ev[pcs[p].clique];
        }
        const uint32_t i = pcs[p].begin + (gi - pcs[p].gofs);
        const uint32_t hi = mdiv(i, q.Lmul, q.Lsh);
        const uint32_t lo = i - hi * q.L;
        T v = prior[q.off + i];
        if (e.mask) {
            const uint64_t d = c.dig[q.hdig + hi] | c.dig[q.ldig + lo];
            if ((d ^ e.want) & e.mask) v = T(0);
        }
        for (uint32_t k = 0; k < q.nchild; k++) {
            const DChild ch = c.ch[q.child0 + k];
            v *= sepc[ch.sep + c.map[ch.mh + hi] + c.map[ch.ml + lo]];
        }
        psi[q.off + i] = v;
        vals[gi] = v;
    }
    __syncthreads();

    // marginalise onto the parent separator: contiguous segments of q.seg
    double* __restrict__ acc = c.acc + (uint64_t)slot * c.sep_stride;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (g.part >= 0) {
        double s = 0.0;
        for (uint32_t k = threadIdx.x; k < g.total; k += kBlock) s += (double)vals[k];
        s = block_sum(s, red);
        if (threadIdx.x == 0) c.part[(uint64_t)slot * c.part_stride + (uint32_t)g.part] = s;
        return;
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
                for (uint32_t k = (uint32_t)lane; k < seg; k += kWave) a += (double)vals[pc.gofs + s * seg + k];
                a = wave_sum(a);
                if (lane == 0) acc[out0 + s] = a;
            }
        } else {
            for (uint32_t s = threadIdx.x; s < nseg; s += kBlock) {
                double a = 0.0;
                for (uint32_t k = 0; k < seg; k++) a += (double)vals[pc.gofs + s * seg + k];
                acc[out0 + s] = a;
            }
        }
    }
}

// After a collect layer: finish each separator message (sum partial sums
// where a segment spanned several tiles), rescale it by an exact power of two
// so its largest entry lies in [0.5, 1), store it in table precision, record
// the exponent, and clear the float64 accumulator for the distribute sweep.
// The root's one-entry virtual separator yields log P(e).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fin_collect(Ctx c, const DSepFin* __restrict__ fins,
                                                        const int32_t* __restrict__ slots) {
    __shared__ double red[kWaves];
    const DSepFin f = fins[blockIdx.x];
    const int slot = slots[blockIdx.y];
    double* __restrict__ acc = c.acc + (uint64_t)slot * c.sep_stride;
    const double* __restrict__ part = c.part + (uint64_t)slot * c.part_stride;
    int32_t* kexp = c.kexp + (uint64_t)slot * c.kexp_stride;

    double mx = 0.0;
    for (uint32_t m = threadIdx.x; m < f.size; m += kBlock) {
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
    mx = block_max(mx, red);

    if (f.edge < 0) {
        if (threadIdx.x == 0) {
            const double z = acc[f.sep];
            acc[f.sep] = 0.0;
            long long ks = c.kappa_total;
            for (int e = 0; e < c.ne; e++) ks += kexp[e];
            if (z > 0.0) {
                c.logpe[slot] = log(z) + 0.69314718055994530942 * (double)ks;
            } else {
                c.logpe[slot] = -INFINITY;
                c.flags[slot] |= c.fp32 ? 2 : 1;
            }
        }
        return;
    }
    int k = 0;
    if (mx > 0.0) {
        frexp(mx, &k);
    } else if (threadIdx.x == 0) {
        c.flags[slot] |= c.fp32 ? 2 : 1;
    }
    const double scale = ldexp(1.0, -k);
    T* __restrict__ sepc = static_cast<T*>(c.sepc) + (uint64_t)slot * c.sep_stride;
    for (uint32_t m = threadIdx.x; m < f.size; m += kBlock) sepc[f.sep + m] = (T)(acc[f.sep + m] * scale);
    if (threadIdx.x == 0) kexp[f.edge] = k;
}

// --------------------------------------------------------------- distribute

// One workgroup marginalises a block of one clique onto one target
// separator: it stages ng groups x nk rows of the clique (each row L
// consecutive entries, read coalesced and extended by the parent's
// distribute ratio on the way in) in LDS, then every separator entry of the
// block is summed by a fixed set of lanes in a fixed order -- no atomics,
// so results do not depend on scheduling.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dist_gather(Ctx c, const DWork* __restrict__ works,
                                                        const int32_t* __restrict__ slots) {
    __shared__ T vals[kTileMax];
    const DWork w = works[blockIdx.x];
    const int slot = slots[blockIdx.y];
    const DTarget tg = c.tg[w.target];
    const DClique q = c.cl[tg.clique];
    const T* __restrict__ psi = static_cast<const T*>(c.psi) + (uint64_t)slot * c.psi_stride + q.off;
    const T* __restrict__ sepd = static_cast<const T*>(c.sepd) + (uint64_t)slot * c.sep_stride;
    const uint32_t* __restrict__ map = c.map;

    const uint32_t n = w.ng * w.nk * q.L;
    for (uint32_t idx = threadIdx.x; idx < n; idx += kBlock) {
        const uint32_t ri = mdiv(idx, q.Lmul, q.Lsh);
        const uint32_t l = idx - ri * q.L;
        const uint32_t gg = mdiv(ri, w.nkmul, w.nksh);
        const uint32_t k = ri - gg * w.nk;
        const uint32_t row = map[tg.rg + w.g0 + gg] + map[tg.rq + w.k0 + k];
        T v = psi[row * q.L + l];
        if (q.pedge >= 0) v *= sepd[q.psep + map[q.pmh + row] + map[q.pml + l]];
        vals[idx] = v;
    }
    __syncthreads();

    // outputs (gg, t); tpo lanes per output, power of two within a wave
    const uint32_t nout = w.ng * tg.nPL;
    uint32_t tpo = 1;
    while (tpo < 64 && tpo * 2 * nout <= (uint32_t)kBlock) tpo *= 2;
    const uint32_t sub = threadIdx.x & (tpo - 1);
    const uint32_t per = w.nk * tg.nQL;  // summands of one output
    double* __restrict__ acc = c.acc + (uint64_t)slot * c.sep_stride;
    double* __restrict__ part = c.part + (uint64_t)slot * c.part_stride;
    for (uint32_t base = 0; base < nout * tpo; base += kBlock) {
        const uint32_t o = (base + threadIdx.x) / tpo;
        double s = 0.0;
        uint32_t gg = 0, t = 0;
        if (o < nout) {
            gg = o / tg.nPL;
            t = o - gg * tg.nPL;
            const uint32_t lp = map[tg.lp + t];
            for (uint32_t j = sub; j < per; j += tpo) {
                const uint32_t k = j / tg.nQL;
                const uint32_t u = j - k * tg.nQL;
                s += (double)vals[(gg * w.nk + k) * q.L + lp + map[tg.lq + u]];
            }
        }
        for (uint32_t o2 = tpo / 2; o2 > 0; o2 >>= 1) s += __shfl_xor(s, (int)o2, kWave);
        if (o < nout && sub == 0) {
            const uint32_t m = map[tg.tb + w.g0 + gg] + map[tg.tv + t];
            if (tg.part0 < 0) acc[tg.sep + m] = s;
            else part[(uint32_t)tg.part0 + m * tg.nchunk + w.chunk] = s;
        }
    }
}

// After a distribute layer, per separator (real or one-variable virtual):
// finish the new separator table S* (summing partials), read the posterior
// marginals of the variables assigned to it, and for a real separator form
// the new/old ratio S*/S (0/0 = 0) rescaled by an exact power of two.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fin_distribute(Ctx c, const DSepFin* __restrict__ fins,
                                                           const int32_t* __restrict__ slots) {
    __shared__ double red[kWaves];
    const DSepFin f = fins[blockIdx.x];
    const int slot = slots[blockIdx.y];
    double* __restrict__ acc = c.acc + (uint64_t)slot * c.sep_stride;
    const double* __restrict__ part = c.part + (uint64_t)slot * c.part_stride;
    if (f.nchunk) {
        for (uint32_t m = threadIdx.x; m < f.size; m += kBlock) {
            double v = 0.0;
            const double* pp = part + f.part0 + (uint64_t)m * f.nchunk;
            for (uint32_t k = 0; k < f.nchunk; k++) v += pp[k];
            acc[f.sep + m] = v;
        }
        __syncthreads();
    }
    // posteriors: each state of each assigned variable is a block-wide sum
    // over the separator entries carrying that state
    double* __restrict__ marg = c.marg + (uint64_t)slot * c.marg_stride;
    for (uint32_t a = 0; a < f.nmv; a++) {
        const DMargVar mv = c.mv[f.mv0 + a];
        const uint32_t per = f.size / mv.card;
        for (uint32_t x = 0; x < mv.card; x++) {
            double s = 0.0;
            for (uint32_t e = threadIdx.x; e < per; e += kBlock) {
                const uint32_t o = e / mv.stride;
                s += acc[f.sep + (o * mv.card + x) * mv.stride + (e - o * mv.stride)];
            }
            s = block_sum(s, red);
            if (threadIdx.x == 0) marg[mv.out + x] = s;
        }
    }
    if (f.edge < 0) return;
    const T* __restrict__ sepc = static_cast<const T*>(c.sepc) + (uint64_t)slot * c.sep_stride;
    T* __restrict__ sepd = static_cast<T*>(c.sepd) + (uint64_t)slot * c.sep_stride;
    double mx = 0.0;
    for (uint32_t m = threadIdx.x; m < f.size; m += kBlock) {
        const double den = (double)sepc[f.sep + m];
        const double r = den == 0.0 ? 0.0 : acc[f.sep + m] / den;
        mx = fmax(mx, r);
    }
    mx = block_max(mx, red);
    int k = 0;
    if (mx > 0.0) frexp(mx, &k);
    const double scale = ldexp(1.0, -k);
    for (uint32_t m = threadIdx.x; m < f.size; m += kBlock) {
        const double den = (double)sepc[f.sep + m];
        const double r = den == 0.0 ? 0.0 : acc[f.sep + m] / den;
        sepd[f.sep + m] = (T)(r * scale);
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

}  // namespace

hipError_t launch_collect(const Ctx& c, int prec, const DGroup* groups, uint32_t ngroups, const int32_t* slots,
                          int nslots, hipStream_t s) {
    if (!ngroups || !nslots) return hipSuccess;
    dim3 grid(ngroups, (unsigned)nslots);
    if (prec) hipLaunchKernelGGL(k_collect<float>, grid, dim3(kBlock), 0, s, c, groups, slots);
    else hipLaunchKernelGGL(k_collect<double>, grid, dim3(kBlock), 0, s, c, groups, slots);
    return hipGetLastError();
}

hipError_t launch_fin_collect(const Ctx& c, int prec, const DSepFin* fins, uint32_t nfins, const int32_t* slots,
                              int nslots, hipStream_t s) {
    if (!nfins || !nslots) return hipSuccess;
    dim3 grid(nfins, (unsigned)nslots);
    if (prec) hipLaunchKernelGGL(k_fin_collect<float>, grid, dim3(kBlock), 0, s, c, fins, slots);
    else hipLaunchKernelGGL(k_fin_collect<double>, grid, dim3(kBlock), 0, s, c, fins, slots);
    return hipGetLastError();
}

hipError_t launch_distribute(const Ctx& c, int prec, const DWork* works, uint32_t nworks, const int32_t* slots,
                             int nslots, hipStream_t s) {
    if (!nworks || !nslots) return hipSuccess;
    dim3 grid(nworks, (unsigned)nslots);
    if (prec) hipLaunchKernelGGL(k_dist_gather<float>, grid, dim3(kBlock), 0, s, c, works, slots);
    else hipLaunchKernelGGL(k_dist_gather<double>, grid, dim3(kBlock), 0, s, c, works, slots);
    return hipGetLastError();
}

hipError_t launch_fin_distribute(const Ctx& c, int prec, const DSepFin* fins, uint32_t nfins, const int32_t* slots,
                                 int nslots, hipStream_t s) {
    if (!nfins || !nslots) return hipSuccess;
    dim3 grid(nfins, (unsigned)nslots);
    if (prec) hipLaunchKernelGGL(k_fin_distribute<float>, grid, dim3(kBlock), 0, s, c, fins, slots);
    else hipLaunchKernelGGL(k_fin_distribute<double>, grid, dim3(kBlock), 0, s, c, fins, slots);
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
