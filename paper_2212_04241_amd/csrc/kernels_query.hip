// Read-out of a joint posterior from a calibrated junction tree (gfx950).
//
// The paper's problem is the conditional probability of the query variables
// given the evidence (Section 1).  After the collect and distribute sweeps,
// the calibrated table of a clique C is proportional to P(X_C, e), so for
// query variables Q that all lie in C the joint posterior P(Q | e) is that
// table summed over C's other variables and normalised.  The calibrated
// table is not stored: every entry is rebuilt from what calibration left in
// device memory, in the order the layer kernels formed it --
//     phi*(i) = prior(i) * [evidence agrees at i]
//               * prod_children collect message(map_f(i))
//               * parent distribute ratio(pmap(i))
// -- with every sum in float64.
//
// Work split: output o (one joint assignment of Q) owns the |C| / n_out
// entries that agree with it; they are enumerated as i = base(o) + off(r)
// by mixed-radix digits, split into chunks of `chunk` consecutive r, and a
// group of tpo lanes (a power of two within one wave) sums one chunk, lanes
// striding by tpo so that consecutive lanes read consecutive entries when
// the clique's fastest variable is not a query variable.  The lane sums are
// combined by a fixed xor-shuffle tree, chunk sums are added in chunk order,
// block sums of the outputs in block order: the result does not depend on
// scheduling, and a call returns the same bits every time.
//
// Scratch: the chunk sums (when an output has more than one chunk), the
// unnormalised outputs and the block sums live in a device buffer that the
// caller provides -- allocated per call by the library, or, for callers
// that cannot allocate, the file-scope array `scratch` below.  Every value
// the kernels read from it is written earlier in the same call, so nothing
// needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace fbn {

// Device memory for the allocation-free joint read-out: one copy per GPU,
// held until the process ends.  Host code never passes this name to a
// kernel or a copy; it uses the address hipGetSymbolAddress returns for the
// current device (joint_static_scratch).
static __device__ __align__(256) double scratch[kJointScratchDoubles];

namespace {

constexpr int kWaveQ = 64;
constexpr int kBlockQ = 256;

__device__ __forceinline__ uint32_t mdiv_q(uint32_t n, uint32_t mul, uint32_t sh) {
    return (uint32_t)(((uint64_t)__umulhi(n, mul) + n) >> sh);
}

// x taken apart into the digits of vars[0..n) (fastest first), each digit
// times the variable's stride in the clique table, summed.
__device__ __forceinline__ uint32_t compose(uint32_t x, const JointVar* vars, uint32_t n) {
    uint32_t i = 0;
    for (uint32_t k = 0; k < n; k++) {
        const uint32_t q = mdiv_q(x, vars[k].cmul, vars[k].csh);
        i += (x - q * vars[k].card) * vars[k].stride;
        x = q;
    }
    return i;
}

// Entry x of a per-slot array: slot-interleaved (x * S + slot) or slot-major.
__device__ __forceinline__ uint64_t slot_index(const Ctx& c, uint32_t x, uint64_t slot, uint32_t stride) {
    return c.S ? (uint64_t)x * c.S + slot : slot * stride + x;
}

template <typename T>
__device__ __forceinline__ double calibrated_entry(const Ctx& c, const DClique& q, const DEvidence& ev,
                                                   uint64_t slot, uint32_t i) {
    const uint32_t hi = mdiv_q(i, q.Lmul, q.Lsh);
    const uint32_t lo = i - hi * q.L;
    if (ev.mask) {
        const uint64_t d = c.dig[q.hdig + hi] | c.dig[q.ldig + lo];
        if ((d ^ ev.want) & ev.mask) return 0.0;
    }
    const T* __restrict__ sepc = static_cast<const T*>(c.sepc);
    const T* __restrict__ sepd = static_cast<const T*>(c.sepd);
    const uint32_t* __restrict__ map = c.map;
    T v = static_cast<const T*>(c.prior)[q.off + i];
    for (uint32_t k = 0; k < q.nchild; k++) {
        const DChild ch = c.ch[q.child0 + k];
        v *= sepc[slot_index(c, ch.sep + map[ch.mh + hi] + map[ch.ml + lo], slot, c.sep_stride)];
    }
    if (q.pedge >= 0) v *= sepd[slot_index(c, q.psep + map[q.pmh + hi] + map[q.pml + lo], slot, c.sep_stride)];
    return (double)v;
}

// Chunk sums: item (o, ch) -> dst[o * nchunk + ch].
template <typename T>
__global__ __launch_bounds__(kBlockQ) void k_joint_sum(Ctx c, DClique q, JointArgs a, double* __restrict__ dst) {
    const uint64_t t = (uint64_t)blockIdx.x * kBlockQ + threadIdx.x;
    const uint64_t item = t / a.tpo;
    const uint32_t sub = (uint32_t)(t % a.tpo);
    const uint64_t items = (uint64_t)a.n_out * a.nchunk;
    const uint64_t slot = (uint64_t)a.slot;
    double s = 0.0;
    if (item < items) {
        const uint32_t o = (uint32_t)(item / a.nchunk);
        const uint32_t ch = (uint32_t)(item % a.nchunk);
        const DEvidence ev = c.ev[slot * c.ev_stride + a.clique];
        const uint32_t base = compose(o, a.qv, a.nq);
        const uint32_t r0 = ch * a.chunk;
        const uint32_t r1 = min(r0 + a.chunk, a.n_r);
        for (uint32_t r = r0 + sub; r < r1; r += a.tpo)
            s += calibrated_entry<T>(c, q, ev, slot, base + compose(r, a.ov, a.no));
    }
    for (uint32_t o2 = a.tpo / 2; o2 > 0; o2 >>= 1) s += __shfl_xor(s, (int)o2, kWaveQ);
    if (item < items && sub == 0) dst[item] = s;
}

__device__ __forceinline__ double block_sum_q(double v, double* red) {
#pragma unroll
    for (int o = kWaveQ / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWaveQ);
    const int lane = threadIdx.x & (kWaveQ - 1), w = threadIdx.x / kWaveQ;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kBlockQ / kWaveQ; k++) s += red[k];
    return s;
}

// Output sums (chunk sums added in chunk order) and one sum per block.
__global__ __launch_bounds__(kBlockQ) void k_joint_fold(const double* __restrict__ part, double* __restrict__ out,
                                                        double* __restrict__ zb, uint32_t n_out, uint32_t nchunk) {
    __shared__ double red[kBlockQ / kWaveQ];
    const uint32_t o = blockIdx.x * kBlockQ + threadIdx.x;
    double m = 0.0;
    if (o < n_out) {
        if (nchunk > 1) {
            const double* p = part + (uint64_t)o * nchunk;
            for (uint32_t k = 0; k < nchunk; k++) m += p[k];
            out[o] = m;
        } else {
            m = out[o];
        }
    }
    m = block_sum_q(m, red);
    if (threadIdx.x == 0) zb[blockIdx.x] = m;
}

// Normalise: every block forms the same total from the block sums, in the
// same order, and divides its outputs by it.
__global__ __launch_bounds__(kBlockQ) void k_joint_norm(double* __restrict__ out, const double* __restrict__ zb,
                                                        uint32_t n_out, uint32_t nb) {
    __shared__ double red[kBlockQ / kWaveQ];
    double z = 0.0;
    for (uint32_t k = threadIdx.x; k < nb; k += kBlockQ) z += zb[k];
    z = block_sum_q(z, red);
    const uint32_t o = blockIdx.x * kBlockQ + threadIdx.x;
    if (o < n_out) out[o] = z > 0.0 ? out[o] / z : 0.0;
}

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
double* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

size_t joint_scratch_doubles(const JointArgs& a) {
    const uint64_t nb = ((uint64_t)a.n_out + kBlockQ - 1) / kBlockQ;
    return (size_t)((uint64_t)a.n_out + nb + (a.nchunk > 1 ? (uint64_t)a.n_out * a.nchunk : 0));
}

hipError_t launch_joint(const Ctx& c, int prec, const DClique& q, const JointArgs& a, double* scratch_dev,
                        hipStream_t s) {
    const uint32_t nb = (a.n_out + kBlockQ - 1) / kBlockQ;
    double* out = scratch_dev;
    double* zb = out + a.n_out;
    double* part = zb + nb;
    double* dst = a.nchunk > 1 ? part : out;
    const uint64_t threads = (uint64_t)a.n_out * a.nchunk * a.tpo;
    const uint64_t blocks = (threads + kBlockQ - 1) / kBlockQ;
    if (!blocks || blocks > 0x7fffffffull) return hipErrorInvalidValue;
    if (prec)
        hipLaunchKernelGGL(k_joint_sum<float>, dim3((unsigned)blocks), dim3(kBlockQ), 0, s, c, q, a, dst);
    else
        hipLaunchKernelGGL(k_joint_sum<double>, dim3((unsigned)blocks), dim3(kBlockQ), 0, s, c, q, a, dst);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_joint_fold, dim3(nb), dim3(kBlockQ), 0, s, part, out, zb, a.n_out, a.nchunk);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_joint_norm, dim3(nb), dim3(kBlockQ), 0, s, out, zb, a.n_out, nb);
    return hipGetLastError();
}

hipError_t joint_static_scratch(double** ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace fbn
