// C ABI of the junction-tree library: network loading and validation, tree
// compilation and device upload, evidence slots, the layer-by-layer launch
// sequence, and result retrieval.  See include/fbn.h for the contract.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/fbn.h"
#include "fbn_internal.h"
#include "kernels.h"
#include "plan.h"

using namespace fbn;

namespace {

thread_local std::string g_err;

fbn_status fail(fbn_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define HIP_OK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(FBN_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------ net validation

fbn_status check_net(Net& net) {
    const int n = net.n;
    for (int v = 0; v < n; v++) {
        if (net.card[v] < 2 || net.card[v] > 65535) return fail(FBN_E_INVALID_ARG, "variable " + std::to_string(v) + ": cardinality out of range");
        for (size_t a = 0; a < net.parents[v].size(); a++) {
            int p = net.parents[v][a];
            if (p < 0 || p >= n || p == v) return fail(FBN_E_INVALID_ARG, "variable " + std::to_string(v) + ": bad parent");
            for (size_t b = 0; b < a; b++)
                if (net.parents[v][b] == p) return fail(FBN_E_INVALID_ARG, "variable " + std::to_string(v) + ": repeated parent");
        }
    }
    // acyclicity by repeatedly removing variables with no remaining parents
    std::vector<int> indeg(n, 0);
    std::vector<std::vector<int>> kids(n);
    for (int v = 0; v < n; v++) {
        indeg[v] = (int)net.parents[v].size();
        for (int p : net.parents[v]) kids[p].push_back(v);
    }
    std::vector<int> ready;
    for (int v = 0; v < n; v++)
        if (!indeg[v]) ready.push_back(v);
    int done = 0;
    while (!ready.empty()) {
        int v = ready.back();
        ready.pop_back();
        done++;
        for (int k : kids[v])
            if (--indeg[k] == 0) ready.push_back(k);
    }
    if (done != n) return fail(FBN_E_INVALID_ARG, "the network has a directed cycle");
    for (int v = 0; v < n; v++) {
        if (net.cpt[v].empty()) continue;
        uint64_t len = (uint64_t)net.card[v];
        for (int p : net.parents[v]) len *= (uint64_t)net.card[p];
        if (net.cpt[v].size() != len) return fail(FBN_E_INVALID_ARG, "variable " + std::to_string(v) + ": CPT length");
        const int r = net.card[v];
        for (uint64_t row = 0; row < len / (uint64_t)r; row++) {
            double s = 0.0;
            for (int x = 0; x < r; x++) {
                double val = net.cpt[v][row * (uint64_t)r + (uint64_t)x];
                if (!std::isfinite(val) || val < 0.0) return fail(FBN_E_INVALID_ARG, "variable " + std::to_string(v) + ": CPT entry not finite and non-negative");
                s += val;
            }
            if (std::fabs(s - 1.0) > 1e-9) return fail(FBN_E_INVALID_ARG, "variable " + std::to_string(v) + ": CPT row does not sum to 1");
        }
    }
    return FBN_OK;
}

// whitespace tokenizer over an in-memory text
struct Lexer {
    const char* p;
    const char* end;
    bool next(std::string& tok) {
        while (p < end && (*p == ' ' || *p == '\n' || *p == '\t' || *p == '\r')) p++;
        if (p >= end) return false;
        const char* s = p;
        while (p < end && !(*p == ' ' || *p == '\n' || *p == '\t' || *p == '\r')) p++;
        tok.assign(s, (size_t)(p - s));
        return true;
    }
    bool integer(long long& x) {
        std::string t;
        if (!next(t)) return false;
        char* e = nullptr;
        errno = 0;
        x = std::strtoll(t.c_str(), &e, 10);
        return errno == 0 && e && *e == 0;
    }
    bool real(double& x) {
        std::string t;
        if (!next(t)) return false;
        char* e = nullptr;
        x = std::strtod(t.c_str(), &e);
        return e && *e == 0;
    }
};

fbn_status parse_net(const char* text, size_t len, Net& net) {
    Lexer lx{text, text + len};
    std::string t;
    long long x = 0, n = 0;
    if (!lx.next(t) || t != "fbn" || !lx.integer(x) || x != 1) return fail(FBN_E_PARSE, "expected 'fbn 1'");
    if (!lx.next(t) || t != "vars" || !lx.integer(n) || n <= 0 || n > 1000000) return fail(FBN_E_PARSE, "expected 'vars n'");
    net.n = (int)n;
    net.card.assign((size_t)n, 0);
    net.parents.assign((size_t)n, {});
    net.cpt.assign((size_t)n, {});
    std::vector<char> declared((size_t)n, 0), has_cpt((size_t)n, 0);
    for (;;) {
        if (!lx.next(t)) return fail(FBN_E_PARSE, "missing 'end'");
        if (t == "end") break;
        if (t == "var") {
            long long v, r, k;
            if (!lx.integer(v) || !lx.integer(r) || !lx.integer(k) || v < 0 || v >= n || k < 0 || k > n || declared[(size_t)v])
                return fail(FBN_E_PARSE, "bad 'var' record");
            declared[(size_t)v] = 1;
            net.card[(size_t)v] = (int)r;
            for (long long i = 0; i < k; i++) {
                long long p;
                if (!lx.integer(p)) return fail(FBN_E_PARSE, "bad parent list");
                net.parents[(size_t)v].push_back((int)p);
            }
        } else if (t == "cpt") {
            long long v, m;
            if (!lx.integer(v) || !lx.integer(m) || v < 0 || v >= n || m <= 0 || has_cpt[(size_t)v])
                return fail(FBN_E_PARSE, "bad 'cpt' record");
            has_cpt[(size_t)v] = 1;
            auto& vals = net.cpt[(size_t)v];
            vals.resize((size_t)m);
            for (long long i = 0; i < m; i++)
                if (!lx.real(vals[(size_t)i])) return fail(FBN_E_PARSE, "bad or missing CPT value");
        } else {
            return fail(FBN_E_PARSE, "unknown record '" + t + "'");
        }
    }
    for (long long v = 0; v < n; v++)
        if (!declared[(size_t)v] || !has_cpt[(size_t)v]) return fail(FBN_E_PARSE, "variable " + std::to_string(v) + " incomplete");
    for (long long v = 0; v < n; v++) {
        uint64_t want = (uint64_t)std::max(net.card[(size_t)v], 0);
        for (int p : net.parents[(size_t)v]) {
            if (p < 0 || p >= n) return fail(FBN_E_PARSE, "bad parent id");
            want *= (uint64_t)std::max(net.card[(size_t)p], 0);
        }
        if (net.cpt[(size_t)v].size() != want) return fail(FBN_E_PARSE, "variable " + std::to_string(v) + ": CPT length");
    }
    return check_net(net);
}

}  // namespace

struct fbn_net {
    Net net;
    // declared names (BIF); empty for .fbn text, whose variables are named
    // by their ids and states by their indices
    std::vector<std::string> names;
    std::vector<std::vector<std::string>> states;
};

// ------------------------------------------------------------------ jt state

struct fbn_jt {
    fbn_jt_options opt{};
    Tree tree;
    Plan plan;
    int device = -1;
    hipStream_t stream = nullptr;
    std::vector<void*> allocs;
    // device plan
    DClique* d_cl = nullptr;
    DChild* d_ch = nullptr;
    DTarget* d_tg = nullptr;
    DMargVar* d_mv = nullptr;
    DWork* d_works = nullptr;
    DWTarget* d_wt = nullptr;
    DPiece* d_pc = nullptr;
    DHomeVar* d_hv = nullptr;
    DGroup* d_groups = nullptr;
    DSepFin* d_fins = nullptr;
    DFinBlk* d_finblks = nullptr;
    uint64_t* d_dig = nullptr;
    uint32_t* d_map = nullptr;
    void* d_prior = nullptr;
    // per-slot state
    void* d_psi = nullptr;
    void* d_sepc = nullptr;
    void* d_sepd = nullptr;
    void* d_acc = nullptr;   // separator sums and partial sums, table precision
    void* d_part = nullptr;
    int32_t* d_kexp = nullptr;
    double* d_marg = nullptr;
    double* d_post = nullptr;
    double* d_logpe = nullptr;
    int32_t* d_flags = nullptr;
    DEvidence* d_ev = nullptr;
    double* d_bmax = nullptr;
    double* d_bmarg = nullptr;
    double* d_rsum = nullptr;   // per slot: root sums in float64
    int32_t* d_slots = nullptr;
    double* d_out_post = nullptr;
    double* d_out_logpe = nullptr;
    int32_t* d_out_flags = nullptr;
    // host staging (pinned when a device is present)
    DEvidence* h_ev = nullptr;
    int32_t* h_slots = nullptr;
    bool h_pinned = false;
    std::vector<char> dirty;
    std::vector<int32_t> staged_slots;  // the slot list now in d_slots
    std::vector<std::vector<std::pair<int32_t, int32_t>>> evidence;  // per slot: (variable, state)
    fbn_jt* twin = nullptr;             // FP32 with fp64_rerun: one-slot FP64 tree of the same network
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
    // evidence lookup: for each variable, the (clique, layout position) pairs
    std::vector<std::vector<std::pair<int, int>>> occ;
    Ctx ctx{};
    uint64_t device_bytes = 0, slot_bytes = 0;
    // graph mode: one captured launch sequence per batch size
    bool use_graph = false;
    std::map<int, hipGraphExec_t> graphs;
    // kernel timing
    struct Rec {
        hipEvent_t a, b;
        int kind;
        double bytes;
    };
    bool prof = false;
    uint32_t prof_mask = (1u << FBN_PROFILE_KINDS) - 1;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    double prof_ms[FBN_PROFILE_KINDS] = {}, prof_bytes[FBN_PROFILE_KINDS] = {};
    int64_t prof_n[FBN_PROFILE_KINDS] = {};
    // per layer: table entries, and separator entries finalised after it
    std::vector<uint64_t> coll_entries, coll_sep, dist_entries, dist_sep;
    // per slot and layer: the table entries its evidence leaves live (the
    // bytes the per-slot layout streams with shrink_evidence)
    std::vector<uint64_t> live_coll, live_dist;
};

namespace {

void* dev_alloc(fbn_jt* jt, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (jt->opt.allocator.alloc) {
        p = jt->opt.allocator.alloc(jt->opt.allocator.ctx, bytes, jt->stream);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) {
        jt->allocs.push_back(p);
        jt->device_bytes += bytes;
    }
    return p;
}

void release(fbn_jt* jt) {
    if (jt->device >= 0) {
        hipSetDevice(jt->device);
        hipStreamSynchronize(jt->stream);
        for (void* p : jt->allocs) {
            if (jt->opt.allocator.alloc) {
                if (jt->opt.allocator.free) jt->opt.allocator.free(jt->opt.allocator.ctx, p, jt->stream);
            } else {
                hipFree(p);
            }
        }
        if (jt->staged) hipEventDestroy(jt->staged);
        for (auto& kv : jt->graphs) hipGraphExecDestroy(kv.second);
        jt->graphs.clear();
        for (auto& r : jt->recs) {
            hipEventDestroy(r.a);
            hipEventDestroy(r.b);
        }
        for (hipEvent_t e : jt->pool) hipEventDestroy(e);
        jt->recs.clear();
        jt->pool.clear();
    }
    jt->allocs.clear();
    if (jt->h_pinned) {
        if (jt->h_ev) hipHostFree(jt->h_ev);
        if (jt->h_slots) hipHostFree(jt->h_slots);
    } else {
        std::free(jt->h_ev);
        std::free(jt->h_slots);
    }
    jt->h_ev = nullptr;
    jt->h_slots = nullptr;
}

template <typename V>
fbn_status upload(fbn_jt* jt, const std::vector<V>& src, V*& dst) {
    dst = static_cast<V*>(dev_alloc(jt, sizeof(V) * std::max<size_t>(src.size(), 1)));
    if (!dst) return fail(FBN_E_NOMEM_DEVICE, "device allocation failed");
    if (!src.empty()) HIP_OK(hipMemcpyAsync(dst, src.data(), sizeof(V) * src.size(), hipMemcpyHostToDevice, jt->stream));
    return FBN_OK;
}

fbn_status wait_staged(fbn_jt* jt) {
    if (jt->staged_pending) {
        HIP_OK(hipEventSynchronize(jt->staged));
        jt->staged_pending = false;
    }
    return FBN_OK;
}

// Per-slot strides and the bytes one slot adds to each per-slot buffer, in
// allocation order.
constexpr int kSlotBuffers = 18;

struct SlotLayout {
    uint64_t psi_stride;
    uint32_t part_stride, kexp_stride, marg_stride, ev_stride, bmax_stride, bmarg_stride;
    size_t unit[kSlotBuffers];
};

SlotLayout slot_layout(const fbn_jt* jt) {
    const Plan& p = jt->plan;
    const size_t w = jt->opt.precision == FBN_FP32_RESCALED ? 4 : 8;
    SlotLayout L{};
    L.psi_stride = std::max<uint64_t>((p.psi_total + 63) / 64 * 64, 64);
    L.part_stride = (p.n_parts + 63) / 64 * 64 + 64;
    L.kexp_stride = (uint32_t)((jt->tree.ne + 1 + 63) / 64 * 64);
    L.marg_stride = p.marg_total;
    L.ev_stride = (uint32_t)jt->tree.nc;
    // per-slot layout: one maximum per block; interleaved: one per large separator
    L.bmax_stride = (uint32_t)std::max<size_t>(p.interleaved ? p.n_bigfin : p.finblks.size(), 1);
    L.bmarg_stride = std::max<uint32_t>(p.n_bmarg, 1);
    // separator sums and partial sums are stored in table precision
    const size_t u[kSlotBuffers] = {w * L.psi_stride, w * p.sep_stride, w * p.sep_stride, w * p.sep_stride,
                                    w * L.part_stride, 4ull * L.kexp_stride, 8ull * L.marg_stride,
                                    8ull * L.marg_stride, 8, 4, sizeof(DEvidence) * L.ev_stride, 4,
                                    8ull * L.marg_stride, 8, 4, 8ull * L.bmax_stride, 8ull * L.bmarg_stride,
                                    8ull * std::max<uint32_t>(p.n_roots, 1)};
    std::copy(u, u + kSlotBuffers, L.unit);
    return L;
}

// Device bytes a jt holds (the plan, the prior and max_slots slots), as
// setup_device allocates them; slot_bytes receives the per-slot share.
uint64_t footprint(const fbn_jt* jt, uint64_t& slot_bytes) {
    const Plan& p = jt->plan;
    auto b = [](const auto& v) { return (uint64_t)sizeof(v[0]) * std::max<uint64_t>(v.size(), 1); };
    uint64_t fixed = b(p.cliques) + b(p.children) + b(p.targets) + b(p.margvars) + b(p.works) + b(p.wtargets) +
                     b(p.pieces) + b(p.homevars) + b(p.groups) + b(p.fins) + b(p.finblks) + b(p.digits) +
                     b(p.maps);
    fixed += (jt->opt.precision == FBN_FP32_RESCALED ? 4ull : 8ull) * std::max<uint64_t>(p.T, 1);
    const SlotLayout L = slot_layout(jt);
    slot_bytes = 0;
    for (size_t u : L.unit) slot_bytes += u;
    return fixed + slot_bytes * (uint64_t)jt->opt.max_slots;
}

fbn_status setup_device(fbn_jt* jt) {
    Plan& p = jt->plan;
    const int S = jt->opt.max_slots;
    const bool f32 = jt->opt.precision == FBN_FP32_RESCALED;
    const size_t w = f32 ? 4 : 8;
    HIP_OK(hipGetDevice(&jt->device));
    jt->stream = static_cast<hipStream_t>(jt->opt.stream);
    HIP_OK(hipEventCreateWithFlags(&jt->staged, hipEventDisableTiming));
    fbn_status st;
    if ((st = upload(jt, p.cliques, jt->d_cl))) return st;
    if ((st = upload(jt, p.children, jt->d_ch))) return st;
    if ((st = upload(jt, p.targets, jt->d_tg))) return st;
    if ((st = upload(jt, p.margvars, jt->d_mv))) return st;
    if ((st = upload(jt, p.works, jt->d_works))) return st;
    if ((st = upload(jt, p.wtargets, jt->d_wt))) return st;
    if ((st = upload(jt, p.pieces, jt->d_pc))) return st;
    if ((st = upload(jt, p.homevars, jt->d_hv))) return st;
    if ((st = upload(jt, p.groups, jt->d_groups))) return st;
    if ((st = upload(jt, p.fins, jt->d_fins))) return st;
    if ((st = upload(jt, p.finblks, jt->d_finblks))) return st;
    if ((st = upload(jt, p.digits, jt->d_dig))) return st;
    if ((st = upload(jt, p.maps, jt->d_map))) return st;
    // prior in table precision (float32: each entry rounded once, to nearest)
    jt->d_prior = dev_alloc(jt, w * std::max<uint64_t>(p.T, 1));
    if (!jt->d_prior) return fail(FBN_E_NOMEM_DEVICE, "device allocation failed");
    if (f32) {
        std::vector<float> pf(p.prior.size());
        for (size_t i = 0; i < pf.size(); i++) pf[i] = (float)p.prior[i];
        HIP_OK(hipMemcpy(jt->d_prior, pf.data(), 4 * pf.size(), hipMemcpyHostToDevice));
    } else {
        HIP_OK(hipMemcpy(jt->d_prior, p.prior.data(), 8 * p.prior.size(), hipMemcpyHostToDevice));
    }
    // per-slot state
    const SlotLayout SL = slot_layout(jt);
    const uint64_t psi_stride = SL.psi_stride;
    const uint32_t part_stride = SL.part_stride, kexp_stride = SL.kexp_stride, marg_stride = SL.marg_stride,
                   ev_stride = SL.ev_stride;
    const uint64_t before = jt->device_bytes;
    void** dsts[kSlotBuffers] = {&jt->d_psi, &jt->d_sepc, &jt->d_sepd, &jt->d_acc, &jt->d_part,
                                 (void**)&jt->d_kexp, (void**)&jt->d_marg, (void**)&jt->d_post,
                                 (void**)&jt->d_logpe, (void**)&jt->d_flags, (void**)&jt->d_ev,
                                 (void**)&jt->d_slots, (void**)&jt->d_out_post, (void**)&jt->d_out_logpe,
                                 (void**)&jt->d_out_flags, (void**)&jt->d_bmax, (void**)&jt->d_bmarg,
                                 (void**)&jt->d_rsum};
    for (int k = 0; k < kSlotBuffers; k++) {
        const size_t bytes = SL.unit[k] * (size_t)S;
        *dsts[k] = dev_alloc(jt, bytes);
        if (!*dsts[k]) return fail(FBN_E_NOMEM_DEVICE, "device allocation failed");
        HIP_OK(launch_zero(*dsts[k], bytes, jt->stream));
    }
    jt->slot_bytes = (jt->device_bytes - before) / (uint64_t)S;
    // host staging
    const size_t evb = sizeof(DEvidence) * ev_stride * (size_t)S;
    if (hipHostMalloc((void**)&jt->h_ev, evb, hipHostMallocDefault) == hipSuccess &&
        hipHostMalloc((void**)&jt->h_slots, 4ull * (size_t)S, hipHostMallocDefault) == hipSuccess) {
        jt->h_pinned = true;
    } else {
        return fail(FBN_E_NOMEM_HOST, "pinned host allocation failed");
    }
    std::memset(jt->h_ev, 0, evb);
    Ctx& c = jt->ctx;
    c.cl = jt->d_cl;
    c.ch = jt->d_ch;
    c.tg = jt->d_tg;
    c.mv = jt->d_mv;
    c.wt = jt->d_wt;
    c.pc = jt->d_pc;
    c.hv = jt->d_hv;
    c.dig = jt->d_dig;
    c.map = jt->d_map;
    c.prior = jt->d_prior;
    c.psi = jt->d_psi;
    c.sepc = jt->d_sepc;
    c.sepd = jt->d_sepd;
    c.acc = jt->d_acc;
    c.part = jt->d_part;
    c.rsum = jt->d_rsum;
    c.kexp = jt->d_kexp;
    c.marg = jt->d_marg;
    c.post = jt->d_post;
    c.logpe = jt->d_logpe;
    c.flags = jt->d_flags;
    c.ev = jt->d_ev;
    c.bmax = jt->d_bmax;
    c.bmarg = jt->d_bmarg;
    c.bmax_stride = SL.bmax_stride;
    c.bmarg_stride = SL.bmarg_stride;
    c.psi_stride = psi_stride;
    c.sep_stride = p.sep_stride;
    c.part_stride = part_stride;
    c.kexp_stride = kexp_stride;
    c.marg_stride = marg_stride;
    c.ev_stride = ev_stride;
    c.nvars = jt->tree.n;
    c.ne = jt->tree.ne;
    c.kappa_total = p.kappa_total;
    c.sep_total = p.sep_total;
    c.nroots = p.n_roots;
    c.S = p.interleaved ? (uint32_t)S : 0u;
    c.fp32 = f32 ? 1 : 0;
    c.tile = p.stage;
    c.dense = jt->opt.shrink_evidence ? 0 : 1;
    c.bcap = jt->opt.slots_per_block;
    HIP_OK(hipStreamSynchronize(jt->stream));
    return FBN_OK;
}

fbn_status check_slots(const fbn_jt* jt, int32_t n, const int32_t* slots) {
    if (n < 0 || n > jt->opt.max_slots || (n > 0 && !slots)) return fail(FBN_E_INVALID_ARG, "bad slot list");
    std::vector<char> seen((size_t)jt->opt.max_slots, 0);
    for (int32_t i = 0; i < n; i++) {
        if (slots[i] < 0 || slots[i] >= jt->opt.max_slots) return fail(FBN_E_INVALID_ARG, "slot out of range");
        if (seen[(size_t)slots[i]]) return fail(FBN_E_INVALID_ARG, "slot listed twice");
        seen[(size_t)slots[i]] = 1;
    }
    return FBN_OK;
}

fbn_status stage_slots(fbn_jt* jt, int32_t n, const int32_t* slots) {
    fbn_status st = wait_staged(jt);
    if (st) return st;
    std::memcpy(jt->h_slots, slots, 4ull * (size_t)n);
    HIP_OK(hipMemcpyAsync(jt->d_slots, jt->h_slots, 4ull * (size_t)n, hipMemcpyHostToDevice, jt->stream));
    const size_t per = (size_t)jt->ctx.ev_stride;
    for (int32_t i = 0; i < n; i++) {
        const int s = slots[i];
        if (!jt->dirty[(size_t)s]) continue;
        int e = s;
        while (e + 1 < jt->opt.max_slots && jt->dirty[(size_t)e + 1]) e++;  // contiguous run
        HIP_OK(hipMemcpyAsync(jt->d_ev + (size_t)s * per, jt->h_ev + (size_t)s * per,
                              sizeof(DEvidence) * per * (size_t)(e - s + 1), hipMemcpyHostToDevice, jt->stream));
        for (int k = s; k <= e; k++) jt->dirty[(size_t)k] = 0;
    }
    HIP_OK(hipEventRecord(jt->staged, jt->stream));
    jt->staged_pending = true;
    jt->staged_slots.assign(slots, slots + n);
    return FBN_OK;
}

// d_slots for a read-back of n slots: reused as is when it already holds
// this list (the usual calibrate-then-fetch), so the read-back records no
// new staging event and a following fbn_set_evidence does not wait for
// the calibration in flight.
fbn_status slots_for_fetch(fbn_jt* jt, int32_t n, const int32_t* slots) {
    if (jt->staged_slots.size() == (size_t)n && std::equal(slots, slots + n, jt->staged_slots.begin()))
        return FBN_OK;
    return stage_slots(jt, n, slots);
}

template <class F>
fbn_status timed(fbn_jt* jt, int kind, double bytes, F launch) {
    if (!jt->prof || !((jt->prof_mask >> kind) & 1u)) {
        HIP_OK(launch());
        return FBN_OK;
    }
    hipEvent_t ev[2];
    for (int k = 0; k < 2; k++) {
        if (jt->pool.empty()) {
            hipEvent_t e;
            HIP_OK(hipEventCreate(&e));
            jt->pool.push_back(e);
        }
        ev[k] = jt->pool.back();
        jt->pool.pop_back();
    }
    HIP_OK(hipEventRecord(ev[0], jt->stream));
    HIP_OK(launch());
    HIP_OK(hipEventRecord(ev[1], jt->stream));
    jt->recs.push_back({ev[0], ev[1], kind, bytes});
    return FBN_OK;
}

fbn_status status_of_flag(int32_t f) {
    if (f & 2) return FBN_E_UNDERFLOW;
    if (f & 1) return FBN_E_ZERO_EVIDENCE;
    return FBN_OK;
}

fbn_status fetch(fbn_jt* jt, int32_t n, double* post, double* logpe, int32_t* flags) {
    HIP_OK(launch_gather(jt->ctx, jt->d_slots, n, post ? jt->d_out_post : nullptr, logpe ? jt->d_out_logpe : nullptr,
                         flags ? jt->d_out_flags : nullptr, jt->stream));
    const size_t per = jt->ctx.marg_stride;
    if (post) HIP_OK(hipMemcpyAsync(post, jt->d_out_post, 8 * per * (size_t)n, hipMemcpyDeviceToHost, jt->stream));
    if (logpe) HIP_OK(hipMemcpyAsync(logpe, jt->d_out_logpe, 8ull * (size_t)n, hipMemcpyDeviceToHost, jt->stream));
    if (flags) HIP_OK(hipMemcpyAsync(flags, jt->d_out_flags, 4ull * (size_t)n, hipMemcpyDeviceToHost, jt->stream));
    return FBN_OK;
}

}  // namespace

static fbn_status enqueue_calibration(fbn_jt* jt, int32_t n);
static fbn_status finish_build(fbn_jt* jt, fbn_jt** out);

// FP32 trees built with fp64_rerun: the slots whose FP32 messages vanished
// (flag bit 1) are recomputed on a one-slot FP64 tree of the same network,
// built on first need, and the FP64 posteriors, log P(e) and flags replace
// the FP32 ones in this tree's per-slot arrays.  flags[i] (raw flags of
// slots[i]) is updated; log_pe[i] too when log_pe is given.
static fbn_status rerun_fp64(fbn_jt* jt, int32_t n, const int32_t* slots, int32_t* flags, double* log_pe) {
    if (!jt->opt.fp64_rerun || jt->opt.precision != FBN_FP32_RESCALED) return FBN_OK;
    for (int32_t i = 0; i < n; i++) {
        if (!(flags[i] & 2)) continue;
        if (!jt->twin) {
            auto* tw = new fbn_jt();
            tw->opt = jt->opt;
            tw->opt.precision = FBN_FP64;
            tw->opt.max_slots = 1;
            tw->opt.layout = FBN_LAYOUT_PER_SLOT;
            tw->opt.shrink_evidence = 0;
            tw->opt.fp64_rerun = 0;
            tw->opt.host_only = 0;
            tw->opt.stream = jt->stream;
            tw->tree = jt->tree;
            fbn_status st = finish_build(tw, &jt->twin);
            if (st) return st;
        }
        fbn_jt* tw = jt->twin;
        const auto& el = jt->evidence[(size_t)slots[i]];
        std::vector<int32_t> vs, ss;
        for (const auto& e : el) {
            vs.push_back(e.first);
            ss.push_back(e.second);
        }
        fbn_status st = fbn_set_evidence(tw, 0, (int32_t)vs.size(), vs.data(), ss.data());
        if (st) return st;
        const int32_t zero = 0;
        if ((st = fbn_calibrate(tw, 1, &zero, nullptr, nullptr))) return st;
        const size_t m = jt->ctx.marg_stride;
        const size_t sl = (size_t)slots[i];
        HIP_OK(hipMemcpyAsync(jt->d_post + sl * m, tw->d_post, 8 * m, hipMemcpyDeviceToDevice, jt->stream));
        HIP_OK(hipMemcpyAsync(jt->d_logpe + sl, tw->d_logpe, 8, hipMemcpyDeviceToDevice, jt->stream));
        HIP_OK(hipMemcpyAsync(jt->d_flags + sl, tw->d_flags, 4, hipMemcpyDeviceToDevice, jt->stream));
        double lp = 0.0;
        int32_t f = 0;
        HIP_OK(hipMemcpyAsync(&lp, tw->d_logpe, 8, hipMemcpyDeviceToHost, jt->stream));
        HIP_OK(hipMemcpyAsync(&f, tw->d_flags, 4, hipMemcpyDeviceToHost, jt->stream));
        HIP_OK(hipStreamSynchronize(jt->stream));
        // bit 2 marks the slot's results as recomputed in FP64: its FP32
        // tables are not valid, and readers of the tables go to the twin
        const int32_t marked = f | 4;
        HIP_OK(hipMemcpyAsync(jt->d_flags + sl, &marked, 4, hipMemcpyHostToDevice, jt->stream));
        HIP_OK(hipStreamSynchronize(jt->stream));
        flags[i] = f;
        if (log_pe) log_pe[i] = lp;
    }
    return FBN_OK;
}

// ====================================================================== ABI

extern "C" {

void fbn_default_options(fbn_jt_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = FBN_FP64;
    opt->max_slots = 1;
    opt->max_clique_entries = 0x7fffffffull;
    opt->host_only = 0;
    opt->tile_entries = 0;
    opt->stream = nullptr;
}

const char* fbn_status_str(fbn_status s) {
    switch (s) {
        case FBN_OK: return "ok";
        case FBN_E_INVALID_ARG: return "invalid argument";
        case FBN_E_PARSE: return "parse error";
        case FBN_E_IO: return "i/o error";
        case FBN_E_NOMEM_HOST: return "out of host memory";
        case FBN_E_NOMEM_DEVICE: return "out of device memory";
        case FBN_E_TOO_LARGE: return "clique too large";
        case FBN_E_ZERO_EVIDENCE: return "evidence has probability zero";
        case FBN_E_STATE: return "invalid state";
        case FBN_E_DEVICE: return "device error";
        case FBN_E_UNDERFLOW: return "float32 underflow";
        default: return "unknown status";
    }
}

const char* fbn_last_error(void) { return g_err.c_str(); }

fbn_status fbn_load_net_mem(const char* text, size_t len, fbn_net** out) {
    if (!text || !out) return fail(FBN_E_INVALID_ARG, "null argument");
    *out = nullptr;
    try {
        auto* h = new fbn_net();
        // .fbn text opens with "fbn"; anything else is read as BIF
        size_t k = 0;
        while (k < len && (text[k] == ' ' || text[k] == '\t' || text[k] == '\n' || text[k] == '\r')) k++;
        fbn_status st;
        if (len - k >= 3 && std::strncmp(text + k, "fbn", 3) == 0) {
            st = parse_net(text, len, h->net);
        } else {
            const std::string err = parse_bif(text, len, h->net, h->names, h->states);
            st = err.empty() ? check_net(h->net) : fail(FBN_E_PARSE, "BIF: " + err);
        }
        if (st) {
            delete h;
            return st;
        }
        *out = h;
        return FBN_OK;
    } catch (const std::bad_alloc&) {
        return fail(FBN_E_NOMEM_HOST, "out of host memory");
    } catch (...) {
        return fail(FBN_E_PARSE, "parse failure");
    }
}

fbn_status fbn_load_net(const char* path, fbn_net** out) {
    if (!path || !out) return fail(FBN_E_INVALID_ARG, "null argument");
    std::ifstream f(path, std::ios::binary);
    if (!f) return fail(FBN_E_IO, std::string("cannot open ") + path);
    std::stringstream ss;
    ss << f.rdbuf();
    std::string s = ss.str();
    return fbn_load_net_mem(s.data(), s.size(), out);
}

fbn_status fbn_net_from_arrays(int32_t n, const int32_t* card, const int32_t* npar, const int32_t* parents,
                               const double* cpt, fbn_net** out) {
    if (!out || n <= 0 || !card || !npar || !cpt) return fail(FBN_E_INVALID_ARG, "null or empty argument");
    *out = nullptr;
    try {
        auto* h = new fbn_net();
        Net& net = h->net;
        net.n = n;
        net.card.assign(card, card + n);
        net.parents.assign((size_t)n, {});
        net.cpt.assign((size_t)n, {});
        size_t po = 0, co = 0;
        for (int v = 0; v < n; v++) {
            if (npar[v] < 0 || (npar[v] > 0 && !parents)) {
                delete h;
                return fail(FBN_E_INVALID_ARG, "bad parent count");
            }
            for (int k = 0; k < npar[v]; k++) net.parents[(size_t)v].push_back(parents[po + (size_t)k]);
            po += (size_t)npar[v];
        }
        for (int v = 0; v < n; v++) {
            uint64_t len = (uint64_t)std::max(card[v], 0);
            for (int p : net.parents[(size_t)v]) {
                if (p < 0 || p >= n) {
                    delete h;
                    return fail(FBN_E_INVALID_ARG, "bad parent id");
                }
                len *= (uint64_t)std::max(card[p], 0);
            }
            net.cpt[(size_t)v].assign(cpt + co, cpt + co + len);
            co += len;
        }
        fbn_status st = check_net(net);
        if (st) {
            delete h;
            return st;
        }
        *out = h;
        return FBN_OK;
    } catch (const std::bad_alloc&) {
        return fail(FBN_E_NOMEM_HOST, "out of host memory");
    }
}

void fbn_free_net(fbn_net* net) { delete net; }

fbn_status fbn_net_n_vars(const fbn_net* net, int32_t* n) {
    if (!net || !n) return fail(FBN_E_INVALID_ARG, "null argument");
    *n = net->net.n;
    return FBN_OK;
}

static fbn_status copy_name(const std::string& s, char* buf, size_t cap) {
    if (!buf || cap < s.size() + 1) return fail(FBN_E_INVALID_ARG, "name buffer too small");
    std::memcpy(buf, s.c_str(), s.size() + 1);
    return FBN_OK;
}

fbn_status fbn_net_var_name(const fbn_net* net, int32_t v, char* buf, size_t cap) {
    if (!net || v < 0 || v >= net->net.n) return fail(FBN_E_INVALID_ARG, "bad variable");
    return copy_name(net->names.empty() ? std::to_string(v) : net->names[(size_t)v], buf, cap);
}

fbn_status fbn_net_state_name(const fbn_net* net, int32_t v, int32_t s, char* buf, size_t cap) {
    if (!net || v < 0 || v >= net->net.n || s < 0 || s >= net->net.card[(size_t)v])
        return fail(FBN_E_INVALID_ARG, "bad variable or state");
    return copy_name(net->states.empty() ? std::to_string(s) : net->states[(size_t)v][(size_t)s], buf, cap);
}

fbn_status fbn_net_find_var(const fbn_net* net, const char* name, int32_t* v) {
    if (!net || !name || !v) return fail(FBN_E_INVALID_ARG, "null argument");
    for (int x = 0; x < net->net.n; x++)
        if ((net->names.empty() ? std::to_string(x) : net->names[(size_t)x]) == name) {
            *v = x;
            return FBN_OK;
        }
    return fail(FBN_E_INVALID_ARG, std::string("no variable named ") + name);
}

fbn_status fbn_net_find_state(const fbn_net* net, int32_t v, const char* name, int32_t* s) {
    if (!net || !name || !s || v < 0 || v >= net->net.n) return fail(FBN_E_INVALID_ARG, "bad argument");
    for (int x = 0; x < net->net.card[(size_t)v]; x++)
        if ((net->states.empty() ? std::to_string(x) : net->states[(size_t)v][(size_t)x]) == name) {
            *s = x;
            return FBN_OK;
        }
    return fail(FBN_E_INVALID_ARG, std::string("no state named ") + name);
}

fbn_status fbn_net_cpt(const fbn_net* net, int32_t v, int32_t* card, int32_t* parents, int32_t par_cap,
                       int32_t* n_parents, double* cpt, size_t cpt_cap, size_t* cpt_len) {
    if (!net || v < 0 || v >= net->net.n) return fail(FBN_E_INVALID_ARG, "bad variable");
    const auto& par = net->net.parents[(size_t)v];
    const auto& tab = net->net.cpt[(size_t)v];
    if ((parents && par_cap < (int32_t)par.size()) || (cpt && cpt_cap < tab.size()))
        return fail(FBN_E_INVALID_ARG, "output too small");
    if (card) *card = net->net.card[(size_t)v];
    if (n_parents) *n_parents = (int32_t)par.size();
    if (cpt_len) *cpt_len = tab.size();
    if (parents) std::copy(par.begin(), par.end(), parents);
    if (cpt) std::copy(tab.begin(), tab.end(), cpt);
    return FBN_OK;
}

static fbn_status finish_build(fbn_jt* jt, fbn_jt** out);

static fbn_status build_jt_impl(const std::vector<const fbn_net*>& nets, const fbn_jt_options* opt_in, fbn_jt** out) {
    *out = nullptr;
    fbn_jt_options opt;
    if (opt_in) opt = *opt_in;
    else fbn_default_options(&opt);
    if (opt.max_slots < 1 || (opt.precision != FBN_FP64 && opt.precision != FBN_FP32_RESCALED) ||
        opt.tile_entries < 0 || opt.tile_entries > kTileMax || opt.layout < FBN_LAYOUT_AUTO ||
        opt.layout > FBN_LAYOUT_INTERLEAVED)
        return fail(FBN_E_INVALID_ARG, "bad options");
    if (opt.slots_per_block != 0 && opt.slots_per_block != 1 && opt.slots_per_block != 2 &&
        opt.slots_per_block != 4 && opt.slots_per_block != 8)
        return fail(FBN_E_INVALID_ARG, "slots_per_block must be 0, 1, 2, 4 or 8");
    if (opt.fin_block != 0 && (opt.fin_block < 64 || opt.fin_block > (int32_t)kFinBlock))
        return fail(FBN_E_INVALID_ARG, "fin_block must be 0 or in [64, 4096]");
    if (opt.max_clique_entries == 0 || opt.max_clique_entries > 0x7fffffffull) opt.max_clique_entries = 0x7fffffffull;
    fbn_jt* jt = nullptr;
    try {
        jt = new fbn_jt();
        jt->opt = opt;
        if (nets.size() == 1) {
            int code = 0;
            std::string err = compile_tree(nets[0]->net, opt.max_clique_entries, jt->tree, code);
            if (!err.empty()) {
                delete jt;
                return fail(code ? code : FBN_E_INVALID_ARG, err);
            }
        } else {
            std::vector<Tree> parts(nets.size());
            uint64_t nv = 0;
            for (size_t k = 0; k < nets.size(); k++) {
                int code = 0;
                std::string err = compile_tree(nets[k]->net, opt.max_clique_entries, parts[k], code);
                if (!err.empty()) {
                    delete jt;
                    return fail(code ? code : FBN_E_INVALID_ARG, "network " + std::to_string(k) + ": " + err);
                }
                nv += (uint64_t)parts[k].n;
            }
            if (nv > 0x7fffffffull) {
                delete jt;
                return fail(FBN_E_TOO_LARGE, "too many variables in the forest");
            }
            jt->tree = merge_forest(parts);
        }
        return finish_build(jt, out);
    } catch (const std::bad_alloc&) {
        if (jt) {
            release(jt);
            delete jt;
        }
        return fail(FBN_E_NOMEM_HOST, "out of host memory");
    } catch (const std::exception& e) {
        if (jt) {
            release(jt);
            delete jt;
        }
        return fail(FBN_E_TOO_LARGE, e.what());
    }
}

// The rest of a build once jt->tree holds the compiled tree and jt->opt the
// options: plan, per-layer counts, evidence lookup, device state.  Frees jt
// and returns the error on failure.
static fbn_status finish_build(fbn_jt* jt, fbn_jt** out) {
    const fbn_jt_options& opt = jt->opt;
    try {
        // default tile: 8 KB of table per slot, so four slots share a workgroup
        // interleaved: one wave per work item, 64 entries each by default
        const bool il = opt.layout == FBN_LAYOUT_INTERLEAVED;
        const int def_tile = il ? 64 : (opt.precision == FBN_FP32_RESCALED ? 1024 : 512);
        const uint32_t max_stage = (uint32_t)kSlotStageBytes / (opt.precision == FBN_FP32_RESCALED ? 4u : 8u);
        build_plan(jt->tree, opt.tile_entries ? opt.tile_entries : def_tile, max_stage, jt->plan, il,
                   (uint32_t)opt.fin_block);
        const std::string bad = check_plan(jt->tree, jt->plan);
        if (!bad.empty()) {
            delete jt;
            return fail(FBN_E_STATE, "internal plan check failed: " + bad);
        }
        {
            const Tree& t = jt->tree;
            const Plan& p = jt->plan;
            jt->coll_entries.assign(p.collect.size(), 0);
            jt->dist_entries.assign(p.distribute.size(), 0);
            for (int c = 0; c < t.nc; c++) {
                jt->coll_entries[(size_t)t.height[(size_t)c]] += t.size[(size_t)c];
                jt->dist_entries[(size_t)t.depth[(size_t)c]] += t.size[(size_t)c];
            }
            auto sep_sum = [&](const std::vector<Layer>& ls, std::vector<uint64_t>& out) {
                out.assign(ls.size(), 0);
                for (size_t k = 0; k < ls.size(); k++)
                    for (uint32_t f = ls[k].fin0; f < ls[k].fin0 + ls[k].nfin; f++) out[k] += p.fins[f].size;
            };
            sep_sum(p.collect, jt->coll_sep);
            sep_sum(p.distribute, jt->dist_sep);
        }
        jt->occ.assign((size_t)jt->tree.n, {});
        for (int c = 0; c < jt->tree.nc; c++)
            for (size_t k = 0; k < jt->tree.vars[(size_t)c].size(); k++)
                jt->occ[(size_t)jt->tree.vars[(size_t)c][k]].push_back({c, (int)k});
        jt->dirty.assign((size_t)opt.max_slots, 0);
        jt->evidence.assign((size_t)opt.max_slots, {});
        jt->live_coll.assign((size_t)opt.max_slots * jt->coll_entries.size(), 0);
        jt->live_dist.assign((size_t)opt.max_slots * jt->dist_entries.size(), 0);
        for (int32_t s = 0; s < opt.max_slots; s++) {
            std::copy(jt->coll_entries.begin(), jt->coll_entries.end(),
                      jt->live_coll.begin() + (size_t)s * jt->coll_entries.size());
            std::copy(jt->dist_entries.begin(), jt->dist_entries.end(),
                      jt->live_dist.begin() + (size_t)s * jt->dist_entries.size());
        }
        if (opt.host_only) {
            jt->device_bytes = footprint(jt, jt->slot_bytes);
        } else {
            fbn_status st = setup_device(jt);
            if (st) {
                std::string keep = g_err;
                release(jt);
                delete jt;
                g_err = keep;
                return st;
            }
        }
        *out = jt;
        return FBN_OK;
    } catch (const std::bad_alloc&) {
        release(jt);
        delete jt;
        return fail(FBN_E_NOMEM_HOST, "out of host memory");
    } catch (const std::exception& e) {
        release(jt);
        delete jt;
        return fail(FBN_E_TOO_LARGE, e.what());
    }
}

fbn_status fbn_build_jt(const fbn_net* net, const fbn_jt_options* opt_in, fbn_jt** out) {
    if (!net || !out) return fail(FBN_E_INVALID_ARG, "null argument");
    return build_jt_impl({net}, opt_in, out);
}

fbn_status fbn_build_forest(const fbn_net* const* nets, int32_t n_nets, const fbn_jt_options* opt_in, fbn_jt** out) {
    if (!nets || !out || n_nets < 1) return fail(FBN_E_INVALID_ARG, "null argument or no networks");
    *out = nullptr;
    std::vector<const fbn_net*> v((size_t)n_nets);
    for (int32_t k = 0; k < n_nets; k++) {
        if (!nets[k]) return fail(FBN_E_INVALID_ARG, "null network");
        v[(size_t)k] = nets[k];
    }
    return build_jt_impl(v, opt_in, out);
}

void fbn_free_jt(fbn_jt* jt) {
    if (!jt) return;
    if (jt->twin) fbn_free_jt(jt->twin);
    release(jt);
    delete jt;
}

fbn_status fbn_set_stream(fbn_jt* jt, void* stream) {
    if (!jt) return fail(FBN_E_INVALID_ARG, "null jt");
    if (jt->opt.host_only) return fail(FBN_E_STATE, "host-only jt");
    fbn_status st = wait_staged(jt);
    if (st) return st;
    HIP_OK(hipStreamSynchronize(jt->stream));
    for (auto& kv : jt->graphs) hipGraphExecDestroy(kv.second);
    jt->graphs.clear();
    jt->stream = static_cast<hipStream_t>(stream);
    jt->opt.stream = stream;
    if (!jt->stream) jt->use_graph = false;
    if (jt->twin) return fbn_set_stream(jt->twin, stream);
    return FBN_OK;
}

fbn_status fbn_set_evidence(fbn_jt* jt, int32_t slot, int32_t n_obs, const int32_t* vars, const int32_t* states) {
    if (!jt) return fail(FBN_E_INVALID_ARG, "null jt");
    if (jt->opt.host_only) return fail(FBN_E_STATE, "host-only jt");
    if (slot < 0 || slot >= jt->opt.max_slots) return fail(FBN_E_INVALID_ARG, "slot out of range");
    if (n_obs < 0 || (n_obs > 0 && (!vars || !states))) return fail(FBN_E_INVALID_ARG, "bad evidence arrays");
    const Tree& t = jt->tree;
    std::vector<char> seen((size_t)t.n, 0);
    for (int32_t k = 0; k < n_obs; k++) {
        const int v = vars[k];
        if (v < 0 || v >= t.n) return fail(FBN_E_INVALID_ARG, "evidence variable out of range");
        if (seen[(size_t)v]) return fail(FBN_E_INVALID_ARG, "evidence variable repeated");
        seen[(size_t)v] = 1;
        if (states[k] < 0 || states[k] >= t.card[(size_t)v]) return fail(FBN_E_INVALID_ARG, "evidence state out of range");
    }
    fbn_status st = wait_staged(jt);
    if (st) return st;
    DEvidence* ev = jt->h_ev + (size_t)slot * jt->ctx.ev_stride;
    std::memset(ev, 0, sizeof(DEvidence) * jt->ctx.ev_stride);
    const Plan& p = jt->plan;
    for (int32_t k = 0; k < n_obs; k++) {
        const int v = vars[k];
        uint32_t bits = 0;
        while ((1u << bits) < (uint32_t)t.card[(size_t)v]) bits++;
        for (const auto& cp : jt->occ[(size_t)v]) {
            const uint32_t sh = p.dig_shift[p.dig_shift0[(size_t)cp.first] + (size_t)cp.second];
            ev[cp.first].mask |= (((uint64_t)1 << bits) - 1) << sh;
            ev[cp.first].want |= (uint64_t)states[k] << sh;
        }
    }
    jt->dirty[(size_t)slot] = 1;
    auto& el = jt->evidence[(size_t)slot];
    el.clear();
    for (int32_t k = 0; k < n_obs; k++) el.push_back({vars[k], states[k]});
    // live entries per layer (shrinking reduction only, for the kernel
    // timing's byte counts): a clique holding observed variables keeps
    // |C| / prod(their cardinalities) entries
    if (jt->opt.shrink_evidence) {
        const size_t nh = jt->coll_entries.size(), nd = jt->dist_entries.size();
        uint64_t* lc = jt->live_coll.data() + (size_t)slot * nh;
        uint64_t* ld = jt->live_dist.data() + (size_t)slot * nd;
        std::copy(jt->coll_entries.begin(), jt->coll_entries.end(), lc);
        std::copy(jt->dist_entries.begin(), jt->dist_entries.end(), ld);
        std::vector<std::pair<int, uint64_t>> div;  // (clique, product of observed cardinalities)
        for (int32_t k = 0; k < n_obs; k++)
            for (const auto& cp : jt->occ[(size_t)vars[k]]) div.push_back({cp.first, (uint64_t)t.card[(size_t)vars[k]]});
        std::sort(div.begin(), div.end());
        for (size_t a = 0; a < div.size();) {
            uint64_t d = 1;
            size_t b = a;
            for (; b < div.size() && div[b].first == div[a].first; b++) d *= div[b].second;
            const uint64_t sz = t.size[(size_t)div[a].first], gone = sz - sz / d;
            lc[(size_t)t.height[(size_t)div[a].first]] -= gone;
            ld[(size_t)t.depth[(size_t)div[a].first]] -= gone;
            a = b;
        }
    }
    return FBN_OK;
}

fbn_status fbn_set_evidence_batch(fbn_jt* jt, int32_t n_slots, const int32_t* slots, const int32_t* offsets,
                                  const int32_t* vars, const int32_t* states) {
    if (!jt || n_slots < 0 || (n_slots > 0 && (!slots || !offsets))) return fail(FBN_E_INVALID_ARG, "bad arguments");
    for (int32_t i = 0; i < n_slots; i++) {
        if (offsets[i + 1] < offsets[i]) return fail(FBN_E_INVALID_ARG, "offsets not ascending");
        fbn_status st = fbn_set_evidence(jt, slots[i], offsets[i + 1] - offsets[i], vars ? vars + offsets[i] : nullptr,
                                         states ? states + offsets[i] : nullptr);
        if (st) return st;
    }
    return FBN_OK;
}

fbn_status fbn_calibrate(fbn_jt* jt, int32_t n, const int32_t* slots, double* log_pe, fbn_status* per_slot) {
    if (!jt) return fail(FBN_E_INVALID_ARG, "null jt");
    if (jt->opt.host_only) return fail(FBN_E_STATE, "host-only jt");
    fbn_status st = check_slots(jt, n, slots);
    if (st) return st;
    if (n == 0) return FBN_OK;
    HIP_OK(hipSetDevice(jt->device));
    if ((st = stage_slots(jt, n, slots))) return st;
    if (jt->use_graph && !jt->prof) {
        // one graph launch replays the whole layer sequence for n slots
        auto it = jt->graphs.find(n);
        if (it == jt->graphs.end()) {
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            HIP_OK(hipStreamBeginCapture(jt->stream, hipStreamCaptureModeThreadLocal));
            st = enqueue_calibration(jt, n);
            hipError_t ec = hipStreamEndCapture(jt->stream, &g);
            if (st) {
                if (g) hipGraphDestroy(g);
                return st;
            }
            if (ec != hipSuccess) return fail(FBN_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
            ec = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            if (ec != hipSuccess) return fail(FBN_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ec));
            it = jt->graphs.emplace(n, ge).first;
        }
        HIP_OK(hipGraphLaunch(it->second, jt->stream));
    } else if ((st = enqueue_calibration(jt, n))) {
        return st;
    }
    if (log_pe || per_slot) {
        std::vector<double> lp((size_t)n);
        std::vector<int32_t> fl((size_t)n);
        if ((st = fetch(jt, n, nullptr, lp.data(), fl.data()))) return st;
        HIP_OK(hipStreamSynchronize(jt->stream));
        if ((st = rerun_fp64(jt, n, slots, fl.data(), lp.data()))) return st;
        for (int32_t i = 0; i < n; i++) {
            if (log_pe) log_pe[i] = lp[(size_t)i];
            if (per_slot) per_slot[i] = status_of_flag(fl[(size_t)i]);
        }
    }
    return FBN_OK;
}

}  // extern "C"

// The launch sequence of one calibration of the n slots staged in d_slots:
// collect layers leaves to root, then distribute layers root to leaves, then
// the posteriors.
// The same sequence on slot-interleaved tables.  wn = table bytes per entry
// times the batch size, for the profiling byte counts.
static fbn_status enqueue_interleaved(fbn_jt* jt, int32_t n, double wn) {
    const Ctx& c = jt->ctx;
    const Plan& p = jt->plan;
    const int prec = jt->opt.precision == FBN_FP32_RESCALED ? 1 : 0;
    hipStream_t s = jt->stream;
    const int32_t* sl = jt->d_slots;
    fbn_status st;
    HIP_OK(launch_begin(c, sl, n, s));
    // the large separators' running maxima start at zero
    if (!p.finblks.empty()) HIP_OK(launch_zero(jt->d_bmax, 8ull * c.bmax_stride * (uint64_t)jt->opt.max_slots, s));
    // a layer's finalisers: the small separators and the first phase of the
    // large ones' blocks in one launch, then the blocks' second phase
    auto fins = [&](const Layer& ly, bool dist, int kind, double bytes) -> fbn_status {
        fbn_status r;
        if (ly.nfin == ly.nbig && !ly.nfb) return FBN_OK;
        if ((r = timed(jt, kind, bytes, [&] {
                 return launch_fin_interleaved(c, prec, dist, jt->d_fins + ly.fin0 + ly.nbig, ly.nfin - ly.nbig,
                                               jt->d_finblks + ly.fb0, ly.nfb, jt->d_fins, sl, n, s);
             })))
            return r;
        if (ly.nfb) {
            const int kb = dist ? kIlFinDistributeB : kIlFinCollectB;
            if ((r = timed(jt, kind, 0.0, [&] {
                     return launch_interleaved(c, prec, kb, jt->d_finblks + ly.fb0, ly.nfb, jt->d_fins, sl, n, s);
                 })))
                return r;
        }
        return FBN_OK;
    };
    for (size_t h = 0; h < p.collect.size(); h++) {
        const Layer& ly = p.collect[h];
        if ((st = timed(jt, 0, 2.0 * wn * (double)jt->coll_entries[h], [&] {
                 return launch_interleaved(c, prec, kIlCollect, jt->d_groups + ly.group0, ly.ngroup, jt->d_fins, sl,
                                           n, s);
             })))
            return st;
        if ((st = fins(ly, false, 1, 2.0 * wn * (double)jt->coll_sep[h]))) return st;
    }
    for (size_t d = 0; d < p.distribute.size(); d++) {
        const Layer& ly = p.distribute[d];
        if ((st = timed(jt, 2, wn * (double)jt->dist_entries[d], [&] {
                 return launch_interleaved(c, prec, kIlDistribute, jt->d_works + ly.group0, ly.ngroup, jt->d_fins, sl,
                                           n, s);
             })))
            return st;
        if ((st = fins(ly, true, 3, 2.0 * wn * (double)jt->dist_sep[d]))) return st;
    }
    return timed(jt, 4, 16.0 * (wn / (prec ? 4.0 : 8.0)) * (double)c.marg_stride,
                 [&] { return launch_marginals_interleaved(c, sl, n, s); });
}

static fbn_status enqueue_calibration(fbn_jt* jt, int32_t n) {
    fbn_status st = FBN_OK;
    const Ctx& c = jt->ctx;
    const Plan& p = jt->plan;
    const int prec = jt->opt.precision == FBN_FP32_RESCALED ? 1 : 0;
    hipStream_t s = jt->stream;
    // clear the per-slot flags of this batch
    HIP_OK(launch_begin(c, jt->d_slots, n, s));
    const double w = prec ? 4.0 : 8.0, nb = (double)n;
    if (p.interleaved) return enqueue_interleaved(jt, n, w * nb);
    // table entries the batch streams per layer: the live ones per slot
    // (every one unless shrink_evidence)
    std::vector<double> ent_c(p.collect.size(), 0.0), ent_d(p.distribute.size(), 0.0);
    if (jt->prof) {
        const bool dense = jt->opt.shrink_evidence == 0;
        for (size_t h = 0; h < ent_c.size(); h++) ent_c[h] = dense ? nb * (double)jt->coll_entries[h] : 0.0;
        for (size_t d = 0; d < ent_d.size(); d++) ent_d[d] = dense ? nb * (double)jt->dist_entries[d] : 0.0;
        if (!dense)
            for (int32_t s : jt->staged_slots) {
                for (size_t h = 0; h < ent_c.size(); h++) ent_c[h] += (double)jt->live_coll[(size_t)s * ent_c.size() + h];
                for (size_t d = 0; d < ent_d.size(); d++) ent_d[d] += (double)jt->live_dist[(size_t)s * ent_d.size() + d];
            }
    }
    // a layer's finalisers: the small separators (a wave or a workgroup
    // each) and the first phase of the large ones' blocks in one launch,
    // then the blocks' second phase; the layer's bytes are booked on the first
    auto finalise = [&](const Layer& ly, bool dist, int kind, double bytes) -> fbn_status {
        fbn_status r;
        if (ly.nfin == ly.nbig && !ly.nfb) return FBN_OK;
        const DSepFin* f = jt->d_fins + ly.fin0 + ly.nbig;
        const uint32_t nf = ly.nfin - ly.nbig;
        const DFinBlk* fb = jt->d_finblks + ly.fb0;
        if ((r = timed(jt, kind, bytes, [&] {
                 return dist ? launch_fin_distribute(c, prec, f, nf, ly.nteam, jt->d_fins, fb, ly.nfb, jt->d_slots, n, s)
                             : launch_fin_collect(c, prec, f, nf, ly.nteam, jt->d_fins, fb, ly.nfb, jt->d_slots, n, s);
             })))
            return r;
        if (ly.nfb &&
            (r = timed(jt, kind, 0.0, [&] {
                 return launch_fin_blocks(c, prec, dist, jt->d_fins, fb, ly.nfb, jt->d_slots, n, s);
             })))
            return r;
        return FBN_OK;
    };
    for (size_t h = 0; h < p.collect.size(); h++) {
        const Layer& ly = p.collect[h];
        // reads the prior, writes the working table
        if ((st = timed(jt, 0, 2.0 * w * ent_c[h], [&] {
                 return launch_collect(c, prec, jt->d_groups + ly.group0, ly.ngroup, ly.stage, jt->d_slots, n, s);
             })))
            return st;
        if ((st = finalise(ly, false, 1, 2.0 * w * nb * (double)jt->coll_sep[h]))) return st;
    }
    for (size_t d = 0; d < p.distribute.size(); d++) {
        const Layer& ly = p.distribute[d];
        // reads the working table
        if ((st = timed(jt, 2, w * ent_d[d], [&] {
                 return launch_distribute(c, prec, jt->d_works + ly.group0, ly.ngroup, ly.stage, jt->d_slots, n, s);
             })))
            return st;
        if ((st = finalise(ly, true, 3, 2.0 * w * nb * (double)jt->dist_sep[d]))) return st;
    }
    if ((st = timed(jt, 4, 16.0 * nb * (double)c.marg_stride, [&] { return launch_marginals(c, jt->d_slots, n, s); })))
        return st;
    return FBN_OK;
}

extern "C" {

fbn_status fbn_set_graph_mode(fbn_jt* jt, int32_t on) {
    if (!jt) return fail(FBN_E_INVALID_ARG, "null jt");
    if (jt->opt.host_only) return fail(FBN_E_STATE, "host-only jt");
    if (on && !jt->stream) return fail(FBN_E_STATE, "graph mode needs a stream");
    jt->use_graph = on != 0;
    return FBN_OK;
}

fbn_status fbn_query_all(fbn_jt* jt, int32_t n, const int32_t* slots, double* out, size_t out_len, double* log_pe,
                         fbn_status* per_slot) {
    if (!jt) return fail(FBN_E_INVALID_ARG, "null jt");
    if (jt->opt.host_only) return fail(FBN_E_STATE, "host-only jt");
    fbn_status st = check_slots(jt, n, slots);
    if (st) return st;
    if (n == 0) return FBN_OK;
    const size_t per = jt->ctx.marg_stride;
    if (out && out_len < per * (size_t)n) return fail(FBN_E_INVALID_ARG, "output too small");
    HIP_OK(hipSetDevice(jt->device));
    if ((st = slots_for_fetch(jt, n, slots))) return st;
    std::vector<double> lp((size_t)n);
    std::vector<int32_t> fl((size_t)n);
    if ((st = fetch(jt, n, out, lp.data(), fl.data()))) return st;
    HIP_OK(hipStreamSynchronize(jt->stream));
    bool rerun = false;
    for (int32_t i = 0; i < n; i++) rerun = rerun || (fl[(size_t)i] & 2);
    if (rerun && jt->opt.fp64_rerun && jt->opt.precision == FBN_FP32_RESCALED) {
        if ((st = rerun_fp64(jt, n, slots, fl.data(), lp.data()))) return st;
        if ((st = slots_for_fetch(jt, n, slots))) return st;
        if ((st = fetch(jt, n, out, nullptr, nullptr))) return st;
        HIP_OK(hipStreamSynchronize(jt->stream));
    }
    for (int32_t i = 0; i < n; i++) {
        if (log_pe) log_pe[i] = lp[(size_t)i];
        if (per_slot) per_slot[i] = status_of_flag(fl[(size_t)i]);
    }
    return FBN_OK;
}

fbn_status fbn_fetch_async(fbn_jt* jt, int32_t n, const int32_t* slots, double* post_out, double* log_pe_out,
                           int32_t* flags_out) {
    if (!jt) return fail(FBN_E_INVALID_ARG, "null jt");
    if (jt->opt.host_only) return fail(FBN_E_STATE, "host-only jt");
    fbn_status st = check_slots(jt, n, slots);
    if (st) return st;
    if (n == 0) return FBN_OK;
    HIP_OK(hipSetDevice(jt->device));
    if ((st = slots_for_fetch(jt, n, slots))) return st;
    return fetch(jt, n, post_out, log_pe_out, flags_out);
}

fbn_status fbn_query_marginals(fbn_jt* jt, int32_t slot, int32_t n_vars, const int32_t* vars, double* out,
                               size_t out_len) {
    if (!jt) return fail(FBN_E_INVALID_ARG, "null jt");
    if (jt->opt.host_only) return fail(FBN_E_STATE, "host-only jt");
    if (slot < 0 || slot >= jt->opt.max_slots) return fail(FBN_E_INVALID_ARG, "slot out of range");
    if (n_vars < 0 || (n_vars > 0 && (!vars || !out))) return fail(FBN_E_INVALID_ARG, "bad arguments");
    size_t need = 0;
    for (int32_t k = 0; k < n_vars; k++) {
        if (vars[k] < 0 || vars[k] >= jt->tree.n) return fail(FBN_E_INVALID_ARG, "variable out of range");
        need += (size_t)jt->tree.card[(size_t)vars[k]];
    }
    if (out_len < need) return fail(FBN_E_INVALID_ARG, "output too small");
    std::vector<double> all(jt->ctx.marg_stride);
    double lp = 0.0;
    fbn_status ps = FBN_OK;
    fbn_status st = fbn_query_all(jt, 1, &slot, all.data(), all.size(), &lp, &ps);
    if (st) return st;
    if (ps) return fail(ps, fbn_status_str(ps));
    size_t o = 0;
    for (int32_t k = 0; k < n_vars; k++) {
        const DHomeVar& h = jt->plan.homevars[(size_t)vars[k]];
        for (uint32_t x = 0; x < h.card; x++) out[o++] = all[h.out + x];
    }
    return FBN_OK;
}

}  // extern "C"

namespace {

// The read-out plan of a joint query: the smallest clique holding every
// query variable (lowest id on ties), and how its entries split into the
// outputs' chunks.
fbn_status joint_plan(const fbn_jt* jt, int32_t slot, int32_t nq, const int32_t* q, size_t out_len, JointArgs& a,
                      int& home) {
    const Tree& t = jt->tree;
    if (slot < 0 || slot >= jt->opt.max_slots) return fail(FBN_E_INVALID_ARG, "slot out of range");
    if (nq < 1 || !q) return fail(FBN_E_INVALID_ARG, "no query variables");
    for (int32_t k = 0; k < nq; k++) {
        if (q[k] < 0 || q[k] >= t.n) return fail(FBN_E_INVALID_ARG, "query variable out of range");
        for (int32_t j = 0; j < k; j++)
            if (q[j] == q[k]) return fail(FBN_E_INVALID_ARG, "query variable repeated");
    }
    home = -1;
    for (int c = 0; c < t.nc; c++) {
        const auto& vs = t.vars[(size_t)c];
        bool all = true;
        for (int32_t k = 0; k < nq && all; k++) all = std::find(vs.begin(), vs.end(), q[k]) != vs.end();
        if (all && (home < 0 || t.size[(size_t)c] < t.size[(size_t)home])) home = c;
    }
    if (home < 0) return fail(FBN_E_INVALID_ARG, "the query variables share no clique");
    const auto& vs = t.vars[(size_t)home];
    std::vector<uint32_t> stride(vs.size());
    uint64_t st = 1;
    for (size_t k = vs.size(); k-- > 0;) {
        stride[k] = (uint32_t)st;
        st *= (uint64_t)t.card[(size_t)vs[k]];
    }
    std::memset(&a, 0, sizeof(a));
    a.clique = (uint32_t)home;
    a.slot = slot;
    uint64_t n_out = 1;
    auto var = [&](size_t k) {
        JointVar jv{};
        jv.card = (uint32_t)t.card[(size_t)vs[k]];
        magic_u32(jv.card, jv.cmul, jv.csh);
        jv.stride = stride[k];
        return jv;
    };
    for (int32_t j = nq; j-- > 0;) {
        const size_t k = (size_t)(std::find(vs.begin(), vs.end(), q[j]) - vs.begin());
        a.qv[a.nq++] = var(k);
        n_out *= (uint64_t)t.card[(size_t)q[j]];
    }
    for (size_t k = vs.size(); k-- > 0;)
        if (std::find(q, q + nq, vs[k]) == q + nq) a.ov[a.no++] = var(k);
    if (out_len < n_out) return fail(FBN_E_INVALID_ARG, "output too small");
    a.n_out = (uint32_t)n_out;
    a.n_r = (uint32_t)(t.size[(size_t)home] / n_out);
    a.tpo = 1;
    while (a.tpo < 64 && a.tpo < a.n_r) a.tpo *= 2;
    a.chunk = a.tpo * 16;
    a.nchunk = (a.n_r + a.chunk - 1) / a.chunk;
    return FBN_OK;
}

// Device memory for one call's scratch, from the jt's allocator when it has
// one; released with temp_free on the same stream.
void* temp_alloc(fbn_jt* jt, size_t bytes) {
    void* p = nullptr;
    if (jt->opt.allocator.alloc) return jt->opt.allocator.alloc(jt->opt.allocator.ctx, bytes, jt->stream);
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

void temp_free(fbn_jt* jt, void* p) {
    if (!p) return;
    if (jt->opt.allocator.alloc) {
        if (jt->opt.allocator.free) jt->opt.allocator.free(jt->opt.allocator.ctx, p, jt->stream);
    } else {
        hipFree(p);
    }
}

// Launch the read-out into dev (joint_scratch_doubles(a) doubles), copy the
// outputs and the slot's flags back, and wait.
fbn_status joint_run(fbn_jt* jt, int home, const JointArgs& a, double* dev, double* out) {
    const int prec = jt->opt.precision == FBN_FP32_RESCALED ? 1 : 0;
    HIP_OK(launch_joint(jt->ctx, prec, jt->plan.cliques[(size_t)home], a, dev, jt->stream));
    int32_t flag = 0;
    HIP_OK(hipMemcpyAsync(out, dev, 8ull * a.n_out, hipMemcpyDeviceToHost, jt->stream));
    HIP_OK(hipMemcpyAsync(&flag, jt->d_flags + a.slot, 4, hipMemcpyDeviceToHost, jt->stream));
    HIP_OK(hipStreamSynchronize(jt->stream));
    const fbn_status ps = status_of_flag(flag);
    if (ps) return fail(ps, fbn_status_str(ps));
    return FBN_OK;
}

}  // namespace

extern "C" {

fbn_status fbn_query_joint(fbn_jt* jt, int32_t slot, int32_t n_q, const int32_t* q_vars, double* out,
                           size_t out_len) {
    if (!jt || !out) return fail(FBN_E_INVALID_ARG, "null argument");
    if (jt->opt.host_only) return fail(FBN_E_STATE, "host-only jt");
    JointArgs a;
    int home = -1;
    fbn_status st = joint_plan(jt, slot, n_q, q_vars, out_len, a, home);
    if (st) return st;
    HIP_OK(hipSetDevice(jt->device));
    if ((st = wait_staged(jt))) return st;
    // a slot whose FP32 tables vanished (flag 2), or whose results were
    // recomputed in FP64 (flag 4), is read from the FP64 tree recalibrated
    // for its evidence when the jt reruns underflows in FP64
    int32_t f0 = 0;
    HIP_OK(hipMemcpyAsync(&f0, jt->d_flags + slot, 4, hipMemcpyDeviceToHost, jt->stream));
    HIP_OK(hipStreamSynchronize(jt->stream));
    const bool twin = jt->opt.fp64_rerun && jt->opt.precision == FBN_FP32_RESCALED && (f0 & 6);
    if (twin) {
        int32_t f = 2;
        if ((st = rerun_fp64(jt, 1, &slot, &f, nullptr))) return st;
    }
    void* dev = temp_alloc(jt, 8 * joint_scratch_doubles(a));
    if (!dev) return fail(FBN_E_NOMEM_DEVICE, "device allocation failed");
    if (twin) {
        JointArgs b = a;
        b.slot = 0;
        st = joint_run(jt->twin, home, b, static_cast<double*>(dev), out);
    } else {
        st = joint_run(jt, home, a, static_cast<double*>(dev), out);
    }
    const std::string keep = g_err;
    hipStreamSynchronize(jt->stream);
    temp_free(jt, dev);
    g_err = keep;
    return st;
}

fbn_status fbn_query_joint_noalloc(fbn_jt* jt, int32_t slot, int32_t n_q, const int32_t* q_vars, double* out,
                                   size_t out_len) {
    if (!jt || !out) return fail(FBN_E_INVALID_ARG, "null argument");
    if (jt->opt.host_only) return fail(FBN_E_STATE, "host-only jt");
    JointArgs a;
    int home = -1;
    fbn_status st = joint_plan(jt, slot, n_q, q_vars, out_len, a, home);
    if (st) return st;
    if (joint_scratch_doubles(a) > kJointScratchDoubles)
        return fail(FBN_E_TOO_LARGE, "the joint read-out needs " + std::to_string(joint_scratch_doubles(a)) +
                                         " scratch doubles, more than the " + std::to_string(kJointScratchDoubles) +
                                         " of the static buffer");
    HIP_OK(hipSetDevice(jt->device));
    if ((st = wait_staged(jt))) return st;
    double* dev = nullptr;
    HIP_OK(joint_static_scratch(&dev));
    return joint_run(jt, home, a, dev, out);
}

fbn_status fbn_jt_stats(const fbn_jt* jt, fbn_jt_stats_t* out) {
    if (!jt || !out) return fail(FBN_E_INVALID_ARG, "null argument");
    const Tree& t = jt->tree;
    std::memset(out, 0, sizeof(*out));
    out->n_vars = t.n;
    out->n_cliques = t.nc;
    out->n_edges = t.ne;
    out->root = t.root;
    out->n_trees = (int32_t)t.roots.size();
    out->interleaved = jt->plan.interleaved ? 1 : 0;
    for (int c = 0; c < t.nc; c++) {
        out->H = std::max(out->H, t.height[(size_t)c]);
        out->D = std::max(out->D, t.depth[(size_t)c]);
        out->T += t.size[(size_t)c];
        out->max_clique = std::max(out->max_clique, t.size[(size_t)c]);
    }
    for (int e = 0; e < t.ne; e++) {
        out->K += t.size[(size_t)t.e_parent[(size_t)e]];
        out->sep_total += t.e_size[(size_t)e];
    }
    out->device_bytes = jt->device_bytes;
    out->slot_bytes = jt->slot_bytes;
    return FBN_OK;
}

fbn_status fbn_jt_clique(const fbn_jt* jt, int32_t c, int32_t* vars, int32_t cap, int32_t* n, int32_t* height,
                         int32_t* depth) {
    if (!jt || c < 0 || c >= jt->tree.nc) return fail(FBN_E_INVALID_ARG, "bad clique");
    const auto& v = jt->tree.vars[(size_t)c];
    for (int32_t k = 0; k < (int32_t)v.size() && k < cap && vars; k++) vars[k] = v[(size_t)k];
    if (n) *n = (int32_t)v.size();
    if (height) *height = jt->tree.height[(size_t)c];
    if (depth) *depth = jt->tree.depth[(size_t)c];
    return FBN_OK;
}

fbn_status fbn_jt_edge(const fbn_jt* jt, int32_t e, int32_t* parent, int32_t* child, int32_t* sep, int32_t cap,
                       int32_t* n) {
    if (!jt || e < 0 || e >= jt->tree.ne) return fail(FBN_E_INVALID_ARG, "bad edge");
    if (parent) *parent = jt->tree.e_parent[(size_t)e];
    if (child) *child = jt->tree.e_child[(size_t)e];
    const auto& s = jt->tree.e_sep[(size_t)e];
    for (int32_t k = 0; k < (int32_t)s.size() && k < cap && sep; k++) sep[k] = s[(size_t)k];
    if (n) *n = (int32_t)s.size();
    return FBN_OK;
}

static const DChild* child_record(const fbn_jt* jt, int32_t e, const DClique** parent) {
    const int p = jt->tree.e_parent[(size_t)e];
    const DClique& d = jt->plan.cliques[(size_t)p];
    const auto& kids = jt->tree.children[(size_t)p];
    for (size_t k = 0; k < kids.size(); k++)
        if (jt->tree.pedge[(size_t)kids[k]] == e) {
            *parent = &d;
            return &jt->plan.children[d.child0 + k];
        }
    return nullptr;
}

fbn_status fbn_jt_index_map(const fbn_jt* jt, int32_t e, int32_t* out, size_t cap) {
    if (!jt || !out || e < 0 || e >= jt->tree.ne) return fail(FBN_E_INVALID_ARG, "bad edge");
    const DClique* d = nullptr;
    const DChild* r = child_record(jt, e, &d);
    if (!r) return fail(FBN_E_STATE, "edge record missing");
    if (cap < d->size) return fail(FBN_E_INVALID_ARG, "output too small");
    const auto& m = jt->plan.maps;
    for (uint32_t j = 0; j < d->size; j++) out[j] = (int32_t)(m[r->mh + j / d->L] + m[r->ml + j % d->L]);
    return FBN_OK;
}

fbn_status fbn_jt_device_index_map(fbn_jt* jt, int32_t e, int32_t* out, size_t cap) {
    if (!jt || !out || e < 0 || e >= jt->tree.ne) return fail(FBN_E_INVALID_ARG, "bad edge");
    if (jt->opt.host_only) return fail(FBN_E_STATE, "host-only jt");
    const DClique* d = nullptr;
    const DChild* r = child_record(jt, e, &d);
    if (!r) return fail(FBN_E_STATE, "edge record missing");
    if (cap < d->size) return fail(FBN_E_INVALID_ARG, "output too small");
    HIP_OK(hipSetDevice(jt->device));
    int32_t* tmp = nullptr;
    HIP_OK(hipMalloc(&tmp, 4ull * d->size));
    hipError_t err = launch_expand_map(jt->d_map, r->mh, r->ml, d->L, d->Lmul, d->Lsh, d->size, tmp, jt->stream);
    if (err == hipSuccess) err = hipMemcpyAsync(out, tmp, 4ull * d->size, hipMemcpyDeviceToHost, jt->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(jt->stream);
    hipFree(tmp);
    if (err != hipSuccess) return fail(FBN_E_DEVICE, hipGetErrorString(err));
    return FBN_OK;
}

fbn_status fbn_jt_profile_enable(fbn_jt* jt, int32_t on) {
    if (!jt) return fail(FBN_E_INVALID_ARG, "null jt");
    if (jt->opt.host_only) return fail(FBN_E_STATE, "host-only jt");
    jt->prof = on != 0;
    return FBN_OK;
}

fbn_status fbn_jt_profile_kinds(fbn_jt* jt, uint32_t mask) {
    if (!jt) return fail(FBN_E_INVALID_ARG, "null jt");
    if (mask >> FBN_PROFILE_KINDS) return fail(FBN_E_INVALID_ARG, "unknown profile kind");
    jt->prof_mask = mask;
    return FBN_OK;
}

fbn_status fbn_jt_profile_read(fbn_jt* jt, double* ms, int64_t* launches, double* bytes) {
    if (!jt) return fail(FBN_E_INVALID_ARG, "null jt");
    if (jt->opt.host_only) return fail(FBN_E_STATE, "host-only jt");
    HIP_OK(hipStreamSynchronize(jt->stream));
    for (auto& r : jt->recs) {
        float t = 0.f;
        HIP_OK(hipEventElapsedTime(&t, r.a, r.b));
        jt->prof_ms[r.kind] += (double)t;
        jt->prof_bytes[r.kind] += r.bytes;
        jt->prof_n[r.kind] += 1;
        jt->pool.push_back(r.a);
        jt->pool.push_back(r.b);
    }
    jt->recs.clear();
    for (int k = 0; k < FBN_PROFILE_KINDS; k++) {
        if (ms) ms[k] = jt->prof_ms[k];
        if (launches) launches[k] = jt->prof_n[k];
        if (bytes) bytes[k] = jt->prof_bytes[k];
        jt->prof_ms[k] = jt->prof_bytes[k] = 0.0;
        jt->prof_n[k] = 0;
    }
    return FBN_OK;
}

fbn_status fbn_jt_elim_order(const fbn_jt* jt, int32_t* order) {
    if (!jt || !order) return fail(FBN_E_INVALID_ARG, "null argument");
    for (int v = 0; v < jt->tree.n; v++) order[v] = jt->tree.elim_order[(size_t)v];
    return FBN_OK;
}

fbn_status fbn_jt_homes(const fbn_jt* jt, int32_t* cpt_home, int32_t* var_home) {
    if (!jt) return fail(FBN_E_INVALID_ARG, "null jt");
    for (int v = 0; v < jt->tree.n; v++) {
        if (cpt_home) cpt_home[v] = jt->tree.cpt_home[(size_t)v];
        if (var_home) var_home[v] = jt->tree.var_home[(size_t)v];
    }
    return FBN_OK;
}

}  // extern "C"
