// Device plan construction.
//
// The paper's key step for the table operations is the index mapping
// between a table and the table it is marginalised onto or extended from
// (Section 2).  Here every map is precomputed once per network.  A separator
// index is a weighted sum of the clique's digits, so with the clique's
// entries split as i = hi * L + lo (L = product of the fastest variables'
// cardinalities) each map is exactly H[hi] + Lo[lo]: two small tables per
// edge instead of one entry per clique entry.  The digits themselves are
// packed into one 64-bit word per entry the same way (hi word | lo word),
// which lets the kernels test evidence and read a home variable's state with
// a mask and a shift.
//
// Work is laid out per layer (Section 2: all the table entries of a layer
// form one parallel task): the entries of every clique in the layer are cut
// into runs and packed into workgroup tiles of at most `tile` entries, so
// many small cliques share a workgroup and a huge clique spreads over many.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <type_traits>

namespace fbn {

void magic_u32(uint32_t d, uint32_t& mul, uint32_t& sh) {
    uint32_t s = 0;
    while ((1ull << s) < d) s++;
    uint64_t m = (((1ull << 32) * ((1ull << s) - d)) / d) + 1;
    mul = (uint32_t)m;
    sh = s;
}

static uint32_t bits_for(int r) {
    uint32_t b = 0;
    while ((1u << b) < (uint32_t)r) b++;
    return b;
}

namespace {

struct Packer {
    Plan& p;
    int tile;
    int32_t open = -1;  // index of the open full group, or -1
    void close() { open = -1; }
    void add_full(uint32_t clique, uint32_t begin, uint32_t count) {
        if (open >= 0) {
            DGroup& g = p.groups[(size_t)open];
            if (g.total + count > (uint32_t)tile || g.npiece >= (uint32_t)kMaxPieces) open = -1;
        }
        if (open < 0) {
            DGroup g{};
            g.piece0 = (uint32_t)p.pieces.size();
            g.npiece = 0;
            g.total = 0;
            g.part = -1;
            p.groups.push_back(g);
            open = (int32_t)p.groups.size() - 1;
        }
        DGroup& g = p.groups[(size_t)open];
        p.pieces.push_back({clique, begin, count, g.total});
        g.npiece++;
        g.total += count;
    }
    void add_part(uint32_t clique, uint32_t begin, uint32_t count, int32_t part) {
        DGroup g{};
        g.piece0 = (uint32_t)p.pieces.size();
        g.npiece = 1;
        g.total = count;
        g.part = part;
        p.pieces.push_back({clique, begin, count, 0});
        p.groups.push_back(g);
    }
};

}  // namespace

std::string check_plan(const Tree& t, const Plan& p) {
    auto bad = [](const std::string& s) { return s; };
    const size_t nc = p.cliques.size();
    if (nc != (size_t)t.nc) return bad("clique count");
    uint64_t sum = 0;
    for (size_t c = 0; c < nc; c++) {
        const DClique& d = p.cliques[c];
        if (d.off != sum || d.size != t.size[c] || d.size == 0) return bad("clique offset/size");
        sum += d.size;
        if (d.L == 0 || d.size % d.L) return bad("split");
        const uint32_t rows = d.size / d.L;
        for (uint32_t x : {0u, d.size - 1, d.size / 2, d.L, d.L - 1})
            if (x < d.size && (uint32_t)(((uint64_t)(((uint64_t)x * d.Lmul) >> 32) + x) >> d.Lsh) != x / d.L)
                return bad("magic division");
        if ((uint64_t)d.hdig + rows > p.digits.size() || (uint64_t)d.ldig + d.L > p.digits.size()) return bad("digit tables");
        const uint32_t psize = (int)c == t.root ? 1u : (uint32_t)t.e_size[(size_t)t.pedge[c]];
        if (d.seg == 0 || d.size != d.seg * psize) return bad("segment");
        if ((uint64_t)d.psep + psize > p.sep_total + 1ull) return bad("parent separator offset");
        auto check_map = [&](uint32_t mh, uint32_t ml, uint32_t limit) -> bool {
            if ((uint64_t)mh + rows > p.maps.size() || (uint64_t)ml + d.L > p.maps.size()) return false;
            uint64_t mx_h = 0, mx_l = 0;
            for (uint32_t r = 0; r < rows; r++) mx_h = std::max<uint64_t>(mx_h, p.maps[mh + r]);
            for (uint32_t l = 0; l < d.L; l++) mx_l = std::max<uint64_t>(mx_l, p.maps[ml + l]);
            return mx_h + mx_l < limit;
        };
        if ((int)c != t.root && !check_map(d.pmh, d.pml, psize)) return bad("parent map range");
        if ((uint64_t)d.child0 + d.nchild > p.children.size() || d.nchild != t.children[c].size()) return bad("children");
        for (uint32_t k = 0; k < d.nchild; k++) {
            const DChild& r = p.children[d.child0 + k];
            if ((uint64_t)r.sep + r.size > p.sep_total) return bad("child separator offset");
            if (!check_map(r.mh, r.ml, r.size)) return bad("child map range");
        }
        if ((uint64_t)d.home0 + d.nhome > p.homes.size()) return bad("homes");
        for (uint32_t k = 0; k < d.nhome; k++) {
            const DHome& h = p.homes[d.home0 + k];
            if ((uint64_t)h.out + h.card > p.marg_total) return bad("home range");
            if (h.mask + 1 < h.card || h.shift >= 64) return bad("home digit");
        }
    }
    if (sum != p.T) return bad("arena size");
    auto check_layers = [&](const std::vector<Layer>& layers, bool collect) -> std::string {
        for (const Layer& ly : layers) {
            if ((uint64_t)ly.group0 + ly.ngroup > p.groups.size()) return "layer groups";
            if ((uint64_t)ly.fin0 + ly.nfin > p.fins.size()) return "layer fins";
            for (uint32_t g = ly.group0; g < ly.group0 + ly.ngroup; g++) {
                const DGroup& G = p.groups[g];
                if (G.total == 0 || G.total > (uint32_t)p.tile || G.total > (uint32_t)kTileMax) return "tile size";
                if (G.npiece == 0 || G.npiece > (uint32_t)kMaxPieces) return "piece count";
                if ((uint64_t)G.piece0 + G.npiece > p.pieces.size()) return "piece range";
                if (G.part >= 0 && (G.npiece != 1 || (uint32_t)G.part >= p.n_parts || !collect)) return "partial group";
                uint32_t ofs = 0;
                for (uint32_t k = 0; k < G.npiece; k++) {
                    const DPiece& pc = p.pieces[G.piece0 + k];
                    if (pc.clique >= nc || pc.count == 0 || pc.gofs != ofs) return "piece layout";
                    const DClique& d = p.cliques[pc.clique];
                    if ((uint64_t)pc.begin + pc.count > d.size) return "piece bounds";
                    if (collect && G.part < 0 && (pc.begin % d.seg || pc.count % d.seg)) return "piece alignment";
                    if (collect && G.part >= 0 && pc.begin / d.seg != (pc.begin + pc.count - 1) / d.seg) return "partial piece spans segments";
                    ofs += pc.count;
                }
                if (ofs != G.total) return "tile total";
            }
            for (uint32_t f = ly.fin0; f < ly.fin0 + ly.nfin; f++) {
                const DSepFin& F = p.fins[f];
                if ((uint64_t)F.sep + F.size > p.sep_total + 1ull) return "fin range";
                if (F.nchunk && (uint64_t)F.part0 + (uint64_t)F.size * F.nchunk > p.n_parts) return "fin partials";
                if (F.edge >= t.ne || (F.edge < 0 && F.size != 1)) return "fin edge";
            }
        }
        return "";
    };
    std::string e = check_layers(p.collect, true);
    if (!e.empty()) return e;
    e = check_layers(p.distribute, false);
    if (!e.empty()) return e;
    if ((uint64_t)p.sep_stride < (uint64_t)p.sep_total + 1) return "separator stride";
    return "";
}

void build_plan(const Tree& t, int tile, Plan& p) {
    p = Plan();
    if (tile <= 0) tile = 2048;
    tile = std::min(tile, kTileMax);
    p.tile = tile;
    const int nc = t.nc;

    // separator arena: edges in id order, then the root's virtual entry
    p.sep_off.resize((size_t)t.ne);
    uint64_t so = 0;
    for (int e = 0; e < t.ne; e++) {
        p.sep_off[(size_t)e] = (uint32_t)so;
        so += t.e_size[(size_t)e];
    }
    if (so + 1 > 0x7fffffffull) throw std::runtime_error("separators too large");
    p.sep_total = (uint32_t)so;
    p.sep_stride = (uint32_t)((so + 1 + 63) / 64 * 64);

    // marginal offsets
    std::vector<uint32_t> marg_off((size_t)t.n);
    uint32_t mo = 0;
    for (int v = 0; v < t.n; v++) {
        marg_off[(size_t)v] = mo;
        p.homevars.push_back({mo, (uint32_t)t.card[(size_t)v]});
        mo += (uint32_t)t.card[(size_t)v];
    }
    p.marg_total = mo;

    std::vector<std::vector<int>> homed((size_t)nc);
    for (int v = 0; v < t.n; v++) homed[(size_t)t.var_home[(size_t)v]].push_back(v);

    // per-clique records, tables in id order
    p.cliques.resize((size_t)nc);
    p.kappa.assign((size_t)nc, 0);
    uint64_t off = 0;
    for (int c = 0; c < nc; c++) {
        const auto& lay = t.vars[(size_t)c];
        const int m = (int)lay.size();
        const uint64_t size = t.size[(size_t)c];
        DClique& d = p.cliques[(size_t)c];
        d = DClique{};
        d.off = off;
        d.size = (uint32_t)size;
        off += size;
        // split point: smallest suffix product >= 64, or the whole clique
        int q = m;
        uint64_t L = 1;
        while (q > 0 && L < 64) {
            q--;
            L *= (uint64_t)t.card[(size_t)lay[(size_t)q]];
        }
        const uint64_t rows = size / L;
        d.L = (uint32_t)L;
        magic_u32(d.L, d.Lmul, d.Lsh);
        // digit bit positions, layout order from the lowest bits
        std::vector<uint32_t> shift((size_t)m), nbits((size_t)m);
        uint32_t sh = 0;
        for (int k = 0; k < m; k++) {
            shift[(size_t)k] = sh;
            nbits[(size_t)k] = bits_for(t.card[(size_t)lay[(size_t)k]]);
            sh += nbits[(size_t)k];
        }
        if (sh > 64) throw std::runtime_error("clique digits exceed 64 bits");
        p.dig_shift0.push_back((uint32_t)p.dig_shift.size());
        for (int k = 0; k < m; k++) p.dig_shift.push_back(shift[(size_t)k]);
        // a factored table: value(row or lo) = sum over positions in [a, b)
        // of digit * weight[position]
        auto table = [&](int a, int b, uint64_t count, const std::vector<uint64_t>& weight, bool packed,
                         auto& pool) -> uint32_t {
            const uint32_t start = (uint32_t)pool.size();
            std::vector<int> dg((size_t)(b - a), 0);
            for (uint64_t x = 0; x < count; x++) {
                uint64_t val = 0;
                for (int k = a; k < b; k++) {
                    const uint64_t digit = (uint64_t)dg[(size_t)(k - a)];
                    val += packed ? (digit << shift[(size_t)k]) : digit * weight[(size_t)k];
                }
                pool.push_back((typename std::remove_reference<decltype(pool)>::type::value_type)val);
                for (int k = b - 1; k >= a; k--) {
                    if (++dg[(size_t)(k - a)] < t.card[(size_t)lay[(size_t)k]]) break;
                    dg[(size_t)(k - a)] = 0;
                }
            }
            return start;
        };
        std::vector<uint64_t> none((size_t)m, 0);
        d.hdig = table(0, q, rows, none, true, p.digits);
        d.ldig = table(q, m, L, none, true, p.digits);
        // parent map (prefix of the layout) and segment length
        if (c == t.root) {
            d.pedge = -1;
            d.psep = p.sep_total;
            d.seg = (uint32_t)size;
            d.pmh = d.pml = 0;
        } else {
            const int e = t.pedge[(size_t)c];
            const int ns = (int)t.e_sep[(size_t)e].size();
            std::vector<uint64_t> w((size_t)m, 0);
            uint64_t s = 1;
            for (int k = ns - 1; k >= 0; k--) {
                w[(size_t)k] = s;
                s *= (uint64_t)t.card[(size_t)lay[(size_t)k]];
            }
            d.pedge = e;
            d.psep = p.sep_off[(size_t)e];
            d.seg = (uint32_t)(size / t.e_size[(size_t)e]);
            d.pmh = table(0, q, rows, w, false, p.maps);
            d.pml = table(q, m, L, w, false, p.maps);
        }
        // child maps: separator variables ascending, last fastest
        d.child0 = (uint32_t)p.children.size();
        d.nchild = (uint16_t)t.children[(size_t)c].size();
        for (int ch : t.children[(size_t)c]) {
            const int e = t.pedge[(size_t)ch];
            const auto& sv = t.e_sep[(size_t)e];
            std::vector<uint64_t> w((size_t)m, 0);
            uint64_t s = 1;
            for (size_t k = sv.size(); k-- > 0;) {
                for (int j = 0; j < m; j++)
                    if (lay[(size_t)j] == sv[k]) w[(size_t)j] = s;
                s *= (uint64_t)t.card[(size_t)sv[k]];
            }
            DChild r{};
            r.sep = p.sep_off[(size_t)e];
            r.size = (uint32_t)t.e_size[(size_t)e];
            r.mh = table(0, q, rows, w, false, p.maps);
            r.ml = table(q, m, L, w, false, p.maps);
            p.children.push_back(r);
        }
        // home variables
        d.home0 = (uint32_t)p.homes.size();
        d.nhome = (uint16_t)homed[(size_t)c].size();
        for (int v : homed[(size_t)c]) {
            int k = 0;
            while (lay[(size_t)k] != v) k++;
            p.homes.push_back({marg_off[(size_t)v], shift[(size_t)k], (1u << nbits[(size_t)k]) - 1u,
                               (uint32_t)t.card[(size_t)v]});
        }
        // scaled prior: max scaled into [0.5, 1) by an exact power of two
        double mx = 0.0;
        for (double x : t.prior[(size_t)c]) mx = std::max(mx, x);
        int kap = 0;
        if (mx > 0.0) std::frexp(mx, &kap);
        p.kappa[(size_t)c] = kap;
        p.kappa_total += kap;
    }
    p.T = off;
    p.prior.resize(off);
    for (int c = 0; c < nc; c++) {
        const auto& src = t.prior[(size_t)c];
        double* dst = p.prior.data() + p.cliques[(size_t)c].off;
        for (size_t i = 0; i < src.size(); i++) dst[i] = std::ldexp(src[i], -p.kappa[(size_t)c]);
    }

    // ---- collect layers (height) and their separator finalisation
    int H = 0, D = 0;
    for (int c = 0; c < nc; c++) {
        H = std::max(H, t.height[(size_t)c]);
        D = std::max(D, t.depth[(size_t)c]);
    }
    p.collect.assign((size_t)H + 1, Layer());
    uint32_t parts = 0;
    for (int h = 0; h <= H; h++) {
        Layer& ly = p.collect[(size_t)h];
        ly.group0 = (uint32_t)p.groups.size();
        Packer pk{p, tile};
        std::vector<DSepFin> fins;
        for (int c = 0; c < nc; c++) {
            if (t.height[(size_t)c] != h) continue;
            const DClique& d = p.cliques[(size_t)c];
            const uint32_t seg = d.seg;
            DSepFin f{};
            f.sep = d.psep;
            f.size = d.size / seg;
            f.edge = d.pedge;
            if (seg <= (uint32_t)tile) {
                const uint32_t per = ((uint32_t)tile / seg) * seg;
                for (uint32_t b = 0; b < d.size; b += per) pk.add_full((uint32_t)c, b, std::min(per, d.size - b));
            } else {
                // nchunk near-equal chunks: [k*seg/nchunk, (k+1)*seg/nchunk)
                const uint32_t nchunk = (seg + (uint32_t)tile - 1) / (uint32_t)tile;
                f.part0 = parts;
                f.nchunk = nchunk;
                for (uint32_t s = 0; s < f.size; s++)
                    for (uint32_t k = 0; k < nchunk; k++) {
                        const uint32_t b = (uint32_t)((uint64_t)k * seg / nchunk);
                        const uint32_t e = (uint32_t)((uint64_t)(k + 1) * seg / nchunk);
                        pk.add_part((uint32_t)c, s * seg + b, e - b, (int32_t)(parts + s * nchunk + k));
                    }
                parts += f.size * nchunk;
            }
            fins.push_back(f);
        }
        ly.ngroup = (uint32_t)p.groups.size() - ly.group0;
        ly.fin0 = (uint32_t)p.fins.size();
        ly.nfin = (uint32_t)fins.size();
        p.fins.insert(p.fins.end(), fins.begin(), fins.end());
    }
    p.n_parts = parts;

    // ---- distribute layers (depth); after layer d the separators towards
    // the children of its cliques are finalised
    p.distribute.assign((size_t)D + 1, Layer());
    for (int dd = 0; dd <= D; dd++) {
        Layer& ly = p.distribute[(size_t)dd];
        ly.group0 = (uint32_t)p.groups.size();
        Packer pk{p, tile};
        std::vector<DSepFin> fins;
        for (int c = 0; c < nc; c++) {
            if (t.depth[(size_t)c] != dd) continue;
            const DClique& d = p.cliques[(size_t)c];
            for (uint32_t b = 0; b < d.size; b += (uint32_t)tile) pk.add_full((uint32_t)c, b, std::min((uint32_t)tile, d.size - b));
            for (int ch : t.children[(size_t)c]) {
                const int e = t.pedge[(size_t)ch];
                DSepFin f{};
                f.sep = p.sep_off[(size_t)e];
                f.size = (uint32_t)t.e_size[(size_t)e];
                f.edge = e;
                fins.push_back(f);
            }
        }
        ly.ngroup = (uint32_t)p.groups.size() - ly.group0;
        ly.fin0 = (uint32_t)p.fins.size();
        ly.nfin = (uint32_t)fins.size();
        p.fins.insert(p.fins.end(), fins.begin(), fins.end());
    }
}

}  // namespace fbn
