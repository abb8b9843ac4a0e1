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
// which lets the kernels test evidence with a mask.
//
// Work is laid out per layer (Section 2: all the table entries of a layer
// form one parallel task).  Collect: the entries of every clique in the
// layer are cut into runs aligned to parent-separator segments and packed
// into workgroup tiles, so many small cliques share a workgroup and a huge
// clique spreads over many.  Distribute: every marginalisation of a clique
// onto a child separator becomes a list of workgroups, each gathering whole
// rows of the clique for a block of separator entries (no atomics).
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

// Table entries one distribute work item stages per slot.
static uint32_t work_entries(const Plan& p, const DWork& w) {
    return w.npiece ? w.total : w.ng * w.nk * p.cliques[p.targets[w.target].clique].L;
}

static uint32_t mdiv_host(uint32_t n, uint32_t mul, uint32_t sh) {
    return (uint32_t)(((uint64_t)(((uint64_t)n * mul) >> 32) + n) >> sh);
}

namespace {

struct Packer {
    Plan& p;
    int tile;
    int32_t open = -1;  // index of the open full group, or -1
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
        open = -1;  // runs of one group must stay contiguous in the run list
        DGroup g{};
        g.piece0 = (uint32_t)p.pieces.size();
        g.npiece = 1;
        g.total = count;
        g.part = part;
        p.pieces.push_back({clique, begin, count, 0});
        p.groups.push_back(g);
    }
};

// Append the mixed-radix enumeration over layout positions `pos` (last
// fastest) of sum_k digit_k * weight[pos_k] to pool; returns its offset.
uint32_t enumerate(const std::vector<int>& pos, const std::vector<int>& card_at, const std::vector<uint64_t>& weight,
                   std::vector<uint32_t>& pool) {
    const uint32_t start = (uint32_t)pool.size();
    uint64_t count = 1;
    for (int k : pos) count *= (uint64_t)card_at[(size_t)k];
    std::vector<int> dg(pos.size(), 0);
    for (uint64_t x = 0; x < count; x++) {
        uint64_t v = 0;
        for (size_t a = 0; a < pos.size(); a++) v += (uint64_t)dg[a] * weight[(size_t)pos[a]];
        if (v > 0xffffffffull) throw std::runtime_error("index table overflow");
        pool.push_back((uint32_t)v);
        for (size_t a = pos.size(); a-- > 0;) {
            if (++dg[a] < card_at[(size_t)pos[a]]) break;
            dg[a] = 0;
        }
    }
    return start;
}

// Finalised in blocks: a real separator above the size threshold, or any
// real or one-variable separator whose entries add many partial sums.
bool is_big(const Plan& p, const DSepFin& f) {
    if (f.edge == -1) return false;
    return (f.size > p.big_separator && f.edge >= 0) || (uint64_t)f.size * f.nchunk > p.fin_work;
}

// Partition a layer's finalisers large-first and split each large one into
// near-equal blocks of at most kFinBlock entries.
void finish_layer(Plan& p, Layer& ly, std::vector<DSepFin>& fins) {
    auto big = [&](const DSepFin& f) { return is_big(p, f); };
    std::stable_partition(fins.begin(), fins.end(), big);
    ly.fin0 = (uint32_t)p.fins.size();
    ly.nfin = (uint32_t)fins.size();
    ly.nbig = (uint32_t)std::count_if(fins.begin(), fins.end(), big);
    // after the large ones, those that get a workgroup team
    std::stable_partition(fins.begin() + ly.nbig, fins.end(),
                          [](const DSepFin& f) { return f.size > kTeamSeparator; });
    ly.nteam = (uint32_t)std::count_if(fins.begin() + ly.nbig, fins.end(),
                                       [](const DSepFin& f) { return f.size > kTeamSeparator; });
    p.fins.insert(p.fins.end(), fins.begin(), fins.end());
    ly.fb0 = (uint32_t)p.finblks.size();
    for (uint32_t f = ly.fin0; f < ly.fin0 + ly.nbig; f++) {
        const DSepFin F = p.fins[f];
        // entries per block: at most fin_block, and at most kFinWork partial sums
        const uint32_t per = (uint32_t)std::max<uint64_t>(
            1, std::min<uint64_t>(p.fin_block, p.fin_work / std::max<uint32_t>(F.nchunk, 1)));
        const uint32_t nblk = (F.size + per - 1) / per;
        uint32_t mw = 0;
        for (uint32_t k = 0; k < F.nmv; k++) mw += p.margvars[F.mv0 + k].card;
        const uint32_t blk0 = (uint32_t)p.finblks.size();
        const uint32_t mx = p.n_bigfin++;
        const uint32_t mbase = p.n_bmarg;
        if ((uint64_t)p.n_bmarg + (uint64_t)mw * nblk > 0x7fffffffull) throw std::runtime_error("finaliser scratch");
        p.n_bmarg += mw * nblk;
        for (uint32_t j = 0; j < nblk; j++) {
            const uint32_t b = (uint32_t)((uint64_t)j * F.size / nblk);
            const uint32_t e = (uint32_t)((uint64_t)(j + 1) * F.size / nblk);
            p.finblks.push_back({f, b, e - b, blk0 + j, blk0, nblk, mbase, mw, mx});
        }
    }
    ly.nfb = (uint32_t)p.finblks.size() - ly.fb0;
}

}  // namespace

std::string check_plan(const Tree& t, const Plan& p) {
    const size_t nc = p.cliques.size();
    if (nc != (size_t)t.nc) return "clique count";
    uint64_t sum = 0;
    for (size_t c = 0; c < nc; c++) {
        const DClique& d = p.cliques[c];
        if (d.off != sum || d.size != t.size[c] || d.size == 0) return "clique offset/size";
        sum += d.size;
        if (d.L == 0 || d.L > (uint32_t)kTileMax || d.size % d.L) return "split";
        const uint32_t rows = d.size / d.L;
        for (uint32_t x : {0u, d.size - 1, d.size / 2, d.L, d.L - 1})
            if (x < d.size && mdiv_host(x, d.Lmul, d.Lsh) != x / d.L) return "magic division";
        if ((uint64_t)d.hdig + rows > p.digits.size() || (uint64_t)d.ldig + d.L > p.digits.size()) return "digit tables";
        const bool is_root = t.pedge[c] < 0;
        const uint32_t psize = is_root ? 1u : (uint32_t)t.e_size[(size_t)t.pedge[c]];
        if (d.seg == 0 || d.size != d.seg * psize) return "segment";
        for (uint32_t i : {0u, d.size - 1, d.size / 2, d.size / 3, d.seg, d.seg - 1, d.L, d.size / 7})
            if (i < d.size && mdiv_host(i, d.segmul, d.segsh) != i / d.seg) return "segment magic";
        if (!is_root && (uint64_t)d.pmh + rows <= p.maps.size() && (uint64_t)d.pml + d.L <= p.maps.size()) {
            // the parent separator leads the layout: entry i lies in its entry
            // i / seg, which the distribute gathers compute instead of loading
            for (uint32_t i : {0u, d.size - 1, d.size / 2, d.size / 3, d.seg, d.seg - 1, d.L, d.size / 7})
                if (i < d.size && p.maps[d.pmh + i / d.L] + p.maps[d.pml + i % d.L] != i / d.seg)
                    return "parent map is not i / seg";
        }
        if ((uint64_t)d.psep + psize > p.sep_real) return "parent separator offset";
        auto check_map = [&](uint32_t mh, uint32_t ml, uint32_t limit) -> bool {
            if ((uint64_t)mh + rows > p.maps.size() || (uint64_t)ml + d.L > p.maps.size()) return false;
            uint64_t mx_h = 0, mx_l = 0;
            for (uint32_t r = 0; r < rows; r++) mx_h = std::max<uint64_t>(mx_h, p.maps[mh + r]);
            for (uint32_t l = 0; l < d.L; l++) mx_l = std::max<uint64_t>(mx_l, p.maps[ml + l]);
            return mx_h + mx_l < limit;
        };
        if (is_root != (d.pedge < 0) || (is_root && (d.psep < p.sep_total || d.psep >= p.sep_real)))
            return "root separator";
        if (!is_root && !check_map(d.pmh, d.pml, psize)) return "parent map range";
        if ((uint64_t)d.child0 + d.nchild > p.children.size() || d.nchild != t.children[c].size()) return "children";
        if (d.psi != kNoPsi && (uint64_t)d.psi + d.size > p.psi_total) return "working-table arena";
        if (d.psi == kNoPsi && (!p.interleaved || d.nchild > kRebuildKidsInterleaved)) return "rebuilt working table";
        for (uint32_t k = 0; k < d.nchild; k++) {
            const DChild& r = p.children[d.child0 + k];
            if ((uint64_t)r.sep + r.size > p.sep_total) return "child separator offset";
            if (!check_map(r.mh, r.ml, r.size)) return "child map range";
        }
    }
    if (sum != p.T) return "arena size";
    // collect layers
    for (const Layer& ly : p.collect) {
        if ((uint64_t)ly.group0 + ly.ngroup > p.groups.size()) return "layer groups";
        if ((uint64_t)ly.fin0 + ly.nfin > p.fins.size()) return "layer fins";
        for (uint32_t g = ly.group0; g < ly.group0 + ly.ngroup; g++) {
            const DGroup& G = p.groups[g];
            if (G.total == 0 || G.total > (uint32_t)p.tile || G.total > (uint32_t)kTileMax) return "tile size";
            if (G.npiece == 0 || G.npiece > (uint32_t)kMaxPieces) return "piece count";
            if ((uint64_t)G.piece0 + G.npiece > p.pieces.size()) return "piece range";
            if (G.part >= 0 && (G.npiece != 1 || (uint32_t)G.part >= p.n_parts)) return "partial group";
            uint32_t ofs = 0;
            for (uint32_t k = 0; k < G.npiece; k++) {
                const DPiece& pc = p.pieces[G.piece0 + k];
                if (pc.clique >= nc || pc.count == 0 || pc.gofs != ofs) return "piece layout";
                const DClique& d = p.cliques[pc.clique];
                if ((uint64_t)pc.begin + pc.count > d.size) return "piece bounds";
                if (G.part < 0 && (pc.begin % d.seg || pc.count % d.seg)) return "piece alignment";
                if (G.part >= 0 && pc.begin / d.seg != (pc.begin + pc.count - 1) / d.seg) return "partial piece spans segments";
                ofs += pc.count;
            }
            if (ofs != G.total) return "tile total";
        }
    }
    // distribute layers
    for (const Layer& ly : p.distribute) {
        if ((uint64_t)ly.group0 + ly.ngroup > p.works.size()) return "layer works";
        if ((uint64_t)ly.fin0 + ly.nfin > p.fins.size()) return "layer fins";
        for (uint32_t w = ly.group0; w < ly.group0 + ly.ngroup; w++) {
            const DWork& W = p.works[w];
            if (p.interleaved && W.npiece > 0) return "packed work in an interleaved plan";
            if (W.npiece > 0) {
                // packed: whole cliques staged in LDS and all their targets
                if (W.npiece > (uint32_t)kMaxPieces || (uint64_t)W.piece0 + W.npiece > p.pieces.size()) return "packed pieces";
                if (W.total == 0 || W.total > (uint32_t)kTileMax) return "packed tile";
                uint32_t ofs = 0;
                for (uint32_t k = 0; k < W.npiece; k++) {
                    const DPiece& pc = p.pieces[W.piece0 + k];
                    if (pc.clique >= nc || pc.begin != 0 || pc.count != p.cliques[pc.clique].size || pc.gofs != ofs)
                        return "packed piece layout";
                    ofs += pc.count;
                }
                if (ofs != W.total) return "packed total";
                if (W.nwt == 0 || W.nwt > (uint32_t)kMaxPieces || (uint64_t)W.wt0 + W.nwt > p.wtargets.size()) return "packed targets";
                uint32_t outs = 0;
                for (uint32_t k = 0; k < W.nwt; k++) {
                    const DWTarget& wt = p.wtargets[W.wt0 + k];
                    if (wt.target >= p.targets.size() || wt.piece >= W.npiece || wt.out0 != outs) return "packed target record";
                    const DTarget& tg = p.targets[wt.target];
                    if (tg.clique != p.pieces[W.piece0 + wt.piece].clique || tg.part0 >= 0) return "packed target clique";
                    outs += tg.G * tg.nPL;
                }
                if (outs != W.nout) return "packed outputs";
                continue;
            }
            if (W.target >= p.targets.size()) return "work target";
            const DTarget& tg = p.targets[W.target];
            if (tg.clique >= nc) return "target clique";
            const DClique& d = p.cliques[tg.clique];
            if (W.ng == 0 || W.nk == 0 || (uint64_t)W.g0 + W.ng > tg.G || (uint64_t)W.k0 + W.nk > tg.NQ) return "work range";
            if ((uint64_t)W.ng * W.nk * d.L > (uint64_t)kTileMax) return "work tile";
            for (uint32_t x : {0u, W.nk - 1, W.nk, W.ng * W.nk - 1})
                if (mdiv_host(x, W.nkmul, W.nksh) != x / W.nk) return "work magic";
            if ((uint64_t)tg.G * tg.NQ * d.L != d.size || (uint64_t)tg.nPL * tg.nQL != d.L) return "target factorisation";
            if (tg.part0 >= 0 && (W.ng != 1 || W.chunk >= tg.nchunk)) return "work partial";
            if (tg.part0 < 0 && (W.k0 != 0 || W.nk != tg.NQ)) return "work rows";
        }
    }
    for (const DTarget& tg : p.targets) {
        if (tg.clique >= nc) return "target clique";
        const DClique& d = p.cliques[tg.clique];
        if ((uint64_t)tg.rg + tg.G > p.maps.size() || (uint64_t)tg.tb + tg.G > p.maps.size() ||
            (uint64_t)tg.rq + tg.NQ > p.maps.size() || (uint64_t)tg.lp + tg.nPL > p.maps.size() ||
            (uint64_t)tg.tv + tg.nPL > p.maps.size() || (uint64_t)tg.lq + tg.nQL > p.maps.size())
            return "target tables";
        // every row and lo offset gathered lies inside the clique
        uint64_t mx_row = 0, mx_q = 0, mx_lp = 0, mx_lq = 0;
        for (uint32_t g = 0; g < tg.G; g++) mx_row = std::max<uint64_t>(mx_row, p.maps[tg.rg + g]);
        for (uint32_t k = 0; k < tg.NQ; k++) mx_q = std::max<uint64_t>(mx_q, p.maps[tg.rq + k]);
        if (mx_row + mx_q >= d.size / d.L) return "target rows";
        for (uint32_t t2 = 0; t2 < tg.nPL; t2++) mx_lp = std::max<uint64_t>(mx_lp, p.maps[tg.lp + t2]);
        for (uint32_t u = 0; u < tg.nQL; u++) mx_lq = std::max<uint64_t>(mx_lq, p.maps[tg.lq + u]);
        if (mx_lp + mx_lq >= d.L) return "target lows";
        // every output index lands inside the separator
        uint64_t mg = 0, mt = 0;
        for (uint32_t g = 0; g < tg.G; g++) mg = std::max<uint64_t>(mg, p.maps[tg.tb + g]);
        for (uint32_t t2 = 0; t2 < tg.nPL; t2++) mt = std::max<uint64_t>(mt, p.maps[tg.tv + t2]);
        const uint64_t sz = (uint64_t)tg.G * tg.nPL;
        if (mg + mt >= sz) return "target output range";
        {
            const uint32_t span = tg.NQ * tg.nQL;  // largest j the gather divides by nQL
            for (uint32_t x : {0u, tg.nQL - 1, tg.nQL, span - 1})
                if (mdiv_host(x, tg.qlmul, tg.qlsh) != x / tg.nQL) return "target nQL magic";
        }
        if ((uint64_t)tg.sep + sz > p.sep_stride) return "target separator offset";
        if (tg.part0 >= 0 && (uint64_t)tg.part0 + sz * tg.nchunk > p.n_parts) return "target partials";
    }
    // finaliser blocks: each large fin of a layer covered by its blocks in order
    for (const std::vector<Layer>* sweep : {&p.collect, &p.distribute})
        for (const Layer& ly : *sweep) {
            if (ly.nbig > ly.nfin || (uint64_t)ly.fb0 + ly.nfb > p.finblks.size()) return "layer fin blocks";
            if ((uint64_t)ly.nbig + ly.nteam > ly.nfin) return "layer fin teams";
            uint32_t b = ly.fb0;
            for (uint32_t f = ly.fin0; f < ly.fin0 + ly.nfin; f++) {
                const DSepFin& F = p.fins[f];
                if ((f < ly.fin0 + ly.nbig) != is_big(p, F)) return "large fin partition";
                if (f >= ly.fin0 + ly.nbig) {
                    // interleaved collect finalisers hold a whole small separator in registers
                    if (p.interleaved && sweep == &p.collect && F.size > kBigSeparatorInterleaved)
                        return "small collect fin size";
                    continue;
                }
                uint32_t mw = 0;
                for (uint32_t k = 0; k < F.nmv; k++) mw += p.margvars[F.mv0 + k].card;
                uint32_t end = 0;
                const uint32_t blk0 = b;
                for (; b < ly.fb0 + ly.nfb && p.finblks[b].fin == f; b++) {
                    const DFinBlk& B = p.finblks[b];
                    if (B.id != b || B.blk0 != blk0 || B.begin != end || B.count == 0 || B.count > p.fin_block ||
                        B.count > kFinBlock)
                        return "fin block layout";
                    if (B.mw != mw || (uint64_t)B.mbase + (uint64_t)B.nblk * mw > p.n_bmarg) return "fin block scratch";
                    if (B.mx != p.finblks[blk0].mx || B.mx >= p.n_bigfin) return "fin block maximum slot";
                    end += B.count;
                }
                if (end != F.size || b - blk0 != p.finblks[blk0].nblk) return "fin block cover";
            }
            if (b != ly.fb0 + ly.nfb) return "fin block count";
        }
    for (const DSepFin& F : p.fins) {
        if ((uint64_t)F.sep + F.size > p.sep_stride) return "fin range";
        if (F.nchunk && (uint64_t)F.part0 + (uint64_t)F.size * F.nchunk > p.n_parts) return "fin partials";
        if (F.edge >= t.ne || F.edge < -2 || (F.edge == -1 && F.size != 1)) return "fin edge";
        if ((uint64_t)F.mv0 + F.nmv > p.margvars.size()) return "fin posterior vars";
        for (uint32_t k = 0; k < F.nmv; k++) {
            const DMargVar& m = p.margvars[F.mv0 + k];
            if ((uint64_t)m.out + m.card > p.marg_total || m.card == 0 || m.stride == 0) return "posterior var range";
            if ((uint64_t)m.stride * m.card > F.size || F.size % ((uint64_t)m.stride * m.card)) return "posterior var stride";
            for (uint32_t x : {0u, m.stride - 1, m.stride, F.size / m.card - 1, F.size - 1})
                if (mdiv_host(x, m.smul, m.ssh) != x / m.stride) return "posterior var magic";
            for (uint32_t x : {0u, m.card - 1, m.card, F.size / m.stride - 1})
                if (mdiv_host(x, m.cmul, m.csh) != x / m.card) return "posterior var card magic";
        }
    }
    if ((uint64_t)p.sep_stride < (uint64_t)p.sep_real) return "separator stride";
    if (p.stage == 0 || p.stage > (uint32_t)kTileMax || p.stage > p.max_stage) return "stage size";
    for (const DGroup& g : p.groups)
        if (g.total > p.stage) return "group exceeds stage";
    for (const DWork& w : p.works)
        if (work_entries(p, w) > p.stage) return "work exceeds stage";
    for (const Layer& ly : p.collect) {
        if (ly.stage == 0 || ly.stage > p.stage) return "collect layer stage";
        for (uint32_t k = ly.group0; k < ly.group0 + ly.ngroup; k++)
            if (p.groups[k].total > ly.stage) return "group exceeds its layer's stage";
    }
    for (const Layer& ly : p.distribute) {
        if (ly.stage == 0 || ly.stage > p.stage) return "distribute layer stage";
        for (uint32_t k = ly.group0; k < ly.group0 + ly.ngroup; k++)
            if (work_entries(p, p.works[k]) > ly.stage) return "work exceeds its layer's stage";
    }
    return "";
}

void build_plan(const Tree& t, int tile, uint32_t max_stage, Plan& p, bool interleaved, uint32_t fin_block) {
    p = Plan();
    p.interleaved = interleaved;
    p.fin_block = interleaved ? kFinBlockInterleaved : (fin_block ? std::min(fin_block, kFinBlock) : kFinBlock);
    p.big_separator = interleaved ? kBigSeparatorInterleaved : kBigSeparator;
    p.fin_work = interleaved ? kFinWorkInterleaved : kFinWork;
    max_stage = std::min<uint32_t>(std::max<uint32_t>(max_stage, 64), (uint32_t)kTileMax);
    p.max_stage = max_stage;
    if (tile <= 0) tile = 2048;
    tile = std::min(tile, (int)max_stage);
    p.tile = tile;
    const int nc = t.nc;

    // ---- separator arena: real edges in id order, one virtual entry per
    // root (a forest of several networks has several), then one-variable
    // virtual separators for private variables
    p.sep_off.resize((size_t)t.ne);
    uint64_t so = 0;
    for (int e = 0; e < t.ne; e++) {
        p.sep_off[(size_t)e] = (uint32_t)so;
        so += t.e_size[(size_t)e];
    }
    p.sep_total = (uint32_t)so;
    std::vector<uint32_t> root_sep((size_t)nc, 0);
    p.n_roots = 0;
    for (int c = 0; c < nc; c++)
        if (t.pedge[(size_t)c] < 0) root_sep[(size_t)c] = p.sep_total + p.n_roots++;
    if (p.n_roots == 0) throw std::runtime_error("tree without a root");
    so += p.n_roots;
    p.sep_real = (uint32_t)so;

    // posterior source: smallest real separator containing the variable
    // (lowest edge id on ties); a variable in no separator lies in exactly
    // one clique and gets a virtual one-variable separator there
    p.post_sep.assign((size_t)t.n, -1);
    std::vector<uint32_t> vsep_off((size_t)t.n, 0);
    for (int e = 0; e < t.ne; e++)
        for (int v : t.e_sep[(size_t)e]) {
            int& s = p.post_sep[(size_t)v];
            if (s < 0 || t.e_size[(size_t)e] < t.e_size[(size_t)s]) s = e;
        }
    for (int v = 0; v < t.n; v++)
        if (p.post_sep[(size_t)v] < 0) {
            vsep_off[(size_t)v] = (uint32_t)so;
            so += (uint64_t)t.card[(size_t)v];
        }
    if (so > 0x7fffffffull) throw std::runtime_error("separators too large");
    p.sep_stride = (uint32_t)((so + 63) / 64 * 64);

    // marginal offsets
    std::vector<uint32_t> marg_off((size_t)t.n);
    uint32_t mo = 0;
    for (int v = 0; v < t.n; v++) {
        marg_off[(size_t)v] = mo;
        p.homevars.push_back({mo, (uint32_t)t.card[(size_t)v]});
        mo += (uint32_t)t.card[(size_t)v];
    }
    p.marg_total = mo;

    // ---- per-clique records, tables in id order
    p.cliques.resize((size_t)nc);
    p.kappa.assign((size_t)nc, 0);
    std::vector<int> splitq((size_t)nc);
    uint64_t off = 0;
    for (int c = 0; c < nc; c++) {
        const auto& lay = t.vars[(size_t)c];
        const int m = (int)lay.size();
        const uint64_t size = t.size[(size_t)c];
        std::vector<int> card_at((size_t)m);
        for (int k = 0; k < m; k++) card_at[(size_t)k] = t.card[(size_t)lay[(size_t)k]];
        DClique& d = p.cliques[(size_t)c];
        d = DClique{};
        d.off = off;
        d.size = (uint32_t)size;
        off += size;
        // split point: smallest suffix product >= 64, or the whole clique
        int q = m;
        uint64_t L = 1;
        // (at most max_stage entries, so that one row fits the LDS stage)
        while (q > 0 && L < 64 && L * (uint64_t)card_at[(size_t)q - 1] <= max_stage) {
            q--;
            L *= (uint64_t)card_at[(size_t)q];
        }
        if (L > (uint64_t)max_stage) throw std::runtime_error("a variable's cardinality is too large for the tile");
        splitq[(size_t)c] = q;
        const uint64_t rows = size / L;
        d.L = (uint32_t)L;
        magic_u32(d.L, d.Lmul, d.Lsh);
        std::vector<int> hi_pos, lo_pos;
        for (int k = 0; k < q; k++) hi_pos.push_back(k);
        for (int k = q; k < m; k++) lo_pos.push_back(k);
        // digit bit positions, layout order from the lowest bits
        std::vector<uint32_t> shift((size_t)m);
        uint32_t sh = 0;
        for (int k = 0; k < m; k++) {
            shift[(size_t)k] = sh;
            sh += bits_for(card_at[(size_t)k]);
        }
        if (sh > 64) throw std::runtime_error("clique digits exceed 64 bits");
        p.dig_shift0.push_back((uint32_t)p.dig_shift.size());
        for (int k = 0; k < m; k++) p.dig_shift.push_back(shift[(size_t)k]);
        {
            // packed digits: enumerate with weights 2^shift (exact in uint64)
            auto packed = [&](const std::vector<int>& pos) {
                const uint32_t start = (uint32_t)p.digits.size();
                uint64_t count = 1;
                for (int k : pos) count *= (uint64_t)card_at[(size_t)k];
                std::vector<int> dg(pos.size(), 0);
                for (uint64_t x = 0; x < count; x++) {
                    uint64_t v = 0;
                    for (size_t a = 0; a < pos.size(); a++) v |= (uint64_t)dg[a] << shift[(size_t)pos[a]];
                    p.digits.push_back(v);
                    for (size_t a = pos.size(); a-- > 0;) {
                        if (++dg[a] < card_at[(size_t)pos[a]]) break;
                        dg[a] = 0;
                    }
                }
                return start;
            };
            d.hdig = packed(hi_pos);
            d.ldig = packed(lo_pos);
        }
        (void)rows;
        // parent map (prefix of the layout) and segment length
        if (t.pedge[(size_t)c] < 0) {
            d.pedge = -1;
            d.psep = root_sep[(size_t)c];
            d.seg = (uint32_t)size;
            d.pmh = d.pml = 0;
        } else {
            const int e = t.pedge[(size_t)c];
            const int ns = (int)t.e_sep[(size_t)e].size();
            std::vector<uint64_t> w((size_t)m, 0);
            uint64_t s = 1;
            for (int k = ns - 1; k >= 0; k--) {
                w[(size_t)k] = s;
                s *= (uint64_t)card_at[(size_t)k];
            }
            d.pedge = e;
            d.psep = p.sep_off[(size_t)e];
            d.seg = (uint32_t)(size / t.e_size[(size_t)e]);
            d.pmh = enumerate(hi_pos, card_at, w, p.maps);
            d.pml = enumerate(lo_pos, card_at, w, p.maps);
        }
        magic_u32(d.seg, d.segmul, d.segsh);
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
            r.mh = enumerate(hi_pos, card_at, w, p.maps);
            r.ml = enumerate(lo_pos, card_at, w, p.maps);
            p.children.push_back(r);
        }
        d.home0 = 0;
        d.nhome = 0;
        // scaled prior: max scaled into [0.5, 1) by an exact power of two
        double mx = 0.0;
        for (double x : t.prior[(size_t)c]) mx = std::max(mx, x);
        int kap = 0;
        if (mx > 0.0) std::frexp(mx, &kap);
        p.kappa[(size_t)c] = kap;
        p.kappa_total += kap;
    }
    p.T = off;
    // working tables: per-slot layout, the prior's arena layout; interleaved,
    // only the cliques with more than kRebuildKidsInterleaved children store
    // one (the distribute rebuilds the others), packed in clique order
    // working tables: which cliques store one is settled with the distribute
    // items below (assign_psi)
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
                        // per-slot partials are chunk-major (chunk k of entry s at
                        // k * size + s), slot-interleaved ones entry-major
                        const uint32_t at = interleaved ? parts + s * nchunk + k : parts + k * f.size + s;
                        pk.add_part((uint32_t)c, s * seg + b, e - b, (int32_t)at);
                    }
                parts += f.size * nchunk;
            }
            fins.push_back(f);
        }
        ly.ngroup = (uint32_t)p.groups.size() - ly.group0;
        finish_layer(p, ly, fins);
    }

    std::vector<char> rebuilt((size_t)nc, 0);
    // ---- distribute layers (depth): marginalise each clique onto each child
    // separator and onto the virtual separator of each private variable
    p.distribute.assign((size_t)D + 1, Layer());
    // interleaved: a distribute work item is walked by one wave, and fewer,
    // longer items mean fewer partial sums for the finalisers to add
    const uint32_t dtile_base = (uint32_t)std::max(interleaved ? 4 * tile : tile, 64);
    for (int dd = 0; dd <= D; dd++) {
        Layer& ly = p.distribute[(size_t)dd];
        ly.group0 = (uint32_t)p.works.size();
        int32_t open_w = -1;  // open packed workgroup of this layer
        std::vector<DSepFin> fins;
        for (int c = 0; c < nc; c++) {
            if (t.depth[(size_t)c] != dd) continue;
            const auto& lay = t.vars[(size_t)c];
            const int m = (int)lay.size();
            const int q = splitq[(size_t)c];
            const DClique& d = p.cliques[(size_t)c];
            std::vector<int> card_at((size_t)m);
            for (int k = 0; k < m; k++) card_at[(size_t)k] = t.card[(size_t)lay[(size_t)k]];
            // strides of the positions among the row digits and the lo digits
            std::vector<uint64_t> rstride((size_t)m, 0), lstride((size_t)m, 0);
            uint64_t s = 1;
            for (int k = q - 1; k >= 0; k--) {
                rstride[(size_t)k] = s;
                s *= (uint64_t)card_at[(size_t)k];
            }
            s = 1;
            for (int k = m - 1; k >= q; k--) {
                lstride[(size_t)k] = s;
                s *= (uint64_t)card_at[(size_t)k];
            }
            // one target per child separator and per private variable
            struct Tgt {
                std::vector<int> vars;  // target variables, ascending = its layout
                uint32_t sep;
                int edge;               // >= 0 real, -2 virtual
            };
            std::vector<Tgt> tgts;
            for (int ch : t.children[(size_t)c]) {
                const int e = t.pedge[(size_t)ch];
                tgts.push_back({t.e_sep[(size_t)e], p.sep_off[(size_t)e], e});
            }
            for (int v : lay)
                if (p.post_sep[(size_t)v] < 0) tgts.push_back({{v}, vsep_off[(size_t)v], -2});
            const uint32_t dtile_c = std::min<uint32_t>(max_stage, std::max(dtile_base, d.L));
            const bool packed = !interleaved && d.size <= dtile_c && tgts.size() <= (size_t)kMaxPieces;
            rebuilt[(size_t)c] = interleaved && d.nchild <= kRebuildKidsInterleaved;
            if (packed) {
                if (open_w >= 0) {
                    const DWork& W = p.works[(size_t)open_w];
                    if (W.total + d.size > dtile_c || W.npiece >= (uint32_t)kMaxPieces ||
                        W.nwt + tgts.size() > (size_t)kMaxPieces)
                        open_w = -1;
                }
                if (open_w < 0) {
                    DWork W{};
                    W.piece0 = (uint32_t)p.pieces.size();
                    W.wt0 = (uint32_t)p.wtargets.size();
                    p.works.push_back(W);
                    open_w = (int32_t)p.works.size() - 1;
                }
                DWork& W = p.works[(size_t)open_w];
                p.pieces.push_back({(uint32_t)c, 0u, d.size, W.total});
                W.npiece++;
                W.total += d.size;
            }
            for (const Tgt& tg0 : tgts) {
                // target strides (ascending variable order, last fastest)
                std::vector<uint64_t> tstride((size_t)m, 0);
                uint64_t ts = 1;
                std::vector<char> keep((size_t)m, 0);
                for (size_t a = tg0.vars.size(); a-- > 0;) {
                    for (int k = 0; k < m; k++)
                        if (lay[(size_t)k] == tg0.vars[a]) {
                            tstride[(size_t)k] = ts;
                            keep[(size_t)k] = 1;
                        }
                    ts *= (uint64_t)t.card[(size_t)tg0.vars[a]];
                }
                const uint64_t tsize = ts;
                std::vector<int> Phi, Qhi, Plo, Qlo;
                for (int k = 0; k < m; k++) {
                    if (k < q) (keep[(size_t)k] ? Phi : Qhi).push_back(k);
                    else (keep[(size_t)k] ? Plo : Qlo).push_back(k);
                }
                DTarget T{};
                T.clique = (uint32_t)c;
                auto prod = [&](const std::vector<int>& ps) {
                    uint64_t x = 1;
                    for (int k : ps) x *= (uint64_t)card_at[(size_t)k];
                    return (uint32_t)x;
                };
                T.G = prod(Phi);
                T.NQ = prod(Qhi);
                T.nPL = prod(Plo);
                T.nQL = prod(Qlo);
                T.rg = enumerate(Phi, card_at, rstride, p.maps);
                T.tb = enumerate(Phi, card_at, tstride, p.maps);
                T.rq = enumerate(Qhi, card_at, rstride, p.maps);
                T.lp = enumerate(Plo, card_at, lstride, p.maps);
                T.tv = enumerate(Plo, card_at, tstride, p.maps);
                T.lq = enumerate(Qlo, card_at, lstride, p.maps);
                T.sep = tg0.sep;
                T.part0 = -1;
                T.nchunk = 0;
                magic_u32(T.nQL, T.qlmul, T.qlsh);
                const uint32_t ti = (uint32_t)p.targets.size();
                const uint32_t dtile = dtile_c;
                const uint64_t group_entries = (uint64_t)T.NQ * d.L;
                if (packed) {
                    DWork& W = p.works[(size_t)open_w];
                    p.wtargets.push_back({ti, W.npiece - 1, W.nout, 0u});
                    W.nwt++;
                    W.nout += T.G * T.nPL;
                } else if (group_entries <= dtile) {
                    const uint32_t per = std::max<uint32_t>(1, (uint32_t)(dtile / group_entries));
                    for (uint32_t g0 = 0; g0 < T.G; g0 += per) {
                        DWork W{};
                        W.target = ti;
                        W.g0 = g0;
                        W.ng = std::min(per, T.G - g0);
                        W.k0 = 0;
                        W.nk = T.NQ;
                        magic_u32(W.nk, W.nkmul, W.nksh);
                        W.chunk = 0;
                        p.works.push_back(W);
                    }
                } else {
                    const uint32_t nk = std::max<uint32_t>(1, dtile / d.L);
                    T.nchunk = (T.NQ + nk - 1) / nk;
                    T.part0 = (int32_t)parts;
                    parts += (uint32_t)(tsize * T.nchunk);
                    for (uint32_t g = 0; g < T.G; g++)
                        for (uint32_t ck = 0; ck < T.nchunk; ck++) {
                            DWork W{};
                            W.target = ti;
                            W.g0 = g;
                            W.ng = 1;
                            W.k0 = ck * nk;
                            W.nk = std::min(nk, T.NQ - W.k0);
                            magic_u32(W.nk, W.nkmul, W.nksh);
                            W.chunk = ck;
                            p.works.push_back(W);
                        }
                }
                p.targets.push_back(T);
                // finalise record with the posterior variables it carries
                DSepFin f{};
                f.sep = tg0.sep;
                f.size = (uint32_t)tsize;
                f.edge = tg0.edge;
                f.nchunk = T.part0 >= 0 ? T.nchunk : 0;
                f.part0 = T.part0 >= 0 ? (uint32_t)T.part0 : 0;
                f.mv0 = (uint32_t)p.margvars.size();
                if (tg0.edge >= 0) {
                    uint64_t st = 1;
                    std::vector<uint64_t> vs(tg0.vars.size());
                    for (size_t a = tg0.vars.size(); a-- > 0;) {
                        vs[a] = st;
                        st *= (uint64_t)t.card[(size_t)tg0.vars[a]];
                    }
                    for (size_t a = 0; a < tg0.vars.size(); a++) {
                        const int v = tg0.vars[a];
                        if (p.post_sep[(size_t)v] != tg0.edge) continue;
                        DMargVar mv{};
                        mv.out = marg_off[(size_t)v];
                        mv.stride = (uint32_t)vs[a];
                        mv.card = (uint32_t)t.card[(size_t)v];
                        magic_u32(mv.stride, mv.smul, mv.ssh);
                        magic_u32(mv.card, mv.cmul, mv.csh);
                        p.margvars.push_back(mv);
                    }
                } else {
                    const int v = tg0.vars[0];
                    DMargVar mv{};
                    mv.out = marg_off[(size_t)v];
                    mv.stride = 1u;
                    mv.card = (uint32_t)t.card[(size_t)v];
                    magic_u32(1u, mv.smul, mv.ssh);
                    magic_u32(mv.card, mv.cmul, mv.csh);
                    p.margvars.push_back(mv);
                }
                f.nmv = (uint32_t)p.margvars.size() - f.mv0;
                fins.push_back(f);
            }
        }
        ly.ngroup = (uint32_t)p.works.size() - ly.group0;
        finish_layer(p, ly, fins);
    }
    p.n_parts = parts;
    // the cliques that store a working table, packed in clique order
    uint64_t po = 0;
    for (int c = 0; c < nc; c++) {
        DClique& d = p.cliques[(size_t)c];
        if (rebuilt[(size_t)c]) {
            d.psi = kNoPsi;
            continue;
        }
        if (po + d.size >= (uint64_t)kNoPsi) throw std::runtime_error("working-table arena");
        d.psi = (uint32_t)po;
        po += d.size;
    }
    p.psi_total = po;
    p.stage = (uint32_t)tile;
    for (const DGroup& g : p.groups) p.stage = std::max(p.stage, g.total);
    for (const DWork& w : p.works) p.stage = std::max(p.stage, work_entries(p, w));
    // a layer stages only what its largest item needs, so layers of small
    // cliques carry more slots per workgroup in less LDS
    for (Layer& ly : p.collect) {
        ly.stage = 64;
        for (uint32_t k = ly.group0; k < ly.group0 + ly.ngroup; k++) ly.stage = std::max(ly.stage, p.groups[k].total);
        ly.stage = std::min(ly.stage, p.stage);
    }
    for (Layer& ly : p.distribute) {
        ly.stage = 64;
        for (uint32_t k = ly.group0; k < ly.group0 + ly.ngroup; k++)
            ly.stage = std::max(ly.stage, work_entries(p, p.works[k]));
        ly.stage = std::min(ly.stage, p.stage);
    }
}

}  // namespace fbn
