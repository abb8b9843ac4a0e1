// Internal types of the junction-tree library: the host-side network and
// tree, and the plain-old-data plan records read by the HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace fbn {

// ---------------------------------------------------------------- host model

// A discrete Bayesian network: a DAG with one CPT per variable, parents in
// listed order and the variable itself fastest (paper, Section 1).
struct Net {
    int n = 0;
    std::vector<int> card;
    std::vector<std::vector<int>> parents;
    std::vector<std::vector<double>> cpt;  // empty vectors: structure only
};

// The compiled junction tree (paper, Section 1: cliques and separators with
// potential tables; Section 2: layers and root selection).
struct Tree {
    int n = 0;
    std::vector<int> card;
    std::vector<int> elim_order;
    int nc = 0;                                  // cliques
    std::vector<std::vector<int>> vars;          // table layout order
    std::vector<uint64_t> size;                  // entries per clique
    int root = 0;                                // first root
    std::vector<int> roots;                      // one per network of a forest
    std::vector<int> parent, pedge, height, depth;
    std::vector<std::vector<int>> children;      // ascending id
    int ne = 0;                                  // edges, by ascending child id
    std::vector<int> e_parent, e_child;
    std::vector<std::vector<int>> e_sep;         // in the order they take in the parent's layout
    std::vector<uint64_t> e_size;
    std::vector<int> cpt_home, var_home;
    std::vector<std::vector<double>> prior;      // per clique, layout order, unscaled
};

// Parse a network in the Bayesian Interchange Format (bif.cpp): variables in
// declaration order, CPTs with the listed parents and the variable fastest.
// Returns "" or the error text; names and states receive the declared names.
std::string parse_bif(const char* text, size_t len, Net& net, std::vector<std::string>& names,
                      std::vector<std::vector<std::string>>& states);

// Returns an empty string on success, else the error text.  code receives
// an fbn_status value.
std::string compile_tree(const Net& net, uint64_t max_entries, Tree& out, int& code);

// Several independent networks as one forest: variables, cliques and edges
// of network k follow those of networks 0..k-1 (ids offset), each network
// keeps its own tree and root.
Tree merge_forest(const std::vector<Tree>& parts);

// ---------------------------------------------------------------- plan records

// One clique as the kernels see it.  Entry i of the table splits as
// i = hi * L + lo, where L is the product of the trailing (fastest)
// variables' cardinalities; every separator index is additive in the
// digits, so each index map is stored factored as H[hi] + L[lo].
struct DClique {
    uint64_t off;        // first entry in the prior / working-table arena
    uint32_t size;       // entries (< 2^31)
    uint32_t L;          // low extent
    uint32_t Lmul, Lsh;  // hi = ((umulhi(i, Lmul) + i) >> Lsh) == i / L
    uint32_t hdig, ldig; // offsets of the packed-digit tables (uint64 pool)
    int32_t pedge;       // edge to the parent, -1 at the root
    uint32_t psep;       // separator-arena offset of the parent separator (root: virtual entry)
    uint32_t pmh, pml;   // parent-map tables (uint32 pool): entry -> parent separator index
    uint32_t seg;        // size / |parent separator| (root: size)
    uint32_t segmul, segsh;  // division by seg: entry i lies in parent-separator entry i / seg
    uint32_t child0;     // first DChild record
    uint32_t home0;      // first DHome record
    uint16_t nchild, nhome;
    uint32_t psi;        // offset in the compact working-table arena, or kNoPsi: psi is rebuilt in the distribute
};

// A child edge seen from its parent clique: where its separator lives and
// the factored index map from parent entries to separator entries.
struct DChild {
    uint32_t sep;        // separator-arena offset
    uint32_t mh, ml;     // map tables (uint32 pool)
    uint32_t size;       // separator entries
};

// A variable whose posterior is read from this clique.
struct DHome {
    uint32_t out;        // offset of its first state in the per-slot marginal arrays
    uint32_t shift;      // bit position of its digit in the packed digits
    uint32_t mask;       // (1 << bits) - 1
    uint32_t card;
};

// A contiguous run of one clique's entries handled inside a workgroup.
struct DPiece {
    uint32_t clique;
    uint32_t begin;      // first entry within the clique
    uint32_t count;
    uint32_t gofs;       // offset of the run inside the workgroup's tile
};

// The work of one workgroup in one layer: a packed list of runs.  In a
// collect layer, a "full" group holds whole parent-separator segments; a
// "part" group holds one chunk of a single segment too long for one tile,
// and writes its partial sum to the partial-sum arena.
struct DGroup {
    uint32_t piece0;
    uint32_t npiece;
    uint32_t total;      // entries in the tile
    int32_t part;        // partial-sum index, or -1 for a full group
};

// Separator finalisation after a layer: one record per separator (the
// root's virtual one-entry separator included, with edge = -1; in the
// distribute sweep also one-variable virtual separators, edge = -2, which
// carry the posterior of a variable that lies in no real separator).
struct DSepFin {
    uint32_t sep;        // separator-arena offset
    uint32_t size;
    uint32_t part0;      // first partial (entry m, chunk c at part0 + m*nchunk + c)
    uint32_t nchunk;     // 0: the layer kernel wrote whole sums
    int32_t edge;        // edge id, -1 root, -2 virtual
    uint32_t mv0, nmv;   // posterior variables read from this separator
    uint32_t pad;
};

// One block of a large separator's finalisation: entries [begin, begin+count)
// of fin `fin`.  The fin's blocks are [blk0, blk0+nblk) in Plan::finblks (so
// this block's maximum lands at slot scratch index id), and their partial
// posterior sums sit at mbase + j*mw (block j), mw = sum of the posterior
// variables' cardinalities.
struct DFinBlk {
    uint32_t fin;
    uint32_t begin, count;
    uint32_t id, blk0, nblk;
    uint32_t mbase, mw;
    uint32_t mx;  // the separator's index among the large ones (its running maximum, interleaved layout)
};

// A variable whose posterior is the marginal of a calibrated separator.
struct DMargVar {
    uint32_t out;        // offset of its first state in the per-slot marginal arrays
    uint32_t stride;     // stride of the variable in the separator layout
    uint32_t card;
    uint32_t smul, ssh;  // division by stride
    uint32_t cmul, csh;  // division by card
    uint32_t pad;
};

// Distribute-sweep marginalisation of clique C onto a target separator S
// (S's variables kept, the rest summed).  With C's entries as rows of L
// (i = row * L + lo):
//   target groups g < G enumerate the digits of S's variables among the row
//   variables; the rows of group g are RG[g] + RQ[k], k < NQ;
//   within a row, output t < nPL gathers the lo offsets LP[t] + LQ[u], u < nQL;
//   output (g, t) is separator entry TB[g] + TV[t].
struct DTarget {
    uint32_t clique;
    uint32_t G, NQ, nPL, nQL;
    uint32_t rg, rq, tb, lp, lq, tv;  // uint32 pool offsets
    uint32_t sep;        // separator-arena offset of S
    int32_t part0;       // partial sums of S when a group's rows span work items, else -1
    uint32_t nchunk;
    uint32_t qlmul, qlsh;  // division by nQL
};

// One workgroup of the distribute gather, in one of two forms.
//   npiece == 0: groups [g0, g0+ng) x rows [k0, k0+nk) of one target, at
//     most one tile of entries (large cliques).
//   npiece  > 0: whole small cliques (runs in Plan::pieces) staged once in
//     LDS, and every target of each of them (records in Plan::wtargets).
struct DWork {
    uint32_t target;
    uint32_t g0, ng, k0, nk;
    uint32_t nkmul, nksh;  // division by nk
    uint32_t chunk;        // k0 / nk
    uint32_t piece0, npiece, total;
    uint32_t wt0, nwt, nout;
};

// A target of a packed distribute workgroup: its clique is run `piece` of
// the workgroup, and its outputs are numbered from out0 within the group.
struct DWTarget {
    uint32_t target, piece, out0, pad;
};

// Per-slot evidence for one clique: entry i survives the reduction when
// ((digits(i) ^ want) & mask) == 0.
struct DEvidence {
    uint64_t want, mask;
};

struct DHomeVar {        // for the posterior finaliser: one per variable
    uint32_t out, card;
};

constexpr int kBlock = 256;       // threads per workgroup
constexpr int kTileMax = 4096;    // entries per workgroup tile
constexpr int kMaxPieces = 32;    // runs (and packed targets) per workgroup
constexpr uint32_t kFinBlock = 4096;  // separator entries per finaliser block at most
constexpr uint32_t kFinBlockInterleaved = 16;  // the same with slot-interleaved tables
constexpr uint32_t kBigSeparatorInterleaved = 16;
// Slot-interleaved: a clique with at most this many children stores no
// working table (DClique::psi = kNoPsi); the distribute rebuilds it from the
// prior, the evidence and the child messages.  The per-slot layout stores
// every working table: there a rebuild gathers each slot's messages apart,
// which measured slower than reading the stored table.
constexpr uint32_t kRebuildKidsInterleaved = 6;
constexpr uint32_t kNoPsi = 0xffffffffu;  // slot-interleaved: larger separators are split into blocks

}  // namespace fbn
