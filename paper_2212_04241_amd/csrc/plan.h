// Device plan: everything the layer kernels read, laid out on the host and
// uploaded once per network.
#pragma once

#include "fbn_internal.h"

namespace fbn {

struct Layer {
    uint32_t group0 = 0, ngroup = 0;  // collect: into Plan::groups; distribute: into Plan::works
    uint32_t fin0 = 0, nfin = 0;      // into Plan::fins (separators finalised after it)
    uint32_t nbig = 0;                // the first nbig fins are large: split over Plan::finblks
    uint32_t fb0 = 0, nfb = 0;        // their blocks, into Plan::finblks
    uint32_t nteam = 0;               // the next nteam fins get a workgroup each, the rest a wave
    uint32_t stage = 0;               // per-slot layout: LDS entries per slot of its largest group / work item
};

constexpr uint32_t kBigSeparator = 1024;  // entries above which a separator is split into blocks
constexpr uint64_t kFinWork = 16384;  // partial sums one finaliser block adds at most (entries x chunks)
constexpr uint64_t kFinWorkInterleaved = 1024;  // the same when one lane adds them all
constexpr uint32_t kTeamSeparator = 256;  // separators above this get a workgroup rather than a wave

struct Plan {
    int tile = 2048;
    bool interleaved = false;         // slot-interleaved tables: one wave per work item, lanes = slots
    uint32_t fin_block = kFinBlock;   // separator entries per finaliser block
    uint32_t big_separator = kBigSeparator;  // larger real separators are finalised in blocks
    uint64_t fin_work = kFinWork;     // partial sums per finaliser block at most
    uint32_t stage = 0;               // LDS entries per slot: largest collect tile or distribute block
    uint32_t max_stage = 0;           // bound on stage
    uint64_t T = 0;                   // prior / working-table entries
    uint64_t psi_total = 0;           // working-table entries per slot (interleaved: storing cliques only)
    uint32_t sep_total = 0;           // separator entries over all edges
    uint32_t n_roots = 0;             // trees of the forest; virtual entries follow sep_total
    uint32_t sep_stride = 0;          // per slot: separators, root entries, virtual separators, rounded
    uint32_t n_parts = 0;             // partial sums per slot
    uint32_t marg_total = 0;          // sum of cardinalities
    int kappa_total = 0;              // sum of clique prior exponents
    std::vector<DClique> cliques;
    std::vector<DChild> children;
    std::vector<DHome> homes;
    std::vector<DHomeVar> homevars;   // per variable
    std::vector<DPiece> pieces;
    std::vector<DGroup> groups;
    std::vector<DSepFin> fins;
    std::vector<DFinBlk> finblks;     // blocks of the large separators, layer by layer
    uint32_t n_bigfin = 0;            // large separators (finalised in blocks), both sweeps
    uint32_t n_bmarg = 0;             // per slot: partial posterior sums of the blocks
    std::vector<DTarget> targets;     // distribute marginalisations
    std::vector<DWork> works;         // distribute workgroups
    std::vector<DWTarget> wtargets;   // targets of packed distribute workgroups
    std::vector<DMargVar> margvars;   // posterior variables per finalised separator
    std::vector<int> post_sep;        // per variable: edge whose separator gives its posterior, -1 virtual
    uint32_t sep_real = 0;            // entries of real separators + the root's virtual entry
    std::vector<Layer> collect;       // by height 0..H
    std::vector<Layer> distribute;    // by depth 0..D
    std::vector<uint64_t> digits;     // packed-digit tables
    std::vector<uint32_t> maps;       // factored index maps
    std::vector<double> prior;        // scaled by 2^-kappa_c per clique, arena order
    std::vector<int> kappa;           // per clique
    std::vector<uint32_t> sep_off;    // per edge
    std::vector<uint32_t> dig_shift;  // per clique, per layout position: bit shift
    std::vector<uint32_t> dig_shift0; // start of each clique's entries in dig_shift
};

// max_stage: entries one workgroup can stage in LDS for one slot (bounds
// every tile, every distribute block and the row length L).  interleaved:
// the work items are sized for one wave each (tile entries), distribute
// work is never packed, and large separators split into blocks of
// kFinBlockInterleaved entries.
void build_plan(const Tree& t, int tile, uint32_t max_stage, Plan& p, bool interleaved = false,
                uint32_t fin_block = 0);

// Checks, on the host, every bound the kernels rely on: tile and run sizes,
// run alignment to separator segments, table offsets and every value of the
// factored maps and packed digits.  Returns "" or the first violation.
std::string check_plan(const Tree& t, const Plan& p);

// Magic numbers for unsigned division by d of numerators below 2^31
// (Granlund and Montgomery, 1994): q = (umulhi(n, mul) + n) >> sh.
void magic_u32(uint32_t d, uint32_t& mul, uint32_t& sh);

}  // namespace fbn
