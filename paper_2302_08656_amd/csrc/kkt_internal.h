// Internal declarations shared by the host symbolic phase, the schedule builder and the
// HIP runtime of the KKT refactorization library.  Not part of the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/kkt.h"

namespace kkt {

// Canonical symbolic factorization (analysis stage).  Permuted index space: row k of
// P A Q is row P[k] of A, column k is column Q[k].
struct Symbolic {
    int32_t n = 0;
    int64_t nnz_a = 0;
    std::vector<int64_t> a_rowptr;
    std::vector<int32_t> a_colind;
    std::vector<int32_t> P, Q, pinv, qinv;
    std::vector<int64_t> colptr;   // combined L+U, CSC, rows ascending per column
    std::vector<int32_t> rowidx;
    std::vector<int32_t> ulen;     // entries above the diagonal per column
    std::vector<int32_t> parent, lev_f, lev_l, lev_u, sn_start;
    std::vector<int64_t> map;      // CSR entry of A -> slot of L+U
    int32_t nsn() const { return (int32_t)sn_start.size() - 1; }
    int64_t nnz_lu() const { return colptr.empty() ? 0 : colptr.back(); }
};

// Status-returning host steps of the analysis.
int validate_pattern(int32_t n, const int64_t *rowptr, const int32_t *colind);
int exact_min_degree(int32_t n, const int64_t *rowptr, const int32_t *colind,
                     std::vector<int32_t> &order);
int pow2_scaling(int32_t n, const int64_t *rowptr, const int32_t *colind, const double *v,
                 bool scale, std::vector<double> &r, std::vector<double> &c);
int analyze_symbolic(int32_t n, const int64_t *rowptr, const int32_t *colind,
                     const double *values, const kkt_opts &o, Symbolic &s);

// Maximum width of a GPU panel (a column range of a structural supernode handled by one
// work item).  Panels never cross supernode boundaries.
constexpr int kPanelMax = 32;
// Width-1 panels of the triangular solves are packed this many to a 256-thread block.
constexpr int kSolvePack = 64;
// Refactorization items whose panel and sources all have at most kSmallW columns and
// kSmallR rows below run on 16 lanes with registers only; the others on 256 threads with
// the source panel staged in LDS.  Targets sharing one source are grouped kGroup per item.
constexpr int kSmallW = 4;
constexpr int kSmallR = 64;
// Narrow items whose panel and sources all have at most kTinyR rows below (tiny items) run
// on kTinyLanes lanes in the launches of levels without wide items.
constexpr int kTinyLanes = 4;
constexpr int kTinyR = 16;
constexpr int kGroup = 32;
constexpr int kMedW = 16;
constexpr int kMedRows = 256;
// rows of a factored panel up to which a 32-column wide item runs in a 256-thread block, and
// the wide items a level needs for its launch to use 256-thread blocks (two per compute
// unit): levels with fewer are bound by one item's latency, which 512 threads shorten
constexpr int kW256Rows = 256;
constexpr int kW256MinItems = 256;
// Solve helpers: a wide panel gets helper items kHelpAhead levels before it when one of
// its rows has at least kHelpMin early entries (columns of panels more than kHelpAhead
// levels below); each helper item sums the early entries of kHelpRows rows.
constexpr int kHelpAhead = 2;
constexpr int kHelpRows = 4;
constexpr int kHelpMin = 32;
// Solve panels of at most kPackW columns are packed whole, kSolvePack rows to an item.
constexpr int kPackW = 4;
// The row-ordered copy of the factor rides with up to kCopyLaunches of the top refactor
// levels that have at most kCopyItems items each.
constexpr int kCopyItems = 16;
constexpr int kCopyLaunches = 4;

// Tunable choices of the schedule builder (kkt_tuning); every value keeps the kernels' limits.
struct SchedParams {
    int32_t panel_max = kPanelMax;   // widest panel cut from a supernode (1..kPanelMax)
    int32_t small_rows = kSmallR;    // narrow path: panels of <= kSmallW columns and <= this many rows below
    int32_t group = kGroup;          // targets of one source grouped into one pull item (1..kGroup)
    int32_t wide256 = 1;             // levels with many wide items, all fitting 256 rows, use 256-thread blocks
    int32_t fuse_chains = 0;         // consecutive panels of a supernode factored by one item when possible
    int32_t tiny_rows = kTinyR;      // tiny items: narrow, every panel <= this many rows below (0 = none)
};

// Device schedule, built on the host once per pattern and uploaded by kkt_bind.
struct Schedule {
    SchedParams params;
    int32_t npan = 0;
    std::vector<int32_t> pan_start;     // [npan+1] first column of each panel
    std::vector<int32_t> pan_r;         // [npan] L rows below the panel (= U columns right)
    // refactorization: launch l runs items [f_lvl[l], f_lvl[l+1]); the first f_nlarge[l] of
    // them take the wide path (in its medium configuration, f_nmed[l] = f_nlarge[l], when
    // every wide item of the level has panels of at most kMedW columns and factors a panel
    // of at most kMedRows rows), the rest the 16-lane path (as extra blocks of the level's
    // wide launch, or as a launch of their own on a level without wide items).  An item owns the target
    // columns of its (source panel, target column) pairs, listed source-major, and then
    // factors its panel (f_item_panel >= 0).  The last f_ntiny[l] narrow items are tiny
    // (4-lane groups in a launch of their own level's narrow kernel).
    std::vector<int32_t> f_lvl, f_nlarge, f_nmed, f_ntiny;
    // levels whose 32-column wide items run in 256-thread blocks (every factored panel of the
    // level has at most 256 rows): 1, else 0
    std::vector<int32_t> f_w256;
    // row-ordered copy: copy_k lists CSR positions, the strictly lower entries first (launch
    // l's: copy_k[copy_lat[l] .. copy_lat[l+1])), then the others (launch l's: copy_k[
    // copy_uat[l] .. copy_uat[l+1])), grouped by the launch that finishes their column;
    // copy_src[q] = csr_src[copy_k[q]].  Launches copy_lvl on (every one with wide items) are
    // the top levels, which leave most of the GPU idle and carry copy chunks.
    int32_t copy_lvl = 0;
    std::vector<int32_t> copy_k, copy_src, copy_lat, copy_uat;
    // forward solve fused with the refactorization: the items of forward level k read only
    // columns final after refactor launch l_ready[k] (and unknowns of lower forward levels)
    std::vector<int32_t> l_ready;
    std::vector<int32_t> f_item_panel;  // (first) panel to factor after the pulls, or -1
    std::vector<int32_t> f_item_npan;   // panels factored by the item (consecutive, one supernode)
    std::vector<int32_t> f_item_pair;   // [nitems+1] range into f_pair_src / f_pair_tgt
    std::vector<int32_t> f_pair_src, f_pair_tgt;
    std::vector<int32_t> f_pair_pos;    // slot of the source's first row in the target column
    std::vector<int64_t> f_pair_rel;    // [npairs+1] range into f_rel
    std::vector<int32_t> f_rel;         // slot of each row R of the source in the target column
    // packed records read by the refactorization kernels (8 x int32 each):
    // itemrec[i] = {panel to factor or -1, first pair, end pair, panels factored, s, w, r,
    //               ldiag[s], s', w', r', ldiag[s']} (s, w, r of the first panel; s', w', r' of
    //               the first pair's source, zero for an item without pairs);
    // pair8[q] = {source panel, f_pair_pos, f_pair_rel (first index), end of q's group,
    //             s, w, r, ldiag[s]}, with s, w, r the panel's first column, width, rows below
    //             (a group: consecutive pairs of one source, at most kGroup);
    // for pairs of narrow items {ldiag[s+1], f_pair_pos, f_pair_rel, ldiag[s+2], ldiag[s+3],
    //             w, r, ldiag[s]} (slots past the width are 0)
    std::vector<int32_t> itemrec, pair8;
    std::vector<int32_t> ldiag;         // slot of the diagonal of each column
    // triangular solves: level l has items [x_lvl[l], x_lvl[l+1]), 4 x int32 each:
    // {1, lanes, s, w}: wide panel of rows s..s+w-1; {0, t0, s, w}: helper summing the
    // early columns of rows s+t0 .. s+t0+kHelpRows-1 of such a panel (kHelpAhead levels
    // before it); {-c, p0, lanes, 0}: pack of c rows of whole panels of width <= kPackW
    // whose row records are x_rows4[p0..] = {row, first external slot, end of external
    // slots, t | w << 8} with t the row's offset in its panel of width w.  `lanes` = lanes
    // per row for the external part (a power of two, 256 / lanes >= rows, at most 64).
    std::vector<int32_t> l_lvl, u_lvl;
    std::vector<int32_t> l_item4, u_item4, l_rows4, u_rows4;
    // per-row records of the CSR copy: forward {first slot, first late slot, diagonal
    // slot, end}; backward {diagonal slot, first early slot, end, 0}
    std::vector<int32_t> rinfo4, urinfo4;
    // forward levels >= l_split and backward levels < u_split run in one persistent launch
    // (with the persistent mode on, every level: l_split = 0, u_split = number of levels)
    int32_t l_split = 0, u_split = 0;
    // combined L+U in CSR for the row-oriented solves.  Rows of helped panels list their L
    // entries as [early | late | in-panel] and their U entries as [in-panel | late | early]:
    // early columns belong to panels more than kHelpAhead levels below in that triangle's
    // order, and helper items kHelpAhead levels early sum them into per-row partial sums (csr_early[i] = end of
    // the early L part, = csr_rowptr[i] when there is none; csr_uearly[i] = start of the
    // early U part, = csr_rowptr[i + 1] when there is none).
    std::vector<int32_t> csr_rowptr, csr_col, csr_src, csr_diag, csr_early, csr_uearly;
    // int32 row pointers of A and column pointers of L+U, as uploaded
    std::vector<int32_t> a_rowptr32, colptr32;
    // value update: per L+U slot {position of its entry in A's CSR value array or -1 for
    // fill-in, that entry's row of A}
    std::vector<int32_t> lu_src;
    double flops = 0.0;
    int64_t nnz_lu_wide = 0;            // L+U entries of columns factored by 512-thread launches
    int64_t nnz_lu_med = 0;             // ... by 256-thread launches of panels up to 16 columns
    int64_t nnz_lu_w256 = 0;            // ... by 256-thread launches of panels up to 32 columns
};

int build_schedule(const Symbolic &s, const SchedParams &prm, Schedule &g);

}  // namespace kkt
