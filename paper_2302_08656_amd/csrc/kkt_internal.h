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
constexpr int kGroup = 32;
constexpr int kPersistItems = 64;

// Device schedule, built on the host once per pattern and uploaded by kkt_bind.
struct Schedule {
    int32_t npan = 0;
    std::vector<int32_t> pan_start;     // [npan+1] first column of each panel
    std::vector<int32_t> pan_r;         // [npan] L rows below the panel (= U columns right)
    // refactorization: launch l runs items [f_lvl[l], f_lvl[l+1]); the first f_nlarge[l] of
    // them take the 256-thread path, the rest the 16-lane path.  An item owns the target
    // columns of its (source panel, target column) pairs, listed source-major, and then
    // factors its panel (f_item_panel >= 0).
    std::vector<int32_t> f_lvl, f_nlarge;
    std::vector<int32_t> f_item_panel;  // panel to factor after the pulls, or -1
    std::vector<int32_t> f_item_pair;   // [nitems+1] range into f_pair_src / f_pair_tgt
    std::vector<int32_t> f_pair_src, f_pair_tgt;
    std::vector<int32_t> f_pair_pos;    // slot of the source's first row in the target column
    std::vector<int64_t> f_pair_rel;    // [npairs+1] range into f_rel
    std::vector<int32_t> f_rel;         // slot of each row R of the source in the target column
    // packed records read by the refactorization kernels (8 x int32 each):
    // item8[i] = {panel to factor or -1, first pair, end pair, 0, s, w, r, ldiag[s]};
    // pair8[q] = {source panel, f_pair_pos, f_pair_rel (first index), target column,
    //             s, w, r, ldiag[s]}, with s, w, r the panel's first column, width, rows below
    std::vector<int32_t> item8, pair8;
    std::vector<int32_t> ldiag;         // slot of the diagonal of each column
    // triangular solves: launch l runs items [x_lvl[l], x_lvl[l+1]); an item is a wide
    // panel (np = 1, pan = panel), a helper (np = 0, pan = panel) or a pack of -np width-1
    // panels (pan = their rows)
    std::vector<int32_t> l_lvl, l_item_p0, l_item_np;
    std::vector<int32_t> u_lvl, u_item_p0, u_item_np;
    // level-sorted panel lists referenced by the solve items
    std::vector<int32_t> l_pan, u_pan;
    // hybrid solves: forward levels >= l_split and backward levels < u_split (the narrow top
    // of the tree, at most kPersistItems items per level) run in one persistent launch
    int32_t l_split = 0, u_split = 0;
    // combined L+U in CSR for the row-oriented solves.  Rows of wide panels list their L
    // entries as [early | late | in-panel]: early columns belong to panels two or more
    // forward levels below, and a helper item one level early sums them into a per-row
    // partial sum (csr_early[i] = end of the early part, = csr_rowptr[i] when there is none).
    std::vector<int32_t> csr_rowptr, csr_col, csr_src, csr_diag, csr_early;
    // value update: for each L+U slot, the CSR entry of A it receives (-1: fill)
    std::vector<int32_t> lu_src;
    // CSC view of A's pattern (positions into the CSR value array)
    std::vector<int32_t> a_cptr, a_cpos, a_rowid;
    double flops = 0.0;
};

int build_schedule(const Symbolic &s, Schedule &g);

}  // namespace kkt
