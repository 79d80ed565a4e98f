// Device schedule of the refactorization and of the triangular solves, built once per
// pattern on the host (the one-time data movement and mapping of Section III).
//
// Panels.  Each structural supernode is cut into panels of at most panel_max consecutive
// columns.  Every column j of a panel [s, e) has the L rows {j+1..e-1} followed by the
// panel's common rows R below e-1, and every row of the panel has the same U columns C to
// the right of e-1; consequently each column k in C holds the rows s..e-1 consecutively.
//
// Refactorization (right-looking over panel levels, values pulled by their owner).  The
// level of a panel is one more than the highest level of any panel S with U(S, T) != 0 or
// L(T, S) != 0.  Launch l (l = 0..max level):
//   - every target column k of a panel S at level l-1 pulls S's update: the rows s..e-1
//     of column k are solved with S's unit lower diagonal block (they become final U
//     entries) and the rows R of column k lose L(R, S) times them;
//   - every panel at level l, whose columns are then complete, is factored densely
//     without pivoting (diagonal block, then the L rows R).
// A column is written only by the one work item that owns it in a launch, so no atomics
// are needed and the result is deterministic.
//
// Triangular solves (row oriented on a combined L+U CSR copy).  Forward level of a panel:
// one more than the highest level of a panel owning a column j of an L entry L(i, j) of one
// of its rows; backward level likewise over U entries to the right.
#include <algorithm>
#include <numeric>

#include "kkt_internal.h"

namespace kkt {

int build_schedule(const Symbolic &s, const SchedParams &prm, Schedule &g) {
    const int32_t n = s.n;
    if (prm.panel_max < 1 || prm.panel_max > kPanelMax || prm.small_rows < 0 || prm.small_rows > kSmallR ||
        prm.group < 1 || prm.group > kGroup || (prm.wide256 != 0 && prm.wide256 != 1) ||
        (prm.fuse_chains != 0 && prm.fuse_chains != 1) || prm.tiny_rows < 0 || prm.tiny_rows > kTinyR)
        return KKT_ERR_ARG;
    g = Schedule{};
    g.params = prm;
    const int64_t nlu = s.nnz_lu();
    if (nlu >= INT32_MAX || s.nnz_a >= INT32_MAX) return KKT_ERR_ARG;   // int32 slots on the device
    // panels
    g.pan_start.clear();
    for (int32_t t = 0; t + 1 < (int32_t)s.sn_start.size(); ++t) {
        const int32_t a = s.sn_start[t], b = s.sn_start[t + 1], w = b - a;
        const int32_t m = (w + prm.panel_max - 1) / prm.panel_max;
        for (int32_t q = 0; q < m; ++q) g.pan_start.push_back(a + (int32_t)((int64_t)w * q / m));
    }
    g.pan_start.push_back(n);
    // int32 copies of the pointer arrays that the device reads (uploaded as they are)
    g.a_rowptr32.resize(n + 1);
    g.colptr32.resize(n + 1);
    for (int32_t i = 0; i <= n; ++i) {
        g.a_rowptr32[i] = (int32_t)s.a_rowptr[i];
        g.colptr32[i] = (int32_t)s.colptr[i];
    }
    const int32_t np = g.npan = (int32_t)g.pan_start.size() - 1;
    std::vector<int32_t> pan_of(n);
    for (int32_t p = 0; p < np; ++p)
        for (int32_t j = g.pan_start[p]; j < g.pan_start[p + 1]; ++j) pan_of[j] = p;
    auto lbeg = [&](int32_t j) { return s.colptr[j] + s.ulen[j] + 1; };
    g.pan_r.resize(np);
    for (int32_t p = 0; p < np; ++p) {
        const int32_t sp = g.pan_start[p], e = g.pan_start[p + 1];
        g.pan_r[p] = (int32_t)(s.colptr[e] - lbeg(e - 1));
        // structure check: column j's L part is {j+1..e-1} followed by R
        const int64_t r0 = lbeg(e - 1);
        for (int32_t j = sp; j < e; ++j) {
            const int64_t l = lbeg(j);
            if (s.colptr[j + 1] - l != (e - 1 - j) + g.pan_r[p]) return KKT_ERR_SCHEDULE;
            for (int32_t t = 0; t < e - 1 - j; ++t)
                if (s.rowidx[l + t] != j + 1 + t) return KKT_ERR_SCHEDULE;
            if (!std::equal(s.rowidx.begin() + l + (e - 1 - j), s.rowidx.begin() + s.colptr[j + 1],
                            s.rowidx.begin() + r0))
                return KKT_ERR_SCHEDULE;
            // U rows s..j-1 directly above the diagonal
            if (s.ulen[j] < j - sp) return KKT_ERR_SCHEDULE;
            for (int32_t t = 0; t < j - sp; ++t)
                if (s.rowidx[s.colptr[j] + s.ulen[j] - (j - sp) + t] != sp + t) return KKT_ERR_SCHEDULE;
        }
    }
    // refactor levels of panels and (source, target) pairs.  A panel T waits for every
    // panel S with U(S, T) != 0 (its columns need S's update) and for every panel S with
    // L(T, S) != 0 (its rows of a later column must be updated by S before T's own update
    // of that column solves them); for symmetric patterns the two sets coincide.
    //
    // Chains (fuse_chains): consecutive panels of one supernode form a chain of levels, one
    // launch per panel.  A panel joins the group of the panel before it when every panel it
    // waits for outside the group is at a level below the group's: the group's item then
    // factors its panels in order and pulls each finished panel's update into the later
    // panels itself (internal pairs, in the group's launch), so the chain costs one launch.
    // Each group is at the level of its first panel; its panels share that level.
    std::vector<int32_t> plev(np, 0), grp(np);
    std::vector<int32_t> sn_of(n);
    for (int32_t t = 0; t + 1 < (int32_t)s.sn_start.size(); ++t)
        for (int32_t j = s.sn_start[t]; j < s.sn_start[t + 1]; ++j) sn_of[j] = t;
    // columns of the L entries of each row (row-wise view of L)
    std::vector<int64_t> lrp(n + 1, 0);
    std::vector<int32_t> lcol;
    if (prm.fuse_chains) {
        for (int32_t j = 0; j < n; ++j)
            for (int64_t p = lbeg(j); p < s.colptr[j + 1]; ++p) lrp[s.rowidx[p] + 1]++;
        for (int32_t i = 0; i < n; ++i) lrp[i + 1] += lrp[i];
        lcol.resize(lrp[n]);
        std::vector<int64_t> nx(lrp.begin(), lrp.end() - 1);
        for (int32_t j = 0; j < n; ++j)
            for (int64_t p = lbeg(j); p < s.colptr[j + 1]; ++p) lcol[nx[s.rowidx[p]]++] = j;
    }
    std::vector<std::pair<int32_t, int32_t>> pairs;   // (source panel, target column)
    for (int32_t T = 0; T < np; ++T) {
        grp[T] = T;
        if (prm.fuse_chains && T > 0 && grp[T - 1] >= 0 && sn_of[g.pan_start[T]] == sn_of[g.pan_start[T - 1]]) {
            // the levels of T's dependencies outside the group of T - 1
            const int32_t G = grp[T - 1];
            int32_t ext = -1;
            for (int32_t k = g.pan_start[T]; k < g.pan_start[T + 1]; ++k)
                for (int64_t p = s.colptr[k]; p < s.colptr[k] + s.ulen[k]; ++p) {
                    const int32_t S = pan_of[s.rowidx[p]];
                    if (S != T && (S < G || S > T)) ext = std::max(ext, plev[S]);
                }
            for (int32_t i = g.pan_start[T]; i < g.pan_start[T + 1]; ++i)
                for (int64_t p = lrp[i]; p < lrp[i + 1]; ++p) {
                    const int32_t S = pan_of[lcol[p]];
                    if (S != T && (S < G || S > T)) ext = std::max(ext, plev[S]);
                }
            if (ext < plev[G]) grp[T] = G;
        }
        const int32_t G = grp[T];
        if (G != T) {
            plev[T] = plev[G];
            for (int32_t k = g.pan_start[T]; k < g.pan_start[T + 1]; ++k)
                for (int64_t p = s.colptr[k]; p < s.colptr[k] + s.ulen[k]; ++p) {
                    const int32_t j = s.rowidx[p];
                    const int32_t S = pan_of[j];
                    if (S != T && j == g.pan_start[S + 1] - 1) pairs.emplace_back(S, k);
                }
        } else {
            for (int32_t k = g.pan_start[T]; k < g.pan_start[T + 1]; ++k)
                for (int64_t p = s.colptr[k]; p < s.colptr[k] + s.ulen[k]; ++p) {
                    const int32_t j = s.rowidx[p];
                    const int32_t S = pan_of[j];
                    if (S == T) continue;
                    plev[T] = std::max(plev[T], plev[S] + 1);
                    if (j == g.pan_start[S + 1] - 1) pairs.emplace_back(S, k);
                }
        }
        // plev[T] is final: push it along the L entries of T's columns (not into its group)
        for (int32_t j = g.pan_start[T]; j < g.pan_start[T + 1]; ++j)
            for (int64_t p = lbeg(j); p < s.colptr[j + 1]; ++p) {
                const int32_t R = pan_of[s.rowidx[p]];
                if (R != T) plev[R] = std::max(plev[R], plev[T] + 1);
            }
    }
    // every target column of S must hold the rows of S consecutively
    for (const auto &pr : pairs) {
        const int32_t S = pr.first, k = pr.second;
        const int32_t sp = g.pan_start[S], e = g.pan_start[S + 1];
        const auto b = s.rowidx.begin() + s.colptr[k], en = s.rowidx.begin() + s.colptr[k] + s.ulen[k];
        const auto it = std::lower_bound(b, en, sp);
        if (en - it < e - sp) return KKT_ERR_SCHEDULE;
        for (int32_t t = 0; t < e - sp; ++t)
            if (it[t] != sp + t) return KKT_ERR_SCHEDULE;
    }
    const int32_t nlev = np ? 1 + *std::max_element(plev.begin(), plev.end()) : 0;
    // group pairs by launch (= source level + 1, or the group's own launch for a pair inside
    // a group), then target column, then source
    std::vector<std::vector<std::pair<int32_t, int32_t>>> by_launch(nlev + 1);
    for (const auto &pr : pairs) {
        const bool inside = grp[pr.first] == grp[pan_of[pr.second]];
        by_launch[plev[pr.first] + (inside ? 0 : 1)].emplace_back(pr.second, pr.first);
    }
    std::vector<std::vector<int32_t>> panels_at(nlev);
    for (int32_t p = 0; p < np; ++p)
        if (grp[p] == p) panels_at[plev[p]].push_back(p);   // group leaders
    std::vector<int32_t> gsize(np, 0);
    for (int32_t p = 0; p < np; ++p) gsize[grp[p]]++;
    auto pw = [&](int32_t p) { return g.pan_start[p + 1] - g.pan_start[p]; };
    auto is_small = [&](int32_t p) { return pw(p) <= kSmallW && g.pan_r[p] <= prm.small_rows; };
    auto is_tiny = [&](int32_t p) { return is_small(p) && g.pan_r[p] <= prm.tiny_rows; };
    g.f_lvl.assign(1, 0);
    g.f_nlarge.clear();
    g.f_nmed.clear();
    g.f_ntiny.clear();
    g.f_w256.clear();
    g.f_item_panel.clear();
    g.f_item_npan.clear();
    g.f_item_pair.assign(1, 0);
    g.f_pair_src.clear();
    g.f_pair_tgt.clear();
    g.f_pair_pos.clear();
    g.f_pair_rel.assign(1, 0);
    g.f_rel.clear();
    std::vector<int32_t> fac_index(np, -1);
    struct Item {
        int32_t panel;
        std::vector<std::pair<int32_t, int32_t>> pairs;   // (source, target)
        bool small;
        double cost;
        int kind = 0;   // 0 wide (up to panel_max columns), 1 medium, 2 narrow, 3 tiny
        int32_t npan = 1;   // panels factored (a group's leader and the panels after it)
    };
    for (int32_t l = 0; l < nlev; ++l) {
        auto &pl = by_launch[l];                  // (target, source)
        std::sort(pl.begin(), pl.end());
        std::vector<Item> items;
        // factor items: the panel (or group of panels) and every pair that targets one of
        // its columns
        for (int32_t T : panels_at[l]) {
            Item it{T, {}, gsize[T] == 1 && is_small(T), 0.0};
            it.npan = gsize[T];
            items.push_back(it);
        }
        for (size_t i = 0; i < items.size(); ++i)
            for (int32_t t = 0; t < items[i].npan; ++t) fac_index[items[i].panel + t] = (int32_t)i;
        // pull-only targets: single-source targets are grouped by source
        std::vector<std::pair<int32_t, int32_t>> single;   // (source, target)
        for (size_t q = 0; q < pl.size();) {
            size_t q1 = q;
            while (q1 < pl.size() && pl[q1].first == pl[q].first) ++q1;
            const int32_t k = pl[q].first, T = pan_of[k];
            if (fac_index[T] >= 0) {
                for (size_t t = q; t < q1; ++t) items[fac_index[T]].pairs.emplace_back(pl[t].second, k);
            } else if (q1 - q == 1) {
                single.emplace_back(pl[q].second, k);
            } else {
                Item it{-1, {}, true, 0.0};
                for (size_t t = q; t < q1; ++t) it.pairs.emplace_back(pl[t].second, k);
                items.push_back(it);
            }
            q = q1;
        }
        std::sort(single.begin(), single.end());
        for (size_t q = 0; q < single.size();) {
            const int32_t S = single[q].first;
            const size_t cap = is_small(S) ? 1 : (size_t)prm.group;
            Item it{-1, {}, true, 0.0};
            size_t q1 = q;
            while (q1 < single.size() && single[q1].first == S && q1 - q < cap) it.pairs.push_back(single[q1++]);
            items.push_back(it);
            q = q1;
        }
        for (auto &it : items) {
            std::sort(it.pairs.begin(), it.pairs.end());
            int32_t mw = it.panel >= 0 ? pw(it.panel) : 0;
            bool tiny = it.small && (it.panel < 0 || is_tiny(it.panel));
            for (const auto &pr : it.pairs) {
                if (!is_small(pr.first)) it.small = false;
                if (!is_tiny(pr.first)) tiny = false;
                it.cost += (double)pw(pr.first) * (pw(pr.first) + g.pan_r[pr.first]);
                mw = std::max(mw, pw(pr.first));
            }
            for (int32_t t = 0; t < (it.panel >= 0 ? it.npan : 0); ++t) {
                const int32_t P = it.panel + t;
                it.cost += (double)pw(P) * pw(P) * (pw(P) + g.pan_r[P]);
            }
            const bool fits_med =
                mw <= kMedW && (it.panel < 0 || pw(it.panel) + g.pan_r[it.panel] <= kMedRows) && it.npan == 1;
            it.kind = it.small ? (tiny ? 3 : 2) : fits_med ? 1 : 0;
        }
        // the medium configuration only where a level has no item that needs the big one
        // (one launch per level for the wide items)
        bool any_big = false, fit256 = true;
        int32_t nbig = 0;
        for (const auto &it : items) {
            any_big |= it.kind == 0;
            nbig += it.kind == 0 || it.kind == 1;
            if (it.kind == 0 && it.panel >= 0 && (pw(it.panel) + g.pan_r[it.panel] > kW256Rows || it.npan > 1))
                fit256 = false;
        }
        if (any_big)
            for (auto &it : items)
                if (it.kind == 1) it.kind = 0;
        g.f_w256.push_back(any_big && fit256 && nbig >= kW256MinItems && prm.wide256 ? 1 : 0);
        for (int32_t T : panels_at[l])
            for (int32_t t = 0; t < gsize[T]; ++t) fac_index[T + t] = -1;
        std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) {
            if (a.kind != b.kind) return a.kind < b.kind;
            return a.cost > b.cost;
        });
        int32_t nlarge = 0, nmed = 0, ntiny = 0;
        for (const auto &it : items) {
            ntiny += it.kind == 3;
            // the wide path solves a source's targets kGroup at a time on the lanes of one
            // wavefront; narrow items take their pairs one at a time
            nlarge += !it.small;
            nmed += it.kind == 1;
            g.f_item_panel.push_back(it.panel);
            g.f_item_npan.push_back(it.npan);
            for (const auto &pr : it.pairs) {
                g.f_pair_src.push_back(pr.first);
                g.f_pair_tgt.push_back(pr.second);
                const int32_t k = pr.second, S = pr.first, sp = g.pan_start[S], e = g.pan_start[S + 1];
                const auto b = s.rowidx.begin() + s.colptr[k];
                const int64_t ps = std::lower_bound(b, b + s.ulen[k], sp) - s.rowidx.begin();
                g.f_pair_pos.push_back((int32_t)ps);
                // rows R of S (ascending) matched against the rest of column k (ascending)
                int64_t p = ps + (e - sp);
                const int64_t pend = s.colptr[k + 1];
                for (int64_t t = lbeg(e - 1); t < s.colptr[e]; ++t) {
                    const int32_t row = s.rowidx[t];
                    while (p < pend && s.rowidx[p] < row) ++p;
                    if (p == pend || s.rowidx[p] != row) return KKT_ERR_SCHEDULE;
                    g.f_rel.push_back((int32_t)p);
                }
                g.f_pair_rel.push_back((int64_t)g.f_rel.size());
            }
            g.f_item_pair.push_back((int32_t)g.f_pair_src.size());
        }
        g.f_nlarge.push_back(nlarge);
        g.f_nmed.push_back(nmed);
        g.f_ntiny.push_back(ntiny);
        g.f_lvl.push_back((int32_t)g.f_item_panel.size());
    }
    if (!by_launch[nlev].empty()) return KKT_ERR_SCHEDULE;   // top panels have no targets
    if (g.f_rel.size() >= (size_t)INT32_MAX) return KKT_ERR_ARG;
    g.ldiag.resize(n);
    for (int32_t j = 0; j < n; ++j) g.ldiag[j] = (int32_t)(s.colptr[j] + s.ulen[j]);
    // packed records: item i = {T, first pair, end pair, panels factored, s, w, r, ldiag[s],
    // s', w', r', ldiag[s']} with T the panel it factors (or -1), s, w, r that panel's first
    // column, width and rows below, and s', w', r' those of its first pair's source; pair q = {S, pos, rel, end of its group, s, w, r, ldiag[s]} with
    // the source panel's geometry
    auto geom = [&](int32_t *o, int32_t P) {
        o[0] = P >= 0 ? g.pan_start[P] : 0;
        o[1] = P >= 0 ? pw(P) : 0;
        o[2] = P >= 0 ? g.pan_r[P] : 0;
        o[3] = P >= 0 ? g.ldiag[g.pan_start[P]] : 0;
    };
    const size_t nitems = g.f_item_panel.size();
    g.itemrec.resize(12 * nitems);
    for (size_t i = 0; i < nitems; ++i) {
        int32_t *o = &g.itemrec[12 * i];
        o[0] = g.f_item_panel[i];
        o[1] = g.f_item_pair[i];
        o[2] = g.f_item_pair[i + 1];
        o[3] = g.f_item_npan[i];
        geom(o + 4, g.f_item_panel[i]);
        geom(o + 8, g.f_item_pair[i] < g.f_item_pair[i + 1] ? g.f_pair_src[g.f_item_pair[i]] : -1);
    }
    // pairs of narrow items (16-lane path) carry the diagonal slots of all source columns
    // instead: {ldiag[s+1], pos, rel, ldiag[s+2], ldiag[s+3], w, r, ldiag[s]} (0 past w).
    // Pairs of wide items carry, in place of the target column, the end of their group: the
    // run of consecutive pairs of one source, at most kGroup long, that the wide path pulls
    // together.
    const size_t npairs = g.f_pair_src.size();
    g.pair8.resize(8 * npairs);
    std::vector<char> narrow_pair(npairs, 0);
    std::vector<int32_t> group_end(npairs, 0);
    for (size_t l = 0; l + 1 < g.f_lvl.size(); ++l) {
        for (int32_t it = g.f_lvl[l] + g.f_nlarge[l]; it < g.f_lvl[l + 1]; ++it)
            for (int32_t q = g.f_item_pair[it]; q < g.f_item_pair[it + 1]; ++q) narrow_pair[q] = 1;
        for (int32_t it = g.f_lvl[l]; it < g.f_lvl[l] + g.f_nlarge[l]; ++it) {
            const int32_t q1 = g.f_item_pair[it + 1];
            for (int32_t g0 = g.f_item_pair[it], g1; g0 < q1; g0 = g1) {
                g1 = g0 + 1;
                while (g1 < q1 && g.f_pair_src[g1] == g.f_pair_src[g0] && g1 - g0 < kGroup) ++g1;
                for (int32_t q = g0; q < g1; ++q) group_end[q] = g1;
            }
        }
    }
    for (size_t q = 0; q < npairs; ++q) {
        int32_t *o = &g.pair8[8 * q];
        const int32_t S = g.f_pair_src[q];
        o[1] = g.f_pair_pos[q];
        o[2] = (int32_t)g.f_pair_rel[q];
        geom(o + 4, S);
        if (narrow_pair[q]) {
            const int32_t sp = g.pan_start[S], w = pw(S);
            auto dslot = [&](int32_t j) { return j < w ? g.ldiag[sp + j] : 0; };
            o[0] = dslot(1);
            o[3] = dslot(2);
            o[4] = dslot(3);
        } else {
            o[0] = S;
            o[3] = group_end[q];
        }
    }
    // solve levels
    std::vector<int32_t> llev(np, 0), ulev(np, 0);
    for (int32_t j = 0; j < n; ++j)
        for (int64_t p = lbeg(j); p < s.colptr[j + 1]; ++p) {
            const int32_t T = pan_of[s.rowidx[p]], S = pan_of[j];
            if (T != S) llev[T] = std::max(llev[T], llev[S] + 1);
        }
    for (int32_t j = n - 1; j >= 0; --j)
        for (int64_t p = s.colptr[j]; p < s.colptr[j] + s.ulen[j]; ++p) {
            const int32_t T = pan_of[s.rowidx[p]], S = pan_of[j];
            if (T != S) ulev[T] = std::max(ulev[T], ulev[S] + 1);
        }
    // solve helpers: a wide panel T (more than kPackW columns) of a triangle with a row of at
    // least kHelpMin early entries (external entries in panels more than kHelpAhead levels
    // below T) gets helper items at level lev[T] - kHelpAhead that sum those entries
    std::vector<char> has_lhelp(np, 0), has_uhelp(np, 0);
    {
        std::vector<int32_t> lcnt(n, 0), ucnt(n, 0);
        for (int32_t j = 0; j < n; ++j) {
            const int32_t S = pan_of[j];
            for (int64_t p = lbeg(j); p < s.colptr[j + 1]; ++p) {
                const int32_t i = s.rowidx[p], T = pan_of[i];
                if (T != S && pw(T) > kPackW && llev[S] < llev[T] - kHelpAhead) lcnt[i]++;
            }
            for (int64_t p = s.colptr[j]; p < s.colptr[j] + s.ulen[j]; ++p) {
                const int32_t i = s.rowidx[p], T = pan_of[i];
                if (T != S && pw(T) > kPackW && ulev[S] < ulev[T] - kHelpAhead) ucnt[i]++;
            }
        }
        for (int32_t i = 0; i < n; ++i) {
            if (lcnt[i] >= kHelpMin) has_lhelp[pan_of[i]] = 1;
            if (ucnt[i] >= kHelpMin) has_uhelp[pan_of[i]] = 1;
        }
    }
    // solve items; pack rows hold the row index only until the CSR copy exists
    auto build_solve = [&](const std::vector<int32_t> &lev, std::vector<int32_t> &lvl, std::vector<int32_t> &item4,
                           std::vector<int32_t> &rows4, const std::vector<char> &has_helper) {
        const int32_t nl = np ? 1 + *std::max_element(lev.begin(), lev.end()) : 0;
        std::vector<std::vector<int32_t>> at(nl), help(nl);
        for (int32_t p = 0; p < np; ++p) {
            at[lev[p]].push_back(p);
            if (has_helper[p]) help[lev[p] - kHelpAhead].push_back(p);
        }
        lvl.assign(1, 0);
        item4.clear();
        rows4.clear();
        auto push = [&](int32_t a, int32_t b, int32_t c, int32_t d) {
            item4.push_back(a);
            item4.push_back(b);
            item4.push_back(c);
            item4.push_back(d);
        };
        for (int32_t l = 0; l < nl; ++l) {
            for (int32_t p : help[l])
                for (int32_t t0 = 0; t0 < pw(p); t0 += kHelpRows) push(0, t0, g.pan_start[p], pw(p));
            std::vector<int32_t> wide, small;
            for (int32_t p : at[l]) (pw(p) > kPackW ? wide : small).push_back(p);
            std::stable_sort(wide.begin(), wide.end(), [&](int32_t a, int32_t b) { return pw(a) > pw(b); });
            // lanes per row: the largest power of two that fits the item's rows in 256 threads,
            // at most one wavefront
            auto lanes_for = [](int32_t rows) {
                int32_t l = 64;
                while (l * rows > 256) l >>= 1;
                return l;
            };
            for (int32_t p : wide) push(1, lanes_for(pw(p)), g.pan_start[p], pw(p));
            // whole small panels, at most kSolvePack rows per pack
            for (size_t q = 0; q < small.size();) {
                const int32_t off = (int32_t)(rows4.size() / 4);
                int32_t c = 0;
                while (q < small.size() && c + pw(small[q]) <= kSolvePack) {
                    const int32_t p = small[q++];
                    for (int32_t t = 0; t < pw(p); ++t, ++c) {
                        rows4.push_back(g.pan_start[p] + t);
                        rows4.push_back(0);
                        rows4.push_back(0);
                        rows4.push_back(t | pw(p) << 8);
                    }
                }
                push(-c, off, lanes_for(c), 0);
            }
            lvl.push_back((int32_t)(item4.size() / 4));
        }
    };
    build_solve(llev, g.l_lvl, g.l_item4, g.l_rows4, has_lhelp);
    build_solve(ulev, g.u_lvl, g.u_item4, g.u_rows4, has_uhelp);
    // with the persistent mode on, one launch per triangle covers every level
    g.l_split = 0;
    g.u_split = (int32_t)g.u_lvl.size() - 1;
    // combined L+U in CSR: row i lists (i, j) by ascending j, csr_src = CSC slot
    g.csr_rowptr.assign(n + 1, 0);
    for (int64_t p = 0; p < nlu; ++p) g.csr_rowptr[s.rowidx[p] + 1]++;
    for (int32_t i = 0; i < n; ++i) g.csr_rowptr[i + 1] += g.csr_rowptr[i];
    g.csr_col.resize(nlu);
    g.csr_src.resize(nlu);
    g.csr_diag.resize(n);
    {
        std::vector<int32_t> nxt(g.csr_rowptr.begin(), g.csr_rowptr.end() - 1);
        for (int32_t j = 0; j < n; ++j)
            for (int64_t p = s.colptr[j]; p < s.colptr[j + 1]; ++p) {
                const int32_t i = s.rowidx[p];
                const int32_t q = nxt[i]++;
                g.csr_col[q] = j;
                g.csr_src[q] = (int32_t)p;
                if (i == j) g.csr_diag[i] = q;
            }
    }
    // rows of helped panels list their external L entries as [early | late] (before the
    // in-panel part) and their external U entries as [late | early] (after it)
    g.csr_early.assign(g.csr_rowptr.begin(), g.csr_rowptr.end() - 1);
    g.csr_uearly.assign(g.csr_rowptr.begin() + 1, g.csr_rowptr.end());
    {
        std::vector<int32_t> tc, ts;
        auto split = [&](int32_t q0, int32_t q1, int32_t T, const std::vector<int32_t> &lev, bool early_first) {
            tc.clear();
            ts.clear();
            int32_t ne = 0;
            for (int pass = 0; pass < 2; ++pass)
                for (int32_t q = q0; q < q1; ++q) {
                    const bool early = lev[pan_of[g.csr_col[q]]] < lev[T] - kHelpAhead;
                    ne += pass == 0 && early;
                    if (early == ((pass == 0) == early_first)) {
                        tc.push_back(g.csr_col[q]);
                        ts.push_back(g.csr_src[q]);
                    }
                }
            std::copy(tc.begin(), tc.end(), g.csr_col.begin() + q0);
            std::copy(ts.begin(), ts.end(), g.csr_src.begin() + q0);
            return ne;
        };
        for (int32_t T = 0; T < np; ++T) {
            const int32_t sp = g.pan_start[T], w = pw(T);
            for (int32_t i = sp; i < sp + w; ++i) {
                const int32_t t = i - sp;
                if (has_lhelp[T]) {
                    const int32_t q0 = g.csr_rowptr[i], q1 = g.csr_diag[i] - t;
                    g.csr_early[i] = q0 + split(q0, q1, T, llev, true);
                }
                if (has_uhelp[T]) {
                    const int32_t q0 = g.csr_diag[i] + (w - t), q1 = g.csr_rowptr[i + 1];
                    g.csr_uearly[i] = q1 - split(q0, q1, T, ulev, false);
                }
            }
        }
    }
    // per-row records and the external ranges of pack rows
    g.rinfo4.resize(4 * (size_t)n);
    g.urinfo4.resize(4 * (size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        g.rinfo4[4 * (size_t)i] = g.csr_rowptr[i];
        g.rinfo4[4 * (size_t)i + 1] = g.csr_early[i];
        g.rinfo4[4 * (size_t)i + 2] = g.csr_diag[i];
        g.rinfo4[4 * (size_t)i + 3] = g.csr_rowptr[i + 1];
        g.urinfo4[4 * (size_t)i] = g.csr_diag[i];
        g.urinfo4[4 * (size_t)i + 1] = g.csr_uearly[i];
        g.urinfo4[4 * (size_t)i + 2] = g.csr_rowptr[i + 1];
        g.urinfo4[4 * (size_t)i + 3] = 0;
    }
    for (size_t k = 0; k < g.l_rows4.size(); k += 4) {
        const int32_t i = g.l_rows4[k], t = g.l_rows4[k + 3] & 255;
        g.l_rows4[k + 1] = g.csr_rowptr[i];
        g.l_rows4[k + 2] = g.csr_diag[i] - t;
    }
    for (size_t k = 0; k < g.u_rows4.size(); k += 4) {
        const int32_t i = g.u_rows4[k], t = g.u_rows4[k + 3] & 255, w = g.u_rows4[k + 3] >> 8;
        g.u_rows4[k + 1] = g.csr_diag[i] + (w - t);
        g.u_rows4[k + 2] = g.csr_rowptr[i + 1];
    }
    // value update: for each factor slot, the position of its entry of A in the CSR value
    // array (-1 for a fill-in slot) and that entry's row of A
    g.lu_src.assign(2 * (size_t)nlu, -1);
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = s.a_rowptr[i]; e < s.a_rowptr[i + 1]; ++e) {
            const int64_t p = s.map[e];
            if (g.lu_src[2 * p] >= 0) return KKT_ERR_SCHEDULE;   // two entries of A in one slot
            g.lu_src[2 * p] = (int32_t)e;
            g.lu_src[2 * p + 1] = i;
        }
    // refactor flops: sum_k 2 |L(:,k)| |U(k,:)| + |L(:,k)|
    std::vector<int64_t> urow(n, 0);
    for (int32_t k = 0; k < n; ++k)
        for (int64_t p = s.colptr[k]; p < s.colptr[k] + s.ulen[k]; ++p) urow[s.rowidx[p]]++;
    double fl = 0.0;
    for (int32_t k = 0; k < n; ++k) {
        const double lk = (double)(s.colptr[k + 1] - lbeg(k));
        fl += 2.0 * lk * (double)urow[k] + lk;
    }
    g.flops = fl;
    // the row-ordered copy of the factor: an entry can be copied once its column is final,
    // i.e. after the launch that factors the column's panel.  copy_k lists the strictly lower
    // (L) entries first, then the others (U and the diagonal); each section by the launch
    // that finishes their column (copy_lat[l], copy_uat[l] = first entry of launch l in each),
    // in factor storage order within a launch, and copy_src[q] = csr_src[copy_k[q]]: a copy
    // reads the factor nearly in order and scatters only its stores.  The forward solve reads
    // only L, so the fused refactorization copies L level by level and spreads U over its top
    // launches.  The top levels (copy_lvl on) have few items and leave most of the GPU idle.
    const int32_t nlev_f = (int32_t)g.f_lvl.size() - 1;
    {
        int32_t win = nlev_f;
        while (win > 0 && g.f_lvl[win] - g.f_lvl[win - 1] <= kCopyItems && g.f_nlarge[win - 1] > 0) --win;
        g.copy_lvl = win;
        std::vector<char> upper(nlu, 0);   // U or diagonal entry (CSR position)
        for (int32_t i = 0; i < n; ++i)
            for (int32_t q = g.csr_rowptr[i]; q < g.csr_rowptr[i + 1]; ++q) upper[q] = g.csr_col[q] >= i;
        // counts per (section, level), then offsets: L section first
        std::vector<int64_t> cnt(2 * (size_t)(nlev_f + 1), 0);
        for (int64_t q = 0; q < nlu; ++q) cnt[upper[q] * (nlev_f + 1) + plev[pan_of[g.csr_col[q]]] + 1]++;
        g.copy_lat.assign(nlev_f + 1, 0);
        g.copy_uat.assign(nlev_f + 1, 0);
        for (int32_t l = 0; l < nlev_f; ++l) g.copy_lat[l + 1] = g.copy_lat[l] + (int32_t)cnt[l + 1];
        g.copy_uat[0] = g.copy_lat[nlev_f];
        for (int32_t l = 0; l < nlev_f; ++l) g.copy_uat[l + 1] = g.copy_uat[l] + (int32_t)cnt[(nlev_f + 1) + l + 1];
        g.copy_k.resize(nlu);
        std::vector<int32_t> nl(g.copy_lat.begin(), g.copy_lat.end() - 1), nu(g.copy_uat.begin(), g.copy_uat.end() - 1);
        for (int64_t q = 0; q < nlu; ++q) {
            const int32_t l = plev[pan_of[g.csr_col[q]]];
            g.copy_k[upper[q] ? nu[l]++ : nl[l]++] = (int32_t)q;
        }
        auto by_slot = [&](int32_t a, int32_t b) { return g.csr_src[a] < g.csr_src[b]; };
        for (int32_t l = 0; l < nlev_f; ++l) {
            std::sort(g.copy_k.begin() + g.copy_lat[l], g.copy_k.begin() + g.copy_lat[l + 1], by_slot);
            std::sort(g.copy_k.begin() + g.copy_uat[l], g.copy_k.begin() + g.copy_uat[l + 1], by_slot);
        }
        g.copy_src.resize(nlu);
        for (int64_t q = 0; q < nlu; ++q) g.copy_src[q] = g.csr_src[g.copy_k[q]];
    }
    // forward solve fused with the refactorization: the ready launch of a forward item is the
    // latest launch that finishes a column whose entries it reads (its own panel's included)
    // or that is the ready launch of an item whose unknowns or partial sums it reads;
    // l_ready[k] = the latest ready launch of the items of forward level k
    {
        const int32_t nit = (int32_t)(g.l_item4.size() / 4);
        std::vector<int32_t> yprod(n, -1), hprod(n, -1), rl(nit, 0);
        bool okp = true;
        auto ready = [&](int32_t q0, int32_t q1, int32_t r) {
            for (int32_t q = q0; q < q1; ++q) {
                const int32_t j = g.csr_col[q];
                r = std::max(r, plev[pan_of[j]]);
                if (yprod[j] < 0) okp = false;
                else r = std::max(r, rl[yprod[j]]);
            }
            return r;
        };
        for (int32_t it = 0; it < nit; ++it) {
            const int32_t *c = &g.l_item4[4 * (size_t)it];
            int32_t r = 0;
            if (c[0] < 0) {                      // pack: rows {row, first external, end external, t|w<<8}
                for (int32_t k = 0; k < -c[0]; ++k) {
                    const int32_t *rr = &g.l_rows4[4 * (size_t)(c[1] + k)];
                    r = ready(rr[1], rr[2], std::max(r, plev[pan_of[rr[0]]]));
                }
                for (int32_t k = 0; k < -c[0]; ++k) yprod[g.l_rows4[4 * (size_t)(c[1] + k)]] = it;
            } else if (c[0] == 0) {              // helper: early entries of kHelpRows rows
                for (int32_t t = c[1]; t < std::min(c[3], c[1] + kHelpRows); ++t) {
                    const int32_t i = c[2] + t;
                    r = ready(g.rinfo4[4 * (size_t)i], g.rinfo4[4 * (size_t)i + 1], r);
                }
                for (int32_t t = c[1]; t < std::min(c[3], c[1] + kHelpRows); ++t) hprod[c[2] + t] = it;
            } else {                             // wide panel: late external entries, partial sums
                r = plev[pan_of[c[2]]];
                for (int32_t t = 0; t < c[3]; ++t) {
                    const int32_t i = c[2] + t;
                    r = ready(g.rinfo4[4 * (size_t)i + 1], g.rinfo4[4 * (size_t)i + 2] - t, r);
                    if (hprod[i] >= 0) r = std::max(r, rl[hprod[i]]);
                }
                for (int32_t t = 0; t < c[3]; ++t) yprod[c[2] + t] = it;
            }
            rl[it] = r;
        }
        if (!okp) return KKT_ERR_SCHEDULE;
        g.l_ready.assign(g.l_lvl.size() - 1, 0);
        for (size_t k = 0; k + 1 < g.l_lvl.size(); ++k)
            for (int32_t it = g.l_lvl[k]; it < g.l_lvl[k + 1]; ++it) g.l_ready[k] = std::max(g.l_ready[k], rl[it]);
    }
    // per launch kind: the 512-thread launch of a level factors its wide items and its narrow
    // ones, the 256-thread launch its medium items and (with no 512-thread launch) the narrow
    // ones; levels without wide items have a narrow launch
    g.nnz_lu_wide = g.nnz_lu_med = g.nnz_lu_w256 = 0;
    for (size_t l = 0; l + 1 < g.f_lvl.size(); ++l) {
        const int32_t nm = g.f_nmed[l], nb = g.f_nlarge[l] - nm;
        for (int32_t it = g.f_lvl[l]; it < g.f_lvl[l + 1]; ++it) {
            const int32_t P = g.f_item_panel[it];
            if (P < 0) continue;
            const int64_t e = s.colptr[g.pan_start[P + g.f_item_npan[it]]] - s.colptr[g.pan_start[P]];
            const bool med = (it >= g.f_lvl[l] + nb && it < g.f_lvl[l] + nb + nm) || (nb == 0 && nm > 0);
            if (nb > 0 && !med) (g.f_w256[l] ? g.nnz_lu_w256 : g.nnz_lu_wide) += e;
            else if (med) g.nnz_lu_med += e;
        }
    }
    return KKT_OK;
}

}  // namespace kkt
