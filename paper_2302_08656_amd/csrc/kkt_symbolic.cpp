// Host analysis stage of the KKT refactorization library (Section II: analysis stage of a
// sparse direct solver -- equilibrate, choose the column order and the pivot order, fix
// the pattern of the factors; Section III, Algorithm 1: factor the first system on the
// CPU, extract the permutations and the L/U structure).
//
// The canonical outputs (P, Q, the combined L+U pattern, elimination tree, levels,
// supernodes, scatter map) are fully determined by these rules:
//  - column order: exact minimum degree on pattern(A + A^T), one vertex at a time, ties
//    broken by the lowest index;
//  - scaling: r_i = 2^-floor(log2 max_j |a_ij|), then c_j the same on R A;
//  - pivots: left-looking LU of the scaled matrix in that column order; each entry is
//    updated as x -= l*u with the product rounded first, in ascending pivot step; the
//    diagonal is kept when it is a nonzero candidate and |x_diag| >= tau * max|cand|,
//    else the largest candidate with the lowest row index wins;
//  - structural zeros are kept.
#include <algorithm>
#include <cmath>
#include <functional>
#include <queue>
#include <set>

#include "kkt_internal.h"

namespace kkt {

int validate_pattern(int32_t n, const int64_t *rowptr, const int32_t *colind) {
    if (n <= 0 || rowptr == nullptr || colind == nullptr) return KKT_ERR_ARG;
    if (rowptr[0] != 0) return KKT_ERR_PATTERN;
    for (int32_t i = 0; i < n; ++i) {
        const int64_t b = rowptr[i], e = rowptr[i + 1];
        if (e < b) return KKT_ERR_PATTERN;
        bool diag = false;
        int32_t prev = -1;
        for (int64_t p = b; p < e; ++p) {
            const int32_t j = colind[p];
            if (j < 0 || j >= n || j <= prev) return KKT_ERR_PATTERN;
            diag |= (j == i);
            prev = j;
        }
        if (!diag) return KKT_ERR_PATTERN;
    }
    return KKT_OK;
}

// ------------------------------------------------------------------------------------
// Exact minimum degree in the quotient-graph representation.  A variable keeps a list of
// variable neighbours (original edges) and a list of adjacent elements (eliminated
// vertices); an element keeps its boundary (the live variables it connects).  Eliminating
// v forms element v with boundary L_v = vars(v) U boundaries of v's elements, absorbs
// v's old elements, and recomputes the exact external degree
// |vars(u) U boundaries(elements(u)) \ {u}| of every u in L_v.
int exact_min_degree(int32_t n, const int64_t *rowptr, const int32_t *colind,
                     std::vector<int32_t> &order) {
    std::vector<std::vector<int32_t>> vars(n), elems(n), bnd(n);
    for (int32_t i = 0; i < n; ++i)
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const int32_t j = colind[p];
            if (j == i) continue;
            vars[i].push_back(j);
            vars[j].push_back(i);
        }
    std::vector<int32_t> degree(n);
    for (int32_t i = 0; i < n; ++i) {
        auto &a = vars[i];
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
        degree[i] = (int32_t)a.size();
    }
    std::set<std::pair<int32_t, int32_t>> queue;
    for (int32_t i = 0; i < n; ++i) queue.emplace(degree[i], i);
    std::vector<char> dead(n, 0);
    std::vector<int64_t> seen(n, -1), absorbed(n, -1);
    int64_t stamp = 0;
    std::vector<int32_t> Lv;
    order.assign(n, -1);
    for (int32_t k = 0; k < n; ++k) {
        const int32_t v = queue.begin()->second;
        queue.erase(queue.begin());
        order[k] = v;
        dead[v] = 1;
        ++stamp;
        seen[v] = stamp;
        Lv.clear();
        for (int32_t w : vars[v])
            if (!dead[w] && seen[w] != stamp) { seen[w] = stamp; Lv.push_back(w); }
        for (int32_t e : elems[v]) {
            for (int32_t w : bnd[e])
                if (!dead[w] && seen[w] != stamp) { seen[w] = stamp; Lv.push_back(w); }
            absorbed[e] = k;
            std::vector<int32_t>().swap(bnd[e]);
        }
        std::vector<int32_t>().swap(vars[v]);
        std::vector<int32_t>().swap(elems[v]);
        bnd[v] = Lv;
        // seen[w] == stamp marks L_v and v: edges between them are now covered by element v
        for (int32_t u : Lv) {
            auto &el = elems[u];
            el.erase(std::remove_if(el.begin(), el.end(), [&](int32_t e) { return absorbed[e] == k; }),
                     el.end());
            el.push_back(v);
            auto &va = vars[u];
            va.erase(std::remove_if(va.begin(), va.end(), [&](int32_t w) { return seen[w] == stamp; }),
                     va.end());
        }
        for (int32_t u : Lv) {
            ++stamp;
            seen[u] = stamp;
            int32_t d = 0;
            for (int32_t w : vars[u])
                if (seen[w] != stamp) { seen[w] = stamp; ++d; }
            for (int32_t e : elems[u])
                for (int32_t w : bnd[e])
                    if (seen[w] != stamp) { seen[w] = stamp; ++d; }
            if (d != degree[u]) {
                queue.erase({degree[u], u});
                degree[u] = d;
                queue.emplace(d, u);
            }
        }
    }
    return KKT_OK;
}

// ------------------------------------------------------------------------------------
static double inv_pow2_floor_log2(double m) {
    if (!(m > 0.0)) return 1.0;
    int e = std::ilogb(m);
    e = std::min(1020, std::max(-1020, e));
    return std::ldexp(1.0, -e);
}

int pow2_scaling(int32_t n, const int64_t *rowptr, const int32_t *colind, const double *v,
                 bool scale, std::vector<double> &r, std::vector<double> &c) {
    r.assign(n, 1.0);
    c.assign(n, 1.0);
    const int64_t nnz = rowptr[n];
    for (int64_t p = 0; p < nnz; ++p)
        if (!std::isfinite(v[p])) return KKT_ERR_NONFINITE;
    if (!scale) return KKT_OK;
    std::vector<double> cmax(n, 0.0);
    for (int32_t i = 0; i < n; ++i) {
        double m = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) m = std::max(m, std::fabs(v[p]));
        r[i] = inv_pow2_floor_log2(m);
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            cmax[colind[p]] = std::max(cmax[colind[p]], std::fabs(r[i] * v[p]));
    }
    for (int32_t j = 0; j < n; ++j) c[j] = inv_pow2_floor_log2(cmax[j]);
    return KKT_OK;
}

// ------------------------------------------------------------------------------------
// Left-looking LU of the scaled matrix in column order Q.  The pivotal rows that column k
// touches are visited in ascending pivot step with a min-heap: starting from the pivotal
// rows of A(:, Q[k]), popping step j applies L(:, j) and pushes the pivotal rows it
// reaches (their steps exceed j), so the updates run in ascending j and the visited set is
// the reach of the column.
int analyze_symbolic(int32_t n, const int64_t *rowptr, const int32_t *colind,
                     const double *values, const kkt_opts &o, Symbolic &s) {
    int rc = validate_pattern(n, rowptr, colind);
    if (rc) return rc;
    if (values == nullptr || o.sn_max_width < 1 || !(o.pivot_tau >= 0.0 && o.pivot_tau <= 1.0))
        return KKT_ERR_ARG;
    if (o.fixed_p && !o.fixed_q) return KKT_ERR_ARG;
    const int64_t nnz = rowptr[n];
    s.n = n;
    s.nnz_a = nnz;
    s.a_rowptr.assign(rowptr, rowptr + n + 1);
    s.a_colind.assign(colind, colind + nnz);
    // columns of A: CSR positions grouped by column, rows ascending
    std::vector<int64_t> acp(n + 1, 0);
    std::vector<int64_t> apos(nnz);
    std::vector<int32_t> arow(nnz);
    for (int64_t p = 0; p < nnz; ++p) acp[colind[p] + 1]++;
    for (int32_t j = 0; j < n; ++j) acp[j + 1] += acp[j];
    {
        std::vector<int64_t> nxt(acp.begin(), acp.end() - 1);
        for (int32_t i = 0; i < n; ++i)
            for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
                const int64_t t = nxt[colind[p]]++;
                apos[t] = p;
                arow[t] = i;
            }
    }
    // column order
    s.Q.resize(n);
    s.qinv.assign(n, -1);
    if (o.fixed_q) {
        for (int32_t k = 0; k < n; ++k) {
            const int32_t q = o.fixed_q[k];
            if (q < 0 || q >= n || s.qinv[q] >= 0) return KKT_ERR_ARG;
            s.qinv[q] = k;
            s.Q[k] = q;
        }
    } else {
        rc = exact_min_degree(n, rowptr, colind, s.Q);
        if (rc) return rc;
        for (int32_t k = 0; k < n; ++k) s.qinv[s.Q[k]] = k;
    }
    if (o.fixed_p) {
        std::vector<char> used(n, 0);
        for (int32_t k = 0; k < n; ++k) {
            const int32_t p = o.fixed_p[k];
            if (p < 0 || p >= n || used[p]) return KKT_ERR_ARG;
            used[p] = 1;
        }
    }
    std::vector<double> r, c;
    rc = pow2_scaling(n, rowptr, colind, values, o.equilibrate != 0, r, c);
    if (rc) return rc;

    // factor storage while the pattern grows: L columns keep original row numbers
    std::vector<std::vector<std::pair<int32_t, double>>> Lcol(n);
    std::vector<std::vector<int32_t>> Ucol(n);        // pivot steps, ascending
    s.P.assign(n, -1);
    s.pinv.assign(n, -1);
    std::vector<double> x(n, 0.0);
    std::vector<char> touched(n, 0);
    std::vector<int32_t> rows;
    std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> steps;
    std::vector<char> queued(n, 0);
    for (int32_t k = 0; k < n; ++k) {
        const int32_t col = s.Q[k];
        rows.clear();
        for (int64_t t = acp[col]; t < acp[col + 1]; ++t) {
            const int32_t i = arow[t];
            x[i] = (r[i] * values[apos[t]]) * c[col];
            touched[i] = 1;
            rows.push_back(i);
            const int32_t j = s.pinv[i];
            if (j >= 0 && !queued[j]) { queued[j] = 1; steps.push(j); }
        }
        while (!steps.empty()) {
            const int32_t j = steps.top();
            steps.pop();
            queued[j] = 0;
            Ucol[k].push_back(j);
            const double xj = x[s.P[j]];
            for (const auto &e : Lcol[j]) {
                const int32_t i = e.first;
                const double t = e.second * xj;
                x[i] = x[i] - t;
                if (!touched[i]) {
                    touched[i] = 1;
                    rows.push_back(i);
                    const int32_t jj = s.pinv[i];
                    if (jj >= 0 && !queued[jj]) { queued[jj] = 1; steps.push(jj); }
                }
            }
        }
        int32_t piv = -1;
        if (o.fixed_p) {
            piv = o.fixed_p[k];
            if (!touched[piv] || s.pinv[piv] >= 0) {
                for (int32_t i : rows) { touched[i] = 0; x[i] = 0.0; }
                return KKT_ERR_SINGULAR;
            }
        } else {
            double big = 0.0;
            bool diag_ok = false;
            for (int32_t i : rows) {
                if (s.pinv[i] >= 0) continue;
                big = std::max(big, std::fabs(x[i]));
                if (i == col) diag_ok = true;
            }
            if (!(big > 0.0)) {
                for (int32_t i : rows) { touched[i] = 0; x[i] = 0.0; }
                return KKT_ERR_SINGULAR;
            }
            if (diag_ok && x[col] != 0.0 && std::fabs(x[col]) >= o.pivot_tau * big) {
                piv = col;
            } else {
                for (int32_t i : rows)
                    if (s.pinv[i] < 0 && std::fabs(x[i]) == big && (piv < 0 || i < piv)) piv = i;
            }
        }
        s.P[k] = piv;
        s.pinv[piv] = k;
        const double ukk = x[piv];
        for (int32_t i : rows)
            if (s.pinv[i] < 0) Lcol[k].emplace_back(i, x[i] / ukk);
        for (int32_t i : rows) { touched[i] = 0; x[i] = 0.0; }
    }
    // canonical combined L+U, CSC in permuted space
    s.colptr.assign(n + 1, 0);
    s.ulen.resize(n);
    for (int32_t k = 0; k < n; ++k) {
        s.ulen[k] = (int32_t)Ucol[k].size();
        s.colptr[k + 1] = s.colptr[k] + (int64_t)Ucol[k].size() + 1 + (int64_t)Lcol[k].size();
    }
    s.rowidx.resize(s.colptr[n]);
    for (int32_t k = 0; k < n; ++k) {
        int64_t p = s.colptr[k];
        for (int32_t j : Ucol[k]) s.rowidx[p++] = j;
        s.rowidx[p++] = k;
        const int64_t l0 = p;
        for (const auto &e : Lcol[k]) s.rowidx[p++] = s.pinv[e.first];
        std::sort(s.rowidx.begin() + l0, s.rowidx.begin() + p);
        std::vector<int32_t>().swap(Ucol[k]);
        std::vector<std::pair<int32_t, double>>().swap(Lcol[k]);
    }
    // elimination tree (first L row below the diagonal) and the three level sets
    s.parent.assign(n, -1);
    s.lev_f.assign(n, 0);
    s.lev_l.assign(n, 0);
    s.lev_u.assign(n, 0);
    for (int32_t k = 0; k < n; ++k) {
        const int64_t d = s.colptr[k] + s.ulen[k];
        for (int64_t p = s.colptr[k]; p < d; ++p) s.lev_f[k] = std::max(s.lev_f[k], s.lev_f[s.rowidx[p]] + 1);
        if (d + 1 < s.colptr[k + 1]) s.parent[k] = s.rowidx[d + 1];
        for (int64_t p = d + 1; p < s.colptr[k + 1]; ++p)
            s.lev_l[s.rowidx[p]] = std::max(s.lev_l[s.rowidx[p]], s.lev_l[k] + 1);
    }
    for (int32_t k = n - 1; k >= 0; --k) {
        const int64_t d = s.colptr[k] + s.ulen[k];
        for (int64_t p = s.colptr[k]; p < d; ++p)
            s.lev_u[s.rowidx[p]] = std::max(s.lev_u[s.rowidx[p]], s.lev_u[k] + 1);
    }
    // structural supernodes.  Row structure of U: transpose of the strictly upper part.
    std::vector<int64_t> urp(n + 1, 0);
    for (int32_t k = 0; k < n; ++k)
        for (int64_t p = s.colptr[k]; p < s.colptr[k] + s.ulen[k]; ++p) urp[s.rowidx[p] + 1]++;
    for (int32_t i = 0; i < n; ++i) urp[i + 1] += urp[i];
    std::vector<int32_t> ucol(urp[n]);
    {
        std::vector<int64_t> nxt(urp.begin(), urp.end() - 1);
        for (int32_t k = 0; k < n; ++k)
            for (int64_t p = s.colptr[k]; p < s.colptr[k] + s.ulen[k]; ++p) ucol[nxt[s.rowidx[p]]++] = k;
    }
    s.sn_start.clear();
    s.sn_start.push_back(0);
    int32_t width = 1;
    for (int32_t j = 1; j < n; ++j) {
        bool join = width < o.sn_max_width;
        // L part of column j-1 must start with row j and continue exactly as column j's L part
        const int64_t lprev = s.colptr[j - 1] + s.ulen[j - 1] + 1, lprev_end = s.colptr[j];
        const int64_t lcur = s.colptr[j] + s.ulen[j] + 1, lcur_end = s.colptr[j + 1];
        if (join) join = (lprev < lprev_end && s.rowidx[lprev] == j) &&
                         (lprev_end - lprev - 1 == lcur_end - lcur) &&
                         std::equal(s.rowidx.begin() + lprev + 1, s.rowidx.begin() + lprev_end,
                                    s.rowidx.begin() + lcur);
        // U row j-1 must start with column j and continue exactly as U row j
        if (join) join = (urp[j] > urp[j - 1] && ucol[urp[j - 1]] == j) &&
                         (urp[j] - urp[j - 1] - 1 == urp[j + 1] - urp[j]) &&
                         std::equal(ucol.begin() + urp[j - 1] + 1, ucol.begin() + urp[j],
                                    ucol.begin() + urp[j]);
        if (join) {
            ++width;
        } else {
            s.sn_start.push_back(j);
            width = 1;
        }
    }
    s.sn_start.push_back(n);
    // scatter map: entry (i, j) of A lands at row pinv[i] of column qinv[j]
    s.map.resize(nnz);
    for (int32_t i = 0; i < n; ++i)
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const int32_t pr = s.pinv[i], pc = s.qinv[colind[p]];
            const auto b = s.rowidx.begin() + s.colptr[pc], e = s.rowidx.begin() + s.colptr[pc + 1];
            const auto it = std::lower_bound(b, e, pr);
            if (it == e || *it != pr) return KKT_ERR_PATTERN;   // impossible by construction
            s.map[p] = it - s.rowidx.begin();
        }
    return KKT_OK;
}

}  // namespace kkt
