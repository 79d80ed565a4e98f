// CDNA4 (gfx950) kernels of the KKT refactorization library.
//
// Value update (Algorithm 1, update the factor object with the new values): power-of-two
// row/column equilibration (the analysis stage equilibrates, Section II) and a gather of
// the scaled values into the combined L+U storage.
// Refactorization (Algorithm 1, refactor without pivoting): one launch per panel level;
// see kkt_schedule.cpp for the schedule.  Each work item is one 64-lane wavefront.
// Triangular solves (Algorithm 1, triangular solve) on a row-ordered copy of L+U, one
// launch per panel level; residuals and Krylov vector work for the refinement.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kkt_kernels.h"

namespace kkt {

__device__ __forceinline__ double bcast(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double inv_pow2_floor_log2(double m) {
    if (!(m > 0.0)) return 1.0;
    int e = ilogb(m);
    e = e > 1020 ? 1020 : (e < -1020 ? -1020 : e);
    return ldexp(1.0, -e);
}

// max of non-negative doubles through their ordered bit patterns
__device__ __forceinline__ void atomic_max_pos(double *addr, double v) {
    atomicMax(reinterpret_cast<unsigned long long *>(addr), (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ double group_sum(double v, int width) {
    for (int o = width / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
    return v;
}

// ---------------------------------------------------------------------------------------
// value update

__global__ void k_row_scale(int n, const int32_t *__restrict__ rowptr, const double *__restrict__ v,
                            int scale, double *__restrict__ r, DevStatus *st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        st->anorm_scaled = 0.0;
        st->anorm = 0.0;
        st->perturbed = 0;
        st->flags = 0;
    }
    if (i >= n) return;
    double m = 0.0;
    int bad = 0;
    for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        const double a = fabs(v[p]);
        bad |= !isfinite(a);
        m = fmax(m, a);
    }
    if (bad) atomicOr(&st->flags, kFlagNonfinite);
    r[i] = scale ? inv_pow2_floor_log2(m) : 1.0;
}

__global__ void k_col_scale(int n, const int32_t *__restrict__ cptr, const int32_t *__restrict__ cpos,
                            const int32_t *__restrict__ rowid, const double *__restrict__ v,
                            const double *__restrict__ r, int scale, double *__restrict__ c) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double m = 0.0;
    for (int t = cptr[j]; t < cptr[j + 1]; ++t) {
        const int p = cpos[t];
        m = fmax(m, fabs(r[rowid[p]] * v[p]));
    }
    c[j] = scale ? inv_pow2_floor_log2(m) : 1.0;
}

// ||A||_inf and ||R A C||_inf (row sums in CSR order)
__global__ void k_norms(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                        const double *__restrict__ v, const double *__restrict__ r,
                        const double *__restrict__ c, DevStatus *st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0, a = 0.0;
    if (i < n) {
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            a = a + fabs(v[p]);
            s = s + fabs((r[i] * v[p]) * c[col[p]]);
        }
    }
    // block max, then one atomic per block
    for (int o = 32; o > 0; o >>= 1) {
        s = fmax(s, __shfl_xor(s, o));
        a = fmax(a, __shfl_xor(a, o));
    }
    if ((threadIdx.x & 63) == 0) {
        atomic_max_pos(&st->anorm_scaled, s);
        atomic_max_pos(&st->anorm, a);
    }
}

__global__ void k_gather_lu(int64_t nlu, const int32_t *__restrict__ src, const int32_t *__restrict__ rowid,
                            const int32_t *__restrict__ col, const double *__restrict__ v,
                            const double *__restrict__ r, const double *__restrict__ c,
                            double *__restrict__ lu) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nlu) return;
    const int e = src[p];
    lu[p] = e < 0 ? 0.0 : (r[rowid[e]] * v[e]) * c[col[e]];
}

__global__ void k_to_csr(int64_t nlu, const int32_t *__restrict__ csr_src, const double *__restrict__ lu,
                         double *__restrict__ lucsr) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nlu) lucsr[q] = lu[csr_src[q]];
}

// ---------------------------------------------------------------------------------------
// refactorization

// first index in [lo, hi) whose row >= key
__device__ __forceinline__ int lower_bound_row(const int32_t *__restrict__ rowidx, int lo, int hi, int key) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rowidx[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

struct RefArgs {
    const int32_t *colptr, *rowidx, *ulen, *pan_start, *pan_r;
    const int32_t *item_panel, *item_tgt, *tgt_col, *tgt_src, *src_panel;
    double *lu;
    DevStatus *st;
    double tiny;
};

// Update of target column k by source panel S: rows s..e-1 of column k become final U
// entries (unit lower solve with S's diagonal block), rows R of S lose L(R, S) times them.
__device__ void pull_update(const RefArgs &a, int k, int S, int lane) {
    const int s = a.pan_start[S], e = a.pan_start[S + 1], w = e - s, r = a.pan_r[S];
    const int c0 = a.colptr[k], c1 = a.colptr[k + 1];
    const int ps = lower_bound_row(a.rowidx, c0, c0 + a.ulen[k], s);
    double u = lane < w ? a.lu[ps + lane] : 0.0;
    for (int j = 0; j + 1 < w; ++j) {
        const double uj = bcast(u, j);
        if (lane > j && lane < w) {
            const int lb = a.colptr[s + j] + a.ulen[s + j] + 1;
            u = fma(-a.lu[lb + (lane - j - 1)], uj, u);
        }
    }
    if (lane < w) a.lu[ps + lane] = u;
    const int r0 = a.colptr[e - 1] + a.ulen[e - 1] + 1;   // rows R in the last column
    for (int i = lane; i < r; i += 64) {
        double acc = 0.0;
        for (int j = 0; j < w; ++j) {
            const int lb = a.colptr[s + j] + a.ulen[s + j] + 1 + (w - 1 - j);
            acc = fma(a.lu[lb + i], bcast(u, j), acc);
        }
        const int row = a.rowidx[r0 + i];
        const int pos = lower_bound_row(a.rowidx, ps + w, c1, row);
        if (pos < c1 && a.rowidx[pos] == row) a.lu[pos] -= acc;
        else atomicOr(&a.st->flags, kFlagInternal);   // the fill pattern guarantees a slot
    }
    // rows of a later source may lie in R: make this update visible to the whole wave
    __threadfence_block();
    __syncthreads();
}

// Dense LU without pivoting of the block column of panel T (diagonal block + rows R).
__device__ void factor_panel(const RefArgs &a, int T, int lane, double *sm) {
    const int s = a.pan_start[T], e = a.pan_start[T + 1], w = e - s, r = a.pan_r[T];
    const double thresh = a.tiny * a.st->anorm_scaled;
    double *D = sm;                    // w x w, column-major
    double *X = sm + kPanelMax * kPanelMax;   // w x 64, one row of R per lane
    for (int jj = 0; jj < w; ++jj) {
        const int seg = a.colptr[s + jj] + a.ulen[s + jj] - jj;
        for (int ii = lane; ii < w; ii += 64) D[jj * w + ii] = a.lu[seg + ii];
    }
    __syncthreads();
    int bad = 0, npert = 0;
    for (int jj = 0; jj < w; ++jj) {
        double p = D[jj * w + jj];
        bad |= !isfinite(p);
        if (fabs(p) < thresh) {
            p = p < 0.0 ? -thresh : thresh;
            ++npert;
        }
        __syncthreads();
        if (lane == 0) D[jj * w + jj] = p;
        for (int ii = jj + 1 + lane; ii < w; ii += 64) D[jj * w + ii] = D[jj * w + ii] / p;
        __syncthreads();
        const int m = w - jj - 1;
        for (int t = lane; t < m * m; t += 64) {
            const int c2 = jj + 1 + t / m, ii = jj + 1 + t % m;
            D[c2 * w + ii] = fma(-D[jj * w + ii], D[c2 * w + jj], D[c2 * w + ii]);
        }
        __syncthreads();
    }
    for (int jj = 0; jj < w; ++jj) {
        const int seg = a.colptr[s + jj] + a.ulen[s + jj] - jj;
        for (int ii = lane; ii < w; ii += 64) a.lu[seg + ii] = D[jj * w + ii];
    }
    for (int i0 = 0; i0 < r; i0 += 64) {
        const int i = i0 + lane;
        if (i < r) {
            for (int jj = 0; jj < w; ++jj) {
                const int seg = a.colptr[s + jj] + a.ulen[s + jj] - jj;
                X[jj * 64 + lane] = a.lu[seg + w + i];
            }
            for (int jj = 0; jj < w; ++jj) {
                const double v = X[jj * 64 + lane] / D[jj * w + jj];
                bad |= !isfinite(v);
                X[jj * 64 + lane] = v;
                for (int c2 = jj + 1; c2 < w; ++c2) X[c2 * 64 + lane] = fma(-v, D[c2 * w + jj], X[c2 * 64 + lane]);
            }
            for (int jj = 0; jj < w; ++jj) {
                const int seg = a.colptr[s + jj] + a.ulen[s + jj] - jj;
                a.lu[seg + w + i] = X[jj * 64 + lane];
            }
        }
    }
    if (lane == 0 && npert) atomicAdd(&a.st->perturbed, (unsigned long long)npert);
    if (__any(bad) && lane == 0) atomicOr(&a.st->flags, kFlagNonfinite);
}

__global__ __launch_bounds__(64) void k_refactor_level(int item0, RefArgs a) {
    __shared__ double sm[kPanelMax * kPanelMax + kPanelMax * 64];
    const int item = item0 + blockIdx.x;
    const int lane = threadIdx.x;
    for (int t = a.item_tgt[item]; t < a.item_tgt[item + 1]; ++t) {
        const int k = a.tgt_col[t];
        for (int q = a.tgt_src[t]; q < a.tgt_src[t + 1]; ++q) pull_update(a, k, a.src_panel[q], lane);
    }
    const int T = a.item_panel[item];
    if (T >= 0) factor_panel(a, T, lane, sm);
}

// ---------------------------------------------------------------------------------------
// triangular solves, one wavefront per item

struct SolveArgs {
    const int32_t *pan_start, *item_p0, *item_np, *pan;
    const int32_t *rowptr, *col, *diag, *P, *Q;
    const double *lucsr, *r, *c;
    const double *b;      // forward: right-hand side (original order)
    double *y;            // forward output / backward input (permuted)
    double *xt;           // backward output (permuted)
    double *x;            // backward output (original order)
};

__global__ __launch_bounds__(64) void k_lsolve_level(int item0, SolveArgs a) {
    __shared__ double ext[kPanelMax];
    const int item = item0 + blockIdx.x, lane = threadIdx.x;
    const int np = a.item_np[item], p0 = a.item_p0[item];
    const int g = lane >> 3, gl = lane & 7;
    if (np < 0) {                                    // pack of width-1 panels
        double acc = 0.0;
        int i = -1;
        if (g < -np) {
            i = a.pan_start[a.pan[p0 + g]];
            for (int q = a.rowptr[i] + gl; q < a.diag[i]; q += 8) acc = fma(a.lucsr[q], a.y[a.col[q]], acc);
        }
        acc = group_sum(acc, 8);
        if (i >= 0 && gl == 0) a.y[i] = a.r[a.P[i]] * a.b[a.P[i]] - acc;
        return;
    }
    const int T = a.pan[p0];
    const int s = a.pan_start[T], w = a.pan_start[T + 1] - s;
    for (int t0 = 0; t0 < w; t0 += 8) {
        const int t = t0 + g;
        double acc = 0.0;
        if (t < w) {
            const int i = s + t;
            for (int q = a.rowptr[i] + gl; q < a.diag[i] - t; q += 8) acc = fma(a.lucsr[q], a.y[a.col[q]], acc);
        }
        acc = group_sum(acc, 8);
        if (t < w && gl == 0) ext[t] = acc;
    }
    __syncthreads();
    double yv = 0.0;
    if (lane < w) yv = a.r[a.P[s + lane]] * a.b[a.P[s + lane]] - ext[lane];
    for (int t = 0; t + 1 < w; ++t) {
        const double yt = bcast(yv, t);
        if (lane > t && lane < w) yv = fma(-a.lucsr[a.diag[s + lane] - (lane - t)], yt, yv);
    }
    if (lane < w) a.y[s + lane] = yv;
}

__global__ __launch_bounds__(64) void k_usolve_level(int item0, SolveArgs a) {
    __shared__ double ext[kPanelMax];
    const int item = item0 + blockIdx.x, lane = threadIdx.x;
    const int np = a.item_np[item], p0 = a.item_p0[item];
    const int g = lane >> 3, gl = lane & 7;
    if (np < 0) {
        double acc = 0.0;
        int i = -1;
        if (g < -np) {
            i = a.pan_start[a.pan[p0 + g]];
            for (int q = a.diag[i] + 1 + gl; q < a.rowptr[i + 1]; q += 8) acc = fma(a.lucsr[q], a.xt[a.col[q]], acc);
        }
        acc = group_sum(acc, 8);
        if (i >= 0 && gl == 0) {
            const double xv = (a.y[i] - acc) / a.lucsr[a.diag[i]];
            a.xt[i] = xv;
            a.x[a.Q[i]] = a.c[a.Q[i]] * xv;
        }
        return;
    }
    const int T = a.pan[p0];
    const int s = a.pan_start[T], w = a.pan_start[T + 1] - s;
    for (int t0 = 0; t0 < w; t0 += 8) {
        const int t = t0 + g;
        double acc = 0.0;
        if (t < w) {
            const int i = s + t;
            for (int q = a.diag[i] + (w - t) + gl; q < a.rowptr[i + 1]; q += 8) acc = fma(a.lucsr[q], a.xt[a.col[q]], acc);
        }
        acc = group_sum(acc, 8);
        if (t < w && gl == 0) ext[t] = acc;
    }
    __syncthreads();
    double val = 0.0, xv = 0.0;
    if (lane < w) val = a.y[s + lane] - ext[lane];
    for (int t = w - 1; t >= 0; --t) {
        if (lane == t) xv = val / a.lucsr[a.diag[s + t]];
        const double xt = bcast(xv, t);
        if (lane < t) val = fma(-a.lucsr[a.diag[s + lane] + (t - lane)], xt, val);
    }
    if (lane < w) {
        a.xt[s + lane] = xv;
        a.x[a.Q[s + lane]] = a.c[a.Q[s + lane]] * xv;
    }
}

// ---------------------------------------------------------------------------------------
// residual, sparse products and Krylov vector kernels (FP64)

__global__ void k_reset_norms(DevStatus *st) {
    st->rnorm = 0.0;
    st->xnorm = 0.0;
    st->bnorm = 0.0;
}

// res = b - A x with infinity norms of res, x and b (8 lanes per row)
__global__ void k_residual(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                           const double *__restrict__ v, const double *__restrict__ x,
                           const double *__restrict__ b, double *__restrict__ res, DevStatus *st) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gid >> 3, gl = gid & 7;
    double s = 0.0;
    if (i < n)
        for (int p = rowptr[i] + gl; p < rowptr[i + 1]; p += 8) s = fma(v[p], x[col[p]], s);
    s = group_sum(s, 8);
    double rn = 0.0, xn = 0.0, bn = 0.0;
    if (i < n && gl == 0) {
        const double ri = b[i] - s;
        res[i] = ri;
        rn = isnan(ri) ? __longlong_as_double(0x7ff8000000000000LL) : fabs(ri);
        xn = isnan(x[i]) ? __longlong_as_double(0x7ff8000000000000LL) : fabs(x[i]);
        bn = fabs(b[i]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        rn = fmax(rn, __shfl_xor(rn, o));
        xn = fmax(xn, __shfl_xor(xn, o));
        bn = fmax(bn, __shfl_xor(bn, o));
    }
    if ((threadIdx.x & 63) == 0) {
        atomic_max_pos(&st->rnorm, rn);
        atomic_max_pos(&st->xnorm, xn);
        atomic_max_pos(&st->bnorm, bn);
    }
}

__global__ void k_spmv(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                       const double *__restrict__ v, const double *__restrict__ x, double *__restrict__ y) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gid >> 3, gl = gid & 7;
    double s = 0.0;
    if (i < n)
        for (int p = rowptr[i] + gl; p < rowptr[i + 1]; p += 8) s = fma(v[p], x[col[p]], s);
    s = group_sum(s, 8);
    if (i < n && gl == 0) y[i] = s;
}

// part[i * nblk + blockIdx.x] = partial dot of V_i with w (fixed order)
__global__ __launch_bounds__(256) void k_multidot(int n, int nv, const double *__restrict__ V, int64_t ldv,
                                                  const double *__restrict__ w, double *__restrict__ part) {
    __shared__ double red[4];
    for (int i = 0; i < nv; ++i) {
        const double *vi = V + (int64_t)i * ldv;
        double s = 0.0;
        for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x)
            s = fma(vi[q], w[q], s);
        s = group_sum(s, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) part[i * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
    }
}

// out[i] = (accumulate ? out[i] : 0) + sum_b part[i * nblk + b]
__global__ __launch_bounds__(256) void k_reduce_parts(int nv, int nblk, const double *__restrict__ part,
                                                      double *__restrict__ out, int accumulate) {
    __shared__ double red[4];
    const int i = blockIdx.x;
    if (i >= nv) return;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += part[i * nblk + b];
    s = group_sum(s, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = (red[0] + red[1]) + (red[2] + red[3]);
        out[i] = accumulate ? out[i] + t : t;
    }
}

// w -= sum_i h[i] V_i
__global__ void k_sub_combo(int n, int nv, const double *__restrict__ V, int64_t ldv,
                            const double *__restrict__ h, double *__restrict__ w) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double s = w[q];
    for (int i = 0; i < nv; ++i) s = fma(-h[i], V[(int64_t)i * ldv + q], s);
    w[q] = s;
}

// x += sum_i y[i] Z_i
__global__ void k_add_combo(int n, int nv, const double *__restrict__ Z, int64_t ldz,
                            const double *__restrict__ y, double *__restrict__ x) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double s = x[q];
    for (int i = 0; i < nv; ++i) s = fma(y[i], Z[(int64_t)i * ldz + q], s);
    x[q] = s;
}

// dst = src / sqrt(*nrm2)   (nrm2 holds a squared norm; zero leaves dst = 0)
__global__ void k_scale_by_norm(int n, const double *__restrict__ src, const double *__restrict__ nrm2,
                                double *__restrict__ dst) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const double t = sqrt(*nrm2);
    if (q < n) dst[q] = t > 0.0 ? src[q] / t : 0.0;
}

}  // namespace kkt
