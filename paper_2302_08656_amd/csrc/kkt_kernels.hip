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

// ||A||_inf and ||R A C||_inf (row sums in CSR order): block maxima into part[2 * block]
__global__ __launch_bounds__(256) void k_norms(int n, const int32_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ col, const double *__restrict__ v,
                                               const double *__restrict__ r, const double *__restrict__ c,
                                               double *__restrict__ part) {
    __shared__ double red[2][4];
    double s = 0.0, a = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double si = 0.0, ai = 0.0;
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            ai = ai + fabs(v[p]);
            si = si + fabs((r[i] * v[p]) * c[col[p]]);
        }
        s = fmax(s, si);
        a = fmax(a, ai);
    }
    for (int o = 32; o > 0; o >>= 1) {
        s = fmax(s, __shfl_xor(s, o));
        a = fmax(a, __shfl_xor(a, o));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s;
        red[1][threadIdx.x >> 6] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
        part[2 * blockIdx.x + 1] = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
    }
}

// dst[j] = max over blocks b of part[nfield * b + j] (NaN propagates), j < nfield
__global__ __launch_bounds__(256) void k_max_parts(int nblk, int nfield, const double *__restrict__ part,
                                                   double *__restrict__ dst) {
    __shared__ double red[4];
    for (int j = 0; j < nfield; ++j) {
        double m = 0.0;
        for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
            const double x = part[nfield * b + j];
            m = (isnan(x) || isnan(m)) ? x + m : fmax(m, x);
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double y = __shfl_xor(m, o);
            m = (isnan(y) || isnan(m)) ? y + m : fmax(m, y);
        }
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = red[0];
            for (int q = 1; q < 4; ++q) t = (isnan(t) || isnan(red[q])) ? t + red[q] : fmax(t, red[q]);
            dst[j] = t;
        }
        __syncthreads();
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
    const int32_t *item_panel, *item_pair, *pair_src, *pair_tgt;
    double *lu;
    DevStatus *st;
    double tiny;
};

// position of the first L entry (row j+1 or below) of column j
__device__ __forceinline__ int lbeg(const RefArgs &a, int j) { return a.colptr[j] + a.ulen[j] + 1; }
// position of row s (the panel's first row) in column j of a panel starting at s
__device__ __forceinline__ int seg(const RefArgs &a, int j, int jj) { return a.colptr[j] + a.ulen[j] - jj; }

__device__ __forceinline__ double perturb(double p, double thresh, int &npert) {
    if (fabs(p) < thresh) {
        ++npert;
        return p < 0.0 ? -thresh : thresh;
    }
    return p;
}

// ----------------------------------------------------------------- 16-lane path

// Update of target column k by a narrow source panel S (w <= kSmallW, r <= kSmallR): rows
// s..e-1 of column k become final U entries (unit lower solve with S's diagonal block) and
// the rows R of S lose L(R, S) times them.
__device__ void small_pull(const RefArgs &a, int k, int S, int gl) {
    const int s = a.pan_start[S], e = a.pan_start[S + 1], w = e - s, r = a.pan_r[S];
    const int c0 = a.colptr[k], c1 = a.colptr[k + 1];
    const int ps = lower_bound_row(a.rowidx, c0, c0 + a.ulen[k], s);
    double u = gl < w ? a.lu[ps + gl] : 0.0;
#pragma unroll
    for (int j = 0; j < kSmallW - 1; ++j) {
        const double uj = __shfl(u, j, 16);
        if (j + 1 < w && gl > j && gl < w) u = fma(-a.lu[lbeg(a, s + j) + (gl - j - 1)], uj, u);
    }
    if (gl < w) a.lu[ps + gl] = u;
    double uu[kSmallW];
    int lb[kSmallW];
#pragma unroll
    for (int j = 0; j < kSmallW; ++j) {
        uu[j] = __shfl(u, j, 16);
        lb[j] = j < w ? lbeg(a, s + j) + (w - 1 - j) : 0;
    }
    const int r0 = lbeg(a, e - 1);
    for (int i = gl; i < r; i += 16) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < kSmallW; ++j)
            if (j < w) acc = fma(a.lu[lb[j] + i], uu[j], acc);
        const int row = a.rowidx[r0 + i];
        const int pos = lower_bound_row(a.rowidx, ps + w, c1, row);
        if (pos < c1 && a.rowidx[pos] == row) a.lu[pos] -= acc;
        else atomicOr(&a.st->flags, kFlagInternal);   // the fill pattern guarantees a slot
    }
    __threadfence_block();   // a later source of the same column may read these rows
}

// Dense LU without pivoting of a narrow panel's block column (w <= kSmallW, r <= kSmallR).
// Returns the number of replaced pivots (the same value on every lane of the group).
__device__ int small_factor(const RefArgs &a, int T, int gl, double thresh) {
    const int s = a.pan_start[T], e = a.pan_start[T + 1], w = e - s, r = a.pan_r[T];
    int sg[kSmallW];
    double d[kSmallW];          // lane gl < w: row gl of the diagonal block
#pragma unroll
    for (int c = 0; c < kSmallW; ++c) {
        sg[c] = c < w ? seg(a, s + c, c) : 0;
        d[c] = (c < w && gl < w) ? a.lu[sg[c] + gl] : 0.0;
    }
    int npert = 0, bad = 0;
    double U[kSmallW][kSmallW];   // final U of the diagonal block, known to every lane
#pragma unroll
    for (int jj = 0; jj < kSmallW; ++jj) {
        if (jj < w) {
            double ur[kSmallW];
#pragma unroll
            for (int c = 0; c < kSmallW; ++c) ur[c] = __shfl(d[c], jj, 16);
            const double p = perturb(ur[jj], thresh, npert);
            bad |= !isfinite(p);
            if (gl == jj) d[jj] = p;
            ur[jj] = p;
#pragma unroll
            for (int c = 0; c < kSmallW; ++c) U[jj][c] = ur[c];
            if (gl > jj && gl < w) {
                const double l = d[jj] / p;
                d[jj] = l;
#pragma unroll
                for (int c = jj + 1; c < kSmallW; ++c)
                    if (c < w) d[c] = fma(-l, ur[c], d[c]);
            }
        }
    }
    if (gl < w) {
#pragma unroll
        for (int c = 0; c < kSmallW; ++c)
            if (c < w) a.lu[sg[c] + gl] = d[c];
    }
    for (int i = gl; i < r; i += 16) {
        double x[kSmallW];
#pragma unroll
        for (int c = 0; c < kSmallW; ++c) x[c] = c < w ? a.lu[sg[c] + w + i] : 0.0;
#pragma unroll
        for (int jj = 0; jj < kSmallW; ++jj) {
            if (jj < w) {
                const double l = x[jj] / U[jj][jj];
                bad |= !isfinite(l);
                x[jj] = l;
#pragma unroll
                for (int c = jj + 1; c < kSmallW; ++c)
                    if (c < w) x[c] = fma(-l, U[jj][c], x[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < kSmallW; ++c)
            if (c < w) a.lu[sg[c] + w + i] = x[c];
    }
    if (bad) atomicOr(&a.st->flags, kFlagNonfinite);
    return npert;
}

// ----------------------------------------------------------------- 256-thread path

constexpr int kLargeThreads = 256;
constexpr int kRChunk = 128;
constexpr int kColCache = 768;     // keeps the block under 64 KiB of LDS
// LDS layout (bytes): Ld | Ub | Lr | Rrow | psbuf | column-row cache per wave
constexpr int kOffLd = 0;
constexpr int kOffUb = kOffLd + kPanelMax * kPanelMax * 8;
constexpr int kOffLr = kOffUb + kPanelMax * kGroup * 8;
constexpr int kOffRrow = kOffLr + kRChunk * kPanelMax * 8;
constexpr int kOffPs = kOffRrow + kRChunk * 4;
constexpr int kOffCol = kOffPs + kGroup * 4;
constexpr int kLargeLds = kOffCol + (kLargeThreads / 64) * kColCache * 4;

__device__ void large_factor(const RefArgs &a, int T, char *sm, double thresh) {
    const int tid = threadIdx.x;
    const int s = a.pan_start[T], e = a.pan_start[T + 1], w = e - s, r = a.pan_r[T];
    double *D = reinterpret_cast<double *>(sm + kOffLd);   // column-major, ld kPanelMax
    double *X = reinterpret_cast<double *>(sm + kOffLr);   // kRChunk rows x w, column-major
    for (int t = tid; t < w * w; t += kLargeThreads) {
        const int jj = t / w, ii = t % w;
        D[jj * kPanelMax + ii] = a.lu[seg(a, s + jj, jj) + ii];
    }
    __syncthreads();
    int npert = 0, bad = 0;
    for (int jj = 0; jj < w; ++jj) {
        const double p = perturb(D[jj * kPanelMax + jj], thresh, npert);
        bad |= !isfinite(p);
        __syncthreads();
        if (tid == 0) D[jj * kPanelMax + jj] = p;
        for (int ii = jj + 1 + tid; ii < w; ii += kLargeThreads) D[jj * kPanelMax + ii] /= p;
        __syncthreads();
        const int m = w - jj - 1;
        for (int t = tid; t < m * m; t += kLargeThreads) {
            const int c2 = jj + 1 + t / m, ii = jj + 1 + t % m;
            D[c2 * kPanelMax + ii] = fma(-D[jj * kPanelMax + ii], D[c2 * kPanelMax + jj], D[c2 * kPanelMax + ii]);
        }
        __syncthreads();
    }
    for (int t = tid; t < w * w; t += kLargeThreads) {
        const int jj = t / w, ii = t % w;
        a.lu[seg(a, s + jj, jj) + ii] = D[jj * kPanelMax + ii];
    }
    for (int i0 = 0; i0 < r; i0 += kRChunk) {
        const int nr = min(kRChunk, r - i0);
        for (int t = tid; t < w * nr; t += kLargeThreads) {
            const int jj = t / nr, i = t % nr;
            X[jj * kRChunk + i] = a.lu[seg(a, s + jj, jj) + w + i0 + i];
        }
        __syncthreads();
        if (tid < nr) {
            for (int jj = 0; jj < w; ++jj) {
                const double l = X[jj * kRChunk + tid] / D[jj * kPanelMax + jj];
                bad |= !isfinite(l);
                X[jj * kRChunk + tid] = l;
                for (int c2 = jj + 1; c2 < w; ++c2)
                    X[c2 * kRChunk + tid] = fma(-l, D[c2 * kPanelMax + jj], X[c2 * kRChunk + tid]);
            }
        }
        __syncthreads();
        for (int t = tid; t < w * nr; t += kLargeThreads) {
            const int jj = t / nr, i = t % nr;
            a.lu[seg(a, s + jj, jj) + w + i0 + i] = X[jj * kRChunk + i];
        }
        __syncthreads();
    }
    if (tid == 0 && npert) atomicAdd(&a.st->perturbed, (unsigned long long)npert);
    if (__any(bad) && (tid & 63) == 0) atomicOr(&a.st->flags, kFlagNonfinite);
}

// All pulls of one item with the source panel staged in LDS, then the panel factorization.
__device__ void large_item(const RefArgs &a, int item, char *sm, double thresh) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double *Ld = reinterpret_cast<double *>(sm + kOffLd);
    double *Ub = reinterpret_cast<double *>(sm + kOffUb);
    double *Lr = reinterpret_cast<double *>(sm + kOffLr);
    int *Rrow = reinterpret_cast<int *>(sm + kOffRrow);
    int *psb = reinterpret_cast<int *>(sm + kOffPs);
    int *colc = reinterpret_cast<int *>(sm + kOffCol) + wv * kColCache;
    const int p1 = a.item_pair[item + 1];
    for (int g0 = a.item_pair[item], g1; g0 < p1; g0 = g1) {
        const int S = a.pair_src[g0];
        g1 = g0 + 1;
        while (g1 < p1 && a.pair_src[g1] == S) ++g1;
        const int s = a.pan_start[S], e = a.pan_start[S + 1], w = e - s, r = a.pan_r[S];
        for (int t = tid; t < w * w; t += kLargeThreads) {
            const int j = t / w, i = t % w;
            if (i > j) Ld[j * kPanelMax + i] = a.lu[lbeg(a, s + j) + (i - j - 1)];
        }
        __syncthreads();
        for (int q = g0 + wv; q < g1; q += kLargeThreads / 64) {
            const int k = a.pair_tgt[q];
            const int c0 = a.colptr[k];
            const int ps = lower_bound_row(a.rowidx, c0, c0 + a.ulen[k], s);
            double u = lane < w ? a.lu[ps + lane] : 0.0;
            for (int j = 0; j + 1 < w; ++j) {
                const double uj = bcast(u, j);
                if (lane > j && lane < w) u = fma(-Ld[j * kPanelMax + lane], uj, u);
            }
            if (lane < w) {
                a.lu[ps + lane] = u;
                Ub[(q - g0) * kPanelMax + lane] = u;
            }
            if (lane == 0) psb[q - g0] = ps;
        }
        __syncthreads();
        const int r0 = lbeg(a, e - 1);
        for (int i0 = 0; i0 < r; i0 += kRChunk) {
            const int nr = min(kRChunk, r - i0);
            for (int t = tid; t < w * nr; t += kLargeThreads) {
                const int j = t / nr, i = t % nr;
                Lr[j * kRChunk + i] = a.lu[lbeg(a, s + j) + (w - 1 - j) + i0 + i];
            }
            for (int i = tid; i < nr; i += kLargeThreads) Rrow[i] = a.rowidx[r0 + i0 + i];
            __syncthreads();
            for (int q = g0 + wv; q < g1; q += kLargeThreads / 64) {
                const int k = a.pair_tgt[q];
                const int lo = psb[q - g0] + w, hi = a.colptr[k + 1];
                const bool cached = hi - lo <= kColCache;
                if (cached)
                    for (int t = lane; t < hi - lo; t += 64) colc[t] = a.rowidx[lo + t];
                __threadfence_block();
                const double *ub = Ub + (q - g0) * kPanelMax;
                for (int i = lane; i < nr; i += 64) {
                    double acc = 0.0;
                    for (int j = 0; j < w; ++j) acc = fma(Lr[j * kRChunk + i], ub[j], acc);
                    const int row = Rrow[i];
                    int pos;
                    if (cached) {
                        int l2 = 0, h2 = hi - lo;
                        while (l2 < h2) {
                            const int mid = (l2 + h2) >> 1;
                            if (colc[mid] < row) l2 = mid + 1;
                            else h2 = mid;
                        }
                        pos = lo + l2;
                    } else {
                        pos = lower_bound_row(a.rowidx, lo, hi, row);
                    }
                    if (pos < hi && a.rowidx[pos] == row) a.lu[pos] -= acc;
                    else atomicOr(&a.st->flags, kFlagInternal);
                }
                __threadfence_block();
            }
            __syncthreads();
        }
        __threadfence_block();
        __syncthreads();
    }
    const int T = a.item_panel[item];
    if (T >= 0) large_factor(a, T, sm, thresh);
}

// One launch per panel level: blocks [0, nlarge) take one large item each, the remaining
// blocks take kLargeThreads/16 small items each (one per 16-lane group).
__global__ __launch_bounds__(256) void k_refactor_level(int item0, int nlarge, int nsmall, RefArgs a) {
    extern __shared__ __align__(16) char dsm[];
    const double thresh = a.tiny * a.st->anorm_scaled;
    if ((int)blockIdx.x < nlarge) {
        large_item(a, item0 + blockIdx.x, dsm, thresh);
        return;
    }
    const int g = (blockIdx.x - nlarge) * (kLargeThreads / 16) + (threadIdx.x >> 4);
    const int gl = threadIdx.x & 15;
    int npert = 0;
    if (g < nsmall) {
        const int item = item0 + nlarge + g;
        for (int q = a.item_pair[item]; q < a.item_pair[item + 1]; ++q)
            small_pull(a, a.pair_tgt[q], a.pair_src[q], gl);
        const int T = a.item_panel[item];
        if (T >= 0) npert = small_factor(a, T, gl, thresh);
    }
    // one counter update per wavefront: group leaders contribute their count
    int c = gl == 0 ? npert : 0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(&a.st->perturbed, (unsigned long long)c);
}

// ---------------------------------------------------------------------------------------
// triangular solves: one 256-thread block per wide panel or per pack of kSolvePack
// width-1 panels (8 lanes per row)

struct SolveArgs {
    const int32_t *pan_start, *item_p0, *item_np, *pan;
    const int32_t *rowptr, *col, *diag, *P, *Q;
    const double *lucsr, *r, *c;
    const double *b;      // forward: right-hand side (original order)
    double *y;            // forward output / backward input (permuted)
    double *xt;           // backward output (permuted)
    double *x;            // backward output (original order)
};

// sum over q in [q0, q1) of lucsr[q] * v[col[q]] on a group of `width` lanes
__device__ __forceinline__ double row_dot(const SolveArgs &a, const double *v, int q0, int q1, int gl, int width) {
    double s0 = 0.0, s1 = 0.0;
    int q = q0 + gl;
    for (; q + width < q1; q += 2 * width) {
        s0 = fma(a.lucsr[q], v[a.col[q]], s0);
        s1 = fma(a.lucsr[q + width], v[a.col[q + width]], s1);
    }
    if (q < q1) s0 = fma(a.lucsr[q], v[a.col[q]], s0);
    return group_sum(s0 + s1, width);
}

__global__ __launch_bounds__(256) void k_lsolve_level(int item0, SolveArgs a) {
    __shared__ double ext[kPanelMax];
    const int item = item0 + blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const int np = a.item_np[item], p0 = a.item_p0[item];
    if (np < 0) {                                    // pack of width-1 panels, 8 lanes each
        const int g = tid >> 3, gl = tid & 7;
        int i = -1, q0 = 0, q1 = 0;
        if (g < -np) {
            i = a.pan_start[a.pan[p0 + g]];
            q0 = a.rowptr[i];
            q1 = a.diag[i];
        }
        const double acc = row_dot(a, a.y, q0, q1, gl, 8);
        if (i >= 0 && gl == 0) a.y[i] = a.r[a.P[i]] * a.b[a.P[i]] - acc;
        return;
    }
    const int T = a.pan[p0];
    const int s = a.pan_start[T], w = a.pan_start[T + 1] - s;
    // external part of each row (columns left of the panel): 32 lanes per row, 8 rows at once
    const int g = tid >> 5, gl = tid & 31;
    for (int t = g; t < w; t += kLargeThreads / 32) {
        const int i = s + t;
        const double acc = row_dot(a, a.y, a.rowptr[i], a.diag[i] - t, gl, 32);
        if (gl == 0) ext[t] = acc;
    }
    __syncthreads();
    if (tid >= 64) return;
    double yv = 0.0;
    if (lane < w) yv = a.r[a.P[s + lane]] * a.b[a.P[s + lane]] - ext[lane];
    for (int t = 0; t + 1 < w; ++t) {
        const double yt = bcast(yv, t);
        if (lane > t && lane < w) yv = fma(-a.lucsr[a.diag[s + lane] - (lane - t)], yt, yv);
    }
    if (lane < w) a.y[s + lane] = yv;
}

__global__ __launch_bounds__(256) void k_usolve_level(int item0, SolveArgs a) {
    __shared__ double ext[kPanelMax];
    const int item = item0 + blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const int np = a.item_np[item], p0 = a.item_p0[item];
    if (np < 0) {
        const int g = tid >> 3, gl = tid & 7;
        int i = -1, q0 = 0, q1 = 0;
        if (g < -np) {
            i = a.pan_start[a.pan[p0 + g]];
            q0 = a.diag[i] + 1;
            q1 = a.rowptr[i + 1];
        }
        const double acc = row_dot(a, a.xt, q0, q1, gl, 8);
        if (i >= 0 && gl == 0) {
            const double xv = (a.y[i] - acc) / a.lucsr[a.diag[i]];
            a.xt[i] = xv;
            a.x[a.Q[i]] = a.c[a.Q[i]] * xv;
        }
        return;
    }
    const int T = a.pan[p0];
    const int s = a.pan_start[T], w = a.pan_start[T + 1] - s;
    const int g = tid >> 5, gl = tid & 31;
    for (int t = g; t < w; t += kLargeThreads / 32) {
        const int i = s + t;
        const double acc = row_dot(a, a.xt, a.diag[i] + (w - t), a.rowptr[i + 1], gl, 32);
        if (gl == 0) ext[t] = acc;
    }
    __syncthreads();
    if (tid >= 64) return;
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

// res = b - A x (8 lanes per row, grid-stride) and block maxima of |res|, |x|, |b| into
// part[3 * block + {0, 1, 2}]
__global__ __launch_bounds__(256) void k_residual(int n, const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col, const double *__restrict__ v,
                                                  const double *__restrict__ x, const double *__restrict__ b,
                                                  double *__restrict__ res, double *__restrict__ part) {
    __shared__ double red[3][4];
    const double qnan = __longlong_as_double(0x7ff8000000000000LL);
    double rn = 0.0, xn = 0.0, bn = 0.0;
    const int gl = threadIdx.x & 7;
    for (int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 3; i < n; i += (gridDim.x * blockDim.x) >> 3) {
        double s = 0.0;
        for (int p = rowptr[i] + gl; p < rowptr[i + 1]; p += 8) s = fma(v[p], x[col[p]], s);
        s = group_sum(s, 8);
        if (gl == 0) {
            const double ri = b[i] - s;
            res[i] = ri;
            rn = isnan(ri) ? qnan : fmax(rn, fabs(ri));
            xn = isnan(x[i]) ? qnan : fmax(xn, fabs(x[i]));
            bn = fmax(bn, fabs(b[i]));
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double r2 = __shfl_xor(rn, o), x2 = __shfl_xor(xn, o);
        rn = (isnan(r2) || isnan(rn)) ? r2 + rn : fmax(rn, r2);
        xn = (isnan(x2) || isnan(xn)) ? x2 + xn : fmax(xn, x2);
        bn = fmax(bn, __shfl_xor(bn, o));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = rn;
        red[1][threadIdx.x >> 6] = xn;
        red[2][threadIdx.x >> 6] = bn;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = red[threadIdx.x][0];
        for (int q = 1; q < 4; ++q) {
            const double y = red[threadIdx.x][q];
            t = (isnan(t) || isnan(y)) ? t + y : fmax(t, y);
        }
        part[3 * blockIdx.x + threadIdx.x] = t;
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
