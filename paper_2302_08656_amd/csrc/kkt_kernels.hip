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

// r_i = 2^-floor(log2 max_j |a_ij|), 8 lanes per row; also clears the status words
__global__ __launch_bounds__(256) void k_row_scale(int n, const int32_t *__restrict__ rowptr,
                                                   const double *__restrict__ v, int scale,
                                                   double *__restrict__ r, DevStatus *st,
                                                   unsigned long long *pcount) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid == 0) {
        st->anorm_scaled = 0.0;
        st->anorm = 0.0;
        st->perturbed = 0;
        st->flags = 0;
        st->abort = 0;
    }
    if (blockIdx.x == 0)
        for (int t = threadIdx.x; t < kCountSlots; t += blockDim.x) pcount[t] = 0;
    const int i = gid >> 3, gl = gid & 7;
    double m = 0.0;
    int bad = 0;
    if (i < n)
        for (int p = rowptr[i] + gl; p < rowptr[i + 1]; p += 8) {
            const double x = fabs(v[p]);
            bad |= !isfinite(x);
            m = fmax(m, x);
        }
    for (int o = 4; o > 0; o >>= 1) {
        m = fmax(m, __shfl_xor(m, o, 8));
        bad |= __shfl_xor(bad, o, 8);
    }
    if (i < n && gl == 0) {
        if (bad) atomicOr(&st->flags, kFlagNonfinite);
        r[i] = scale ? inv_pow2_floor_log2(m) : 1.0;
    }
}

// c_j from the row-scaled matrix, 8 lanes per column of the CSC view
__global__ __launch_bounds__(256) void k_col_scale(int n, const int32_t *__restrict__ cptr,
                                                   const int32_t *__restrict__ cpos,
                                                   const int32_t *__restrict__ rowid,
                                                   const double *__restrict__ v, const double *__restrict__ r,
                                                   int scale, double *__restrict__ c) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = gid >> 3, gl = gid & 7;
    double m = 0.0;
    if (j < n)
        for (int t = cptr[j] + gl; t < cptr[j + 1]; t += 8) {
            const int p = cpos[t];
            m = fmax(m, fabs(r[rowid[p]] * v[p]));
        }
    for (int o = 4; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 8));
    if (j < n && gl == 0) c[j] = scale ? inv_pow2_floor_log2(m) : 1.0;
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

// st->perturbed = sum of the spread counter slots
__global__ __launch_bounds__(256) void k_sum_counts(const unsigned long long *__restrict__ pcount,
                                                    unsigned long long *out) {
    __shared__ unsigned long long red[4];
    unsigned long long c = 0;
    for (int i = threadIdx.x; i < kCountSlots; i += blockDim.x) c += pcount[i];
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
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

constexpr int kBlock = 256;   // threads of the elementwise, small-item and solve blocks

typedef double double4_t __attribute__((ext_vector_type(4)));

// Optional phase timestamps of the wide refactorization items (development builds only):
// with KKT_PHASE_TRACE defined, thread 0 of each item records the constant-rate clock at
// each phase boundary into kkt_phase_buf[item * 8 + phase].
#ifdef KKT_PHASE_TRACE
__device__ unsigned long long *kkt_phase_buf;
#define KKT_PHASE(item, k)                                                             \
    do {                                                                               \
        if (threadIdx.x == 0 && kkt_phase_buf) kkt_phase_buf[(item) * 8 + (k)] = wall_clock64(); \
    } while (0)
#else
#define KKT_PHASE(item, k) \
    do {                   \
    } while (0)
#endif

// pan[S] = {first column, width, rows below, 0}; pair[q] = {source panel, slot of the
// source's first row in the target column, first index into rel, target column}
struct RefArgs {
    const int32_t *ldiag;      // slot of the diagonal of each column
    const int4 *pan;
    const int32_t *item_panel, *item_pair;
    const int4 *pair;
    const int32_t *rel;
    double *lu;
    DevStatus *st;
    unsigned long long *pcount;   // replaced-pivot counter, spread over kCountSlots slots
    double tiny;
    int use_mfma;                 // dense update blocks on the matrix cores
};

// slot of the first L entry (row j+1 or below) of column j
__device__ __forceinline__ int lbeg(const RefArgs &a, int j) { return a.ldiag[j] + 1; }
// slot of row s (the panel's first row) in column j = s + jj of a panel starting at s
__device__ __forceinline__ int seg(const RefArgs &a, int j, int jj) { return a.ldiag[j] - jj; }

__device__ __forceinline__ double perturb(double p, double thresh, int &npert) {
    if (fabs(p) < thresh) {
        ++npert;
        return p < 0.0 ? -thresh : thresh;
    }
    return p;
}

// ----------------------------------------------------------------- 16-lane path

// Update of target column k by a narrow source panel S (w <= kSmallW, r <= kSmallR): rows
// s..e-1 of column k (from slot ps on) become final U entries (unit lower solve with S's
// diagonal block) and the rows R of S lose L(R, S) times them.
__device__ __forceinline__ void small_pull(const RefArgs &a, int4 pr, int gl) {
    const int4 pn = a.pan[pr.x];
    const int s = pn.x, w = pn.y, r = pn.z, ps = pr.y;
    const int32_t *rel = a.rel + pr.z;
    // diagonal slots of the source's columns, one per lane, then shared by shuffles
    const int ldg = gl < w ? a.ldiag[s + gl] : 0;
    int ld[kSmallW];
#pragma unroll
    for (int j = 0; j < kSmallW; ++j) ld[j] = __shfl(ldg, j, 16);
    double l_row[kSmallW - 1];   // L(s + gl, s + j) for j < gl
#pragma unroll
    for (int j = 0; j < kSmallW - 1; ++j) l_row[j] = (j + 1 < w && gl > j && gl < w) ? a.lu[ld[j] + (gl - j)] : 0.0;
    double u = gl < w ? a.lu[ps + gl] : 0.0;
#pragma unroll
    for (int j = 0; j < kSmallW - 1; ++j) {
        const double uj = __shfl(u, j, 16);
        if (j + 1 < w && gl > j && gl < w) u = fma(-l_row[j], uj, u);
    }
    if (gl < w) a.lu[ps + gl] = u;
    double uu[kSmallW];
    int lb[kSmallW];
#pragma unroll
    for (int j = 0; j < kSmallW; ++j) {
        uu[j] = __shfl(u, j, 16);
        lb[j] = ld[j] + 1 + (w - 1 - j);
    }
    for (int i = gl; i < r; i += 16) {
        const int pos = rel[i];
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < kSmallW; ++j)
            if (j < w) acc = fma(a.lu[lb[j] + i], uu[j], acc);
        a.lu[pos] -= acc;
    }
    __threadfence_block();   // a later source of the same column may read these rows
}

// Dense LU without pivoting of a narrow panel's block column (w <= kSmallW, r <= kSmallR).
// Returns the number of replaced pivots (the same value on every lane of the group).
__device__ __forceinline__ int small_factor(const RefArgs &a, int T, int gl, double thresh) {
    const int4 pn = a.pan[T];
    const int s = pn.x, w = pn.y, r = pn.z;
    const int ldg = gl < w ? a.ldiag[s + gl] : 0;
    int sg[kSmallW];
    double d[kSmallW];          // lane gl < w: row gl of the diagonal block
#pragma unroll
    for (int c = 0; c < kSmallW; ++c) sg[c] = __shfl(ldg, c, 16) - c;
#pragma unroll
    for (int c = 0; c < kSmallW; ++c) d[c] = (c < w && gl < w) ? a.lu[sg[c] + gl] : 0.0;
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

// kBlock/16 items per block, one per 16-lane group
__global__ __launch_bounds__(256) void k_refactor_small(int item0, int nsmall, RefArgs a) {
    const double thresh = a.tiny * a.st->anorm_scaled;
    const int g = blockIdx.x * (kBlock / 16) + (threadIdx.x >> 4);
    const int gl = threadIdx.x & 15;
    int npert = 0;
    if (g < nsmall) {
        const int item = item0 + g;
        for (int q = a.item_pair[item]; q < a.item_pair[item + 1]; ++q) small_pull(a, a.pair[q], gl);
        const int T = a.item_panel[item];
        if (T >= 0) npert = small_factor(a, T, gl, thresh);
    }
    // one counter update per wavefront: group leaders contribute their count
    int c = gl == 0 ? npert : 0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0 && c)
        atomicAdd(&a.pcount[(blockIdx.x * 4 + (threadIdx.x >> 6)) % kCountSlots], (unsigned long long)c);
}

// ----------------------------------------------------------------- 512-thread path

constexpr int kBigThreads = 512;
constexpr int kRChunk = 256;
// LDS layout (bytes): Ld (source diagonal block, later the factored panel's U) | Ub (solved
// rows per target) | Lr (a chunk of the source's L rows)
constexpr int kOffLd = 0;
constexpr int kOffUb = kOffLd + kPanelMax * kPanelMax * 8;
constexpr int kOffLr = kOffUb + kPanelMax * kGroup * 8;
constexpr int kStagePairs = 256;
constexpr int kOffPairs = kOffLr + kRChunk * kPanelMax * 8 + kPanelMax * 4;
constexpr int kLargeLds = kOffPairs + kStagePairs * 16;

// Dense LU without pivoting of a wide panel's block column: the diagonal block in the
// registers of wavefront 0 (lane = row), then every row below on its own thread.
__device__ __forceinline__ void large_factor(const RefArgs &a, int T, char *sm, double thresh) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int4 pn = a.pan[T];
    const int s = pn.x, w = pn.y, r = pn.z;
    double *D = reinterpret_cast<double *>(sm + kOffLd);   // D[c * kPanelMax + row]
    int *sgs = reinterpret_cast<int *>(sm + kOffUb);        // slot of row s in each column
    if (tid < w) sgs[tid] = seg(a, s + tid, tid);
    __syncthreads();
    int npert = 0, bad = 0;
    if (tid < 64) {
        double d[kPanelMax];
#pragma unroll
        for (int c = 0; c < kPanelMax; ++c) d[c] = (c < w && lane < w) ? a.lu[sgs[c] + lane] : 0.0;
#pragma unroll
        for (int jj = 0; jj < kPanelMax; ++jj) {
            if (jj < w) {
                const double p = perturb(bcast(d[jj], jj), thresh, npert);
                bad |= !isfinite(p);
                if (lane == jj) d[jj] = p;
                const double l = d[jj] / p;
                const bool below = lane > jj && lane < w;
                if (below) d[jj] = l;
#pragma unroll
                for (int c = jj + 1; c < kPanelMax; ++c) {
                    if (c < w) {
                        const double ujc = bcast(d[c], jj);
                        if (below) d[c] = fma(-l, ujc, d[c]);
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < kPanelMax; ++c) {
            if (c < w && lane < w) {
                a.lu[sgs[c] + lane] = d[c];
                D[c * kPanelMax + lane] = d[c];
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < r; i += kBigThreads) {
        double x[kPanelMax];
#pragma unroll
        for (int c = 0; c < kPanelMax; ++c) x[c] = c < w ? a.lu[sgs[c] + w + i] : 0.0;
#pragma unroll
        for (int jj = 0; jj < kPanelMax; ++jj) {
            if (jj < w) {
                const double l = x[jj] / D[jj * kPanelMax + jj];
                bad |= !isfinite(l);
                x[jj] = l;
#pragma unroll
                for (int c = jj + 1; c < kPanelMax; ++c)
                    if (c < w) x[c] = fma(-l, D[c * kPanelMax + jj], x[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < kPanelMax; ++c)
            if (c < w) a.lu[sgs[c] + w + i] = x[c];
    }
    if (tid == 0 && npert) atomicAdd(&a.pcount[blockIdx.x % kCountSlots], (unsigned long long)npert);
    if (__any(bad) && lane == 0) atomicOr(&a.st->flags, kFlagNonfinite);
}

// All pulls of one item with the source panel staged in LDS, then the panel factorization.
__global__ __launch_bounds__(kBigThreads) void k_refactor_large(int item0, RefArgs a) {
    extern __shared__ __align__(16) char sm[];
    const double thresh = a.tiny * a.st->anorm_scaled;
    const int item = item0 + blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int nw = kBigThreads / 64;
    KKT_PHASE(item, 0);
    double *Ld = reinterpret_cast<double *>(sm + kOffLd);
    double *Ub = reinterpret_cast<double *>(sm + kOffUb);
    double *Lr = reinterpret_cast<double *>(sm + kOffLr);
    const int p1 = a.item_pair[item + 1];
    int *lds = reinterpret_cast<int *>(sm + kOffLr + kRChunk * kPanelMax * 8);   // diagonal slots
    int4 *prs = reinterpret_cast<int4 *>(sm + kOffPairs);                          // staged pairs
    const int pbeg = a.item_pair[item];
    const int npr = p1 - pbeg;
    const bool staged = npr <= kStagePairs;
    if (staged)
        for (int t = tid; t < npr; t += kBigThreads) prs[t] = a.pair[pbeg + t];
    __syncthreads();
    auto pr_at = [&](int q) { return staged ? prs[q - pbeg] : a.pair[q]; };
    KKT_PHASE(item, 1);
    for (int g0 = pbeg, g1; g0 < p1; g0 = g1) {
        const int S = pr_at(g0).x;
        g1 = g0 + 1;
        while (g1 < p1 && pr_at(g1).x == S) ++g1;
        const int4 pn = a.pan[S];
        const int s = pn.x, w = pn.y, r = pn.z;
        if (tid < w) lds[tid] = a.ldiag[s + tid];
        __syncthreads();
        for (int t = tid; t < w * w; t += kBigThreads) {
            const int j = t / w, i = t % w;
            if (i > j) Ld[j * kPanelMax + i] = a.lu[lds[j] + (i - j)];
        }
        __syncthreads();
        KKT_PHASE(item, 2);
        // rows of S in each target: unit lower solve with S's diagonal block, one lane per
        // target (wavefront 0; groups hold at most kGroup targets); the lane keeps its
        // target's rows in registers
        if (wv == 0 && lane < g1 - g0) {
            const int ps = pr_at(g0 + lane).y;
            double u[kPanelMax];
#pragma unroll
            for (int j = 0; j < kPanelMax; ++j) u[j] = j < w ? a.lu[ps + j] : 0.0;
#pragma unroll
            for (int t = 1; t < kPanelMax; ++t) {
                if (t < w) {
                    double acc = u[t];
#pragma unroll
                    for (int j = 0; j < t; ++j) acc = fma(-Ld[j * kPanelMax + t], u[j], acc);
                    u[t] = acc;
                }
            }
#pragma unroll
            for (int j = 0; j < kPanelMax; ++j) {
                if (j < w) {
                    a.lu[ps + j] = u[j];
                    Ub[lane * kPanelMax + j] = u[j];
                }
            }
        }
        __syncthreads();
        KKT_PHASE(item, 3);
        // rows R of each target: chunks of S's L rows staged in LDS, precomputed slots
        for (int i0 = 0; i0 < r; i0 += kRChunk) {
            const int nr = min(kRChunk, r - i0);
            for (int t = tid; t < w * nr; t += kBigThreads) {
                const int j = t / nr, i = t % nr;
                Lr[j * kRChunk + i] = a.lu[lds[j] + 1 + (w - 1 - j) + i0 + i];
            }
            __syncthreads();
            const int m = g1 - g0;
            if (a.use_mfma && m > 1) {
                // update block Lr (nr x w) times the solved rows (w x m) on the matrix cores:
                // 16x16 output tiles, k in steps of 4; lane holds A[lane % 16][lane / 16],
                // B[lane / 16][lane % 16] and the four outputs D[lane / 16 + 4 v][lane % 16]
                const int mt = (nr + 15) >> 4, nt = (m + 15) >> 4;
                const int li = lane & 15, lk = lane >> 4;
                for (int tile = wv; tile < mt * nt; tile += nw) {
                    const int ti = tile % mt, tt = tile / mt;
                    const int ia = ti * 16 + li, tb = tt * 16 + li;
                    double4_t acc = {0.0, 0.0, 0.0, 0.0};
                    for (int k0 = 0; k0 < w; k0 += 4) {
                        const int k = k0 + lk;
                        const double av = (k < w && ia < nr) ? Lr[k * kRChunk + ia] : 0.0;
                        const double bv = (k < w && tb < m) ? Ub[tb * kPanelMax + k] : 0.0;
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                    }
                    if (tb < m) {
                        const int32_t *rel = a.rel + pr_at(g0 + tb).z + i0;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int i = ti * 16 + lk + 4 * v;
                            if (i < nr) a.lu[rel[i]] -= acc[v];
                        }
                    }
                }
            } else {
                for (int q = g0 + wv; q < g1; q += nw) {
                    const int32_t *rel = a.rel + pr_at(q).z + i0;
                    const double *ub = Ub + (q - g0) * kPanelMax;
                    for (int i = lane; i < nr; i += 64) {
                        double acc = 0.0;
                        for (int j = 0; j < w; ++j) acc = fma(Lr[j * kRChunk + i], ub[j], acc);
                        a.lu[rel[i]] -= acc;
                    }
                }
            }
            __syncthreads();
        }
        __threadfence_block();
        __syncthreads();
        KKT_PHASE(item, 4);
    }
    const int T = a.item_panel[item];
    if (T >= 0) large_factor(a, T, sm, thresh);
    KKT_PHASE(item, 5);
}

// ---------------------------------------------------------------------------------------
// triangular solves: one 256-thread block per wide panel or per pack of kSolvePack
// width-1 panels (kPackLanes lanes per row)

constexpr int kPackLanes = kBlock / kSolvePack;

struct SolveArgs {
    const int32_t *pan_start, *item_p0, *item_np, *pan;
    const int32_t *rowptr, *col, *diag, *early, *P, *Q;
    const double *lucsr, *r, *c;
    const double *b;      // forward: right-hand side (original order)
    double *y;            // forward output / backward input (permuted)
    double *xt;           // backward output (permuted)
    double *x;            // backward output (original order)
    double *psum;         // forward: partial sums of the early L columns of helped rows
};

// sum over q in [q0, q1) of lucsr[q] * v[col[q]] on a group of `width` lanes; four
// independent gathers in flight per lane
__device__ __forceinline__ double row_dot(const SolveArgs &a, const double *v, int q0, int q1, int gl, int width) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int q = q0 + gl;
    for (; q + 3 * width < q1; q += 4 * width) {
        const int c0 = a.col[q], c1 = a.col[q + width], c2 = a.col[q + 2 * width], c3 = a.col[q + 3 * width];
        s0 = fma(a.lucsr[q], v[c0], s0);
        s1 = fma(a.lucsr[q + width], v[c1], s1);
        s2 = fma(a.lucsr[q + 2 * width], v[c2], s2);
        s3 = fma(a.lucsr[q + 3 * width], v[c3], s3);
    }
    for (; q < q1; q += width) s0 = fma(a.lucsr[q], v[a.col[q]], s0);
    return group_sum((s0 + s1) + (s2 + s3), width);
}

// In-panel block of a wide panel staged in LDS by the whole block (one parallel round):
// blk[t * kPanelMax + i] = entry (s + i, s + t) of L (t < i) or U (t > i); blk[i * 33] = U(i, i).
__device__ __forceinline__ void stage_inpanel(const SolveArgs &a, int s, int w, double *blk) {
    for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
        const int i = e / w, t = e % w;
        blk[t * kPanelMax + i] = a.lucsr[a.diag[s + i] + (t - i)];
    }
}

// Forward substitution inside a panel of w <= kPanelMax rows (lane = row); yv enters as the
// row's right-hand side minus its external part.
__device__ __forceinline__ double inpanel_forward(const double *blk, int w, int lane, double yv) {
    for (int t = 0; t + 1 < w; ++t) {
        const double yt = bcast(yv, t);
        if (lane > t && lane < w) yv = fma(-blk[t * kPanelMax + lane], yt, yv);
    }
    return yv;
}

// Backward substitution inside a panel (lane = row); val enters as y minus the external
// part; returns the lane's unknown.
__device__ __forceinline__ double inpanel_backward(const double *blk, int w, int lane, double val) {
    double xv = 0.0;
    for (int t = w - 1; t >= 0; --t) {
        if (lane == t) xv = val / blk[t * kPanelMax + t];
        const double xt = bcast(xv, t);
        if (lane < t) val = fma(-blk[t * kPanelMax + lane], xt, val);
    }
    return xv;
}

__global__ __launch_bounds__(256) void k_lsolve_level(int item0, SolveArgs a) {
    __shared__ double ext[kPanelMax];
    __shared__ double blk[kPanelMax * kPanelMax];
    const int item = item0 + blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const int np = a.item_np[item], p0 = a.item_p0[item];
    if (np < 0) {                                    // pack of width-1 panels, 8 lanes each
        const int g = tid / kPackLanes, gl = tid % kPackLanes;
        int i = -1, q0 = 0, q1 = 0;
        if (g < -np) {
            i = a.pan[p0 + g];
            q0 = a.rowptr[i];
            q1 = a.diag[i];
        }
        const double acc = row_dot(a, a.y, q0, q1, gl, kPackLanes);
        if (i >= 0 && gl == 0) a.y[i] = a.r[a.P[i]] * a.b[a.P[i]] - acc;
        return;
    }
    const int T = a.pan[p0];
    const int s = a.pan_start[T], w = a.pan_start[T + 1] - s;
    const int g = tid >> 5, gl = tid & 31;
    if (np == 0) {                                   // early partial sums of panel T's rows
        for (int t = g; t < w; t += kBlock / 32) {
            const int i = s + t;
            const double acc = row_dot(a, a.y, a.rowptr[i], a.early[i], gl, 32);
            if (gl == 0) a.psum[i] = acc;
        }
        return;
    }
    stage_inpanel(a, s, w, blk);
    // late part of each row (columns left of the panel), 32 lanes per row, 8 rows at once
    for (int t = g; t < w; t += kBlock / 32) {
        const int i = s + t;
        const int e = a.early[i];
        double acc = row_dot(a, a.y, e, a.diag[i] - t, gl, 32);
        if (gl == 0) ext[t] = e > a.rowptr[i] ? acc + a.psum[i] : acc;
    }
    __syncthreads();
    if (tid >= 64) return;
    double yv = 0.0;
    if (lane < w) yv = a.r[a.P[s + lane]] * a.b[a.P[s + lane]] - ext[lane];
    yv = inpanel_forward(blk, w, lane, yv);
    if (lane < w) a.y[s + lane] = yv;
}

__global__ __launch_bounds__(256) void k_usolve_level(int item0, SolveArgs a) {
    __shared__ double ext[kPanelMax];
    __shared__ double blk[kPanelMax * kPanelMax];
    const int item = item0 + blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const int np = a.item_np[item], p0 = a.item_p0[item];
    if (np < 0) {
        const int g = tid / kPackLanes, gl = tid % kPackLanes;
        int i = -1, q0 = 0, q1 = 0;
        if (g < -np) {
            i = a.pan[p0 + g];
            q0 = a.diag[i] + 1;
            q1 = a.rowptr[i + 1];
        }
        const double acc = row_dot(a, a.xt, q0, q1, gl, kPackLanes);
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
    stage_inpanel(a, s, w, blk);
    for (int t = g; t < w; t += kBlock / 32) {
        const int i = s + t;
        const double acc = row_dot(a, a.xt, a.diag[i] + (w - t), a.rowptr[i + 1], gl, 32);
        if (gl == 0) ext[t] = acc;
    }
    __syncthreads();
    if (tid >= 64) return;
    double val = 0.0;
    if (lane < w) val = a.y[s + lane] - ext[lane];
    const double xv = inpanel_backward(blk, w, lane, val);
    if (lane < w) {
        a.xt[s + lane] = xv;
        a.x[a.Q[s + lane]] = a.c[a.Q[s + lane]] * xv;
    }
}

// ---------------------------------------------------------------------------------------
// persistent triangular solves (the narrow top of the tree): blocks take the solve items of
// a range of levels from a queue in level order.
// Every unknown starts as a signaling-NaN sentinel (arithmetic never produces one) and is
// published by one 64-bit device-coherent store, so the value is its own ready flag.
// A read of a not-yet-published unknown waits (bounded); items only depend on items that
// were taken earlier, so the earliest unfinished item can always proceed.

constexpr unsigned long long kUnset = 0x7ff4dead0badf00dULL;   // signaling NaN
constexpr int kSpinLimit = 1 << 21;

__device__ __forceinline__ unsigned long long load_coherent(const double *p) {
    return __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void publish(double *p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// value of an unknown, waiting until it is published; on timeout or abort returns 0 and
// raises *abort (the solve result is then invalid and reported as a device error)
__device__ __forceinline__ double wait_value(const double *p, int *abort) {
    unsigned long long b = load_coherent(p);
    if (b != kUnset) return __longlong_as_double((long long)b);
    for (int it = 0; it < kSpinLimit; ++it) {
        __builtin_amdgcn_s_sleep(2);
        b = load_coherent(p);
        if (b != kUnset) return __longlong_as_double((long long)b);
        if ((it & 63) == 63 &&
            __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return 0.0;
    }
    atomicOr(abort, 1);
    return 0.0;
}

// row_dot with waits; same summation order, so both solve modes give identical results
__device__ __forceinline__ double row_dot_wait(const SolveArgs &a, const double *v, int q0, int q1, int gl,
                                               int width, int *abort) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int q = q0 + gl;
    for (; q + 3 * width < q1; q += 4 * width) {
        const int c0 = a.col[q], c1 = a.col[q + width], c2 = a.col[q + 2 * width], c3 = a.col[q + 3 * width];
        s0 = fma(a.lucsr[q], wait_value(v + c0, abort), s0);
        s1 = fma(a.lucsr[q + width], wait_value(v + c1, abort), s1);
        s2 = fma(a.lucsr[q + 2 * width], wait_value(v + c2, abort), s2);
        s3 = fma(a.lucsr[q + 3 * width], wait_value(v + c3, abort), s3);
    }
    for (; q < q1; q += width) s0 = fma(a.lucsr[q], wait_value(v + a.col[q], abort), s0);
    return group_sum((s0 + s1) + (s2 + s3), width);
}

// y[:] = xt[:] = psum[:] = unset, work queues cleared
__global__ void k_solve_reset(int n, double *__restrict__ y, double *__restrict__ xt, double *__restrict__ psum,
                              DevStatus *st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const double u = __longlong_as_double((long long)kUnset);
    if (i < n) {
        y[i] = u;
        xt[i] = u;
        psum[i] = u;
    }
    if (i < 4) st->queue[i] = 0;
}

__device__ __forceinline__ int next_item(int *queue) {
    __shared__ int s_item;
    if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    return item;
}

__global__ __launch_bounds__(256) void k_lsolve_persistent(int i0, int i1, SolveArgs a, int *queue, int *abort) {
    __shared__ double ext[kPanelMax];
    __shared__ double blk[kPanelMax * kPanelMax];
    const int tid = threadIdx.x, lane = tid & 63;
    for (;;) {
        const int item = i0 + next_item(queue);
        if (item >= i1 || __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
        const int np = a.item_np[item], p0 = a.item_p0[item];
        if (np < 0) {                                    // pack of width-1 panels, 8 lanes each
            const int g = tid / kPackLanes, gl = tid % kPackLanes;
            int i = -1, q0 = 0, q1 = 0;
            if (g < -np) {
                i = a.pan[p0 + g];
                q0 = a.rowptr[i];
                q1 = a.diag[i];
            }
            const double acc = row_dot_wait(a, a.y, q0, q1, gl, kPackLanes, abort);
            if (i >= 0 && gl == 0) publish(a.y + i, a.r[a.P[i]] * a.b[a.P[i]] - acc);
            continue;
        }
        const int T = a.pan[p0];
        const int s = a.pan_start[T], w = a.pan_start[T + 1] - s;
        const int g = tid >> 5, gl = tid & 31;
        if (np == 0) {                                   // early partial sums of panel T's rows
            for (int t = g; t < w; t += kBlock / 32) {
                const int i = s + t;
                const double acc = row_dot_wait(a, a.y, a.rowptr[i], a.early[i], gl, 32, abort);
                if (gl == 0) publish(a.psum + i, acc);
            }
            continue;
        }
        stage_inpanel(a, s, w, blk);
        for (int t = g; t < w; t += kBlock / 32) {
            const int i = s + t;
            const int e = a.early[i];
            const double acc = row_dot_wait(a, a.y, e, a.diag[i] - t, gl, 32, abort);
            if (gl == 0) ext[t] = e > a.rowptr[i] ? acc + wait_value(a.psum + i, abort) : acc;
        }
        __syncthreads();
        if (tid < 64) {
            double yv = 0.0;
            if (lane < w) yv = a.r[a.P[s + lane]] * a.b[a.P[s + lane]] - ext[lane];
            yv = inpanel_forward(blk, w, lane, yv);
            if (lane < w) publish(a.y + s + lane, yv);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_usolve_persistent(int i0, int i1, SolveArgs a, int *queue, int *abort) {
    __shared__ double ext[kPanelMax];
    __shared__ double blk[kPanelMax * kPanelMax];
    const int tid = threadIdx.x, lane = tid & 63;
    for (;;) {
        const int item = i0 + next_item(queue);
        if (item >= i1 || __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
        const int np = a.item_np[item], p0 = a.item_p0[item];
        if (np < 0) {
            const int g = tid / kPackLanes, gl = tid % kPackLanes;
            int i = -1, q0 = 0, q1 = 0;
            if (g < -np) {
                i = a.pan[p0 + g];
                q0 = a.diag[i] + 1;
                q1 = a.rowptr[i + 1];
            }
            const double acc = row_dot_wait(a, a.xt, q0, q1, gl, kPackLanes, abort);
            if (i >= 0 && gl == 0) {
                const double xv = (a.y[i] - acc) / a.lucsr[a.diag[i]];
                a.x[a.Q[i]] = a.c[a.Q[i]] * xv;
                publish(a.xt + i, xv);
            }
            continue;
        }
        const int T = a.pan[p0];
        const int s = a.pan_start[T], w = a.pan_start[T + 1] - s;
        const int g = tid >> 5, gl = tid & 31;
        stage_inpanel(a, s, w, blk);
        for (int t = g; t < w; t += kBlock / 32) {
            const int i = s + t;
            const double acc = row_dot_wait(a, a.xt, a.diag[i] + (w - t), a.rowptr[i + 1], gl, 32, abort);
            if (gl == 0) ext[t] = acc;
        }
        __syncthreads();
        if (tid < 64) {
            double val = 0.0;
            if (lane < w) val = a.y[s + lane] - ext[lane];
            const double xv = inpanel_backward(blk, w, lane, val);
            if (lane < w) {
                a.x[a.Q[s + lane]] = a.c[a.Q[s + lane]] * xv;
                publish(a.xt + s + lane, xv);
            }
        }
        __syncthreads();
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
