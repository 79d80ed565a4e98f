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

#include <cstddef>
#include <cstdint>
#include <type_traits>

#include "kkt_kernels.h"

namespace kkt {

__device__ __forceinline__ double bcast(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float bcast(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Barrier over the block for data exchanged through LDS only: global memory operations of
// the waves may stay in flight across it (a plain __syncthreads waits for them).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// the equilibration scale 2^-floor(log2 m) (1 for m <= 0 or NaN) is kept as its exponent e,
// clamped to +-1020 so that 2^-e is a normal number; scale_of(e) rebuilds the scale exactly
__device__ __forceinline__ int pow2_floor_log2(double m) {
    if (!(m > 0.0)) return 0;
    const int e = ilogb(m);
    return e > 1020 ? 1020 : (e < -1020 ? -1020 : e);
}
__device__ __forceinline__ double scale_of(int e) { return ldexp(1.0, -e); }
__device__ __forceinline__ double inv_pow2_floor_log2(double m) { return scale_of(pow2_floor_log2(m)); }


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

// Clears the status words and the replaced-pivot counter slots of a refactorization (one
// block, launched before k_row_scale, whose blocks may raise the non-finite flag).
__device__ __forceinline__ void clear_status_body(DevStatus *st, unsigned long long *pcount) {
    if (threadIdx.x == 0) {
        st->anorm_scaled = 0.0;
        st->anorm = 0.0;
        st->perturbed = 0;
        st->flags = 0;
        st->abort = 0;
    }
    for (int t = threadIdx.x; t < kCountSlots; t += blockDim.x) pcount[t] = 0;
}

// The per-call inputs of the recorded graphs (the values of A, the right-hand side): a
// one-thread launch stores them before a replay and the recorded kernels read them here, so
// one recording serves every call.
struct CallPtrs {
    const double *v;
    const double *b;
};

// stores the call's inputs and clears the status words and pivot counters of the call
// (one block of 256 threads)
__global__ __launch_bounds__(256) void k_set_call(CallPtrs *dst, const double *v, const double *b, DevStatus *st,
                                                  unsigned long long *pcount) {
    clear_status_body(st, pcount);
    if (threadIdx.x == 0) {
        dst->v = v;
        dst->b = b;
    }
}

// a pointer stored by an earlier launch, read past the non-coherent caches
__device__ __forceinline__ const double *call_ptr(const double *const *p) {
    return reinterpret_cast<const double *>(__hip_atomic_load(reinterpret_cast<const unsigned long long *>(p),
                                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Rows of the update passes taken by one group of 8 lanes: the group issues the loads of
// all its rows together, so a wavefront has that many times more loads in flight (the passes
// are bound by the latency of their dependent loads, not by bandwidth).
constexpr int kRowsPerGroup = 4;

// the row pointers of rows i0 .. i0 + kRowsPerGroup (0 past n)
__device__ __forceinline__ void group_rows(const int32_t *__restrict__ rowptr, int n, int i0,
                                           int (&rp)[kRowsPerGroup + 1]) {
#pragma unroll
    for (int k = 0; k <= kRowsPerGroup; ++k) rp[k] = i0 + k <= n ? rowptr[i0 + k] : 0;
}

// r_i = 2^-floor(log2 max_j |a_ij|), 8 lanes per row, kRowsPerGroup rows per group; a
// non-finite value raises the flag
__device__ __forceinline__ void row_scale_body(int blk, int n, const int32_t *__restrict__ rowptr,
                                               const double *__restrict__ v, int scale, double *__restrict__ r,
                                               int16_t *__restrict__ er, DevStatus *st) {
    const int gid = blk * blockDim.x + threadIdx.x;
    const int i0 = (gid >> 3) * kRowsPerGroup, gl = gid & 7;
    int rp[kRowsPerGroup + 1];
    group_rows(rowptr, n, i0, rp);
    double m[kRowsPerGroup];
    int bad = 0;
#pragma unroll
    for (int k = 0; k < kRowsPerGroup; ++k) {
        const int p = rp[k] + gl;
        m[k] = p < rp[k + 1] ? fabs(v[p]) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kRowsPerGroup; ++k) {
        bad |= !isfinite(m[k]);
        for (int p = rp[k] + gl + 8; p < rp[k + 1]; p += 8) {
            const double x = fabs(v[p]);
            bad |= !isfinite(x);
            m[k] = fmax(m[k], x);
        }
    }
    for (int o = 4; o > 0; o >>= 1) {
#pragma unroll
        for (int k = 0; k < kRowsPerGroup; ++k) m[k] = fmax(m[k], __shfl_xor(m[k], o, 8));
        bad |= __shfl_xor(bad, o, 8);
    }
    if (gl == 0 && i0 < n) {
        if (bad) atomicOr(&st->flags, kFlagNonfinite);
#pragma unroll
        for (int k = 0; k < kRowsPerGroup; ++k)
            if (i0 + k < n) {
                const int e = scale ? pow2_floor_log2(m[k]) : 0;
                r[i0 + k] = scale_of(e);
                er[i0 + k] = (int16_t)e;
            }
    }
}

__global__ __launch_bounds__(256) void k_row_scale(int n, const int32_t *__restrict__ rowptr,
                                                   const CallPtrs *call, int scale,
                                                   double *__restrict__ r, int16_t *__restrict__ er,
                                                   DevStatus *st) {
    row_scale_body(blockIdx.x, n, rowptr, call_ptr(&call->v), scale, r, er, st);
}

// c from the row-scaled matrix and the scaled values into the factor, per column j
// of the factor (column Q[j] of A), its slots in storage order: src[p] = {position of slot
// p's entry of A in the CSR value array, or -1 for a fill-in slot; that entry's row i of A}.
// c[Q[j]] = 2^-floor(log2 max_i |r_i a_i,Q[j]|); then lu[p] = (r_i a) c (exact in FP64;
// rounded once when the factor is FP32), 0 for fill-in.  The factor is written in its own
// order (no scattered stores); the first kColRegs slots of each lane keep r_i a in registers
// between the two sweeps, later slots of a long column are gathered again.  kColLanes lanes
// per column, so that each lane has several gathers in flight.
constexpr int kColLanes = 8;
constexpr int kColRegs = 4;

template <class T>
__device__ __forceinline__ void col_store_body(int blk, int n, const int32_t *__restrict__ colptr,
                                               const int2 *__restrict__ src, const int32_t *__restrict__ Q,
                                               const double *__restrict__ v, const int16_t *__restrict__ er,
                                               int scale, double *__restrict__ c, int16_t *__restrict__ ec,
                                               T *__restrict__ lu) {
    const int gid = blk * blockDim.x + threadIdx.x;
    const int j = gid / kColLanes, gl = gid % kColLanes;
    const int p0 = j < n ? colptr[j] : 0, p1 = j < n ? colptr[j + 1] : 0;
    int2 e[kColRegs];
#pragma unroll
    for (int k = 0; k < kColRegs; ++k) {
        const int p = p0 + gl + kColLanes * k;
        e[k] = p < p1 ? src[p] : int2{-1, 0};
    }
    double ra[kColRegs];
#pragma unroll
    for (int k = 0; k < kColRegs; ++k) ra[k] = e[k].x >= 0 ? scale_of(er[e[k].y]) * v[e[k].x] : 0.0;
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < kColRegs; ++k) m = fmax(m, fabs(ra[k]));
    for (int p = p0 + gl + kColLanes * kColRegs; p < p1; p += kColLanes) {
        const int2 f = src[p];
        if (f.x >= 0) m = fmax(m, fabs(scale_of(er[f.y]) * v[f.x]));
    }
    for (int o = kColLanes / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, kColLanes));
    const int ej = scale ? pow2_floor_log2(m) : 0;
    const double cj = scale_of(ej);
    if (j < n && gl == 0) {
        c[Q[j]] = cj;
        ec[Q[j]] = (int16_t)ej;
    }
#pragma unroll
    for (int k = 0; k < kColRegs; ++k) {
        const int p = p0 + gl + kColLanes * k;
        if (p < p1) lu[p] = e[k].x >= 0 ? (T)(ra[k] * cj) : T(0);
    }
    for (int p = p0 + gl + kColLanes * kColRegs; p < p1; p += kColLanes) {
        const int2 f = src[p];
        lu[p] = f.x >= 0 ? (T)((scale_of(er[f.y]) * v[f.x]) * cj) : T(0);
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_col_store(int n, const int32_t *__restrict__ colptr,
                                                   const int2 *__restrict__ src, const int32_t *__restrict__ Q,
                                                   const CallPtrs *call, const int16_t *__restrict__ er,
                                                   int scale, double *__restrict__ c, int16_t *__restrict__ ec,
                                                   T *__restrict__ lu) {
    col_store_body<T>(blockIdx.x, n, colptr, src, Q, call_ptr(&call->v), er, scale, c, ec, lu);
}

// The row sums of |A| and |R A C| in CSR order, kRowsPerGroup rows per group of 8 lanes
// (grid-stride): the lanes load 8 consecutive entries of each row at once and leave their
// terms in LDS, and lane k of the group adds row k's terms in CSR order (so the sums are
// the sequential ones, bit for bit); block maxima into part[2 * block].  blockDim.x <= 256.
__device__ __forceinline__ void norms_body(int blk, int nblk, int n, const int32_t *__restrict__ rowptr,
                                           const int32_t *__restrict__ col, const double *__restrict__ v,
                                           const double *__restrict__ r, const int16_t *__restrict__ ec,
                                           double *__restrict__ part) {
    __shared__ double red[2][4];
    __shared__ double terms[256 / 8][kRowsPerGroup][2][8];   // per group: row, {|r a c|, |a|}, entry
    const int gl = threadIdx.x & 7, grp = threadIdx.x >> 3;
    double (*T)[2][8] = terms[grp];
    double s = 0.0, a = 0.0;
    for (int i0 = ((blk * blockDim.x + threadIdx.x) >> 3) * kRowsPerGroup; i0 < n;
         i0 += ((nblk * blockDim.x) >> 3) * kRowsPerGroup) {
        int rp[kRowsPerGroup + 1];
        group_rows(rowptr, n, i0, rp);
        double ri[kRowsPerGroup], vv[kRowsPerGroup], cj[kRowsPerGroup];
        int cc[kRowsPerGroup];
#pragma unroll
        for (int k = 0; k < kRowsPerGroup; ++k) {
            const int p = rp[k] + gl;
            const bool h = p < rp[k + 1];
            ri[k] = i0 + k < n ? r[i0 + k] : 0.0;
            vv[k] = h ? v[p] : 0.0;
            cc[k] = h ? col[p] : 0;
        }
#pragma unroll
        for (int k = 0; k < kRowsPerGroup; ++k) cj[k] = rp[k] + gl < rp[k + 1] ? scale_of(ec[cc[k]]) : 0.0;
#pragma unroll
        for (int k = 0; k < kRowsPerGroup; ++k) {
            T[k][0][gl] = fabs((ri[k] * vv[k]) * cj[k]);
            T[k][1][gl] = fabs(vv[k]);
        }
        __builtin_amdgcn_wave_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        // lane k: row k's first (up to) 8 terms in order
        const int k = gl < kRowsPerGroup ? gl : 0;
        const int len0 = min(8, rp[k + 1] - rp[k]);
        double si = 0.0, ai = 0.0;
        if (gl < kRowsPerGroup)
            for (int t = 0; t < len0; ++t) {
                si = si + T[k][0][t];
                ai = ai + T[k][1][t];
            }
        // longer rows: the group loads each further chunk of 8, the row's lane adds it
#pragma unroll
        for (int kk = 0; kk < kRowsPerGroup; ++kk) {
            for (int q = rp[kk] + 8; q < rp[kk + 1]; q += 8) {
                __builtin_amdgcn_wave_barrier();
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                const bool h = q + gl < rp[kk + 1];
                const double x = h ? v[q + gl] : 0.0;
                T[0][0][gl] = h ? fabs((ri[kk] * x) * scale_of(ec[col[q + gl]])) : 0.0;
                T[0][1][gl] = fabs(x);
                __builtin_amdgcn_wave_barrier();
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                if (gl == kk) {
                    const int cnt = min(8, rp[kk + 1] - q);
                    for (int t = 0; t < cnt; ++t) {
                        si = si + T[0][0][t];
                        ai = ai + T[0][1][t];
                    }
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (gl < kRowsPerGroup) {
            s = fmax(s, si);
            a = fmax(a, ai);
        }
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
        part[2 * blk] = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
        part[2 * blk + 1] = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
    }
}

__global__ __launch_bounds__(256) void k_norms(int n, const int32_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ col, const CallPtrs *call,
                                               const double *__restrict__ r, const int16_t *__restrict__ ec,
                                               double *__restrict__ part) {
    norms_body(blockIdx.x, gridDim.x, n, rowptr, col, call_ptr(&call->v), r, ec, part);
}

// max that propagates a NaN of either side
__device__ __forceinline__ double max_nan(double m, double x) {
    return (isnan(x) || isnan(m)) ? x + m : fmax(m, x);
}

// dst[j] = max over blocks b of part[nfield * b + j] (NaN propagates), j < nfield; each
// thread keeps four maxima so that its loads are in flight together
__device__ __forceinline__ void max_parts_body(int nblk, int nfield, const double *__restrict__ part,
                                               double *__restrict__ dst) {
    __shared__ double red[4];
    for (int j = 0; j < nfield; ++j) {
        double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
        const int step = blockDim.x;
        int b = threadIdx.x;
        for (; b + 3 * step < nblk; b += 4 * step) {
            const double x0 = part[nfield * b + j], x1 = part[nfield * (b + step) + j];
            const double x2 = part[nfield * (b + 2 * step) + j], x3 = part[nfield * (b + 3 * step) + j];
            m0 = max_nan(m0, x0);
            m1 = max_nan(m1, x1);
            m2 = max_nan(m2, x2);
            m3 = max_nan(m3, x3);
        }
        for (; b < nblk; b += step) m0 = max_nan(m0, part[nfield * b + j]);
        double m = max_nan(max_nan(m0, m1), max_nan(m2, m3));
        for (int o = 32; o > 0; o >>= 1) m = max_nan(m, __shfl_xor(m, o));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = red[0];
            for (int q = 1; q < 4; ++q) t = max_nan(t, red[q]);
            dst[j] = t;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_max_parts(int nblk, int nfield, const double *__restrict__ part,
                                                   double *__restrict__ dst) {
    max_parts_body(nblk, nfield, part, dst);
}

// st->perturbed = sum of the spread counter slots
__device__ __forceinline__ void sum_counts_body(const unsigned long long *__restrict__ pcount,
                                                unsigned long long *out) {
    __shared__ unsigned long long red[4];
    unsigned long long c = 0;
    for (int i = threadIdx.x; i < kCountSlots; i += blockDim.x) c += pcount[i];
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_sum_counts(const unsigned long long *__restrict__ pcount,
                                                    unsigned long long *out) {
    sum_counts_body(pcount, out);
}

// Two ranges [a0, a1) and [b0, b1) of the row-ordered copy list (entries of the strictly
// lower and of the upper section)
struct CopyRanges {
    int a0, a1, b0, b1;
};

// lucsr[copy_k[q]] = lu[copy_src[q]] for q in the ranges (copy_src[q]: factor slot of CSR
// position copy_k[q]), by block b of nb blocks of nthreads threads
template <class T>
__device__ __forceinline__ void copy_ranges(const int32_t *__restrict__ copy_k, const int32_t *__restrict__ copy_src,
                                            const T *__restrict__ lu, T *__restrict__ lucsr, const CopyRanges &c,
                                            int b, int nb, int nthreads) {
    const int na = c.a1 - c.a0, tot = na + (c.b1 - c.b0);
    for (int t = b * nthreads + (int)threadIdx.x; t < tot; t += nb * nthreads) {
        const int q = t < na ? c.a0 + t : c.b0 + (t - na);
        lucsr[copy_k[q]] = lu[copy_src[q]];
    }
}

// the copy on all blocks but the last when pcount is set: that one sums the replaced-pivot
// counter slots into *pout (every refactorization launch has finished)
template <class T>
__global__ __launch_bounds__(256) void k_to_csr(CopyRanges c, const int32_t *__restrict__ copy_k,
                                                const int32_t *__restrict__ copy_src, const T *__restrict__ lu,
                                                T *__restrict__ lucsr, const unsigned long long *__restrict__ pcount,
                                                unsigned long long *pout) {
    const int nb = (int)gridDim.x - (pcount ? 1 : 0);
    if ((int)blockIdx.x == nb) {
        sum_counts_body(pcount, pout);
        return;
    }
    copy_ranges(copy_k, copy_src, lu, lucsr, c, blockIdx.x, nb, blockDim.x);
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
typedef float float4_t __attribute__((ext_vector_type(4)));

// Two consecutive values of the factor type, for paired LDS reads and writes.
template <class T> struct Pair;
template <> struct Pair<double> { using type = double2; };
template <> struct Pair<float> { using type = float2; };

// Packed records, an item three int4, a pair two:
//   item[3i]   = {panel to factor or -1, first pair, end of pairs, panels factored}
//   item[3i+1] = {its first column s, width w, rows below r, slot of the diagonal of column s}
//   item[3i+2] = the same for the source of its first pair (zero without pairs)
// An item that factors several panels (consecutive panels of one supernode) factors them in
// order; its pairs list the pulls from outside first, then the pulls of each of its panels
// into the later ones, by source: a panel is factored before the first pull whose source
// it is, and after the pulls into it.
//   pair[2q]   = {source panel, slot of the source's first row in the target column,
//                 first index into rel, end of the group of q: the consecutive pairs of one
//                 source, at most kGroup, pulled together}
//   pair[2q+1] = {source's first column, width, rows below, slot of its first diagonal}
// T: the type in which the factor is stored and refactored (double, or float for the
// mixed-precision path).
template <class T>
struct RefArgs {
    const int32_t *ldiag;      // slot of the diagonal of each column
    const int4 *item;
    const int4 *pair;
    const int32_t *rel;
    T *lu;
    DevStatus *st;
    unsigned long long *pcount;   // replaced-pivot counter, spread over kCountSlots slots
    double tiny;
    int use_mfma;                 // dense update blocks on the matrix cores
    // row-ordered copy of the factor: lucsr[copy_k[q]] = lu[copy_src[q]] (copy_k: CSR
    // positions, copy_src: their factor slots)
    const int32_t *copy_k;
    const int32_t *copy_src;
    T *lucsr;
    // panel geometry (first column, rows below) for items that factor several panels
    const int32_t *pan_start;
    const int32_t *pan_r;
};

// the tiny-pivot threshold tiny * ||A~||_inf of the current refactorization, in T
template <class T>
__device__ __forceinline__ T pivot_threshold(const RefArgs<T> &a) {
    return (T)(a.tiny * a.st->anorm_scaled);
}

template <class T>
__device__ __forceinline__ T perturb(T p, T thresh, int &npert) {
    if (fabs(p) < thresh) {
        ++npert;
        return p < T(0) ? -thresh : thresh;
    }
    return p;
}

// ----------------------------------------------------------------- 16-lane path

// Source side of the update of target column k by a narrow source panel S (w <= kSmallW,
// r <= kSmallRows * kL), loaded by one group of kL lanes (16, or 4 for tiny items): S's
// diagonal block rows, its L rows and the slots of those rows in the target; lane gl holds
// rows gl, gl + kL, ...  Independent of the target's values, so the next pair's source side
// is loaded while the current pair is applied.
constexpr int kSmallRows = kSmallR / 16;
static_assert(kTinyR == kSmallRows * kTinyLanes, "tiny items fill the rows of a 4-lane group");
template <class T>
struct SmallSrc {
    int ps, w, r;
    int pos[kSmallRows];
    T l_row[kSmallW - 1];          // L(s + gl, s + j) for j < gl
    T lr[kSmallRows][kSmallW];     // L(R_i, s + j) for this lane's rows i
};

// pa, pb: the pair's record {ldiag[s+1], pos, rel, ldiag[s+2]}, {ldiag[s+3], w, r, ldiag[s]}
template <int kL, class T>
__device__ __forceinline__ void small_load_src(const RefArgs<T> &a, int4 pa, int4 pb, int gl, SmallSrc<T> &x) {
    const int ld[kSmallW] = {pb.w, pa.x, pa.w, pb.x};
    x.ps = pa.y;
    x.w = pb.y;
    x.r = pb.z;
    const int w = x.w, r = x.r;
    const int32_t *rel = a.rel + pa.z;
#pragma unroll
    for (int j = 0; j < kSmallW - 1; ++j) x.l_row[j] = (j + 1 < w && gl > j && gl < w) ? a.lu[ld[j] + (gl - j)] : T(0);
#pragma unroll
    for (int k = 0; k < kSmallRows; ++k) {
        const int i = gl + kL * k;
        x.pos[k] = i < r ? rel[i] : 0;
#pragma unroll
        for (int j = 0; j < kSmallW; ++j) x.lr[k][j] = (i < r && j < w) ? a.lu[ld[j] + 1 + (w - 1 - j) + i] : T(0);
    }
}

// Target side: rows s..s+w-1 of column k (from slot ps on) become final U entries (unit
// lower solve with S's diagonal block) and the rows R of S lose L(R, S) times them.
template <int kL, class T>
__device__ __forceinline__ void small_apply(const RefArgs<T> &a, const SmallSrc<T> &x, int gl) {
    const int w = x.w, r = x.r;
    // one round: the target's rows of S and of R
    T u = gl < w ? a.lu[x.ps + gl] : T(0);
    T tv[kSmallRows];
#pragma unroll
    for (int k = 0; k < kSmallRows; ++k) tv[k] = gl + kL * k < r ? a.lu[x.pos[k]] : T(0);
#pragma unroll
    for (int j = 0; j < kSmallW - 1; ++j) {
        const T uj = __shfl(u, j, kL);
        if (j + 1 < w && gl > j && gl < w) u = fma(-x.l_row[j], uj, u);
    }
    if (gl < w) a.lu[x.ps + gl] = u;
    T uu[kSmallW];
#pragma unroll
    for (int j = 0; j < kSmallW; ++j) uu[j] = __shfl(u, j, kL);
#pragma unroll
    for (int k = 0; k < kSmallRows; ++k) {
        if (gl + kL * k < r) {
            T acc = T(0);
#pragma unroll
            for (int j = 0; j < kSmallW; ++j)
                if (j < w) acc = fma(x.lr[k][j], uu[j], acc);
            a.lu[x.pos[k]] = tv[k] - acc;
        }
    }
    __threadfence_block();   // a later source of the same column may read these rows
}

// Dense LU without pivoting of a narrow panel's block column (w <= kSmallW,
// r <= kSmallRows * kL) by a group of kL lanes.  pn = {s, w, r, slot of the first
// diagonal}.  Returns the number of replaced pivots (the same value on every lane of the
// group).
template <int kL, class T>
__device__ __forceinline__ int small_factor(const RefArgs<T> &a, int4 pn, int ldg, int gl, T thresh) {
    const int w = pn.y, r = pn.z;
    int sg[kSmallW];
#pragma unroll
    for (int c = 0; c < kSmallW; ++c) sg[c] = __shfl(ldg, c, kL) - c;
    // one round: the diagonal block (lane gl < w holds row gl) and this lane's rows below
    T d[kSmallW];
#pragma unroll
    for (int c = 0; c < kSmallW; ++c) d[c] = (c < w && gl < w) ? a.lu[sg[c] + gl] : T(0);
    constexpr int kRows = kSmallRows;
    T x[kRows][kSmallW];
#pragma unroll
    for (int k = 0; k < kRows; ++k)
#pragma unroll
        for (int c = 0; c < kSmallW; ++c) x[k][c] = (c < w && gl + kL * k < r) ? a.lu[sg[c] + w + gl + kL * k] : T(0);
    int npert = 0, bad = 0;
    T U[kSmallW][kSmallW];   // final U of the diagonal block, known to every lane
#pragma unroll
    for (int jj = 0; jj < kSmallW; ++jj) {
        if (jj < w) {
            T ur[kSmallW];
#pragma unroll
            for (int c = 0; c < kSmallW; ++c) ur[c] = __shfl(d[c], jj, kL);
            const T p = perturb(ur[jj], thresh, npert);
            bad |= !isfinite(p);
            if (gl == jj) d[jj] = p;
            ur[jj] = p;
#pragma unroll
            for (int c = 0; c < kSmallW; ++c) U[jj][c] = ur[c];
            if (gl > jj && gl < w) {
                const T l = d[jj] / p;
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
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        if (gl + kL * k < r) {
#pragma unroll
            for (int jj = 0; jj < kSmallW; ++jj) {
                if (jj < w) {
                    const T l = x[k][jj] / U[jj][jj];
                    bad |= !isfinite(l);
                    x[k][jj] = l;
#pragma unroll
                    for (int c = jj + 1; c < kSmallW; ++c)
                        if (c < w) x[k][c] = fma(-l, U[jj][c], x[k][c]);
                }
            }
#pragma unroll
            for (int c = 0; c < kSmallW; ++c)
                if (c < w) a.lu[sg[c] + w + gl + kL * k] = x[k][c];
        }
    }
    if (bad) atomicOr(&a.st->flags, kFlagNonfinite);
    return npert;
}

// One item per group of kL lanes (16; 4 for tiny items, whose panels have at most kTinyR
// rows below, so a wavefront keeps four times as many of them in flight).  kPipe: the next
// pair's source side is loaded while the current pair is applied (fewer dependent rounds
// per item, more registers: for levels with few items); otherwise one pair at a time (more
// items in flight).  Group g runs narrow item item0 + g when g < nsmall; the wavefront's
// perturbed pivots go to counter slot `slot`.  No block-wide synchronisation: the groups of
// a block are independent.  Every entry receives the same operations in the same order
// whatever kL is.
template <class T, bool kPipe, int kL = 16>
__device__ __forceinline__ void small_group(int item0, int nsmall, const RefArgs<T> &a, int g, int slot) {
    const T thresh = pivot_threshold(a);
    const int gl = threadIdx.x & (kL - 1);
    int npert = 0;
    if (g < nsmall) {
        const int item = item0 + g;
        const int4 ia = a.item[3 * item], ib = a.item[3 * item + 1];
        // one round: the records of up to kL pairs (lane t holds pair p0 + t) and the
        // diagonal slots of the panel to factor
        const int p0 = ia.y, np = ia.z - ia.y;
        int4 ra = int4{0, 0, 0, 0}, rb = int4{0, 0, 0, 0};
        if (gl < np) {
            ra = a.pair[2 * (p0 + gl)];
            rb = a.pair[2 * (p0 + gl) + 1];
        }
        const int ldg = (ia.x >= 0 && ib.y > 1 && gl > 0 && gl < ib.y) ? a.ldiag[ib.x + gl] : ib.w;
        auto rec = [&](int q, int4 &pa, int4 &pb) {
            if (q >= kL) {   // items with more than kL pairs read the rest on demand
                pa = a.pair[2 * (p0 + q)];
                pb = a.pair[2 * (p0 + q) + 1];
                return;
            }
            pa = int4{__shfl(ra.x, q, kL), __shfl(ra.y, q, kL), __shfl(ra.z, q, kL), __shfl(ra.w, q, kL)};
            pb = int4{__shfl(rb.x, q, kL), __shfl(rb.y, q, kL), __shfl(rb.z, q, kL), __shfl(rb.w, q, kL)};
        };
        if constexpr (kPipe) {
            if (np > 0) {
                SmallSrc<T> cur, nxt;
                int4 pa, pb;
                rec(0, pa, pb);
                small_load_src<kL>(a, pa, pb, gl, cur);
                for (int q = 0; q < np; ++q) {
                    if (q + 1 < np) {
                        rec(q + 1, pa, pb);
                        small_load_src<kL>(a, pa, pb, gl, nxt);
                    }
                    small_apply<kL>(a, cur, gl);
                    cur = nxt;
                }
            }
        } else {
            for (int q = 0; q < np; ++q) {
                SmallSrc<T> cur;
                int4 pa, pb;
                rec(q, pa, pb);
                small_load_src<kL>(a, pa, pb, gl, cur);
                small_apply<kL>(a, cur, gl);
            }
        }
        if (ia.x >= 0) npert = small_factor<kL>(a, ib, ldg, gl, thresh);
    }
    // one counter update per wavefront: group leaders contribute their count
    int c = gl == 0 ? npert : 0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(&a.pcount[slot % kCountSlots], (unsigned long long)c);
}

template <class T>
__device__ __forceinline__ void copy_block(const RefArgs<T> &a, const CopyRanges &c, int b, int nb, int nthreads) {
    copy_ranges(a.copy_k, a.copy_src, a.lu, a.lucsr, c, b, nb, nthreads);
}

// A level without wide items: its nsmall narrow items, the last ntiny of them tiny.  The
// first blocks run the others, kBlock / 16 to a block, the next ones the tiny items,
// kBlock / kTinyLanes to a block; the blocks after them copy the ranges c of the
// row-ordered factor (columns final before the launch)
template <class T, bool kPipe>
__global__ __launch_bounds__(256) void k_refactor_small(int item0, int nsmall, int ntiny, RefArgs<T> a,
                                                        CopyRanges c) {
    const int nn = nsmall - ntiny;
    const int nsb = (nn + kBlock / 16 - 1) / (kBlock / 16);
    const int ntb = (ntiny + kBlock / kTinyLanes - 1) / (kBlock / kTinyLanes);
    const int b = blockIdx.x, slot = b * 4 + (threadIdx.x >> 6);
    if (b < nsb) {
        small_group<T, kPipe>(item0, nn, a, b * (kBlock / 16) + (threadIdx.x >> 4), slot);
    } else if (b < nsb + ntb) {
        small_group<T, kPipe, kTinyLanes>(item0 + nn, ntiny, a,
                                          (b - nsb) * (kBlock / kTinyLanes) + (threadIdx.x / kTinyLanes), slot);
    } else {
        copy_block(a, c, b - nsb - ntb, gridDim.x - nsb - ntb, kBlock);
    }
}

// ----------------------------------------------------------------- 512-thread path

constexpr int kStagePairs = 256;

// LDS row stride (values) of per-lane rows that the lanes of a wavefront read or write at
// the same column at once: FP64 rows start four banks apart, so 16 consecutive lanes touch
// distinct banks, and the alignment of paired reads is kept
constexpr int kRowLd = kPanelMax + 2;

// Update tiles on the matrix cores, 16x16 outputs with k in steps of 4: lane holds
// A[lane % 16][lane / 16] and B[lane / 16][lane % 16]; its four outputs are rows row(lk, v)
// (lk = lane / 16, v = 0..3) of column lane % 16 (the FP64 and FP32 instructions place them
// differently).
template <class T> struct Mfma;
template <> struct Mfma<double> {
    using acc_t = double4_t;
    static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <> struct Mfma<float> {
    using acc_t = float4_t;
    static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

// Configurations of the wide path: threads per block, minimum waves per SIMD, source L rows
// staged per chunk, widest panel (target and sources) and update tiles per wavefront and
// pass.  LDS layout (bytes): Ld (the pivot rows of the panel being factored) | Ub (solved
// rows per target) | Lr (a chunk of the source's L rows) | lds (the diagonal slots of the
// current and the next group's source, two buffers) | sgs (slot of row s in each column of
// the panel to factor) | flg (pivot rows published by the panel sweep) | staged pair
// records.
template <class TV, int NT, int WV, int CH, int MW, int TI>
struct WideCfg {
    using T = TV;   // factor type
    static constexpr int kThreads = NT;
    static constexpr int kWaves = WV;
    static constexpr int kChunk = CH;
    static constexpr int kMaxW = MW;
    static constexpr int kTiles = TI;
    static constexpr int kOffLd = 0;
    static constexpr int kOffUb = kOffLd + kMaxW * kPanelMax * (int)sizeof(T);
    static constexpr int kOffLr = kOffUb + kRowLd * kGroup * (int)sizeof(T);
    static constexpr int kOffLds = kOffLr + kChunk * kMaxW * (int)sizeof(T);
    static constexpr int kOffSgs = kOffLds + 2 * kPanelMax * 4;
    static constexpr int kOffFlg = kOffSgs + kPanelMax * 4;
    static constexpr int kOffPairs = kOffFlg + kPanelMax * 4;
    static constexpr int kLds = kOffPairs + kStagePairs * 32;
    static_assert(kOffPairs % 16 == 0, "staged pair records are read as int4");
};
// panels up to 32 columns: one block per CU
template <class T> using BigCfg = WideCfg<T, 512, 2, 256, 32, 4>;
// panels up to 16 columns: four blocks per CU
template <class T> using MedCfg = WideCfg<T, 256, 4, 128, 16, 2>;
// panels up to 32 columns whose factored panels have at most 256 rows: two blocks per CU
template <class T> using W256Cfg = WideCfg<T, 256, 2, 128, 32, 4>;

// Panel sweeps in registers.  A row of a panel of width w <= KW lives in registers
// x[0..KW-1] with zeros past column w.  Step j of the elimination consumes x[0] (column j)
// and moves the remaining columns down by one while it applies the step's update, so every
// register index is static while the loop over j stays rolled; the update of column c at
// step j is the same FMA, in the same order, as in the unshifted form.
// The window narrows in four phases of K_p = KW, 3KW/4, KW/2, KW/4 registers: phase p runs
// steps [b_p, b_{p+1}), b_0 = 0, b_{p+1} = max(b_p, w - K_{p+1}), b_4 = w, so that no step
// carries more than KW/4 columns past the panel's remaining ones.
// The register freed at the top of the window takes, for a row of the diagonal block (a
// future pivot row), a zero, so that its window holds zeros past its remaining columns when
// it is published; such a row keeps its multipliers in LDS.  A row below the block takes its
// multiplier L(row, j) there instead: phase p's n_p = b_{p+1} - b_p multipliers then sit, in
// order, in registers [K_p - n_p, K_p) when the sweep ends (K_p - n_p >= K_{p+1}, so later
// phases leave them alone), and stay in registers until the panel is stored.
// The pivot row (LDS, 16-byte aligned) is read into registers in one round before the FMAs;
// otherwise the compiler interleaves one LDS round trip per pair of columns.
template <int KW, class T>
__device__ __forceinline__ void load_lds_row(T (&rw)[kPanelMax], const T *row) {
    using P2 = typename Pair<T>::type;
    const P2 *r2 = reinterpret_cast<const P2 *>(row);
#pragma unroll
    for (int c = 0; c < KW / 2; ++c) {
        const P2 v = r2[c];
        rw[2 * c] = v.x;
        rw[2 * c + 1] = v.y;
    }
}

// x[c] = lu[base[c] + off] for c < w, 0 beyond (every address in bounds)
template <int KW, class T>
__device__ __forceinline__ void load_row(T (&x)[kPanelMax], const T *lu, const int *base, int w, int off) {
#pragma unroll
    for (int c = 0; c < KW; ++c) {
        const T v = lu[base[c < w ? c : 0] + off];
        x[c] = c < w ? v : T(0);
    }
}

// window sizes of the four phases of a sweep of width class KW
template <int KW> struct Phases {
    static constexpr int K0 = KW, K1 = 3 * KW / 4, K2 = KW / 2, K3 = KW / 4;
    static_assert(K3 >= 2 && K3 % 2 == 0, "even windows of at least two columns");
};

// first steps b[0..4] of the four phases of a sweep of w columns
template <int KW>
__device__ __forceinline__ void phase_bounds(int w, int (&b)[5]) {
    using P = Phases<KW>;
    b[0] = 0;
    b[1] = max(b[0], w - P::K1);
    b[2] = max(b[1], w - P::K2);
    b[3] = max(b[2], w - P::K3);
    b[4] = w;
}

// One step of the panel sweep on a row (window K) with pivot row urow; a row of the diagonal
// block (diag) stores its multiplier to *lslot.
template <int K, class T>
__device__ __forceinline__ void sweep_step(T (&x)[kPanelMax], const T *urow, bool diag, T *lslot, int &bad) {
    T rw[kPanelMax];
    load_lds_row<K>(rw, urow);
    __builtin_amdgcn_sched_barrier(0);
    const T l = x[0] / rw[0];
    bad |= !isfinite(l);
#pragma unroll
    for (int c = 1; c < K; ++c) x[c - 1] = fma(-l, rw[c], x[c]);
    x[K - 1] = diag ? T(0) : l;
    if (diag) *lslot = l;
}

// Stores the multipliers L(row, i), i < w, of a row below the diagonal block after the whole
// sweep to lu[sgs[i] + row]: register c belongs to the phase p with K_{p+1} <= c < K_p.
template <int KW, class T>
__device__ __forceinline__ void store_multipliers(const T (&x)[kPanelMax], T *lu, const int *sgs, int row,
                                                  const int (&b)[5]) {
    using P = Phases<KW>;
#pragma unroll
    for (int c = 0; c < KW; ++c) {
        const int p = c >= P::K1 ? 0 : c >= P::K2 ? 1 : c >= P::K3 ? 2 : 3;
        const int kp = p == 0 ? P::K0 : p == 1 ? P::K1 : p == 2 ? P::K2 : P::K3;
        const int first = kp - (b[p + 1] - b[p]);
        if (c >= first) lu[sgs[b[p] + c - first] + row] = x[c];
    }
}

// Dense LU without pivoting of a wide panel's block column (w + r rows, w columns).  The
// block's threads own one panel row each: wavefront 0 rows 0..63 (the diagonal block and the
// first L rows), the others 64 rows each, the wavefront that shares wavefront 0's SIMD last
// (for 512 threads), so that wavefront 0 runs alone on its SIMD for panels of up to 448
// rows.  Wavefront 0 runs the whole sweep without waiting: at step j lane j perturbs its
// pivot if tiny, publishes its window U(j, j..) in LDS (Us[j * kPanelMax + c] = U(j, j + c),
// zero past the panel) and raises flg[j] (ordered after the row by an LDS-only release), and
// every later row of the wavefront takes its multiplier and update from it.  The other
// wavefronts follow, waiting (bounded) on flg[j] before step j.  No global memory operation
// is outstanding inside the sweep: the multipliers stay in registers or LDS and are stored
// when it ends.  Rows beyond the threads of the block are eliminated afterwards from the
// finished Us.  sgs[c] = slot of row s in column s + c (staged by the caller); row t of the
// panel is at slot sgs[c] + t.  The diagonal block's multipliers go to Ltri (the chunk area
// of the pulls, free here): Ltri[t * kPanelMax + j] = L(t, j).
constexpr int kSweepSpin = 1 << 22;

template <class C, int KW>
__device__ __forceinline__ void large_factor_w(const RefArgs<typename C::T> &a, int w, int r, char *sm,
                                               typename C::T thresh) {
    using T = typename C::T;
    using P2 = typename Pair<T>::type;
    using P = Phases<KW>;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    T *Us = reinterpret_cast<T *>(sm + C::kOffLd);
    T *Ltri = reinterpret_cast<T *>(sm + C::kOffLr);
    const int *sgs = reinterpret_cast<const int *>(sm + C::kOffSgs);
    int *flg = reinterpret_cast<int *>(sm + C::kOffFlg);
    const int nrow = w + r;
    const int row = (C::kThreads == 512 ? (wv < 4 ? wv : wv == 4 ? 7 : wv - 1) : wv) * 64 + lane;
    const bool diag = row < w;
    int b[5];
    phase_bounds<KW>(w, b);
    int npert = 0, bad = 0;
    T x[kPanelMax];
#pragma unroll
    for (int c = 0; c < kPanelMax; ++c) x[c] = T(0);
    if (row < nrow) load_row<KW>(x, a.lu, sgs, w, row);
    if (tid < kPanelMax) flg[tid] = 0;
    lds_barrier();
    if (wv == 0) {
        auto run = [&](auto kc, int j0, int j1) {
            constexpr int K = decltype(kc)::value;
#pragma unroll 1
            for (int j = j0; j < j1; ++j) {
                if (lane == j) {
                    x[0] = perturb(x[0], thresh, npert);
                    bad |= !isfinite(x[0]);
                    P2 *o = reinterpret_cast<P2 *>(Us + j * kPanelMax);
#pragma unroll
                    for (int c = 0; c < K / 2; ++c) o[c] = P2{x[2 * c], x[2 * c + 1]};
                }
                // this wavefront's own reads of row j follow its writes in LDS order; the
                // compiler is kept from moving them ahead (no instruction is emitted)
                __builtin_amdgcn_wave_barrier();
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                if (lane > j && row < nrow)
                    sweep_step<K>(x, Us + j * kPanelMax, diag, Ltri + lane * kPanelMax + j, bad);
                if (lane == j) {
                    // the other wavefronts may read row j once it is complete in LDS (long
                    // since, by now: the wait is off the sweep's chain)
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                    __hip_atomic_store(flg + j, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        };
        run(std::integral_constant<int, P::K0>{}, b[0], b[1]);
        run(std::integral_constant<int, P::K1>{}, b[1], b[2]);
        run(std::integral_constant<int, P::K2>{}, b[2], b[3]);
        run(std::integral_constant<int, P::K3>{}, b[3], b[4]);
    } else if (row - lane < nrow) {             // a wavefront with rows to eliminate
        bool ok = true;
        auto run = [&](auto kc, int j0, int j1) {
            constexpr int K = decltype(kc)::value;
#pragma unroll 1
            for (int j = j0; j < j1 && ok; ++j) {
                int spin = 0;
                while (__hip_atomic_load(flg + j, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == 0) {
                    if (++spin > kSweepSpin) break;
                    __builtin_amdgcn_s_sleep(1);
                }
                if (spin > kSweepSpin) {
                    if (lane == 0) atomicOr(&a.st->flags, kFlagInternal);
                    ok = false;
                } else if (row < nrow) {
                    sweep_step<K>(x, Us + j * kPanelMax, false, Ltri, bad);
                }
            }
        };
        run(std::integral_constant<int, P::K0>{}, b[0], b[1]);
        run(std::integral_constant<int, P::K1>{}, b[1], b[2]);
        run(std::integral_constant<int, P::K2>{}, b[2], b[3]);
        run(std::integral_constant<int, P::K3>{}, b[3], b[4]);
    }
    lds_barrier();
    // U rows of the diagonal block (diagonal included) from LDS: row j's window covers its
    // w - j remaining columns
    for (int t = tid; t < w * KW; t += C::kThreads) {
        const int j = t / KW, c = t % KW;
        if (j + c < w) a.lu[sgs[j + c] + j] = Us[j * kPanelMax + c];
    }
    // multipliers of the diagonal block from LDS, of the rows below it from registers
    for (int t = tid; t < w * kPanelMax; t += C::kThreads) {
        const int i = t / kPanelMax, j = t % kPanelMax;
        if (j < i) a.lu[sgs[j] + i] = Ltri[t];
    }
    if (!diag && row < nrow) store_multipliers<KW>(x, a.lu, sgs, row, b);
    // rows beyond the threads of the block
    for (int i = tid + C::kThreads; i < nrow; i += C::kThreads) {
        load_row<KW>(x, a.lu, sgs, w, i);
#pragma unroll 1
        for (int j = b[0]; j < b[1]; ++j) sweep_step<P::K0>(x, Us + j * kPanelMax, false, Ltri, bad);
#pragma unroll 1
        for (int j = b[1]; j < b[2]; ++j) sweep_step<P::K1>(x, Us + j * kPanelMax, false, Ltri, bad);
#pragma unroll 1
        for (int j = b[2]; j < b[3]; ++j) sweep_step<P::K2>(x, Us + j * kPanelMax, false, Ltri, bad);
#pragma unroll 1
        for (int j = b[3]; j < b[4]; ++j) sweep_step<P::K3>(x, Us + j * kPanelMax, false, Ltri, bad);
        store_multipliers<KW>(x, a.lu, sgs, i, b);
    }
    if (npert) atomicAdd(&a.pcount[blockIdx.x % kCountSlots], (unsigned long long)npert);   // row j counts pivot j
    if (__any(bad) && lane == 0) atomicOr(&a.st->flags, kFlagNonfinite);
}

template <class C>
__device__ __forceinline__ void large_factor(const RefArgs<typename C::T> &a, int4 pn, char *sm,
                                             typename C::T thresh) {
    // the panel's geometry is the same for the whole block: scalar from here on
    pn.y = __builtin_amdgcn_readfirstlane(pn.y);
    pn.z = __builtin_amdgcn_readfirstlane(pn.z);
    if constexpr (C::kMaxW > 16) {
        if (pn.y > 16) {
            large_factor_w<C, 32>(a, pn.y, pn.z, sm, thresh);
            return;
        }
    }
    if (pn.y > 8) large_factor_w<C, 16>(a, pn.y, pn.z, sm, thresh);
    else large_factor_w<C, 8>(a, pn.y, pn.z, sm, thresh);
}

// Rows of the source panel S (width w) in the targets of a group: the unit lower solve
// U(S, t) = L_SS^-1 A(S, t) for each target column t.  Wavefront v takes targets v, v + nw,
// ... (NT of them); lane c < w holds row c of S in each (u[k]).  Lcol holds the columns of
// L_SS in LDS, unshifted: Lcol[j * kPanelMax + c] = L(c, j) for j < c < w, zero for c <= j.
// Step j broadcasts the finished entry of row j of each target (readlane) and applies it to
// the rows below it (lanes c <= j add zero products), so every entry receives the same FMAs
// in the same order as a row-by-row forward substitution.  The next step's column is read
// while the current one is applied.
template <int NT, class T>
__device__ __forceinline__ void lower_run(const T *Lcol, T (&u)[NT], int w, int lane) {
    T l = Lcol[lane];
#pragma unroll 1
    for (int j = 0; j + 1 < w; ++j) {
        const T ln = Lcol[(j + 1) * kPanelMax + lane];
#pragma unroll
        for (int k = 0; k < NT; ++k) u[k] = fma(-l, bcast(u[k], j), u[k]);
        l = ln;
    }
}

// All pulls of one item, one group (one source S, up to kGroup target columns) at a time,
// then the panel factorization.  Per group: the loads of the update's destination slots and
// current values, of S's first chunk of L rows and of the lower solve's operands are issued
// together; the lower solve runs on all wavefronts; the update of the rows R of the targets
// runs on the matrix cores (16x16 tiles of Lr (nr x w) times the solved rows (w x m)).  The
// diagonal slots of the next group's source are loaded during the current group.
template <class C>
__device__ __forceinline__ void wide_item(const int item, const RefArgs<typename C::T> &a, char *sm) {
    using T = typename C::T;
    using MM = Mfma<T>;
    const T thresh = pivot_threshold(a);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int nw = C::kThreads / 64;
    constexpr int NT = (kGroup + nw - 1) / nw;       // targets per wavefront in the lower solve
    constexpr int kJ = C::kThreads / C::kChunk;      // source columns staged per round
    constexpr int kLr = C::kMaxW / kJ;               // rounds
    constexpr int kTiles = C::kTiles;
    static_assert(C::kThreads % C::kChunk == 0 && C::kMaxW % kJ == 0, "staging rounds");
    T *Ub = reinterpret_cast<T *>(sm + C::kOffUb);
    T *Lr = reinterpret_cast<T *>(sm + C::kOffLr);
    int *ldsb = reinterpret_cast<int *>(sm + C::kOffLds);
    int *sgs = reinterpret_cast<int *>(sm + C::kOffSgs);
    int4 *prs = reinterpret_cast<int4 *>(sm + C::kOffPairs);
    const int4 ia = a.item[3 * item], ib = a.item[3 * item + 1], ic = a.item[3 * item + 2];
    const int pbeg = ia.y, p1 = ia.z;
    const int npan = ia.x >= 0 ? max(1, ia.w) : 0;
    int done = 0;   // panels of the item factored so far
    // pair records pbeg .. are staged in LDS, kStagePairs at a time: a window [wbeg, wend)
    // holds the current group and the first pair of the next one
    int wbeg = pbeg, wend = min(p1, pbeg + kStagePairs);
    // one round: the pair records, the slots of the (first) panel to factor and the
    // diagonal slots of the first group's source
    for (int t = tid; t < 2 * (wend - wbeg); t += C::kThreads) prs[t] = a.pair[2 * wbeg + t];
    if (ia.x >= 0 && tid < ib.y) sgs[tid] = a.ldiag[ib.x + tid] - tid;
    if (p1 > pbeg && tid < ic.y) ldsb[tid] = tid == 0 ? ic.w : a.ldiag[ic.x + tid];
    lds_barrier();
    auto pra = [&](int q) { return prs[2 * (q - wbeg)]; };
    auto prb = [&](int q) { return prs[2 * (q - wbeg) + 1]; };
    // factors the item's next panel (the first one's geometry is ib, the others' is read)
    auto factor_next = [&]() {
        int4 pn = ib;
        if (done > 0) {
            const int P = ia.x + done;
            const int s0 = a.pan_start[P];
            pn = int4{s0, a.pan_start[P + 1] - s0, a.pan_r[P], a.ldiag[s0]};
            if (tid < pn.y) sgs[tid] = a.ldiag[s0 + tid] - tid;
            __syncthreads();
        }
        large_factor<C>(a, pn, sm, thresh);
        // the factored panel is read by the item's later pulls
        __threadfence_block();
        __syncthreads();
        ++done;
    };
    const int li = lane & 15, lk = lane >> 4;
    // destination slots of the four outputs of this lane in update tile `tile` of a group
    // (g0, m targets; mt row tiles of a chunk of nr rows from i0): q[v], valid where ok[v].
    // A group has at most kGroup = 32 targets, so tile / mt is 0 or 1.  The loads are only
    // issued here; their values are consumed later.
    auto tile_slots = [&](int g0, int m, int tile, int mt, int nr, int i0, int (&q)[4], bool (&ok)[4]) {
        const int tt = tile >= mt ? 1 : 0, ti = tile - tt * mt, tb = tt * 16 + li;
        const bool okt = tile < 2 * mt && tb < m;
        const int rb = pra(g0 + (okt ? tb : 0)).z + i0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = ti * 16 + MM::row(lk, v);
            ok[v] = okt && i < nr;
            q[v] = a.rel[rb + (ok[v] ? i : 0)];
        }
    };
    int buf = 0;
    for (int g0 = pbeg, g1; g0 < p1; g0 = g1, buf ^= 1) {
        if (wend < p1 && g0 + kGroup >= wend) {
            // the group or the next one's first pair is past the staged window: restage
            // from g0 (every wavefront is done with the records of the previous groups)
            wbeg = g0;
            wend = min(p1, g0 + kStagePairs);
            for (int t = tid; t < 2 * (wend - wbeg); t += C::kThreads) prs[t] = a.pair[2 * wbeg + t];
            __syncthreads();
        }
        const int4 pa0 = pra(g0);
        const int S = pa0.x;
        g1 = __builtin_amdgcn_readfirstlane(pa0.w);
        // a pull from one of the item's own panels: factor the panels up to it first
        while (done < npan && S >= ia.x + done && S < ia.x + npan) factor_next();
        const int4 pn = prb(g0);
        const int w = __builtin_amdgcn_readfirstlane(pn.y), r = __builtin_amdgcn_readfirstlane(pn.z);
        const int m = g1 - g0;
        const int *lds = ldsb + buf * kPanelMax;
        // the next group's diagonal slots, stored to the other buffer when this group ends
        int ndiag = 0, ndiag0 = 0;
        bool nstore = false;
        if (g1 < p1) {
            const int4 pq = prb(g1);
            nstore = tid < pq.y;
            ndiag = a.ldiag[nstore ? pq.x + tid : 0];
            ndiag0 = pq.w;
        }
        const bool mf = a.use_mfma && m > 1;
        const int nt = (m + 15) >> 4;
        const int nr0 = min(C::kChunk, r), mt0 = (nr0 + 15) >> 4;
        // (1) destination slots of this wavefront's first update tiles
        int pslot[kTiles][4];
        bool pok[kTiles][4];
        T pcur[kTiles][4];
        if (mf) {
#pragma unroll
            for (int k = 0; k < kTiles; ++k) tile_slots(g0, m, wv * kTiles + k, mt0, nr0, 0, pslot[k], pok[k]);
        }
        // (2) the first chunk of S's L rows: column j = lj + k kJ, row lrow of the chunk
        const int lrow = tid % C::kChunk, lj = tid / C::kChunk;
        T lv[kLr];
#pragma unroll
        for (int k = 0; k < kLr; ++k) {
            const int j = lj + k * kJ, dj = lds[j];
            const bool ok = lrow < nr0 && j < w;
            lv[k] = a.lu[ok ? dj + 1 + (w - 1 - j) + lrow : 0];
        }
        // (3) the columns of L_SS (entry e = j kPanelMax + c of Lcol: L(c, j), zero unless
        // j < c < w) and the rows of S in this wavefront's targets
        constexpr int kLc = C::kMaxW * kPanelMax / C::kThreads;
        static_assert(C::kMaxW * kPanelMax % C::kThreads == 0, "Lcol rounds");
        T lc[kLc];
#pragma unroll
        for (int k = 0; k < kLc; ++k) {
            const int e = tid + k * C::kThreads, j = e / kPanelMax, c = e % kPanelMax, dj = lds[j];
            lc[k] = a.lu[j < c && c < w ? dj + (c - j) : 0];
        }
        int ps[NT], tg[NT];
        bool own[NT];
        T u[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            tg[k] = wv + k * nw;
            own[k] = tg[k] < m && lane < w;
            ps[k] = pra(g0 + (tg[k] < m ? tg[k] : 0)).y;
            u[k] = a.lu[own[k] ? ps[k] + lane : 0];
        }
        // (4) the chunk and the columns to LDS
#pragma unroll
        for (int k = 0; k < kLr; ++k) {
            const int j = lj + k * kJ;
            if (lrow < nr0 && j < w) Lr[j * C::kChunk + lrow] = lv[k];
        }
        T *Lcol = reinterpret_cast<T *>(sm + C::kOffLd);
#pragma unroll
        for (int k = 0; k < kLc; ++k) {
            const int e = tid + k * C::kThreads, j = e / kPanelMax, c = e % kPanelMax;
            Lcol[e] = j < c && c < w ? lc[k] : T(0);
        }
#pragma unroll
        for (int k = 0; k < NT; ++k) u[k] = own[k] ? u[k] : T(0);
        lds_barrier();
        // (5) the lower solve on every wavefront; the solved rows to the factor and to Ub;
        // then the current values at the slots (in flight during the barrier and the products)
        lower_run<NT>(Lcol, u, w, lane);
#pragma unroll
        for (int k = 0; k < NT; ++k)
            if (own[k]) {
                a.lu[ps[k] + lane] = u[k];
                Ub[tg[k] * kRowLd + lane] = u[k];
            }
        if (mf) {
#pragma unroll
            for (int k = 0; k < kTiles; ++k)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    pslot[k][v] = pok[k][v] ? pslot[k][v] : -1;
                    pcur[k][v] = a.lu[pok[k][v] ? pslot[k][v] : 0];
                }
        }
        lds_barrier();   // Ub is complete; the loads and stores above stay in flight
        // rows R of each target: chunks of S's L rows in LDS, precomputed slots
        for (int i0 = 0; i0 < r; i0 += C::kChunk) {
            const int nr = min(C::kChunk, r - i0);
            if (i0 > 0) {
                lds_barrier();   // every wavefront is done with the previous chunk
#pragma unroll
                for (int k = 0; k < kLr; ++k) {
                    const int j = lj + k * kJ, dj = lds[j];
                    const bool ok = lrow < nr && j < w;
                    lv[k] = a.lu[ok ? dj + 1 + (w - 1 - j) + i0 + lrow : 0];
                }
#pragma unroll
                for (int k = 0; k < kLr; ++k) {
                    const int j = lj + k * kJ;
                    if (lrow < nr && j < w) Lr[j * C::kChunk + lrow] = lv[k];
                }
                lds_barrier();
            }
            if (mf) {
                const int mt = (nr + 15) >> 4;
                for (int tile0 = wv * kTiles, pass = 0; tile0 < mt * nt; tile0 += nw * kTiles, ++pass) {
                    typename MM::acc_t acc[kTiles];
#pragma unroll
                    for (int k = 0; k < kTiles; ++k) acc[k] = typename MM::acc_t{T(0), T(0), T(0), T(0)};
                    int ia2[kTiles], tb[kTiles];
                    bool okt[kTiles];
#pragma unroll
                    for (int k = 0; k < kTiles; ++k) {
                        const int tile = tile0 + k, tt = tile >= mt ? 1 : 0;
                        okt[k] = tile < mt * nt;
                        ia2[k] = (tile - tt * mt) * 16 + li;
                        tb[k] = tt * 16 + li;
                    }
                    for (int k0 = 0; k0 < w; k0 += 4) {
                        const int kk = k0 + lk;
                        T av[kTiles], bv[kTiles];
#pragma unroll
                        for (int k = 0; k < kTiles; ++k) {
                            const bool ok = okt[k] && kk < w;
                            av[k] = (ok && ia2[k] < nr) ? Lr[kk * C::kChunk + ia2[k]] : T(0);
                            bv[k] = (ok && tb[k] < m) ? Ub[tb[k] * kRowLd + kk] : T(0);
                        }
#pragma unroll
                        for (int k = 0; k < kTiles; ++k) acc[k] = MM::step(av[k], bv[k], acc[k]);
                    }
                    int slot[kTiles][4];
                    T cur[kTiles][4];
                    if (i0 == 0 && pass == 0) {
#pragma unroll
                        for (int k = 0; k < kTiles; ++k)
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                slot[k][v] = pslot[k][v];
                                cur[k][v] = pcur[k][v];
                            }
                    } else {
#pragma unroll
                        for (int k = 0; k < kTiles; ++k) {
                            bool ok[4];
                            tile_slots(g0, m, tile0 + k, mt, nr, i0, slot[k], ok);
#pragma unroll
                            for (int v = 0; v < 4; ++v) slot[k][v] = ok[v] ? slot[k][v] : -1;
                        }
#pragma unroll
                        for (int k = 0; k < kTiles; ++k)
#pragma unroll
                            for (int v = 0; v < 4; ++v) cur[k][v] = a.lu[slot[k][v] >= 0 ? slot[k][v] : 0];
                    }
#pragma unroll
                    for (int k = 0; k < kTiles; ++k)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (slot[k][v] >= 0) a.lu[slot[k][v]] = cur[k][v] - acc[k][v];
                }
            } else {
                for (int q = g0 + wv; q < g1; q += nw) {
                    const int32_t *rel = a.rel + pra(q).z + i0;
                    const T *ub = Ub + (q - g0) * kRowLd;
                    for (int i = lane; i < nr; i += 64) {
                        T acc = T(0);
                        for (int j = 0; j < w; ++j) acc = fma(Lr[j * C::kChunk + i], ub[j], acc);
                        a.lu[rel[i]] -= acc;
                    }
                }
            }
        }
        if (nstore) ldsb[(buf ^ 1) * kPanelMax + tid] = tid == 0 ? ndiag0 : ndiag;
        // the updated targets are read by the item's factorization
        __threadfence_block();
        __syncthreads();
    }
    while (done < npan) factor_next();
}

// One launch per level: block b < nwide runs wide item item0 + b; the next f.nsolve blocks
// run the forward-solve items f.j0 .. f.j1 - 1 (one forward level; they read only columns and
// unknowns final before the launch), ahead of the narrow items so that they start beside the
// factor work; the next ones run the level's narrow items small0 .. small0 + nsmall - 1,
// C::kThreads / 16 to a block (they touch other columns than the wide items, so one launch
// needs no ordering between them); any blocks after those copy the ranges c of the
// row-ordered factor (columns that no launch from this one on writes).
// Block blk of nblk of one level launch (the work of one handle: its wide items, narrow
// items and copy chunk).
template <class TF> struct SolveArgs;
// the forward items [j0, j1) of the solve s (one forward level: independent items) run by
// nsolve extra blocks of a refactor launch
template <class T> struct FuseArgs {
    SolveArgs<T> s;
    int j0, j1, nsolve;
};
template <class T> __device__ void fused_forward_block(const FuseArgs<T> &f, int blk, char *sm);

template <class C>
__device__ __forceinline__ void refactor_block(int blk, int nblk, int item0, const RefArgs<typename C::T> &a,
                                               int nwide, int small0, int nsmall, const CopyRanges &c,
                                               const FuseArgs<typename C::T> &f, char *sm) {
    const int nsb = (nsmall + C::kThreads / 16 - 1) / (C::kThreads / 16);
    if (blk >= nwide && blk < nwide + f.nsolve) {
        fused_forward_block(f, blk - nwide, sm);
        return;
    }
    if (blk >= nwide + f.nsolve + nsb) {
        const int b = blk - nwide - f.nsolve - nsb, nbc = nblk - nwide - f.nsolve - nsb;
        copy_block(a, c, b, nbc, C::kThreads);
        return;
    }
    if (blk >= nwide) {
        const int b = blk - nwide - f.nsolve;
        small_group<typename C::T, (C::kMaxW > 16)>(small0, nsmall, a, b * (C::kThreads / 16) + (threadIdx.x >> 4),
                                                    b * (C::kThreads / 64) + (threadIdx.x >> 6));
        return;
    }
    wide_item<C>(item0 + blk, a, sm);
}

template <class C>
__global__ __launch_bounds__(C::kThreads, C::kWaves) void k_refactor_wide(int item0, RefArgs<typename C::T> a,
                                                                         int nwide, int small0, int nsmall,
                                                                         CopyRanges c, FuseArgs<typename C::T> f) {
    extern __shared__ __align__(16) char sm[];
    refactor_block<C>(blockIdx.x, gridDim.x, item0, a, nwide, small0, nsmall, c, f, sm);
}

// ---------------------------------------------------------------------------------------
// triangular solves.  Items (one 256-thread block each): a pack of up to kSolvePack rows of
// whole panels of at most kPackW columns (a group of lanes per row for the part outside
// the panel, then the in-panel substitution in kPackW synchronised steps), a wide panel (a
// group of lanes per row outside the panel, then a register substitution inside it on
// wavefront 0), or a helper that sums the early columns of kHelpRows rows of a wide panel
// kHelpAhead levels ahead.  Records:
//   item {-c, p0, lanes, 0} pack of c rows listed at rows[p0..]; {1, lanes, s, w} wide
//   panel of rows s..s+w-1; {0, t0, s, w} helper for rows s+t0 .. of that panel;
//   pack row {i, first external slot, end of external slots, t | w << 8};
//   rinfo[i] forward {first slot, first late slot, diagonal slot, end}, backward
//   {diagonal slot, first early slot, end, 0}.
//
// Every item is written once for two execution modes: level launches (kWait = false: all
// inputs were written by earlier launches) and one persistent launch per triangle (kWait =
// true: an unknown is read with a device-coherent load and waited for while it still holds
// the unset sentinel; results are published with device-coherent stores).  The arithmetic
// is the same in both modes.  TF is the type of the stored factor (FP64, or FP32 in the
// mixed-precision path); each factor value is widened to FP64 as it is read, so the
// right-hand sides, the unknowns and every sum stay FP64.

template <class TF>
struct SolveArgs {
    const int4 *item, *rows, *rinfo;
    const int32_t *col, *Q;
    const TF *lucsr;
    const double *c;
    const double *bp;     // forward right-hand side r[P[i]] * b[P[i]] (permuted order)
    double *y;            // forward output / backward input (permuted)
    double *xt;           // backward output (permuted)
    double *x;            // backward output (original order)
    double *psum;         // forward: partial sums of the early L columns of helped rows
    double *usum;         // backward: partial sums of the early U columns of helped rows
    int *abort;           // persistent mode: raised by a wait that timed out
    int *tick;            // persistent mode: next item to take (forward, backward)
};

constexpr unsigned long long kUnset = 0x7ff4dead0badf00dULL;   // signaling NaN
constexpr int kSpinLimit = 1 << 21;

__device__ __forceinline__ unsigned long long load_coherent(const double *p) {
    return __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

// waits until *p no longer holds the sentinel; on timeout or abort returns 0 and raises
// *abort (the solve result is then invalid and reported as a device error)
__device__ __noinline__ double wait_slow(const double *p, int *abort) {
    for (int it = 0; it < kSpinLimit; ++it) {
        __builtin_amdgcn_s_sleep(2);
        const unsigned long long b = load_coherent(p);
        if (b != kUnset) return __longlong_as_double((long long)b);
        if ((it & 63) == 63 && __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return 0.0;
    }
    atomicOr(abort, 1);
    return 0.0;
}

// re-reads every still-unset entry of a batch together until none is left (bounded; on
// timeout or abort the unset entries read as 0 and *abort is raised)
template <int B>
__device__ __forceinline__ void wait_batch(unsigned long long (&bb)[B], const double *v, const int (&cc)[B],
                                           int *abort) {
    bool pend = false;
#pragma unroll
    for (int k = 0; k < B; ++k) pend |= bb[k] == kUnset;
    for (int it = 1; pend; ++it) {
        __builtin_amdgcn_s_sleep(2);
#pragma unroll
        for (int k = 0; k < B; ++k)
            if (bb[k] == kUnset) bb[k] = load_coherent(v + cc[k]);
        pend = false;
#pragma unroll
        for (int k = 0; k < B; ++k) pend |= bb[k] == kUnset;
        const bool stop = it >= kSpinLimit ||
                          ((it & 63) == 0 && __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (pend && stop) {
            if (it >= kSpinLimit) atomicOr(abort, 1);
#pragma unroll
            for (int k = 0; k < B; ++k)
                if (bb[k] == kUnset) bb[k] = 0ULL;
            pend = false;
        }
    }
}

template <bool kWait>
__device__ __forceinline__ double get_value(const double *p, int *abort) {
    if constexpr (kWait) {
        const unsigned long long b = load_coherent(p);
        return b != kUnset ? __longlong_as_double((long long)b) : wait_slow(p, abort);
    } else {
        return *p;
    }
}

template <bool kWait>
__device__ __forceinline__ void put_value(double *p, double v) {
    if constexpr (kWait)
        __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

// sum over q in [q0, q1) of lucsr[q] * v[col[q]] on a group of `width` lanes.  A lane's
// entries are taken four at a time into four accumulators, a remainder of fewer than four
// into the first.  Loads go in batches of B entries per lane: the batch's indices and
// factor values in one round, then its unknowns in one round.
template <bool kWait, int B, class TF>
__device__ __forceinline__ double sdot(const SolveArgs<TF> &a, const double *v, int q0, int q1, int gl, int width) {
    static_assert(B % 4 == 0, "batch of whole groups of four");
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int q = q0 + gl; q < q1; q += B * width) {
        const int rem = (q1 - q + width - 1) / width;
        int cc[B];
        double ll[B], vv[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const bool h = k < rem;
            cc[k] = h ? a.col[q + k * width] : 0;
            ll[k] = h ? (double)a.lucsr[q + k * width] : 0.0;
        }
        if constexpr (kWait) {
            unsigned long long bb[B];
#pragma unroll
            for (int k = 0; k < B; ++k) bb[k] = k < rem ? load_coherent(v + cc[k]) : 0ULL;
            wait_batch<B>(bb, v, cc, a.abort);
#pragma unroll
            for (int k = 0; k < B; ++k) vv[k] = __longlong_as_double((long long)bb[k]);
        } else {
#pragma unroll
            for (int k = 0; k < B; ++k) vv[k] = k < rem ? v[cc[k]] : 0.0;
        }
#pragma unroll
        for (int k0 = 0; k0 < B; k0 += 4) {
            const int r4 = rem - k0;
            if (r4 >= 4) {
                s0 = fma(ll[k0], vv[k0], s0);
                s1 = fma(ll[k0 + 1], vv[k0 + 1], s1);
                s2 = fma(ll[k0 + 2], vv[k0 + 2], s2);
                s3 = fma(ll[k0 + 3], vv[k0 + 3], s3);
            } else {
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    if (k < r4) s0 = fma(ll[k0 + k], vv[k0 + k], s0);
            }
        }
    }
    return group_sum((s0 + s1) + (s2 + s3), width);
}

// Forward substitution inside a panel of w <= kPanelMax rows (lane = row): Lrow[t] =
// L(lane, t) for t < lane, zero otherwise; yv enters as the row's right-hand side minus its
// external part.
__device__ __forceinline__ double inpanel_forward(const double (&Lrow)[kPanelMax], int w, int lane, double yv) {
#pragma unroll
    for (int t = 0; t + 1 < kPanelMax; ++t) {
        if (t + 1 < w) {
            const double yt = bcast(yv, t);
            const double nv = fma(-Lrow[t], yt, yv);
            yv = lane > t ? nv : yv;
        }
    }
    return yv;
}

// Backward substitution inside a panel (lane = row): Urow[t] = U(lane, t) for t > lane,
// rdv = 1 / U(lane, lane), taken before the substitution so that no division sits on its
// dependency chain; val enters as y minus the external part; returns the lane's unknown.
__device__ __forceinline__ double inpanel_backward(const double (&Urow)[kPanelMax], double rdv, int w, int lane,
                                                   double val) {
    double xv = 0.0;
#pragma unroll
    for (int t = kPanelMax - 1; t >= 0; --t) {
        if (t < w) {
            const double q = val * rdv;         // final in lane t
            const double xt = bcast(q, t);
            xv = lane == t ? q : xv;
            const double nv = fma(-Urow[t], xt, val);
            val = lane < t ? nv : val;
        }
    }
    return xv;
}

// ext[kPanelMax], blk[kPanelMax * kRowLd] (16-byte aligned) and ys[kSolvePack] are LDS of
// the caller.  The block has 256 threads or more; threads past 256 take no row and only
// join the barriers.
template <bool kWait, class TF>
__device__ __forceinline__ void lsolve_item(const SolveArgs<TF> &a, int item, double *ext, double *blk, double *ys) {
    const int4 it = a.item[item];
    const int tid = threadIdx.x, lane = tid & 63;
    if (it.x < 0) {                                     // pack of whole small panels
        const int lanes = it.z, g = tid / lanes, gl = tid % lanes;
        const int4 rr = g < -it.x ? a.rows[it.y + g] : int4{-1, 0, 0, 0};
        const int t = rr.w & 255;
        const bool lead = rr.x >= 0 && gl == 0;
        double bv = 0.0, Lp[kPackW - 1];
#pragma unroll
        for (int k = 0; k < kPackW - 1; ++k) Lp[k] = lead && k < t ? (double)a.lucsr[rr.z + k] : 0.0;
        if (lead) bv = a.bp[rr.x];
        const double acc = sdot<kWait, 4>(a, a.y, rr.y, rr.z, gl, lanes);
        double yv = bv - acc;
        // in-panel substitution: step k solves the rows at offset k of their panels
#pragma unroll
        for (int k = 0; k < kPackW; ++k) {
            if (lead && t == k) {
#pragma unroll
                for (int k2 = 0; k2 < k; ++k2) yv = fma(-Lp[k2], ys[g - k + k2], yv);
                ys[g] = yv;
                put_value<kWait>(a.y + rr.x, yv);
            }
            __syncthreads();
        }
        return;
    }
    const int s = it.z, w = it.w;
    if (it.x == 0) {                                    // early partial sums, one wavefront per row
        const int t = it.y + (tid >> 6);
        if (t < w && t < it.y + kHelpRows) {
            const int4 ri = a.rinfo[s + t];
            const double acc = sdot<kWait, 8>(a, a.y, ri.x, ri.y, lane, 64);
            if (lane == 0) put_value<kWait>(a.psum + s + t, acc);
        }
        return;
    }
    // wide panel: the in-panel rows are staged in LDS (blk[r * kRowLd + t] = L(r, t),
    // zero on and above the diagonal) alongside the first loads of the external part
    {
        const int lanes = it.y, t = tid / lanes, gl = tid % lanes;
        const int4 ri = a.rinfo[s + min(t, w - 1)];
        for (int e = tid; e < w * kPanelMax; e += blockDim.x) {
            const int r = e / kPanelMax, c = e % kPanelMax;
            const int d = a.rinfo[s + r].z;
            blk[r * kRowLd + c] = c < r ? (double)a.lucsr[d - r + c] : 0.0;
        }
        if (t < w) {
            const double bv = gl == 0 ? a.bp[s + t] : 0.0;
            const bool helped = ri.y > ri.x;
            const double ps = helped && gl == 0 ? get_value<kWait>(a.psum + s + t, a.abort) : 0.0;
            const double acc = sdot<kWait, 8>(a, a.y, ri.y, ri.z - t, gl, lanes);
            if (gl == 0) ext[t] = bv - (helped ? acc + ps : acc);
        }
    }
    __syncthreads();
    if (tid < 64) {
        double Lrow[kPanelMax];
        load_lds_row<kPanelMax>(Lrow, blk + min(lane, kPanelMax - 1) * kRowLd);
        double yv = lane < w ? ext[lane] : 0.0;
        yv = inpanel_forward(Lrow, w, lane, yv);
        if (lane < w) put_value<kWait>(a.y + s + lane, yv);
    }
    __syncthreads();
}

template <bool kWait, class TF>
__device__ __forceinline__ void usolve_item(const SolveArgs<TF> &a, int item, double *ext, double *blk) {
    const int4 it = a.item[item];
    const int tid = threadIdx.x, lane = tid & 63;
    if (it.x < 0) {                                     // pack of whole small panels
        __shared__ double xs[kSolvePack];
        const int lanes = it.z, g = tid / lanes, gl = tid % lanes;
        const int4 rr = g < -it.x ? a.rows[it.y + g] : int4{-1, 0, 0, 0};
        const int t = rr.w & 255, w = rr.w >> 8;
        const int e = w - 1 - t;                        // in-panel entries right of the diagonal
        const bool lead = rr.x >= 0 && gl == 0;
        double yv = 0.0, dd = 1.0, ci = 0.0, Up[kPackW - 1];
        int qi = 0;
        const int d = rr.y - (w - t);                   // diagonal slot
#pragma unroll
        for (int k = 0; k < kPackW - 1; ++k) Up[k] = lead && k < e ? (double)a.lucsr[d + 1 + k] : 0.0;
        if (lead) {
            yv = a.y[rr.x];
            dd = (double)a.lucsr[d];
            qi = a.Q[rr.x];
            ci = a.c[qi];
        }
        const double rdd = 1.0 / dd;                    // off the substitution's chain
        const double acc = sdot<kWait, 4>(a, a.xt, rr.y, rr.z, gl, lanes);
        double val = yv - acc;
        // step k solves the rows k places before the end of their panels; the row's
        // in-panel terms are taken from the right
#pragma unroll
        for (int k = 0; k < kPackW; ++k) {
            if (lead && e == k) {
#pragma unroll
                for (int k2 = k - 1; k2 >= 0; --k2) val = fma(-Up[k2], xs[g + 1 + k2], val);
                const double xv = val * rdd;
                xs[g] = xv;
                a.x[qi] = ci * xv;
                put_value<kWait>(a.xt + rr.x, xv);
            }
            __syncthreads();
        }
        return;
    }
    const int s = it.z, w = it.w;
    if (it.x == 0) {                                    // early partial sums, one wavefront per row
        const int t = it.y + (tid >> 6);
        if (t < w && t < it.y + kHelpRows) {
            const int4 ri = a.rinfo[s + t];
            const double acc = sdot<kWait, 8>(a, a.xt, ri.y, ri.z, lane, 64);
            if (lane == 0) put_value<kWait>(a.usum + s + t, acc);
        }
        return;
    }
    // in-panel rows staged in LDS: blk[r * kRowLd + t] = U(r, t) for t > r, else zero
    double dv = 1.0, yv = 0.0, ci = 0.0;
    int qi = 0;
    {
        for (int e = tid; e < w * kPanelMax; e += kBlock) {
            const int r = e / kPanelMax, c = e % kPanelMax;
            const int d = a.rinfo[s + r].x;
            blk[r * kRowLd + c] = c > r && c < w ? (double)a.lucsr[d + (c - r)] : 0.0;
        }
        if (tid < w) {
            const int i = s + tid;
            dv = (double)a.lucsr[a.rinfo[i].x];
            yv = a.y[i];
            qi = a.Q[i];
            ci = a.c[qi];
        }
        const int lanes = it.y, t = tid / lanes, gl = tid % lanes;
        if (t < w) {
            const int4 ri = a.rinfo[s + t];
            const bool helped = ri.y < ri.z;
            const double us = helped && gl == 0 ? get_value<kWait>(a.usum + s + t, a.abort) : 0.0;
            const double acc = sdot<kWait, 8>(a, a.xt, ri.x + (w - t), ri.y, gl, lanes);
            if (gl == 0) ext[t] = helped ? acc + us : acc;
        }
    }
    __syncthreads();
    if (tid < 64) {
        double Urow[kPanelMax];
        load_lds_row<kPanelMax>(Urow, blk + min(lane, kPanelMax - 1) * kRowLd);
        const double val = lane < w ? yv - ext[lane] : 0.0;
        const double xv = inpanel_backward(Urow, 1.0 / dv, w, lane, val);
        if (lane < w) {
            a.x[qi] = ci * xv;
            put_value<kWait>(a.xt + s + lane, xv);
        }
    }
    __syncthreads();
}

template <class TF>
__global__ __launch_bounds__(256) void k_lsolve_level(int item0, SolveArgs<TF> a) {
    __shared__ double ext[kPanelMax], ys[kSolvePack];
    __shared__ __align__(16) double blk[kPanelMax * kRowLd];
    lsolve_item<false>(a, item0 + blockIdx.x, ext, blk, ys);
}

template <class TF>
__global__ __launch_bounds__(256) void k_usolve_level(int item0, SolveArgs<TF> a) {
    __shared__ double ext[kPanelMax];
    __shared__ __align__(16) double blk[kPanelMax * kRowLd];
    usolve_item<false>(a, item0 + blockIdx.x, ext, blk);
}

// Persistent solves: the items of levels [i0, i1) in level order; an item only reads
// unknowns of items of lower levels, i.e. of smaller index.  Two ways to hand out items:
//  - fixed (kTicket = false): item i0 + k on block k % gridDim.x, each block in increasing
//    order.  The unfinished item of smallest index can always proceed once its block runs,
//    so the launch drains when every block is resident at once (a cooperative launch on a
//    device the launch has to itself);
//  - ticket (kTicket = true): running blocks take items from a counter (*tick, zeroed by
//    k_solve_reset), each block in increasing order.  A block takes a ticket only while it
//    runs and works through its tickets in order, so the unfinished item of smallest index
//    is always held by a running block that is working on it: the launch drains on whatever
//    share of the device it gets, with other streams' kernels beside it.  The next ticket
//    is requested at the start of an item and read at its end, so the counter's round trip
//    overlaps the item's loads; the counter still costs a round trip per item, which is why
//    the fixed order is kept for a device that the solve has to itself.
// LDS of the persistent and fused forward loops: ext, ys, the ticket and the staged panel
struct SolveLds {
    double ext[kPanelMax];
    double ys[kSolvePack];
    int next;
    int pad[3];
    double blk[kPanelMax * kRowLd];
};
static_assert(offsetof(SolveLds, blk) % 16 == 0, "the staged panel is read in 16-byte pairs");

// The ticket loop (blocks take items i0 + *tick++ in increasing order, see above) over the
// forward (kFwd) or backward items [i0, i1).
template <bool kFwd, class TF>
__device__ __forceinline__ void ticket_items(int i0, int i1, const SolveArgs<TF> &a, int *tick, SolveLds &L) {
    if (threadIdx.x == 0) L.next = atomicAdd(tick, 1);
    __syncthreads();
    int cur = L.next;
    while (i0 + cur < i1) {
        int nt = 0;
        if (threadIdx.x == 0) nt = atomicAdd(tick, 1);
        if constexpr (kFwd) lsolve_item<true>(a, i0 + cur, L.ext, L.blk, L.ys);
        else usolve_item<true>(a, i0 + cur, L.ext, L.blk);
        __syncthreads();                     // every thread is done with the item and `next`
        if (threadIdx.x == 0) L.next = nt;
        __syncthreads();
        cur = L.next;
    }
}

template <bool kFwd, bool kTicket, class TF>
__device__ __forceinline__ void persistent_items(int i0, int i1, const SolveArgs<TF> &a, int *tick) {
    __shared__ SolveLds L;
    if constexpr (!kTicket) {
        for (int item = i0 + blockIdx.x; item < i1; item += gridDim.x) {
            if constexpr (kFwd) lsolve_item<true>(a, item, L.ext, L.blk, L.ys);
            else usolve_item<true>(a, item, L.ext, L.blk);
        }
        return;
    }
    ticket_items<kFwd>(i0, i1, a, tick, L);
}

template <class TF, bool kTicket>
__global__ __launch_bounds__(256) void k_lsolve_persistent(int i0, int i1, SolveArgs<TF> a) {
    persistent_items<true, kTicket>(i0, i1, a, a.tick);
}

template <class TF, bool kTicket>
__global__ __launch_bounds__(256) void k_usolve_persistent(int i0, int i1, SolveArgs<TF> a) {
    persistent_items<false, kTicket>(i0, i1, a, a.tick + 1);
}

// Block blk of the f.nsolve extra blocks of a refactorization launch that run the items of
// one forward level (every input final before the launch, as in a level launch), with the
// launch's dynamic LDS
template <class T>
__device__ __forceinline__ void fused_forward_block(const FuseArgs<T> &f, int blk, char *sm) {
    SolveLds &L = *reinterpret_cast<SolveLds *>(sm);
    // an item that uses LDS ends with a barrier, so the next one may overwrite it
    for (int item = f.j0 + blk; item < f.j1; item += f.nsolve) lsolve_item<false>(f.s, item, L.ext, L.blk, L.ys);
}

// bp = r[P] .* b[P] (b = b0, or the recorded call's right-hand side when b0 is null); with
// mark, every unknown of the persistent mode starts unset; the first ntick item tickets start
// at zero (ntick <= n, or the grid covers ntick threads)
__device__ __forceinline__ void solve_reset_body(int i, int n, const double *__restrict__ b,
                                                 const double *__restrict__ r, const int32_t *__restrict__ P,
                                                 double *__restrict__ bp, double *__restrict__ y,
                                                 double *__restrict__ xt, double *__restrict__ psum,
                                                 double *__restrict__ usum, int mark, int ntick,
                                                 int *__restrict__ tick) {
    if (i < ntick) tick[i] = 0;
    if (i < n) {
        const int pi = P[i];
        bp[i] = r[pi] * b[pi];
        if (mark) {
            const double u = __longlong_as_double((long long)kUnset);
            y[i] = u;
            xt[i] = u;
            psum[i] = u;
            usum[i] = u;
        }
    }
}

__global__ void k_solve_reset(int n, const double *__restrict__ b0, const CallPtrs *call,
                              const double *__restrict__ r, const int32_t *__restrict__ P, double *__restrict__ bp,
                              double *__restrict__ y, double *__restrict__ xt, double *__restrict__ psum,
                              double *__restrict__ usum, int mark, int ntick, int *__restrict__ tick) {
    const double *__restrict__ b = b0 ? b0 : call_ptr(&call->b);   // b0 null: the recorded call's
    solve_reset_body(blockIdx.x * blockDim.x + threadIdx.x, n, b, r, P, bp, y, xt, psum, usum, mark, ntick, tick);
}

// The column pass of the value update with the solve's set-up for the recorded call's
// right-hand side (k_solve_reset with the unknowns marked unset) on its first nset blocks:
// the set-up reads only the row scales and the call's inputs, so its blocks run beside the
// column pass's gathers instead of in a launch of their own.
template <class T>
__global__ __launch_bounds__(256) void k_col_store_setup(int n, const int32_t *__restrict__ colptr,
                                                         const int2 *__restrict__ src,
                                                         const int32_t *__restrict__ Q, const CallPtrs *call,
                                                         const int16_t *__restrict__ er, int scale,
                                                         double *__restrict__ c, int16_t *__restrict__ ec,
                                                         T *__restrict__ lu, int nset, const double *__restrict__ r,
                                                         const int32_t *__restrict__ P, double *__restrict__ bp,
                                                         double *__restrict__ y, double *__restrict__ xt,
                                                         double *__restrict__ psum, double *__restrict__ usum,
                                                         int ntick, int *__restrict__ tick) {
    if ((int)blockIdx.x < nset) {
        solve_reset_body(blockIdx.x * blockDim.x + threadIdx.x, n, call_ptr(&call->b), r, P, bp, y, xt, psum, usum,
                         1, ntick, tick);
        return;
    }
    col_store_body<T>(blockIdx.x - nset, n, colptr, src, Q, call_ptr(&call->v), er, scale, c, ec, lu);
}

// Approximate triangular solves for the preconditioner inside refinement (the triangular
// solves replaced by Jacobi or Gauss-Seidel iterations): sweeps over the CSR copy of L+U in
// the permuted, scaled space.  Each triangle starts from the zero vector (yin / xin null).
// Jacobi: 8 lanes per row, no dependency between rows (every sweep reads the previous
// iterate only).  One sweep of the unit lower triangle: yout = bp - (L - I) yin.
template <class TF>
__global__ __launch_bounds__(256) void k_jacobi_l(int n, const int4 *__restrict__ rinfo, const int32_t *__restrict__ col,
                                                  const TF *__restrict__ lucsr, const double *__restrict__ bp,
                                                  const double *__restrict__ yin, double *__restrict__ yout) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gid >> 3, gl = gid & 7;
    if (i >= n) return;                                 // whole 8-lane groups
    const int4 ri = rinfo[i];                           // L entries of row i: [x, z)
    double s = 0.0;
    if (yin)
        for (int q = ri.x + gl; q < ri.z; q += 8) s = fma((double)lucsr[q], yin[col[q]], s);
    s = group_sum(s, 8);
    if (gl == 0) yout[i] = bp[i] - s;
}

// One sweep of the upper triangle: xout = D^-1 (y - (U - D) xin).
template <class TF>
__global__ __launch_bounds__(256) void k_jacobi_u(int n, const int4 *__restrict__ urinfo,
                                                  const int32_t *__restrict__ col, const TF *__restrict__ lucsr,
                                                  const double *__restrict__ y, const double *__restrict__ xin,
                                                  double *__restrict__ xout) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gid >> 3, gl = gid & 7;
    if (i >= n) return;
    const int4 ri = urinfo[i];                          // diagonal at x, U entries (x, z)
    double s = 0.0;
    if (xin)
        for (int q = ri.x + 1 + gl; q < ri.z; q += 8) s = fma((double)lucsr[q], xin[col[q]], s);
    s = group_sum(s, 8);
    if (gl == 0) xout[i] = (y[i] - s) / (double)lucsr[ri.x];
}

// Block Gauss-Seidel sweeps: the rows are cut into chunks of kGsChunk consecutive permuted
// rows, one 256-thread block per chunk.  A row reads the values of its own chunk from the
// current sweep and every other value from the previous iterate (Jacobi between chunks):
// 8 lanes per row sum the entries outside the chunk while the entries inside it are staged
// as a dense triangle in LDS, then wavefront 0 substitutes inside the chunk in registers.
constexpr int kGsChunk = kPanelMax;

// yout = chunk-wise solve of L_cc yout_c = bp_c - L_c,out yin (unit L_cc)
template <class TF>
__global__ __launch_bounds__(256) void k_bgs_l(int n, const int4 *__restrict__ rinfo, const int32_t *__restrict__ col,
                                               const TF *__restrict__ lucsr, const double *__restrict__ bp,
                                               const double *__restrict__ yin, double *__restrict__ yout) {
    __shared__ double ext[kGsChunk];
    __shared__ __align__(16) double blk[kGsChunk * kRowLd];
    const int c0 = blockIdx.x * kGsChunk, w = min(kGsChunk, n - c0);
    const int tid = threadIdx.x, t = tid >> 3, gl = tid & 7;
    for (int e = tid; e < kGsChunk * kRowLd; e += kBlock) blk[e] = 0.0;
    __syncthreads();
    double s = 0.0;
    if (t < w) {
        const int4 ri = rinfo[c0 + t];                  // L entries of the row: [x, z)
        for (int q = ri.x + gl; q < ri.z; q += 8) {
            const int j = col[q];
            const double l = (double)lucsr[q];
            if (j >= c0) blk[t * kRowLd + (j - c0)] = l;
            else if (yin) s = fma(l, yin[j], s);
        }
    }
    s = group_sum(s, 8);
    if (t < w && gl == 0) ext[t] = bp[c0 + t] - s;
    __syncthreads();
    if (tid < 64) {
        double Lrow[kPanelMax];
        load_lds_row<kPanelMax>(Lrow, blk + min(tid, kGsChunk - 1) * kRowLd);
        double yv = tid < w ? ext[tid] : 0.0;
        yv = inpanel_forward(Lrow, w, tid, yv);
        if (tid < w) yout[c0 + tid] = yv;
    }
}

// xout = chunk-wise solve of U_cc xout_c = y_c - U_c,out xin
template <class TF>
__global__ __launch_bounds__(256) void k_bgs_u(int n, const int4 *__restrict__ urinfo, const int32_t *__restrict__ col,
                                               const TF *__restrict__ lucsr, const double *__restrict__ y,
                                               const double *__restrict__ xin, double *__restrict__ xout) {
    __shared__ double ext[kGsChunk], dg[kGsChunk];
    __shared__ __align__(16) double blk[kGsChunk * kRowLd];
    const int c0 = blockIdx.x * kGsChunk, w = min(kGsChunk, n - c0), c1 = c0 + w;
    const int tid = threadIdx.x, t = tid >> 3, gl = tid & 7;
    for (int e = tid; e < kGsChunk * kRowLd; e += kBlock) blk[e] = 0.0;
    __syncthreads();
    double s = 0.0;
    int4 ri = int4{0, 0, 0, 0};
    if (t < w) {
        ri = urinfo[c0 + t];                            // diagonal at x, U entries (x, z)
        for (int q = ri.x + 1 + gl; q < ri.z; q += 8) {
            const int j = col[q];
            const double u = (double)lucsr[q];
            if (j < c1) blk[t * kRowLd + (j - c0)] = u;
            else if (xin) s = fma(u, xin[j], s);
        }
    }
    s = group_sum(s, 8);
    if (t < w && gl == 0) {
        ext[t] = y[c0 + t] - s;
        dg[t] = (double)lucsr[ri.x];
    }
    __syncthreads();
    if (tid < 64) {
        double Urow[kPanelMax];
        load_lds_row<kPanelMax>(Urow, blk + min(tid, kGsChunk - 1) * kRowLd);
        const double val = tid < w ? ext[tid] : 0.0;
        const double xv = inpanel_backward(Urow, tid < w ? 1.0 / dg[tid] : 1.0, w, tid, val);
        if (tid < w) xout[c0 + tid] = xv;
    }
}

// x[Q[i]] = c[Q[i]] xt[i]: back to the original ordering and scaling
__global__ __launch_bounds__(256) void k_unpermute(int n, const int32_t *__restrict__ Q, const double *__restrict__ c,
                                                   const double *__restrict__ xt, double *__restrict__ x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int qi = Q[i];
        x[qi] = c[qi] * xt[i];
    }
}

// ---------------------------------------------------------------------------------------
// residual, sparse products and Krylov vector kernels (FP64)

// res = b - A x (8 lanes per row, kRowsPerGroup rows per group, grid-stride) and block
// maxima of |res|, |x|, |b| into part[3 * block + {0, 1, 2}]
__global__ __launch_bounds__(256) void k_residual(int n, const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col, const double *__restrict__ v,
                                                  const double *__restrict__ x, const double *__restrict__ b,
                                                  double *__restrict__ res, double *__restrict__ part) {
    __shared__ double red[3][4];
    const double qnan = __longlong_as_double(0x7ff8000000000000LL);
    double rn = 0.0, xn = 0.0, bn = 0.0;
    const int gl = threadIdx.x & 7;
    for (int i0 = ((blockIdx.x * blockDim.x + threadIdx.x) >> 3) * kRowsPerGroup; i0 < n;
         i0 += ((gridDim.x * blockDim.x) >> 3) * kRowsPerGroup) {
        int rp[kRowsPerGroup + 1];
        group_rows(rowptr, n, i0, rp);
        double vv[kRowsPerGroup], xv[kRowsPerGroup];
        int cc[kRowsPerGroup];
#pragma unroll
        for (int k = 0; k < kRowsPerGroup; ++k) {
            const int p = rp[k] + gl;
            const bool h = p < rp[k + 1];
            vv[k] = h ? v[p] : 0.0;
            cc[k] = h ? col[p] : 0;
        }
#pragma unroll
        for (int k = 0; k < kRowsPerGroup; ++k) xv[k] = rp[k] + gl < rp[k + 1] ? x[cc[k]] : 0.0;
#pragma unroll
        for (int k = 0; k < kRowsPerGroup; ++k) {
            double sk = vv[k] * xv[k];
            for (int p = rp[k] + gl + 8; p < rp[k + 1]; p += 8) sk = fma(v[p], x[col[p]], sk);
            sk = group_sum(sk, 8);
            const int i = i0 + k;
            if (gl == 0 && i < n) {
                const double ri = b[i] - sk;
                res[i] = ri;
                rn = isnan(ri) ? qnan : fmax(rn, fabs(ri));
                xn = isnan(x[i]) ? qnan : fmax(xn, fabs(x[i]));
                bn = fmax(bn, fabs(b[i]));
            }
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
