// C ABI of the KKT refactorization library: handle lifetime, workspace binding, and the
// enqueueing of the value update, refactorization, solves and FGMRES refinement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <type_traits>
#include <vector>

#include "kkt_kernels.h"
#include "kkt_kernels.hip"

using namespace kkt;

namespace {

// device pointers carved out of the caller's workspace
struct Dev {
    int32_t *a_rowptr, *a_colind;
    int2 *lu_src;       // per factor slot: {CSR position of its entry of A or -1, that entry's row}
    int32_t *colptr, *rowidx, *ulen, *pan_start, *pan_r;
    int32_t *f_rel, *ldiag;
    int4 *itemrec, *pair8;
    unsigned long long *pcount;
    int4 *l_item4, *u_item4, *l_rows4, *u_rows4, *rinfo4, *urinfo4;
    int32_t *csr_col, *copy_k, *copy_src, *P, *Q;
    void *lu, *lucsr;   // factor values (FP64, or FP32 with factor_precision = KKT_FP32)
    double *r, *c, *y, *xt, *psum, *usum, *bp, *bsave;
    int16_t *er, *ec;   // exponents of the scale factors: r_i = 2^-er[i], c_j = 2^-ec[j]
    double *V, *Z, *w, *res, *part, *hbuf, *ybuf;
    DevStatus *st;
    ResNorms *rn;
    int *tick;          // ticket counters of the persistent solves (forward, backward, fused tail)
    CallPtrs *call;     // the values and right-hand side of the current call (recorded graphs)
};

// most blocks of a refactor launch that run forward-solve items (kkt_refactor_refine; at 70k
// 128 and 512 measured 1% and 0.4% slower)
constexpr int kFuseSolveBlocks = 256;
// most copy blocks of a refactor launch per compute unit (1: 1.3% slower at 70k, 16: same)
constexpr int kCopyBlocksPerCu = 4;
constexpr int kDotBlocks = 512;
constexpr int kNormRowBlocks = 4096;   // most blocks of the row-norm pass (8 lanes per row)
// narrow items per level up to which the pipelined variant runs (a tiny item counts a quarter:
// its 4-lane group keeps four times as many items in flight)
constexpr int kSmallPipeMax = 100000;
constexpr int kNormBlocks = 4096;
constexpr int kMaxSweeps = 1024;       // largest approx_sweeps accepted
constexpr int kMaxRestart = 64;

struct Carver {
    char *base;
    size_t off = 0;
    template <class T> T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

}  // namespace

struct kkt_handle {
    kkt_opts opts{};
    Symbolic sym;
    Schedule sch;
    bool bound = false;
    bool factored = false;
    int device = -1;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int32_t max_nrhs = 1;
    Dev d{};
    const double *d_values = nullptr;
    // host staging for small read-backs: the pinned buffer made by kkt_bind, or the handle's
    // own array (pageable) for a handle bound by kkt_bind_scratch that never had one
    double *h_small = nullptr;
    double *h_pinned = nullptr;
    double h_stage[4 * (kMaxRestart + 2) + 32] = {};
    // bound to the library's static scratch array: nothing is allocated after the bind (no
    // graph is recorded; the level launches go one by one)
    bool on_scratch = false;
    // the persistent solves take items by ticket (persistent_solve = 2, or a device without
    // cooperative launches): safe when other streams share the device
    bool tickets = false;
    int grid_l = 1, grid_u = 1;  // co-resident blocks of the persistent solve kernels
    int ncu = 1;                 // compute units of the bound device
    // the refactorization's per-level launches, recorded once per bind on the capture stream
    // (created at the first bind) and replayed on the caller's stream
    hipStream_t cap = nullptr;
    hipGraphExec_t levels = nullptr;
    hipEvent_t levels_done = nullptr;   // recorded after every replay, on the caller's stream
    bool levels_failed = false;
    // kkt_refactor_refine: the level launches with the forward solve riding in them,
    // recorded at its first call
    hipGraphExec_t fused = nullptr;
    bool fused_failed = false;
    // launch profiler
    bool prof = false;
    kkt_profile acc{};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
    std::vector<int> ev_count;     // launches bracketed by each pending pair
    int ev_open = -1;              // pending pair whose end is not recorded yet (a run of launches)
    hipStream_t ev_open_s = nullptr;
};

namespace {

void carve(const kkt_handle *h, char *base, Dev &d, size_t *bytes) {
    const Symbolic &s = h->sym;
    const Schedule &g = h->sch;
    const size_t n = s.n, nlu = s.nnz_lu(), na = s.nnz_a;
    const int m = h->opts.gmres_restart;
    const size_t fb = h->opts.factor_precision == KKT_FP32 ? sizeof(float) : sizeof(double);
    Carver c{base};
    d.a_rowptr = c.take<int32_t>(n + 1);
    d.a_colind = c.take<int32_t>(na);
    d.lu_src = c.take<int2>(std::max<size_t>(1, nlu));
    d.colptr = c.take<int32_t>(n + 1);
    d.rowidx = c.take<int32_t>(nlu);
    d.ulen = c.take<int32_t>(n);
    d.pan_start = c.take<int32_t>(g.pan_start.size());
    d.pan_r = c.take<int32_t>(g.pan_r.size());
    d.itemrec = c.take<int4>(std::max<size_t>(3, g.itemrec.size() / 4));
    d.pair8 = c.take<int4>(std::max<size_t>(2, g.pair8.size() / 4));
    d.ldiag = c.take<int32_t>(n);
    d.f_rel = c.take<int32_t>(std::max<size_t>(1, g.f_rel.size()));
    d.pcount = c.take<unsigned long long>(kCountSlots);
    d.l_item4 = c.take<int4>(std::max<size_t>(1, g.l_item4.size() / 4));
    d.u_item4 = c.take<int4>(std::max<size_t>(1, g.u_item4.size() / 4));
    d.l_rows4 = c.take<int4>(std::max<size_t>(1, g.l_rows4.size() / 4));
    d.u_rows4 = c.take<int4>(std::max<size_t>(1, g.u_rows4.size() / 4));
    d.rinfo4 = c.take<int4>(n);
    d.urinfo4 = c.take<int4>(n);
    d.csr_col = c.take<int32_t>(nlu);
    d.copy_k = c.take<int32_t>(std::max<size_t>(1, g.copy_k.size()));
    d.copy_src = c.take<int32_t>(std::max<size_t>(1, g.copy_src.size()));
    d.P = c.take<int32_t>(n);
    d.Q = c.take<int32_t>(n);
    d.r = c.take<double>(n);
    d.c = c.take<double>(n);
    d.er = c.take<int16_t>(n);
    d.ec = c.take<int16_t>(n);
    d.lu = c.take<char>(nlu * fb);
    d.lucsr = c.take<char>(nlu * fb);
    d.y = c.take<double>(n);
    d.xt = c.take<double>(n);
    d.psum = c.take<double>(n);
    d.usum = c.take<double>(n);
    d.bp = c.take<double>(n);
    d.bsave = c.take<double>(n);
    d.V = c.take<double>((size_t)(m + 1) * n);
    d.Z = c.take<double>((size_t)m * n);
    d.w = c.take<double>(n);
    d.res = c.take<double>(n);
    d.part = c.take<double>(std::max((size_t)kDotBlocks * (m + 2), (size_t)kNormBlocks * 3));
    d.hbuf = c.take<double>(4 * (size_t)(m + 2));
    d.ybuf = c.take<double>((size_t)m + 2);
    d.st = c.take<DevStatus>(1);
    d.rn = c.take<ResNorms>(1);
    d.tick = c.take<int>(3);
    d.call = c.take<CallPtrs>(1);
    *bytes = c.off + 256;
}

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Runs f with a value of the handle's factor type (double, or float for KKT_FP32).
template <class F>
auto by_precision(const kkt_handle *h, F &&f) {
    if (h->opts.factor_precision == KKT_FP32) return f(float{});
    return f(double{});
}

#define HIPCHK(x)                                  \
    do {                                           \
        if ((x) != hipSuccess) return KKT_ERR_DEVICE; \
    } while (0)

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }
// blocks of the update passes: 8 lanes per kRowsPerGroup rows, kColLanes lanes per column
inline int row_blocks(int n) {
    return (int)std::max<unsigned>(1, blocks_for((int64_t)(n + kRowsPerGroup - 1) / kRowsPerGroup * 8, 256));
}
inline int col_blocks(int n) { return (int)std::max<unsigned>(1, blocks_for((int64_t)n * kColLanes, 256)); }
inline int norm_blocks(int n) { return std::min(kNormRowBlocks, row_blocks(n)); }
// blocks of `threads` threads for ns narrow items, the last nt of them tiny (one 16-lane
// group per item, one kTinyLanes-lane group per tiny item)
inline int narrow_blocks(int ns, int nt, int threads) {
    if (ns == 0) return 0;
    return (int)(blocks_for(ns - nt, threads / 16) + blocks_for(nt, threads / kTinyLanes));
}

// ends the open run of launches of the profiler (records its end event)
void close_run(kkt_handle *h) {
    if (h->ev_open < 0) return;
    (void)hipEventRecord(h->ev_pending[h->ev_open].second.second, h->ev_open_s);
    h->ev_open = -1;
}

// Runs `launch` (which enqueues one kernel on s); with the profiler on, brackets it with a
// pair of events attributed to kernel class cls.  run: consecutive launches of one class on
// one stream (the refactorization's levels) share one pair, so the events' own cost (a few
// microseconds a pair) is not counted once per launch.
template <class F>
void timed(kkt_handle *h, int cls, hipStream_t s, F &&launch, bool run = false) {
    if (!h->prof) {
        launch();
        return;
    }
    if (h->ev_open >= 0) {
        if (run && h->ev_pending[h->ev_open].first == cls && h->ev_open_s == s) {
            launch();
            h->ev_count[h->ev_open] += 1;
            return;
        }
        close_run(h);
    }
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (!h->ev_free.empty()) {
        ev = h->ev_free.back();
        h->ev_free.pop_back();
    } else if (hipEventCreate(&ev.first) != hipSuccess || hipEventCreate(&ev.second) != hipSuccess) {
        launch();
        return;
    }
    (void)hipEventRecord(ev.first, s);
    launch();
    h->ev_pending.emplace_back(cls, ev);
    h->ev_count.push_back(1);
    if (run) {
        h->ev_open = (int)h->ev_pending.size() - 1;
        h->ev_open_s = s;
    } else {
        (void)hipEventRecord(ev.second, s);
    }
}

void fold_events(kkt_handle *h);

// waits for the stream, then folds the profiler's completed events
hipError_t sync_fold(kkt_handle *h, hipStream_t s) {
    close_run(h);
    const hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess && !h->ev_pending.empty()) fold_events(h);
    return e;
}

// folds completed event pairs into the profile (call after the stream was synchronized)
void fold_events(kkt_handle *h) {
    for (size_t i = 0; i < h->ev_pending.size(); ++i) {
        const auto &pe = h->ev_pending[i];
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, pe.second.first, pe.second.second) == hipSuccess) {
            h->acc.ms[pe.first] += ms;
            h->acc.launches[pe.first] += h->ev_count[i];
        }
        h->ev_free.push_back(pe.second);
    }
    h->ev_pending.clear();
    h->ev_count.clear();
}

template <class T>
int upload(T *dst, const std::vector<T> &src, hipStream_t s) {
    if (src.empty()) return KKT_OK;
    HIPCHK(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return KKT_OK;
}

// x = Q C (L U)^-1 P R b for one column (both in original order)
// One launch of a persistent solve kernel over items [i0, i1) with at most as many blocks
// as the device holds at once: cooperative for the fixed item order (every block resident),
// plain for the ticket order (progress does not need residency).
template <class K, class A>
hipError_t launch_persistent(K kernel, bool ticket, int grid, int i0, int i1, A &a, hipStream_t s) {
    if (ticket) {
        kernel<<<grid, kBlock, 0, s>>>(i0, i1, a);
        return hipGetLastError();
    }
    void *args[] = {&i0, &i1, &a};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kernel), dim3(grid), dim3(kBlock), args, 0, s);
}

// forward = false: the forward part already ran (the fused refactorization), only the
// backward part is enqueued
template <class TF>
int enqueue_solve_t(kkt_handle *h, const double *b, double *x, hipStream_t s, bool forward) {
    const Schedule &g = h->sch;
    const Dev &d = h->d;
    const int n = h->sym.n;
    const bool pers = h->opts.persistent_solve != 0;
    SolveArgs<TF> a{d.l_item4, d.l_rows4, d.rinfo4, d.csr_col, d.Q, static_cast<const TF *>(d.lucsr), d.c, d.bp, d.y,
                    d.xt, x, d.psum, d.usum, &d.st->abort, d.tick};
    if (forward)
        timed(h, KKT_PROF_LSOLVE, s, [&] {
            k_solve_reset<<<blocks_for(n, 256), 256, 0, s>>>(n, b, d.call, d.r, d.P, d.bp, d.y, d.xt, d.psum, d.usum,
                                                             pers ? 1 : 0, pers ? 2 : 0, d.tick);
        });
    // forward: level launches below l_split, then the persistent launch
    const int lsplit = !forward ? 0 : pers ? g.l_split : (int)g.l_lvl.size() - 1;
    for (int l = 0; l < lsplit; ++l) {
        const int cnt = g.l_lvl[l + 1] - g.l_lvl[l];
        if (cnt) timed(h, KKT_PROF_LSOLVE, s, [&] { k_lsolve_level<TF><<<cnt, kBlock, 0, s>>>(g.l_lvl[l], a); });
    }
    const int li0 = g.l_lvl[lsplit], li1 = forward ? g.l_lvl.back() : li0;
    if (li1 > li0) {
        hipError_t e = hipSuccess;
        timed(h, KKT_PROF_LSOLVE, s,
              [&] {
                  const int gr = std::min(li1 - li0, h->grid_l);
                  e = h->tickets ? launch_persistent(k_lsolve_persistent<TF, true>, true, gr, li0, li1, a, s)
                                 : launch_persistent(k_lsolve_persistent<TF, false>, false, gr, li0, li1, a, s);
              });
        HIPCHK(e);
    }
    // backward: the persistent launch for levels below u_split, then level launches
    a.item = d.u_item4;
    a.rows = d.u_rows4;
    a.rinfo = d.urinfo4;
    const int usplit = pers ? g.u_split : 0;
    const int ui1 = g.u_lvl[usplit];
    if (ui1 > 0) {
        hipError_t e = hipSuccess;
        timed(h, KKT_PROF_USOLVE, s,
              [&] {
                  const int gr = std::min(ui1, h->grid_u);
                  e = h->tickets ? launch_persistent(k_usolve_persistent<TF, true>, true, gr, 0, ui1, a, s)
                                 : launch_persistent(k_usolve_persistent<TF, false>, false, gr, 0, ui1, a, s);
              });
        HIPCHK(e);
    }
    for (size_t l = usplit; l + 1 < g.u_lvl.size(); ++l) {
        const int cnt = g.u_lvl[l + 1] - g.u_lvl[l];
        if (cnt) timed(h, KKT_PROF_USOLVE, s, [&] { k_usolve_level<TF><<<cnt, kBlock, 0, s>>>(g.u_lvl[l], a); });
    }
    HIPCHK(hipGetLastError());
    return KKT_OK;
}

int enqueue_solve(kkt_handle *h, const double *b, double *x, hipStream_t s, bool forward = true) {
    return by_precision(h, [&](auto tag) { return enqueue_solve_t<decltype(tag)>(h, b, x, s, forward); });
}

// stores the call's values (and right-hand side, or null) for the recorded kernels and
// clears the status words (before anything of the call can raise a flag)
int set_call(kkt_handle *h, const double *v, const double *b, hipStream_t s) {
    timed(h, KKT_PROF_UPDATE, s, [&] { k_set_call<<<1, 256, 0, s>>>(h->d.call, v, b, h->d.st, h->d.pcount); });
    HIPCHK(hipGetLastError());
    return KKT_OK;
}

// value update of the values stored by set_call: scale factors, scaled values into the
// factor, norms; with setup, the column pass also runs the solve's set-up for the stored
// right-hand side (the unknowns marked unset, ntick tickets cleared)
int enqueue_update(kkt_handle *h, hipStream_t s, bool setup = false, int ntick = 0) {
    const Dev &d = h->d;
    const int n = h->sym.n;
    const int eq = h->opts.equilibrate != 0;
    timed(h, KKT_PROF_UPDATE, s, [&] {
        k_row_scale<<<row_blocks(n), 256, 0, s>>>(n, d.a_rowptr, d.call, eq, d.r, d.er, d.st);
    });
    timed(h, KKT_PROF_UPDATE, s, [&] {
        by_precision(h, [&](auto tag) {
            using T = decltype(tag);
            if (setup) {
                const int nset = (int)blocks_for(std::max(n, ntick), 256);
                k_col_store_setup<T><<<nset + col_blocks(n), 256, 0, s>>>(
                    n, d.colptr, d.lu_src, d.Q, d.call, d.er, eq, d.c, d.ec, static_cast<T *>(d.lu), nset, d.r, d.P,
                    d.bp, d.y, d.xt, d.psum, d.usum, ntick, d.tick);
            } else {
                k_col_store<T><<<col_blocks(n), 256, 0, s>>>(n, d.colptr, d.lu_src, d.Q, d.call, d.er, eq, d.c,
                                                          d.ec, static_cast<T *>(d.lu));
            }
            return 0;
        });
    });
    const int nbn = norm_blocks(n);
    timed(h, KKT_PROF_UPDATE, s, [&] { k_norms<<<nbn, 256, 0, s>>>(n, d.a_rowptr, d.a_colind, d.call, d.r, d.ec, d.part); });
    timed(h, KKT_PROF_UPDATE, s, [&] { k_max_parts<<<1, 256, 0, s>>>(nbn, 2, d.part, &d.st->anorm_scaled); });
    HIPCHK(hipGetLastError());
    return KKT_OK;
}

// extra blocks of `threads` threads of a refactor launch that copy `entries` entries of the
// row-ordered factor (they run after the factor work of the launch, in its tail)
int copy_blocks(const kkt_handle *h, int entries, int threads) {
    return entries > 0 ? std::min(kCopyBlocksPerCu * h->ncu, (int)blocks_for(entries, threads)) : 0;
}
int copy_count(const CopyRanges &c) { return (c.a1 - c.a0) + (c.b1 - c.b0); }

// kkt_refactor's row-ordered copy: the entries of every column final before the top levels
// ride in up to kCopyLaunches of the top launches, chunk c of ncopy of each section; the rest
// follows the last level
int copy_carriers(const Schedule &g) {
    return std::min<int>(kCopyLaunches, (int)g.f_lvl.size() - 1 - g.copy_lvl);
}
CopyRanges copy_chunk(const Schedule &g, int c, int ncopy) {
    const int64_t nl = g.copy_lat[g.copy_lvl], u0 = g.copy_uat[0], nu = g.copy_uat[g.copy_lvl] - u0;
    return CopyRanges{(int)(nl * c / ncopy), (int)(nl * (c + 1) / ncopy), (int)(u0 + nu * c / ncopy),
                      (int)(u0 + nu * (c + 1) / ncopy)};
}
CopyRanges copy_rest(const Schedule &g, int ncopy) {
    const int u0 = g.copy_uat[0], n = (int)g.copy_k.size();
    return CopyRanges{ncopy > 0 ? g.copy_lat[g.copy_lvl] : 0, u0, ncopy > 0 ? g.copy_uat[g.copy_lvl] : u0, n};
}

// the value update (of the values stored by set_call), the level launches of the
// refactorization, the row-ordered copy and the pivot count; they read only workspace
// buffers, so one recording serves every later call.
// fused: the forward solve of the right-hand side set up by k_solve_reset rides in the same
// launches, so no launch waits on another queue.  Each launch has extra blocks that copy the
// entries of the columns finished by the launches before it into the row-ordered copy; each
// wide launch also has extra blocks that run the next forward level once every column its
// items read was copied by an earlier launch (its lower levels ran in earlier launches; its
// items are independent, as in a level launch).  What is left after the last level runs in
// a copy launch and a ticket-ordered forward launch of its own.
template <class T>
int enqueue_levels_t(kkt_handle *h, hipStream_t s, bool fused) {
    using Big = BigCfg<T>;
    using Med = MedCfg<T>;
    using W256 = W256Cfg<T>;
    const Schedule &g = h->sch;
    const Dev &d = h->d;
    const double tiny = std::is_same<T, float>::value ? h->opts.tiny_pivot_fp32 : h->opts.tiny_pivot;
    RefArgs<T> a{d.ldiag, d.itemrec, d.pair8, d.f_rel, static_cast<T *>(d.lu), d.st, d.pcount,
                 tiny, h->opts.dense_mfma != 0, d.copy_k, d.copy_src, static_cast<T *>(d.lucsr),
                 d.pan_start, d.pan_r};
    const int nlev = (int)g.f_lvl.size() - 1;
    const int ncopy = fused ? 0 : copy_carriers(g);   // kkt_refactor: launches that carry a chunk of the copy
    // fused: the upper section spread evenly over the top launches (as far as final)
    const int u0 = g.copy_uat[0], nup = (int)g.copy_k.size() - u0, ntop = nlev - g.copy_lvl;
    int ucopied = u0, ktop = 0;
    const SolveArgs<T> fs{d.l_item4, d.l_rows4, d.rinfo4, d.csr_col, d.Q, static_cast<const T *>(d.lucsr), d.c,
                          d.bp, d.y, d.xt, nullptr, d.psum, d.usum, &d.st->abort, d.tick + 2};
    const int nfl = (int)g.l_lvl.size() - 1;
    {
        // fused: the column pass also sets up the solve (bp from the stored right-hand side,
        // the unset unknowns and the tickets, the forward tail's included)
        const int rc = enqueue_update(h, s, fused, 3);
        if (rc) return rc;
    }
    int copied = 0, solved = 0;   // fused: levels whose columns a launch copies, forward levels launched
    for (int l = 0; l < nlev; ++l) {
        // the kinds of items of a level touch disjoint target columns, so one launch runs the
        // wide items (32- or 16-column configuration) and the narrow ones together; a level
        // without wide items has a launch of the narrow kernel
        const int nm = g.f_nmed[l], nb = g.f_nlarge[l] - nm, ns = g.f_lvl[l + 1] - g.f_lvl[l] - nb - nm;
        const int i0 = g.f_lvl[l];
        if (ns && !nb && !nm) {
            // with fused, extra blocks copy the lower entries of the columns of the levels since
            // the last launch
            const CopyRanges c{fused ? g.copy_lat[copied] : 0, fused ? g.copy_lat[l] : 0, 0, 0};
            if (fused) copied = l;
            const int nt = g.f_ntiny[l];
            const int grid = narrow_blocks(ns, nt, kBlock) + copy_blocks(h, copy_count(c), kBlock);
            // many items: keep more in flight; few: shorten each item's dependent chain (only
            // items that pull have one; a level of leaves keeps the plain variant's occupancy)
            const bool pulls = g.f_item_pair[i0 + ns] > g.f_item_pair[i0];
            const bool pipe = pulls && (ns - nt) + (nt + kTinyLanes - 1) / kTinyLanes <= kSmallPipeMax;
            timed(h, KKT_PROF_REFACTOR_SMALL, s, [&] {
                if (!pipe)
                    k_refactor_small<T, false><<<grid, kBlock, 0, s>>>(i0, ns, nt, a, c);
                else
                    k_refactor_small<T, true><<<grid, kBlock, 0, s>>>(i0, ns, nt, a, c);
            }, true);
        }
        if (!nb && !nm) continue;
        // otherwise the narrow items are extra blocks of the level's wide launch, and so is a
        // chunk of the row-ordered copy (columns already final): on the top levels; with fused
        // the lower entries of the columns of the levels since the last launch, and on the top
        // levels a share of the upper ones
        const int s0 = i0 + nb + nm, mb = nb ? ns : 0, mm = nb ? 0 : ns;
        const int cc = l - g.copy_lvl;
        CopyRanges c = cc >= 0 && cc < ncopy ? copy_chunk(g, cc, ncopy) : CopyRanges{0, 0, 0, 0};
        FuseArgs<T> f{fs, 0, 0, 0};
        if (fused) {
            if (solved < nfl && g.l_ready[solved] < copied) {
                f.j0 = g.l_lvl[solved];
                f.j1 = g.l_lvl[solved + 1];
                f.nsolve = std::min(f.j1 - f.j0, kFuseSolveBlocks);
                ++solved;
            }
            c = CopyRanges{g.copy_lat[copied], g.copy_lat[l], 0, 0};
            copied = l;
            if (cc >= 0) {
                const int uend = std::min<int>(g.copy_uat[l], (int)(u0 + (int64_t)nup * (++ktop) / ntop));
                if (uend > ucopied) {
                    c.b0 = ucopied;
                    c.b1 = uend;
                    ucopied = uend;
                }
            }
        }
        const int threads = nb ? (g.f_w256[l] ? W256::kThreads : Big::kThreads) : Med::kThreads;
        const int cb = copy_blocks(h, copy_count(c), threads);
        if (nb && g.f_w256[l])
            timed(h, KKT_PROF_REFACTOR_W256, s, [&] {
                const int grid = nb + (int)blocks_for(mb, W256::kThreads / 16) + f.nsolve + cb;
                k_refactor_wide<W256><<<grid, W256::kThreads, W256::kLds, s>>>(i0, a, nb, s0, mb, c, f);
            }, true);
        else if (nb)
            timed(h, KKT_PROF_REFACTOR_LARGE, s, [&] {
                const int grid = nb + (int)blocks_for(mb, Big::kThreads / 16) + f.nsolve + cb;
                k_refactor_wide<Big><<<grid, Big::kThreads, Big::kLds, s>>>(i0, a, nb, s0, mb, c, f);
            }, true);
        else
            timed(h, KKT_PROF_REFACTOR_MEDIUM, s, [&] {
                const int grid = nm + (int)blocks_for(mm, Med::kThreads / 16) + f.nsolve + cb;
                k_refactor_wide<Med><<<grid, Med::kThreads, Med::kLds, s>>>(i0, a, nm, s0, mm, c, f);
            }, true);
    }
    // the rest of the copy: the columns of the top levels (all of it without such levels), or
    // with fused the lower entries of the columns of the levels since the last launch and the
    // upper entries not copied yet; then the remaining forward levels
    const CopyRanges rest = fused ? CopyRanges{g.copy_lat[copied], u0, ucopied, (int)g.copy_k.size()}
                                  : copy_rest(g, ncopy);
    // the copy's last block sums the replaced-pivot counters (a launch of their own without a copy)
    const bool copy_rest_left = copy_count(rest) > 0;
    if (copy_rest_left)
        timed(h, KKT_PROF_TO_CSR, s, [&] {
            k_to_csr<T><<<blocks_for(copy_count(rest), 256) + 1, 256, 0, s>>>(rest, d.copy_k, d.copy_src, a.lu,
                                                                             a.lucsr, d.pcount, &d.st->perturbed);
        });
    if (fused && solved < nfl) {
        const int j0 = g.l_lvl[solved], j1 = g.l_lvl[nfl];
        timed(h, KKT_PROF_LSOLVE, s, [&] {
            k_lsolve_persistent<T, true><<<std::min(j1 - j0, h->grid_l), kBlock, 0, s>>>(j0, j1, fs);
        });
    }
    if (!copy_rest_left)
        timed(h, KKT_PROF_UPDATE, s, [&] { k_sum_counts<<<1, 256, 0, s>>>(d.pcount, &d.st->perturbed); });
    HIPCHK(hipGetLastError());
    return KKT_OK;
}

int enqueue_levels(kkt_handle *h, hipStream_t s, bool fused = false) {
    return by_precision(h, [&](auto tag) { return enqueue_levels_t<decltype(tag)>(h, s, fused); });
}

// dst[0..nv) = V[0..nv) . w  (deterministic two-pass reduction)
void enqueue_dots(kkt_handle *h, int nv, const double *V, const double *w, double *dst, int accumulate,
                  hipStream_t s) {
    const int n = h->sym.n;
    timed(h, KKT_PROF_KRYLOV, s, [&] { k_multidot<<<kDotBlocks, 256, 0, s>>>(n, nv, V, (int64_t)n, w, h->d.part); });
    timed(h, KKT_PROF_KRYLOV, s, [&] { k_reduce_parts<<<nv, 256, 0, s>>>(nv, kDotBlocks, h->d.part, dst, accumulate); });
}

// infinity norms of b - A x into the status block; returns berr on the host (and the
// status block read with it in *sto)
int residual_berr(kkt_handle *h, const double *x, const double *b, double *berr, double *den, hipStream_t s,
                  DevStatus *sto = nullptr) {
    const Dev &d = h->d;
    const int n = h->sym.n;
    timed(h, KKT_PROF_RESIDUAL, s, [&] {
        k_residual<<<kNormBlocks, 256, 0, s>>>(n, d.a_rowptr, d.a_colind, h->d_values, x, b, d.res, d.part);
    });
    timed(h, KKT_PROF_RESIDUAL, s, [&] { k_max_parts<<<1, 256, 0, s>>>(kNormBlocks, 3, d.part, &d.rn->rnorm); });
    // the residual norms are carved right after the status block: one read-back takes both
    const size_t off = static_cast<size_t>(reinterpret_cast<const char *>(d.rn) - reinterpret_cast<const char *>(d.st));
    if (off < sizeof(DevStatus) || off + sizeof(ResNorms) > sizeof(h->h_stage)) return KKT_ERR_DEVICE;
    HIPCHK(hipMemcpyAsync(h->h_small, d.st, off + sizeof(ResNorms), hipMemcpyDeviceToHost, s));
    HIPCHK(sync_fold(h, s));
    DevStatus st;
    ResNorms rn;
    std::memcpy(&st, h->h_small, sizeof(st));
    std::memcpy(&rn, reinterpret_cast<const char *>(h->h_small) + off, sizeof(rn));
    if (sto) *sto = st;
    if (st.abort) return KKT_ERR_DEVICE;
    *den = st.anorm * rn.xnorm + rn.bnorm;
    if (*den == 0.0) *berr = rn.rnorm == 0.0 ? 0.0 : INFINITY;
    else *berr = rn.rnorm / *den;
    return KKT_OK;
}

// Approximate preconditioner application: `sweeps` sweeps per triangle, each triangle from
// the zero vector, Jacobi (kind 0) or block Gauss-Seidel over chunks of kGsChunk rows
// (kind 1).  The exact solve's helper sums (psum, usum) serve as second iterate buffers.
template <class TF>
int enqueue_approx_solve_t(kkt_handle *h, const double *b, double *x, int sweeps, hipStream_t s) {
    const Dev &d = h->d;
    const TF *lucsr = static_cast<const TF *>(d.lucsr);
    const int n = h->sym.n;
    const bool gs = h->opts.approx_kind == 1;
    const unsigned nb8 = blocks_for((int64_t)n * 8, 256), nb = blocks_for(n, 256);
    const unsigned nch = blocks_for(n, kGsChunk);
    timed(h, KKT_PROF_LSOLVE, s, [&] {
        k_solve_reset<<<nb, 256, 0, s>>>(n, b, d.call, d.r, d.P, d.bp, d.y, d.xt, d.psum, d.usum, 0, 0, d.tick);
    });
    const double *yin = nullptr;
    double *ybuf[2] = {d.psum, d.y};
    for (int k = 0; k < sweeps; ++k) {
        double *yout = ybuf[k & 1];
        timed(h, KKT_PROF_LSOLVE, s, [&] {
            if (gs) k_bgs_l<TF><<<nch, kBlock, 0, s>>>(n, d.rinfo4, d.csr_col, lucsr, d.bp, yin, yout);
            else k_jacobi_l<TF><<<nb8, 256, 0, s>>>(n, d.rinfo4, d.csr_col, lucsr, d.bp, yin, yout);
        });
        yin = yout;
    }
    const double *xin = nullptr;
    double *xbuf[2] = {d.xt, d.usum};
    for (int k = 0; k < sweeps; ++k) {
        double *xout = xbuf[k & 1];
        timed(h, KKT_PROF_USOLVE, s, [&] {
            if (gs) k_bgs_u<TF><<<nch, kBlock, 0, s>>>(n, d.urinfo4, d.csr_col, lucsr, yin, xin, xout);
            else k_jacobi_u<TF><<<nb8, 256, 0, s>>>(n, d.urinfo4, d.csr_col, lucsr, yin, xin, xout);
        });
        xin = xout;
    }
    timed(h, KKT_PROF_USOLVE, s, [&] { k_unpermute<<<nb, 256, 0, s>>>(n, d.Q, d.c, xin, x); });
    HIPCHK(hipGetLastError());
    return KKT_OK;
}

int enqueue_approx_solve(kkt_handle *h, const double *b, double *x, int sweeps, hipStream_t s) {
    return by_precision(h, [&](auto tag) { return enqueue_approx_solve_t<decltype(tag)>(h, b, x, sweeps, s); });
}

// FGMRES on one column from the first solve x = M^-1 b.  fused: the refactorization and the
// forward part of that solve were enqueued together; the backward part is enqueued here and
// the factorization's status is checked with the first residual (a failed factorization
// returns its error with info = {0, error, inf, perturbed pivots}, as kkt_refine does).
int fgmres_column(kkt_handle *h, const double *b, double *x, kkt_info *info, hipStream_t s, bool fused = false) {
    const Dev &d = h->d;
    const int n = h->sym.n;
    const int m = h->opts.gmres_restart;
    const double tol = h->opts.berr_tol;
    int rc = enqueue_solve(h, b, x, s, !fused);
    if (rc) return rc;
    int64_t pert = 0;
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), gv(m + 1), yv(m);
    int it = 0;
    double berr = 0.0, den = 0.0;
    int status = KKT_OK;
    const unsigned nb = blocks_for(n, 256);
    for (bool first = true;; first = false) {
        DevStatus st{};
        rc = residual_berr(h, x, b, &berr, &den, s, &st);
        if (fused && first) {
            pert = (int64_t)st.perturbed;
            const int fst = ((st.flags & kFlagInternal) || st.abort) ? KKT_ERR_DEVICE
                            : (st.flags & kFlagNonfinite)            ? KKT_ERR_NONFINITE
                                                                     : KKT_OK;
            if (fst < 0) {
                if (info) *info = kkt_info{0, fst, INFINITY, pert};
                return fst;
            }
        }
        if (rc) return rc;
        if (berr <= tol) { status = KKT_OK; break; }
        if (it >= h->opts.max_iters || !std::isfinite(berr)) { status = KKT_WARN_NOT_CONVERGED; break; }
        const double target = tol * den;
        double *beta2 = d.hbuf + 3 * (m + 2);
        enqueue_dots(h, 1, d.res, d.res, beta2, 0, s);
        timed(h, KKT_PROF_KRYLOV, s, [&] { k_scale_by_norm<<<nb, 256, 0, s>>>(n, d.res, beta2, d.V); });
        std::fill(gv.begin(), gv.end(), 0.0);
        int jend = -1;
        for (int j = 0; j < m; ++j) {
            double *vj = d.V + (size_t)j * n, *zj = d.Z + (size_t)j * n;
            rc = h->opts.approx_sweeps > 0 ? enqueue_approx_solve(h, vj, zj, h->opts.approx_sweeps, s)
                                           : enqueue_solve(h, vj, zj, s);
            if (rc) return rc;
            timed(h, KKT_PROF_RESIDUAL, s, [&] {
                k_spmv<<<blocks_for((int64_t)n * 8, 256), 256, 0, s>>>(n, d.a_rowptr, d.a_colind, h->d_values, zj, d.w);
            });
            double *h1 = d.hbuf, *h2 = d.hbuf + (m + 2), *hn2 = d.hbuf + 2 * (m + 2);
            enqueue_dots(h, j + 1, d.V, d.w, h1, 0, s);
            timed(h, KKT_PROF_KRYLOV, s, [&] { k_sub_combo<<<nb, 256, 0, s>>>(n, j + 1, d.V, n, h1, d.w); });
            enqueue_dots(h, j + 1, d.V, d.w, h2, 0, s);
            timed(h, KKT_PROF_KRYLOV, s, [&] { k_sub_combo<<<nb, 256, 0, s>>>(n, j + 1, d.V, n, h2, d.w); });
            enqueue_dots(h, 1, d.w, d.w, hn2, 0, s);
            timed(h, KKT_PROF_KRYLOV, s,
                  [&] { k_scale_by_norm<<<nb, 256, 0, s>>>(n, d.w, hn2, d.V + (size_t)(j + 1) * n); });
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(h->h_small, d.hbuf, sizeof(double) * 4 * (m + 2), hipMemcpyDeviceToHost, s));
            HIPCHK(sync_fold(h, s));
            const double *hs = h->h_small;
            if (j == 0) gv[0] = std::sqrt(hs[3 * (m + 2)]);
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hs[i] + hs[(m + 2) + i];
            const double hn = std::sqrt(hs[2 * (m + 2)]);
            H[(size_t)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double a0 = H[(size_t)i * m + j], b0 = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a0 + sn[i] * b0;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a0 + cs[i] * b0;
            }
            const double a0 = H[(size_t)j * m + j], b0 = H[(size_t)(j + 1) * m + j];
            const double rr = std::hypot(a0, b0);
            cs[j] = rr > 0.0 ? a0 / rr : 1.0;
            sn[j] = rr > 0.0 ? b0 / rr : 0.0;
            H[(size_t)j * m + j] = rr;
            H[(size_t)(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            ++it;
            jend = j;
            if (std::fabs(gv[j + 1]) <= target || it >= h->opts.max_iters || hn == 0.0) break;
        }
        for (int i = jend; i >= 0; --i) {
            double t = gv[i];
            for (int q = i + 1; q <= jend; ++q) t -= H[(size_t)i * m + q] * yv[q];
            yv[i] = H[(size_t)i * m + i] != 0.0 ? t / H[(size_t)i * m + i] : 0.0;
        }
        std::memcpy(h->h_small, yv.data(), sizeof(double) * (jend + 1));
        HIPCHK(hipMemcpyAsync(d.ybuf, h->h_small, sizeof(double) * (jend + 1), hipMemcpyHostToDevice, s));
        timed(h, KKT_PROF_KRYLOV, s, [&] { k_add_combo<<<nb, 256, 0, s>>>(n, jend + 1, d.Z, n, d.ybuf, x); });
        HIPCHK(hipGetLastError());
        // the staging buffer is reused by the next read-back: wait for the upload
        HIPCHK(sync_fold(h, s));
    }
    if (info) {
        info->iters = it;
        info->berr = berr;
        info->status = status;
        if (fused) info->perturbed_pivots = pert;
    }
    return status;
}

}  // namespace

extern "C" {

void kkt_default_opts(kkt_opts *o) {
    if (!o) return;
    o->pivot_tau = 0.0;
    o->tiny_pivot = std::ldexp(1.0, -40);
    o->equilibrate = 1;
    o->gmres_restart = 30;
    o->max_iters = 100;
    o->berr_tol = 1e-10;
    o->sn_max_width = 256;
    o->fixed_p = nullptr;
    o->fixed_q = nullptr;
    o->dense_mfma = 1;
    o->persistent_solve = 1;
    o->graph_refactor = 1;
    o->approx_sweeps = 0;
    o->factor_precision = KKT_FP64;
    o->tiny_pivot_fp32 = std::ldexp(1.0, -26);
    o->approx_kind = 0;
}

int kkt_analyze(int32_t n, const int64_t *rowptr, const int32_t *colind, const double *values_k1,
                const kkt_opts *opts, kkt_handle **out) {
    if (!out) return KKT_ERR_ARG;
    *out = nullptr;
    kkt_opts o;
    kkt_default_opts(&o);
    if (opts) o = *opts;
    if (o.gmres_restart < 1 || o.gmres_restart > kMaxRestart || o.max_iters < 0 || !(o.berr_tol >= 0.0) ||
        !(o.tiny_pivot >= 0.0) || o.approx_sweeps < 0 || o.approx_sweeps > kMaxSweeps ||
        (o.factor_precision != KKT_FP64 && o.factor_precision != KKT_FP32) || !(o.tiny_pivot_fp32 >= 0.0) ||
        (o.approx_kind != 0 && o.approx_kind != 1) || o.persistent_solve < 0 || o.persistent_solve > 2)
        return KKT_ERR_ARG;
    kkt_handle *h = new (std::nothrow) kkt_handle;
    if (!h) return KKT_ERR_NOMEM;
    int rc;
    try {
        rc = analyze_symbolic(n, rowptr, colind, values_k1, o, h->sym);
        if (rc == KKT_OK) rc = build_schedule(h->sym, SchedParams{}, h->sch);
    } catch (const std::bad_alloc &) {
        rc = KKT_ERR_NOMEM;
    }
    if (rc != KKT_OK) {
        delete h;
        return rc;
    }
    o.fixed_p = nullptr;   // borrowed for the call only
    o.fixed_q = nullptr;
    h->opts = o;
    h->tickets = o.persistent_solve == 2;
    *out = h;
    return KKT_OK;
}

int kkt_clone(const kkt_handle *src, kkt_handle **out) {
    if (!src || !out) return KKT_ERR_ARG;
    *out = nullptr;
    kkt_handle *h = new (std::nothrow) kkt_handle;
    if (!h) return KKT_ERR_NOMEM;
    try {
        h->opts = src->opts;
        h->sym = src->sym;
        h->sch = src->sch;
        h->tickets = src->opts.persistent_solve == 2;
    } catch (const std::bad_alloc &) {
        delete h;
        return KKT_ERR_NOMEM;
    }
    *out = h;
    return KKT_OK;
}

int kkt_get_stats(const kkt_handle *h, kkt_stats *out) {
    if (!h || !out) return KKT_ERR_ARG;
    const Symbolic &s = h->sym;
    out->n = s.n;
    out->nsn = s.nsn();
    out->nnz_a = s.nnz_a;
    out->nnz_lu = s.nnz_lu();
    auto mx = [](const std::vector<int32_t> &v) { return v.empty() ? 0 : 1 + *std::max_element(v.begin(), v.end()); };
    out->levels_f = mx(s.lev_f);
    out->levels_l = mx(s.lev_l);
    out->levels_u = mx(s.lev_u);
    out->gpu_levels_f = (int32_t)h->sch.f_lvl.size() - 1;
    out->gpu_levels_l = (int32_t)h->sch.l_lvl.size() - 1;
    out->gpu_levels_u = (int32_t)h->sch.u_lvl.size() - 1;
    const bool pers = h->opts.persistent_solve != 0;
    out->persistent_levels_l = pers ? out->gpu_levels_l - h->sch.l_split : 0;
    out->persistent_levels_u = pers ? h->sch.u_split : 0;
    out->flops_refactor = h->sch.flops;
    out->nnz_lu_wide = h->sch.nnz_lu_wide;
    out->nnz_lu_medium = h->sch.nnz_lu_med;
    {
        const int nc = copy_carriers(h->sch);
        out->copy_in_levels = nc > 0 ? copy_count(copy_chunk(h->sch, 0, 1)) : 0;
    }
    out->nnz_lu_w256 = h->sch.nnz_lu_w256;
    return KKT_OK;
}

int kkt_export_symbolic(const kkt_handle *h, int32_t *P, int32_t *Q, int64_t *colptr, int32_t *rowidx,
                        int32_t *parent, int32_t *lev_f, int32_t *lev_l, int32_t *lev_u, int32_t *sn_start,
                        int64_t *map) {
    if (!h) return KKT_ERR_ARG;
    const Symbolic &s = h->sym;
    auto cp = [](auto *dst, const auto &v) {
        if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
    };
    cp(P, s.P);
    cp(Q, s.Q);
    cp(colptr, s.colptr);
    cp(rowidx, s.rowidx);
    cp(parent, s.parent);
    cp(lev_f, s.lev_f);
    cp(lev_l, s.lev_l);
    cp(lev_u, s.lev_u);
    cp(sn_start, s.sn_start);
    cp(map, s.map);
    return KKT_OK;
}

int kkt_workspace_bytes(const kkt_handle *h, int32_t max_nrhs, size_t *bytes) {
    if (!h || !bytes || max_nrhs < 1) return KKT_ERR_ARG;
    Dev probe{};
    carve(h, nullptr, probe, bytes);
    return KKT_OK;
}

}  // extern "C"

// Static device scratch of kkt_bind_scratch, one copy per device (each holds it until the
// process ends).  Host code never passes `scratch` itself to the device: its device address
// is taken once per device with hipGetSymbolAddress and kept in g_scratch_ptr.
static __device__ __align__(256) char scratch[KKT_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
kkt_handle *g_scratch_owner[kMaxDevices] = {};   // the handle bound to that device's scratch

// drops h's claim on its device's scratch array (the caller holds g_scratch_mu)
void release_scratch_locked(kkt_handle *h) {
    if (h->on_scratch && h->device >= 0 && h->device < kMaxDevices && g_scratch_owner[h->device] == h)
        g_scratch_owner[h->device] = nullptr;
    h->on_scratch = false;
}

// drops the recorded graphs (their addresses belong to the current workspace); the last
// replay may still run on a caller's stream
int drop_graphs(kkt_handle *h) {
    if (h->levels || h->fused) HIPCHK(hipEventSynchronize(h->levels_done));
    if (h->levels) HIPCHK(hipGraphExecDestroy(h->levels));
    if (h->fused) HIPCHK(hipGraphExecDestroy(h->fused));
    h->levels = nullptr;
    h->fused = nullptr;
    return KKT_OK;
}

// Common part of kkt_bind and kkt_bind_scratch: checks the size, records the device,
// uploads the structure into ws and waits.  no_alloc: take no pinned buffer, create no
// stream, event or graph (the level launches then go one by one).
int bind_common(kkt_handle *h, char *ws, size_t bytes, int32_t max_nrhs, hipStream_t stream, bool no_alloc) {
    size_t need = 0;
    Dev probe{};
    carve(h, nullptr, probe, &need);
    if (bytes < need) return KKT_ERR_NOMEM;
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    int ncu = 0;
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int ok = by_precision(h, [&](auto tag) {
        using T = decltype(tag);
        int bl = 0, bu = 0;
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_refactor_wide<BigCfg<T>>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, BigCfg<T>::kLds) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void *>(&k_refactor_wide<W256Cfg<T>>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, W256Cfg<T>::kLds) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void *>(&k_refactor_wide<MedCfg<T>>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, MedCfg<T>::kLds) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &bl, reinterpret_cast<const void *>(&k_lsolve_persistent<T, false>), kBlock, 0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &bu, reinterpret_cast<const void *>(&k_usolve_persistent<T, false>), kBlock, 0) != hipSuccess)
            return -1;
        h->grid_l = std::max(1, bl) * std::max(1, ncu);
        h->grid_u = std::max(1, bu) * std::max(1, ncu);
        return 0;
    });
    if (ok != 0) return KKT_ERR_DEVICE;
    h->ncu = std::max(1, ncu);
    {
        int coop = 0;
        HIPCHK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
        if (!coop) h->tickets = true;   // the fixed item order needs a cooperative launch
    }
    if (h->device >= 0 && h->device != dev) return KKT_ERR_STATE;   // rebinding keeps the device
    h->device = dev;
    h->bound = false;      // until the new workspace holds the structure
    h->factored = false;
    if (!h->h_pinned && !no_alloc)
        HIPCHK(hipHostMalloc(&h->h_pinned, sizeof(double) * 4 * (kMaxRestart + 2) + 256));
    h->h_small = h->h_pinned ? h->h_pinned : h->h_stage;
    {
        const int rc = drop_graphs(h);   // recorded with the previous workspace's addresses
        if (rc) return rc;
    }
    h->levels_failed = false;
    h->fused_failed = false;
    if (!no_alloc) {
        if (!h->cap) HIPCHK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
        if (!h->levels_done) HIPCHK(hipEventCreateWithFlags(&h->levels_done, hipEventDisableTiming));
    }
    carve(h, ws, h->d, &need);
    const Symbolic &s = h->sym;
    const Schedule &g = h->sch;
    const Dev &d = h->d;
    int rc = KKT_OK;
    rc |= upload(d.a_rowptr, g.a_rowptr32, stream);
    rc |= upload(d.a_colind, s.a_colind, stream);
    rc |= upload(reinterpret_cast<int32_t *>(d.lu_src), g.lu_src, stream);
    rc |= upload(d.colptr, g.colptr32, stream);
    rc |= upload(d.rowidx, s.rowidx, stream);
    rc |= upload(d.ulen, s.ulen, stream);
    rc |= upload(d.pan_start, g.pan_start, stream);
    rc |= upload(d.pan_r, g.pan_r, stream);
    rc |= upload(reinterpret_cast<int32_t *>(d.itemrec), g.itemrec, stream);
    rc |= upload(reinterpret_cast<int32_t *>(d.pair8), g.pair8, stream);
    rc |= upload(d.ldiag, g.ldiag, stream);
    rc |= upload(d.f_rel, g.f_rel, stream);
    rc |= upload(reinterpret_cast<int32_t *>(d.l_item4), g.l_item4, stream);
    rc |= upload(reinterpret_cast<int32_t *>(d.u_item4), g.u_item4, stream);
    rc |= upload(reinterpret_cast<int32_t *>(d.l_rows4), g.l_rows4, stream);
    rc |= upload(reinterpret_cast<int32_t *>(d.u_rows4), g.u_rows4, stream);
    rc |= upload(reinterpret_cast<int32_t *>(d.rinfo4), g.rinfo4, stream);
    rc |= upload(reinterpret_cast<int32_t *>(d.urinfo4), g.urinfo4, stream);
    rc |= upload(d.csr_col, g.csr_col, stream);
    rc |= upload(d.copy_k, g.copy_k, stream);
    rc |= upload(d.copy_src, g.copy_src, stream);
    rc |= upload(d.P, s.P, stream);
    rc |= upload(d.Q, s.Q, stream);
    if (rc) return KKT_ERR_DEVICE;
    HIPCHK(hipMemsetAsync(d.st, 0, sizeof(DevStatus), stream));
    HIPCHK(hipStreamSynchronize(stream));
    h->ws = ws;
    h->ws_bytes = bytes;
    h->max_nrhs = max_nrhs;
    h->on_scratch = no_alloc;
    h->bound = true;
    h->factored = false;
    return KKT_OK;
}

}  // namespace

extern "C" {

int kkt_bind(kkt_handle *h, void *d_workspace, size_t bytes, int32_t max_nrhs, hipStream_t stream) {
    if (!h || !d_workspace || max_nrhs < 1) return KKT_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256) return KKT_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    release_scratch_locked(h);
    return bind_common(h, static_cast<char *>(d_workspace), bytes, max_nrhs, stream, false);
}

int kkt_bind_scratch(kkt_handle *h, int32_t max_nrhs, hipStream_t stream) {
    if (!h || max_nrhs < 1) return KKT_ERR_ARG;
    size_t need = 0;
    Dev probe{};
    carve(h, nullptr, probe, &need);
    if (need > KKT_SCRATCH_BYTES) return KKT_ERR_NOMEM;   // beyond the static array
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return KKT_ERR_DEVICE;
    if (h->device >= 0 && h->device != dev) return KKT_ERR_STATE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {   // once per device, with that device current
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return KKT_ERR_DEVICE;
        g_scratch_ptr[dev] = p;
    }
    // the previous holder of this device's array loses its binding (its structure and
    // factors are about to be overwritten)
    kkt_handle *prev = g_scratch_owner[dev];
    if (prev && prev != h) {
        prev->bound = false;
        prev->factored = false;
        prev->on_scratch = false;
    }
    g_scratch_owner[dev] = nullptr;
    h->on_scratch = false;
    const int rc = bind_common(h, static_cast<char *>(g_scratch_ptr[dev]), KKT_SCRATCH_BYTES, max_nrhs, stream, true);
    if (rc == KKT_OK) g_scratch_owner[dev] = h;
    return rc;
}

namespace {

// records the level launches on the capture stream into h->levels; on any failure the
// calls fall back to launching them one by one
void record_levels(kkt_handle *h) {
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        h->levels_failed = true;
        return;
    }
    const int rc = enqueue_levels(h, h->cap);
    const hipError_t e = hipStreamEndCapture(h->cap, &graph);
    if (rc != KKT_OK || e != hipSuccess || !graph ||
        hipGraphInstantiate(&h->levels, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        h->levels = nullptr;
        h->levels_failed = true;
    }
    if (graph) (void)hipGraphDestroy(graph);
}

// records the level launches with the forward solve riding in them into h->fused; on any
// failure kkt_refactor_refine runs the two calls
void record_fused(kkt_handle *h) {
    hipGraph_t graph = nullptr;
    bool ok = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        const int rc = enqueue_levels(h, h->cap, true);
        const hipError_t e = hipStreamEndCapture(h->cap, &graph);
        ok = rc == KKT_OK && e == hipSuccess && graph &&
             hipGraphInstantiate(&h->fused, graph, nullptr, nullptr, 0) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        h->fused = nullptr;
        h->fused_failed = true;
    }
    if (graph) (void)hipGraphDestroy(graph);
}

// the level launches with the forward solve riding in them, replayed from h->fused (recorded
// at the first call) or, without graphs, with the profiler on or on a capturing stream,
// launched one by one
int run_fused_levels(kkt_handle *h, hipStream_t s) {
    if (h->opts.graph_refactor && !h->prof && !h->fused_failed && !h->on_scratch) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIPCHK(hipStreamIsCapturing(s, &cs));
        if (cs == hipStreamCaptureStatusNone) {
            if (!h->fused) record_fused(h);
            if (h->fused) {
                HIPCHK(hipGraphLaunch(h->fused, s));
                HIPCHK(hipEventRecord(h->levels_done, s));
                return KKT_OK;
            }
        }
    }
    return enqueue_levels(h, s, true);
}

int run_levels(kkt_handle *h, hipStream_t s) {
    if (h->opts.graph_refactor && !h->prof && !h->levels_failed && !h->on_scratch) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIPCHK(hipStreamIsCapturing(s, &cs));
        if (cs == hipStreamCaptureStatusNone) {
            if (!h->levels) record_levels(h);
            if (h->levels) {
                HIPCHK(hipGraphLaunch(h->levels, s));
                HIPCHK(hipEventRecord(h->levels_done, s));
                return KKT_OK;
            }
        }
    }
    return enqueue_levels(h, s);
}

}  // namespace

int kkt_refactor(kkt_handle *h, const double *d_values, hipStream_t stream) {
    if (!h || !d_values) return KKT_ERR_ARG;
    if (!h->bound) return KKT_ERR_STATE;
    DeviceGuard dg(h->device);
    if (!dg.ok) return KKT_ERR_DEVICE;
    int rc = set_call(h, d_values, nullptr, stream);
    if (!rc) rc = run_levels(h, stream);
    if (rc) return rc;
    h->d_values = d_values;
    h->factored = true;
    return KKT_OK;
}

int kkt_refactor_refine(kkt_handle *h, const double *d_values, const double *d_b, double *d_x, kkt_info *info,
                        hipStream_t stream) {
    if (!h || !d_values || !d_b || !d_x) return KKT_ERR_ARG;
    if (!h->bound) return KKT_ERR_STATE;
    DeviceGuard dg(h->device);
    if (!dg.ok) return KKT_ERR_DEVICE;
    const Dev &d = h->d;
    const int n = h->sym.n;
    const double *b = d_b;
    if (b == d_x) {   // the residuals read b after x is written
        HIPCHK(hipMemcpyAsync(d.bsave, b, sizeof(double) * n, hipMemcpyDeviceToDevice, stream));
        b = d.bsave;
    }
    int rc = set_call(h, d_values, b, stream);
    if (rc) return rc;
    rc = run_fused_levels(h, stream);
    if (rc) return rc;
    h->d_values = d_values;
    h->factored = true;
    kkt_info inf{};
    rc = fgmres_column(h, b, d_x, &inf, stream, true);
    if (info && (rc >= 0 || inf.status < 0)) *info = inf;   // a failed factorization fills inf
    return rc;
}

int kkt_refactor_status(kkt_handle *h, int64_t *perturbed, hipStream_t stream) {
    if (!h) return KKT_ERR_ARG;
    if (!h->factored) return KKT_ERR_STATE;
    DeviceGuard dg(h->device);
    if (!dg.ok) return KKT_ERR_DEVICE;
    HIPCHK(hipMemcpyAsync(h->h_small, h->d.st, sizeof(DevStatus), hipMemcpyDeviceToHost, stream));
    HIPCHK(sync_fold(h, stream));
    DevStatus st;
    std::memcpy(&st, h->h_small, sizeof(st));
    if (perturbed) *perturbed = (int64_t)st.perturbed;
    if ((st.flags & kFlagInternal) || st.abort) return KKT_ERR_DEVICE;
    if (st.flags & kFlagNonfinite) return KKT_ERR_NONFINITE;
    return st.perturbed ? KKT_WARN_PIVOT_PERTURBED : KKT_OK;
}

int kkt_solve(kkt_handle *h, const double *d_b, double *d_x, int32_t nrhs, int64_t ld, hipStream_t stream) {
    if (!h || !d_b || !d_x || nrhs < 1 || ld < h->sym.n) return KKT_ERR_ARG;
    if (!h->factored) return KKT_ERR_STATE;
    DeviceGuard dg(h->device);
    if (!dg.ok) return KKT_ERR_DEVICE;
    for (int32_t j = 0; j < nrhs; ++j) {
        const int rc = enqueue_solve(h, d_b + (size_t)j * ld, d_x + (size_t)j * ld, stream);
        if (rc) return rc;
    }
    return KKT_OK;
}

int kkt_solve_approx(kkt_handle *h, const double *d_b, double *d_x, int32_t nrhs, int64_t ld, hipStream_t stream) {
    if (!h || !d_b || !d_x || nrhs < 1 || ld < h->sym.n || h->opts.approx_sweeps < 1) return KKT_ERR_ARG;
    if (!h->factored) return KKT_ERR_STATE;
    DeviceGuard dg(h->device);
    if (!dg.ok) return KKT_ERR_DEVICE;
    for (int32_t j = 0; j < nrhs; ++j) {
        const double *b = d_b + (size_t)j * ld;
        double *x = d_x + (size_t)j * ld;
        if (b == x) {   // the sweeps read b after x is written
            HIPCHK(hipMemcpyAsync(h->d.bsave, b, sizeof(double) * h->sym.n, hipMemcpyDeviceToDevice, stream));
            b = h->d.bsave;
        }
        const int rc = enqueue_approx_solve(h, b, x, h->opts.approx_sweeps, stream);
        if (rc) return rc;
    }
    return KKT_OK;
}

int kkt_refine(kkt_handle *h, const double *d_b, double *d_x, int32_t nrhs, int64_t ld, kkt_info *info,
               hipStream_t stream) {
    if (!h || !d_b || !d_x || nrhs < 1 || ld < h->sym.n) return KKT_ERR_ARG;
    if (!h->factored) return KKT_ERR_STATE;
    DeviceGuard dg(h->device);
    if (!dg.ok) return KKT_ERR_DEVICE;
    int64_t pert = 0;
    const int fst = kkt_refactor_status(h, &pert, stream);
    if (fst < 0) {
        if (info)
            for (int32_t j = 0; j < nrhs; ++j) info[j] = kkt_info{0, fst, INFINITY, pert};
        return fst;
    }
    int worst = KKT_OK;
    for (int32_t j = 0; j < nrhs; ++j) {
        const double *b = d_b + (size_t)j * ld;
        double *x = d_x + (size_t)j * ld;
        if (b == x) {
            HIPCHK(hipMemcpyAsync(h->d.bsave, b, sizeof(double) * h->sym.n, hipMemcpyDeviceToDevice, stream));
            b = h->d.bsave;
        }
        kkt_info inf{};
        const int rc = fgmres_column(h, b, x, &inf, stream);
        if (rc < 0) return rc;
        inf.perturbed_pivots = pert;
        if (info) info[j] = inf;
        worst = std::max(worst, rc);
    }
    return worst;
}

int kkt_get_tuning(const kkt_handle *h, kkt_tuning *t) {
    if (!h || !t) return KKT_ERR_ARG;
    t->panel_max = h->sch.params.panel_max;
    t->small_rows = h->sch.params.small_rows;
    t->group = h->sch.params.group;
    t->wide256 = h->sch.params.wide256;
    t->fuse_chains = h->sch.params.fuse_chains;
    t->tiny_rows = h->sch.params.tiny_rows;
    return KKT_OK;
}

}  // extern "C"

namespace {

// drops the device binding of h (after its last work finished): the recorded graph goes,
// the workspace is no longer used
int unbind(kkt_handle *h) {
    {
        const int rc = drop_graphs(h);
        if (rc) return rc;
    }
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        release_scratch_locked(h);
    }
    h->bound = false;
    h->factored = false;
    h->ws = nullptr;
    return KKT_OK;
}

int set_schedule(kkt_handle *h, const SchedParams &p) {
    Schedule g;
    int rc;
    try {
        rc = build_schedule(h->sym, p, g);
    } catch (const std::bad_alloc &) {
        rc = KKT_ERR_NOMEM;
    }
    if (rc != KKT_OK) return rc;
    h->sch = std::move(g);
    return KKT_OK;
}

}  // namespace

extern "C" {

int kkt_set_tuning(kkt_handle *h, const kkt_tuning *t) {
    if (!h || !t) return KKT_ERR_ARG;
    if (h->device >= 0) {
        DeviceGuard dg(h->device);
        if (!dg.ok) return KKT_ERR_DEVICE;
        const int rc = unbind(h);
        if (rc) return rc;
    }
    return set_schedule(h, SchedParams{t->panel_max, t->small_rows, t->group, t->wide256, t->fuse_chains,
                                       t->tiny_rows});
}

int kkt_autotune(kkt_handle *h, const double *d_values, int32_t reps, kkt_tuning *best, double *best_ms,
                 hipStream_t stream) {
    if (!h || !d_values || reps < 1) return KKT_ERR_ARG;
    if (h->device >= 0) {
        DeviceGuard dg(h->device);
        if (!dg.ok) return KKT_ERR_DEVICE;
        const int rc = unbind(h);
        if (rc) return rc;
    }
    const SchedParams start = h->sch.params;
    SchedParams win = start;
    double win_ms = INFINITY;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int rc = KKT_OK;
    for (int32_t pm : {32, 16, 8})
        for (int32_t sr : {64, 32})
            for (int32_t gr : {32, 16})
            for (int32_t w2 : {1, 0})
            for (int32_t fc : {0, 1}) {
                rc = set_schedule(h, SchedParams{pm, sr, gr, w2, fc, start.tiny_rows});
                if (rc == KKT_ERR_SCHEDULE) { rc = KKT_OK; continue; }   // not a valid cut for this pattern
                if (rc) break;
                size_t bytes = 0;
                Dev probe{};
                carve(h, nullptr, probe, &bytes);
                void *ws = nullptr;
                if (hipMalloc(&ws, bytes) != hipSuccess) { rc = KKT_ERR_NOMEM; break; }
                float ms = 0.0f;
                rc = bind_common(h, static_cast<char *>(ws), bytes, 1, stream, false);
                if (!rc) rc = kkt_refactor(h, d_values, stream);   // records the graph
                if (!rc && hipEventRecord(e0, stream) != hipSuccess) rc = KKT_ERR_DEVICE;
                for (int32_t k = 0; k < reps && !rc; ++k) rc = kkt_refactor(h, d_values, stream);
                if (!rc && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    rc = KKT_ERR_DEVICE;
                if (!rc) {
                    int64_t pert = 0;
                    const int st = kkt_refactor_status(h, &pert, stream);
                    if (st < 0) rc = st;
                }
                (void)hipStreamSynchronize(stream);
                const int urc = unbind(h);
                (void)hipFree(ws);
                if (rc) break;
                if (urc) { rc = urc; break; }
                if (ms / reps < win_ms) {
                    win_ms = ms / reps;
                    win = SchedParams{pm, sr, gr, w2, fc, start.tiny_rows};
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const int rc2 = set_schedule(h, rc ? start : win);
    if (rc) return rc;
    if (rc2) return rc2;
    if (best) {
        best->panel_max = win.panel_max;
        best->small_rows = win.small_rows;
        best->group = win.group;
        best->wide256 = win.wide256;
        best->fuse_chains = win.fuse_chains;
        best->tiny_rows = win.tiny_rows;
    }
    if (best_ms) *best_ms = win_ms;
    return KKT_OK;
}

int kkt_export_factors(kkt_handle *h, double *h_lu, double *h_r, double *h_c, hipStream_t stream) {
    if (!h || !h_lu) return KKT_ERR_ARG;
    if (!h->factored) return KKT_ERR_STATE;
    DeviceGuard dg(h->device);
    if (!dg.ok) return KKT_ERR_DEVICE;
    const size_t nlu = (size_t)h->sym.nnz_lu();
    if (h->opts.factor_precision == KKT_FP32) {
        // FP32 factors are widened (exactly) into the caller's FP64 array
        std::vector<float> tmp;
        try {
            tmp.resize(nlu);
        } catch (const std::bad_alloc &) {
            return KKT_ERR_NOMEM;
        }
        HIPCHK(hipMemcpyAsync(tmp.data(), h->d.lu, sizeof(float) * nlu, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        for (size_t k = 0; k < nlu; ++k) h_lu[k] = (double)tmp[k];
    } else {
        HIPCHK(hipMemcpyAsync(h_lu, h->d.lu, sizeof(double) * nlu, hipMemcpyDeviceToHost, stream));
    }
    if (h_r) HIPCHK(hipMemcpyAsync(h_r, h->d.r, sizeof(double) * h->sym.n, hipMemcpyDeviceToHost, stream));
    if (h_c) HIPCHK(hipMemcpyAsync(h_c, h->d.c, sizeof(double) * h->sym.n, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    return KKT_OK;
}

int kkt_profile_enable(kkt_handle *h, int32_t on) {
    if (!h) return KKT_ERR_ARG;
    close_run(h);
    h->prof = on != 0;
    if (h->prof) h->acc = kkt_profile{};
    return KKT_OK;
}

int kkt_profile_read(kkt_handle *h, kkt_profile *out, hipStream_t stream) {
    if (!h || !out) return KKT_ERR_ARG;
    close_run(h);
    if (!h->ev_pending.empty()) HIPCHK(sync_fold(h, stream));
    *out = h->acc;
    return KKT_OK;
}

void kkt_destroy(kkt_handle *h) {
    if (!h) return;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        release_scratch_locked(h);
    }
    // order: wait for the last replay and for every profiled launch, then release the graph,
    // the capture stream, the events and last the pinned staging buffer
    if (h->device >= 0) {
        DeviceGuard g(h->device);
        close_run(h);
        if (h->levels_done) (void)hipEventSynchronize(h->levels_done);
        for (auto &pe : h->ev_pending) (void)hipEventSynchronize(pe.second.second);
        if (h->cap) (void)hipStreamSynchronize(h->cap);
        if (h->levels) (void)hipGraphExecDestroy(h->levels);
        if (h->fused) (void)hipGraphExecDestroy(h->fused);
        if (h->cap) (void)hipStreamDestroy(h->cap);
        if (h->levels_done) (void)hipEventDestroy(h->levels_done);
        for (auto &pe : h->ev_pending) h->ev_free.push_back(pe.second);
        for (auto &ev : h->ev_free) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
    }
    if (h->h_pinned) (void)hipHostFree(h->h_pinned);
    delete h;
}

const char *kkt_strerror(int status) {
    switch (status) {
        case KKT_OK: return "ok";
        case KKT_WARN_PIVOT_PERTURBED: return "tiny pivots were replaced during refactorization";
        case KKT_WARN_NOT_CONVERGED: return "iterative refinement did not reach the backward-error target";
        case KKT_ERR_ARG: return "invalid argument";
        case KKT_ERR_PATTERN: return "invalid sparsity pattern";
        case KKT_ERR_SINGULAR: return "structurally or numerically singular at analysis";
        case KKT_ERR_NONFINITE: return "non-finite value in matrix or factors";
        case KKT_ERR_STATE: return "call out of order";
        case KKT_ERR_NOMEM: return "out of memory or workspace too small";
        case KKT_ERR_DEVICE: return "HIP runtime error";
        case KKT_ERR_SCHEDULE: return "internal GPU schedule invariant or limit violated";
        default: return "unknown status";
    }
}

}  // extern "C"
#include "kkt_batch.hip"
