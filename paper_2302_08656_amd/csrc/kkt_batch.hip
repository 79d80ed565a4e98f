// Batched refactorization: several bound handles (same device, same factor precision; the
// same or different patterns) refactored by one launch per dependency level across the
// whole batch, the value update merged likewise, and every launch of a batch step recorded
// once into a HIP graph that later steps replay.  Included by kkt_runtime.hip (it needs the
// handle's internals).
//
// Each launch is cut into shares, one per handle: share p runs blocks [blk0, blk0 + nblk)
// of the launch with that handle's arguments, exactly the blocks a launch of the handle
// alone would run, so every handle's result is bitwise the same as refactoring it alone.

namespace kkt {

// Everything the batched kernels read of one handle.
template <class T>
struct BatchSys {
    RefArgs<T> ref;
    const int32_t *a_rowptr, *a_colind, *colptr, *Q;
    const int2 *lu_src;
    double *r, *c, *part;
    int16_t *er, *ec;
    int n, eq, nb_norm;
    CopyRanges rest;   // the copy after the last level
};

// One handle's share of a batched launch.
struct BatchPart {
    int sys, blk0, nblk, item0, nwide, small0, nsmall;
    CopyRanges c;   // the level's chunk of the row-ordered copy
    int pad0;
};

// the share that runs block b (shares are sorted by blk0, the first starts at 0)
__device__ __forceinline__ int find_part(const BatchPart *__restrict__ parts, int nparts, int b) {
    int lo = 0, hi = nparts - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (parts[mid].blk0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <class T>
__global__ __launch_bounds__(256) void k_batch_clear(const BatchSys<T> *__restrict__ sys) {
    clear_status_body(sys[blockIdx.x].ref.st, sys[blockIdx.x].ref.pcount);
}

template <class T>
__global__ __launch_bounds__(256) void k_batch_rows(const BatchSys<T> *__restrict__ sys,
                                                    const BatchPart *__restrict__ parts, int nparts,
                                                    const double *const *__restrict__ vals) {
    const BatchPart P = parts[find_part(parts, nparts, blockIdx.x)];
    const BatchSys<T> &S = sys[P.sys];
    row_scale_body(blockIdx.x - P.blk0, S.n, S.a_rowptr, vals[P.sys], S.eq, S.r, S.er, S.ref.st);
}

template <class T>
__global__ __launch_bounds__(256) void k_batch_cols(const BatchSys<T> *__restrict__ sys,
                                                    const BatchPart *__restrict__ parts, int nparts,
                                                    const double *const *__restrict__ vals) {
    const BatchPart P = parts[find_part(parts, nparts, blockIdx.x)];
    const BatchSys<T> &S = sys[P.sys];
    col_store_body<T>(blockIdx.x - P.blk0, S.n, S.colptr, S.lu_src, S.Q, vals[P.sys], S.er, S.eq, S.c, S.ec,
                      S.ref.lu);
}

template <class T>
__global__ __launch_bounds__(256) void k_batch_rowsums(const BatchSys<T> *__restrict__ sys,
                                                       const BatchPart *__restrict__ parts, int nparts,
                                                       const double *const *__restrict__ vals) {
    const BatchPart P = parts[find_part(parts, nparts, blockIdx.x)];
    const BatchSys<T> &S = sys[P.sys];
    norms_body(blockIdx.x - P.blk0, P.nblk, S.n, S.a_rowptr, S.a_colind, vals[P.sys], S.r, S.ec, S.part);
}

template <class T>
__global__ __launch_bounds__(256) void k_batch_norms(const BatchSys<T> *__restrict__ sys) {
    const BatchSys<T> &S = sys[blockIdx.x];
    max_parts_body(S.nb_norm, 2, S.part, &S.ref.st->anorm_scaled);
}

template <class C>
__global__ __launch_bounds__(C::kThreads, C::kWaves) void k_batch_level(const BatchSys<typename C::T> *__restrict__ sys,
                                                                       const BatchPart *__restrict__ parts,
                                                                       int nparts) {
    extern __shared__ __align__(16) char sm[];
    const BatchPart P = parts[find_part(parts, nparts, blockIdx.x)];
    const RefArgs<typename C::T> a = sys[P.sys].ref;
    refactor_block<C>(blockIdx.x - P.blk0, P.nblk, P.item0, a, P.nwide, P.small0, P.nsmall, P.c,
                      FuseArgs<typename C::T>{}, sm);
}

// the copy after the last level and the replaced-pivot sums
template <class T>
__global__ void k_batch_copy(const BatchSys<T> *__restrict__ sys, const BatchPart *__restrict__ parts, int nparts) {
    const BatchPart P = parts[find_part(parts, nparts, blockIdx.x)];
    const BatchSys<T> &S = sys[P.sys];
    copy_ranges(S.ref.copy_k, S.ref.copy_src, S.ref.lu, S.ref.lucsr, S.rest, blockIdx.x - P.blk0, P.nblk,
                blockDim.x);
}

template <class T>
__global__ __launch_bounds__(256) void k_batch_counts(const BatchSys<T> *__restrict__ sys) {
    sum_counts_body(sys[blockIdx.x].ref.pcount, &sys[blockIdx.x].ref.st->perturbed);
}

}  // namespace kkt

// worker threads (and streams) of kkt_batch_refine
constexpr int kBatchRefineThreads = 8;

struct kkt_batch {
    std::vector<kkt_handle *> hs;
    std::vector<char *> ws;        // each handle's workspace when the batch was made
    int device = -1;
    bool fp32 = false;
    char *dmem = nullptr;          // device: systems, shares, value-pointer table
    void *d_sys = nullptr;
    const double **d_vals = nullptr;
    const double **h_vals = nullptr;   // pinned staging of the value pointers
    hipEvent_t vals_done = nullptr;    // the last upload of h_vals has been read
    // launches of a step: kind (0 clear, 1 rows, 2 cols, 3 scatter, 4 norms, 5 level,
    // 6 copy, 7 counts), grid, first share, shares
    struct Launch {
        int kind, grid, p0, np;
    };
    std::vector<Launch> launches;
    BatchPart *d_parts = nullptr;
    hipStream_t cap = nullptr;
    hipGraphExec_t graph = nullptr;
    hipEvent_t graph_done = nullptr;
    bool graph_failed = false;
    // concurrent refinement: one stream per worker thread, and an event that orders them
    // after the caller's stream
    std::vector<hipStream_t> rstreams;
    hipEvent_t ready = nullptr;
};

namespace {

template <class T>
BatchSys<T> batch_sys(const kkt_handle *h) {
    const Dev &d = h->d;
    const Schedule &g = h->sch;
    BatchSys<T> b{};
    b.ref = RefArgs<T>{d.ldiag, d.itemrec, d.pair8, d.f_rel, static_cast<T *>(d.lu), d.st, d.pcount,
                       std::is_same<T, float>::value ? h->opts.tiny_pivot_fp32 : h->opts.tiny_pivot,
                       h->opts.dense_mfma != 0, d.copy_k, d.copy_src, static_cast<T *>(d.lucsr),
                       d.pan_start, d.pan_r};
    b.a_rowptr = d.a_rowptr;
    b.a_colind = d.a_colind;
    b.colptr = d.colptr;
    b.Q = d.Q;
    b.lu_src = d.lu_src;
    b.r = d.r;
    b.c = d.c;
    b.er = d.er;
    b.ec = d.ec;
    b.part = d.part;
    b.n = h->sym.n;
    b.eq = h->opts.equilibrate != 0;
    b.nb_norm = norm_blocks(h->sym.n);
    b.rest = copy_rest(g, copy_carriers(g));
    return b;
}

template <class T>
int batch_build(kkt_batch *b, std::vector<BatchPart> &parts, std::vector<char> &sysbytes) {
    using Big = BigCfg<T>;
    const int count = (int)b->hs.size();
    std::vector<BatchSys<T>> sys(count);
    for (int i = 0; i < count; ++i) sys[i] = batch_sys<T>(b->hs[i]);
    sysbytes.resize(sizeof(BatchSys<T>) * count);
    std::memcpy(sysbytes.data(), sys.data(), sysbytes.size());
    auto add = [&](int kind, const std::vector<BatchPart> &ps) {
        int grid = 0;
        for (const auto &p : ps) grid = std::max(grid, p.blk0 + p.nblk);
        if (grid == 0 && kind != 0 && kind != 4 && kind != 7) return;
        b->launches.push_back({kind, kind == 0 || kind == 4 || kind == 7 ? count : grid, (int)parts.size(),
                               (int)ps.size()});
        parts.insert(parts.end(), ps.begin(), ps.end());
    };
    auto shares = [&](auto nblk_of) {
        std::vector<BatchPart> ps;
        int blk = 0;
        for (int i = 0; i < count; ++i) {
            BatchPart p{};
            p.sys = i;
            p.blk0 = blk;
            p.nblk = nblk_of(i, p);
            if (p.nblk > 0) {
                ps.push_back(p);
                blk += p.nblk;
            }
        }
        return ps;
    };
    add(0, {});
    add(1, shares([&](int i, BatchPart &) { return row_blocks(sys[i].n); }));
    add(2, shares([&](int i, BatchPart &) { return col_blocks(sys[i].n); }));
    add(3, shares([&](int i, BatchPart &) { return sys[i].nb_norm; }));
    add(4, {});
    int nlev = 0;
    for (auto *h : b->hs) nlev = std::max(nlev, (int)h->sch.f_lvl.size() - 1);
    for (int l = 0; l < nlev; ++l) {
        add(5, shares([&](int i, BatchPart &p) {
            const kkt_handle *h = b->hs[i];
            const Schedule &g = h->sch;
            if (l + 1 >= (int)g.f_lvl.size()) return 0;
            const int i0 = g.f_lvl[l], nw = g.f_nlarge[l], ns = g.f_lvl[l + 1] - i0 - nw;
            const int ncopy = copy_carriers(g), cc = l - g.copy_lvl;
            const bool copy = cc >= 0 && cc < ncopy && nw > 0;
            p.item0 = i0;
            p.nwide = nw;
            p.small0 = i0 + nw;
            p.nsmall = ns;
            p.c = copy ? copy_chunk(g, cc, ncopy) : CopyRanges{0, 0, 0, 0};
            const int cb = copy_count(p.c) > 0 ? h->ncu : 0;
            return nw + (int)blocks_for(ns, Big::kThreads / 16) + cb;
        }));
    }
    add(6, shares([&](int i, BatchPart &) { return (int)blocks_for(copy_count(sys[i].rest), 256); }));
    add(7, {});
    return KKT_OK;
}

template <class T>
int batch_enqueue(kkt_batch *b, hipStream_t s) {
    using Big = BigCfg<T>;
    const auto *sys = static_cast<const BatchSys<T> *>(b->d_sys);
    for (const auto &L : b->launches) {
        const BatchPart *p = b->d_parts + L.p0;
        switch (L.kind) {
            case 0: k_batch_clear<T><<<L.grid, 256, 0, s>>>(sys); break;
            case 1: k_batch_rows<T><<<L.grid, 256, 0, s>>>(sys, p, L.np, b->d_vals); break;
            case 2: k_batch_cols<T><<<L.grid, 256, 0, s>>>(sys, p, L.np, b->d_vals); break;
            case 3: k_batch_rowsums<T><<<L.grid, 256, 0, s>>>(sys, p, L.np, b->d_vals); break;
            case 4: k_batch_norms<T><<<L.grid, 256, 0, s>>>(sys); break;
            case 5: k_batch_level<Big><<<L.grid, Big::kThreads, Big::kLds, s>>>(sys, p, L.np); break;
            case 6: k_batch_copy<T><<<L.grid, 256, 0, s>>>(sys, p, L.np); break;
            case 7: k_batch_counts<T><<<L.grid, 256, 0, s>>>(sys); break;
        }
    }
    HIPCHK(hipGetLastError());
    return KKT_OK;
}

int batch_enqueue_any(kkt_batch *b, hipStream_t s) {
    return b->fp32 ? batch_enqueue<float>(b, s) : batch_enqueue<double>(b, s);
}

void batch_free(kkt_batch *b) {
    if (b->device >= 0) {
        DeviceGuard g(b->device);
        if (b->graph_done) (void)hipEventSynchronize(b->graph_done);
        if (b->vals_done) (void)hipEventSynchronize(b->vals_done);
        if (b->cap) (void)hipStreamSynchronize(b->cap);
        if (b->graph) (void)hipGraphExecDestroy(b->graph);
        if (b->cap) (void)hipStreamDestroy(b->cap);
        if (b->graph_done) (void)hipEventDestroy(b->graph_done);
        for (hipStream_t st : b->rstreams) (void)hipStreamDestroy(st);
        if (b->ready) (void)hipEventDestroy(b->ready);
        if (b->vals_done) (void)hipEventDestroy(b->vals_done);
        if (b->dmem) (void)hipFree(b->dmem);
        if (b->h_vals) (void)hipHostFree(b->h_vals);
    }
    delete b;
}

}  // namespace

extern "C" {

int kkt_batch_create(kkt_handle *const *handles, int32_t count, kkt_batch **out) {
    if (!out) return KKT_ERR_ARG;
    *out = nullptr;
    if (!handles || count < 1) return KKT_ERR_ARG;
    for (int32_t i = 0; i < count; ++i) {
        if (!handles[i]) return KKT_ERR_ARG;
        for (int32_t j = 0; j < i; ++j)
            if (handles[j] == handles[i]) return KKT_ERR_ARG;   // one workspace, one slot
        if (!handles[i]->bound) return KKT_ERR_STATE;
        if (handles[i]->device != handles[0]->device ||
            handles[i]->opts.factor_precision != handles[0]->opts.factor_precision)
            return KKT_ERR_ARG;
    }
    kkt_batch *b = new (std::nothrow) kkt_batch;
    if (!b) return KKT_ERR_NOMEM;
    b->hs.assign(handles, handles + count);
    for (auto *h : b->hs) b->ws.push_back(h->ws);
    b->device = handles[0]->device;
    b->fp32 = handles[0]->opts.factor_precision == KKT_FP32;
    DeviceGuard dg(b->device);
    if (!dg.ok) { batch_free(b); return KKT_ERR_DEVICE; }
    std::vector<BatchPart> parts;
    std::vector<char> sysbytes;
    int rc;
    try {
        rc = b->fp32 ? batch_build<float>(b, parts, sysbytes) : batch_build<double>(b, parts, sysbytes);
    } catch (const std::bad_alloc &) {
        rc = KKT_ERR_NOMEM;
    }
    if (rc) { batch_free(b); return rc; }
    const size_t off_parts = (sysbytes.size() + 255) & ~size_t(255);
    const size_t off_vals = (off_parts + parts.size() * sizeof(BatchPart) + 255) & ~size_t(255);
    const size_t total = off_vals + sizeof(double *) * count;
    if (hipMalloc(&b->dmem, total) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&b->h_vals), sizeof(double *) * count) != hipSuccess ||
        hipEventCreateWithFlags(&b->vals_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->graph_done, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ready, hipEventDisableTiming) != hipSuccess) {
        batch_free(b);
        return KKT_ERR_DEVICE;
    }
    for (int i = 0; i < std::min(count, kBatchRefineThreads); ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            batch_free(b);
            return KKT_ERR_DEVICE;
        }
        b->rstreams.push_back(st);
    }
    // refinements of several handles run at once on those streams: their persistent solves
    // take items by ticket (bitwise the same results as the fixed order)
    for (auto *h : b->hs) h->tickets = true;
    {
        const hipError_t e = b->fp32 ? hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch_level<BigCfg<float>>),
                                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                                           BigCfg<float>::kLds)
                                     : hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch_level<BigCfg<double>>),
                                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                                           BigCfg<double>::kLds);
        if (e != hipSuccess) {
            batch_free(b);
            return KKT_ERR_DEVICE;
        }
    }
    b->d_sys = b->dmem;
    b->d_parts = reinterpret_cast<BatchPart *>(b->dmem + off_parts);
    b->d_vals = reinterpret_cast<const double **>(b->dmem + off_vals);
    if (hipMemcpy(b->d_sys, sysbytes.data(), sysbytes.size(), hipMemcpyHostToDevice) != hipSuccess ||
        (!parts.empty() && hipMemcpy(b->d_parts, parts.data(), parts.size() * sizeof(BatchPart),
                                     hipMemcpyHostToDevice) != hipSuccess) ||
        hipEventRecord(b->vals_done, nullptr) != hipSuccess) {
        batch_free(b);
        return KKT_ERR_DEVICE;
    }
    *out = b;
    return KKT_OK;
}

int kkt_batch_refactor(kkt_batch *b, const double *const *d_values, hipStream_t stream) {
    if (!b || !d_values) return KKT_ERR_ARG;
    const int count = (int)b->hs.size();
    for (int i = 0; i < count; ++i) {
        if (!d_values[i]) return KKT_ERR_ARG;
        if (!b->hs[i]->bound || b->hs[i]->ws != b->ws[i]) return KKT_ERR_STATE;   // unbound or rebound since
    }
    DeviceGuard dg(b->device);
    if (!dg.ok) return KKT_ERR_DEVICE;
    // the pinned staging of the value pointers is rewritten once its last upload was read
    HIPCHK(hipEventSynchronize(b->vals_done));
    for (int i = 0; i < count; ++i) b->h_vals[i] = d_values[i];
    HIPCHK(hipMemcpyAsync(b->d_vals, b->h_vals, sizeof(double *) * count, hipMemcpyHostToDevice, stream));
    HIPCHK(hipEventRecord(b->vals_done, stream));
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHK(hipStreamIsCapturing(stream, &cs));
    int rc = KKT_OK;
    if (!b->graph && !b->graph_failed && cs == hipStreamCaptureStatusNone) {
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            const int erc = batch_enqueue_any(b, b->cap);
            const hipError_t e = hipStreamEndCapture(b->cap, &graph);
            if (erc || e != hipSuccess || !graph || hipGraphInstantiate(&b->graph, graph, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGetLastError();
                b->graph = nullptr;
                b->graph_failed = true;
            }
            if (graph) (void)hipGraphDestroy(graph);
        } else {
            (void)hipGetLastError();
            b->graph_failed = true;
        }
    }
    if (b->graph && cs == hipStreamCaptureStatusNone) {
        HIPCHK(hipGraphLaunch(b->graph, stream));
        HIPCHK(hipEventRecord(b->graph_done, stream));
    } else {
        rc = batch_enqueue_any(b, stream);
        if (rc) return rc;
    }
    for (int i = 0; i < count; ++i) {
        b->hs[i]->d_values = d_values[i];
        b->hs[i]->factored = true;
    }
    return KKT_OK;
}

int kkt_batch_refine(kkt_batch *b, const double *const *d_b, double *const *d_x, kkt_info *info,
                     hipStream_t stream) {
    if (!b || !d_b || !d_x) return KKT_ERR_ARG;
    const int count = (int)b->hs.size();
    for (int i = 0; i < count; ++i)
        if (!d_b[i] || !d_x[i]) return KKT_ERR_ARG;
    DeviceGuard dg(b->device);
    if (!dg.ok) return KKT_ERR_DEVICE;
    // the refinement streams start after everything enqueued on the caller's stream so far
    HIPCHK(hipEventRecord(b->ready, stream));
    for (hipStream_t st : b->rstreams) HIPCHK(hipStreamWaitEvent(st, b->ready, 0));
    std::vector<int> rcs(count, KKT_OK);
    std::vector<kkt_info> infs(count);
    std::atomic<int> next(0);
    auto work = [&](hipStream_t st) {
        (void)hipSetDevice(b->device);
        for (int i; (i = next.fetch_add(1)) < count;)
            rcs[i] = kkt_refine(b->hs[i], d_b[i], d_x[i], 1, b->hs[i]->sym.n, &infs[i], st);
    };
    std::vector<std::thread> pool;
    try {
        for (size_t t = 1; t < b->rstreams.size(); ++t) pool.emplace_back(work, b->rstreams[t]);
    } catch (...) {
        // fewer threads: the remaining handles go to the ones that started
    }
    work(b->rstreams[0]);
    for (auto &t : pool) t.join();
    int worst = KKT_OK;
    for (int i = 0; i < count; ++i) {
        if (info) info[i] = infs[i];
        if (rcs[i] < 0 && worst >= 0) worst = rcs[i];
        else if (worst >= 0) worst = std::max(worst, rcs[i]);
    }
    return worst;
}

void kkt_batch_destroy(kkt_batch *b) {
    if (b) batch_free(b);
}

}  // extern "C"
