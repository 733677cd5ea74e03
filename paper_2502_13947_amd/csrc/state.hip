// The main loop of Alg. 2 inside the library: a run's state (solution set,
// fields, energies, Tabu statistics, keys, the sub-QUBO batch and its
// annealer buffers, the best solution) and the fixed sequence of launches of
// one outer iteration.  Every per-iteration scalar (iteration number t for
// the mutation rate and the random keys, the annealer's instance base, the
// trace position) lives in a device record that the last kernel of the
// iteration advances, so one captured iteration replays every later one.
#include <algorithm>
#include <vector>

#include "qb_internal.h"

struct qb_state_s {
    qb_problem P = nullptr;
    int n = 0, z = 0, k = 0;
    qb_run_cfg cfg{};
    std::vector<int32_t> job_m;
    float scales[7] = {0};
    qb_batch batch = nullptr;     // z * k jobs, solution-major
    qb_batch ib = nullptr;        // initial pass: z jobs of init_m (block after block) or z * L0 (at once)
    qb_batch empty = nullptr;     // No_IM: no jobs, so every variable is a mutation candidate
    int L0 = 0;                   // blocks of the initial pass
    uint32_t inst0 = 0;           // instance base after the initial pass
    int tile_esz = 1;             // bytes per dense tile element
    bool learned = false, tracing = false, random_select = false, no_im = false;
    qb_state_buffers b{};         // buffers in use
    // owned internals
    void *itiles = nullptr;
    int32_t *iF0 = nullptr;
    uint8_t *iy0 = nullptr, *iY = nullptr;
    int64_t *ie = nullptr;
    int64_t *KR = nullptr, *K0 = nullptr;
    int32_t *orderR = nullptr, *kcount = nullptr;
    int32_t *thr = nullptr, *thr_init = nullptr;
    double *rate_tab = nullptr;
    qb_iter *it = nullptr;
    std::vector<void *> owned;
    hipStream_t cap = nullptr;    // capture stream of the iteration graph
    hipGraphExec_t graph = nullptr;
    bool timing = false;          // stage events of eager iterations
    hipEvent_t ev[QB_NSTAGE + 1] = {nullptr};
};

namespace {

__global__ void k_fill_i64(int64_t *__restrict__ p, int64_t v) { p[0] = v; }

// idx of the initial pass, block l of init_m for every job: job q (of
// solution q / per_sol) takes variables l m .. l m + m - 1, l = l0 + q mod
// per_sol (per_sol = 1: block after block; per_sol = L0: every block at once)
__global__ void k_block_idx(int32_t *__restrict__ idx, int jobs, int per_sol, int m, int l0)
{
    const int q = blockIdx.x;
    if (q >= jobs) return;
    const int l = l0 + q % per_sol;
    for (int a = threadIdx.x; a < m; a += blockDim.x) idx[(int64_t)q * m + a] = l * m + a;
}

__global__ void k_set_iter(qb_iter *__restrict__ it, int t, uint32_t inst, int keep_trn)
{
    it->t = t;
    it->inst = inst;
    if (!keep_trn) it->trn = 0;
    it->pad = 0;
}

// end of an outer iteration: E_best of iteration t recorded, t + 1, the
// instance base moved past this iteration's jobs, the trace rows counted
// when they were written (the trace kernel's own room test)
__global__ void k_advance(qb_iter *__restrict__ it, uint32_t jobs, int total, int64_t cap, int tracing,
                          const int64_t *__restrict__ ebest, int64_t *__restrict__ trace, int ntrace)
{
    const int t = it->t;
    if (trace && t < ntrace) trace[t] = ebest[0];
    it->t = t + 1;
    it->inst += jobs;
    if (tracing && (int64_t)it->trn + total <= cap) it->trn += total;
}

template <typename T>
bool alloc(qb_state S, T **p, size_t count)
{
    void *v = nullptr;
    if (hipMalloc(&v, std::max<size_t>(count * sizeof(T), 16)) != hipSuccess) return false;
    if (hipMemset(v, 0, std::max<size_t>(count * sizeof(T), 16)) != hipSuccess) {
        (void)hipFree(v);
        return false;
    }
    S->owned.push_back(v);
    *p = (T *)v;
    return true;
}

// borrowed when given, else owned
template <typename T>
bool use(qb_state S, T **dst, T *given, size_t count)
{
    if (given) {
        *dst = given;
        return true;
    }
    return alloc(S, dst, count);
}

qb_status st_extract(qb_state S, qb_batch b, void *tiles, int32_t *F0, uint8_t *y0, hipStream_t s)
{
    if (S->P->sparse)
        return qb_extract_ell(S->P, b, S->b.X, S->b.H, (uint32_t *)tiles, nullptr, F0, y0, s);
    return qb_extract(S->P, b, S->b.X, S->b.H, tiles, nullptr, F0, y0, s);
}

qb_status st_anneal(qb_state S, qb_batch b, const void *tiles, const int32_t *F0, const uint8_t *y0,
                    int nsw, const int32_t *thr, uint32_t inst_base, const qb_iter *it, uint8_t *Y, int64_t *e,
                    hipStream_t s)
{
    const qb_run_cfg &c = S->cfg;
    if (S->P->sparse)
        return qb_anneal_ell_x(b, S->P->ellw, (const uint32_t *)tiles, F0, y0, nsw, c.B, thr, c.R, c.anneal_rw,
                               c.seed, inst_base, it, Y, e, s);
    return qb_anneal_x(b, tiles, S->P->int8_ok, F0, y0, nsw, c.B, thr, c.R, c.seed, inst_base, it, Y, e, s);
}

// rank-k field update, energy and best after a change dX
qb_status st_field_energy_best(qb_state S, hipStream_t s)
{
    qb_status rc = qb_rankk(S->P, S->z, S->b.dX, S->b.H, S->cfg.rankk_variant, s);
    if (rc == QB_OK) rc = qb_energy(S->n, S->z, S->b.X, S->b.H, S->b.E, s);
    if (rc == QB_OK) rc = qb_best(S->n, S->z, S->b.X, S->b.E, S->b.ebest, S->b.xbest, s);
    return rc;
}

// write-back of the batch's annealing (Y, e against y0), then the update
qb_status st_apply(qb_state S, qb_batch b, const uint8_t *Y, const int64_t *e, const uint8_t *y0, hipStream_t s)
{
    qb_status rc = qb_zero(S->b.dX, (size_t)S->z * S->n, s);
    if (rc == QB_OK)
        rc = qb_writeback(b, S->cfg.R, Y, e, y0, S->b.X, S->b.dX, nullptr,
                          (S->cfg.flags & QB_RUN_WB_NOT_WORSE) ? QB_WB_NOT_WORSE : 0, s);
    if (rc == QB_OK) rc = st_field_energy_best(S, s);
    return rc;
}

#define ST_TRY(expr)                       \
    do {                                   \
        const qb_status _r = (expr);       \
        if (_r != QB_OK) return _r;        \
    } while (0)

// One outer iteration of Alg. 2 (the sequence stated in qb.h).  `timed`:
// record the stage events (eager iterations only).
qb_status st_iteration(qb_state S, hipStream_t s, bool timed)
{
    const qb_run_cfg &c = S->cfg;
    const qb_state_buffers &B = S->b;
    const int n = S->n, z = S->z;
    qb_batch b = S->batch;
    auto mark = [&](int i) -> qb_status {
        if (timed) QB_TRY_HIP(hipEventRecord(S->ev[i], s));
        return QB_OK;
    };
    ST_TRY(mark(0));
    ST_TRY(qb_tabu(S->P, z, B.X, B.H, B.E, c.alpha, c.tenure, c.aspiration, B.T, B.LF, s));
    ST_TRY(qb_best(n, z, B.X, B.E, B.ebest, B.xbest, s));
    ST_TRY(mark(1));
    ST_TRY(qb_keys(S->P, z, B.X, B.T, c.W1, c.W2, c.W3, std::max(c.alpha, 1), B.K, s));
    ST_TRY(qb_rank(n, z, B.K, B.order, s));
    if (S->learned || S->tracing)
        ST_TRY(qb_features(S->P, z, B.X, B.H, B.T, B.LF, B.G, c.alpha, S->scales, B.F, s));
    if (S->learned) {
        ST_TRY(qb_mlp_score((int64_t)z * n, B.F, c.mlp_W_d, nullptr, B.KL, s));
        ST_TRY(qb_rank(n, z, B.KL, B.orderL, s));
        ST_TRY(qb_select(b, B.orderL, s));
    } else if (S->random_select) {
        ST_TRY(qb_random_keys_x(n, z, 0, S->it, c.seed, S->KR, s));
        ST_TRY(qb_rank(n, z, S->KR, S->orderR, s));
        ST_TRY(qb_select(b, S->orderR, s));
    } else {
        ST_TRY(qb_select(b, B.order, s));
    }
    ST_TRY(mark(2));
    if (!S->no_im) {
        ST_TRY(st_extract(S, b, B.tiles, B.F0, B.y0, s));
        ST_TRY(mark(3));
        ST_TRY(st_anneal(S, b, B.tiles, B.F0, B.y0, c.nsw, S->thr, 0, S->it, B.Y, B.e, s));
        ST_TRY(mark(4));
        if (S->learned || S->tracing) ST_TRY(qb_gain_update(b, c.R, B.Y, B.e, B.y0, B.G, s));
        if (S->tracing)
            ST_TRY(qb_trace_x(b, c.R, B.F, B.Y, B.e, B.y0, B.trace_F, B.trace_L, S->it, c.trace_capacity, s));
        ST_TRY(st_apply(S, b, B.Y, B.e, B.y0, s));
    } else {
        ST_TRY(mark(3));
        ST_TRY(mark(4));
    }
    ST_TRY(mark(5));
    ST_TRY(qb_zero(B.dX, (size_t)z * n, s));
    qb_batch mb = S->no_im ? S->empty : b;
    if (S->random_select)
        ST_TRY(qb_mutate_x(mb, S->K0, S->orderR, 0.0, 0, S->it, S->rate_tab, c.max_iters, c.seed, B.X, B.dX,
                           S->kcount, s));
    else
        ST_TRY(qb_mutate_x(mb, B.K, B.order, 0.0, 0, S->it, S->rate_tab, c.max_iters, c.seed, B.X, B.dX,
                           S->kcount, s));
    ST_TRY(st_field_energy_best(S, s));
    k_advance<<<1, 1, 0, s>>>(S->it, S->no_im ? 0u : (uint32_t)b->J, b->total, c.trace_capacity,
                              S->tracing ? 1 : 0, B.ebest, B.ebest_trace, c.max_iters);
    QB_LAUNCH_CHECK();
    ST_TRY(mark(6));
    return QB_OK;
}

}  // namespace

extern "C" void qb_state_destroy(qb_state S)
{
    if (!S) return;
    if (S->graph) (void)hipGraphExecDestroy(S->graph);
    for (hipEvent_t e : S->ev)
        if (e) (void)hipEventDestroy(e);
    if (S->cap) (void)hipStreamDestroy(S->cap);
    qb_batch_destroy(S->batch);
    qb_batch_destroy(S->ib);
    qb_batch_destroy(S->empty);
    for (void *p : S->owned) (void)hipFree(p);
    delete S;
}

extern "C" qb_status qb_state_create(qb_state *out, qb_problem P, const qb_run_cfg *cfg, const qb_state_buffers *bufs,
                                    void *stream)
{
    if (!out || !P || !cfg) return QB_E_ARG;
    *out = nullptr;
    const qb_run_cfg &c = *cfg;
    const int n = P->n;
    if (c.z < 1 || c.k < 1 || !c.job_m_h || !c.thr_h || c.nsw < 1 || c.B < 1 || c.B > 16 || c.R < 1 || c.R > 16)
        return QB_E_ARG;
    if (c.alpha < 0 || c.tenure < 0 || c.max_iters < 1 || c.trace_capacity < 0 || (c.flags & ~31)) return QB_E_ARG;
    if (c.init_m < 0 || c.init_m > 1024 || (c.init_m > 0 && (c.init_m > n || c.nsw_init < 1 || !c.thr_init_h)))
        return QB_E_ARG;
    const bool learned = (c.flags & QB_RUN_LEARNED) != 0;
    if (learned && (!c.mlp_W_d || (c.flags & (QB_RUN_RANDOM_SELECT | QB_RUN_NO_IM | QB_RUN_WB_NOT_WORSE))))
        return QB_E_ARG;
    if ((learned || c.trace_capacity > 0) && !c.scales_h) return QB_E_ARG;
    const int z = c.z, k = c.k;
    const int L0 = c.init_m ? n / c.init_m : 0;
    // every instance number of the run stays below 2^28
    const uint64_t insts = (uint64_t)z * L0 + (uint64_t)z * k * (uint64_t)c.max_iters;
    if (insts > (1ull << 28)) return QB_E_RANGE;

    qb_state S = new qb_state_s();
    S->P = P;
    S->n = n;
    S->z = z;
    S->k = k;
    S->cfg = c;
    S->job_m.assign(c.job_m_h, c.job_m_h + (size_t)z * k);
    S->cfg.job_m_h = nullptr;
    S->cfg.thr_h = nullptr;
    S->cfg.thr_init_h = nullptr;
    S->cfg.scales_h = nullptr;
    if (c.scales_h) std::copy(c.scales_h, c.scales_h + 7, S->scales);
    S->learned = learned;
    S->tracing = c.trace_capacity > 0;
    S->random_select = (c.flags & QB_RUN_RANDOM_SELECT) != 0;
    S->no_im = (c.flags & QB_RUN_NO_IM) != 0;
    S->L0 = L0;
    S->tile_esz = P->int8_ok ? 1 : 2;
    hipStream_t s = qb_stream(stream);
    qb_status rc = QB_OK;
    auto fail = [&](qb_status r) {
        qb_state_destroy(S);
        return r;
    };

    std::vector<int32_t> sol((size_t)z * k);
    for (int p = 0; p < z; ++p)
        for (int q = 0; q < k; ++q) sol[(size_t)p * k + q] = p;
    if ((rc = qb_batch_create(&S->batch, n, z, z * k, sol.data(), S->job_m.data(), nullptr)) != QB_OK) return fail(rc);
    if (S->no_im && (rc = qb_batch_create(&S->empty, n, z, 0, nullptr, nullptr, nullptr)) != QB_OK) return fail(rc);
    if (L0 > 0) {
        const bool jac = (c.flags & QB_RUN_INIT_JACOBI) != 0;
        const int jobs = jac ? z * L0 : z;
        std::vector<int32_t> isol(jobs), isz(jobs, c.init_m);
        for (int q = 0; q < jobs; ++q) isol[q] = jac ? q / L0 : q;
        if ((rc = qb_batch_create(&S->ib, n, z, jobs, isol.data(), isz.data(), nullptr)) != QB_OK) return fail(rc);
    }
    const qb_batch b = S->batch;
    auto tile_bytes = [&](qb_batch bb) -> size_t {
        if (P->sparse) return sizeof(uint32_t) * ((size_t)bb->total * P->ellw + (size_t)bb->dblk_words);
        return (size_t)bb->tile_elems * S->tile_esz;
    };
    const size_t zn = (size_t)z * n;
    qb_state_buffers g{};
    if (bufs) g = *bufs;
    qb_state_buffers &B = S->b;
    bool ok = use(S, &B.X, g.X, zn) && use(S, &B.H, g.H, zn) && use(S, &B.E, g.E, (size_t)z) &&
              use(S, &B.xbest, g.xbest, (size_t)n) && use(S, &B.ebest, g.ebest, 1) &&
              use(S, &B.ebest_trace, g.ebest_trace, (size_t)c.max_iters) && use(S, &B.T, g.T, zn) &&
              use(S, &B.LF, g.LF, zn) && use(S, &B.G, g.G, zn) && use(S, &B.K, g.K, zn) &&
              use(S, &B.order, g.order, zn) && use(S, &B.dX, g.dX, zn) &&
              use(S, (uint8_t **)&B.tiles, (uint8_t *)g.tiles, tile_bytes(b)) && use(S, &B.F0, g.F0, (size_t)b->total) &&
              use(S, &B.y0, g.y0, (size_t)b->total) && use(S, &B.Y, g.Y, (size_t)b->total * c.R) &&
              use(S, &B.e, g.e, (size_t)b->J * c.R) && alloc(S, &S->kcount, (size_t)z) && alloc(S, &S->it, 1) &&
              alloc(S, &S->rate_tab, (size_t)c.max_iters) && alloc(S, &S->thr, (size_t)c.nsw << c.B);
    if (ok && (learned || S->tracing)) ok = use(S, &B.F, g.F, zn * 8);
    if (ok && learned) ok = use(S, &B.KL, g.KL, zn) && use(S, &B.orderL, g.orderL, zn);
    if (ok && S->tracing)
        ok = use(S, &B.trace_F, g.trace_F, (size_t)c.trace_capacity * 8) &&
             use(S, &B.trace_L, g.trace_L, (size_t)c.trace_capacity);
    if (ok && S->random_select)
        ok = alloc(S, &S->KR, zn) && alloc(S, &S->K0, zn) && alloc(S, &S->orderR, zn);
    if (ok && L0 > 0) {
        const qb_batch ib = S->ib;
        ok = alloc(S, (uint8_t **)&S->itiles, tile_bytes(ib)) && alloc(S, &S->iF0, (size_t)ib->total) &&
             alloc(S, &S->iy0, (size_t)ib->total) && alloc(S, &S->iY, (size_t)ib->total * c.R) &&
             alloc(S, &S->ie, (size_t)ib->J * c.R) && alloc(S, &S->thr_init, (size_t)c.nsw_init << c.B);
    }
    if (!ok) return fail(QB_E_HIP);
    if (((uintptr_t)B.tiles & 15) || (B.F && ((uintptr_t)B.F & 15))) return fail(QB_E_ARG);
    std::vector<double> rates(c.max_iters);
    for (int t = 0; t < c.max_iters; ++t) rates[t] = qb_mutation_rate(t);
    if (hipMemcpyAsync(S->rate_tab, rates.data(), sizeof(double) * c.max_iters, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(S->thr, c.thr_h, sizeof(int32_t) * ((size_t)c.nsw << c.B), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        (L0 > 0 && hipMemcpyAsync(S->thr_init, c.thr_init_h, sizeof(int32_t) * ((size_t)c.nsw_init << c.B),
                                  hipMemcpyHostToDevice, s) != hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(QB_E_HIP);
    if (hipStreamCreateWithFlags(&S->cap, hipStreamNonBlocking) != hipSuccess) return fail(QB_E_HIP);
    *out = S;
    return QB_OK;
}

extern "C" qb_status qb_state_get_buffers(qb_state S, qb_state_buffers *out)
{
    if (!S || !out) return QB_E_ARG;
    *out = S->b;
    return QB_OK;
}

extern "C" qb_batch qb_state_batch(qb_state S) { return S ? S->batch : nullptr; }

extern "C" qb_status qb_state_init(qb_state S, void *stream)
{
    if (!S) return QB_E_ARG;
    hipStream_t s = qb_stream(stream);
    const qb_run_cfg &c = S->cfg;
    const qb_state_buffers &B = S->b;
    const int n = S->n, z = S->z;
    ST_TRY(qb_init_solutions(n, z, c.seed, B.X, s));
    ST_TRY(qb_field(S->P, z, B.X, B.H, s));
    ST_TRY(qb_energy(n, z, B.X, B.H, B.E, s));
    k_fill_i64<<<1, 1, 0, s>>>(B.ebest, INT64_MAX);
    QB_LAUNCH_CHECK();
    ST_TRY(qb_best(n, z, B.X, B.E, B.ebest, B.xbest, s));
    uint32_t inst = 0;
    if (S->L0 > 0) {
        const qb_batch ib = S->ib;
        const int m0 = c.init_m;
        const bool jac = (c.flags & QB_RUN_INIT_JACOBI) != 0;
        const int rounds = jac ? 1 : S->L0;
        for (int l = 0; l < rounds; ++l) {
            k_block_idx<<<ib->J, 256, 0, s>>>(ib->idx_d, ib->J, jac ? S->L0 : 1, m0, jac ? 0 : l);
            QB_LAUNCH_CHECK();
            ST_TRY(st_extract(S, ib, S->itiles, S->iF0, S->iy0, s));
            ST_TRY(st_anneal(S, ib, S->itiles, S->iF0, S->iy0, c.nsw_init, S->thr_init, inst, nullptr, S->iY, S->ie,
                             s));
            inst += (uint32_t)ib->J;
            ST_TRY(st_apply(S, ib, S->iY, S->ie, S->iy0, s));
        }
    }
    S->inst0 = inst;
    k_set_iter<<<1, 1, 0, s>>>(S->it, 0, inst, 0);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

extern "C" qb_status qb_iterate(qb_state S, int32_t iters, int32_t graph, int32_t patience, int32_t *ran,
                               void *stream)
{
    if (!S || iters < 0 || patience < 0) return QB_E_ARG;
    if (ran) *ran = 0;
    hipStream_t s = qb_stream(stream);
    if (graph && !S->graph && iters > 0) {
        // one iteration on the state's own stream, captured once
        QB_TRY_HIP(hipStreamBeginCapture(S->cap, hipStreamCaptureModeRelaxed));
        const qb_status rc = st_iteration(S, S->cap, false);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(S->cap, &g);
        if (rc != QB_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) {
            qb_set_hip_error(e);
            return QB_E_HIP;
        }
        const hipError_t e2 = hipGraphInstantiate(&S->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) {
            S->graph = nullptr;
            qb_set_hip_error(e2);
            return QB_E_HIP;
        }
    }
    int64_t best = 0;
    int stall = 0;
    if (patience > 0) {
        QB_TRY_HIP(hipMemcpyAsync(&best, S->b.ebest, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        QB_TRY_HIP(hipStreamSynchronize(s));
    }
    for (int i = 0; i < iters; ++i) {
        if (graph)
            QB_TRY_HIP(hipGraphLaunch(S->graph, s));
        else
            ST_TRY(st_iteration(S, s, S->timing));
        if (ran) *ran = i + 1;
        if (patience > 0) {
            int64_t eb = 0;
            QB_TRY_HIP(hipMemcpyAsync(&eb, S->b.ebest, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            QB_TRY_HIP(hipStreamSynchronize(s));
            stall = eb < best ? 0 : stall + 1;
            best = eb;
            if (stall >= patience) break;
        }
    }
    return QB_OK;
}

extern "C" qb_status qb_state_get_iteration(qb_state S, int32_t *t_h, uint32_t *inst_h, int64_t *trace_rows_h,
                                           void *stream)
{
    if (!S) return QB_E_ARG;
    hipStream_t s = qb_stream(stream);
    qb_iter h{};
    QB_TRY_HIP(hipMemcpyAsync(&h, S->it, sizeof(qb_iter), hipMemcpyDeviceToHost, s));
    QB_TRY_HIP(hipStreamSynchronize(s));
    if (t_h) *t_h = h.t;
    if (inst_h) *inst_h = h.inst;
    if (trace_rows_h) *trace_rows_h = h.trn;
    return QB_OK;
}

extern "C" qb_status qb_state_set_iteration(qb_state S, int32_t t, void *stream)
{
    if (!S || t < 0 || t >= S->cfg.max_iters) return QB_E_ARG;
    const uint32_t per = S->no_im ? 0u : (uint32_t)S->batch->J;
    k_set_iter<<<1, 1, 0, qb_stream(stream)>>>(S->it, t, S->inst0 + per * (uint32_t)t, 1);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

extern "C" qb_status qb_apply(qb_state S, void *stream)
{
    if (!S) return QB_E_ARG;
    return st_apply(S, S->batch, S->b.Y, S->b.e, S->b.y0, qb_stream(stream));
}

extern "C" qb_status qb_state_set_variants(qb_state S, int32_t rankk_variant, int32_t anneal_rw)
{
    if (!S || rankk_variant < 0 || rankk_variant > 3 || anneal_rw < 0 || anneal_rw > 16) return QB_E_ARG;
    S->cfg.rankk_variant = rankk_variant;
    S->cfg.anneal_rw = anneal_rw;
    if (S->graph) {
        // the captured iteration holds the old launches
        (void)hipGraphExecDestroy(S->graph);
        S->graph = nullptr;
    }
    return QB_OK;
}

extern "C" qb_status qb_state_enable_timing(qb_state S, int32_t on)
{
    if (!S) return QB_E_ARG;
    if (on && !S->ev[0])
        for (hipEvent_t &e : S->ev) QB_TRY_HIP(hipEventCreate(&e));
    S->timing = on != 0;
    return QB_OK;
}

extern "C" qb_status qb_state_stage_ms(qb_state S, float *ms_h, void *stream)
{
    if (!S || !ms_h || !S->ev[0]) return QB_E_ARG;
    QB_TRY_HIP(hipStreamSynchronize(qb_stream(stream)));
    for (int i = 0; i < QB_NSTAGE; ++i) QB_TRY_HIP(hipEventElapsedTime(&ms_h[i], S->ev[i], S->ev[i + 1]));
    return QB_OK;
}

extern "C" qb_status qb_state_check(qb_state S, void *stream)
{
    if (!S) return QB_E_ARG;
    qb_status r = qb_check(S->P, stream);
    const qb_status r1 = qb_batch_check(S->batch, stream);
    const qb_status r2 = S->ib ? qb_batch_check(S->ib, stream) : QB_OK;
    if (r == QB_OK) r = r1;
    if (r == QB_OK) r = r2;
    return r;
}
