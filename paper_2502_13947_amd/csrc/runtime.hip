// Orchestration helpers: HIP-graph capture of the outer loop of Alg. 2 and
// the autotuner of result-invariant kernel variants.
#include <mutex>
#include <vector>

#include "qb_internal.h"

hipError_t qb_cu_count(int *out)
{
    static std::mutex mu;
    static int cached[64] = {0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if (dev >= 0 && dev < 64 && cached[dev]) {
        *out = cached[dev];
        return hipSuccess;
    }
    int v = 0;
    e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < 64) cached[dev] = v;
    *out = v;
    return hipSuccess;
}

extern "C" qb_status qb_graph_begin(void *stream)
{
    hipStream_t s = qb_stream(stream);
    if (!s) return QB_E_ARG;   // the legacy default stream cannot be captured
    QB_TRY_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    return QB_OK;
}

extern "C" qb_status qb_graph_end(void *stream, void **graph_exec_out)
{
    if (!graph_exec_out) return QB_E_ARG;
    *graph_exec_out = nullptr;
    hipGraph_t g = nullptr;
    QB_TRY_HIP(hipStreamEndCapture(qb_stream(stream), &g));
    hipGraphExec_t ge = nullptr;
    hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        qb_set_hip_error(e);
        return QB_E_HIP;
    }
    *graph_exec_out = ge;
    return QB_OK;
}

extern "C" qb_status qb_graph_launch(void *graph_exec, void *stream)
{
    if (!graph_exec) return QB_E_ARG;
    QB_TRY_HIP(hipGraphLaunch((hipGraphExec_t)graph_exec, qb_stream(stream)));
    return QB_OK;
}

extern "C" void qb_graph_destroy(void *graph_exec)
{
    if (graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)graph_exec);
}

// ------------------------------------------------------------------ autotuner
// Times every applicable rank-k variant on the caller's (dX, H) and returns
// the fastest.  All variants must produce identical fields (checked on the
// host); a mismatch is reported as QB_E_STATE.  H_d is left unchanged.  Not a
// hot call: it allocates scratch and synchronises.
extern "C" qb_status qb_autotune_rankk(qb_problem P, int32_t z, const int8_t *dX_d, const int32_t *H_d,
                                      int32_t reps, int32_t *variant_out, float *ms_out, void *stream)
{
    if (!P || z < 1 || !dX_d || !H_d || !variant_out || reps < 1) return QB_E_ARG;
    hipStream_t s = qb_stream(stream);
    const size_t bytes = sizeof(int32_t) * (size_t)z * P->n;
    int32_t *Hw = nullptr;
    QB_TRY_HIP(hipMalloc(&Hw, bytes));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipFree(Hw);
        return QB_E_HIP;
    }
    std::vector<int32_t> ref, cur;
    int best = 1;
    float best_ms = 1e30f;
    qb_status rc = QB_OK;
    const int cand[3] = {1, 2, 3};
    if (P->sparse) best = 3;
    for (int vi = 0; vi < 3 && rc == QB_OK; ++vi) {
        const int v = cand[vi];
        if (P->sparse != (v == 3)) continue;
        if (v == 2 && (!P->int8_ok || !P->Qp)) continue;
        float tot = 0.f;
        for (int r = 0; r < reps + 1 && rc == QB_OK; ++r) {
            if (hipMemcpyAsync(Hw, H_d, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) { rc = QB_E_HIP; break; }
            if (hipEventRecord(e0, s) != hipSuccess) { rc = QB_E_HIP; break; }
            rc = qb_rankk(P, z, dX_d, Hw, v, stream);
            if (rc != QB_OK) break;
            float ms = 0.f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = QB_E_HIP;
                break;
            }
            if (r > 0) tot += ms;   // first run is a warm-up
        }
        if (rc != QB_OK) break;
        cur.resize((size_t)z * P->n);
        if (hipMemcpy(cur.data(), Hw, bytes, hipMemcpyDeviceToHost) != hipSuccess) { rc = QB_E_HIP; break; }
        if (ref.empty())
            ref = cur;
        else if (ref != cur)
            rc = QB_E_STATE;
        const float avg = tot / reps;
        if (avg < best_ms) { best_ms = avg; best = v; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(Hw);
    if (rc != QB_OK) return rc;
    *variant_out = best;
    if (ms_out) *ms_out = best_ms;
    return QB_OK;
}

// Times qb_anneal_ell for every replicas-per-workgroup choice that fits and
// returns the fastest; every choice must give the same (Y, e) (checked on the
// host, QB_E_STATE otherwise).  Not a hot call: allocates scratch, syncs.
extern "C" qb_status qb_autotune_anneal_ell(qb_batch b, int32_t W, const uint32_t *tile_d, const int32_t *F0_d,
                                           const uint8_t *y0_d, int32_t nsw, int32_t B, const int32_t *thr_d,
                                           int32_t R, uint64_t seed, uint32_t inst_base, int32_t reps,
                                           int32_t *rw_out, float *ms_out, void *stream)
{
    if (!b || !rw_out || reps < 1 || R < 1 || R > 16) return QB_E_ARG;
    hipStream_t s = qb_stream(stream);
    const size_t ybytes = (size_t)b->total * R, ebytes = sizeof(int64_t) * (size_t)b->J * R;
    uint8_t *Yw = nullptr;
    int64_t *ew = nullptr;
    if (hipMalloc(&Yw, ybytes ? ybytes : 1) != hipSuccess || hipMalloc(&ew, ebytes ? ebytes : 8) != hipSuccess) {
        if (Yw) (void)hipFree(Yw);
        return QB_E_HIP;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipFree(Yw);
        (void)hipFree(ew);
        return QB_E_HIP;
    }
    std::vector<uint8_t> Yref, Ycur;
    std::vector<int64_t> eref, ecur;
    int best = 0;
    float best_ms = 1e30f;
    qb_status rc = QB_OK;
    for (int rw = 1; rw <= 16 && rc == QB_OK; rw <<= 1) {
        if (rw > R && rw > 1) break;
        float tot = 0.f;
        qb_status r0 = QB_OK;
        for (int r = 0; r < reps + 1; ++r) {
            if (hipEventRecord(e0, s) != hipSuccess) { r0 = QB_E_HIP; break; }
            r0 = qb_anneal_ell(b, W, tile_d, F0_d, y0_d, nsw, B, thr_d, R, rw, seed, inst_base, Yw, ew, stream);
            if (r0 != QB_OK) break;
            float ms = 0.f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                r0 = QB_E_HIP;
                break;
            }
            if (r > 0) tot += ms;
        }
        if (r0 == QB_E_CAPACITY) break;   // larger rw do not fit either
        if (r0 != QB_OK) { rc = r0; break; }
        Ycur.resize(ybytes);
        ecur.resize((size_t)b->J * R);
        if (hipMemcpy(Ycur.data(), Yw, ybytes, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(ecur.data(), ew, ebytes, hipMemcpyDeviceToHost) != hipSuccess) {
            rc = QB_E_HIP;
            break;
        }
        if (Yref.empty() && eref.empty()) {
            Yref = Ycur;
            eref = ecur;
        } else if (Yref != Ycur || eref != ecur) {
            rc = QB_E_STATE;
        }
        const float avg = tot / reps;
        if (avg < best_ms) {
            best_ms = avg;
            best = rw;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(Yw);
    (void)hipFree(ew);
    if (rc != QB_OK) return rc;
    if (best == 0) return QB_E_CAPACITY;
    *rw_out = best;
    if (ms_out) *ms_out = best_ms;
    return QB_OK;
}

// Plan autotuner of the dense annealer (qb_anneal): coordinate descent over
// the result-invariant knobs of qb_anneal_plan on the caller's batch -- the
// kernel of each size class present (largest class first), then the
// persistent queue with its grid and its order, then the consumers' loads in
// flight -- timing `reps` launches of each candidate after one warm-up
// launch and keeping a change only when it is faster.  Every candidate's Y
// and e are compared with the first plan's (QB_E_STATE on any difference).
// The best plan is left set on the batch.  Not a hot call: it allocates
// scratch and synchronises.
namespace {

struct PlanTimer {
    qb_batch b;
    const void *tile;
    int int8_tile;
    const int32_t *F0;
    const uint8_t *y0;
    int nsw, B;
    const int32_t *thr;
    int R;
    uint64_t seed;
    uint32_t inst;
    int reps;
    hipStream_t s;
    uint8_t *Yw = nullptr;
    int64_t *ew = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<uint8_t> Yref, Ycur;
    std::vector<int64_t> eref, ecur;

    qb_status time(const qb_anneal_plan &p, float *ms_out)
    {
        b->plan = p;
        float tot = 0.f;
        for (int r = 0; r < reps + 1; ++r) {
            QB_TRY_HIP(hipEventRecord(e0, s));
            const qb_status rc = qb_anneal(b, tile, int8_tile, F0, y0, nsw, B, thr, R, seed, inst, Yw, ew, s);
            if (rc != QB_OK) return rc;
            float ms = 0.f;
            QB_TRY_HIP(hipEventRecord(e1, s));
            QB_TRY_HIP(hipEventSynchronize(e1));
            QB_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (r > 0) tot += ms;
        }
        const size_t ybytes = (size_t)b->total * R;
        Ycur.resize(ybytes);
        ecur.resize((size_t)b->J * R);
        QB_TRY_HIP(hipMemcpy(Ycur.data(), Yw, ybytes, hipMemcpyDeviceToHost));
        QB_TRY_HIP(hipMemcpy(ecur.data(), ew, sizeof(int64_t) * ecur.size(), hipMemcpyDeviceToHost));
        if (Yref.empty() && eref.empty()) {
            Yref = Ycur;
            eref = ecur;
        } else if (Yref != Ycur || eref != ecur) {
            return QB_E_STATE;
        }
        *ms_out = tot / reps;
        return QB_OK;
    }
};

}  // namespace

extern "C" qb_status qb_autotune_anneal(qb_batch b, const void *tile_d, int32_t int8_tile, const int32_t *F0_d,
                                       const uint8_t *y0_d, int32_t nsw, int32_t B, const int32_t *thr_d, int32_t R,
                                       uint64_t seed, uint32_t inst_base, int32_t reps, qb_anneal_plan *plan_out,
                                       float *ms_out, void *stream)
{
    if (!b || !tile_d || !F0_d || !y0_d || !thr_d || reps < 1 || R < 1 || R > 16) return QB_E_ARG;
    if (b->J == 0) {
        if (plan_out) *plan_out = b->plan;
        if (ms_out) *ms_out = 0.f;
        return QB_OK;
    }
    PlanTimer T{b, tile_d, int8_tile, F0_d, y0_d, nsw, B, thr_d, R, seed, inst_base, reps, qb_stream(stream)};
    const size_t ybytes = (size_t)b->total * R, ebytes = sizeof(int64_t) * (size_t)b->J * R;
    qb_status rc = QB_OK;
    if (hipMalloc(&T.Yw, ybytes ? ybytes : 1) != hipSuccess || hipMalloc(&T.ew, ebytes ? ebytes : 8) != hipSuccess ||
        hipEventCreate(&T.e0) != hipSuccess || hipEventCreate(&T.e1) != hipSuccess)
        rc = QB_E_HIP;
    const qb_anneal_plan start = b->plan;
    qb_anneal_plan best = start;
    float best_ms = 0.f;
    if (rc == QB_OK) rc = T.time(best, &best_ms);
    auto trial = [&](const qb_anneal_plan &p) {
        if (rc != QB_OK) return;
        float ms = 0.f;
        rc = T.time(p, &ms);
        if (rc == QB_OK && ms < best_ms) {
            best_ms = ms;
            best = p;
        }
    };
    // the kernel of each class present, largest class first
    for (int c = 0; c < QB_NCLASS && rc == QB_OK; ++c) {
        if (b->cls_end[c] <= b->cls_begin[c]) continue;
        const qb_anneal_plan base = best;
        for (int k : {QB_ANNEAL_MULTI_WAVE_GLOBAL, QB_ANNEAL_ONE_WAVE, QB_ANNEAL_ONE_WAVE_REG, QB_ANNEAL_AUTO}) {
            if (k == base.kernel[c]) continue;
            qb_anneal_plan p = base;
            p.kernel[c] = k;
            trial(p);
        }
    }
    // persistent queue: grid and order
    {
        const qb_anneal_plan base = best;
        for (int w : {1, 2, 4}) {
            qb_anneal_plan p = base;
            p.persistent = 1;
            p.wgs_per_cu = w;
            if (p.persistent != base.persistent || p.wgs_per_cu != base.wgs_per_cu) trial(p);
        }
        if (base.persistent) {
            qb_anneal_plan p = base;
            p.persistent = 0;
            trial(p);
        }
    }
    {
        qb_anneal_plan p = best;
        p.lpt = 1 - p.lpt;
        trial(p);
    }
    {
        qb_anneal_plan p = best;
        p.depth = p.depth == 8 ? 16 : 8;
        trial(p);
    }
    b->plan = rc == QB_OK ? best : start;
    if (T.e0) (void)hipEventDestroy(T.e0);
    if (T.e1) (void)hipEventDestroy(T.e1);
    if (T.Yw) (void)hipFree(T.Yw);
    if (T.ew) (void)hipFree(T.ew);
    if (rc != QB_OK) return rc;
    if (plan_out) *plan_out = best;
    if (ms_out) *ms_out = best_ms;
    return QB_OK;
}
