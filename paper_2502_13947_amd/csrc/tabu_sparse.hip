// Tabu search (Alg. 1 of the IC-D^2S paper) on a sparse problem: one
// 1024-thread workgroup (sixteen waves, four per SIMD) per solution.
//
// The step is the dense kernel's: thread t owns the variables j = e*1024 + t
// (e < EPT) and keeps in registers the biased move value D_j and the step
// U_j after which j is free again; every lane keys its allowed variables (move << EB | element), the
// wave minimum comes from DPP, the sixteen wave winners meet in LDS with one
// barrier per step.  What changes is the field update: flipping i moves
// D_j only for the neighbours j of i (the O(n) update of the Tabu section,
// here O(degree)).  The neighbour list is read once by the whole workgroup
// (uniform address, scalar loads); each entry's owner patches its own
// element through a scalar switch on the (uniform) element index.  The
// factor 2(1-2x_j) is taken from the x bits when an element is touched, so
// no per-element copy of it is kept.  The flip count and last-flip step go
// straight to the output arrays (a vector atomic add and a store by the
// owner, neither waited for), which keeps the registers for D and U.
#include "qb_internal.h"

namespace {

constexpr int TB = QB_TABU_SP_THREADS;
constexpr int NW = TB / 64;
constexpr int TMASK = TB - 1;
constexpr int TSHIFT = 10;
static_assert(TB == 1 << TSHIFT, "thread count must be 2^TSHIFT");

#define QB_SWITCH20(CASE)                                                                              \
    CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) \
    CASE(12) CASE(13) CASE(14) CASE(15) CASE(16) CASE(17) CASE(18) CASE(19)

// Calls f on every word of row i's ELL entries (zero words included up to
// the next multiple of four), 16-byte loads one chunk ahead of their use.
template <typename Fn>
__device__ __forceinline__ void for_row(const uint32_t *__restrict__ ell, int W, const int32_t *__restrict__ ecnt,
                                        int i, Fn &f)
{
    const uint4 *row = reinterpret_cast<const uint4 *>(ell + (int64_t)i * W);
    const int c4 = (ecnt[i] + 3) >> 2;
    uint4 cur = c4 > 0 ? row[0] : make_uint4(0, 0, 0, 0);
    for (int t = 0; t < c4; ++t) {
        const uint4 nxt = t + 1 < c4 ? row[t + 1] : make_uint4(0, 0, 0, 0);
        f(cur.x);
        f(cur.y);
        f(cur.z);
        f(cur.w);
        cur = nxt;
    }
}

template <int EPT>
__global__ void __launch_bounds__(TB) k_tabu_sp(const uint32_t *__restrict__ ell, int W,
                                                const int32_t *__restrict__ ecnt,
                                                const int32_t *__restrict__ diag, int n,
                                                uint8_t *__restrict__ X, int32_t *__restrict__ H,
                                                int64_t *__restrict__ E, int alpha, int tenure, int asp,
                                                int32_t *__restrict__ Tout, int32_t *__restrict__ LFout,
                                                uint32_t bias)
{
    static_assert(EPT <= 20, "switch covers 20 elements");
    constexpr int EB = qb_ceil_log2(EPT);
    constexpr uint32_t EMASK = (1u << EB) - 1u;
    __shared__ uint64_t red[2][NW];
    __shared__ uint64_t red2[NW];
    __shared__ int32_t list[TB];
    __shared__ int lcount;

    const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t ro = (int64_t)p * n;
    const uint32_t dpad = 0xFFFFFFFFu >> EB;

    uint32_t Db[EPT];   // D + bias
    int32_t U[EPT];     // tabu through step U
    uint64_t xb = 0;    // x bits of the owned variables
    uint64_t pb = 0;    // flipped since the last improvement
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int j = e * TB + tid;
        U[e] = 0;
        if (j < n) {
            Tout[ro + j] = 0;
            LFout[ro + j] = 0;
            const int32_t x = X[ro + j] & 1;
            xb |= (uint64_t)x << e;
            Db[e] = (uint32_t)(diag[j] + (x ? -2 : 2) * H[ro + j]) + bias;
        } else {
            Db[e] = dpad;
            U[e] = 0x7fffffff;
        }
    }
    int64_t OV = E[p], OVmin = OV;

    for (int step = 1; step <= alpha; ++step) {
        const int64_t tau = OVmin - OV + (int64_t)bias;
        const uint32_t tb = tau <= 0 ? 0u : (uint32_t)tau;
        const int32_t free_at = step - 1;
        uint32_t best = 0xFFFFFFFFu;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const bool allowed = U[e] <= free_at || (asp && Db[e] < tb);
            const uint32_t key = (Db[e] << EB) | (uint32_t)e;
            best = min(best, allowed ? key : 0xFFFFFFFFu);
        }
        const uint32_t wmin = qb_wave_min_u32(best);
        uint64_t wkey = ~0ull;
        if (wmin != 0xFFFFFFFFu) {
            const uint64_t who = __ballot(best == wmin);
            const int L = __builtin_ctzll(who);
            const int ew = (int)(wmin & EMASK);
            const uint32_t xw = (uint32_t)__builtin_amdgcn_readlane((int)((xb >> ew) & 1ull), L);
            wkey = qb_tabu_winner(wmin >> EB, ew * TB + wid * 64 + L, xw);
        }
        if (lane == 0) red[step & 1][wid] = wkey;
        __syncthreads();
        uint64_t kb = red[step & 1][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) kb = min(kb, red[step & 1][w]);
        if (kb == ~0ull) {
            uint32_t b2 = 0xFFFFFFFFu;
#pragma unroll
            for (int e = 0; e < EPT; ++e) b2 = min(b2, (Db[e] << EB) | (uint32_t)e);
            const uint32_t w2 = qb_wave_min_u32(b2);
            const uint64_t who = __ballot(b2 == w2);
            const int L = __builtin_ctzll(who);
            const int ew = (int)(w2 & EMASK);
            const uint32_t xw = (uint32_t)__builtin_amdgcn_readlane((int)((xb >> ew) & 1ull), L);
            if (lane == 0) red2[wid] = qb_tabu_winner(w2 >> EB, ew * TB + wid * 64 + L, xw);
            __syncthreads();
            kb = red2[0];
#pragma unroll
            for (int w = 1; w < NW; ++w) kb = min(kb, red2[w]);
        }
        const uint32_t dib = (uint32_t)(kb >> 32);
        const int i = __builtin_amdgcn_readfirstlane((int)((uint32_t)kb >> 1));
        const int32_t s = (kb & 1) ? -1 : 1;   // direction of x_i
        OV += (int64_t)(int32_t)(dib - bias);

        // neighbours j of i: h_j += s Q_ji, so D_j += 2(1-2x_j) s Q_ji
        auto nb = [&](uint32_t wd) {
            const int c = qb_ell_col(wd);
            if (wd != 0u && tid == (c & TMASK)) {
                const int32_t dv = s * qb_ell_val(wd);
                switch (c >> TSHIFT) {
#define QB_NB_CASE(K)                                                                        \
    case K:                                                                                  \
        if constexpr (K < EPT) Db[K] += (uint32_t)(((xb >> K) & 1ull) ? -2 * dv : 2 * dv); \
        break;
                    QB_SWITCH20(QB_NB_CASE)
#undef QB_NB_CASE
                default: break;
                }
            }
        };
        for_row(ell, W, ecnt, i, nb);
        if (tid == (i & TMASK)) {
            // the zeroing stores above precede the first step's barrier
            __hip_atomic_fetch_add(Tout + ro + i, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            LFout[ro + i] = step;
            xb ^= 1ull << (i >> TSHIFT);
            pb ^= 1ull << (i >> TSHIFT);
            switch (i >> TSHIFT) {
#define QB_OWNER_CASE(K)                                                         \
    case K:                                                                      \
        if constexpr (K < EPT) {                                                 \
            Db[K] = 2u * bias - dib;                                             \
            U[K] = step + max(max(U[K] - (step - 1), 0) + tenure - 1, 0);        \
        }                                                                        \
        break;
                QB_SWITCH20(QB_OWNER_CASE)
#undef QB_OWNER_CASE
            default: break;
            }
        }
        if (OV < OVmin) {
            OVmin = OV;
            pb = 0;
        }
    }

    // field of the final x from D, then moved to x_min = x ^ pb by the
    // neighbour lists of the differing variables
    int32_t h[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int j = e * TB + tid;
        h[e] = 0;
        if (j < n) {
            const int32_t sg = ((xb >> e) & 1ull) ? -2 : 2;
            h[e] = ((int32_t)(Db[e] - bias) - diag[j]) * sg / 4;
        }
    }
    for (int e = 0; e < EPT; ++e) {
        if (tid == 0) lcount = 0;
        __syncthreads();
        if (e * TB + tid < n && ((pb >> e) & 1ull)) {
            const int pos = atomicAdd(&lcount, 1);
            const int jj = e * TB + tid;
            list[pos] = ((xb >> e) & 1ull) ? -(jj + 1) : (jj + 1);
        }
        __syncthreads();
        const int cnt = lcount;
        for (int u = 0; u < cnt; ++u) {
            const int32_t v = list[u];
            const int32_t sg = v < 0 ? -1 : 1;
            const int jv = __builtin_amdgcn_readfirstlane(v < 0 ? -v - 1 : v - 1);
            // the diagonal term of x_jv itself
            if (tid == (jv & TMASK)) {
                switch (jv >> TSHIFT) {
#define QB_DIAG_CASE(K)                                                      \
    case K:                                                                  \
        if constexpr (K < EPT) h[K] += sg * diag[jv];                        \
        break;
                    QB_SWITCH20(QB_DIAG_CASE)
#undef QB_DIAG_CASE
                default: break;
                }
            }
            auto hup = [&](uint32_t wd) {
                const int c = qb_ell_col(wd);
                if (wd != 0u && tid == (c & TMASK)) {
                    const int32_t dv = sg * qb_ell_val(wd);
                    switch (c >> TSHIFT) {
#define QB_H_CASE(K)                                                         \
    case K:                                                                  \
        if constexpr (K < EPT) h[K] += dv;                                   \
        break;
                        QB_SWITCH20(QB_H_CASE)
#undef QB_H_CASE
                    default: break;
                    }
                }
            };
            for_row(ell, W, ecnt, jv, hup);
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int j = e * TB + tid;
        if (j < n) {
            X[ro + j] = (uint8_t)(((xb ^ pb) >> e) & 1ull);
            H[ro + j] = h[e];
        }
    }
    if (tid == 0) E[p] = OVmin;
}

#undef QB_SWITCH20

}  // namespace

qb_status qb_tabu_sparse_launch(qb_problem P, int z, uint8_t *X, int32_t *H, int64_t *E, int alpha, int tenure,
                                int asp, int32_t *T, int32_t *LF, hipStream_t s)
{
    const int ept = qb_tabu_sp_ept(P->n);
    if (ept == 0) return QB_E_CAPACITY;
    const int64_t dmax = (int64_t)P->qmax + 2 * P->eta_max;
    const uint32_t bias = (uint32_t)dmax;
#define QB_T(K)                                                                                     \
    if (ept == K) {                                                                                \
        if (2 * dmax + 1 >= (int64_t)(0xFFFFFFFFu >> qb_ceil_log2(K))) return QB_E_RANGE;          \
        k_tabu_sp<K><<<z, TB, 0, s>>>(P->ell, P->ellw, P->ecnt, P->diag, P->n, X, H, E, alpha, tenure, asp, T, \
                                      LF, bias);                                                   \
        QB_LAUNCH_CHECK();                                                                         \
        return QB_OK;                                                                              \
    }
    QB_T(1) QB_T(2) QB_T(3) QB_T(4) QB_T(5) QB_T(6) QB_T(7) QB_T(8) QB_T(10) QB_T(12) QB_T(14) QB_T(16)
    QB_T(20)
#undef QB_T
    return QB_E_CAPACITY;
}
