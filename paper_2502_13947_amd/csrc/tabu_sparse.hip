// Tabu search (Alg. 1 of the IC-D^2S paper) on a sparse problem: one
// 1024-thread workgroup (sixteen waves, four per SIMD) per solution.
//
// Thread t owns the variables j = e*1024 + t (e < EPT) and keeps in
// registers, per variable, the key ((D_j + bias) << EB | element), with bit
// 31 set while j is tabu, and the step U_j after which j is free again, as
// the dense kernel does: each step takes the unsigned minimum of the keys
// (the smallest free key) and the signed one (the smallest tabu key, which
// aspirates whenever any does), the wave minimum comes from DPP, and the
// wave winners meet in LDS with one barrier per step, where a DPP minimum
// over lanes picks the smallest (32-bit (key, wave) when the move values
// allow, else 64-bit (move, index, x)).  What changes from the dense kernel
// is the field update: flipping i moves D_j only for the neighbours j of i
// (the O(n) update of the Tabu section, here O(degree)), each a shift-add
// into the key.
//
// Before the barrier every wave copies the neighbour row of its own
// candidate from the ELL into LDS, so the winner's row is on chip when the
// step resolves and no memory round trip follows the barrier; each wave then
// applies only the entries whose variable it owns (a ballot), the owning
// lane through a scalar switch on the element index.  The factor 2(1-2x_j)
// is taken from the x bits when an element is touched.  The flip count and
// last-flip step go straight to the output arrays (a vector atomic add and a
// store by the owner, neither waited for), which keeps the registers for the
// keys and U.
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

// Calls f on the W words of row i of the ELL (zero words included), reading
// 16 words at a time with the next chunk in flight; the allocation has 16
// spare words after the last row, and words past W are not passed to f.
template <typename Fn>
__device__ __forceinline__ void for_row(const uint32_t *__restrict__ ell, int W, int i, Fn &f)
{
    const uint4 *row = reinterpret_cast<const uint4 *>(ell + (int64_t)i * W);
    uint4 c0 = row[0], c1 = row[1], c2 = row[2], c3 = row[3];
    for (int t0 = 0; t0 < W; t0 += 16) {
        uint4 n0 = make_uint4(0, 0, 0, 0), n1 = n0, n2 = n0, n3 = n0;
        if (t0 + 16 < W) {
            const uint4 *nx = row + ((t0 + 16) >> 2);
            n0 = nx[0];
            n1 = nx[1];
            n2 = nx[2];
            n3 = nx[3];
        }
        const uint32_t w[16] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w,
                                c2.x, c2.y, c2.z, c2.w, c3.x, c3.y, c3.z, c3.w};
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (t0 + u < W) f(w[u]);
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
}

constexpr int WB = qb_ceil_log2(NW);

template <int EPT, bool K32>
__global__ void __launch_bounds__(TB) k_tabu_sp(const uint32_t *__restrict__ ell, int W,
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
    extern __shared__ uint32_t rowbuf[];   // [2][NW][W]

    const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wid_u = __builtin_amdgcn_readfirstlane(wid);
    const int64_t ro = (int64_t)p * n;
    constexpr uint32_t TBIT = 0x80000000u;       // set in a key while the variable is tabu
    // padding elements carry the largest possible key, tabu for ever
    const uint32_t dpad = 0x7FFFFFFFu >> EB;

    uint32_t Kb[EPT];   // ((D + bias) << EB | e) | TBIT if tabu
    int32_t U[EPT];     // tabu through step U
    int32_t nexp = 0x7fffffff;   // smallest U among the thread's tabu variables
    uint32_t xb = 0;    // x bits of the owned variables (EPT <= 20)
    uint32_t pb = 0;    // flipped since the last improvement
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int j = e * TB + tid;
        U[e] = 0;
        if (j < n) {
            Tout[ro + j] = 0;
            LFout[ro + j] = 0;
            const int32_t x = X[ro + j] & 1;
            xb |= (uint32_t)x << e;
            Kb[e] = (((uint32_t)(diag[j] + (x ? -2 : 2) * H[ro + j]) + bias) << EB) | (uint32_t)e;
        } else {
            Kb[e] = (dpad << EB) | (uint32_t)e | TBIT;
            U[e] = 0x7fffffff;
        }
    }
    int64_t OV = E[p];
    int64_t gap = 0;    // OV - OV_min, never negative
    constexpr uint32_t KNONE = 0xFFFFFFFFu;

    for (int step = 1; step <= alpha; ++step) {
        // aspiration: a tabu key k aspirates when (k >> EB) < OV_min - OV + bias,
        // that is k < tbk (zero when nothing can aspirate)
        uint32_t tbk = 0;
        {
            const uint32_t gh = (uint32_t)((uint64_t)gap >> 32), gl = (uint32_t)gap;
            if (asp && gh == 0u && gl < bias) tbk = (bias - gl) << EB;
        }
        const int32_t free_at = step - 1;
        if (free_at >= nexp) {
            // a tabu variable of this thread is free again (every variable
            // that is not tabu has U <= free_at already, padding never frees)
            nexp = 0x7fffffff;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const bool freed = U[e] <= free_at;
                Kb[e] &= freed ? ~TBIT : ~0u;
                nexp = min(nexp, freed ? 0x7fffffff : U[e]);
            }
        }
        // smallest free key (unsigned minimum: tabu keys carry bit 31) and
        // smallest tabu key (signed minimum); the smallest tabu key
        // aspirates whenever any does
        uint32_t m1 = KNONE;
        int32_t m2 = 0x7fffffff;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            m1 = min(m1, Kb[e]);
            m2 = min(m2, (int32_t)Kb[e]);
        }
        const uint32_t kfa = (uint32_t)max((int32_t)m1, -1);   // KNONE when every key is tabu
        const uint32_t kta = (uint32_t)m2 ^ TBIT;              // >= TBIT (never aspirates) when none is
        const uint32_t best = min(kfa, kta < tbk ? kta : KNONE);
        const uint32_t wmin = qb_wave_min_u32_b(best);
        // the wave's winner slot for minimum key wm among the lanes' keys
        // bsel (a whole-wave call), and the copy of its candidate row;
        // padding keys never win a 32-bit slot
        auto slot_of = [&](uint32_t wm, uint32_t bsel) -> uint64_t {
            const uint64_t who = __ballot(bsel == wm);
            const int L = __builtin_ctzll(who);
            const int ew = (int)(wm & EMASK);
            const uint32_t xw = ((uint32_t)__builtin_amdgcn_readlane((int)xb, L) >> ew) & 1u;
            const int iw = ew * TB + wid * 64 + L;
            uint32_t *rb = rowbuf + ((step & 1) * NW + wid) * W;
            if (iw < n)
                for (int t = lane; t < W; t += 64) rb[t] = ell[(int64_t)iw * W + t];
            if constexpr (K32) {
                if (wm >= (1u << (31 - WB))) return ~0ull;
                return ((uint64_t)(((uint32_t)L << 1) | xw) << 32) | ((wm << WB) | (uint32_t)wid);
            } else {
                return qb_tabu_winner(wm >> EB, iw, xw);
            }
        };
        uint64_t wkey = ~0ull;
        if (wmin != KNONE) wkey = slot_of(wmin, best);
        if (lane == 0) red[step & 1][wid] = wkey;
        __syncthreads();
        uint32_t dib;
        int i;
        int32_t s;                                 // direction of x_i
        if constexpr (K32) {
            uint32_t key = 0, hi = 0;
            if (!qb_pick32<NW>(red[step & 1], lane, key, hi)) {
                // every variable is tabu and none aspirates: argmin over all of them
                const uint32_t b2 = min(kfa, kta);
                const uint32_t w2 = qb_wave_min_u32_b(b2);
                const uint64_t k2 = slot_of(w2, b2);
                if (lane == 0) red2[wid] = k2;
                __syncthreads();
                qb_pick32<NW>(red2, lane, key, hi);
            }
            const uint32_t wm = key >> WB;
            dib = wm >> EB;
            i = (int)(wm & EMASK) * TB + (int)(key & (NW - 1)) * 64 + (int)(hi >> 1);
            s = (hi & 1u) ? -1 : 1;
        } else {
            uint64_t kb = qb_min_winners<NW>(red[step & 1], lane);
            if (kb == ~0ull) {
                // every variable is tabu and none aspirates: argmin over all of them
                const uint32_t b2 = min(kfa, kta);
                const uint32_t w2 = qb_wave_min_u32_b(b2);
                const uint64_t k2 = slot_of(w2, b2);
                if (lane == 0) red2[wid] = k2;
                __syncthreads();
                kb = qb_min_winners<NW>(red2, lane);
            }
            dib = (uint32_t)(kb >> 32);
            i = __builtin_amdgcn_readfirstlane((int)((uint32_t)kb >> 1));
            s = (kb & 1) ? -1 : 1;
        }
        const int32_t dmove = (int32_t)(dib - bias);
        OV += dmove;
        gap += dmove;

        // neighbours j of i: h_j += s Q_ji, so D_j += 2(1-2x_j) s Q_ji
        auto nb = [&](uint32_t wd) {
            const int c = qb_ell_col(wd);
            if (wd != 0u && ((c >> 6) & (NW - 1)) == wid_u && lane == (c & 63)) {
                const int32_t dv = s * qb_ell_val(wd);
                switch (c >> TSHIFT) {
#define QB_NB_CASE(K)                                                                        \
    case K:                                                                                  \
        if constexpr (K < EPT)                                                               \
            Kb[K] += (uint32_t)(((xb >> K) & 1u) ? -2 * dv : 2 * dv) << EB;                  \
        break;
                    QB_SWITCH20(QB_NB_CASE)
#undef QB_NB_CASE
                default: break;
                }
            }
        };
        {
            const uint32_t *rb = rowbuf + ((step & 1) * NW + ((i >> 6) & (NW - 1))) * W;
            for (int t0 = 0; t0 < W; t0 += 64) {
                const uint32_t wd = t0 + lane < W ? rb[t0 + lane] : 0u;
                const int c = qb_ell_col(wd);
                uint64_t mine = __ballot(wd != 0u && ((c >> 6) & (NW - 1)) == wid);
                while (mine) {
                    const int t = __builtin_ctzll(mine);
                    mine &= mine - 1;
                    nb((uint32_t)__builtin_amdgcn_readlane((int)wd, t));
                }
            }
        }
        if (tid == (i & TMASK)) {
            // the zeroing stores above precede the first step's barrier
            __hip_atomic_fetch_add(Tout + ro + i, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            LFout[ro + i] = step;
            xb ^= 1u << (i >> TSHIFT);
            pb ^= 1u << (i >> TSHIFT);
            switch (i >> TSHIFT) {
#define QB_OWNER_CASE(K)                                                         \
    case K:                                                                      \
        if constexpr (K < EPT) {                                                 \
            const int32_t Un = step + max(max(U[K] - (step - 1), 0) + tenure - 1, 0); \
            U[K] = Un;                                                           \
            Kb[K] = ((2u * bias - dib) << EB) | (uint32_t)K;                     \
            if (Un > step) {                                                     \
                Kb[K] |= TBIT;                                                   \
                nexp = min(nexp, Un);                                            \
            }                                                                    \
        }                                                                        \
        break;
                QB_SWITCH20(QB_OWNER_CASE)
#undef QB_OWNER_CASE
            default: break;
            }
        }
        if ((int32_t)((uint64_t)gap >> 32) < 0) {
            // a new best: x_min is the current x
            gap = 0;
            pb = 0;
        }
    }
    const int64_t OVmin = OV - gap;

    // field of the final x from D, then moved to x_min = x ^ pb by the
    // neighbour lists of the differing variables
    int32_t h[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int j = e * TB + tid;
        h[e] = 0;
        if (j < n) {
            const int32_t sg = ((xb >> e) & 1u) ? -2 : 2;
            h[e] = ((int32_t)(((Kb[e] & ~TBIT) >> EB) - bias) - diag[j]) * sg / 4;
        }
    }
    for (int e = 0; e < EPT; ++e) {
        if (tid == 0) lcount = 0;
        __syncthreads();
        if (e * TB + tid < n && ((pb >> e) & 1u)) {
            const int pos = atomicAdd(&lcount, 1);
            const int jj = e * TB + tid;
            list[pos] = ((xb >> e) & 1u) ? -(jj + 1) : (jj + 1);
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
            for_row(ell, W, jv, hup);
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int j = e * TB + tid;
        if (j < n) {
            X[ro + j] = (uint8_t)(((xb ^ pb) >> e) & 1u);
            H[ro + j] = h[e];
        }
    }
    if (tid == 0) E[p] = OVmin;
}

#undef QB_SWITCH20

}  // namespace

qb_status qb_tabu_tree_launch(qb_problem P, int z, uint8_t *X, int32_t *H, int64_t *E, int alpha, int tenure,
                              int asp, int32_t *T, int32_t *LF, hipStream_t s);

qb_status qb_tabu_sparse_launch(qb_problem P, int z, uint8_t *X, int32_t *H, int64_t *E, int alpha, int tenure,
                                int asp, int32_t *T, int32_t *LF, hipStream_t s)
{
    if (P->tabu_variant != QB_TABU_LANES) {
        const qb_status rc = qb_tabu_tree_launch(P, z, X, H, E, alpha, tenure, asp, T, LF, s);
        if ((rc != QB_E_CAPACITY && rc != QB_E_RANGE) || P->tabu_variant == QB_TABU_TREE) return rc;
    }
    const int ept = qb_tabu_sp_ept(P->n);
    if (ept == 0) return QB_E_CAPACITY;
    const int64_t dmax = (int64_t)P->qmax + 2 * P->eta_max;
    const uint32_t bias = (uint32_t)dmax;
    // each wave's candidate row, double-buffered by step parity
    const size_t lds = sizeof(uint32_t) * 2 * NW * (size_t)P->ellw;
    if (lds > 64 * 1024) return QB_E_CAPACITY;
#define QB_T(K)                                                                                     \
    if (ept == K) {                                                                                \
        if (2 * dmax + 1 >= (int64_t)(0x7FFFFFFFu >> qb_ceil_log2(K))) return QB_E_RANGE;          \
        if (lds > 48 * 1024) {                                                                     \
            QB_TRY_HIP(hipFuncSetAttribute((const void *)k_tabu_sp<K, true>,                       \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)); \
            QB_TRY_HIP(hipFuncSetAttribute((const void *)k_tabu_sp<K, false>,                      \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)); \
        }                                                                                          \
        if (((2 * dmax + 1) << qb_ceil_log2(K)) < (int64_t(1) << (31 - WB)))                         \
            k_tabu_sp<K, true><<<z, TB, lds, s>>>(P->ell, P->ellw, P->diag, P->n, X, H, E, alpha, tenure, \
                                                  asp, T, LF, bias);                                 \
        else                                                                                       \
            k_tabu_sp<K, false><<<z, TB, lds, s>>>(P->ell, P->ellw, P->diag, P->n, X, H, E, alpha,      \
                                                   tenure, asp, T, LF, bias);                        \
        QB_LAUNCH_CHECK();                                                                         \
        return QB_OK;                                                                              \
    }
    QB_T(1) QB_T(2) QB_T(3) QB_T(4) QB_T(5) QB_T(6) QB_T(7) QB_T(8) QB_T(10) QB_T(12) QB_T(14) QB_T(16)
    QB_T(20)
#undef QB_T
    return QB_E_CAPACITY;
}
