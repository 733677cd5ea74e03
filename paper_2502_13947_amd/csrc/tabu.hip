// Tabu search (Alg. 1 of the IC-D^2S paper) on gfx950: one workgroup per
// solution, of 1024 threads (sixteen waves, four per SIMD, so the per-step
// element work is spread thin and one wave's latency overlaps the others'
// work), or of 512 threads at the sizes where eight waves measured faster
// (qb_tabu_threads).
//
// Thread t owns the variables j = e*TB + t (e < EPT) and keeps in
// registers, per variable: the move value D_j = Q_jj + 2(1-2x_j)h_j (biased
// to be non-negative), the factor S_j = 2(1-2x_j), and the step U_j after
// which the variable is free again.  U replaces the tenure vector of the
// listing: "C_j <= 0 at step t" is exactly "U_j <= t-1" when U is updated
// only for the flipped variable, so no per-step decrement pass is needed.
//
// One step: every lane forms a 32-bit key (move value, element) for each of
// its allowed variables (not tabu, or aspirating: OV + D < OV_min) and keeps
// the minimum; the wave minimum comes from DPP row operations and the row
// broadcasts; index order inside a wave is (element, lane), so the lowest
// lane holding the minimal key gives the lowest index; the sixteen wave
// winners meet in LDS (one barrier per step, double-buffered slots, the
// step loop run in pairs so every slot address is fixed), where a DPP
// minimum over lanes picks the smallest (32-bit (key, wave) when the move
// values allow, else 64-bit (move, index, x)).  The chosen variable's row is
// read from the Tabu copy of Q, where each thread's elements lie in one
// padded, naturally aligned slot of up to 16 bytes, or in a few aligned
// chunks beyond that (qb_tabu_pos), so a wave issues one vector load per
// slot or chunk rather than one byte load per element; every D is updated by
// one multiply-add and the owner of the flipped variable patches its own
// element.  x_min is never copied: per-variable "flipped since the last
// improvement" bits recover it, and the field is moved to x_min with the
// rows of the differing variables.
#include <algorithm>

#include "qb_internal.h"

#include <type_traits>

namespace {

// Cross-wave winner in 32 bits (K32): the slot's low word is
// (wave minimum key << WB) | wave and its high word (lane << 1) | x, with
// NW = TB / 64 waves and WB = log2 NW.  Within a wave the ballot already
// took the lowest lane among equal keys, and across waves (move, element,
// wave) orders exactly as (move, index) since index = element * TB + wave *
// 64 + lane; so a 32-bit DPP minimum over the slots picks the winner and one
// readlane of the winning slot's high word gives its lane and x.  Used when
// every real key fits 31 - WB bits.
template <int TB>
struct TabuShape {
    static constexpr int NW = TB / 64;
    static constexpr int WB = qb_ceil_log2(NW);
    static_assert(TB == 512 || TB == 1024, "eight or sixteen waves");
};

constexpr int qb_pow2_at_least(int v) { return v <= 1 ? 1 : 2 * qb_pow2_at_least((v + 1) / 2); }

// Thread tid's elements of one row of the Tabu copy of Q (the order of
// qb_tabu_pos), sign-extended: up to 16 bytes one naturally aligned load of
// the thread's padded slot; beyond, one load per chunk, chunks of SZ
// elements from element START on.
template <typename QT, int EPT, int TB, int START = 0, int SZ = 16 / (int)sizeof(QT)>
__device__ __forceinline__ void tabu_row(const QT *row, uint32_t tid, int32_t (&q)[EPT])
{
    constexpr int BYTES_ALL = EPT * (int)sizeof(QT);
    if constexpr (START == 0 && BYTES_ALL <= 16 && qb_pow2_at_least(BYTES_ALL) != BYTES_ALL) {
        constexpr int SLOT = qb_pow2_at_least(BYTES_ALL);     // bytes
        const uint8_t *p = reinterpret_cast<const uint8_t *>(row) + tid * (uint32_t)SLOT;
        uint32_t w[4];
        if constexpr (SLOT == 16) {
            const uint4 v = *reinterpret_cast<const uint4 *>(p);
            w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
        } else if constexpr (SLOT == 8) {
            const uint2 v = *reinterpret_cast<const uint2 *>(p);
            w[0] = v.x; w[1] = v.y; w[2] = 0u; w[3] = 0u;
        } else {
            w[0] = *reinterpret_cast<const uint32_t *>(p); w[1] = w[2] = w[3] = 0u;
        }
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const uint32_t word = w[(k * (int)sizeof(QT)) / 4];
            const int sh = ((k * (int)sizeof(QT)) % 4) * 8;
            q[k] = sizeof(QT) == 1 ? (int32_t)(int8_t)(word >> sh) : (int32_t)(int16_t)(word >> sh);
        }
    } else if constexpr (SZ >= 1 && START < EPT) {
        if constexpr (EPT - START >= SZ) {
            constexpr int BYTES = SZ * (int)sizeof(QT);
            const uint8_t *p = reinterpret_cast<const uint8_t *>(row + START * TB) + tid * (uint32_t)BYTES;
            uint32_t w[(BYTES + 3) / 4];
            if constexpr (BYTES == 16) {
                const uint4 v = *reinterpret_cast<const uint4 *>(p);
                w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
            } else if constexpr (BYTES == 8) {
                const uint2 v = *reinterpret_cast<const uint2 *>(p);
                w[0] = v.x; w[1] = v.y;
            } else if constexpr (BYTES == 4) {
                w[0] = *reinterpret_cast<const uint32_t *>(p);
            } else if constexpr (BYTES == 2) {
                w[0] = *reinterpret_cast<const uint16_t *>(p);
            } else {
                w[0] = *p;
            }
#pragma unroll
            for (int k = 0; k < SZ; ++k) {
                const uint32_t word = w[(k * (int)sizeof(QT)) / 4];
                const int sh = ((k * (int)sizeof(QT)) % 4) * 8;
                q[START + k] = sizeof(QT) == 1 ? (int32_t)(int8_t)(word >> sh) : (int32_t)(int16_t)(word >> sh);
            }
            tabu_row<QT, EPT, TB, START + SZ, SZ>(row, tid, q);
        } else {
            tabu_row<QT, EPT, TB, START, SZ / 2>(row, tid, q);
        }
    }
}

template <int EPT, typename QT, bool K32, int TB>
__global__ void __launch_bounds__(TB) k_tabu(const QT *__restrict__ Qt, int ldp, const int16_t *__restrict__ Q16,
                                             int n, uint8_t *__restrict__ X, int32_t *__restrict__ H,
                                             int64_t *__restrict__ E, int alpha, int tenure, int asp,
                                             int32_t *__restrict__ Tout, int32_t *__restrict__ LFout,
                                             uint32_t bias)
{
    constexpr int NW = TabuShape<TB>::NW, WB = TabuShape<TB>::WB;
    constexpr int EB = qb_ceil_log2(EPT);           // bits of the element index
    constexpr uint32_t EMASK = (1u << EB) - 1u;
    __shared__ uint64_t red[2][NW];
    __shared__ uint64_t red2[NW];
    __shared__ int32_t list[TB];
    __shared__ int lcount;
    extern __shared__ int32_t tl[];              // [0,n): flips, [n,2n): last-flip step
    int32_t *Ts = tl, *Ls = tl + n;

    const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t ro = (int64_t)p * n;
    constexpr uint32_t TBIT = 0x80000000u;       // set in a key while the variable is tabu
    constexpr uint32_t KNONE = 0xFFFFFFFFu;
    // padding elements carry the largest possible key, tabu for ever
    const uint32_t dpad = 0x7FFFFFFFu >> EB;

    uint32_t Kb[EPT];      // ((D + bias) << EB | e) | TBIT if tabu
    int32_t S[EPT];        // 2 (1 - 2 x) << EB
    int32_t U[EPT];        // tabu through step U
    uint32_t xb = 0;       // x bits of the owned variables (EPT <= 16)
    uint32_t pb = 0;       // flipped since the last improvement
    int32_t nexp = 0x7fffffff;   // smallest U among the thread's tabu variables
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int j = e * TB + tid;
        U[e] = 0;
        if (j < n) {
            const int32_t x = X[ro + j] & 1;
            const int32_t qjj = Q16[(int64_t)j * n + j];
            S[e] = (x ? -2 : 2) << EB;
            xb |= (uint32_t)x << e;
            Kb[e] = (((uint32_t)(qjj + (x ? -2 : 2) * H[ro + j]) + bias) << EB) | (uint32_t)e;
            Ts[j] = 0;
            Ls[j] = 0;
        } else {
            S[e] = 2 << EB;
            Kb[e] = (dpad << EB) | (uint32_t)e | TBIT;
            U[e] = 0x7fffffff;                   // never allowed
        }
    }
    int64_t OV = E[p];
    int64_t gap = 0;       // OV - OV_min, never negative
    const int wu = __builtin_amdgcn_readfirstlane(wid);

    // One step; consecutive steps alternate the two slot buffers, so the loop
    // runs in pairs and every LDS address is fixed.
    auto one_step = [&](const int step, uint64_t *slots) {
        // aspiration: a tabu key k aspirates when (k >> EB) < OV_min - OV + bias,
        // that is k < tbk (zero when nothing can aspirate)
        uint32_t tbk = 0;
        {
            const uint32_t gh = (uint32_t)((uint64_t)gap >> 32), gl = (uint32_t)gap;
            if (asp && gh == 0u && gl < bias) tbk = (bias - gl) << EB;
        }
        const int32_t free_at = step - 1;
        if (free_at >= nexp) {
            // a tabu variable of this thread is free again.  Every variable
            // that is not tabu has U <= free_at already (clearing its bit is a
            // no-op), and padding never frees (U = INT_MAX), so no per-element
            // branch is needed
            nexp = 0x7fffffff;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const bool freed = U[e] <= free_at;
                Kb[e] &= freed ? ~TBIT : ~0u;
                nexp = min(nexp, freed ? 0x7fffffff : U[e]);
            }
        }
        // smallest free key (tabu keys carry bit 31, so they lose the
        // unsigned minimum) and smallest tabu key (they win the signed one);
        // the smallest tabu key aspirates whenever any does
        uint32_t m1 = KNONE;
        int32_t m2 = 0x7fffffff;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            m1 = min(m1, Kb[e]);
            m2 = min(m2, (int32_t)Kb[e]);
        }
        const uint32_t fk = (uint32_t)max((int32_t)m1, -1);    // KNONE when every key is tabu
        const uint32_t tk = (uint32_t)m2 ^ TBIT;               // >= TBIT (never aspirates) when none is
        const uint32_t best = min(fk, tk < tbk ? tk : KNONE);
        const uint32_t wmin = qb_wave_min_u32_b(best);
        // the wave's winner slot for minimum key wm among the lanes' keys bsel
        // (a whole-wave call); padding keys never win a K32 slot
        auto slot_of = [&](uint32_t wm, uint32_t bsel) -> uint64_t {
            // lowest index among the minimal moves: the lowest lane holding the
            // minimal move value, then that lane's own lowest element
            const uint64_t who = __ballot(bsel == wm);
            const int L = __builtin_ctzll(who);
            const int ew = (int)(wm & EMASK);
            const uint32_t xw = ((uint32_t)__builtin_amdgcn_readlane((int)xb, L) >> ew) & 1u;
            if constexpr (K32) {
                if (wm >= (1u << (31 - WB))) return ~0ull;
                return ((uint64_t)(((uint32_t)L << 1) | xw) << 32) | ((wm << WB) | (uint32_t)wu);
            } else {
                return qb_tabu_winner(wm >> EB, ew * TB + wu * 64 + L, xw);
            }
        };
        uint64_t wkey = ~0ull;
        if (wmin != KNONE) wkey = slot_of(wmin, best);
        if (lane == 0) slots[wid] = wkey;
        __syncthreads();
        uint32_t dib;
        int i;
        int32_t s;                                 // direction of x_i
        if constexpr (K32) {
            uint32_t key = 0, hi = 0;
            if (!qb_pick32<NW>(slots, lane, key, hi)) {
                // every variable is tabu and none aspirates: argmin over all of them
                const uint32_t b2 = min(fk, tk);
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
            uint64_t kb = qb_min_winners<NW>(slots, lane);
            if (kb == ~0ull) {
                // every variable is tabu and none aspirates: argmin over all of them
                const uint32_t b2 = min(fk, tk);
                const uint32_t w2 = qb_wave_min_u32_b(b2);
                const uint64_t k2 = slot_of(w2, b2);
                if (lane == 0) red2[wid] = k2;
                __syncthreads();
                kb = qb_min_winners<NW>(red2, lane);
            }
            dib = (uint32_t)(kb >> 32);
            i = (int)((uint32_t)kb >> 1);
            s = (kb & 1) ? -1 : 1;
        }
        const int32_t dmove = (int32_t)(dib - bias);
        OV += dmove;
        gap += dmove;
        // the row base is uniform (scalar registers); each lane adds its own
        // 32-bit chunk offsets
        int32_t q[EPT];
        tabu_row<QT, EPT, TB>(Qt + (uint32_t)i * (uint32_t)ldp, (uint32_t)tid, q);
        // h_j += s Q_ji  =>  D_j += S_j s Q_ji, applied to the key above its
        // element bits (the owner is patched below)
        if (s > 0) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) Kb[e] += (uint32_t)__mul24(q[e], S[e]);
        } else {
#pragma unroll
            for (int e = 0; e < EPT; ++e) Kb[e] -= (uint32_t)__mul24(q[e], S[e]);
        }
        const int ti = i & (TB - 1);
        if (tid == ti) {
            // the owner patches its element ei and bumps the counters without
            // waiting on LDS
            const int ei = i / TB;
            xb ^= 1u << ei;
            pb ^= 1u << ei;
            atomicAdd(&Ts[i], 1);
            Ls[i] = step;
            // tenure from this step on (the remaining tenure of an aspirated
            // variable carries over), and the new key: minus the old move value
            auto tabu_until = [&](int32_t u) { return step + max(max(u - (step - 1), 0) + tenure - 1, 0); };
            auto new_key = [&](int32_t un, uint32_t e) {
                uint32_t kn = ((2u * bias - dib) << EB) | e;
                if (un > step) {
                    kn |= TBIT;
                    nexp = min(nexp, un);
                }
                return kn;
            };
            auto patch = [&](auto ec) {
                constexpr int e = decltype(ec)::value;
                if constexpr (e < EPT) {
                    const int32_t Un = tabu_until(U[e]);
                    U[e] = Un;
                    S[e] = -S[e];
                    Kb[e] = new_key(Un, (uint32_t)e);
                }
            };
            static_assert(EPT <= 16, "sixteen cases");
            if constexpr (EPT <= 10) {
                // the uniform ei indexes the register arrays (selects over
                // the few elements)
                const int32_t Un = tabu_until(U[ei]);
                U[ei] = Un;
                S[ei] = -S[ei];
                Kb[ei] = new_key(Un, (uint32_t)ei);
            } else switch (ei) {
                // a scalar branch per element: an index into the larger
                // arrays would send them to scratch memory
#define QB_TABU_CASE(c) \
    case c: patch(std::integral_constant<int, c>{}); break;
                QB_TABU_CASE(0) QB_TABU_CASE(1) QB_TABU_CASE(2) QB_TABU_CASE(3)
                QB_TABU_CASE(4) QB_TABU_CASE(5) QB_TABU_CASE(6) QB_TABU_CASE(7)
                QB_TABU_CASE(8) QB_TABU_CASE(9) QB_TABU_CASE(10) QB_TABU_CASE(11)
                QB_TABU_CASE(12) QB_TABU_CASE(13) QB_TABU_CASE(14) QB_TABU_CASE(15)
#undef QB_TABU_CASE
            default: break;
            }
        }
        if ((int32_t)((uint64_t)gap >> 32) < 0) {
            // a new best: x_min is the current x
            gap = 0;
            pb = 0;
        }
    };

    int step = 1;
    for (; step < alpha; step += 2) {
        one_step(step, red[1]);
        one_step(step + 1, red[0]);
    }
    if (step == alpha) one_step(step, red[1]);
    const int64_t OVmin = OV - gap;

    // field of the final x from D, then moved to x_min = x ^ pb row by row
    int32_t h[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int j = e * TB + tid;
        h[e] = 0;
        if (j < n) {
            const int32_t qjj = Q16[(int64_t)j * n + j];
            h[e] = ((int32_t)(((Kb[e] & ~TBIT) >> EB) - bias) - qjj) * (S[e] >> EB) / 4;
        }
    }
#pragma unroll
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
            int32_t q[EPT];
            tabu_row<QT, EPT, TB>(Qt + (uint32_t)(v < 0 ? -v - 1 : v - 1) * (uint32_t)ldp, (uint32_t)tid, q);
#pragma unroll
            for (int e2 = 0; e2 < EPT; ++e2) h[e2] += sg * q[e2];
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int j = e * TB + tid;
        if (j < n) {
            X[ro + j] = (uint8_t)(((xb ^ pb) >> e) & 1u);
            H[ro + j] = h[e];
            Tout[ro + j] = Ts[j];
            LFout[ro + j] = Ls[j];
        }
    }
    if (tid == 0) E[p] = OVmin;
}

template <int EPT, typename QT, bool K32, int TB>
qb_status launch_one(const QT *Qt, int ldp, qb_problem P, int z, uint8_t *X, int32_t *H, int64_t *E, int alpha,
                     int tenure, int asp, int32_t *T, int32_t *LF, uint32_t bias, hipStream_t s)
{
    const size_t lds = sizeof(int32_t) * 2 * (size_t)P->n;
    QB_TRY_HIP(hipFuncSetAttribute((const void *)k_tabu<EPT, QT, K32, TB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
    k_tabu<EPT, QT, K32, TB><<<z, TB, lds, s>>>(Qt, ldp, P->Q, P->n, X, H, E, alpha, tenure, asp, T, LF, bias);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

// The 32-bit winner key when every real key fits 31 - WB bits, else 64 bits.
template <int EPT, typename QT, int TB>
qb_status launch_keyed(const QT *Qt, int ldp, qb_problem P, int z, uint8_t *X, int32_t *H, int64_t *E,
                       int alpha, int tenure, int asp, int32_t *T, int32_t *LF, int64_t dmax, hipStream_t s)
{
    if (2 * dmax + 1 >= (int64_t)(0x7FFFFFFFu >> qb_ceil_log2(EPT))) return QB_E_RANGE;
    const uint32_t bias = (uint32_t)dmax;
    if (((2 * dmax + 1) << qb_ceil_log2(EPT)) < (int64_t(1) << (31 - TabuShape<TB>::WB)))
        return launch_one<EPT, QT, true, TB>(Qt, ldp, P, z, X, H, E, alpha, tenure, asp, T, LF, bias, s);
    return launch_one<EPT, QT, false, TB>(Qt, ldp, P, z, X, H, E, alpha, tenure, asp, T, LF, bias, s);
}

template <typename QT>
qb_status launch_tabu(qb_problem P, const QT *Qt, int ldp, int z, uint8_t *X, int32_t *H, int64_t *E, int alpha,
                      int tenure, int asp, int32_t *T, int32_t *LF, hipStream_t s)
{
    const int ept = P->tabu_ept, tb = P->tabu_tb;
    if (ept == 0 || ldp != qb_tabu_pitch(tb, ept, (int)sizeof(QT))) return QB_E_CAPACITY;
    const int64_t dmax = (int64_t)P->qmax + 2 * P->eta_max;
#define QB_T(K, W)                                                                                 \
    if (ept == K && tb == W)                                                                      \
        return launch_keyed<K, QT, W>(Qt, ldp, P, z, X, H, E, alpha, tenure, asp, T, LF, dmax, s);
    // eight waves only where qb_tabu_threads picks them (5, 6 or 10 elements)
    QB_T(5, 512) QB_T(6, 512) QB_T(10, 512)
    QB_T(1, 1024) QB_T(2, 1024) QB_T(3, 1024) QB_T(4, 1024) QB_T(5, 1024) QB_T(6, 1024)
    QB_T(7, 1024) QB_T(8, 1024) QB_T(10, 1024) QB_T(12, 1024) QB_T(14, 1024) QB_T(16, 1024)
#undef QB_T
    return QB_E_CAPACITY;
}

}  // namespace

qb_status qb_tabu_sparse_launch(qb_problem P, int z, uint8_t *X, int32_t *H, int64_t *E, int alpha, int tenure,
                                int asp, int32_t *T, int32_t *LF, hipStream_t s);

extern "C" qb_status qb_tabu(qb_problem P, int32_t z, uint8_t *X_d, int32_t *H_d, int64_t *E_d,
                            int32_t alpha, int32_t tenure, int32_t aspiration, int32_t *T_d,
                            int32_t *LF_d, void *stream)
{
    if (!P || z < 1 || !X_d || !H_d || !E_d || !T_d || !LF_d || alpha < 0 || tenure < 0)
        return QB_E_ARG;
    // a tenure that reaches past the last step keeps a variable tabu to the
    // end either way: alpha + 1 gives the same search and keeps the kernels'
    // step and counter arithmetic far from int32 overflow
    tenure = (int32_t)std::min<int64_t>(tenure, (int64_t)alpha + 1);
    hipStream_t s = qb_stream(stream);
    if (P->sparse)
        return qb_tabu_sparse_launch(P, z, X_d, H_d, E_d, alpha, tenure, aspiration != 0, T_d, LF_d, s);
    if (P->tabu_ept == 0) return QB_E_CAPACITY;
    if (P->int8_ok)
        return launch_tabu<int8_t>(P, (const int8_t *)P->Qt, P->ldp, z, X_d, H_d, E_d, alpha, tenure,
                                   aspiration != 0, T_d, LF_d, s);
    return launch_tabu<int16_t>(P, (const int16_t *)P->Qt, P->ldp, z, X_d, H_d, E_d, alpha, tenure,
                                aspiration != 0, T_d, LF_d, s);
}
