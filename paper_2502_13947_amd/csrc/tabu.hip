// Tabu search (Alg. 1 of the IC-D^2S paper) on gfx950: one 1024-thread
// workgroup per solution.  Every thread keeps EPT variables' local field,
// tenure counter and diagonal entry in registers (flip counts and last-flip
// steps, touched only by the owner of the flipped variable, live in LDS); one
// step is a
// lexicographic (move value, index) argmin (wave shuffles + one LDS exchange,
// a single barrier per step thanks to double-buffered slots), then the
// chosen variable's row of Q (int8 copy when it fits) updates every field.
// x_min is never copied: a per-variable "flipped since the last improvement"
// bit recovers it at the end, and the field is moved to x_min by the rows of
// the differing variables.
#include "qb_internal.h"

namespace {

constexpr int TB = 1024;           // threads per solution
constexpr int NW = TB / 64;        // waves

// (move value, index, x) packed so that unsigned order = (move asc, index asc)
__device__ __forceinline__ uint64_t pack_move(int32_t d, int j, uint32_t x)
{
    return ((uint64_t)((uint32_t)d ^ 0x80000000u) << 32) | ((uint64_t)(uint32_t)j << 1) | x;
}

template <int EPT, typename QT>
__global__ void __launch_bounds__(TB) k_tabu(const int16_t *__restrict__ Q16, const QT *__restrict__ Qr,
                                             int n, uint8_t *__restrict__ X, int32_t *__restrict__ H,
                                             int64_t *__restrict__ E, int alpha, int tenure, int asp,
                                             int32_t *__restrict__ Tout, int32_t *__restrict__ LFout)
{
    __shared__ uint64_t red[2][NW];
    __shared__ uint64_t red2[NW];
    __shared__ int32_t list[TB];
    __shared__ int lcount;
    extern __shared__ int32_t tl[];           // [0,n): flip counts, [n,2n): last-flip steps
    int32_t *Ts = tl, *Ls = tl + n;

    const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t rowoff = (int64_t)p * n;
    int32_t h[EPT], C[EPT], qd[EPT];
    uint32_t xb = 0, pb = 0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int j = tid + TB * e;
        h[e] = 0; qd[e] = 0; C[e] = 0;
        if (j < n) {
            Ts[j] = 0;
            Ls[j] = 0;
            h[e] = H[rowoff + j];
            qd[e] = Q16[(int64_t)j * n + j];
            xb |= (uint32_t)(X[rowoff + j] & 1) << e;
        }
    }
    int64_t OV = E[p], OVmin = OV;

    for (int step = 1; step <= alpha; ++step) {
        uint64_t best = ~0ull;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int j = tid + TB * e;
            if (j < n) {
                const uint32_t xe = (xb >> e) & 1u;
                const int32_t d = qd[e] + 2 * (xe ? -h[e] : h[e]);
                const bool allowed = C[e] <= 0 || (asp && OV + d < OVmin);
                const uint64_t key = pack_move(d, j, xe);
                if (allowed && key < best) best = key;
            }
        }
        best = qb_wave_min_u64(best);
        if (lane == 0) red[step & 1][wid] = best;
        __syncthreads();
        uint64_t kb = red[step & 1][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) kb = min(kb, red[step & 1][w]);
        if (kb == ~0ull) {
            // every variable is tabu and none aspirates: argmin over all
            uint64_t b2 = ~0ull;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int j = tid + TB * e;
                if (j < n) {
                    const uint32_t xe = (xb >> e) & 1u;
                    const int32_t d = qd[e] + 2 * (xe ? -h[e] : h[e]);
                    b2 = min(b2, pack_move(d, j, xe));
                }
            }
            b2 = qb_wave_min_u64(b2);
            if (lane == 0) red2[wid] = b2;
            __syncthreads();
            kb = red2[0];
#pragma unroll
            for (int w = 1; w < NW; ++w) kb = min(kb, red2[w]);
        }
        const int32_t di = (int32_t)((uint32_t)(kb >> 32) ^ 0x80000000u);
        const int i = (int)((kb >> 1) & 0x7fffffffu);
        const int32_t sgn = (kb & 1) ? -1 : 1;
        OV += di;
        const QT *row = Qr + (int64_t)i * n;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int j = tid + TB * e;
            if (j < n) h[e] += sgn * (int32_t)row[j];
            if (j == i) {
                xb ^= 1u << e;
                pb ^= 1u << e;
                Ts[j] += 1;
                Ls[j] = step;
                C[e] += tenure;
            }
            if (C[e] > 0) C[e] -= 1;
        }
        if (OV < OVmin) {
            OVmin = OV;
            pb = 0;
        }
    }

    // move the field from the final x to x_min = x ^ pb
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        if (tid == 0) lcount = 0;
        __syncthreads();
        const int j = tid + TB * e;
        if (j < n && ((pb >> e) & 1u)) {
            const int pos = atomicAdd(&lcount, 1);
            list[pos] = ((xb >> e) & 1u) ? -(j + 1) : (j + 1);
        }
        __syncthreads();
        const int cnt = lcount;
        for (int u = 0; u < cnt; ++u) {
            const int32_t v = list[u];
            const int32_t s = v < 0 ? -1 : 1;
            const QT *row = Qr + (int64_t)(v < 0 ? -v - 1 : v - 1) * n;
#pragma unroll
            for (int e2 = 0; e2 < EPT; ++e2) {
                const int jj = tid + TB * e2;
                if (jj < n) h[e2] += s * (int32_t)row[jj];
            }
        }
        __syncthreads();
    }
    xb ^= pb;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int j = tid + TB * e;
        if (j < n) {
            X[rowoff + j] = (uint8_t)((xb >> e) & 1u);
            H[rowoff + j] = h[e];
            Tout[rowoff + j] = Ts[j];
            LFout[rowoff + j] = Ls[j];
        }
    }
    if (tid == 0) E[p] = OVmin;
}

template <typename QT>
qb_status launch_tabu(qb_problem P, const QT *Qr, int z, uint8_t *X, int32_t *H, int64_t *E,
                      int alpha, int tenure, int asp, int32_t *T, int32_t *LF, hipStream_t s)
{
    const int ept = (P->n + TB - 1) / TB;
    const size_t lds = sizeof(int32_t) * 2 * (size_t)P->n;
#define QB_TABU_CASE(K)                                                                       \
    case K:                                                                                   \
        (void)hipFuncSetAttribute((const void *)k_tabu<K, QT>,                                      \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);            \
        k_tabu<K, QT><<<z, TB, lds, s>>>(P->Q, Qr, P->n, X, H, E, alpha, tenure, asp, T, LF); \
        break;
    switch (ept) {
        QB_TABU_CASE(1)
        QB_TABU_CASE(2)
        QB_TABU_CASE(3)
        QB_TABU_CASE(4)
        QB_TABU_CASE(5)
        QB_TABU_CASE(6)
        QB_TABU_CASE(7)
        QB_TABU_CASE(8)
        QB_TABU_CASE(10)
        QB_TABU_CASE(12)
        QB_TABU_CASE(16)
    case 9:
        (void)hipFuncSetAttribute((const void *)k_tabu<10, QT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_tabu<10, QT><<<z, TB, lds, s>>>(P->Q, Qr, P->n, X, H, E, alpha, tenure, asp, T, LF);
        break;
    case 11:
        (void)hipFuncSetAttribute((const void *)k_tabu<12, QT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_tabu<12, QT><<<z, TB, lds, s>>>(P->Q, Qr, P->n, X, H, E, alpha, tenure, asp, T, LF);
        break;
    case 13:
    case 14:
    case 15:
        (void)hipFuncSetAttribute((const void *)k_tabu<16, QT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_tabu<16, QT><<<z, TB, lds, s>>>(P->Q, Qr, P->n, X, H, E, alpha, tenure, asp, T, LF);
        break;
    default: return QB_E_CAPACITY;
    }
#undef QB_TABU_CASE
    QB_LAUNCH_CHECK();
    return QB_OK;
}

}  // namespace

extern "C" qb_status qb_tabu(qb_problem P, int32_t z, uint8_t *X_d, int32_t *H_d, int64_t *E_d,
                            int32_t alpha, int32_t tenure, int32_t aspiration, int32_t *T_d,
                            int32_t *LF_d, void *stream)
{
    if (!P || z < 1 || !X_d || !H_d || !E_d || !T_d || !LF_d || alpha < 0 || tenure < 0)
        return QB_E_ARG;
    if (P->n > 16 * TB) return QB_E_CAPACITY;
    hipStream_t s = qb_stream(stream);
    if (P->int8_ok)
        return launch_tabu<int8_t>(P, P->Q8, z, X_d, H_d, E_d, alpha, tenure, aspiration != 0, T_d,
                                   LF_d, s);
    return launch_tabu<int16_t>(P, P->Q, z, X_d, H_d, E_d, alpha, tenure, aspiration != 0, T_d, LF_d,
                                s);
}
