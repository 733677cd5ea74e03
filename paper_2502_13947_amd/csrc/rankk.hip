// Rank-k local-field update H[p] += Q dX[p] (the Tabu section's O(n)
// move-value update generalised to every variable a stage changed).
//
// VALU variant: per (solution, column slice) the changed variables of dX[p]
// are compacted into an LDS list, then every thread adds +-Q[j][i] for its
// columns i (Q is symmetric, so column j of Q is row j: coalesced reads).
#include "qb_internal.h"

namespace {

constexpr int RK_CHUNK = 4096;

template <typename QT, int CPT>
__global__ void __launch_bounds__(256) k_rankk_valu(const QT *__restrict__ Q, int n, const int8_t *__restrict__ dX,
                                                    int32_t *__restrict__ H)
{
    __shared__ int32_t list[RK_CHUNK];
    __shared__ int cnt;
    const int p = blockIdx.y, tid = threadIdx.x;
    const int i0 = blockIdx.x * 256 * CPT;
    const int8_t *d = dX + (int64_t)p * n;
    int32_t acc[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) acc[c] = 0;
    for (int j0 = 0; j0 < n; j0 += RK_CHUNK) {
        if (tid == 0) cnt = 0;
        __syncthreads();
        for (int t = tid; t < RK_CHUNK; t += 256) {
            const int j = j0 + t;
            if (j < n) {
                const int v = d[j];
                if (v) list[atomicAdd(&cnt, 1)] = v > 0 ? (j + 1) : -(j + 1);
            }
        }
        __syncthreads();
        const int c_n = cnt;
        for (int u = 0; u < c_n; ++u) {
            const int32_t v = list[u];
            const int32_t s = v < 0 ? -1 : 1;
            const QT *row = Q + (int64_t)(v < 0 ? -v - 1 : v - 1) * n;
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int i = i0 + tid + 256 * c;
                if (i < n) acc[c] += s * (int32_t)row[i];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int i = i0 + tid + 256 * c;
        if (i < n && acc[c]) H[(int64_t)p * n + i] += acc[c];
    }
}

}  // namespace

extern "C" qb_status qb_rankk(qb_problem P, int32_t z, const int8_t *dX_d, int32_t *H_d, int32_t variant,
                             void *stream)
{
    if (!P || z < 1 || z > 65535 || !dX_d || !H_d || variant < 0 || variant > 2) return QB_E_ARG;
    if (variant == 2 && !P->int8_ok) return QB_E_UNSUPPORTED;
    hipStream_t s = qb_stream(stream);
    constexpr int CPT = 4;
    dim3 grid((P->n + 256 * CPT - 1) / (256 * CPT), z);
    if (variant == 2) return QB_E_UNSUPPORTED;   // MFMA path: see rankk_mfma
    if (P->int8_ok)
        k_rankk_valu<int8_t, CPT><<<grid, 256, 0, s>>>(P->Q8, P->n, dX_d, H_d);
    else
        k_rankk_valu<int16_t, CPT><<<grid, 256, 0, s>>>(P->Q, P->n, dX_d, H_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}
