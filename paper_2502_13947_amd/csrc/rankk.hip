// Rank-k local-field update H[p] += Q dX[p] (the Tabu section's O(n)
// move-value update generalised to every variable a stage changed).
//
// VALU variant (any Q, best for few solutions or few changed variables): per (solution, column slice) the changed variables of dX[p]
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

// ------------------------------------------------------------------ MFMA variant
// H (z x n) += dX (z x n, int8) . Q (n x n, int8): a real dense contraction.
// Q is symmetric, so the B operand's column i is row i of the padded copy Qp
// (K-contiguous, like the A operand's rows of dX).  v_mfma_i32_16x16x64_i8
// with int32 accumulation is exact (|sum| <= n * 127 * 1).  Workgroup tile:
// 64 solutions x 128 columns, four waves of 32 x 64 (2 x 4 MFMA tiles);
// K is split across blockIdx.z and the partial sums are added with integer
// atomics (exact and order independent).
typedef int v4i __attribute__((ext_vector_type(4)));

template <int AW>
__device__ __forceinline__ v4i load_a16(const int8_t *__restrict__ row, int kk, int n)
{
    v4i v = {0, 0, 0, 0};
    if (kk + 16 <= n) {
        if constexpr (AW == 16) {
            v = *reinterpret_cast<const v4i *>(row + kk);
        } else if constexpr (AW == 8) {
            const int2 lo = *reinterpret_cast<const int2 *>(row + kk);
            const int2 hi = *reinterpret_cast<const int2 *>(row + kk + 8);
            v = v4i{lo.x, lo.y, hi.x, hi.y};
        } else if constexpr (AW == 4) {
            const int *w = reinterpret_cast<const int *>(row + kk);
            v = v4i{w[0], w[1], w[2], w[3]};
        } else {
            uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
            for (int b = 0; b < 16; ++b) w[b >> 2] |= (uint32_t)(uint8_t)row[kk + b] << (8 * (b & 3));
            v = v4i{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
        }
    } else if (kk < n) {
        uint32_t w[4] = {0, 0, 0, 0};
        for (int b = 0; b < 16 && kk + b < n; ++b) w[b >> 2] |= (uint32_t)(uint8_t)row[kk + b] << (8 * (b & 3));
        v = v4i{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
    }
    return v;
}

template <int AW>
__global__ void __launch_bounds__(256) k_rankk_mfma(const int8_t *__restrict__ dX, int n, int z,
                                                    const int8_t *__restrict__ Qp, int ldp, int32_t *__restrict__ H,
                                                    int kchunk)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int n0 = blockIdx.x * 128 + (wave & 1) * 64;
    const int kend_all = (n + 63) & ~63;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(kbeg + kchunk, kend_all);
    const int r16 = lane & 15, g = lane >> 4;
    v4i acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4i{0, 0, 0, 0};
    const int8_t *arow[2];
    bool aok[2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
        const int p = m0 + mi * 16 + r16;
        aok[mi] = p < z;
        arow[mi] = dX + (int64_t)(aok[mi] ? p : 0) * n;
    }
    const int8_t *brow[4];
    bool bok[4];
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
        const int i = n0 + ni * 16 + r16;
        bok[ni] = i < n;
        brow[ni] = Qp + (int64_t)(bok[ni] ? i : 0) * ldp;
    }
    for (int k0 = kbeg; k0 < kend; k0 += 64) {
        const int kk = k0 + g * 16;
        v4i a[2], b[4];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) a[mi] = aok[mi] ? load_a16<AW>(arow[mi], kk, n) : v4i{0, 0, 0, 0};
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
            b[ni] = bok[ni] ? *reinterpret_cast<const v4i *>(brow[ni] + kk) : v4i{0, 0, 0, 0};
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
                acc[mi][ni] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
    }
    // 16x16 result layout: lane holds rows 4g..4g+3 of column r16
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = m0 + mi * 16 + 4 * g + r;
                const int i = n0 + ni * 16 + r16;
                const int32_t v = acc[mi][ni][r];
                if (p < z && i < n && v != 0) atomicAdd(&H[(int64_t)p * n + i], v);
            }
}

// Sparse product over the row-major ELL: H[p][i] (+)= Q_ii V[p][i] +
// sum_t val_t V[p][col_t].  One thread per (i, p); a row's words are read as
// 16-byte vectors (the width is a multiple of 4, and the zero words past a
// row's last entry add 0).
template <typename VT, bool ACC>
__global__ void __launch_bounds__(256) k_ell_spmm(const uint32_t *__restrict__ ell, const int32_t *__restrict__ ecnt,
                                                  const int32_t *__restrict__ diag, int n, int W,
                                                  const VT *__restrict__ V, int32_t *__restrict__ H)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int p = blockIdx.y;
    if (i >= n) return;
    const VT *v = V + (int64_t)p * n;
    int32_t acc = diag[i] * (int32_t)v[i];
    const uint4 *row = reinterpret_cast<const uint4 *>(ell + (int64_t)i * W);
    const int c4 = (ecnt[i] + 3) >> 2;
    for (int t = 0; t < c4; ++t) {
        const uint4 w = row[t];
        acc += qb_ell_val(w.x) * (int32_t)v[qb_ell_col(w.x)];
        acc += qb_ell_val(w.y) * (int32_t)v[qb_ell_col(w.y)];
        acc += qb_ell_val(w.z) * (int32_t)v[qb_ell_col(w.z)];
        acc += qb_ell_val(w.w) * (int32_t)v[qb_ell_col(w.w)];
    }
    int32_t *h = H + (int64_t)p * n + i;
    *h = ACC ? *h + acc : acc;
}

}  // namespace

qb_status qb_field_ell_launch(qb_problem P, int z, const uint8_t *X, int32_t *H, hipStream_t s)
{
    dim3 grid((P->n + 255) / 256, z);
    k_ell_spmm<uint8_t, false><<<grid, 256, 0, s>>>(P->ell, P->ecnt, P->diag, P->n, P->ellw, X, H);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

qb_status qb_rankk_mfma_launch(qb_problem P, int z, const int8_t *dX, int32_t *H, hipStream_t s)
{
    const int n = P->n;
    const int gx = (n + 127) / 128, gy = (z + 63) / 64;
    const int nk = (n + 63) / 64;
    int split = (512 + gx * gy - 1) / (gx * gy);
    split = split < 1 ? 1 : split > nk ? nk : split;
    const int kchunk = 64 * ((nk + split - 1) / split);
    split = (nk * 64 + kchunk - 1) / kchunk;
    dim3 grid(gx, gy, split);
    const int8_t *Qp = (const int8_t *)P->Qp;
    if (n % 16 == 0)
        k_rankk_mfma<16><<<grid, 256, 0, s>>>(dX, n, z, Qp, P->ldp, H, kchunk);
    else if (n % 8 == 0)
        k_rankk_mfma<8><<<grid, 256, 0, s>>>(dX, n, z, Qp, P->ldp, H, kchunk);
    else if (n % 4 == 0)
        k_rankk_mfma<4><<<grid, 256, 0, s>>>(dX, n, z, Qp, P->ldp, H, kchunk);
    else
        k_rankk_mfma<1><<<grid, 256, 0, s>>>(dX, n, z, Qp, P->ldp, H, kchunk);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

extern "C" qb_status qb_rankk(qb_problem P, int32_t z, const int8_t *dX_d, int32_t *H_d, int32_t variant,
                             void *stream)
{
    if (!P || z < 1 || z > 65535 || !dX_d || !H_d || variant < 0 || variant > 3) return QB_E_ARG;
    hipStream_t s = qb_stream(stream);
    if (P->sparse) {
        if (variant != 0 && variant != 3) return QB_E_UNSUPPORTED;
        dim3 g((P->n + 255) / 256, z);
        k_ell_spmm<int8_t, true><<<g, 256, 0, s>>>(P->ell, P->ecnt, P->diag, P->n, P->ellw, dX_d, H_d);
        QB_LAUNCH_CHECK();
        return QB_OK;
    }
    if (variant == 3 || (variant == 2 && !P->int8_ok)) return QB_E_UNSUPPORTED;
    constexpr int CPT = 4;
    dim3 grid((P->n + 256 * CPT - 1) / (256 * CPT), z);
    if (variant == 0) variant = (P->int8_ok && P->Qp && z >= 32) ? 2 : 1;
    if (variant == 2) {
        if (!P->Qp) return QB_E_UNSUPPORTED;
        return qb_rankk_mfma_launch(P, z, dX_d, H_d, s);
    }
    if (P->int8_ok)
        k_rankk_valu<int8_t, CPT><<<grid, 256, 0, s>>>(P->Q8, P->n, dX_d, H_d);
    else
        k_rankk_valu<int16_t, CPT><<<grid, 256, 0, s>>>(P->Q, P->n, dX_d, H_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}
