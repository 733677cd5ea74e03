// Learned sub-QUBO selection: per-variable features, a BF16 MLP scorer with
// bit-reproducible inference, improvement traces, and the training step.
//
// Inference sums every layer in index order in FP32 starting from the bias,
// on operands that are BF16 values; the product of two BF16 values is exact
// in FP32, so the result does not depend on whether a multiply-add is fused,
// and the host reference reproduces it bit for bit.  Hidden activations are
// rounded to BF16 (round to nearest even).  The score is mapped to an
// order-preserving int64 key so that the plain path's rank and selection
// kernels serve the learned path unchanged.
#include <math.h>

#include <mutex>

#include "qb_internal.h"

namespace {

constexpr int NPARAM = 4801;
constexpr int OW1 = 0, OB1 = 512, OW2 = 576, OB2 = 4672, OW3 = 4736, OB3 = 4800;

__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ------------------------------------------------------------------ features
__global__ void __launch_bounds__(256) k_features(int n, int z, const int32_t *__restrict__ diag,
                                                  const int64_t *__restrict__ eta, const int32_t *__restrict__ cnt,
                                                  const int32_t *__restrict__ H, const int32_t *__restrict__ T,
                                                  const int32_t *__restrict__ LF, const int32_t *__restrict__ G,
                                                  int alpha, float s0, float s1, float s2, float s3, float s4,
                                                  float s5, float s6, uint16_t *__restrict__ F)
{
    __shared__ int32_t part[4];
    const int p = blockIdx.x;
    const int64_t ro = (int64_t)p * n;
    int32_t tm = 1;
    for (int j = threadIdx.x; j < n; j += 256) tm = max(tm, T[ro + j]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tm = max(tm, __shfl_xor(tm, o, 64));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = tm;
    __syncthreads();
    const int32_t Tp = max(max(part[0], part[1]), max(part[2], part[3]));
    for (int j = threadIdx.x; j < n; j += 256) {
        const int64_t at = ro + j;
        const int32_t dev = abs(2 * cnt[j] - z);
        const int32_t age = LF[at] > 0 ? alpha - LF[at] : alpha;
        float f[8];
        f[0] = (float)H[at] * s0;
        f[1] = (float)diag[j] * s1;
        f[2] = (float)T[at] * s2;
        f[3] = (float)age * s3;
        f[4] = (float)G[at] * s4;
        f[5] = (float)eta[j] * s5;
        f[6] = (float)(z - dev) * s6;
        f[7] = (float)(Tp - T[at]) / (float)Tp;
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = (uint32_t)bf16_rne(f[2 * k]) | ((uint32_t)bf16_rne(f[2 * k + 1]) << 16);
        *reinterpret_cast<uint4 *>(F + at * 8) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// ------------------------------------------------------------------ inference
__device__ __forceinline__ float mlp_forward(const uint16_t *__restrict__ W, const float (&x)[8])
{
    float h1[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) {
        float acc = bf16_f(W[OB1 + k]);
#pragma unroll
        for (int i = 0; i < 8; ++i) acc = acc + bf16_f(W[OW1 + k * 8 + i]) * x[i];
        h1[k] = bf16_f(bf16_rne(acc > 0.0f ? acc : 0.0f));
    }
    float s = bf16_f(W[OB3]);
    for (int k = 0; k < 64; ++k) {
        float acc = bf16_f(W[OB2 + k]);
#pragma unroll
        for (int i = 0; i < 64; ++i) acc = acc + bf16_f(W[OW2 + k * 64 + i]) * h1[i];
        s = s + bf16_f(W[OW3 + k]) * bf16_f(bf16_rne(acc > 0.0f ? acc : 0.0f));
    }
    return s;
}

__global__ void __launch_bounds__(256) k_mlp_score(int64_t count, const uint16_t *__restrict__ F,
                                                   const uint16_t *__restrict__ W, float *__restrict__ score,
                                                   int64_t *__restrict__ K)
{
    const int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (e >= count) return;
    const uint4 v = *reinterpret_cast<const uint4 *>(F + e * 8);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    float x[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        x[2 * k] = bf16_f((uint16_t)(w[k] & 0xffffu));
        x[2 * k + 1] = bf16_f((uint16_t)(w[k] >> 16));
    }
    float s = mlp_forward(W, x);
    if (s == 0.0f) s = 0.0f;   // one key for -0 and +0
    if (score) score[e] = s;
    const uint32_t u = __float_as_uint(s);
    const uint32_t key = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    K[e] = (int64_t)key - 2147483648LL;
}

// ------------------------------------------------------------------ traces
// Sample of (p, S_a) of job q: its features and the label "changed by the
// chosen replica of a job that lowered the sub-QUBO energy".
__global__ void __launch_bounds__(256) k_trace(int n, int R, const int32_t *__restrict__ sol,
                                               const int32_t *__restrict__ off, const int32_t *__restrict__ idx,
                                               const uint16_t *__restrict__ F, const uint8_t *__restrict__ Y,
                                               const int64_t *__restrict__ e, const uint8_t *__restrict__ y0,
                                               uint16_t *__restrict__ outF, uint8_t *__restrict__ outL,
                                               const qb_iter *__restrict__ it, int64_t cap, int total)
{
    const int q = blockIdx.x;
    const int base = off[q], m = off[q + 1] - base, p = sol[q];
    if (it) {
        // appended after the rows already written, only while the ring has room
        const int64_t at = it->trn;
        if (at + total > cap) return;
        outF += at * 8;
        outL += at;
    }
    bool failed;
    const int rb = qb_best_replica(e + (size_t)q * R, R, &failed);
    // a job without a finished replica gives no gain (and its Y is not read)
    const bool gain = rb >= 0 && e[(size_t)q * R + rb] < 0;
    const uint8_t *Yr = Y + (size_t)base * R + (size_t)(rb < 0 ? 0 : rb) * m;
    for (int a = threadIdx.x; a < m; a += 256) {
        const int j = idx[base + a];
        *reinterpret_cast<uint4 *>(outF + (int64_t)(base + a) * 8) =
            *reinterpret_cast<const uint4 *>(F + ((int64_t)p * n + j) * 8);
        outL[base + a] = (uint8_t)(gain && Yr[a] != y0[base + a]);
    }
}

// G[p][j] = gain (-e, saturated to int32) of the chosen replica, for every
// variable that job changed.
__global__ void __launch_bounds__(256) k_gain(int n, int R, const int32_t *__restrict__ sol,
                                              const int32_t *__restrict__ off, const int32_t *__restrict__ idx,
                                              const uint8_t *__restrict__ Y, const int64_t *__restrict__ e,
                                              const uint8_t *__restrict__ y0, int32_t *__restrict__ G)
{
    const int q = blockIdx.x;
    const int base = off[q], m = off[q + 1] - base, p = sol[q];
    bool failed;
    const int rb = qb_best_replica(e + (size_t)q * R, R, &failed);
    if (rb < 0) return;                       // no finished replica: nothing changed
    const int64_t g = -e[(size_t)q * R + rb];
    const int32_t gs = (int32_t)max(min(g, (int64_t)INT32_MAX), (int64_t)INT32_MIN);
    const uint8_t *Yr = Y + (size_t)base * R + (size_t)rb * m;
    for (int a = threadIdx.x; a < m; a += 256)
        if (Yr[a] != y0[base + a]) G[(int64_t)p * n + idx[base + a]] = gs;
}

// ------------------------------------------------------------------ training
// Forward and backward of 64 samples per workgroup (one wave).  The three
// 64x64x64 products -- the second layer's forward pass Z2 = H1 W2^T, the
// backward pass dH1 = dZ2 W2 and the weight gradient dW2 = dZ2^T H1 -- run
// on the matrix cores (v_mfma_f32_16x16x16_bf16: BF16 operands, FP32
// accumulation).  H1 and W2 are BF16 already; the FP32 dZ2 enters as a pair
// of BF16 numbers hi + lo (hi = BF16(dZ2), lo = BF16(dZ2 - hi), 16 bits of
// mantissa together), each product taking hi and then lo into the same
// accumulator.  The first layer, the output layer, the biases and the loss
// stay on FP32 VALU, sample by sample in index order.  Each workgroup's gradient lands in its own row of `partial`
// (deterministic: the matrix cores' summation order is fixed).
//
// Operand layouts of the 16x16x16 product, lane l = 16 g + r (g < 4):
// A[row r][k 4g .. 4g+3], B[k 4g .. 4g+3][column r], and the result
// D[rows 4g .. 4g+3][column r]; every operand is read as 4 consecutive BF16
// (8 bytes) from an LDS array laid out along k.
typedef short mlp_v4s __attribute__((ext_vector_type(4)));
typedef float mlp_v4f __attribute__((ext_vector_type(4)));

constexpr int MP64 = 68;   // row pitch (BF16) of the 64 x 64 LDS operands: 8-byte aligned, banks spread

__device__ __forceinline__ mlp_v4s mlp_ld4(const uint16_t *row, int k)
{
    return *reinterpret_cast<const mlp_v4s *>(row + k);
}

__global__ void __launch_bounds__(64) k_mlp_grad(int B, const uint16_t *__restrict__ feat,
                                                 const uint8_t *__restrict__ label,
                                                 const uint16_t *__restrict__ W, float *__restrict__ partial,
                                                 float *__restrict__ lossp)
{
    __shared__ float xs[64][8], dss[64], ls[64];
    __shared__ uint64_t m1s[64];
    __shared__ __align__(16) uint16_t w2b[64][MP64], w2t[64][MP64];   // W2[k][i], W2^T[i][k]
    __shared__ __align__(16) uint16_t h1b[64][MP64], h1t[64][MP64];   // H1[s][i], H1^T[i][s]
    __shared__ __align__(16) uint16_t z2b[64][MP64], z2t[64][MP64];   // hi of dZ2[s][k], of dZ2^T[k][s]
    __shared__ __align__(16) uint16_t z2l[64][MP64], z2tl[64][MP64];  // lo of the same
    __shared__ float h2f[64][65], dz2f[64][65], dz1f[64][65];
    const int t = threadIdx.x;
    const int b = blockIdx.x * 64 + t;
    const bool ok = b < B;
    const int r16 = t & 15, g = t >> 4;

    for (int e = t; e < 64 * 64; e += 64) {
        const uint16_t w = W[OW2 + e];
        w2b[e >> 6][e & 63] = w;
        w2t[e & 63][e >> 6] = w;
    }
    float x[8];
    if (ok) {
        const uint4 v = *reinterpret_cast<const uint4 *>(feat + (int64_t)b * 8);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[2 * k] = bf16_f((uint16_t)(w[k] & 0xffffu));
            x[2 * k + 1] = bf16_f((uint16_t)(w[k] >> 16));
        }
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = 0.0f;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) xs[t][i] = x[i];
    // first layer, as in inference (thread = sample)
    uint64_t m1 = 0;
#pragma unroll
    for (int k = 0; k < 64; ++k) {
        float acc = bf16_f(W[OB1 + k]);
#pragma unroll
        for (int i = 0; i < 8; ++i) acc = acc + bf16_f(W[OW1 + k * 8 + i]) * x[i];
        m1 |= (uint64_t)(acc > 0.0f) << k;
        const uint16_t hb = bf16_rne(acc > 0.0f ? acc : 0.0f);
        h1b[t][k] = hb;
        h1t[k][t] = hb;
    }
    m1s[t] = m1;
    __syncthreads();

    // second layer on the matrix cores: Z2[s][k] = b2[k] + sum_i H1[s][i] W2[k][i];
    // h2 = BF16(relu(Z2)), stored as -0 where Z2 <= 0 (the ReLU mask)
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
            const float bias = bf16_f(W[OB2 + 16 * ni + r16]);
            mlp_v4f acc = {bias, bias, bias, bias};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(mlp_ld4(h1b[16 * mi + r16], 16 * ks + 4 * g),
                                                                mlp_ld4(w2b[16 * ni + r16], 16 * ks + 4 * g), acc,
                                                                0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float z = acc[r];
                h2f[16 * mi + 4 * g + r][16 * ni + r16] = z > 0.0f ? bf16_f(bf16_rne(z)) : -0.0f;
            }
        }
    __syncthreads();

    // output layer, loss and dZ2 (thread = sample)
    {
        float sc = bf16_f(W[OB3]);
        for (int k = 0; k < 64; ++k) sc = sc + bf16_f(W[OW3 + k]) * h2f[t][k];
        const float y = ok && label[b] ? 1.0f : 0.0f;
        const float ds = ok ? (1.0f / (1.0f + expf(-sc)) - y) / (float)B : 0.0f;
        ls[t] = ok ? ((sc > 0.0f ? sc + log1pf(expf(-sc)) : log1pf(expf(sc))) - y * sc) : 0.0f;
        dss[t] = ds;
        for (int k = 0; k < 64; ++k) {
            const float dz2 = __builtin_signbit(h2f[t][k]) ? 0.0f : ds * bf16_f(W[OW3 + k]);
            dz2f[t][k] = dz2;
            const uint16_t hi = bf16_rne(dz2);
            const uint16_t lo = bf16_rne(dz2 - bf16_f(hi));
            z2b[t][k] = hi;
            z2t[k][t] = hi;
            z2l[t][k] = lo;
            z2tl[k][t] = lo;
        }
    }
    __syncthreads();

    // backward into the first layer on the matrix cores:
    // dH1[s][i] = sum_k dZ2[s][k] W2[k][i], dZ1 = dH1 where the first layer was positive
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
            mlp_v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const mlp_v4s bw = mlp_ld4(w2t[16 * ni + r16], 16 * ks + 4 * g);
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(mlp_ld4(z2b[16 * mi + r16], 16 * ks + 4 * g), bw,
                                                                acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(mlp_ld4(z2l[16 * mi + r16], 16 * ks + 4 * g), bw,
                                                                acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int sr = 16 * mi + 4 * g + r, ic = 16 * ni + r16;
                dz1f[sr][ic] = ((m1s[sr] >> ic) & 1ull) ? acc[r] : 0.0f;
            }
        }

    float *out = partial + (int64_t)blockIdx.x * NPARAM;
    // dW2[k][i] = sum_s dZ2[s][k] H1[s][i] on the matrix cores
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
            mlp_v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const mlp_v4s bh = mlp_ld4(h1t[16 * ni + r16], 16 * ks + 4 * g);
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(mlp_ld4(z2t[16 * mi + r16], 16 * ks + 4 * g), bh,
                                                                acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(mlp_ld4(z2tl[16 * mi + r16], 16 * ks + 4 * g), bh,
                                                                acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) out[OW2 + (16 * mi + 4 * g + r) * 64 + 16 * ni + r16] = acc[r];
        }
    __syncthreads();

    // the small sums on VALU, over the samples in index order (thread = unit)
    {
        float gb2 = 0.0f, gb1 = 0.0f, gw3 = 0.0f, g1[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int bb = 0; bb < 64; ++bb) {
            const float d1 = dz1f[bb][t];
#pragma unroll
            for (int i = 0; i < 8; ++i) g1[i] = g1[i] + d1 * xs[bb][i];
            gb2 = gb2 + dz2f[bb][t];
            gb1 = gb1 + d1;
            gw3 = gw3 + dss[bb] * h2f[bb][t];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) out[OW1 + t * 8 + i] = g1[i];
        out[OB2 + t] = gb2;
        out[OB1 + t] = gb1;
        out[OW3 + t] = gw3;
    }
    if (t == 0) {
        float gb3 = 0.0f, l = 0.0f;
        for (int bb = 0; bb < 64; ++bb) {
            gb3 = gb3 + dss[bb];
            l = l + ls[bb];
        }
        out[OB3] = gb3;
        lossp[blockIdx.x] = l;
    }
}

__global__ void k_mlp_reduce(int nblk, const float *__restrict__ partial, const float *__restrict__ lossp, int B,
                             float *__restrict__ grad, float *__restrict__ loss)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < NPARAM) {
        float g = 0.0f;
        for (int w = 0; w < nblk; ++w) g = g + partial[(int64_t)w * NPARAM + k];
        grad[k] = g;
    }
    if (k == 0 && loss) {
        float l = 0.0f;
        for (int w = 0; w < nblk; ++w) l = l + lossp[w];
        *loss = l / (float)B;
    }
}

// Initial parameters: weights uniform on [-a, a) per layer from Philox
// words (parameter k: word k mod 4 at counter (k/4, 0, 0, 5<<28)), the
// 24-bit draw r = (u >> 8) 2^-24 scaled as (2r - 1) a in one FP32 rounding;
// biases zero; W = BF16(master).
__global__ void k_mlp_init(uint32_t s0, uint32_t s1, float a1, float a2, float a3, float *__restrict__ master,
                           uint16_t *__restrict__ Wbf)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NPARAM) return;
    const float a = k < OB1 ? a1 : (k >= OW2 && k < OB2) ? a2 : (k >= OW3 && k < OB3) ? a3 : 0.0f;
    float w = 0.0f;
    if (a != 0.0f) {
        const uint4 r = qb_philox(make_uint4((uint32_t)k >> 2, 0u, 0u, 5u << 28), s0, s1);
        const uint32_t u = (k & 3) == 0 ? r.x : (k & 3) == 1 ? r.y : (k & 3) == 2 ? r.z : r.w;
        const float c = 2.0f * ((float)(u >> 8) * (1.0f / 16777216.0f)) - 1.0f;
        w = c * a;
    }
    master[k] = w;
    Wbf[k] = bf16_rne(w);
}

__global__ void k_adam(const float *__restrict__ grad, float *__restrict__ master, float *__restrict__ m,
                       float *__restrict__ v, float lr, float beta1, float beta2, float eps, float c1, float c2,
                       uint16_t *__restrict__ Wbf)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NPARAM) return;
    const float g = grad[k];
    m[k] = beta1 * m[k] + (1.0f - beta1) * g;
    v[k] = beta2 * v[k] + (1.0f - beta2) * g * g;
    const float mh = m[k] / c1, vh = v[k] / c2;
    master[k] = master[k] - lr * mh / (sqrtf(vh) + eps);
    Wbf[k] = bf16_rne(master[k]);
}

}  // namespace

extern "C" qb_status qb_features(qb_problem P, int32_t z, const uint8_t *X_d, const int32_t *H_d, const int32_t *T_d,
                                const int32_t *LF_d, const int32_t *G_d, int32_t alpha, const float *scales_h,
                                uint16_t *F_d, void *stream)
{
    if (!P || z < 1 || !X_d || !H_d || !T_d || !LF_d || !G_d || !scales_h || !F_d || alpha < 0) return QB_E_ARG;
    if ((uintptr_t)F_d & 15) return QB_E_ARG;
    hipStream_t s = qb_stream(stream);
    qb_status rc = qb_column_counts(P, z, X_d, stream);
    if (rc != QB_OK) return rc;
    k_features<<<z, 256, 0, s>>>(P->n, z, P->diag, P->eta, P->colcnt, H_d, T_d, LF_d, G_d, alpha, scales_h[0],
                                 scales_h[1], scales_h[2], scales_h[3], scales_h[4], scales_h[5], scales_h[6], F_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

extern "C" qb_status qb_mlp_score(int64_t count, const uint16_t *F_d, const uint16_t *W_d, float *score_d,
                                 int64_t *K_d, void *stream)
{
    if (count < 1 || !F_d || !W_d || !K_d) return QB_E_ARG;
    if ((uintptr_t)F_d & 15) return QB_E_ARG;
    k_mlp_score<<<(unsigned)((count + 255) / 256), 256, 0, qb_stream(stream)>>>(count, F_d, W_d, score_d, K_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

qb_status qb_trace_x(qb_batch b, int32_t R, const uint16_t *F_d, const uint8_t *Y_d, const int64_t *e_d,
                     const uint8_t *y0_d, uint16_t *outF_d, uint8_t *outL_d, const qb_iter *it, int64_t cap,
                     void *stream)
{
    if (!b || R < 1 || R > 16 || !F_d || !Y_d || !e_d || !y0_d || !outF_d || !outL_d) return QB_E_ARG;
    if (((uintptr_t)F_d & 15) || ((uintptr_t)outF_d & 15)) return QB_E_ARG;
    if (b->J == 0) return QB_OK;
    k_trace<<<b->J, 256, 0, qb_stream(stream)>>>(b->n, R, b->sol_d, b->off_d, b->idx_d, F_d, Y_d, e_d, y0_d, outF_d,
                                                 outL_d, it, cap, b->total);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

extern "C" qb_status qb_trace(qb_batch b, int32_t R, const uint16_t *F_d, const uint8_t *Y_d, const int64_t *e_d,
                             const uint8_t *y0_d, uint16_t *outF_d, uint8_t *outL_d, void *stream)
{
    return qb_trace_x(b, R, F_d, Y_d, e_d, y0_d, outF_d, outL_d, nullptr, 0, stream);
}

extern "C" qb_status qb_gain_update(qb_batch b, int32_t R, const uint8_t *Y_d, const int64_t *e_d,
                                   const uint8_t *y0_d, int32_t *G_d, void *stream)
{
    if (!b || R < 1 || R > 16 || !Y_d || !e_d || !y0_d || !G_d) return QB_E_ARG;
    if (b->J == 0) return QB_OK;
    k_gain<<<b->J, 256, 0, qb_stream(stream)>>>(b->n, R, b->sol_d, b->off_d, b->idx_d, Y_d, e_d, y0_d, G_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

extern "C" size_t qb_mlp_train_workspace(int32_t B)
{
    const size_t nblk = (size_t)(B + 63) / 64;
    return sizeof(float) * (nblk * NPARAM + nblk);
}

extern "C" qb_status qb_mlp_grad(int32_t B, const uint16_t *feat_d, const uint8_t *label_d, const uint16_t *W_d,
                                float *grad_d, float *loss_d, void *work_d, void *stream)
{
    if (B < 1 || !feat_d || !label_d || !W_d || !grad_d || !work_d) return QB_E_ARG;
    if ((uintptr_t)feat_d & 15) return QB_E_ARG;
    hipStream_t s = qb_stream(stream);
    const int nblk = (B + 63) / 64;
    float *partial = (float *)work_d;
    float *lossp = partial + (size_t)nblk * NPARAM;
    k_mlp_grad<<<nblk, 64, 0, s>>>(B, feat_d, label_d, W_d, partial, lossp);
    k_mlp_reduce<<<(NPARAM + 255) / 256, 256, 0, s>>>(nblk, partial, lossp, B, grad_d, loss_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

// ------------------------------------------------------------------ no allocation
// qb_mlp_grad for callers that cannot allocate (graph capture, tight training
// loops): the per-workgroup partial sums live in this file-scope device array
// instead of a caller workspace.  In host code `scratch` names a host-side
// stand-in, never the device memory: its device address is taken once per
// device with hipGetSymbolAddress and only that address is passed to the
// kernels.  k_mlp_grad writes every entry of the rows it uses, so nothing is
// cleared between calls; calls that overlap on one GPU share the array and
// race.
constexpr int NOALLOC_MAX_B = QB_MLP_GRAD_NOALLOC_MAX_B;
constexpr size_t NOALLOC_FLOATS = (size_t)((NOALLOC_MAX_B + 63) / 64) * (NPARAM + 1);
static __device__ __align__(256) float scratch[NOALLOC_FLOATS];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static float *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {nullptr};

// the device address of `scratch` on the current device (set up on the first
// call there)
static qb_status scratch_address(float **out)
{
    int dev = -1;
    QB_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return QB_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        QB_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return QB_E_HIP;
        g_scratch_ptr[dev] = (float *)p;
    }
    *out = g_scratch_ptr[dev];
    return QB_OK;
}

extern "C" qb_status qb_mlp_grad_noalloc(int32_t B, const uint16_t *feat_d, const uint8_t *label_d,
                                        const uint16_t *W_d, float *grad_d, float *loss_d, void *stream)
{
    if (B < 1 || !feat_d || !label_d || !W_d || !grad_d) return QB_E_ARG;
    if ((uintptr_t)feat_d & 15) return QB_E_ARG;
    if (B > NOALLOC_MAX_B) return QB_E_CAPACITY;
    float *partial = nullptr;
    const qb_status rc = scratch_address(&partial);
    if (rc != QB_OK) return rc;
    hipStream_t s = qb_stream(stream);
    const int nblk = (B + 63) / 64;
    float *lossp = partial + (size_t)nblk * NPARAM;
    k_mlp_grad<<<nblk, 64, 0, s>>>(B, feat_d, label_d, W_d, partial, lossp);
    k_mlp_reduce<<<(NPARAM + 255) / 256, 256, 0, s>>>(nblk, partial, lossp, B, grad_d, loss_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

extern "C" qb_status qb_mlp_init(uint64_t seed, float a1, float a2, float a3, float *master_d, uint16_t *W_d,
                                 void *stream)
{
    if (!master_d || !W_d) return QB_E_ARG;
    k_mlp_init<<<(NPARAM + 255) / 256, 256, 0, qb_stream(stream)>>>((uint32_t)seed, (uint32_t)(seed >> 32), a1, a2,
                                                                     a3, master_d, W_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

extern "C" qb_status qb_mlp_adam(const float *grad_d, float *master_d, float *m_d, float *v_d, int32_t step, float lr,
                                float beta1, float beta2, float eps, uint16_t *W_d, void *stream)
{
    if (!grad_d || !master_d || !m_d || !v_d || !W_d || step < 1) return QB_E_ARG;
    const float c1 = 1.0f - powf(beta1, (float)step);
    const float c2 = 1.0f - powf(beta2, (float)step);
    k_adam<<<(NPARAM + 255) / 256, 256, 0, qb_stream(stream)>>>(grad_d, master_d, m_d, v_d, lr, beta1, beta2, eps, c1,
                                                                c2, W_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}
