// Tabu search (Alg. 1 of the IC-D^2S paper) on a sparse problem with the
// move values in a min-tree in LDS: one wave per solution.
//
// A step of Alg. 1 flips the allowed variable of least move value, and the
// flip changes only a handful of move values: the flipped variable's own
// (negated), its neighbours' (the O(degree) update of the Tabu section) and
// the tabu state of the variable whose tenure runs out.  So instead of an
// argmin over all n values per step, the kernel keeps the move values in
// LDS under one level of 64-leaf nodes and repairs only the nodes a step
// touches.
//
// Layout per solution (one 64-lane workgroup, all state in LDS):
//   dl[j]  move value D_j + bias (uint16; bias bounds |D|),
//   Ul[j]  the last step at which j is tabu (0: free),
//   xw, pw bit vectors of x and of "flipped since the last improvement",
//   per node q (leaves 64q .. 64q+63): the least key over its free leaves,
//   the least key over its tabu leaves and the least Ul over its tabu
//   leaves (the step after which one of them becomes free).
// A key is (D_j + bias) << IB | j, so the unsigned minimum is the least move
// value, then the lowest index, exactly the oracle's tie rule.
//
// Step t: the wave reads every node (a few per lane) and takes the two
// minima; the smallest tabu key is allowed when it reaches OV + D < OV_min
// (aspiration), and when nothing is free and nothing aspirates it wins
// anyway (the argmin over all).  The winner's ELL row is requested from
// memory at once; while it is in flight the wave rewrites the winner's leaf
// and recomputes its node and every node whose least tabu step has passed.
// Then each lane with a neighbour c updates D_c in place: a key that fell
// only needs an LDS atomic minimum on its node, a key that rose is a repair
// only when it was its node's minimum.  Every node is exact for step t+1
// when the step ends.
#include "qb_internal.h"

namespace {

constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr int TT_MAX_NR = 8;   // nodes per lane: n <= 64 * 64 * 8

// Wave minimum left in lane 63 (the row minima by quad and mirror moves,
// then the row broadcasts); the other lanes hold partial minima.
__device__ __forceinline__ uint32_t min_to63(uint32_t v)
{
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x142, 0xA, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x143, 0xC, 0xF, false));
    return v;
}

// Two wave minima at once (the steps interleaved), returned uniform.
__device__ __forceinline__ void min2_uniform(uint32_t &a, uint32_t &b)
{
#define TT_STEP(CTL, RM, ID)                                                                     \
    a = min(a, (uint32_t)__builtin_amdgcn_update_dpp((ID), (int)a, CTL, RM, 0xF, false));       \
    b = min(b, (uint32_t)__builtin_amdgcn_update_dpp((ID), (int)b, CTL, RM, 0xF, false));
    TT_STEP(0xB1, 0xF, 0)
    TT_STEP(0x4E, 0xF, 0)
    TT_STEP(0x141, 0xF, 0)
    TT_STEP(0x140, 0xF, 0)
    TT_STEP(0x142, 0xA, -1)
    TT_STEP(0x143, 0xC, -1)
#undef TT_STEP
    a = (uint32_t)__builtin_amdgcn_readlane((int)a, 63);
    b = (uint32_t)__builtin_amdgcn_readlane((int)b, 63);
}

struct TreeLds {
    int32_t *Ul;
    uint2 *nd;       // (least free key, least tabu key) per node, NR * 64 slots
    uint32_t *ne;    // least Ul over the node's tabu leaves, NR * 64 slots
    uint32_t *xw;
    uint32_t *pw;
    uint16_t *dl;
};

// Slots past the last node hold empty nodes, so every lane reads its NR
// slots unconditionally.
__device__ __forceinline__ TreeLds tree_lds(uint32_t *sm, int NN, int NR)
{
    const int NP = NN << 6, NXW = NP >> 5;
    TreeLds L;
    L.Ul = (int32_t *)sm;
    L.nd = (uint2 *)(sm + NP);
    L.ne = sm + NP + 2 * 64 * NR;
    L.xw = L.ne + 64 * NR;
    L.pw = L.xw + NXW;
    L.dl = (uint16_t *)(L.pw + NXW);
    return L;
}

// Node q from its leaves, tabu meaning "Ul > t" (the state at step t + 1).
__device__ __forceinline__ void recompute(const TreeLds &L, int q, int t, int n, int IB, int lane)
{
    const int j = (q << 6) + lane;
    const uint32_t d = L.dl[j];
    const int32_t u = L.Ul[j];
    uint32_t f = NONE, g = NONE, e = NONE;
    if (j < n) {
        const uint32_t key = (d << IB) | (uint32_t)j;
        if (u > t) {
            g = key;
            e = (uint32_t)u;
        } else {
            f = key;
        }
    }
    f = min_to63(f);
    g = min_to63(g);
    e = min_to63(e);
    if (lane == 63) {
        L.nd[q] = make_uint2(f, g);
        L.ne[q] = e;
    }
}

template <int NR>
__global__ void __launch_bounds__(64) k_tabu_tree(const uint32_t *__restrict__ ell, int W,
                                                  const int32_t *__restrict__ diag, int n,
                                                  uint8_t *__restrict__ X, int32_t *__restrict__ H,
                                                  int64_t *__restrict__ E, int alpha, int tenure, int asp,
                                                  int32_t *__restrict__ Tout, int32_t *__restrict__ LFout,
                                                  uint32_t bias, int IB)
{
    extern __shared__ __align__(16) uint32_t sm[];
    const int p = blockIdx.x, lane = threadIdx.x;
    const int NN = (n + 63) >> 6, NP = NN << 6, NXW = NP >> 5;
    const TreeLds L = tree_lds(sm, NN, NR);
    const int64_t ro = (int64_t)p * n;
    const uint32_t IMASK = (1u << IB) - 1u;

    // leaves from x and the field: D_j = Q_jj + 2(1 - 2x_j) h_j
    for (int j0 = 0; j0 < NP; j0 += 64) {
        const int j = j0 + lane;
        uint32_t x = 0, dv = 0;
        if (j < n) {
            Tout[ro + j] = 0;
            LFout[ro + j] = 0;
            x = X[ro + j] & 1u;
            dv = (uint32_t)(diag[j] + (x ? -2 : 2) * H[ro + j] + (int32_t)bias);
        }
        L.dl[j] = (uint16_t)dv;
        L.Ul[j] = 0;
        const uint64_t bx = __ballot(x != 0u);
        if (lane < 2) {
            L.xw[(j0 >> 5) + lane] = lane ? (uint32_t)(bx >> 32) : (uint32_t)bx;
            L.pw[(j0 >> 5) + lane] = 0u;
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        L.nd[lane + 64 * r] = make_uint2(NONE, NONE);
        L.ne[lane + 64 * r] = NONE;
    }
    __syncthreads();
    for (int q = 0; q < NN; ++q) recompute(L, q, 0, n, IB, lane);
    __syncthreads();

    int64_t OV = E[p];
    int64_t gap = 0;   // OV - OV_min, never negative

    for (int step = 1; step <= alpha; ++step) {
        // the least free key and the least tabu key over all nodes
        uint32_t fm = NONE, tm = NONE;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const uint2 v = L.nd[lane + 64 * r];
            fm = min(fm, v.x);
            tm = min(tm, v.y);
        }
        min2_uniform(fm, tm);
        // a tabu key aspirates when D < OV_min - OV = -gap
        uint32_t tbk = 0;
        if (asp && gap < (int64_t)bias) tbk = (bias - (uint32_t)gap) << IB;
        uint32_t best = fm;
        if (tm < tbk) best = min(best, tm);
        if (best == NONE) best = tm;   // everything tabu and nothing aspirates
        const int i = (int)(best & IMASK);
        const uint32_t dib = best >> IB;

        // the winner's row, in flight while its own leaf and node are redone
        uint32_t wd = 0u;
        if (lane < W) wd = ell[(int64_t)i * W + lane];

        const uint32_t xword = L.xw[i >> 5];
        const int32_t Ui = L.Ul[i];
        const uint32_t bit = 1u << (i & 31);
        const int32_t s = (xword & bit) ? -1 : 1;   // h_j += s Q_ji
        const int32_t Un = step + max(max(Ui - (step - 1), 0) + tenure - 1, 0);
        const int32_t dmove = (int32_t)dib - (int32_t)bias;
        OV += dmove;
        gap += dmove;
        const bool improved = gap < 0;
        if (improved) gap = 0;
        if (lane == 0) {
            L.Ul[i] = Un;
            L.dl[i] = (uint16_t)(2u * bias - dib);   // D_i -> -D_i
            L.xw[i >> 5] = xword ^ bit;
            if (!improved) __hip_atomic_fetch_xor(L.pw + (i >> 5), bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if (improved)   // x_min is the current x
            for (int w = lane; w < NXW; w += 64) L.pw[w] = 0u;

        recompute(L, i >> 6, step, n, IB, lane);
        // nodes with a tabu leaf that is free at step + 1
        uint32_t nev[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) nev[r] = L.ne[lane + 64 * r];
        uint64_t exm[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) exm[r] = __ballot(nev[r] <= (uint32_t)step);
#pragma unroll
        for (int r = 0; r < NR; ++r)
            for (uint64_t m = exm[r]; m; m &= m - 1) recompute(L, __builtin_ctzll(m) + 64 * r, step, n, IB, lane);

        // neighbours: D_c += 2(1 - 2x_c) s Q_ci
        bool need = false;
        int cq = 0;
        if (wd != 0u) {
            const int c = qb_ell_col(wd);
            const int32_t v = qb_ell_val(wd);
            cq = c >> 6;
            const uint32_t xcw = L.xw[c >> 5];
            const uint32_t dold = L.dl[c];
            const int32_t uc = L.Ul[c];
            const uint2 nq = L.nd[cq];
            const int32_t sg = ((xcw >> (c & 31)) & 1u) ? -2 : 2;
            const uint32_t dnew = (uint32_t)((int32_t)dold + sg * s * v);
            L.dl[c] = (uint16_t)dnew;
            const uint32_t kold = (dold << IB) | (uint32_t)c, knew = (dnew << IB) | (uint32_t)c;
            const bool tb = uc > step;
            if (knew < kold) {
                __hip_atomic_fetch_min(tb ? &L.nd[cq].y : &L.nd[cq].x, knew, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            } else {
                need = knew > kold && (tb ? nq.y : nq.x) == kold;
            }
        }
        for (uint64_t m = __ballot(need); m;) {
            const int q = __builtin_amdgcn_readlane(cq, __builtin_ctzll(m));
            recompute(L, q, step, n, IB, lane);
            m &= ~__ballot(need && cq == q);
        }
        // the flip count and last-flip step go out after the row has been
        // waited for, so that wait never covers them
        if (lane == 0) {
            __hip_atomic_fetch_add(Tout + ro + i, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            LFout[ro + i] = step;
        }
    }
    __syncthreads();

    // field of the final x from D (h_j = (D_j - Q_jj) / (2(1 - 2x_j))), kept
    // in Ul, then moved to x_min = x ^ pw by the rows of the differing
    // variables (their own diagonal term and their neighbours)
    for (int j = lane; j < n; j += 64) {
        const int32_t sg = ((L.xw[j >> 5] >> (j & 31)) & 1u) ? -2 : 2;
        L.Ul[j] = ((int32_t)L.dl[j] - (int32_t)bias - diag[j]) * sg / 4;
    }
    __syncthreads();
    for (int w = lane; w < NXW; w += 64) {
        for (uint32_t bits = L.pw[w]; bits; bits &= bits - 1u) {
            const int j = (w << 5) + __builtin_ctz(bits);
            const int32_t sg = ((L.xw[w] >> (j & 31)) & 1u) ? -1 : 1;
            __hip_atomic_fetch_add(L.Ul + j, sg * diag[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            for (int t = 0; t < W; ++t) {
                const uint32_t w2 = ell[(int64_t)j * W + t];
                if (w2 == 0u) break;
                __hip_atomic_fetch_add(L.Ul + qb_ell_col(w2), sg * qb_ell_val(w2), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
    __syncthreads();
    for (int j = lane; j < n; j += 64) {
        X[ro + j] = (uint8_t)(((L.xw[j >> 5] ^ L.pw[j >> 5]) >> (j & 31)) & 1u);
        H[ro + j] = L.Ul[j];
    }
    if (lane == 0) E[p] = OV - gap;
}

}  // namespace

// LDS bytes of the tree kernel for n variables.
size_t qb_tabu_tree_lds(int n)
{
    const size_t NN = ((size_t)n + 63) / 64, NP = NN * 64, NR = (NN + 63) / 64;
    return NP * 4 + NR * 64 * 12 + NP / 32 * 8 + NP * 2;
}

// QB_E_CAPACITY when the problem does not fit the tree kernel (the caller
// then runs the lane kernel), QB_E_RANGE when its keys cannot hold the move
// values.
qb_status qb_tabu_tree_launch(qb_problem P, int z, uint8_t *X, int32_t *H, int64_t *E, int alpha, int tenure,
                              int asp, int32_t *T, int32_t *LF, hipStream_t s)
{
    const int n = P->n;
    const size_t lds = qb_tabu_tree_lds(n);
    if (P->ellw > 64 || n > 64 * 64 * TT_MAX_NR || lds > 160 * 1024) return QB_E_CAPACITY;
    const int64_t dmax = (int64_t)P->qmax + 2 * P->eta_max;
    const int IB = qb_ceil_log2(n);
    if (2 * dmax > 0xFFFF || ((2 * dmax + 1) << IB) >= (int64_t(1) << 32)) return QB_E_RANGE;
    const int NR = (n + 4095) / 4096;
#define QB_TT(K)                                                                                              \
    if (NR == K) {                                                                                            \
        QB_TRY_HIP(hipFuncSetAttribute((const void *)k_tabu_tree<K>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                       (int)lds));                                                            \
        k_tabu_tree<K><<<z, 64, lds, s>>>(P->ell, P->ellw, P->diag, n, X, H, E, alpha, tenure, asp, T, LF,     \
                                          (uint32_t)dmax, IB);                                                \
    }
    QB_TT(1) QB_TT(2) QB_TT(3) QB_TT(4) QB_TT(5) QB_TT(6) QB_TT(7) QB_TT(8)
#undef QB_TT
    QB_LAUNCH_CHECK();
    return QB_OK;
}
