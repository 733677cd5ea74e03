// Tabu search (Alg. 1 of the IC-D^2S paper) on a sparse problem with the
// move values in a min-tree in LDS: one wave per solution.
//
// A step of Alg. 1 flips the allowed variable of least move value, and the
// flip changes only a handful of move values: the flipped variable's own
// (negated), its neighbours' (the O(degree) update of the Tabu section) and
// the tabu state of the variable whose tenure runs out.  So instead of an
// argmin over all n values per step, the kernel keeps the move values of the
// free variables under one level of 64-leaf nodes in LDS and repairs only
// the nodes a step touches, while the few tabu variables (about `tenure` of
// them) sit in slots held in registers.
//
// Layout per solution (one 64-lane workgroup):
//   dl[j]   x_j << 15 | (D_j + bias) (uint16 in LDS; bias bounds |D|, and
//           2 bias < 2^15 - 1; one more leaf past the last node holds the
//           all-ones value, the sentinel of the empty slots),
//   Ul[j]   the last step at which j is tabu (0: free; LDS),
//   pw      bit vector of "flipped since the last improvement",
//   nf[q]   the least key over the free leaves of node q (leaves 64q..64q+63),
//   slots   S (variable, last tabu step) pairs per lane for tabu variables;
//           the variable that turns tabu at step t goes to row 0 of lane
//           t mod 64, and the rows rotate by one after every 64 steps, so
//           that slot last took a variable 64 S steps earlier: it is empty
//           unless that occupant's tenure was extended (then the first empty
//           slot),
//   ob      bit vector of tabu variables that found no slot (normally empty;
//           scanned at every step while it is not, so the result never
//           depends on the slot count).
// A key is (D_j + bias) << IB | j, so the unsigned minimum is the least move
// value, then the lowest index: the oracle's tie rule.
//
// Step t: the least free key is the minimum over the nodes and over the
// slots whose tenure ran out at t (they rejoin the tree with an LDS atomic
// minimum); the least tabu key comes from the remaining slots, each reading
// its variable's current move value.  The smallest tabu key is allowed when
// it reaches OV + D < OV_min (aspiration); when nothing is free and nothing
// aspirates it wins anyway (the argmin over all).  The winner's ELL row is
// requested from memory at once; while it is in flight the wave reads the
// winner's node once, takes the winner's x and tabu step from its lane,
// rewrites the leaf in that lane's registers and recomputes the node from
// them, and moves the winner into a slot when it becomes tabu.  Then each
// lane with a neighbour c updates D_c in place: for a free c a key that fell
// needs only an atomic minimum on its node, a key that rose is a node repair
// only when it was the node's minimum; a tabu c needs nothing, its slot
// reads the new value at the next step.
//
// Invariant at the start of step t: a node's value is the minimum over a set
// of its leaves that holds every leaf free at t, except possibly those whose
// tenure ends exactly at t (they are still in slots and enter the minimum
// from there), and no leaf tabu at t.
#include "qb_internal.h"

namespace {

constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr int TT_MAX_NR = 8;   // nodes per lane: n <= 64 * 64 * 8

// Wave minimum left in lane 63: the row minima by quad and mirror moves,
// then the row broadcasts (the other lanes hold partial minima).
__device__ __forceinline__ uint32_t min_to63(uint32_t a)
{
    a = min(a, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)a, 0xB1, 0xF, 0xF, false));    // quad_perm [1,0,3,2]
    a = min(a, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)a, 0x4E, 0xF, 0xF, false));    // quad_perm [2,3,0,1]
    a = min(a, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)a, 0x141, 0xF, 0xF, false));   // row_half_mirror
    a = min(a, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)a, 0x140, 0xF, 0xF, false));   // row_mirror
    a = min(a, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)a, 0x142, 0xA, 0xF, false));  // row_bcast 15
    a = min(a, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)a, 0x143, 0xC, 0xF, false));  // row_bcast 31
    return a;
}

// Wave minimum, returned uniform.
__device__ __forceinline__ uint32_t min_uniform(uint32_t a)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)min_to63(a), 63);
}

// Wave sum, uniform (the overflow path only).
__device__ __forceinline__ int wave_sum(int v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return __builtin_amdgcn_readfirstlane(v);
}

struct TreeLds {
    int32_t *Ul;
    uint32_t *nf;    // NR * 64 slots, NONE past the last node
    uint32_t *pw;
    uint32_t *ob;
    uint32_t *dump;  // 64 words: where the lanes that must not store a value store it
    uint16_t *dl;
};

__device__ __forceinline__ TreeLds tree_lds(uint32_t *sm, int NN, int NR)
{
    const int NP = NN << 6, NXW = NP >> 5;
    TreeLds L;
    L.Ul = (int32_t *)sm;
    L.nf = sm + NP;
    L.pw = L.nf + 64 * NR;
    L.ob = L.pw + NXW;
    L.dump = L.ob + NXW;
    L.dl = (uint16_t *)(L.dump + 64);
    return L;
}

// A store of a uniform value by one lane without a branch: the other lanes
// store into their own word of the dump area (so no two lanes meet in a bank).
template <typename T>
__device__ __forceinline__ T *one_lane(const TreeLds &L, T *addr, int lane, int writer)
{
    return lane == writer ? addr : reinterpret_cast<T *>(L.dump + lane);
}

constexpr uint32_t DMASK = 0x7FFFu;   // the move-value field of a leaf

// nf[q] from leaf values already in registers (lane L: leaf 64q + L), free
// meaning Ul <= t (the state at step t + 1).
__device__ __forceinline__ void node_from(const TreeLds &L, int q, uint32_t d, int32_t u, int t, int n, int IB,
                                          int lane)
{
    const int j = (q << 6) + lane;
    const uint32_t f = (j < n && u <= t) ? (((d & DMASK) << IB) | (uint32_t)j) : NONE;
    *one_lane(L, L.nf + q, lane, 63) = min_to63(f);
}

__device__ __forceinline__ void recompute(const TreeLds &L, int q, int t, int n, int IB, int lane)
{
    const int j = (q << 6) + lane;
    node_from(L, q, L.dl[j], L.Ul[j], t, n, IB, lane);
}

template <int NR, int S>
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
    const int SENT = NP;              // the sentinel leaf of the empty slots
    constexpr int32_t NEVER = 0x7FFFFFFF;

    // leaves from x and the field: D_j = Q_jj + 2(1 - 2x_j) h_j
    for (int j0 = 0; j0 < NP; j0 += 64) {
        const int j = j0 + lane;
        uint32_t x = 0, dv = 0;
        if (j < n) {
            Tout[ro + j] = 0;
            LFout[ro + j] = 0;
            x = X[ro + j] & 1u;
            dv = (uint32_t)(diag[j] + (x ? -2 : 2) * H[ro + j] + (int32_t)bias) | (x << 15);
        }
        L.dl[j] = (uint16_t)dv;
        L.Ul[j] = 0;
        if (lane < 2) {
            L.pw[(j0 >> 5) + lane] = 0u;
            L.ob[(j0 >> 5) + lane] = 0u;
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) L.nf[lane + 64 * r] = NONE;
    if (lane == 0) L.dl[SENT] = (uint16_t)DMASK;
    __syncthreads();
    for (int q = 0; q < NN; ++q) recompute(L, q, 0, n, IB, lane);
    __syncthreads();

    // tabu slots: variable and its last tabu step; an empty slot holds the
    // sentinel leaf (its key is above every real key, so it never wins and
    // never aspirates) and a step that never comes (it never expires)
    int sj[S], su[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        sj[s] = SENT;
        su[s] = NEVER;
    }
    int ovf = 0;        // tabu variables outside the slots (their bits in ob)
    int bi = 0;         // the variable flipped at step 64 b + lane of the current batch b
    int64_t OV = E[p];
    int64_t OVmin = OV;
    // gap = OV - OV_min >= 0 in 32 bits: exact from each batch start (where it
    // is recomputed, saturated at GCAP) for as long as it stays below GCAP;
    // a step moves it by |D_i| < 2^15, so within a batch a saturated gap stays
    // above GCAP - 2^21, far above every value its two tests (gap < bias, and
    // gap + D_i < 0) tell apart
    constexpr int32_t GCAP = 1 << 30;
    int32_t gap = 0;
    const int ten1 = max(tenure - 1, 0);

    // steps in batches of 64 (batch b: steps 64 b .. 64 b + 63), the flip
    // counts sent at the end of each
    for (int b0 = 0; b0 <= alpha; b0 += 64) {
        const int shi = min(b0 + 63, alpha);
        gap = OV - OVmin < (int64_t)GCAP ? (int32_t)(OV - OVmin) : GCAP;
        for (int step = max(b0, 1); step <= shi; ++step) {
            // a tabu key k aspirates when D < OV_min - OV = -gap, that is k < tbk
            uint32_t tbk = 0;
            if (asp && gap < (int32_t)bias) tbk = (bias - (uint32_t)gap) << IB;
            // candidates: the free keys (nodes, and slots whose tenure ended:
            // free at this step) and the tabu keys (the other slots) that
            // aspirate
            uint32_t fm = NONE;
            uint32_t nv[NR], dv[S];
#pragma unroll
            for (int r = 0; r < NR; ++r) nv[r] = L.nf[lane + 64 * r];
#pragma unroll
            for (int s = 0; s < S; ++s) dv[s] = L.dl[sj[s]];
            __builtin_amdgcn_sched_barrier(0);   // every read issued before the first wait: one round trip
            // a slot's key is a candidate when it is below st: all ones for a
            // slot whose tenure ended (free), tbk for a tabu one (aspiration);
            // formed while the reads are in flight, so each slot needs one
            // compare and one select after them
            uint32_t sk[S], st[S];
            bool sx[S];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                sx[s] = su[s] < step;
                st[s] = sx[s] ? NONE : tbk;
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) fm = min(fm, nv[r]);
            uint32_t cm = NONE;   // least slot candidate, apart from fm's chain
#pragma unroll
            for (int s = 0; s < S; ++s) {
                sk[s] = (__builtin_amdgcn_ubfe(dv[s], 0, 15) << IB) | (uint32_t)sj[s];
                cm = min(cm, sk[s] < st[s] ? sk[s] : NONE);
            }
            fm = min(fm, cm);
            uint32_t tov = NONE;   // least tabu key among the overflow bits
            if (ovf > 0) {
                // tabu variables without a slot: scan their bits
                int freed = 0;
                for (int w = lane; w < NXW; w += 64) {
                    uint32_t keep = L.ob[w];
                    for (uint32_t bits = keep; bits; bits &= bits - 1u) {
                        const int j = (w << 5) + __builtin_ctz(bits);
                        const uint32_t key = (((uint32_t)L.dl[j] & DMASK) << IB) | (uint32_t)j;
                        if (L.Ul[j] < step) {
                            fm = min(fm, key);
                            __hip_atomic_fetch_min(L.nf + (j >> 6), key, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                            keep &= ~(1u << (j & 31));
                            ++freed;
                        } else {
                            tov = min(tov, key);
                            if (key < tbk) fm = min(fm, key);
                        }
                    }
                    L.ob[w] = keep;
                }
                ovf -= wave_sum(freed);
            }
            uint32_t best = min_uniform(fm);
            if (best == NONE) {
                // everything tabu and nothing aspirates: the least tabu key
                uint32_t tm = tov;
#pragma unroll
                for (int s = 0; s < S; ++s) tm = min(tm, sx[s] ? NONE : sk[s]);
                best = min_uniform(tm);
            }
            const int i = (int)(best & IMASK);
            const uint32_t dib = best >> IB;

            // the winner's row, in flight while its own leaf and node are redone
            uint32_t wd = 0u;
            if (lane < W) wd = ell[(int64_t)i * W + lane];

            // the winner's node, read once: its lane gives x_i and U_i, and the
            // node is recomputed from registers with the winner's leaf rewritten
            const int qi = i >> 6, li = i & 63;
            const int jl = (qi << 6) + lane;
            uint32_t dl_l = L.dl[jl];
            int32_t ul_l = L.Ul[jl];

            // slots whose tenure ended rejoin the tree (issued after the node
            // read, which waits for nothing of theirs, and before the node's
            // recompute is stored, which must land after them: the winner may
            // be one of these variables)
#pragma unroll
            for (int s = 0; s < S; ++s) {
                __hip_atomic_fetch_min(sx[s] ? L.nf + (sj[s] >> 6) : L.dump + lane, sx[s] ? sk[s] : NONE,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                sj[s] = sx[s] ? SENT : sj[s];
                su[s] = sx[s] ? NEVER : su[s];
            }
            const uint32_t di = (uint32_t)__builtin_amdgcn_readlane((int)dl_l, li);
            const int32_t Ui = __builtin_amdgcn_readlane(ul_l, li);
            const uint32_t xi = di >> 15;
            const uint32_t bit = 1u << (i & 31);
            const int32_t sgn = xi ? -1 : 1;   // h_j += sgn Q_ji
            // the last tabu step: step + max(max(Ui - step + 1, 0) + tenure - 1, 0),
            // which equals max(Ui + tenure, step + max(tenure - 1, 0)); any
            // value past alpha means tabu to the end, so it is held at
            // alpha + 1 (repeated extensions cannot grow it)
            const int32_t Un = min(max(Ui + tenure, step + ten1), alpha + 1);
            const int32_t dmove = (int32_t)dib - (int32_t)bias;
            const uint32_t dnew_i = 2u * bias - dib;   // D_i -> -D_i
            OV += dmove;
            gap += dmove;
            const bool improved = gap < 0;
            if (improved) {
                gap = 0;
                OVmin = OV;
            } else {
                gap = min(gap, GCAP);
            }
            if (lane == li) {
                dl_l = ((xi ^ 1u) << 15) | dnew_i;
                ul_l = Un;
            }
            // (lane li's leaf of the node is i itself: jl == i there)
            *one_lane(L, L.dl + jl, lane, li) = (uint16_t)dl_l;
            *one_lane(L, L.Ul + jl, lane, li) = ul_l;
            if (improved) {   // x_min is the current x
                for (int w = lane; w < NXW; w += 64) L.pw[w] = 0u;
            } else {
                __hip_atomic_fetch_xor(one_lane(L, L.pw + (i >> 5), lane, 0), bit, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            // i leaves the free set, changes its key or (tabu before and after)
            // stays out of it
            node_from(L, qi, dl_l, ul_l, step, n, IB, lane);

            // the slots: a free variable that turns tabu goes into the ring
            // position of this step (row 0, lane step mod 64), whose last
            // occupant came 64 S steps ago or earlier (the rows rotate every
            // 64 steps), so with 64 S >= tenure it is empty unless that
            // variable's tenure was extended; else into the first empty slot,
            // else the overflow bits (where a tabu variable sits never changes
            // a key or a result).  A tabu variable that flips again keeps its
            // slot with the new step, or leaves it at tenure 0.  Either way one
            // slot (row ps, lane plane) takes the pair (sjv, suv): row 0
            // without a branch, the other rows (only after a search) behind
            // one uniform branch.
            const bool was_tabu = Ui >= step, now_tabu = Un > step;
            int ps = -1, plane = 0, sjv = i;
            int32_t suv = Un;
            if (!was_tabu) {
                if (now_tabu) {
                    plane = step & 63;
                    ps = 0;
                    if (__builtin_amdgcn_readlane(sj[0], plane) != SENT) {
                        ps = -1;
                        // the highest row with an empty slot: row r is the ring
                        // row again after r rotations, and row 0 (this batch's
                        // ring row, whose later lanes the next steps take) only
                        // when no other row has one
#pragma unroll
                        for (int s = 0; s < S; ++s) {
                            const uint64_t em = __ballot(sj[s] == SENT);
                            if (em) {
                                ps = s;
                                plane = (int)__builtin_ctzll(em);
                            }
                        }
                        if (ps < 0) {
                            if (lane == 0)
                                __hip_atomic_fetch_or(L.ob + (i >> 5), bit, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_WORKGROUP);
                            ++ovf;
                        }
                    }
                }
            } else {
                // i sits in a slot (an expired slot was emptied above, so only
                // a tabu i can), or in the overflow bits
#pragma unroll
                for (int s = S - 1; s >= 0; --s) {
                    const uint64_t em = __ballot(sj[s] == i);
                    if (em) {
                        ps = s;
                        plane = (int)__builtin_ctzll(em);
                    }
                }
                if (!now_tabu) {
                    sjv = SENT;
                    suv = NEVER;
                    if (ps < 0) {
                        // tenure 0: free again at once (the node above took it back)
                        if (lane == 0)
                            __hip_atomic_fetch_and(L.ob + (i >> 5), ~bit, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                        --ovf;
                    }
                }
            }
            {
                const int trow = lane == plane ? ps : -1;   // the row this lane rewrites, if any
                sj[0] = trow == 0 ? sjv : sj[0];
                su[0] = trow == 0 ? suv : su[0];
                if (S > 1 && ps > 0) {
#pragma unroll
                    for (int s = 1; s < S; ++s) {
                        const bool mine = trow == s;
                        sj[s] = mine ? sjv : sj[s];
                        su[s] = mine ? suv : su[s];
                    }
                }
            }

            // neighbours: D_c += 2(1 - 2x_c) sgn Q_ci, without a branch (a lane
            // without a neighbour reads leaf 0 and stores into the dump area):
            // the leaf, its tabu step and its node are read in one round trip
            bool need;
            int cq;
            {
                const bool has = wd != 0u;
                const int c = qb_ell_col(wd);
                const int32_t v = qb_ell_val(wd);
                cq = c >> 6;
                const uint32_t lold = L.dl[c];
                const int32_t uc = L.Ul[c];
                const uint32_t nq = L.nf[cq];
                __builtin_amdgcn_sched_barrier(0);
                const int32_t sg = (lold >> 15) ? -2 : 2;
                const uint32_t dold = lold & DMASK;
                const uint32_t dnew = (uint32_t)((int32_t)dold + sg * sgn * v);
                *(has ? L.dl + c : reinterpret_cast<uint16_t *>(L.dump + lane)) = (uint16_t)((lold & ~DMASK) | dnew);
                // free at step + 1: the tree holds it (or may, when its tenure ends now)
                const bool intree = has && uc <= step;
                const uint32_t kold = (dold << IB) | (uint32_t)c, knew = (dnew << IB) | (uint32_t)c;
                const bool fell = intree && knew < kold;
                __hip_atomic_fetch_min(fell ? L.nf + cq : L.dump + lane, fell ? knew : NONE, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                // a key that rose repairs its node only when it was the node's minimum
                need = intree && knew > kold && nq == kold;
            }
            for (uint64_t m = __ballot(need); m;) {
                const int q = __builtin_amdgcn_readlane(cq, __builtin_ctzll(m));
                recompute(L, q, step, n, IB, lane);
                m &= ~__ballot(need && cq == q);
            }
            // the flip count and last-flip step: lane (step mod 64) keeps this
            // step's flip, and every 64 steps the wave sends the 64 of them at
            // once (an atomic add and an atomic maximum each, so a variable
            // flipped twice in a batch is counted twice and keeps its later step)
            bi = lane == (step & 63) ? i : bi;
        }
        if (lane <= shi - b0 && b0 + lane >= 1) {
            __hip_atomic_fetch_add(Tout + ro + bi, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_max(LFout + ro + bi, b0 + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // the next batch's ring row becomes row 0
        if (S > 1) {
            const int j0 = sj[0], u0 = su[0];
#pragma unroll
            for (int s = 0; s + 1 < S; ++s) {
                sj[s] = sj[s + 1];
                su[s] = su[s + 1];
            }
            sj[S - 1] = j0;
            su[S - 1] = u0;
        }
    }
    __syncthreads();

    // field of the final x from D (h_j = (D_j - Q_jj) / (2(1 - 2x_j))), kept
    // in Ul, then moved to x_min = x ^ pw by the rows of the differing
    // variables (their own diagonal term and their neighbours)
    for (int j = lane; j < n; j += 64) {
        const uint32_t lj = L.dl[j];
        const int32_t sg = (lj >> 15) ? -2 : 2;
        L.Ul[j] = ((int32_t)(lj & DMASK) - (int32_t)bias - diag[j]) * sg / 4;
    }
    __syncthreads();
    for (int w = lane; w < NXW; w += 64) {
        for (uint32_t bits = L.pw[w]; bits; bits &= bits - 1u) {
            const int j = (w << 5) + __builtin_ctz(bits);
            const int32_t sg = (L.dl[j] >> 15) ? -1 : 1;
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
        X[ro + j] = (uint8_t)(((uint32_t)L.dl[j] >> 15) ^ ((L.pw[j >> 5] >> (j & 31)) & 1u));
        H[ro + j] = L.Ul[j];
    }
    if (lane == 0) E[p] = OVmin;
}

}  // namespace

// LDS bytes of the tree kernel for n variables.
size_t qb_tabu_tree_lds(int n)
{
    const size_t NN = ((size_t)n + 63) / 64, NP = NN * 64, NR = (NN + 63) / 64;
    return NP * 4 + NR * 64 * 4 + NP / 32 * 8 + 64 * 4 + NP * 2 + 4;
}

qb_status qb_tabu_tree_fits(qb_problem P)
{
    const int n = P->n;
    if (!P->sparse || P->ellw > 64 || n > 64 * 64 * TT_MAX_NR || qb_tabu_tree_lds(n) > 160 * 1024)
        return QB_E_CAPACITY;
    const int64_t dmax = (int64_t)P->qmax + 2 * P->eta_max;
    if (2 * dmax >= (int64_t)DMASK || ((2 * dmax + 1) << qb_ceil_log2(n)) >= (int64_t(1) << 32)) return QB_E_RANGE;
    return QB_OK;
}

// QB_E_CAPACITY when the problem does not fit the tree kernel (the caller
// then runs the lane kernel), QB_E_RANGE when its keys cannot hold the move
// values.  Slots per lane: enough for `tenure` tabu variables with 16 to
// spare, at most eight (beyond, the overflow bits take the rest).
qb_status qb_tabu_tree_launch(qb_problem P, int z, uint8_t *X, int32_t *H, int64_t *E, int alpha, int tenure,
                              int asp, int32_t *T, int32_t *LF, hipStream_t s)
{
    const qb_status fit = qb_tabu_tree_fits(P);
    if (fit != QB_OK) return fit;
    const int n = P->n;
    const size_t lds = qb_tabu_tree_lds(n);
    const int64_t dmax = (int64_t)P->qmax + 2 * P->eta_max;
    const int IB = qb_ceil_log2(n);
    const int NR = (n + 4095) / 4096;
    const int need = (int)std::min<int64_t>((int64_t)tenure + 16, n);
    const int S = need <= 64 ? 1 : need <= 128 ? 2 : need <= 192 ? 3 : need <= 256 ? 4 : 8;
#define QB_TT(K, SL)                                                                                           \
    if (NR == K && S == SL) {                                                                                  \
        QB_TRY_HIP(hipFuncSetAttribute((const void *)k_tabu_tree<K, SL>,                                       \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));                 \
        k_tabu_tree<K, SL><<<z, 64, lds, s>>>(P->ell, P->ellw, P->diag, n, X, H, E, alpha, tenure, asp, T, LF, \
                                              (uint32_t)dmax, IB);                                             \
    }
#define QB_TT3(K) QB_TT(K, 1) QB_TT(K, 2) QB_TT(K, 3) QB_TT(K, 4) QB_TT(K, 8)
    QB_TT3(1) QB_TT3(2) QB_TT3(3) QB_TT3(4) QB_TT3(5) QB_TT3(6) QB_TT3(7) QB_TT3(8)
#undef QB_TT3
#undef QB_TT
    QB_LAUNCH_CHECK();
    return QB_OK;
}
