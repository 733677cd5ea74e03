// Problem handle, initial solutions, local field, exact energy, best tracking,
// host-side schedule tables.  Eq. 1 and Alg. 2 of the IC-D^2S paper.
#include <math.h>

#include <algorithm>
#include <cstring>

#include "qb_internal.h"

static thread_local int32_t g_last_hip_error = 0;
void qb_set_hip_error(hipError_t e) { g_last_hip_error = (int32_t)e; }

extern "C" int32_t qb_last_hip_error(void) { return g_last_hip_error; }
extern "C" const char *qb_version(void) { return "qb-gfx950 0.1"; }

extern "C" const char *qb_status_str(qb_status s)
{
    switch (s) {
    case QB_OK: return "ok";
    case QB_E_ARG: return "invalid argument";
    case QB_E_NOT_SYMMETRIC: return "Q is not symmetric";
    case QB_E_RANGE: return "value range exceeds the exact integer arithmetic";
    case QB_E_OVERLAP: return "jobs of one solution overlap";
    case QB_E_CAPACITY: return "size beyond kernel capacity";
    case QB_E_HIP: return "HIP runtime error";
    case QB_E_STATE: return "device-side check failed";
    case QB_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

// ------------------------------------------------------------------ problem scan
// One pass over Q in 64x64 tiles: symmetry (each tile against its mirror,
// both staged through LDS so every global read is coalesced), max |Q|, and
// the sum of squared off-diagonal entries.
__global__ void __launch_bounds__(256) k_problem_scan(const int16_t *__restrict__ Q, int n,
                                                      int32_t *__restrict__ flags, int32_t *__restrict__ qmax,
                                                      unsigned long long *__restrict__ sumsq)
{
    __shared__ int16_t A[64][65], B[64][65];
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    for (int t = threadIdx.x; t < 64 * 64; t += 256) {
        const int r = t >> 6, c = t & 63;
        A[r][c] = (r0 + r < n && c0 + c < n) ? Q[(int64_t)(r0 + r) * n + c0 + c] : 0;
        B[r][c] = (c0 + r < n && r0 + c < n) ? Q[(int64_t)(c0 + r) * n + r0 + c] : 0;
    }
    __syncthreads();
    int32_t amax = 0, bad = 0;
    unsigned long long sq = 0;
    for (int t = threadIdx.x; t < 64 * 64; t += 256) {
        const int r = t >> 6, c = t & 63;
        const int32_t v = A[r][c];
        bad |= v != B[c][r];
        amax = max(amax, v < 0 ? -v : v);
        if (r0 + r != c0 + c) sq += (unsigned long long)(v * v);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        amax = max(amax, __shfl_xor(amax, o, 64));
        bad |= __shfl_xor(bad, o, 64);
        sq += __shfl_xor(sq, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(qmax, amax);
        if (bad) atomicOr(flags, 1);
        if (sq) atomicAdd(sumsq, sq);
    }
}

// eta_j = sum_i |Q_ij| (Weight_Effect_Extraction); coalesced over j.
__global__ void k_eta(const int16_t *__restrict__ Q, int n, int64_t *__restrict__ eta)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int64_t acc = 0;
    for (int i = 0; i < n; ++i) {
        const int32_t v = Q[(int64_t)i * n + j];
        acc += v < 0 ? -v : v;
    }
    eta[j] = acc;
}

// Row-padded copy of Q (pitch ld elements, zero padding), int8 or int16.
template <typename T>
__global__ void k_pad_copy(const int16_t *__restrict__ Q, int n, int ld, T *__restrict__ out)
{
    const int i = blockIdx.y;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ld; j += gridDim.x * blockDim.x)
        out[(int64_t)i * ld + j] = j < n ? (T)Q[(int64_t)i * n + j] : (T)0;
}

// Rows of Q in the dense Tabu kernel's thread order (qb_tabu_pos), zero
// past column n.
template <typename T>
__global__ void k_tabu_copy(const int16_t *__restrict__ Q, int n, int ld, int ept, int tb, T *__restrict__ out)
{
    const int i = blockIdx.y;
    // the ept * tb elements of a row; a slot's padding is left as it is
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ept * tb; j += gridDim.x * blockDim.x) {
        const int pos = qb_tabu_pos(j / tb, j % tb, ept, (int)sizeof(T), tb);
        out[(int64_t)i * ld + pos] = j < n ? (T)Q[(int64_t)i * n + j] : (T)0;
    }
}

__global__ void k_diag(const int16_t *__restrict__ Q, int n, int32_t *__restrict__ diag)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) diag[j] = Q[(int64_t)j * n + j];
}

__global__ void k_to_int8(const int16_t *__restrict__ Q, int8_t *__restrict__ Q8, int64_t count)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x)
        Q8[t] = (int8_t)Q[t];
}

extern "C" qb_status qb_problem_create_dense(qb_problem *out, int32_t n, const int16_t *Q_d,
                                            void *stream)
{
    if (!out || !Q_d || n < 1 || n > 65535) return QB_E_ARG;
    *out = nullptr;
    hipStream_t s = qb_stream(stream);
    qb_problem P = new qb_problem_s();
    P->n = n;
    P->Q = Q_d;
    struct Scan {
        int32_t flags, qmax;
        unsigned long long sumsq;
    };
    Scan *scan_d = nullptr;
    Scan scan_h{};
    qb_status rc = QB_OK;
    auto fail = [&](qb_status r) {
        rc = r;
        return r;
    };
    do {
        if (hipMalloc(&scan_d, sizeof(Scan)) != hipSuccess) { fail(QB_E_HIP); break; }
        if (hipMemsetAsync(scan_d, 0, sizeof(Scan), s) != hipSuccess) { fail(QB_E_HIP); break; }
        dim3 grid((n + 63) / 64, (n + 63) / 64);
        k_problem_scan<<<grid, 256, 0, s>>>(Q_d, n, &scan_d->flags, &scan_d->qmax, &scan_d->sumsq);
        if (hipMemcpyAsync(&scan_h, scan_d, sizeof(Scan), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            fail(QB_E_HIP);
            break;
        }
        if (scan_h.flags) { fail(QB_E_NOT_SYMMETRIC); break; }
        const int64_t bound = (2 * (int64_t)n + 1) * (int64_t)scan_h.qmax;
        if (bound >= (int64_t(1) << 31)) { fail(QB_E_RANGE); break; }
        P->qmax = scan_h.qmax;
        P->int8_ok = scan_h.qmax <= 127;
        P->sigma = sqrt((double)scan_h.sumsq / (double)n);
        if (hipMalloc(&P->eta, sizeof(int64_t) * n) != hipSuccess ||
            hipMalloc(&P->colcnt, sizeof(int32_t) * n) != hipSuccess ||
            hipMalloc(&P->diag, sizeof(int32_t) * n) != hipSuccess ||
            hipMalloc(&P->status, sizeof(int32_t)) != hipSuccess) {
            fail(QB_E_HIP);
            break;
        }
        if (hipMemsetAsync(P->status, 0, sizeof(int32_t), s) != hipSuccess) {
            fail(QB_E_HIP);
            break;
        }
        k_eta<<<(n + 255) / 256, 256, 0, s>>>(Q_d, n, P->eta);
        k_diag<<<(n + 255) / 256, 256, 0, s>>>(Q_d, n, P->diag);
        if (P->int8_ok) {
            if (hipMalloc(&P->Q8, (size_t)n * n) != hipSuccess) { fail(QB_E_HIP); break; }
            k_to_int8<<<1024, 256, 0, s>>>(Q_d, P->Q8, (int64_t)n * n);
        }
        std::vector<int64_t> eta_h(n);
        if (hipMemcpyAsync(eta_h.data(), P->eta, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            fail(QB_E_HIP);
            break;
        }
        P->eta_max = *std::max_element(eta_h.begin(), eta_h.end());
        // the dense Tabu kernel's workgroup: the preferred size, unless its
        // wider element field leaves too few key bits for these move values
        // (the 1024-thread kernel then takes the range it always had)
        int tb = qb_tabu_threads(n);
        int ept = qb_tabu_ept(n, tb);
        const int64_t dmax = (int64_t)P->qmax + 2 * P->eta_max;
        if (tb != QB_TABU_THREADS && ept && 2 * dmax + 1 >= (int64_t)(0x7FFFFFFFu >> qb_ceil_log2(ept))) {
            tb = QB_TABU_THREADS;
            ept = qb_tabu_ept(n, tb);
        }
        if (ept) {
            P->tabu_tb = tb;
            P->tabu_ept = ept;
            const size_t esz = P->int8_ok ? 1 : 2;
            P->ldp = qb_tabu_pitch(tb, ept, (int)esz);
            if (hipMalloc(&P->Qp, esz * (size_t)n * P->ldp) != hipSuccess ||
                hipMalloc(&P->Qt, esz * (size_t)n * P->ldp) != hipSuccess) {
                fail(QB_E_HIP);
                break;
            }
            // zero first: the copy kernel leaves the slots' padding alone
            if (hipMemsetAsync(P->Qt, 0, esz * (size_t)n * P->ldp, s) != hipSuccess) {
                fail(QB_E_HIP);
                break;
            }
            dim3 g((P->ldp + 255) / 256, n);
            if (P->int8_ok) {
                k_pad_copy<int8_t><<<g, 256, 0, s>>>(Q_d, n, P->ldp, (int8_t *)P->Qp);
                k_tabu_copy<int8_t><<<g, 256, 0, s>>>(Q_d, n, P->ldp, ept, tb, (int8_t *)P->Qt);
            } else {
                k_pad_copy<int16_t><<<g, 256, 0, s>>>(Q_d, n, P->ldp, (int16_t *)P->Qp);
                k_tabu_copy<int16_t><<<g, 256, 0, s>>>(Q_d, n, P->ldp, ept, tb, (int16_t *)P->Qt);
            }
            if (hipGetLastError() != hipSuccess) {
                fail(QB_E_HIP);
                break;
            }
        }
        // the derived copies are complete before the handle is returned, so
        // calls on other streams may use them at once
        if (hipStreamSynchronize(s) != hipSuccess) {
            fail(QB_E_HIP);
            break;
        }
    } while (0);
    if (scan_d) (void)hipFree(scan_d);
    if (rc != QB_OK) {
        qb_problem_destroy(P);
        return rc;
    }
    *out = P;
    return QB_OK;
}

// ------------------------------------------------------------------ sparse problem
// One thread per row: structure (columns strictly ascending and in range),
// diagonal, off-diagonal count, eta, max |Q|, squared off-diagonal sum, and
// symmetry (each off-diagonal entry is looked up in its mirror row by binary
// search; a row that is itself unsorted is flagged as malformed).
__global__ void __launch_bounds__(256) k_csr_scan(int n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col,
                                                  const int16_t *__restrict__ val, int32_t *__restrict__ diag,
                                                  int32_t *__restrict__ deg, int64_t *__restrict__ eta,
                                                  int32_t *__restrict__ flags, int32_t *__restrict__ qmax,
                                                  int32_t *__restrict__ dmax, unsigned long long *__restrict__ sumsq)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int32_t amax = 0, bad = 0, asym = 0, d = 0;
    unsigned long long sq = 0;
    if (i < n) {
        const int a = rp[i], b = rp[i + 1];
        int prev = -1;
        int32_t dg = 0;
        int64_t et = 0;
        for (int t = a; t < b; ++t) {
            const int c = col[t];
            if (c <= prev || c >= n) {
                bad = 1;
                break;
            }
            prev = c;
            const int32_t v = val[t];
            const int32_t av = v < 0 ? -v : v;
            amax = max(amax, av);
            et += av;
            if (c == i) {
                dg = v;
                continue;
            }
            ++d;
            sq += (unsigned long long)(av * av);
            int lo = rp[c], hi = rp[c + 1] - 1;
            bool found = false;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int cm = col[mid];
                if (cm == i) {
                    found = val[mid] == v;
                    break;
                }
                if (cm < i)
                    lo = mid + 1;
                else
                    hi = mid - 1;
            }
            asym |= !found;
        }
        diag[i] = dg;
        deg[i] = d;
        eta[i] = et;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        amax = max(amax, __shfl_xor(amax, o, 64));
        d = max(d, __shfl_xor(d, o, 64));
        bad |= __shfl_xor(bad, o, 64);
        asym |= __shfl_xor(asym, o, 64);
        sq += __shfl_xor(sq, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(qmax, amax);
        atomicMax(dmax, d);
        if (bad) atomicOr(flags, 2);
        if (asym) atomicOr(flags, 1);
        if (sq) atomicAdd(sumsq, sq);
    }
}

// Off-diagonal entries of row i into ELL words [i*W, i*W + deg), zeros after.
__global__ void k_csr_to_ell(int n, int W, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                             const int16_t *__restrict__ val, uint32_t *__restrict__ ell,
                             int32_t *__restrict__ ecnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t *row = ell + (int64_t)i * W;
    int k = 0;
    for (int t = rp[i]; t < rp[i + 1]; ++t) {
        const int c = col[t];
        if (c != i) row[k++] = qb_ell_word(val[t], c);
    }
    ecnt[i] = k;
    for (; k < W; ++k) row[k] = 0u;
}

extern "C" qb_status qb_problem_create_csr(qb_problem *out, int32_t n, const int32_t *rowptr_d,
                                          const int32_t *col_d, const int16_t *val_d, void *stream)
{
    if (!out || !rowptr_d || n < 1 || n > 65535) return QB_E_ARG;
    *out = nullptr;
    hipStream_t s = qb_stream(stream);
    std::vector<int32_t> rp(n + 1);
    QB_TRY_HIP(hipMemcpyAsync(rp.data(), rowptr_d, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s));
    QB_TRY_HIP(hipStreamSynchronize(s));
    if (rp[0] != 0) return QB_E_ARG;
    for (int i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return QB_E_ARG;
    const int64_t nnz = rp[n];
    if (nnz > 0 && (!col_d || !val_d)) return QB_E_ARG;
    qb_problem P = new qb_problem_s();
    P->n = n;
    P->sparse = 1;
    struct Scan {
        int32_t flags, qmax, dmax, pad;
        unsigned long long sumsq;
    };
    Scan *scan_d = nullptr;
    int32_t *deg_d = nullptr;
    Scan scan_h{};
    qb_status rc = QB_OK;
    do {
        if (hipMalloc(&scan_d, sizeof(Scan)) != hipSuccess || hipMalloc(&deg_d, sizeof(int32_t) * n) != hipSuccess ||
            hipMalloc(&P->eta, sizeof(int64_t) * n) != hipSuccess ||
            hipMalloc(&P->colcnt, sizeof(int32_t) * n) != hipSuccess ||
            hipMalloc(&P->diag, sizeof(int32_t) * n) != hipSuccess ||
            hipMalloc(&P->ecnt, sizeof(int32_t) * n) != hipSuccess ||
            hipMalloc(&P->status, sizeof(int32_t)) != hipSuccess) {
            rc = QB_E_HIP;
            break;
        }
        if (hipMemsetAsync(scan_d, 0, sizeof(Scan), s) != hipSuccess ||
            hipMemsetAsync(P->status, 0, sizeof(int32_t), s) != hipSuccess) {
            rc = QB_E_HIP;
            break;
        }
        k_csr_scan<<<(n + 255) / 256, 256, 0, s>>>(n, rowptr_d, col_d, val_d, P->diag, deg_d, P->eta, &scan_d->flags,
                                                   &scan_d->qmax, &scan_d->dmax, &scan_d->sumsq);
        if (hipMemcpyAsync(&scan_h, scan_d, sizeof(Scan), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = QB_E_HIP;
            break;
        }
        if (scan_h.flags & 2) { rc = QB_E_ARG; break; }
        if (scan_h.flags & 1) { rc = QB_E_NOT_SYMMETRIC; break; }
        const int64_t bound = (2 * (int64_t)n + 1) * (int64_t)scan_h.qmax;
        if (bound >= (int64_t(1) << 31)) { rc = QB_E_RANGE; break; }
        P->qmax = scan_h.qmax;
        P->int8_ok = scan_h.qmax <= 127;
        P->sigma = sqrt((double)scan_h.sumsq / (double)n);
        P->ellw = std::max(4, (scan_h.dmax + 3) & ~3);
        // 16 spare zero words after the last row: row readers fetch whole
        // 16-word chunks and ignore the words past the row
        const size_t ell_words = (size_t)n * P->ellw + 16;
        if (hipMalloc(&P->ell, sizeof(uint32_t) * ell_words) != hipSuccess ||
            hipMemsetAsync(P->ell + (size_t)n * P->ellw, 0, sizeof(uint32_t) * 16, s) != hipSuccess) {
            rc = QB_E_HIP;
            break;
        }
        k_csr_to_ell<<<(n + 255) / 256, 256, 0, s>>>(n, P->ellw, rowptr_d, col_d, val_d, P->ell, P->ecnt);
        std::vector<int64_t> eta_h(n);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(eta_h.data(), P->eta, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = QB_E_HIP;
            break;
        }
        P->eta_max = *std::max_element(eta_h.begin(), eta_h.end());
    } while (0);
    if (scan_d) (void)hipFree(scan_d);
    if (deg_d) (void)hipFree(deg_d);
    if (rc != QB_OK) {
        qb_problem_destroy(P);
        return rc;
    }
    *out = P;
    return QB_OK;
}

extern "C" void qb_problem_destroy(qb_problem P)
{
    if (!P) return;
    if (P->Q8) (void)hipFree(P->Q8);
    if (P->Qp) (void)hipFree(P->Qp);
    if (P->Qt) (void)hipFree(P->Qt);
    if (P->eta) (void)hipFree(P->eta);
    if (P->colcnt) (void)hipFree(P->colcnt);
    if (P->diag) (void)hipFree(P->diag);
    if (P->ell) (void)hipFree(P->ell);
    if (P->ecnt) (void)hipFree(P->ecnt);
    if (P->status) (void)hipFree(P->status);
    delete P;
}

extern "C" qb_status qb_problem_get_info(qb_problem P, qb_problem_info *info)
{
    if (!P || !info) return QB_E_ARG;
    info->n = P->n;
    info->int8_ok = P->int8_ok;
    info->qmax = P->qmax;
    info->eta_max = P->eta_max;
    info->sigma = P->sigma;
    info->sparse = P->sparse;
    info->ell_width = P->ellw;
    if (!P->sparse) {
        info->tabu_kernel = P->tabu_ept ? 0 : -1;
    } else {
        const bool tree = P->tabu_variant != QB_TABU_LANES && qb_tabu_tree_fits(P) == QB_OK;
        const bool lanes = P->tabu_variant != QB_TABU_TREE && qb_tabu_sp_ept(P->n) != 0;
        info->tabu_kernel = tree ? QB_TABU_TREE : lanes ? QB_TABU_LANES : -1;
    }
    return QB_OK;
}

extern "C" qb_status qb_problem_set_tabu_variant(qb_problem P, int32_t variant)
{
    if (!P || !P->sparse || variant < QB_TABU_AUTO || variant > QB_TABU_TREE) return QB_E_ARG;
    P->tabu_variant = variant;
    return QB_OK;
}

extern "C" qb_status qb_problem_eta(qb_problem P, int64_t *eta_d, void *stream)
{
    if (!P || !eta_d) return QB_E_ARG;
    QB_TRY_HIP(hipMemcpyAsync(eta_d, P->eta, sizeof(int64_t) * P->n, hipMemcpyDeviceToDevice,
                              qb_stream(stream)));
    return QB_OK;
}

extern "C" qb_status qb_check(qb_problem P, void *stream)
{
    if (!P) return QB_E_ARG;
    hipStream_t s = qb_stream(stream);
    int32_t flags = 0;
    QB_TRY_HIP(hipMemcpyAsync(&flags, P->status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    QB_TRY_HIP(hipStreamSynchronize(s));
    if (!flags) return QB_OK;
    QB_TRY_HIP(hipMemsetAsync(P->status, 0, sizeof(int32_t), s));
    QB_TRY_HIP(hipStreamSynchronize(s));
    return (flags & QB_FLAG_RANGE) ? QB_E_RANGE : QB_E_STATE;
}

// ------------------------------------------------------------------ a1 init
__global__ void k_init_x(int n, int z, uint32_t k0, uint32_t k1, uint8_t *__restrict__ X)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;   // group of 4 variables
    const int p = blockIdx.y;
    if (4 * g >= n) return;
    const uint4 o = qb_philox(make_uint4((uint32_t)g, (uint32_t)p, 0u, 3u << 28), k0, k1);
    uint8_t *row = X + (int64_t)p * n;
#pragma unroll
    for (int w = 0; w < 4; ++w)
        if (4 * g + w < n) row[4 * g + w] = (uint8_t)(qb_word(o, w) >> 31);
}

extern "C" qb_status qb_init_solutions(int32_t n, int32_t z, uint64_t seed, uint8_t *X_d,
                                      void *stream)
{
    if (n < 1 || z < 1 || z > 65535 || !X_d) return QB_E_ARG;
    dim3 grid(((n + 3) / 4 + 255) / 256, z);
    k_init_x<<<grid, 256, 0, qb_stream(stream)>>>(n, z, (uint32_t)seed, (uint32_t)(seed >> 32), X_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

// ------------------------------------------------------------------ field H = X Q
// Block: 256 columns i x 8 solutions; X chunk staged through LDS.
__global__ void __launch_bounds__(256) k_field(const int16_t *__restrict__ Q, int n, int z,
                                               const uint8_t *__restrict__ X, int32_t *__restrict__ H)
{
    constexpr int ZT = 8, JC = 256;
    __shared__ uint8_t xs[ZT][JC];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int p0 = blockIdx.y * ZT;
    int32_t acc[ZT] = {0};
    for (int j0 = 0; j0 < n; j0 += JC) {
        __syncthreads();
        for (int t = threadIdx.x; t < ZT * JC; t += 256) {
            const int pp = t / JC, jj = t % JC;
            xs[pp][jj] = (p0 + pp < z && j0 + jj < n) ? X[(int64_t)(p0 + pp) * n + j0 + jj] : 0;
        }
        __syncthreads();
        if (i < n) {
            const int jn = min(JC, n - j0);
            for (int jj = 0; jj < jn; ++jj) {
                const int32_t q = Q[(int64_t)(j0 + jj) * n + i];
#pragma unroll
                for (int pp = 0; pp < ZT; ++pp) acc[pp] += q * xs[pp][jj];
            }
        }
    }
    if (i < n)
#pragma unroll
        for (int pp = 0; pp < ZT; ++pp)
            if (p0 + pp < z) H[(int64_t)(p0 + pp) * n + i] = acc[pp];
}

qb_status qb_rankk_mfma_launch(qb_problem P, int z, const int8_t *dX, int32_t *H, hipStream_t s);
qb_status qb_field_ell_launch(qb_problem P, int z, const uint8_t *X, int32_t *H, hipStream_t s);

extern "C" qb_status qb_field(qb_problem P, int32_t z, const uint8_t *X_d, int32_t *H_d, void *stream)
{
    if (!P || z < 1 || z > 65535 || !X_d || !H_d) return QB_E_ARG;
    if (P->sparse) return qb_field_ell_launch(P, z, X_d, H_d, qb_stream(stream));
    if (P->int8_ok && P->Qp && z >= 32) {
        // H = 0 + X Q on the int8 matrix cores (X in {0,1} read as int8)
        qb_status rc = qb_zero(H_d, sizeof(int32_t) * (size_t)z * P->n, stream);
        if (rc != QB_OK) return rc;
        return qb_rankk_mfma_launch(P, z, (const int8_t *)X_d, H_d, qb_stream(stream));
    }
    dim3 grid((P->n + 255) / 256, (z + 7) / 8);
    k_field<<<grid, 256, 0, qb_stream(stream)>>>(P->Q, P->n, z, X_d, H_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

// ------------------------------------------------------------------ energy
__global__ void __launch_bounds__(256) k_energy(int n, const uint8_t *__restrict__ X,
                                                const int32_t *__restrict__ H, int64_t *__restrict__ E)
{
    __shared__ int64_t part[4];
    const int p = blockIdx.x;
    const uint8_t *x = X + (int64_t)p * n;
    const int32_t *h = H + (int64_t)p * n;
    int64_t acc = 0;
    for (int i = threadIdx.x; i < n; i += 256)
        if (x[i]) acc += h[i];
    acc = qb_wave_sum_i64(acc);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) E[p] = part[0] + part[1] + part[2] + part[3];
}

extern "C" qb_status qb_energy(int32_t n, int32_t z, const uint8_t *X_d, const int32_t *H_d,
                              int64_t *E_d, void *stream)
{
    if (n < 1 || z < 1 || !X_d || !H_d || !E_d) return QB_E_ARG;
    k_energy<<<z, 256, 0, qb_stream(stream)>>>(n, X_d, H_d, E_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

// ------------------------------------------------------------------ best tracking
__global__ void __launch_bounds__(256) k_best(int n, int z, const uint8_t *__restrict__ X,
                                              const int64_t *__restrict__ E, int64_t *__restrict__ ebest,
                                              uint8_t *__restrict__ xbest)
{
    __shared__ int64_t se[4];
    __shared__ int sp[4];
    __shared__ int winner;
    int64_t be = INT64_MAX;
    int bp = -1;
    for (int p = threadIdx.x; p < z; p += 256)
        if (E[p] < be) { be = E[p]; bp = p; }   // ascending p: first minimum kept
    // the smallest (E, p) of the block: shuffles within each wave, then the
    // four wave results
    auto take = [&](int64_t oe, int op) {
        if (op >= 0 && (bp < 0 || oe < be || (oe == be && op < bp))) {
            be = oe;
            bp = op;
        }
    };
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t oe = __shfl_xor(be, o, 64);
        const int op = __shfl_xor(bp, o, 64);
        take(oe, op);
    }
    if ((threadIdx.x & 63) == 0) {
        se[threadIdx.x >> 6] = be;
        sp[threadIdx.x >> 6] = bp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 1; t < 4; ++t) take(se[t], sp[t]);
        winner = (bp >= 0 && be < *ebest) ? bp : -1;
        if (winner >= 0) *ebest = be;
    }
    __syncthreads();
    const int w = winner;
    if (w < 0) return;
    for (int j = threadIdx.x; j < n; j += 256) xbest[j] = X[(int64_t)w * n + j];
}

extern "C" qb_status qb_best(int32_t n, int32_t z, const uint8_t *X_d, const int64_t *E_d,
                            int64_t *ebest_d, uint8_t *xbest_d, void *stream)
{
    if (n < 1 || z < 1 || !X_d || !E_d || !ebest_d || !xbest_d) return QB_E_ARG;
    k_best<<<1, 256, 0, qb_stream(stream)>>>(n, z, X_d, E_d, ebest_d, xbest_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

// ------------------------------------------------------------------ zero fill
__global__ void k_zero16(uint4 *__restrict__ p, int64_t n16)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n16;
         t += (int64_t)gridDim.x * blockDim.x)
        p[t] = make_uint4(0, 0, 0, 0);
}
__global__ void k_zero1(uint8_t *__restrict__ p, int64_t n)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        p[t] = 0;
}

extern "C" qb_status qb_zero(void *buf_d, size_t bytes, void *stream)
{
    if (!buf_d) return bytes ? QB_E_ARG : QB_OK;
    if (!bytes) return QB_OK;
    hipStream_t s = qb_stream(stream);
    if (((uintptr_t)buf_d & 15) == 0 && (bytes & 15) == 0) {
        const int64_t n16 = (int64_t)(bytes / 16);
        const int blocks = (int)std::min<int64_t>((n16 + 255) / 256, 4096);
        k_zero16<<<blocks, 256, 0, s>>>((uint4 *)buf_d, n16);
    } else {
        const int blocks = (int)std::min<int64_t>(((int64_t)bytes + 255) / 256, 4096);
        k_zero1<<<blocks, 256, 0, s>>>((uint8_t *)buf_d, (int64_t)bytes);
    }
    QB_LAUNCH_CHECK();
    return QB_OK;
}

// ------------------------------------------------------------------ host tables
// Cosine-waveform temperature and its quantised Metropolis thresholds.  The
// expressions are written in the order the header documents so that any
// IEEE-754 double implementation with the same libm reproduces them exactly.
extern "C" qb_status qb_threshold_table(int32_t nsw, int32_t B, double tmax, double tmin,
                                       int32_t *thr_h)
{
    if (nsw < 1 || B < 1 || B > 16 || !thr_h || !(tmax >= 0.0) || !(tmin >= 0.0)) return QB_E_ARG;
    const int nb = 1 << B;
    for (int s = 0; s < nsw; ++s) {
        double T;
        if (nsw <= 1)
            T = tmax;
        else
            T = tmin + 0.5 * (tmax - tmin) * (1.0 + cos(M_PI * (double)s / (double)(nsw - 1)));
        for (int b = 0; b < nb; ++b) {
            const double v = T * (-log(((double)b + 0.5) / (double)nb));
            thr_h[(int64_t)s * nb + b] = v >= 2147483647.0 ? 2147483647 : (int32_t)floor(v);
        }
    }
    return QB_OK;
}

extern "C" double qb_mutation_rate(int32_t t)
{
    return 0.3 * (1.0 + cos(M_PI * (double)t / 15.0)) * pow(0.99, (double)t);
}
