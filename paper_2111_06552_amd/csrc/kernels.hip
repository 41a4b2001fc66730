// HIP kernels of the GCG eigensolver for gfx950 (MI355X, CDNA4).
//
// Memory layout: every block of vectors is row-major (n x ld); sparse matrices
// are CSR with int32 indices.  Row-streaming kernels (SpMM, CG updates) give
// each work-group a contiguous chunk of rows; work-group ids are remapped so
// that the chunks resident on one XCD (work-groups are dispatched round-robin
// over the 8 XCDs) are contiguous, which keeps the stencil neighbours of a
// chunk in that XCD's L2.  Reductions over rows write one partial per
// work-group and column and are finished by a single work-group in a fixed
// order, so every result is bitwise reproducible.
//
// The dense tall-skinny products (block inner products X^T Y and the
// multi-vector combinations X S of Section 3.2) run on the FP64 matrix cores
// with v_mfma_f64_16x16x4f64.
#include "internal.h"

#include <algorithm>

namespace gcge {

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 operand layout (lane l of the wave, li = l % 16,
// lk = l / 16): lane l supplies A[li][lk] and B[lk][li]; accumulator register
// r of lane l holds D[lk + 4 r][li].

constexpr int NXCD = 8;

// Logical block id such that blocks dispatched to the same XCD get a
// contiguous range of logical ids (bijection on [0, nb)).
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
    const int q = nb / NXCD, r = nb % NXCD, x = bid % NXCD, j = bid / NXCD;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + j;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

int row_chunks(int64_t n, int k) {
    (void)k;
    int64_t per = std::max<int64_t>(64, (n + 2047) / 2048);
    return (int)((n + per - 1) / per);
}

static inline int64_t rows_per_chunk(int64_t n, int nparts) { return (n + nparts - 1) / nparts; }

// ---------------------------------------------------------------------------
// SpMM: one group of G lanes per row, lane l of the group owns columns
// l, l + G, ... (CT of them).
// ---------------------------------------------------------------------------
template <typename T, int G, int CT, int MODE, int RED>
__global__ __launch_bounds__(256) void k_spmm(int64_t n, const int32_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ colind, const T *__restrict__ va,
                                              const T *__restrict__ vb, const T *__restrict__ dg,
                                              const T *__restrict__ sigma, const T *__restrict__ X, int64_t ldx,
                                              int k, T *__restrict__ Y, int64_t ldy, const T *__restrict__ Z,
                                              int64_t ldz, T *__restrict__ part, int nparts, int64_t rows_per,
                                              const int *__restrict__ skip) {
    if (skip != nullptr && skip[0] == 0) return;
    constexpr int NG = 256 / G;
    const int tid = threadIdx.x, grp = tid / G, lig = tid % G;
    const int chunk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t r0 = (int64_t)chunk * rows_per;
    const int64_t r1 = min(n, r0 + rows_per);
    int col[CT];
    bool cv[CT];
    T sg[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        col[t] = lig + G * t;
        cv[t] = col[t] < k;
        sg[t] = (MODE != 0 && cv[t]) ? sigma[col[t]] : T(0);
    }
    T red1[CT], red2[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) red1[t] = red2[t] = T(0);

    for (int64_t row = r0 + grp; row < r1; row += NG) {
        int e0 = rowptr[row], e1 = rowptr[row + 1];
        if (G == 64) {
            e0 = __builtin_amdgcn_readfirstlane(e0);
            e1 = __builtin_amdgcn_readfirstlane(e1);
        }
        T acc[CT], accb[CT];
#pragma unroll
        for (int t = 0; t < CT; ++t) acc[t] = accb[t] = T(0);
#pragma unroll 4
        for (int e = e0; e < e1; ++e) {
            const int64_t c = colind[e];
            const T a = va[e];
            const T b = (MODE == 2) ? vb[e] : T(0);
            const T *xr = X + c * ldx;
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                if (cv[t]) {
                    const T x = xr[col[t]];
                    acc[t] = fma(a, x, acc[t]);
                    if (MODE == 2) accb[t] = fma(b, x, accb[t]);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            if (!cv[t]) continue;
            T y = acc[t], bx = T(0);
            if (MODE == 1) {
                const T xs = X[row * ldx + col[t]];
                bx = (dg != nullptr) ? dg[row] * xs : xs;
                y = fma(-sg[t], bx, y);
            } else if (MODE == 2) {
                bx = accb[t];
                y = fma(-sg[t], bx, y);
            }
            Y[row * ldy + col[t]] = y;
            if (RED == 1) {
                red1[t] = fma(y, y, red1[t]);
                red2[t] = fma(bx, bx, red2[t]);
            } else if (RED == 2) {
                red1[t] = fma(y, Z[row * ldz + col[t]], red1[t]);
            }
        }
    }
    if (RED != 0) {
        __shared__ T sh[2][NG][G * CT];
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            sh[0][grp][lig + G * t] = red1[t];
            sh[1][grp][lig + G * t] = red2[t];
        }
        __syncthreads();
        for (int c = tid; c < G * CT; c += 256) {
            if (c >= k) continue;
            T s1 = T(0), s2 = T(0);
            for (int g = 0; g < NG; ++g) {
                s1 += sh[0][g][c];
                s2 += sh[1][g][c];
            }
            part[(size_t)c * nparts + chunk] = s1;
            if (RED == 1) part[(size_t)(k + c) * nparts + chunk] = s2;
        }
    }
}

template <typename T, int MODE, int RED>
static hipError_t spmm_dispatch(const DevCsr<T> &A, const T *vb, const T *dg, const T *sigma, const T *X,
                                int64_t ldx, int k, T *Y, int64_t ldy, const T *Z, int64_t ldz, T *part,
                                int nparts, const int *skip, hipStream_t st) {
    const int64_t rp = rows_per_chunk(A.n, nparts);
    dim3 grid(nparts), block(256);
#define GCGE_SPMM_LAUNCH(G, CT)                                                                          \
    hipLaunchKernelGGL((k_spmm<T, G, CT, MODE, RED>), grid, block, 0, st, A.n, A.rowptr, A.colind, A.val, \
                       vb, dg, sigma, X, ldx, k, Y, ldy, Z, ldz, part, nparts, rp, skip)
    if (k <= 16) GCGE_SPMM_LAUNCH(16, 1);
    else if (k <= 32) GCGE_SPMM_LAUNCH(32, 1);
    else if (k <= 64) GCGE_SPMM_LAUNCH(64, 1);
    else GCGE_SPMM_LAUNCH(64, 2);
#undef GCGE_SPMM_LAUNCH
    return hipGetLastError();
}

template <typename T>
hipError_t spmm(const DevCsr<T> &A, const T *vb, const T *dg, const T *sigma, int mode, int red, const T *X,
                int64_t ldx, int k, T *Y, int64_t ldy, const T *Z, int64_t ldz, T *part, int nparts,
                hipStream_t st) {
    if (A.n == 0 || k == 0) return hipSuccess;
    if (k > 128) return hipErrorInvalidValue;
    if (nparts <= 0) {
        if (red != 0) return hipErrorInvalidValue;
        nparts = row_chunks(A.n, k);
    }
#define GCGE_SPMM_CASE(M, R) \
    if (mode == M && red == R) return spmm_dispatch<T, M, R>(A, vb, dg, sigma, X, ldx, k, Y, ldy, Z, ldz, part, nparts, nullptr, st)
    GCGE_SPMM_CASE(0, 0);
    GCGE_SPMM_CASE(1, 0);
    GCGE_SPMM_CASE(2, 0);
    GCGE_SPMM_CASE(1, 1);
    GCGE_SPMM_CASE(2, 1);
    GCGE_SPMM_CASE(0, 2);
#undef GCGE_SPMM_CASE
    return hipErrorInvalidValue;
}

template hipError_t spmm<double>(const DevCsr<double> &, const double *, const double *, const double *, int, int,
                                 const double *, int64_t, int, double *, int64_t, const double *, int64_t,
                                 double *, int, hipStream_t);
template <>
hipError_t spmm<float>(const DevCsr<float> &A, const float *vb, const float *dg, const float *sigma, int mode,
                       int red, const float *X, int64_t ldx, int k, float *Y, int64_t ldy, const float *Z,
                       int64_t ldz, float *part, int nparts, hipStream_t st) {
    if (A.n == 0 || k == 0) return hipSuccess;
    if (k > 128) return hipErrorInvalidValue;
    if (nparts <= 0) {
        if (red != 0) return hipErrorInvalidValue;
        nparts = row_chunks(A.n, k);
    }
    if (mode == 0 && red == 0)
        return spmm_dispatch<float, 0, 0>(A, vb, dg, sigma, X, ldx, k, Y, ldy, Z, ldz, part, nparts, nullptr, st);
    if (mode == 0 && red == 2)
        return spmm_dispatch<float, 0, 2>(A, vb, dg, sigma, X, ldx, k, Y, ldy, Z, ldz, part, nparts, nullptr, st);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t cg_spmm(const DevCsr<T> &M, const T *p, T *q, int64_t ld, int k, T *part, int nparts, const int *flags,
                   hipStream_t st) {
    if (M.n == 0 || k == 0) return hipSuccess;
    if (k > 128) return hipErrorInvalidValue;
    return spmm_dispatch<T, 0, 2>(M, nullptr, nullptr, nullptr, p, ld, k, q, ld, p, ld, part, nparts, flags, st);
}
template hipError_t cg_spmm<double>(const DevCsr<double> &, const double *, double *, int64_t, int, double *, int,
                                    const int *, hipStream_t);
template hipError_t cg_spmm<float>(const DevCsr<float> &, const float *, float *, int64_t, int, float *, int,
                                   const int *, hipStream_t);

// ---------------------------------------------------------------------------
// fixed-order column sums of partials (one work-group, 16 waves)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T colsum_wave(const T *__restrict__ part, int nparts, int c, int lane) {
    T s = T(0);
    for (int p = lane; p < nparts; p += 64) s += part[(size_t)c * nparts + p];
    return wave_sum(s);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_colsum(const T *__restrict__ part, int nparts, int k, double *out) {
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int c = w; c < k; c += 16) {
        const T s = colsum_wave(part, nparts, c, lane);
        if (lane == 0) out[c] = (double)s;
    }
}

template <typename T>
hipError_t colsum(const T *part, int nparts, int k, double *out, hipStream_t st) {
    if (k == 0) return hipSuccess;
    hipLaunchKernelGGL(k_colsum<T>, dim3(1), dim3(1024), 0, st, part, nparts, k, out);
    return hipGetLastError();
}
template hipError_t colsum<double>(const double *, int, int, double *, hipStream_t);
template hipError_t colsum<float>(const float *, int, int, double *, hipStream_t);

// ---------------------------------------------------------------------------
// column-wise CG (STEP 6)
// ---------------------------------------------------------------------------
template <typename T, int G, int CT>
__global__ __launch_bounds__(256) void k_cg_init(int64_t n, int k, const double *__restrict__ R, int64_t ldr,
                                                 const double *__restrict__ rscale, T *__restrict__ r,
                                                 T *__restrict__ p, T *__restrict__ x, int64_t ld,
                                                 T *__restrict__ part, int nparts, int64_t rows_per) {
    constexpr int NG = 256 / G;
    const int tid = threadIdx.x, grp = tid / G, lig = tid % G;
    const int chunk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t r0 = (int64_t)chunk * rows_per, r1 = min(n, r0 + rows_per);
    T acc[CT];
    double sc[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        acc[t] = T(0);
        const int c = lig + G * t;
        sc[t] = (c < k && rscale != nullptr) ? rscale[c] : 1.0;
    }
    for (int64_t row = r0 + grp; row < r1; row += NG) {
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            const int c = lig + G * t;
            if (c >= k) continue;
            const T v = (T)(R[row * ldr + c] * sc[t]);
            r[row * ld + c] = v;
            p[row * ld + c] = v;
            x[row * ld + c] = T(0);
            acc[t] = fma(v, v, acc[t]);
        }
    }
    __shared__ T sh[NG][G * CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) sh[grp][lig + G * t] = acc[t];
    __syncthreads();
    for (int c = tid; c < G * CT; c += 256) {
        if (c >= k) continue;
        T s = T(0);
        for (int g = 0; g < NG; ++g) s += sh[g][c];
        part[(size_t)c * nparts + chunk] = s;
    }
}

template <typename T, int G, int CT>
__global__ __launch_bounds__(256) void k_cg_update_r(int64_t n, int k, const T *__restrict__ q,
                                                     T *__restrict__ r, int64_t ld, T *__restrict__ part,
                                                     int nparts, int64_t rows_per, CgState<T> cs) {
    if (cs.flags[1] == 0) return;
    constexpr int NG = 256 / G;
    const int tid = threadIdx.x, grp = tid / G, lig = tid % G;
    const int chunk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t r0 = (int64_t)chunk * rows_per, r1 = min(n, r0 + rows_per);
    T acc[CT], al[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        acc[t] = T(0);
        const int c = lig + G * t;
        al[t] = (c < k) ? cs.alpha[c] : T(0);
    }
    for (int64_t row = r0 + grp; row < r1; row += NG) {
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            const int c = lig + G * t;
            if (c >= k) continue;
            const T v = fma(-al[t], q[row * ld + c], r[row * ld + c]);
            r[row * ld + c] = v;
            acc[t] = fma(v, v, acc[t]);
        }
    }
    __shared__ T sh[NG][G * CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) sh[grp][lig + G * t] = acc[t];
    __syncthreads();
    for (int c = tid; c < G * CT; c += 256) {
        if (c >= k) continue;
        T s = T(0);
        for (int g = 0; g < NG; ++g) s += sh[g][c];
        part[(size_t)c * nparts + chunk] = s;
    }
}

template <typename T, int G, int CT>
__global__ __launch_bounds__(256) void k_cg_update_xp(int64_t n, int k, T *__restrict__ x, T *__restrict__ p,
                                                      const T *__restrict__ r, int64_t ld, int64_t rows_per,
                                                      CgState<T> cs) {
    if (cs.flags[1] == 0) return;
    constexpr int NG = 256 / G;
    const int tid = threadIdx.x, grp = tid / G, lig = tid % G;
    const int chunk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t r0 = (int64_t)chunk * rows_per, r1 = min(n, r0 + rows_per);
    T al[CT], be[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        const int c = lig + G * t;
        al[t] = (c < k) ? cs.alpha[c] : T(0);
        be[t] = (c < k) ? cs.beta[c] : T(0);
    }
    for (int64_t row = r0 + grp; row < r1; row += NG) {
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            const int c = lig + G * t;
            if (c >= k) continue;
            const T pv = p[row * ld + c];
            x[row * ld + c] = fma(al[t], pv, x[row * ld + c]);
            p[row * ld + c] = fma(be[t], pv, r[row * ld + c]);
        }
    }
}

// flags[0] = active columns, flags[1] = columns with a nonzero step this iteration
template <typename T>
__global__ __launch_bounds__(1024) void k_cg_init_finish(const T *__restrict__ part, int nparts, int k,
                                                         CgState<T> cs) {
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int c = w; c < k; c += 16) {
        const T s = colsum_wave(part, nparts, c, lane);
        if (lane == 0) {
            cs.rr[c] = s;
            cs.rr0[c] = s;
            cs.active[c] = (s > T(0)) ? 1 : 0;
            cs.its[c] = 0;
            cs.alpha[c] = T(0);
            cs.beta[c] = T(0);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int na = 0;
        for (int c = 0; c < k; ++c) na += cs.active[c];
        cs.flags[0] = na;
        cs.flags[1] = 0;
    }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_cg_alpha(const T *__restrict__ part, int nparts, int k, CgState<T> cs) {
    if (cs.flags[0] == 0) {
        if (threadIdx.x == 0) cs.flags[1] = 0;
        return;
    }
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int c = w; c < k; c += 16) {
        const T pq = colsum_wave(part, nparts, c, lane);
        if (lane == 0) {
            T al = T(0);
            if (cs.active[c]) {
                if (pq > T(0)) {
                    al = cs.rr[c] / pq;
                    cs.its[c] += 1;
                } else {
                    cs.active[c] = 0;   // p^T (A - theta B) p <= 0: freeze the column
                }
            }
            cs.alpha[c] = al;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int live = 0, na = 0;
        for (int c = 0; c < k; ++c) {
            live += (cs.alpha[c] != T(0)) ? 1 : 0;
            na += cs.active[c];
        }
        cs.flags[0] = na;
        cs.flags[1] = live;
    }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_cg_beta(const T *__restrict__ part, int nparts, int k, T tol2,
                                                  CgState<T> cs) {
    if (cs.flags[1] == 0) return;
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int c = w; c < k; c += 16) {
        const T rrn = colsum_wave(part, nparts, c, lane);
        if (lane == 0) {
            T be = T(0);
            if (cs.alpha[c] != T(0)) {
                be = rrn / cs.rr[c];
                cs.rr[c] = rrn;
                if (rrn <= tol2 * cs.rr0[c]) cs.active[c] = 0;
            }
            cs.beta[c] = be;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int na = 0;
        for (int c = 0; c < k; ++c) na += cs.active[c];
        cs.flags[0] = na;
    }
}

#define GCGE_ROW_LAUNCH(KERNEL, T, k, ...)                                                              \
    do {                                                                                               \
        if ((k) <= 16) hipLaunchKernelGGL((KERNEL<T, 16, 1>), grid, block, 0, st, __VA_ARGS__);        \
        else if ((k) <= 32) hipLaunchKernelGGL((KERNEL<T, 32, 1>), grid, block, 0, st, __VA_ARGS__);   \
        else if ((k) <= 64) hipLaunchKernelGGL((KERNEL<T, 64, 1>), grid, block, 0, st, __VA_ARGS__);   \
        else hipLaunchKernelGGL((KERNEL<T, 64, 2>), grid, block, 0, st, __VA_ARGS__);                  \
    } while (0)

template <typename T>
hipError_t cg_init(const double *R, int64_t ldr, const double *rscale, int k, int64_t n, T *r, T *p, T *x,
                   int64_t ld, T *part, int nparts, CgState<T> cs, hipStream_t st) {
    (void)cs;
    if (k > 128) return hipErrorInvalidValue;
    dim3 grid(nparts), block(256);
    const int64_t rp = rows_per_chunk(n, nparts);
    GCGE_ROW_LAUNCH(k_cg_init, T, k, n, k, R, ldr, rscale, r, p, x, ld, part, nparts, rp);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_init_finish(const T *part, int nparts, int k, CgState<T> cs, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_init_finish<T>, dim3(1), dim3(1024), 0, st, part, nparts, k, cs);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_alpha(const T *part, int nparts, int k, CgState<T> cs, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_alpha<T>, dim3(1), dim3(1024), 0, st, part, nparts, k, cs);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_update_r(int64_t n, int k, const T *q, T *r, int64_t ld, T *part, int nparts, CgState<T> cs,
                       hipStream_t st) {
    if (k > 128) return hipErrorInvalidValue;
    dim3 grid(nparts), block(256);
    const int64_t rp = rows_per_chunk(n, nparts);
    GCGE_ROW_LAUNCH(k_cg_update_r, T, k, n, k, q, r, ld, part, nparts, rp, cs);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_beta(const T *part, int nparts, int k, double rel_tol, CgState<T> cs, hipStream_t st) {
    const T tol2 = (T)(rel_tol * rel_tol);
    hipLaunchKernelGGL(k_cg_beta<T>, dim3(1), dim3(1024), 0, st, part, nparts, k, tol2, cs);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_update_xp(int64_t n, int k, T *x, T *p, const T *r, int64_t ld, CgState<T> cs, hipStream_t st) {
    if (k > 128) return hipErrorInvalidValue;
    const int nparts = row_chunks(n, k);
    dim3 grid(nparts), block(256);
    const int64_t rp = rows_per_chunk(n, nparts);
    GCGE_ROW_LAUNCH(k_cg_update_xp, T, k, n, k, x, p, r, ld, rp, cs);
    return hipGetLastError();
}

#define GCGE_CG_INST(T)                                                                                          \
    template hipError_t cg_init<T>(const double *, int64_t, const double *, int, int64_t, T *, T *, T *, int64_t, \
                                   T *, int, CgState<T>, hipStream_t);                                            \
    template hipError_t cg_init_finish<T>(const T *, int, int, CgState<T>, hipStream_t);                          \
    template hipError_t cg_alpha<T>(const T *, int, int, CgState<T>, hipStream_t);                                \
    template hipError_t cg_update_r<T>(int64_t, int, const T *, T *, int64_t, T *, int, CgState<T>, hipStream_t); \
    template hipError_t cg_beta<T>(const T *, int, int, double, CgState<T>, hipStream_t);                         \
    template hipError_t cg_update_xp<T>(int64_t, int, T *, T *, const T *, int64_t, CgState<T>, hipStream_t);
GCGE_CG_INST(double)
GCGE_CG_INST(float)
#undef GCGE_CG_INST

// ---------------------------------------------------------------------------
// Block inner product C = X^T diag(d) Y on the FP64 matrix cores.
// A work-group (4 waves) owns one (TM x TN) output tile over one chunk of
// rows; each wave streams every 4th group of 4 rows and feeds them straight
// from global memory into v_mfma_f64_16x16x4f64 (the 16 consecutive columns
// of a row that one MFMA operand needs are one 128-byte load).  The four
// waves' tiles are summed in LDS in a fixed order and written as one partial;
// a second kernel sums the partials over the chunks.
// ---------------------------------------------------------------------------
struct GTile {
    const double *xp;
    int64_t ldx;
    int xcol0;   // first column of the strip within its segment
    int ncol;    // valid columns of the strip (<= TM)
    int crow0;   // row of C that holds the strip's first column
};
constexpr int MAX_GT = 48;
struct GramParams {
    int64_t n;
    int ntile;
    GTile t[MAX_GT];
    const double *Y;
    int64_t ldy;
    int k;
    int nyt;
    const double *d;
    double *part;
    int nchunk;
    int64_t rows_per;
};

template <int MB, int NB>
__global__ __launch_bounds__(256) void k_gram(GramParams P) {
    constexpr int TM = 16 * MB, TN = 16 * NB;
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int per_chunk = P.ntile * P.nyt;
    const int chunk = lid / per_chunk, rem = lid % per_chunk;
    const int ti = rem / P.nyt, yt = rem % P.nyt;
    const GTile tl = P.t[ti];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, li = lane % 16, lk = lane / 16;
    const int64_t r0 = (int64_t)chunk * P.rows_per, r1 = min(P.n, r0 + P.rows_per);
    d4 acc[MB][NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    int xc[MB], yc[NB];
    bool xv[MB], yv[NB];
#pragma unroll
    for (int a = 0; a < MB; ++a) {
        xc[a] = tl.xcol0 + a * 16 + li;
        xv[a] = (a * 16 + li) < tl.ncol;
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        yc[b] = yt * TN + b * 16 + li;
        yv[b] = yc[b] < P.k;
    }
    for (int64_t rb = r0 + wave * 4; rb < r1; rb += 16) {
        const int64_t row = rb + lk;
        const bool rv = row < r1;
        const double *xr = tl.xp + row * tl.ldx;
        const double *yr = P.Y + row * P.ldy;
        const double dw = (P.d != nullptr && rv) ? P.d[row] : 1.0;
        double av[MB], bv[NB];
#pragma unroll
        for (int a = 0; a < MB; ++a) av[a] = (rv && xv[a]) ? xr[xc[a]] : 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) bv[b] = (rv && yv[b]) ? yr[yc[b]] * dw : 0.0;
#pragma unroll
        for (int a = 0; a < MB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __shared__ double sh[TM * TN];
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int a = 0; a < MB; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int idx = (a * 16 + lk + 4 * r) * TN + b * 16 + li;
                        sh[idx] = (w == 0 ? 0.0 : sh[idx]) + acc[a][b][r];
                    }
        }
        __syncthreads();
    }
    double *dst = P.part + ((size_t)(ti * P.nyt + yt) * P.nchunk + chunk) * (TM * TN);
    for (int e = threadIdx.x; e < TM * TN; e += 256) dst[e] = sh[e];
}

template <int MB, int NB>
__global__ __launch_bounds__(256) void k_gram_reduce(GramParams P, double *C, int64_t ldc) {
    constexpr int TM = 16 * MB, TN = 16 * NB;
    const int tp = blockIdx.x;
    const int ti = tp / P.nyt, yt = tp % P.nyt;
    const GTile tl = P.t[ti];
    const double *src = P.part + (size_t)tp * P.nchunk * (TM * TN);
    for (int e = threadIdx.x; e < TM * TN; e += 256) {
        const int i = e / TN, j = e % TN;
        const int cj = yt * TN + j;
        if (i >= tl.ncol || cj >= P.k) continue;
        double s = 0.0;
        for (int c = 0; c < P.nchunk; ++c) s += src[(size_t)c * (TM * TN) + e];
        C[(int64_t)(tl.crow0 + i) * ldc + cj] = s;
    }
}

hipError_t gram(int64_t n, const Segs &X, const double *Y, int64_t ldy, int k, const double *d, double *C,
                int64_t ldc, Workspace &ws, hipStream_t st) {
    const int m = X.total();
    if (m == 0 || k == 0) return hipSuccess;
    int MB, NB;
    if (m <= 16 && k <= 16) { MB = 1; NB = 1; }
    else if (m <= 32 && k <= 32) { MB = 2; NB = 2; }
    else if (k <= 16) { MB = 4; NB = 1; }
    else { MB = 4; NB = 4; }
    const int TM = 16 * MB, TN = 16 * NB;
    GramParams P;
    P.n = n;
    P.ntile = 0;
    int crow = 0;
    for (int s = 0; s < X.nseg; ++s) {
        for (int c0 = 0; c0 < X.s[s].ncol; c0 += TM) {
            if (P.ntile >= MAX_GT) return hipErrorInvalidValue;
            P.t[P.ntile++] = GTile{X.s[s].p, X.s[s].ld, c0, std::min(TM, X.s[s].ncol - c0), crow + c0};
        }
        crow += X.s[s].ncol;
    }
    P.Y = Y;
    P.ldy = ldy;
    P.k = k;
    P.nyt = (k + TN - 1) / TN;
    P.d = d;
    const int tiles = P.ntile * P.nyt;
    int nchunk = std::max(1, 2048 / tiles);
    nchunk = (int)std::min<int64_t>(nchunk, std::max<int64_t>(1, (n + 255) / 256));
    int64_t rp = (n + nchunk - 1) / nchunk;
    rp = (rp + 15) / 16 * 16;
    nchunk = (int)((n + rp - 1) / rp);
    P.nchunk = nchunk;
    P.rows_per = rp;
    hipError_t e = ws.ensure_part((size_t)tiles * nchunk * TM * TN * sizeof(double));
    if (e != hipSuccess) return e;
    P.part = ws.part;
    dim3 grid(tiles * nchunk), block(256);
#define GCGE_GRAM(MBv, NBv)                                                                     \
    if (MB == MBv && NB == NBv) {                                                               \
        hipLaunchKernelGGL((k_gram<MBv, NBv>), grid, block, 0, st, P);                          \
        hipLaunchKernelGGL((k_gram_reduce<MBv, NBv>), dim3(tiles), block, 0, st, P, C, ldc);     \
    }
    GCGE_GRAM(1, 1)
    GCGE_GRAM(2, 2)
    GCGE_GRAM(4, 1)
    GCGE_GRAM(4, 4)
#undef GCGE_GRAM
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Y = alpha * X S + beta * Y on the FP64 matrix cores: 64 x 64 output tiles,
// 4 waves of 32 x 32 each, the X and S tiles staged through LDS in K-chunks of
// 16 columns.  X is read as up to MAX_SEG column segments.
// ---------------------------------------------------------------------------
struct GemmParams {
    int64_t n;
    int nseg;
    Seg s[MAX_SEG];
    int soff[MAX_SEG];
    const double *S;
    int64_t lds;
    int k;
    double alpha, beta;
    double *Y;
    int64_t ldy;
    int nct;
};

__global__ __launch_bounds__(256) void k_gemm(GemmParams P) {
    constexpr int BM = 64, BN = 64, BK = 16;
    __shared__ double Vt[BM][BK + 1];
    __shared__ double St[BK][BN];
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int rt = lid / P.nct, ct = lid % P.nct;
    const int64_t row0 = (int64_t)rt * BM;
    const int col0 = ct * BN;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, li = lane % 16, lk = lane / 16;
    const int wr = wave / 2, wc = wave % 2;
    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    for (int sgi = 0; sgi < P.nseg; ++sgi) {
        const Seg sg = P.s[sgi];
        const int soff = P.soff[sgi];
        for (int kc = 0; kc < sg.ncol; kc += BK) {
            {
                const int r = tid / 4, c4 = (tid % 4) * 4;
                const int64_t row = row0 + r;
                const bool rv = row < P.n;
                const double *src = sg.p + row * sg.ld + kc + c4;
#pragma unroll
                for (int q = 0; q < 4; ++q) Vt[r][c4 + q] = (rv && kc + c4 + q < sg.ncol) ? src[q] : 0.0;
            }
            {
                const int kr = tid / 16, c4 = (tid % 16) * 4;
                const int srow = kc + kr;
                const bool sv = srow < sg.ncol;
                const double *src = P.S + (int64_t)(soff + srow) * P.lds + col0 + c4;
#pragma unroll
                for (int q = 0; q < 4; ++q) St[kr][c4 + q] = (sv && col0 + c4 + q < P.k) ? src[q] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < BK; ks += 4) {
                double av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) av[a] = Vt[wr * 32 + a * 16 + li][ks + lk];
#pragma unroll
                for (int b = 0; b < 2; ++b) bv[b] = St[ks + lk][wc * 32 + b * 16 + li];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + wr * 32 + a * 16 + lk + 4 * r;
                const int col = col0 + wc * 32 + b * 16 + li;
                if (row < P.n && col < P.k) {
                    double v = P.alpha * acc[a][b][r];
                    if (P.beta != 0.0) v = fma(P.beta, P.Y[row * P.ldy + col], v);
                    P.Y[row * P.ldy + col] = v;
                }
            }
}

hipError_t gemm(int64_t n, const Segs &X, const double *S, int64_t lds, int k, double alpha, double beta,
                double *Y, int64_t ldy, hipStream_t st) {
    if (n == 0 || k == 0) return hipSuccess;
    GemmParams P;
    P.n = n;
    P.nseg = X.nseg;
    int off = 0;
    for (int s = 0; s < X.nseg; ++s) {
        P.s[s] = X.s[s];
        P.soff[s] = off;
        off += X.s[s].ncol;
    }
    P.S = S;
    P.lds = lds;
    P.k = k;
    P.alpha = alpha;
    P.beta = beta;
    P.Y = Y;
    P.ldy = ldy;
    P.nct = (k + 63) / 64;
    const int64_t nrt = (n + 63) / 64;
    const int64_t nb = nrt * P.nct;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gemm, dim3((unsigned)nb), dim3(256), 0, st, P);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small elementwise kernels
// ---------------------------------------------------------------------------
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_copy_cols(int64_t n, int k, const TI *__restrict__ X, int64_t ldx,
                                                   TO *__restrict__ Y, int64_t ldy, const double *__restrict__ scale) {
    const int64_t total = n * k;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
        const int64_t i = t / k;
        const int j = (int)(t % k);
        double v = (double)X[i * ldx + j];
        if (scale != nullptr) v *= scale[j];
        Y[i * ldy + j] = (TO)v;
    }
}

static inline unsigned ew_grid(int64_t total) {
    int64_t b = (total + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

template <typename TI, typename TO>
hipError_t copy_cols(int64_t n, int k, const TI *X, int64_t ldx, TO *Y, int64_t ldy, const double *scale,
                     hipStream_t st) {
    if (n == 0 || k == 0) return hipSuccess;
    hipLaunchKernelGGL((k_copy_cols<TI, TO>), dim3(ew_grid(n * k)), dim3(256), 0, st, n, k, X, ldx, Y, ldy, scale);
    return hipGetLastError();
}
template hipError_t copy_cols<double, double>(int64_t, int, const double *, int64_t, double *, int64_t,
                                              const double *, hipStream_t);
template hipError_t copy_cols<float, double>(int64_t, int, const float *, int64_t, double *, int64_t,
                                             const double *, hipStream_t);
template hipError_t copy_cols<double, float>(int64_t, int, const double *, int64_t, float *, int64_t,
                                             const double *, hipStream_t);

// one thread per row; columns move left in increasing order, so a source is
// always read before its slot is overwritten
__global__ __launch_bounds__(256) void k_shift_cols_left(int64_t n, double *X, int64_t ld, int dst, int src,
                                                         int cnt) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double *row = X + i * ld;
        for (int j = 0; j < cnt; ++j) row[dst + j] = row[src + j];
    }
}

hipError_t shift_cols_left(int64_t n, double *X, int64_t ld, int dst, int src, int cnt, hipStream_t st) {
    if (n == 0 || cnt == 0 || dst == src) return hipSuccess;
    if (dst > src) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_shift_cols_left, dim3(ew_grid(n)), dim3(256), 0, st, n, X, ld, dst, src, cnt);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_gather_cols(int64_t n, int k, const double *__restrict__ X, int64_t ldx,
                                                     const int *__restrict__ perm, double *__restrict__ Y,
                                                     int64_t ldy) {
    const int64_t total = n * k;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
        const int64_t i = t / k;
        const int j = (int)(t % k);
        Y[i * ldy + j] = X[i * ldx + perm[j]];
    }
}

hipError_t gather_cols(int64_t n, int k, const double *X, int64_t ldx, const int *perm, double *Y, int64_t ldy,
                       hipStream_t st) {
    if (n == 0 || k == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_cols, dim3(ew_grid(n * k)), dim3(256), 0, st, n, k, X, ldx, perm, Y, ldy);
    return hipGetLastError();
}

// SplitMix64 (Steele, Lea, Flood 2014): draw idx of the stream seeded with s is
// mix64(s + (idx + 1) * 0x9E3779B97F4A7C15).
__device__ __forceinline__ uint64_t splitmix64_draw(uint64_t seed, uint64_t idx) {
    uint64_t z = seed + (idx + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_fill_random(int64_t n, int k, int col0, uint64_t seed, double *X,
                                                     int64_t ld) {
    const int64_t total = n * k;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
        const int64_t i = t / k;
        const int j = (int)(t % k);
        const uint64_t z = splitmix64_draw(seed, (uint64_t)(col0 + j) * (uint64_t)n + (uint64_t)i);
        const double u = (double)(z >> 11) * 0x1.0p-53;
        X[i * ld + j] = 2.0 * u - 1.0;
    }
}

hipError_t fill_random(int64_t n, int k, int col0, uint64_t seed, double *X, int64_t ld, hipStream_t st) {
    if (n == 0 || k == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_random, dim3(ew_grid(n * k)), dim3(256), 0, st, n, k, col0, seed, X, ld);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_shift_values(int64_t nnz, const double *__restrict__ a,
                                                      const double *__restrict__ b, double theta, double *m) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * 256)
        m[e] = (b != nullptr) ? fma(-theta, b[e], a[e]) : a[e];
}

__global__ __launch_bounds__(256) void k_shift_diag(int64_t n, const int32_t *__restrict__ dpos,
                                                    const double *__restrict__ dg, double theta, double *m) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        m[dpos[i]] = fma(-theta, (dg != nullptr) ? dg[i] : 1.0, m[dpos[i]]);
}

__global__ __launch_bounds__(256) void k_to_f32(int64_t nnz, const double *__restrict__ m, float *m32) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * 256)
        m32[e] = (float)m[e];
}

hipError_t shift_values(int64_t nnz, const double *a, const double *b, int64_t n, const int32_t *dpos,
                        const double *dg, double theta, double *m, float *m32, hipStream_t st) {
    if (nnz > 0)
        hipLaunchKernelGGL(k_shift_values, dim3(ew_grid(nnz)), dim3(256), 0, st, nnz, a, b, theta, m);
    if (b == nullptr && dpos != nullptr && theta != 0.0 && n > 0)
        hipLaunchKernelGGL(k_shift_diag, dim3(ew_grid(n)), dim3(256), 0, st, n, dpos, dg, theta, m);
    if (m32 != nullptr && nnz > 0) hipLaunchKernelGGL(k_to_f32, dim3(ew_grid(nnz)), dim3(256), 0, st, nnz, m, m32);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// eigenvalue gradients over a sparsity pattern: one wave per row, lanes over
// the eigenpairs; each stored entry is a fixed-order wave reduction.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pattern_grad(int64_t n, const int32_t *__restrict__ rowptr,
                                                      const int32_t *__restrict__ colind,
                                                      const double *__restrict__ X, int64_t ldx, int nev,
                                                      const double *__restrict__ w, double *__restrict__ gval) {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t row = (int64_t)blockIdx.x * 4 + wave; row < n; row += nw) {
        const int e0 = __builtin_amdgcn_readfirstlane(rowptr[row]);
        const int e1 = __builtin_amdgcn_readfirstlane(rowptr[row + 1]);
        double xr[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = lane + 64 * t;
            xr[t] = (c < nev) ? X[row * ldx + c] * w[c] : 0.0;
        }
        for (int e = e0; e < e1; ++e) {
            const int64_t cc = colind[e];
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int c = lane + 64 * t;
                if (c < nev) s = fma(xr[t], X[cc * ldx + c], s);
            }
            s = wave_sum(s);
            if (lane == 0) gval[e] = s;
        }
    }
}

hipError_t pattern_grad(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *X, int64_t ldx,
                        int nev, const double *w, double *gval, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (nev > 256) return hipErrorInvalidValue;
    const int64_t blocks = std::min<int64_t>((n + 3) / 4, 65536);
    hipLaunchKernelGGL(k_pattern_grad, dim3((unsigned)blocks), dim3(256), 0, st, n, rowptr, colind, X, ldx, nev, w,
                       gval);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_diag_grad(int64_t n, const double *__restrict__ X, int64_t ldx, int nev,
                                                   const double *__restrict__ w, double *__restrict__ gd) {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t row = (int64_t)blockIdx.x * 4 + wave; row < n; row += nw) {
        double s = 0.0;
        for (int c = lane; c < nev; c += 64) {
            const double x = X[row * ldx + c];
            s = fma(w[c] * x, x, s);
        }
        s = wave_sum(s);
        if (lane == 0) gd[row] = s;
    }
}

hipError_t diag_grad(int64_t n, const double *X, int64_t ldx, int nev, const double *w, double *gd, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 3) / 4, 65536);
    hipLaunchKernelGGL(k_diag_grad, dim3((unsigned)blocks), dim3(256), 0, st, n, X, ldx, nev, w, gd);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// value scatter into the union pattern, row scaling by a diagonal
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scatter_values(int64_t nnz, const int32_t *__restrict__ map,
                                                        const double *__restrict__ src, double *__restrict__ dst) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * 256)
        dst[map[e]] = src[e];
}

hipError_t scatter_values(int64_t nnz, const int32_t *map, const double *src, double *dst, hipStream_t st) {
    if (nnz == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_values, dim3(ew_grid(nnz)), dim3(256), 0, st, nnz, map, src, dst);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_scale_rows(int64_t n, int k, const double *__restrict__ d,
                                                    const double *__restrict__ X, int64_t ldx, double *__restrict__ Y,
                                                    int64_t ldy) {
    const int64_t total = n * k;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
        const int64_t i = t / k;
        const int j = (int)(t % k);
        Y[i * ldy + j] = d[i] * X[i * ldx + j];
    }
}

hipError_t scale_rows(int64_t n, int k, const double *d, const double *X, int64_t ldx, double *Y, int64_t ldy,
                      hipStream_t st) {
    if (n == 0 || k == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_rows, dim3(ew_grid(n * k)), dim3(256), 0, st, n, k, d, X, ldx, Y, ldy);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
static hipError_t grow(void **p, size_t *cap, size_t bytes) {
    if (bytes <= *cap) return hipSuccess;
    if (*p) {
        hipError_t e = hipFree(*p);
        if (e != hipSuccess) return e;
        *p = nullptr;
        *cap = 0;
    }
    size_t nb = std::max<size_t>(bytes, 4096);
    nb = nb + nb / 4;
    hipError_t e = hipMalloc(p, nb);
    if (e != hipSuccess) return e;
    *cap = nb;
    return hipSuccess;
}

hipError_t Workspace::ensure_part(size_t bytes) { return grow((void **)&part, &part_bytes, bytes); }
hipError_t Workspace::ensure_small(size_t bytes) { return grow((void **)&small, &small_bytes, bytes); }
hipError_t Workspace::ensure_colvec(size_t bytes) { return grow((void **)&colvec, &colvec_bytes, bytes); }
hipError_t Workspace::ensure_flags() {
    if (iflags) return hipSuccess;
    return hipMalloc((void **)&iflags, 8 * sizeof(int));
}
hipError_t Workspace::ensure_pinned(size_t bytes) {
    if (bytes <= pinned_bytes) return hipSuccess;
    if (pinned) {
        hipError_t e = hipHostFree(pinned);
        if (e != hipSuccess) return e;
        pinned = nullptr;
        pinned_bytes = 0;
    }
    size_t nb = std::max<size_t>(bytes, 4096);
    nb = nb + nb / 4;
    hipError_t e = hipHostMalloc((void **)&pinned, nb, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    pinned_bytes = nb;
    return hipSuccess;
}
void Workspace::release() {
    if (part) (void)hipFree(part);
    if (small) (void)hipFree(small);
    if (colvec) (void)hipFree(colvec);
    if (iflags) (void)hipFree(iflags);
    if (pinned) (void)hipHostFree(pinned);
    part = small = colvec = nullptr;
    iflags = nullptr;
    pinned = nullptr;
    part_bytes = small_bytes = colvec_bytes = pinned_bytes = 0;
}

}  // namespace gcge
