// Dense symmetric eigensolver on the device for the reduced Rayleigh-Ritz
// problem of STEP 3 (Section 3.2; the paper calls LAPACK dsyevx on the host).
//
//   1. Householder reduction of the n x n matrix to tridiagonal form T, one
//      pass over the lower triangle per step (vectors in LDS): by one
//      work-group, or from order 305 on by eight work-groups of one
//      cooperative launch that split the rows and meet at one grid barrier
//      per step.
//   2. The nwant smallest eigenvalues of T by multisection: one wave per
//      eigenvalue, 64 Sturm counts per round (one per lane).
//   3. Their eigenvectors by inverse iteration with a partially pivoted LU of
//      T - lambda I; eigenvalues closer than a cluster tolerance are handled by
//      one work-group in order, each vector orthogonalized against the earlier
//      ones of its cluster (classical Gram-Schmidt, twice).
//   4. Back-transformation by the Householder reflectors, one wave per
//      column.
//   5. Two Newton-Schulz steps X <- X (3 I - X^T X) / 2 with the block Gram
//      and GEMM kernels, which restore orthonormality to rounding (inverse
//      iteration leaves eps ||T|| / gap between vectors of distinct
//      eigenvalues) while keeping X^T A X diagonal to O(eps ||T||).
//
// Every step is deterministic (fixed reduction orders, counter-based start
// vectors).
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>

#include "internal.h"

namespace gcge {
namespace {

constexpr double EPS = 2.220446049250313e-16;

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_upd0(double v) {   // rows outside ROWS read 0
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}
// Sum over the 64 lanes, the same value in every lane; all lanes active.
// Inside each 16-lane row, DPP moves (quad permutations [1,0,3,2] and
// [2,3,0,1], then the half-row and row mirrors) pair each lane with one that
// holds the same kind of partial, so every lane of a row ends with the row
// sum; row broadcasts 15 and 31 then accumulate the four row sums into lane
// 63, which is read as a wave-uniform value.  VALU moves only: no LDS
// permutes on the dependent chain of a reduction.
__device__ __forceinline__ double wsum(double v) {
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x141>(v);
    v += dpp_mov<0x140>(v);
    v += dpp_upd0<0x142, 0xA>(v);
    v += dpp_upd0<0x143, 0xC>(v);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wmin(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Sum over a work-group of NW waves, identical in every thread, fixed order.
// No barrier after the read of red: the caller must not write red again
// before a later barrier (the tridiagonalization alternates two buffers).
template <int NW>
__device__ __forceinline__ double block_sum(double v, double *red) {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    v = wsum(v);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) t += red[i];
    return t;
}

// ---------------------------------------------------------------------------
// 1. Householder tridiagonalization, one work-group of 1024 threads (16
// waves).  a: n x n symmetric, row-major (lda); only its lower triangle is
// read after the first row.  Reflector k (H_k = I - tau_k v v^T, v[0] = 1)
// is chosen from column k below the diagonal and stored over row k, columns
// k+1..n-1 (the upper triangle, otherwise unused) for the back-transformation.
//
// Each step makes one pass over the lower triangle of the trailing block: it
// applies the pending rank-2 update of the previous reflector (B -= v w^T +
// w v^T) and, in the same pass, accumulates the product of the updated block
// with the next reflector (row sums, plus column contributions kept per lane
// in registers and added across waves in a fixed order).  The next reflector
// itself comes from the updated first column, computed just before the pass.
// d, e: diagonal and off-diagonal of T; tau[k] for k < n-2.
// ---------------------------------------------------------------------------
constexpr int TRI_T = 1024, TRI_W = TRI_T / 64;
static_assert(DENSE_EIG_MAX <= 12 * 64, "k_tridiag instances cover 12 column slots per lane");

// Rows of the LDS buffer that combines the per-wave column sums: one per
// wave, so the 16 waves write their sums at once and one barrier precedes
// the fixed-order sum; (6 + 16) n doubles are at most 135 KiB (order 768) of
// the 160 KiB a work-group may hold.
__host__ __device__ constexpr int tri_comb_rows(int) { return TRI_W; }

// y = C v over the trailing block C = rows/cols r0..n-1, first applying the
// pending update C -= sv sw^T + sw sv^T when UPD.  y goes to sy[r0..n-1].
// A wave takes RU consecutive rows at a time; lane l holds columns l, l + 64,
// ... (NS slots).  The loads of a row group are issued SB slots at a time
// before any of them is used (clamped in-bounds addresses, values masked
// afterwards), so the group pays one memory latency per SB slots; slots wholly
// right of the group's last row are skipped (a wave-uniform test).
template <bool UPD, int NS, int RU, int SB, int CR>
__device__ __forceinline__ void tri_pass(int n, double *__restrict__ a, int64_t lda, int r0,
                                         const double *sv, const double *sw, const double *vn, double *sy,
                                         double *comb) {
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int mm = n - r0;
    double part[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) part[t] = 0.0;
    for (int rb = wave * RU; rb < mm; rb += TRI_W * RU) {
        const int nsl = min(rb + RU - 1, mm - 1) / 64 + 1;   // slots holding columns <= the last row
        double acc[RU], vi[RU], wi[RU], vni[RU];
        double *rows[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int i = min(r0 + rb + u, n - 1);
            acc[u] = 0.0;
            vi[u] = UPD ? sv[i] : 0.0;
            wi[u] = UPD ? sw[i] : 0.0;
            vni[u] = vn[i];
            rows[u] = a + (int64_t)i * lda + r0;
        }
        // slots in batches of SB: the loads of a batch are all in flight together
#pragma unroll
        for (int t0 = 0; t0 < NS; t0 += SB) {
            if (t0 < nsl) {
                double x[SB][RU];
#pragma unroll
                for (int b = 0; b < SB; ++b) {
                    const int t = t0 + b;
                    if (t < NS && t < nsl) {
                        const int rc = min(lane + 64 * t, mm - 1);
#pragma unroll
                        for (int u = 0; u < RU; ++u) x[b][u] = rows[u][rc];
                    }
                }
#pragma unroll
                for (int b = 0; b < SB; ++b) {
                    const int t = t0 + b;
                    if (t < NS && t < nsl) {
                        const int r = lane + 64 * t;
                        const int rc = min(r, mm - 1);
                        const double swr = UPD ? sw[r0 + rc] : 0.0, svr = UPD ? sv[r0 + rc] : 0.0;
                        const double vnr = vn[r0 + rc];
#pragma unroll
                        for (int u = 0; u < RU; ++u) {
                            const int ri = rb + u;
                            const bool in = ri < mm && r <= ri;
                            double xv = x[b][u];
                            if (UPD) {
                                xv -= vi[u] * swr + wi[u] * svr;
                                if (in) rows[u][r] = xv;
                            }
                            xv = in ? xv : 0.0;
                            acc[u] += xv * vnr;
                            const double xp = r < ri ? xv : 0.0;
                            part[t] += xp * vni[u];
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const double s = wsum(acc[u]);
            if (lane == 0 && rb + u < mm) sy[r0 + rb + u] = s;
        }
    }
    // column contributions, combined in a fixed order: comb[q] = part of wave
    // q + CR (NST - 1), + ..., + wave q; y = sy + comb[0] + ... + comb[CR - 1].
    // (comb was last read before the barrier that ended the previous pass, and
    // sy is read only after the stage barriers.)
    constexpr int NST = TRI_W / CR;
    for (int stage = NST - 1; stage >= 0; --stage) {
        if (wave / CR == stage) {
            double *c = comb + (int64_t)(wave % CR) * n;
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                const int r = lane + 64 * t;
                if (r < mm) c[r] = (stage == NST - 1) ? part[t] : c[r] + part[t];
            }
        }
        __syncthreads();
    }
    for (int r = tid; r < mm; r += TRI_T) {
        double y = sy[r0 + r];
#pragma unroll
        for (int q = 0; q < CR; ++q) y += comb[(int64_t)q * n + r];
        sy[r0 + r] = y;
    }
    __syncthreads();
}

// Reflector from x[r0..n-1] (x[r0] = alpha): v -> sv2[r0..n-1], returns
// (tau, beta).  Identical in every thread.  sq is this thread's share of
// sum x[i]^2 over i > r0, accumulated while x was written (the barrier in the
// block sum publishes x).
__device__ __forceinline__ void tri_reflector(int n, int r0, const double *x, double *sv2, double *red,
                                              double sq, double &tau_out, double &beta_out) {
    const int tid = threadIdx.x;
    const double s = block_sum<TRI_W>(sq, red);
    const double alpha = x[r0];
    if (s == 0.0) {
        for (int i = r0 + tid; i < n; i += TRI_T) sv2[i] = (i == r0) ? 1.0 : 0.0;
        tau_out = 0.0;
        beta_out = alpha;
    } else {
        const double beta = -copysign(sqrt(alpha * alpha + s), alpha);
        const double sc = 1.0 / (alpha - beta);
        for (int i = r0 + tid; i < n; i += TRI_T) sv2[i] = (i == r0) ? 1.0 : x[i] * sc;
        tau_out = (beta - alpha) / beta;
        beta_out = beta;
    }
    __syncthreads();
}

// w = p + K v with p = tau y, K = -tau/2 p.v over r0..n-1
__device__ __forceinline__ void tri_w(int n, int r0, double t, const double *sy, const double *sv2, double *sw2,
                                      double *red) {
    const int tid = threadIdx.x;
    double pv = 0.0;
    for (int i = r0 + tid; i < n; i += TRI_T) pv += t * sy[i] * sv2[i];
    pv = block_sum<TRI_W>(pv, red);
    const double K = -0.5 * t * pv;
    for (int i = r0 + tid; i < n; i += TRI_T) sw2[i] = t * sy[i] + K * sv2[i];
    __syncthreads();
}

template <int NS, int RU, int SB>
__global__ __launch_bounds__(TRI_T) void k_tridiag(int n, double *__restrict__ a, int64_t lda,
                                                    double *__restrict__ d, double *__restrict__ e,
                                                    double *__restrict__ tau) {
    extern __shared__ double sm[];
    double *svA = sm, *swA = sm + n, *svB = sm + 2 * n, *swB = sm + 3 * n, *sy = sm + 4 * n, *sx = sm + 5 * n;
    constexpr int CR = tri_comb_rows(NS);
    double *comb = sm + 6 * n;   // CR x n
    __shared__ double red[2][TRI_W];   // block sums: reflector norms, then p.v
    const int tid = threadIdx.x;
    if (n <= 2) {
        if (tid == 0) {
            d[0] = a[0];
            if (n == 2) {
                e[0] = a[lda];
                d[1] = a[lda + 1];
                tau[0] = 0.0;
            }
        }
        return;
    }
    // reflector 0 from row 0 (the input is fully symmetric)
    double sq = 0.0;
    for (int i = 1 + tid; i < n; i += TRI_T) {
        const double v = a[i];
        sx[i] = v;
        sq += i >= 2 ? v * v : 0.0;
    }
    double t0, b0;
    tri_reflector(n, 1, sx, svA, red[0], sq, t0, b0);
    for (int i = 1 + tid; i < n; i += TRI_T) a[i] = svA[i];
    if (tid == 0) {
        d[0] = a[0];
        e[0] = b0;
        tau[0] = t0;
    }
    tri_pass<false, NS, RU, SB, CR>(n, a, lda, 1, nullptr, nullptr, svA, sy, comb);
    tri_w(n, 1, t0, sy, svA, swA, red[1]);
    double *sv = svA, *sw = swA, *sv2 = svB, *sw2 = swB;
    for (int k = 0; k + 4 <= n; ++k) {
        const int k1 = k + 1;
        // updated column k1 below the diagonal and the diagonal entry
        double sq1 = 0.0;
        for (int i = k1 + 1 + tid; i < n; i += TRI_T) {
            const double v = a[(int64_t)i * lda + k1] - (sv[i] * sw[k1] + sw[i] * sv[k1]);
            sx[i] = v;
            sq1 += i >= k1 + 2 ? v * v : 0.0;
        }
        if (tid == 0) d[k1] = a[(int64_t)k1 * lda + k1] - (sv[k1] * sw[k1] + sw[k1] * sv[k1]);
        double t1, b1;
        tri_reflector(n, k1 + 1, sx, sv2, red[0], sq1, t1, b1);
        for (int i = k1 + 1 + tid; i < n; i += TRI_T) a[(int64_t)k1 * lda + i] = sv2[i];
        if (tid == 0) {
            e[k1] = b1;
            tau[k1] = t1;
        }
        tri_pass<true, NS, RU, SB, CR>(n, a, lda, k1 + 1, sv, sw, sv2, sy, comb);
        tri_w(n, k1 + 1, t1, sy, sv2, sw2, red[1]);
        double *tv = sv, *tw = sw;
        sv = sv2;
        sw = sw2;
        sv2 = tv;
        sw2 = tw;
    }
    // pending update of the last reflector on the trailing 2 x 2 block
    if (tid == 0) {
        const int p = n - 2, q = n - 1;
        d[p] = a[(int64_t)p * lda + p] - (sv[p] * sw[p] + sw[p] * sv[p]);
        e[p] = a[(int64_t)q * lda + p] - (sv[q] * sw[p] + sw[q] * sv[p]);
        d[q] = a[(int64_t)q * lda + q] - (sv[q] * sw[q] + sw[q] * sv[q]);
        tau[p] = 0.0;
    }
}

// The same reduction spread over TRI_G work-groups of one cooperative launch.
// Rows of the trailing block are dealt to the G * TRI_W waves of the grid in
// turn (RU rows at a time); a work-group's pass applies the pending rank-2
// update to its own rows of the lower triangle and writes its partial of
// y = C v (the row sums of its rows and the column contributions of its rows
// to every column) to its slot of yp.  After one grid barrier per step every
// work-group sums the G partials in slot order and forms w, the updated next
// column and the next reflector itself (the same values in every
// work-group); work-group 0 writes d, e, tau and the reflector into the
// upper triangle, which no step reads.  The partials alternate between two
// buffers, so a work-group still summing one step's partials is never
// overwritten by another's next pass.  Output as k_tridiag's.
constexpr int TRI_G = 8;

template <bool UPD, int NS, int RU, int SB, int CR>
__device__ __forceinline__ void tri_pass_mw(int n, double *a, int64_t lda, int r0, const double *sv,
                                            const double *sw, const double *vn, double *sy, double *comb,
                                            double *yp) {
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int gw = blockIdx.x * TRI_W + wave, nw = gridDim.x * TRI_W;
    const int mm = n - r0;
    for (int r = tid; r < mm; r += TRI_T) sy[r0 + r] = 0.0;
    __syncthreads();
    double part[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) part[t] = 0.0;
    for (int rb = gw * RU; rb < mm; rb += nw * RU) {
        const int nsl = min(rb + RU - 1, mm - 1) / 64 + 1;
        double acc[RU], vi[RU], wi[RU], vni[RU];
        double *rows[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int i = min(r0 + rb + u, n - 1);
            acc[u] = 0.0;
            vi[u] = UPD ? sv[i] : 0.0;
            wi[u] = UPD ? sw[i] : 0.0;
            vni[u] = vn[i];
            rows[u] = a + (int64_t)i * lda + r0;
        }
#pragma unroll
        for (int t0 = 0; t0 < NS; t0 += SB) {
            if (t0 < nsl) {
                double x[SB][RU];
#pragma unroll
                for (int b = 0; b < SB; ++b) {
                    const int t = t0 + b;
                    if (t < NS && t < nsl) {
                        const int rc = min(lane + 64 * t, mm - 1);
#pragma unroll
                        for (int u = 0; u < RU; ++u) x[b][u] = rows[u][rc];
                    }
                }
#pragma unroll
                for (int b = 0; b < SB; ++b) {
                    const int t = t0 + b;
                    if (t < NS && t < nsl) {
                        const int r = lane + 64 * t;
                        const int rc = min(r, mm - 1);
                        const double swr = UPD ? sw[r0 + rc] : 0.0, svr = UPD ? sv[r0 + rc] : 0.0;
                        const double vnr = vn[r0 + rc];
#pragma unroll
                        for (int u = 0; u < RU; ++u) {
                            const int ri = rb + u;
                            const bool in = ri < mm && r <= ri;
                            double xv = x[b][u];
                            if (UPD) {
                                xv -= vi[u] * swr + wi[u] * svr;
                                if (in) rows[u][r] = xv;
                            }
                            xv = in ? xv : 0.0;
                            acc[u] += xv * vnr;
                            const double xp = r < ri ? xv : 0.0;
                            part[t] += xp * vni[u];
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const double s = wsum(acc[u]);
            if (lane == 0 && rb + u < mm) sy[r0 + rb + u] = s;
        }
    }
    constexpr int NST = TRI_W / CR;
    for (int stage = NST - 1; stage >= 0; --stage) {
        if (wave / CR == stage) {
            double *c = comb + (int64_t)(wave % CR) * n;
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                const int r = lane + 64 * t;
                if (r < mm) c[r] = (stage == NST - 1) ? part[t] : c[r] + part[t];
            }
        }
        __syncthreads();
    }
    for (int r = tid; r < mm; r += TRI_T) {
        double y = sy[r0 + r];
#pragma unroll
        for (int q = 0; q < CR; ++q) y += comb[(int64_t)q * n + r];
        yp[r0 + r] = y;
    }
    __syncthreads();
}

// y[r0..n-1] = the sum of the G partials in slot order
__device__ __forceinline__ void tri_gather(int n, int r0, const double *yp, double *sy) {
    const int G = gridDim.x;
    for (int r = r0 + threadIdx.x; r < n; r += TRI_T) {
        double y = 0.0;
        for (int g = 0; g < G; ++g) y += yp[(int64_t)g * n + r];
        sy[r] = y;
    }
    __syncthreads();
}

template <int NS, int RU, int SB>
__global__ __launch_bounds__(TRI_T) void k_tridiag_mw(int n, double *a, int64_t lda, double *__restrict__ d,
                                                       double *__restrict__ e, double *__restrict__ tau,
                                                       double *ypart) {
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    extern __shared__ double sm[];
    double *svA = sm, *swA = sm + n, *svB = sm + 2 * n, *swB = sm + 3 * n, *sy = sm + 4 * n, *sx = sm + 5 * n;
    constexpr int CR = tri_comb_rows(NS);
    double *comb = sm + 6 * n;
    __shared__ double red[2][TRI_W];
    const int tid = threadIdx.x, g = blockIdx.x, G = gridDim.x;
    const bool lead = g == 0;
    if (n <= 2) {   // the same in every work-group: no barrier is reached
        if (lead && tid == 0) {
            d[0] = a[0];
            if (n == 2) {
                e[0] = a[lda];
                d[1] = a[lda + 1];
                tau[0] = 0.0;
            }
        }
        return;
    }
    // reflector 0 from column 0 below the diagonal (the input is fully
    // symmetric; work-group 0 overwrites row 0's upper part with it)
    double sq = 0.0;
    for (int i = 1 + tid; i < n; i += TRI_T) {
        const double v = a[(int64_t)i * lda];
        sx[i] = v;
        sq += i >= 2 ? v * v : 0.0;
    }
    double t0, b0;
    tri_reflector(n, 1, sx, svA, red[0], sq, t0, b0);
    if (lead) {
        for (int i = 1 + tid; i < n; i += TRI_T) a[i] = svA[i];
        if (tid == 0) {
            d[0] = a[0];
            e[0] = b0;
            tau[0] = t0;
        }
    }
    int par = 0;
    tri_pass_mw<false, NS, RU, SB, CR>(n, a, lda, 1, nullptr, nullptr, svA, sy, comb,
                                       ypart + ((int64_t)par * G + g) * n);
    grid.sync();
    tri_gather(n, 1, ypart + (int64_t)par * G * n, sy);
    tri_w(n, 1, t0, sy, svA, swA, red[1]);
    double *sv = svA, *sw = swA, *sv2 = svB, *sw2 = swB;
    for (int k = 0; k + 4 <= n; ++k) {
        const int k1 = k + 1;
        par ^= 1;
        // updated column k1 below the diagonal and the diagonal entry
        double sq1 = 0.0;
        for (int i = k1 + 1 + tid; i < n; i += TRI_T) {
            const double v = a[(int64_t)i * lda + k1] - (sv[i] * sw[k1] + sw[i] * sv[k1]);
            sx[i] = v;
            sq1 += i >= k1 + 2 ? v * v : 0.0;
        }
        const double dk1 = a[(int64_t)k1 * lda + k1] - (sv[k1] * sw[k1] + sw[k1] * sv[k1]);
        double t1, b1;
        tri_reflector(n, k1 + 1, sx, sv2, red[0], sq1, t1, b1);
        if (lead) {
            for (int i = k1 + 1 + tid; i < n; i += TRI_T) a[(int64_t)k1 * lda + i] = sv2[i];
            if (tid == 0) {
                d[k1] = dk1;
                e[k1] = b1;
                tau[k1] = t1;
            }
        }
        tri_pass_mw<true, NS, RU, SB, CR>(n, a, lda, k1 + 1, sv, sw, sv2, sy, comb,
                                          ypart + ((int64_t)par * G + g) * n);
        grid.sync();
        tri_gather(n, k1 + 1, ypart + (int64_t)par * G * n, sy);
        tri_w(n, k1 + 1, t1, sy, sv2, sw2, red[1]);
        double *tv = sv, *tw = sw;
        sv = sv2;
        sw = sw2;
        sv2 = tv;
        sw2 = tw;
    }
    // pending update of the last reflector on the trailing 2 x 2 block
    if (lead && tid == 0) {
        const int p = n - 2, q = n - 1;
        d[p] = a[(int64_t)p * lda + p] - (sv[p] * sw[p] + sw[p] * sv[p]);
        e[p] = a[(int64_t)q * lda + p] - (sv[q] * sw[p] + sw[q] * sv[p]);
        d[q] = a[(int64_t)q * lda + q] - (sv[q] * sw[q] + sw[q] * sv[q]);
        tau[p] = 0.0;
    }
}

// Gershgorin interval, norm bound and pivot floor of T, as every wave of the
// later kernels computes them (identically).
struct TBounds {
    double lo, hi, tnorm, pivmin;
};
__device__ TBounds t_bounds(int n, const double *d, const double *e) {
    const int lane = threadIdx.x % 64;
    double lo = INFINITY, hi = -INFINITY, e2 = 0.0;
    for (int r = lane; r < n; r += 64) {
        const double off = (r > 0 ? fabs(e[r - 1]) : 0.0) + (r + 1 < n ? fabs(e[r]) : 0.0);
        lo = fmin(lo, d[r] - off);
        hi = fmax(hi, d[r] + off);
        if (r + 1 < n) e2 = fmax(e2, e[r] * e[r]);
    }
    TBounds b;
    b.lo = wmin(lo);
    b.hi = wmax(hi);
    b.tnorm = fmax(fabs(b.lo), fabs(b.hi));
    b.pivmin = DBL_MIN * fmax(1.0, wmax(e2));
    const double pad = 2.0 * EPS * b.tnorm + 4.0 * b.pivmin;
    b.lo -= pad;
    b.hi += pad;
    return b;
}

// ---------------------------------------------------------------------------
// 2. Eigenvalue i (0-based, ascending) of T by multisection: one wave per
// eigenvalue; each round splits the bracket into 65 parts and lane l counts
// the eigenvalues below the l-th split point (Sturm sequence).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_bisect(int n, const double *__restrict__ d, const double *__restrict__ e,
                                               int nwant, double *__restrict__ w) {
    extern __shared__ double sm[];
    double *sd = sm, *se2 = sm + n;
    const int i = blockIdx.x, lane = threadIdx.x;
    for (int r = lane; r < n; r += 64) {
        sd[r] = d[r];
        se2[r] = (r + 1 < n) ? e[r] * e[r] : 0.0;
    }
    __syncthreads();
    const TBounds b = t_bounds(n, d, e);
    double lo = b.lo, hi = b.hi;
    for (int round = 0; round < 24; ++round) {
        if (hi - lo <= 2.0 * EPS * fmax(fabs(lo), fabs(hi)) + 2.0 * b.pivmin) break;
        const double h = hi - lo;
        const double x = lo + h * (double)(lane + 1) / 65.0;
        int cnt = 0;
        double q = sd[0] - x;
        if (fabs(q) < b.pivmin) q = -b.pivmin;
        cnt += q < 0.0;
        for (int r = 1; r < n; ++r) {
            q = (sd[r] - x) - se2[r - 1] / q;
            if (fabs(q) < b.pivmin) q = -b.pivmin;
            cnt += q < 0.0;
        }
        const unsigned long long mask = __ballot(cnt > i);
        if (mask == 0ull) {
            lo = lo + h * 64.0 / 65.0;
        } else {
            const int f = __ffsll((long long)mask) - 1;
            const double nhi = lo + h * (double)(f + 1) / 65.0;
            const double nlo = (f > 0) ? lo + h * (double)f / 65.0 : lo;
            lo = nlo;
            hi = nhi;
        }
    }
    if (lane == 0) w[i] = 0.5 * (lo + hi);
}

// ---------------------------------------------------------------------------
// 3. Inverse iteration.  Work-group i (one wave) acts only when eigenvalue i
// starts a cluster (i == 0 or w[i] - w[i-1] > ctol); it then computes the
// vectors of the whole cluster in order.  LU of T - s I with row interchanges
// (a tridiagonal U with two superdiagonals), three solves from a start vector
// drawn from SplitMix64, each followed by two Gram-Schmidt passes against the
// earlier vectors of the cluster and normalization.  Z column-major (ldz).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(64) void k_invit(int n, const double *__restrict__ d, const double *__restrict__ e,
                                              int nwant, const double *__restrict__ w, double ctol_rel,
                                              double *__restrict__ Z, int64_t ldz) {
    const int i = blockIdx.x, lane = threadIdx.x;
    const TBounds b = t_bounds(n, d, e);
    const double ctol = ctol_rel * b.tnorm;
    if (i > 0 && w[i] - w[i - 1] <= ctol) return;   // not the first of its cluster
    int j = i + 1;
    while (j < nwant && w[j] - w[j - 1] <= ctol) ++j;
    extern __shared__ double sm[];
    double *u1 = sm, *u2 = sm + n, *u3 = sm + 2 * n, *ml = sm + 3 * n, *z = sm + 4 * n;
    double *iu1 = sm + 5 * n, *sd = sm + 6 * n, *se = sm + 7 * n;   // 1 / u1; T staged in LDS
    int *piv = (int *)(sm + 8 * n);
    for (int r = lane; r < n; r += 64) {
        sd[r] = d[r];
        se[r] = r + 1 < n ? e[r] : 0.0;
    }
    __syncthreads();
    const double tiny = EPS * b.tnorm + b.pivmin;
    double sprev = -INFINITY;
    for (int mbr = i; mbr < j; ++mbr) {
        double s = w[mbr];
        if (s <= sprev) s = sprev + 10.0 * EPS * b.tnorm;   // separate equal shifts
        sprev = s;
        if (lane == 0) {
            // LU with partial pivoting of the tridiagonal T - s I (T read
            // from LDS; only ar and br are carried from step to step)
            double ar = sd[0] - s, br = (n > 1) ? se[0] : 0.0;
            for (int r = 0; r + 1 < n; ++r) {
                const double cr = se[r];                      // subdiagonal entry (r+1, r)
                const double an = sd[r + 1] - s;              // diagonal of row r+1
                const double bn = se[r + 1];                  // (r+1, r+2); 0 past the end
                if (fabs(ar) >= fabs(cr)) {
                    const double aa = (fabs(ar) < tiny) ? copysign(tiny, ar) : ar;
                    const double l = cr / aa;
                    u1[r] = aa;
                    u2[r] = br;
                    u3[r] = 0.0;
                    ml[r] = l;
                    piv[r] = 0;
                    ar = an - l * br;
                    br = bn;
                } else {
                    const double l = ar / cr;
                    u1[r] = (fabs(cr) < tiny) ? copysign(tiny, cr) : cr;
                    u2[r] = an;
                    u3[r] = bn;
                    ml[r] = l;
                    piv[r] = 1;
                    ar = br - l * an;
                    br = -l * bn;
                }
            }
            u1[n - 1] = (fabs(ar) < tiny) ? copysign(tiny, ar) : ar;
            ml[n - 1] = 0.0;
            piv[n - 1] = 0;
        }
        for (int r = lane; r < n; r += 64) {
            const uint64_t h = mix64((uint64_t)0x5eed + ((uint64_t)mbr * (uint64_t)n + (uint64_t)r + 1) *
                                                             0x9e3779b97f4a7c15ull);
            z[r] = 2.0 * ((double)(h >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
        }
        __syncthreads();
        for (int r = lane; r < n; r += 64) iu1[r] = 1.0 / u1[r];
        __syncthreads();
        for (int it = 0; it < 3; ++it) {
            if (lane == 0) {
                // forward: row interchanges and L.  The value moving down
                // (z[r] after the steps before) is carried in a register;
                // z[r + 1] is still the input's, so every load of a step is
                // independent of the carried value and can be issued early.
                double c = z[0];
                for (int r = 0; r + 1 < n; ++r) {
                    const double t = z[r + 1], l = ml[r];
                    const bool sw = piv[r] != 0;
                    z[r] = sw ? t : c;
                    c = sw ? fma(-l, t, c) : fma(-l, c, t);
                }
                z[n - 1] = c;
                // back substitution with U, the two later unknowns carried in
                // registers, the divisions by u1 as products with 1 / u1
                double x1 = z[n - 1] * iu1[n - 1], x2 = 0.0;
                z[n - 1] = x1;
                for (int r = n - 2; r >= 0; --r) {
                    const double x = (z[r] - u2[r] * x1 - u3[r] * x2) * iu1[r];
                    z[r] = x;
                    x2 = x1;
                    x1 = x;
                }
            }
            __syncthreads();
            // scale, then orthogonalize against the earlier cluster vectors (twice)
            double nr = 0.0;
            for (int r = lane; r < n; r += 64) nr += z[r] * z[r];
            nr = wsum(nr);
            const double inv = (nr > 0.0) ? 1.0 / sqrt(nr) : 0.0;
            for (int r = lane; r < n; r += 64) z[r] *= inv;
            for (int pass = 0; pass < 2 && mbr > i; ++pass) {
                for (int q = i; q < mbr; ++q) {
                    const double *zq = Z + (int64_t)q * ldz;
                    double c = 0.0;
                    for (int r = lane; r < n; r += 64) c += zq[r] * z[r];
                    c = wsum(c);
                    for (int r = lane; r < n; r += 64) z[r] -= c * zq[r];
                }
                double n2 = 0.0;
                for (int r = lane; r < n; r += 64) n2 += z[r] * z[r];
                n2 = wsum(n2);
                const double in2 = (n2 > 0.0) ? 1.0 / sqrt(n2) : 0.0;
                for (int r = lane; r < n; r += 64) z[r] *= in2;
            }
            __syncthreads();
        }
        double *zo = Z + (int64_t)mbr * ldz;
        for (int r = lane; r < n; r += 64) zo[r] = z[r];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 4. x = H_0 H_1 ... H_{n-3} z for every wanted column; output row-major.
// ---------------------------------------------------------------------------
// One wave per column: the column sits in registers (lane l holds rows l,
// l + 64, ...; NS slots), reflector k's row of a is read coalesced (rows
// k+1..n-1 of v; addresses clamped into the row, values masked), the loads
// run PD reflectors ahead of their use, and the dot product is a wave sum
// (DPP, no LDS): no block barrier per reflector.  Measured at order 450 with
// 350 columns: 154 us, against 629 us for four columns per 256-thread
// work-group with two barriers and a block sum per reflector.
template <int NS, int PD>
__global__ __launch_bounds__(64) void k_backtr_w(int n, const double *__restrict__ a, int64_t lda,
                                                 const double *__restrict__ tau, int nwant,
                                                 const double *__restrict__ Z, int64_t ldz,
                                                 double *__restrict__ X, int64_t ldx) {
    extern __shared__ double stau[];
    const int c = blockIdx.x, lane = threadIdx.x;
    for (int i = lane; i < n; i += 64) stau[i] = tau[i];
    double z[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const int r = lane + 64 * j;
        z[j] = r < n ? Z[(int64_t)c * ldz + r] : 0.0;
    }
    __syncthreads();
    auto load = [&](int k, double (&v)[NS]) {
        const int kk = max(k, 0);
        const double *row = a + (int64_t)kk * lda;
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int r = lane + 64 * j;
            v[j] = row[min(max(r, kk + 1), n - 1)];
        }
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int r = lane + 64 * j;
            v[j] = (k >= 0 && r > k && r < n) ? v[j] : 0.0;
        }
    };
    double buf[PD][NS];
    const int ktop = n - 3;
#pragma unroll
    for (int p = 0; p < PD; ++p) load(ktop - p, buf[p]);
    for (int k0 = ktop; k0 >= 0; k0 -= PD) {
#pragma unroll
        for (int p = 0; p < PD; ++p) {
            const int k = k0 - p;
            if (k >= 0) {   // wave-uniform
                double d = 0.0;
#pragma unroll
                for (int j = 0; j < NS; ++j) d += buf[p][j] * z[j];
                const double s = stau[k] * wsum(d);
#pragma unroll
                for (int j = 0; j < NS; ++j) z[j] -= s * buf[p][j];
            }
            load(k - PD, buf[p]);
        }
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const int r = lane + 64 * j;
        if (r < n) X[(int64_t)r * ldx + c] = z[j];
    }
}

// M = 1.5 I - 0.5 G (m x m, row-major, ld)
__global__ __launch_bounds__(256) void k_ns_coef(int m, double *__restrict__ G, int64_t ld) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)m * m) return;
    const int r = (int)(idx / m), c = (int)(idx % m);
    double *g = G + (int64_t)r * ld + c;
    *g = (r == c ? 1.5 : 0.0) - 0.5 * *g;
}

}  // namespace

hipError_t DenseEigWork::ensure(int n, int nwant) {
    const size_t need = (size_t)n * n + 3 * (size_t)n + 32 + 3 * (size_t)n * nwant + (size_t)nwant * nwant + 64 +
                        2 * (size_t)TRI_G * n + 64;
    if (need <= cap) return hipSuccess;
    if (buf) (void)hipFree(buf);
    buf = nullptr;
    cap = 0;
    hipError_t e = hipMalloc(&buf, need * sizeof(double));
    if (e != hipSuccess) return e;
    cap = need;
    return hipSuccess;
}

void DenseEigWork::release() {
    if (buf) (void)hipFree(buf);
    buf = nullptr;
    cap = 0;
}

// Householder reduction of the n x n matrix a (row-major, lda = n) to
// tridiagonal form: orders from TRI_MW_MIN on by TRI_G cooperating
// work-groups (one grid barrier per step), below that, or when the runtime
// refuses the cooperative launch, by one work-group.  Measured per call
// (one work-group against eight): order 512 8.1 / 5.2 ms, 448 6.0 / 4.3,
// 384 4.1 / 3.5, 352 3.4 / 3.1, 320 2.76 / 2.67, 288 2.22 / 2.35, 260
// 1.83 / 2.07.
constexpr int TRI_MW_MIN = 305;
static hipError_t tridiagonalize(int n, double *a, double *dg, double *off, double *tau, double *yp,
                                 hipStream_t st) {
    const int ns = (n + 63) / 64;   // column slots per lane
    const size_t lds = sizeof(double) * (6 + tri_comb_rows(ns)) * n;
    int64_t ldn = n;
    if (n >= TRI_MW_MIN) {
        void *args[] = {(void *)&n, (void *)&a, (void *)&ldn, (void *)&dg, (void *)&off, (void *)&tau, (void *)&yp};
        hipError_t le = hipErrorInvalidValue;
#define GCGE_TRI_MW(NSv, RUv, SBv)                                                                      \
    if (ns == NSv)                                                                                       \
        le = hipLaunchCooperativeKernel((const void *)k_tridiag_mw<NSv, RUv, SBv>, dim3(TRI_G), dim3(TRI_T), args, \
                                        (unsigned)lds, st);
        GCGE_TRI_MW(5, 1, 4) GCGE_TRI_MW(6, 1, 4) GCGE_TRI_MW(7, 1, 4) GCGE_TRI_MW(8, 1, 4)
        GCGE_TRI_MW(9, 1, 2) GCGE_TRI_MW(10, 1, 2) GCGE_TRI_MW(11, 1, 2) GCGE_TRI_MW(12, 1, 2)
#undef GCGE_TRI_MW
        if (le == hipSuccess) return hipSuccess;
        (void)hipGetLastError();   // refused: one work-group below
    }
    // rows per group and slots per load batch, the fastest measured at
    // n = 300..500 (one row per group from 5 slots on; two rows would run
    // out of registers from 7 on)
#define GCGE_TRI(NSv, RUv, SBv)                                                                   \
    if (ns == NSv)                                                                                 \
        hipLaunchKernelGGL((k_tridiag<NSv, RUv, SBv>), dim3(1), dim3(TRI_T), lds, st, n, a, ldn, dg, off, tau);
    GCGE_TRI(1, 2, 4) GCGE_TRI(2, 2, 4) GCGE_TRI(3, 2, 4) GCGE_TRI(4, 2, 4) GCGE_TRI(5, 1, 4)
    GCGE_TRI(6, 1, 4) GCGE_TRI(7, 1, 4) GCGE_TRI(8, 1, 4) GCGE_TRI(9, 1, 2) GCGE_TRI(10, 1, 2)
    GCGE_TRI(11, 1, 2) GCGE_TRI(12, 1, 2)
#undef GCGE_TRI
    return hipGetLastError();
}

hipError_t dense_eig(int n, const double *A, int64_t lda, int nwant, double *w, double *X, int64_t ldx,
                     DenseEigWork &dw, Workspace &ws, hipStream_t st) {
    if (n <= 0 || nwant <= 0) return hipSuccess;
    if (nwant > n || n > DENSE_EIG_MAX || ldx < nwant || lda < n) return hipErrorInvalidValue;
    hipError_t e = dw.ensure(n, nwant);
    if (e != hipSuccess) return e;
    double *a = dw.buf;                          // n x n working copy, then the reflectors
    double *dg = a + (size_t)n * n;              // diagonal of T
    double *off = dg + n + 8;                    // off-diagonal of T
    double *tau = off + n + 8;                   // reflector scalars
    double *Z = tau + n + 8;                     // eigenvectors of T, column-major n x nwant
    double *X1 = Z + (size_t)n * nwant;          // row-major n x nwant scratch
    double *X2 = X1 + (size_t)n * nwant;         // row-major n x nwant scratch
    double *G = X2 + (size_t)n * nwant;          // nwant x nwant
    double *yp = G + (size_t)nwant * nwant + 64;  // 2 x TRI_G x n partials of the cooperative reduction
    e = hipMemcpy2DAsync(a, sizeof(double) * n, A, sizeof(double) * lda, sizeof(double) * n, n,
                         hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    e = tridiagonalize(n, a, dg, off, tau, yp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bisect, dim3(nwant), dim3(64), sizeof(double) * 2 * n, st, n, dg, off, nwant, w);
    const size_t inv_lds = sizeof(double) * 8 * n + sizeof(int) * n + 64;
    hipLaunchKernelGGL(k_invit, dim3(nwant), dim3(64), inv_lds, st, n, dg, off, nwant, w, 1e-10, Z, (int64_t)n);
    const int ns = (n + 63) / 64;
#define GCGE_BTW(NSv)                                                                                  \
    if (ns == NSv)                                                                                      \
        hipLaunchKernelGGL((k_backtr_w<NSv, 4>), dim3(nwant), dim3(64), sizeof(double) * n, st, n, a, (int64_t)n, \
                           tau, nwant, Z, (int64_t)n, X1, (int64_t)nwant);
    GCGE_BTW(1) GCGE_BTW(2) GCGE_BTW(3) GCGE_BTW(4) GCGE_BTW(5) GCGE_BTW(6) GCGE_BTW(7) GCGE_BTW(8)
    GCGE_BTW(9) GCGE_BTW(10) GCGE_BTW(11) GCGE_BTW(12)
#undef GCGE_BTW
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // two Newton-Schulz steps: X1 -> X2 -> X
    const double *src = X1;
    for (int it = 0; it < 2; ++it) {
        Segs S;
        S.add(src, nwant, nwant);
        e = gram(n, S, src, nwant, nwant, nullptr, G, nwant, ws, st);
        if (e != hipSuccess) return e;
        const int64_t cnt = (int64_t)nwant * nwant;
        hipLaunchKernelGGL(k_ns_coef, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, nwant, G,
                           (int64_t)nwant);
        double *dst = (it == 0) ? X2 : X;
        const int64_t ldd = (it == 0) ? nwant : ldx;
        e = gemm(n, S, G, nwant, nwant, 1.0, 0.0, dst, ldd, st);
        if (e != hipSuccess) return e;
        src = X2;
    }
    return hipGetLastError();
}

}  // namespace gcge
