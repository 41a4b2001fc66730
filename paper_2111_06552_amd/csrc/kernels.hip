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
#include <mutex>
#include <unordered_map>

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

// Rows visited by one work-group of a row-streaming kernel.  The rows are
// split into one contiguous range per XCD (work-groups are dispatched
// round-robin over the XCDs), and inside that range the XCD's work-groups take
// interleaved groups of ng rows: the resident work-groups of an XCD sweep one
// compact front, so the stencil neighbours one or two grid lines back are
// still in that XCD's L2 when they are gathered again.
struct RowWalk {
    int64_t first, end, stride;
};
__device__ __forceinline__ RowWalk row_walk(int64_t n, int ng) {
    const int nb = gridDim.x, b = blockIdx.x;
    const int nx = nb < NXCD ? nb : NXCD;
    const int x = b % nx, w = b / nx;
    const int nw = nb / nx + (x < nb % nx ? 1 : 0);
    const int64_t per = (n + nx - 1) / nx;
    const int64_t r0 = min(n, (int64_t)x * per), r1 = min(n, r0 + per);
    return RowWalk{r0 + (int64_t)w * ng, r1, (int64_t)nw * ng};
}

// Row blocks of the SpMM over a unit order: the logical row space of
// ceil(n/64) 64-row units is split into one contiguous range of whole units
// per XCD and walked like row_walk in blocks of ng rows (ng divides 64);
// logical row l is physical row uorder[l / 64] * 64 + l % 64 (identity when
// uorder is null).
__device__ __forceinline__ RowWalk unit_walk(int64_t n, int ng) {
    const int nb = gridDim.x, b = blockIdx.x;
    const int nx = nb < NXCD ? nb : NXCD;
    const int x = b % nx, w = b / nx;
    const int nw = nb / nx + (x < nb % nx ? 1 : 0);
    const int64_t nu = (n + 63) / 64;
    const int64_t per = (nu + nx - 1) / nx * 64;
    const int64_t nl = nu * 64;
    const int64_t r0 = min(nl, (int64_t)x * per), r1 = min(nl, r0 + per);
    return RowWalk{r0 + (int64_t)w * ng, r1, (int64_t)nw * ng};
}
__device__ __forceinline__ int64_t unit_row(const int32_t *uorder, int64_t l) {
    return uorder != nullptr ? (int64_t)uorder[l >> 6] * 64 + (l & 63) : l;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

static int num_cu() {
    static const int v = [] {
        int dev = 0, c = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1)
            c = 256;
        return c;
    }();
    return v;
}

int max_row_parts() { return num_cu() * 8; }

// Work-groups of 256 threads that are resident at once for `fn` (occupancy
// query, cached per kernel): row-streaming kernels are launched with exactly
// that many work-groups (capped by the number of work units), so all of them
// run in one wave of residency and finish together.
static int resident_grid(const void *fn, int64_t units, int block = 256) {
    static std::mutex mu;
    static std::unordered_map<const void *, int> cache;
    int nb = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(fn);
        if (it != cache.end()) {
            nb = it->second;
        } else {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, 0) != hipSuccess || nb < 1) nb = 4;
            nb = std::min(nb, 8);
            cache[fn] = nb;
        }
    }
    const int64_t g = (int64_t)num_cu() * nb;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, std::max<int64_t>(units, 1)));
}

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
                                              const int *__restrict__ skip, Affine<T> af) {
    if (skip != nullptr && skip[0] == 0) return;
    constexpr int NG = 256 / G;
    const int tid = threadIdx.x, grp = tid / G, lig = tid % G;
    const int chunk = blockIdx.x;
    const RowWalk rw = row_walk(n, NG);
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

    for (int64_t base = rw.first; base < rw.end; base += rw.stride) {
        const int64_t row = base + grp;
        if (row >= rw.end) break;
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
            } else if (MODE >= 3) {
                const T w = af.w != nullptr ? af.ws * af.w[row] : af.ws;
                const T bb = af.b != nullptr ? af.b[row * af.ldb + col[t]] : T(0);
                const T zz = af.z != nullptr ? af.z[row * af.ldz + col[t]] : T(0);
                y = fma(w, bb - y, zz);
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
            part[(size_t)c * gridDim.x + chunk] = s1;
            if (RED == 1) part[(size_t)(k + c) * gridDim.x + chunk] = s2;
        }
    }
}

// 16-byte vector of V elements (double2, float4) for aligned row segments.
template <typename T, int V>
struct alignas(sizeof(T) * V) Vec {
    T v[V];
};
template <typename T, int V>
__device__ __forceinline__ Vec<T, V> vld(const T *p) {
    return *reinterpret_cast<const Vec<T, V> *>(p);
}
template <typename T, int V>
__device__ __forceinline__ void vst(T *p, const Vec<T, V> &x) {
    *reinterpret_cast<Vec<T, V> *>(p) = x;
}
// streaming store (not kept in L2): the SpMM's output rows, so that L2 keeps
// the gathered input rows instead of dirty output lines
template <typename T, int V>
__device__ __forceinline__ void vst_nt(T *p, const Vec<T, V> &x) {
#pragma unroll
    for (int v = 0; v < V; ++v) __builtin_nontemporal_store(x.v[v], p + v);
}

// SpMM with the sparsity pattern of each block of RS consecutive rows staged
// in LDS: the work-group loads the block's row pointers, then its column
// indices and values with one coalesced sweep, and the row groups gather the
// vector rows with the indices read from LDS (no per-lane broadcast loads,
// one dependent global round trip per row instead of three).  Blocks whose
// nonzeros do not fit the staging area fall back to global index loads.
// 16-byte vector accesses: a group of G lanes per row, lane l owns columns
// V*l .. V*l+V-1; the nonzeros of a row are taken in batches of 7, all seven
// gathered vector rows being requested before they are used.  Requires
// 16-byte aligned rows and leading dimensions that cover round_up(k, V)
// columns: the tail lane reads padding columns of the inputs (never part of a
// result); it writes the padding columns of the output too, except in MODE 4
// (the affine epilogue for caller-owned outputs).
template <typename T, int G, int V, int MODE, int RED>
__global__ __launch_bounds__(256) void k_spmms(int64_t n, const int32_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ colind, const T *__restrict__ va,
                                               const T *__restrict__ vb, const T *__restrict__ dg,
                                               const T *__restrict__ sigma, const T *__restrict__ X, int64_t ldx,
                                               int k, T *__restrict__ Y, int64_t ldy, const T *__restrict__ Z,
                                               int64_t ldz, T *__restrict__ part, int nparts, int64_t rows_per,
                                               const int *__restrict__ skip, const int32_t *__restrict__ uorder,
                                               Affine<T> af) {
    if (skip != nullptr && skip[0] == 0) return;
    // batches of 7 nonzeros: one batch per row of a 7-point stencil, four per 27-point row
    constexpr int NG = 256 / G, U = 7;
    constexpr int RS = NG > 32 ? NG : 32;   // rows per staged block (divides 64)
    constexpr int RPG = RS / NG;            // rows per group per block
    constexpr int CAP = 1024;               // staged nonzeros per block
    __shared__ int s_rp[RS + 1];
    __shared__ int s_ci[CAP];
    __shared__ T s_va[CAP];
    __shared__ T s_vb[MODE == 2 ? CAP : 1];
    const int tid = threadIdx.x, grp = tid / G, lig = tid % G;
    const int chunk = blockIdx.x;
    const RowWalk rw = unit_walk(n, RS);
    const int c0 = lig * V;
    const bool on = c0 < k;
    const int c0l = on ? c0 : 0;   // load column (lanes past k read column 0)
    T sg[V], red1[V], red2[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        sg[v] = (MODE != 0 && c0 + v < k) ? sigma[c0 + v] : T(0);
        red1[v] = red2[v] = T(0);
    }
    for (int64_t lb = rw.first; lb < rw.end; lb += rw.stride) {
        const int64_t base = unit_row(uorder, lb);
        const int nrows = (int)min((int64_t)RS, n - base);
        if (nrows <= 0) continue;   // past the last row (uniform over the work-group)
        for (int t = tid; t <= nrows; t += 256) s_rp[t] = rowptr[base + t];
        __syncthreads();
        const int eb = s_rp[0], ne = s_rp[nrows] - eb;
        const bool staged = ne <= CAP;
        if (staged) {
            for (int t = tid; t < ne; t += 256) {
                s_ci[t] = colind[eb + t];
                s_va[t] = va[eb + t];
                if (MODE == 2) s_vb[t] = vb[eb + t];
            }
        }
        __syncthreads();
        for (int j = 0; j < RPG; ++j) {
            const int lr = j * NG + grp;
            if (lr >= nrows) break;
            const int64_t row = base + lr;
            const int e0 = s_rp[lr] - eb, e1 = s_rp[lr + 1] - eb;
            Vec<T, V> acc, accb, xself;   // xself: the gathered own row (FP32 RED 2, below)
            bool found = false;
#pragma unroll
            for (int v = 0; v < V; ++v) acc.v[v] = accb.v[v] = xself.v[v] = T(0);
            // Slots past the row end re-read the row's last entry (a valid
            // address) with a zero weight, and lanes past column k read column
            // 0: every load is unconditional, so the eight gathers of a batch
            // are all in flight before the first one is used.
            for (int e = e0; e < e1; e += U) {
                int cc[U];
                T av[U], bv[U];
                if (staged) {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int ee = min(e + u, e1 - 1);
                        const bool ok = e + u < e1;
                        cc[u] = s_ci[ee];
                        const T a = s_va[ee];
                        av[u] = ok ? a : T(0);
                        if (MODE == 2) {
                            const T b = s_vb[ee];
                            bv[u] = ok ? b : T(0);
                        } else {
                            bv[u] = T(0);
                        }
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int ee = eb + min(e + u, e1 - 1);
                        const bool ok = e + u < e1;
                        cc[u] = colind[ee];
                        const T a = va[ee];
                        av[u] = ok ? a : T(0);
                        if (MODE == 2) {
                            const T b = vb[ee];
                            bv[u] = ok ? b : T(0);
                        } else {
                            bv[u] = T(0);
                        }
                    }
                }
                Vec<T, V> xv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) xv[u] = vld<T, V>(X + (int64_t)cc[u] * ldx + c0l);
                if (RED == 2 && sizeof(T) == 4) {
                    // the dot q . p of the CG needs p's own row, which the
                    // diagonal entry has just gathered (saves a load in FP32)
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (cc[u] == (int)row) {
                            xself = xv[u];
                            found = true;
                        }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        acc.v[v] = fma(av[u], xv[u].v[v], acc.v[v]);
                        if (MODE == 2) accb.v[v] = fma(bv[u], xv[u].v[v], accb.v[v]);
                    }
            }
            if (!on) continue;
            T bx[V];
#pragma unroll
            for (int v = 0; v < V; ++v) bx[v] = T(0);
            if (MODE == 1) {
                const Vec<T, V> xs = vld<T, V>(X + row * ldx + c0);
                const T dw = (dg != nullptr) ? dg[row] : T(1);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    bx[v] = dw * xs.v[v];
                    acc.v[v] = fma(-sg[v], bx[v], acc.v[v]);
                }
            } else if (MODE == 2) {
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    bx[v] = accb.v[v];
                    acc.v[v] = fma(-sg[v], bx[v], acc.v[v]);
                }
            } else if (MODE >= 3) {
                const T w = af.w != nullptr ? af.ws * af.w[row] : af.ws;
                Vec<T, V> bb, zz;
#pragma unroll
                for (int v = 0; v < V; ++v) bb.v[v] = zz.v[v] = T(0);
                if (af.b != nullptr) bb = vld<T, V>(af.b + row * af.ldb + c0);
                if (af.z != nullptr) zz = vld<T, V>(af.z + row * af.ldz + c0);
#pragma unroll
                for (int v = 0; v < V; ++v) acc.v[v] = fma(w, bb.v[v] - acc.v[v], zz.v[v]);
            }
            if (MODE == 4 && c0 + V > k) {   // tail lane: the padding columns of Y are left untouched
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if (c0 + v < k) Y[row * ldy + c0 + v] = acc.v[v];
            } else {
                vst_nt<T, V>(Y + row * ldy + c0, acc);
            }
            if (RED == 1) {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if (c0 + v < k) {
                        red1[v] = fma(acc.v[v], acc.v[v], red1[v]);
                        red2[v] = fma(bx[v], bx[v], red2[v]);
                    }
            } else if (RED == 2) {
                Vec<T, V> z = xself;
                if (!(sizeof(T) == 4 && found && Z == X && ldz == ldx)) z = vld<T, V>(Z + row * ldz + c0);
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if (c0 + v < k) red1[v] = fma(acc.v[v], z.v[v], red1[v]);
            }
        }
        __syncthreads();
    }
    if (RED != 0) {
        __shared__ T sh[2][NG][G * V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            sh[0][grp][c0 + v] = red1[v];
            sh[1][grp][c0 + v] = red2[v];
        }
        __syncthreads();
        for (int c = tid; c < G * V; c += 256) {
            if (c >= k) continue;
            T s1 = T(0), s2 = T(0);
            for (int g = 0; g < NG; ++g) {
                s1 += sh[0][g][c];
                s2 += sh[1][g][c];
            }
            part[(size_t)c * gridDim.x + chunk] = s1;
            if (RED == 1) part[(size_t)(k + c) * gridDim.x + chunk] = s2;
        }
    }
}

template <typename T>
static inline bool aligned16(const T *p) {
    return p == nullptr || ((uintptr_t)p % 16) == 0;
}

template <typename T, int MODE, int RED>
static hipError_t spmm_dispatch(const DevCsr<T> &A, const T *vb, const T *dg, const T *sigma, const T *X,
                                int64_t ldx, int k, T *Y, int64_t ldy, const T *Z, int64_t ldz, T *part,
                                int *nparts, const int *skip, hipStream_t st, const Affine<T> &af = Affine<T>{}) {
    dim3 block(256);
    constexpr int V = 16 / sizeof(T);
    const int kp = (k + V - 1) / V * V;
    const bool vec = aligned16(X) && aligned16(Y) && aligned16(Z) && ldx % V == 0 && ldy % V == 0 &&
                     (Z == nullptr || ldz % V == 0) && kp <= ldx && kp <= ldy && (Z == nullptr || kp <= ldz) &&
                     kp <= 64 * V && aligned16(af.b) && aligned16(af.z) &&
                     (af.b == nullptr || (af.ldb % V == 0 && kp <= af.ldb)) &&
                     (af.z == nullptr || (af.ldz % V == 0 && kp <= af.ldz));
    const void *fn = nullptr;
    int units = 1;
    if (vec) {
        const int lanes = (k + V - 1) / V;
        const int G = lanes <= 4 ? 4 : lanes <= 8 ? 8 : lanes <= 16 ? 16 : lanes <= 32 ? 32 : 64;
        const int RS = std::max(256 / G, 32);
        units = (int)std::min<int64_t>((A.n + 63) / 64 * (64 / RS), 1 << 30);
#define GCGE_SPMMS(Gv)                                                                                   \
    if (G == Gv) {                                                                                       \
        fn = (const void *)k_spmms<T, Gv, V, MODE, RED>;                                                 \
        const int g = resident_grid(fn, units);                                                          \
        if (nparts) *nparts = g;                                                                         \
        hipLaunchKernelGGL((k_spmms<T, Gv, V, MODE, RED>), dim3(g), block, 0, st, A.n, A.rowptr, A.colind, \
                           A.val, vb, dg, sigma, X, ldx, k, Y, ldy, Z, ldz, part, g, (int64_t)0, skip,      \
                           A.uorder, af);                                                               \
    }
        GCGE_SPMMS(4) else GCGE_SPMMS(8) else GCGE_SPMMS(16) else GCGE_SPMMS(32) else GCGE_SPMMS(64)
#undef GCGE_SPMMS
        return hipGetLastError();
    }
    const int G = k <= 16 ? 16 : k <= 32 ? 32 : 64;
    const int CT = k <= 64 ? 1 : 2;
    units = (int)std::min<int64_t>((A.n + 256 / G - 1) / (256 / G), 1 << 30);
#define GCGE_SPMM1(Gv, CTv)                                                                              \
    if (G == Gv && CT == CTv) {                                                                          \
        fn = (const void *)k_spmm<T, Gv, CTv, MODE, RED>;                                                \
        const int g = resident_grid(fn, units);                                                          \
        if (nparts) *nparts = g;                                                                         \
        hipLaunchKernelGGL((k_spmm<T, Gv, CTv, MODE, RED>), dim3(g), block, 0, st, A.n, A.rowptr, A.colind, \
                           A.val, vb, dg, sigma, X, ldx, k, Y, ldy, Z, ldz, part, g, (int64_t)0, skip, af); \
    }
    GCGE_SPMM1(16, 1) else GCGE_SPMM1(32, 1) else GCGE_SPMM1(64, 1) else GCGE_SPMM1(64, 2)
#undef GCGE_SPMM1
    return hipGetLastError();
}

template <typename T>
hipError_t spmm(const DevCsr<T> &A, const T *vb, const T *dg, const T *sigma, int mode, int red, const T *X,
                int64_t ldx, int k, T *Y, int64_t ldy, const T *Z, int64_t ldz, T *part, int *nparts,
                hipStream_t st) {
    if (nparts) *nparts = 0;
    if (A.n == 0 || k == 0) return hipSuccess;
    if (k > 128) return hipErrorInvalidValue;
    if (red != 0 && (part == nullptr || nparts == nullptr)) return hipErrorInvalidValue;
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
                                 double *, int *, hipStream_t);
template <>
hipError_t spmm<float>(const DevCsr<float> &A, const float *vb, const float *dg, const float *sigma, int mode,
                       int red, const float *X, int64_t ldx, int k, float *Y, int64_t ldy, const float *Z,
                       int64_t ldz, float *part, int *nparts, hipStream_t st) {
    if (nparts) *nparts = 0;
    if (A.n == 0 || k == 0) return hipSuccess;
    if (k > 128) return hipErrorInvalidValue;
    if (red != 0 && (part == nullptr || nparts == nullptr)) return hipErrorInvalidValue;
    if (mode == 0 && red == 0)
        return spmm_dispatch<float, 0, 0>(A, vb, dg, sigma, X, ldx, k, Y, ldy, Z, ldz, part, nparts, nullptr, st);
    if (mode == 0 && red == 2)
        return spmm_dispatch<float, 0, 2>(A, vb, dg, sigma, X, ldx, k, Y, ldy, Z, ldz, part, nparts, nullptr, st);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t cg_spmm(const DevCsr<T> &M, const T *p, T *q, int64_t ld, int k, T *part, int *nparts, const int *flags,
                   hipStream_t st) {
    if (M.n == 0 || k == 0) return hipSuccess;
    if (k > 128) return hipErrorInvalidValue;
    return spmm_dispatch<T, 0, 2>(M, nullptr, nullptr, nullptr, p, ld, k, q, ld, p, ld, part, nparts, flags, st);
}
template hipError_t cg_spmm<double>(const DevCsr<double> &, const double *, double *, int64_t, int, double *, int *,
                                    const int *, hipStream_t);
template hipError_t cg_spmm<float>(const DevCsr<float> &, const float *, float *, int64_t, int, float *, int *,
                                   const int *, hipStream_t);

template <typename T>
hipError_t spmm_affine(const DevCsr<T> &A, const T *X, int64_t ldx, int k, T *Y, int64_t ldy, const Affine<T> &af,
                       hipStream_t st, const T *zdot, int64_t ldzdot, T *part, int *nparts, const int *skip) {
    if (nparts) *nparts = 0;
    if (A.n == 0 || k == 0) return hipSuccess;
    if (k > 128) return hipErrorInvalidValue;
    if (zdot != nullptr) {
        if (part == nullptr || nparts == nullptr) return hipErrorInvalidValue;
        if (af.exact)
            return spmm_dispatch<T, 4, 2>(A, nullptr, nullptr, nullptr, X, ldx, k, Y, ldy, zdot, ldzdot, part,
                                          nparts, skip, st, af);
        return spmm_dispatch<T, 3, 2>(A, nullptr, nullptr, nullptr, X, ldx, k, Y, ldy, zdot, ldzdot, part, nparts,
                                      skip, st, af);
    }
    if (af.exact)
        return spmm_dispatch<T, 4, 0>(A, nullptr, nullptr, nullptr, X, ldx, k, Y, ldy, nullptr, 0, nullptr, nullptr,
                                      skip, st, af);
    return spmm_dispatch<T, 3, 0>(A, nullptr, nullptr, nullptr, X, ldx, k, Y, ldy, nullptr, 0, nullptr, nullptr,
                                  skip, st, af);
}
template hipError_t spmm_affine<double>(const DevCsr<double> &, const double *, int64_t, int, double *, int64_t,
                                        const Affine<double> &, hipStream_t, const double *, int64_t, double *,
                                        int *, const int *);
template hipError_t spmm_affine<float>(const DevCsr<float> &, const float *, int64_t, int, float *, int64_t,
                                       const Affine<float> &, hipStream_t, const float *, int64_t, float *, int *,
                                       const int *);

// ---------------------------------------------------------------------------
// fixed-order column sums of partials (one work-group, 16 waves)
// ---------------------------------------------------------------------------
// Wave w sums the partials of columns c = c0 + w + 16 i (i < 8, c < k) of the
// layout part[c * nparts + p]: lane l accumulates p = l, l + 64, ... in
// increasing order (four rows of partials of all eight columns in flight),
// then the lanes are combined by wave_sum.  out[i] is valid in every lane.
template <typename T>
__device__ __forceinline__ void colsums_wave(const T *__restrict__ part, int nparts, int k, int c0, int w,
                                             int lane, T out[8]) {
    T s[8];
    bool own[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        s[i] = T(0);
        own[i] = c0 + w + 16 * i < k;
    }
    const T *base = part + (size_t)(c0 + w) * nparts;
    int p = lane;
    for (; p + 192 < nparts; p += 256) {
        T v[4][8];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int i = 0; i < 8; ++i) v[u][i] = own[i] ? base[(size_t)16 * i * nparts + p + 64 * u] : T(0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int i = 0; i < 8; ++i) s[i] += v[u][i];
    }
    for (; p < nparts; p += 64)
#pragma unroll
        for (int i = 0; i < 8; ++i) s[i] += own[i] ? base[(size_t)16 * i * nparts + p] : T(0);
#pragma unroll
    for (int i = 0; i < 8; ++i) out[i] = wave_sum(s[i]);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_colsum(const T *__restrict__ part, int nparts, int k, double *out) {
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int c0 = 0; c0 < k; c0 += 128) {
        T sums[8];
        colsums_wave(part, nparts, k, c0, w, lane, sums);
        if (lane == 0)
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (c0 + w + 16 * i < k) out[c0 + w + 16 * i] = (double)sums[i];
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
    const int chunk = blockIdx.x;
    const RowWalk rw = row_walk(n, NG);
    T acc[CT];
    double sc[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        acc[t] = T(0);
        const int c = lig + G * t;
        sc[t] = (c < k && rscale != nullptr) ? rscale[c] : 1.0;
    }
    for (int64_t base = rw.first; base < rw.end; base += rw.stride) {
        const int64_t row = base + grp;
        if (row >= rw.end) break;
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            const int c = lig + G * t;
            if (c >= k) continue;
            const T v = (T)(R[row * ldr + c] * sc[t]);
            r[row * ld + c] = v;
            p[row * ld + c] = v;
            if (x != nullptr) x[row * ld + c] = T(0);
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
        part[(size_t)c * gridDim.x + chunk] = s;
    }
}



// k_cg_init in the layout of k_cg_update_r_pk: thread t owns vector column t
// mod ldv of row offset t / ldv, U rows per step; r and p (and x = 0) are
// written as 16-byte vectors (padding columns of a partial vector get 0), the
// RHS is read with scalar loads (R may start at any column).
template <typename T, int V, int U>
__global__ __launch_bounds__(256) void k_cg_init_pk(int64_t n, int ldv, int k, const double *__restrict__ R,
                                                    int64_t ldr, const double *__restrict__ rscale,
                                                    T *__restrict__ r, T *__restrict__ p, T *__restrict__ x,
                                                    T *__restrict__ part) {
    __shared__ T sh[256 * V];
    const int tid = threadIdx.x;
    const int RW = 256 / ldv;
    const int ro = tid / ldv, c0 = (tid % ldv) * V;
    const bool act = ro < RW && c0 < k;
    const int64_t ld = (int64_t)ldv * V;
    double sc[V];
    T acc[V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
        const bool on = act && c0 + e < k;
        sc[e] = on ? (rscale != nullptr ? rscale[c0 + e] : 1.0) : 0.0;
        acc[e] = T(0);
    }
    const RowWalk rw{(int64_t)blockIdx.x * RW * U, n, (int64_t)gridDim.x * RW * U};
    if (act) {
        for (int64_t row0 = rw.first; row0 < rw.end; row0 += rw.stride) {
            double rv[U][V];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t row = min(row0 + u * RW + ro, n - 1);   // clamped: always in bounds
#pragma unroll
                for (int e = 0; e < V; ++e) rv[u][e] = c0 + e < k ? R[row * ldr + c0 + e] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t row = row0 + u * RW + ro;
                if (row >= n) continue;
                Vec<T, V> v, z;
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    v.v[e] = (T)(rv[u][e] * sc[e]);
                    z.v[e] = T(0);
                    if (c0 + e < k) acc[e] = fma(v.v[e], v.v[e], acc[e]);
                }
                vst<T, V>(r + row * ld + c0, v);
                vst<T, V>(p + row * ld + c0, v);
                if (x != nullptr) vst<T, V>(x + row * ld + c0, z);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < V; ++e) sh[tid * V + e] = acc[e];
    __syncthreads();
    for (int c = tid; c < k; c += 256) {
        T sum = T(0);
        for (int o = 0; o < RW; ++o) sum += sh[(o * ldv + c / V) * V + c % V];
        part[(size_t)c * gridDim.x + blockIdx.x] = sum;
    }
}

// Vector forms of the two CG update passes (16-byte accesses; same layout
// conditions as k_spmms).
template <typename T, int G, int V>
__global__ __launch_bounds__(256) void k_cg_update_r_v(int64_t n, int k, const T *__restrict__ q,
                                                       T *__restrict__ r, int64_t ld, T *__restrict__ part,
                                                       int nparts, int64_t rows_per, CgState<T> cs) {
    if (cs.flags[1] == 0) return;
    constexpr int NG = 256 / G;
    const int tid = threadIdx.x, grp = tid / G, lig = tid % G;
    const int chunk = blockIdx.x;
    const RowWalk rw = row_walk(n, NG);
    const int c0 = lig * V;
    const bool on = c0 < k;
    T acc[V], al[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        acc[v] = T(0);
        al[v] = (c0 + v < k) ? cs.alpha[c0 + v] : T(0);
    }
    if (on) {
        for (int64_t base = rw.first; base < rw.end; base += rw.stride) {
        const int64_t row = base + grp;
        if (row >= rw.end) break;
            const Vec<T, V> qv = vld<T, V>(q + row * ld + c0);
            Vec<T, V> rv = vld<T, V>(r + row * ld + c0);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                rv.v[v] = fma(-al[v], qv.v[v], rv.v[v]);
                if (c0 + v < k) acc[v] = fma(rv.v[v], rv.v[v], acc[v]);
            }
            vst<T, V>(r + row * ld + c0, rv);
        }
    }
    __shared__ T sh[NG][G * V];
#pragma unroll
    for (int v = 0; v < V; ++v) sh[grp][c0 + v] = acc[v];
    __syncthreads();
    for (int c = tid; c < G * V; c += 256) {
        if (c >= k) continue;
        T s = T(0);
        for (int g = 0; g < NG; ++g) s += sh[g][c];
        part[(size_t)c * gridDim.x + chunk] = s;
    }
}

template <typename T, int G, int V>
__global__ __launch_bounds__(256) void k_cg_update_xp_v(int64_t n, int k, T *__restrict__ x, T *__restrict__ p,
                                                        const T *__restrict__ r, int64_t ld, int64_t rows_per,
                                                        CgState<T> cs) {
    if (cs.flags[1] == 0) return;
    constexpr int NG = 256 / G;
    const int tid = threadIdx.x, grp = tid / G, lig = tid % G;
    const RowWalk rw = row_walk(n, NG);
    const int c0 = lig * V;
    if (c0 >= k) return;
    T al[V], be[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        al[v] = (c0 + v < k) ? cs.alpha[c0 + v] : T(0);
        be[v] = (c0 + v < k) ? cs.beta[c0 + v] : T(0);
    }
    for (int64_t base = rw.first; base < rw.end; base += rw.stride) {
        const int64_t row = base + grp;
        if (row >= rw.end) break;
        const Vec<T, V> pv = vld<T, V>(p + row * ld + c0);
        const Vec<T, V> rv = vld<T, V>(r + row * ld + c0);
        Vec<T, V> xv = vld<T, V>(x + row * ld + c0), pn;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            xv.v[v] = fma(al[v], pv.v[v], xv.v[v]);
            pn.v[v] = fma(be[v], pv.v[v], rv.v[v]);
        }
        vst<T, V>(x + row * ld + c0, xv);
        vst<T, V>(p + row * ld + c0, pn);
    }
}

// The CG vectors are n x ld row-major blocks with ld a multiple of V, so each
// block is one flat array of n * ld / V 16-byte vectors whose vector v holds
// columns (v mod ld/V) * V .. + V-1 of row v / (ld/V).  The flat kernels below
// stream those arrays with every lane busy; columns k .. ld-1 are left as they
// are.

// x += alpha p, p = r + beta p (per column): one vector per thread, one pass;
// vectors of columns >= k are not touched.
template <typename T, int V>
__global__ __launch_bounds__(256) void k_cg_update_xp_flat(int64_t nvec, int ldv, int k, T *__restrict__ x,
                                                           T *__restrict__ p, const T *__restrict__ r,
                                                           CgState<T> cs) {
    if (cs.flags[1] == 0) return;
    __shared__ T sab[2][128];
    for (int c = threadIdx.x; c < ldv * V; c += 256) {
        sab[0][c] = c < k ? cs.alpha[c] : T(0);
        sab[1][c] = c < k ? cs.beta[c] : T(0);
    }
    __syncthreads();
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= nvec) return;
    const int c0 = (int)(v % ldv) * V;
    if (c0 >= k) return;
    T *xp = x + v * V, *pp = p + v * V;
    const Vec<T, V> pv = vld<T, V>(pp), rv = vld<T, V>(r + v * V);
    Vec<T, V> xv = vld<T, V>(xp), pn;
#pragma unroll
    for (int e = 0; e < V; ++e) {
        const bool on = c0 + e < k;
        xv.v[e] = on ? fma(sab[0][c0 + e], pv.v[e], xv.v[e]) : xv.v[e];
        pn.v[e] = on ? fma(sab[1][c0 + e], pv.v[e], rv.v[e]) : pv.v[e];
    }
    vst<T, V>(xp, xv);
    vst<T, V>(pp, pn);
}

// With a search-direction history the iterate is not updated per step: step
// i writes p_(i+1) = s + beta p_i (s = r, or z when preconditioned) to a new
// slot of an n x ld ring, and x = sum_i alpha_i p_i is formed afterwards by
// k_cg_fold, which takes the terms in the order of the steps with the same
// fused multiply-adds as k_cg_update_xp_flat, so the result is the same to
// the bit; per step the two passes over x are saved.  After a step with no
// column updated (flags[1] = 0, some still active) p is carried over
// unchanged, as the in-place update leaves it; once no column is active the
// later steps are skipped and their alphas are zero.
//
// The direction update is a flat pass (one 16-byte vector per thread, as
// k_cg_update_xp_flat) whose stores stream past L2: the new slot's lines are
// not in L2, and the streaming stores measured 13 % faster than plain ones
// (0.48 against 0.55 ms for 50 FP64 columns of 2^21 rows, 3 n k 8 bytes).
template <typename T, int V>
__global__ __launch_bounds__(256) void k_cg_update_p_flat(int64_t nvec, int ldv, int k, const T *__restrict__ p,
                                                          T *__restrict__ pn, const T *__restrict__ s,
                                                          CgState<T> cs) {
    if (cs.flags[0] == 0) return;
    const bool carry = cs.flags[1] == 0;
    __shared__ T sb[128];
    for (int c = threadIdx.x; c < ldv * V; c += 256) sb[c] = c < k ? cs.beta[c] : T(0);
    __syncthreads();
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= nvec) return;
    const int c0 = (int)(v % ldv) * V;
    if (c0 >= k) return;
    const Vec<T, V> pv = vld<T, V>(p + v * V), sv = vld<T, V>(s + v * V);
    Vec<T, V> out;
#pragma unroll
    for (int e = 0; e < V; ++e) out.v[e] = (!carry && c0 + e < k) ? fma(sb[c0 + e], pv.v[e], sv.v[e]) : pv.v[e];
    vst_nt<T, V>(pn + v * V, out);
}

// The fold uses the layout of k_cg_update_r_pk: thread t owns vector column
// t mod ldv of row offset t / ldv, U rows per step, so the alphas of its
// columns stay fixed and the alpha table is read into LDS once per
// work-group (a resident grid); rows past n are clamped for the loads and
// not stored.
// x (+)= sum over steps j = first .. first+count-1 of alpha_j p_j, per
// column, j ascending (x = 0 first when init).  p_j is slot j mod H of the
// ring (slot stride sstride elements), alpha_j row j mod H of ar (row stride
// astride).  Terms with alpha = 0 are left out (a skipped step's slot may
// hold anything); vectors of columns >= k are not touched.  The loads of two
// terms are in flight together.
template <typename T, int V, int U>
__global__ __launch_bounds__(256) void k_cg_fold(int64_t n, int ldv, int k, T *__restrict__ x,
                                                 const T *__restrict__ hist, int64_t sstride, int H,
                                                 const T *__restrict__ ar, int astride, int first, int count,
                                                 int init) {
    __shared__ T sa[CG_HIST_MAX][128];
    for (int i = threadIdx.x; i < count * ldv * V; i += 256) {
        const int j = i / (ldv * V), c = i % (ldv * V);
        sa[j][c] = c < k ? ar[(int64_t)((first + j) % H) * astride + c] : T(0);
    }
    __syncthreads();
    const int tid = threadIdx.x;
    const int RW = 256 / ldv;
    const int ro = tid / ldv, c0 = (tid % ldv) * V;
    if (ro >= RW || c0 >= k) return;
    const int64_t ld = (int64_t)ldv * V;
    const RowWalk rw{(int64_t)blockIdx.x * RW * U, n, (int64_t)gridDim.x * RW * U};
    for (int64_t row0 = rw.first; row0 < rw.end; row0 += rw.stride) {
        Vec<T, V> acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = min(row0 + u * RW + ro, n - 1);
            if (init) {
#pragma unroll
                for (int e = 0; e < V; ++e) acc[u].v[e] = T(0);
            } else {
                acc[u] = vld<T, V>(x + row * ld + c0);
            }
        }
        for (int j = 0; j < count; j += 2) {
            const bool two = j + 1 < count;
            const T *s0 = hist + (int64_t)((first + j) % H) * sstride;
            const T *s1 = two ? hist + (int64_t)((first + j + 1) % H) * sstride : s0;
            Vec<T, V> p0[U], p1[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t row = min(row0 + u * RW + ro, n - 1);
                p0[u] = vld<T, V>(s0 + row * ld + c0);
                p1[u] = vld<T, V>(s1 + row * ld + c0);
            }
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const T a0 = sa[j][c0 + e], a1 = two ? sa[j + 1][c0 + e] : T(0);
                const bool c_on = c0 + e < k;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (c_on && a0 != T(0)) acc[u].v[e] = fma(a0, p0[u].v[e], acc[u].v[e]);
                    if (c_on && a1 != T(0)) acc[u].v[e] = fma(a1, p1[u].v[e], acc[u].v[e]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = row0 + u * RW + ro;
            if (row < n) vst<T, V>(x + row * ld + c0, acc[u]);
        }
    }
}

// r -= alpha q with the partial sums of r.r per column.  Thread t of a
// work-group owns vector column t mod ldv of row offset t / ldv, so one pass
// of the work-group covers RW = 256 / ldv consecutive whole rows (a contiguous
// stretch of memory) with every lane but the last 256 mod ldv busy; each
// thread takes U such passes at once (2U loads in flight) and keeps one
// accumulator.  Lanes whose columns are all >= k do nothing.  Chunks of RW * U
// rows follow the XCD-aware row walk; the per-thread sums are added per column
// in row-offset order in LDS.
template <typename T, int V, int U>
__global__ __launch_bounds__(256) void k_cg_update_r_pk(int64_t n, int ldv, int k, const T *__restrict__ q,
                                                        T *__restrict__ r, T *__restrict__ part, CgState<T> cs) {
    if (cs.flags[1] == 0) return;
    __shared__ T sh[256 * V];
    const int tid = threadIdx.x;
    const int RW = 256 / ldv;
    const int ro = tid / ldv, c0 = (tid % ldv) * V;
    const bool act = ro < RW && c0 < k;
    const int64_t ld = (int64_t)ldv * V;
    T al[V], acc[V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
        al[e] = (act && c0 + e < k) ? cs.alpha[c0 + e] : T(0);
        acc[e] = T(0);
    }
    // plain interleaved walk: no reuse across rows, so no XCD partition
    const RowWalk rw{(int64_t)blockIdx.x * RW * U, n, (int64_t)gridDim.x * RW * U};
    if (act) {
        for (int64_t row0 = rw.first; row0 < rw.end; row0 += rw.stride) {
            Vec<T, V> qv[U], rv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t row = min(row0 + u * RW + ro, rw.end - 1);   // clamped: always in bounds
                qv[u] = vld<T, V>(q + row * ld + c0);
                rv[u] = vld<T, V>(r + row * ld + c0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t row = row0 + u * RW + ro;
                if (row < rw.end) {
#pragma unroll
                    for (int e = 0; e < V; ++e) {
                        rv[u].v[e] = fma(-al[e], qv[u].v[e], rv[u].v[e]);
                        if (c0 + e < k) acc[e] = fma(rv[u].v[e], rv[u].v[e], acc[e]);
                    }
                    vst<T, V>(r + row * ld + c0, rv[u]);
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < V; ++e) sh[tid * V + e] = acc[e];
    __syncthreads();
    for (int c = tid; c < k; c += 256) {
        T sum = T(0);
        for (int o = 0; o < RW; ++o) sum += sh[(o * ldv + c / V) * V + c % V];
        part[(size_t)c * gridDim.x + blockIdx.x] = sum;
    }
}

// flags[0] = active columns, flags[1] = columns with a nonzero step this iteration
template <typename T>
__global__ __launch_bounds__(1024) void k_cg_init_finish(const T *__restrict__ part, int nparts, int k,
                                                         CgState<T> cs) {
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int c0 = 0; c0 < k; c0 += 128) {
        T sums[8];
        colsums_wave(part, nparts, k, c0, w, lane, sums);
        if (lane == 0)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int c = c0 + w + 16 * i;
                if (c >= k) continue;
                const T s = sums[i];
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
        // a step past convergence: alpha = 0 (with a search-direction
        // history, every iteration's alpha is read when x is formed)
        for (int c = threadIdx.x; c < k; c += 1024) cs.alpha[c] = T(0);
        if (threadIdx.x == 0) cs.flags[1] = 0;
        return;
    }
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int c0 = 0; c0 < k; c0 += 128) {
        T sums[8];
        colsums_wave(part, nparts, k, c0, w, lane, sums);
        if (lane == 0)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int c = c0 + w + 16 * i;
                if (c >= k) continue;
                const T pq = sums[i];
                T al = T(0);
                if (cs.active[c]) {
                    if (pq > T(0)) {
                        al = (cs.rz != nullptr ? cs.rz[c] : cs.rr[c]) / pq;
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
    for (int c0 = 0; c0 < k; c0 += 128) {
        T sums[8];
        colsums_wave(part, nparts, k, c0, w, lane, sums);
        if (lane == 0)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int c = c0 + w + 16 * i;
                if (c >= k) continue;
                const T rrn = sums[i];
                T be = T(0);
                if (cs.alpha[c] != T(0)) {
                    be = rrn / cs.rr[c];
                    cs.rr[c] = rrn;
                    if (rrn <= tol2 * cs.rr0[c]) cs.active[c] = 0;
                }
                if (cs.rz == nullptr) cs.beta[c] = be;   // preconditioned: beta comes from r . z
            }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int na = 0;
        for (int c = 0; c < k; ++c) na += cs.active[c];
        cs.flags[0] = na;
    }
}

// Column-parallel alpha and beta (CgState::done set): one work-group per
// column sums that column's partials (thread t takes partials t, t + 256, ...
// in order, then the waves in order) and updates the column as k_cg_alpha /
// k_cg_beta do; the last work-group to finish (a counter it resets) counts
// the active and updated columns into flags.  Each column's sum is one fixed
// order, so results are reproducible.
template <typename T>
__device__ __forceinline__ T col_partial_sum(const T *__restrict__ part, int nparts, int c) {
    __shared__ T red[4];
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const T *base = part + (size_t)c * nparts;
    T s = T(0);
    for (int p = tid; p < nparts; p += 256) s += base[p];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}

// true in every thread of the work-group that finishes last (after its
// column's writes, which the fence publishes)
__device__ __forceinline__ bool last_of_grid(unsigned *done) {
    __shared__ bool last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

template <typename T>
__global__ __launch_bounds__(256) void k_cg_alpha_c(const T *__restrict__ part, int nparts, int k, CgState<T> cs) {
    const int c = blockIdx.x;
    if (cs.flags[0] == 0) {
        if (threadIdx.x == 0) cs.alpha[c] = T(0);
    } else {
        const T pq = col_partial_sum(part, nparts, c);
        if (threadIdx.x == 0) {
            T al = T(0);
            if (cs.active[c]) {
                if (pq > T(0)) {
                    al = (cs.rz != nullptr ? cs.rz[c] : cs.rr[c]) / pq;
                    cs.its[c] += 1;
                } else {
                    cs.active[c] = 0;   // p^T (A - theta B) p <= 0: freeze the column
                }
            }
            cs.alpha[c] = al;
        }
    }
    if (last_of_grid(cs.done) && threadIdx.x == 0) {
        int live = 0, na = 0;
        if (cs.flags[0] != 0)
            for (int j = 0; j < k; ++j) {
                live += (cs.alpha[j] != T(0)) ? 1 : 0;
                na += cs.active[j];
            }
        cs.flags[0] = na;
        cs.flags[1] = live;
        *cs.done = 0u;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_cg_beta_c(const T *__restrict__ part, int nparts, int k, T tol2,
                                                   CgState<T> cs) {
    if (cs.flags[1] == 0) return;   // the same in every work-group: the counter is not touched
    const int c = blockIdx.x;
    const T rrn = col_partial_sum(part, nparts, c);
    if (threadIdx.x == 0) {
        T be = T(0);
        if (cs.alpha[c] != T(0)) {
            be = rrn / cs.rr[c];
            cs.rr[c] = rrn;
            if (rrn <= tol2 * cs.rr0[c]) cs.active[c] = 0;
        }
        if (cs.rz == nullptr) cs.beta[c] = be;   // preconditioned: beta comes from r . z
    }
    if (last_of_grid(cs.done) && threadIdx.x == 0) {
        int na = 0;
        for (int j = 0; j < k; ++j) na += cs.active[j];
        cs.flags[0] = na;
        *cs.done = 0u;
    }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_pcg_rz(const T *__restrict__ part, int nparts, int k, int init,
                                                 CgState<T> cs) {
    if (!init && cs.flags[1] == 0) return;
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int c0 = 0; c0 < k; c0 += 128) {
        T sums[8];
        colsums_wave(part, nparts, k, c0, w, lane, sums);
        if (lane == 0)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int c = c0 + w + 16 * i;
                if (c >= k) continue;
                const T s = sums[i];
                if (init) {
                    cs.rz[c] = s;
                    cs.beta[c] = T(0);
                } else if (cs.alpha[c] != T(0)) {
                    cs.beta[c] = s / cs.rz[c];
                    cs.rz[c] = s;
                } else {
                    cs.beta[c] = T(0);
                }
            }
    }
}

// Column-dot partials: 64 lanes per row (two columns each), 4 rows per
// work-group step; the four row groups are summed in LDS in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void k_coldot_part(int64_t n, int k, const T *__restrict__ X, int64_t ldx,
                                                     const T *__restrict__ Y, int64_t ldy, T *__restrict__ part) {
    const int tid = threadIdx.x, grp = tid / 64, lane = tid % 64;
    T s0 = T(0), s1 = T(0);
    const int c0 = lane, c1 = lane + 64;
    for (int64_t r = (int64_t)blockIdx.x * 4 + grp; r < n; r += (int64_t)gridDim.x * 4) {
        if (c0 < k) s0 = fma(X[r * ldx + c0], Y[r * ldy + c0], s0);
        if (c1 < k) s1 = fma(X[r * ldx + c1], Y[r * ldy + c1], s1);
    }
    __shared__ T sh[4][128];
    sh[grp][c0] = s0;
    sh[grp][c1] = s1;
    __syncthreads();
    if (tid < 128 && tid < k) {
        const T v = ((sh[0][tid] + sh[1][tid]) + sh[2][tid]) + sh[3][tid];
        part[(size_t)tid * gridDim.x + blockIdx.x] = v;
    }
}

// Launch a row kernel instance with its resident grid; the grid size is
// stored in *np_out (the number of partials per column) when np_out != nullptr.
#define GCGE_ROW_GO(INST, units, np_out, ...)                                              \
    do {                                                                                   \
        const int g_ = resident_grid((const void *)INST, (units));                         \
        if (np_out) *(np_out) = g_;                                                        \
        hipLaunchKernelGGL(INST, dim3(g_), dim3(256), 0, st, __VA_ARGS__);                 \
    } while (0)

template <typename T>
hipError_t cg_init(const double *R, int64_t ldr, const double *rscale, int k, int64_t n, T *r, T *p, T *x,
                   int64_t ld, T *part, int *nparts, CgState<T> cs, hipStream_t st) {
    (void)cs;
    if (k > 128) return hipErrorInvalidValue;
    constexpr int V = 16 / sizeof(T);
    if (ld % V == 0 && (k + V - 1) / V * V <= ld && ld <= 64 * V && aligned16(r) && aligned16(p) && aligned16(x)) {
        const int ldv = (int)(ld / V);
        const int64_t units = (n + 4 * (256 / ldv) - 1) / (4 * (256 / ldv));
        GCGE_ROW_GO((k_cg_init_pk<T, V, 4>), units, nparts, n, ldv, k, R, ldr, rscale, r, p, x, part);
        return hipGetLastError();
    }
    const int G = k <= 16 ? 16 : k <= 32 ? 32 : 64, CT = k <= 64 ? 1 : 2;
    const int64_t units = (n + 256 / G - 1) / (256 / G);
    int g = 0;
#define GCGE_CGI(Gv, CTv)                                                                       \
    if (G == Gv && CT == CTv) {                                                                 \
        g = resident_grid((const void *)k_cg_init<T, Gv, CTv>, units);                          \
        hipLaunchKernelGGL((k_cg_init<T, Gv, CTv>), dim3(g), dim3(256), 0, st, n, k, R, ldr, rscale, r, p, x, \
                           ld, part, g, (int64_t)0);                                            \
    }
    GCGE_CGI(16, 1) else GCGE_CGI(32, 1) else GCGE_CGI(64, 1) else GCGE_CGI(64, 2)
#undef GCGE_CGI
    *nparts = g;
    return hipGetLastError();
}

template <typename T>
hipError_t cg_init_finish(const T *part, int nparts, int k, CgState<T> cs, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_init_finish<T>, dim3(1), dim3(1024), 0, st, part, nparts, k, cs);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_alpha(const T *part, int nparts, int k, CgState<T> cs, hipStream_t st) {
    if (cs.done != nullptr && k > 0) hipLaunchKernelGGL(k_cg_alpha_c<T>, dim3(k), dim3(256), 0, st, part, nparts, k, cs);
    else hipLaunchKernelGGL(k_cg_alpha<T>, dim3(1), dim3(1024), 0, st, part, nparts, k, cs);
    return hipGetLastError();
}

template <typename T>
static inline bool cg_vec_ok(int k, int64_t ld, const T *a, const T *b, const T *c) {
    constexpr int V = 16 / sizeof(T);
    const int kp = (k + V - 1) / V * V;
    return ld % V == 0 && kp <= ld && kp <= 64 * V && aligned16(a) && aligned16(b) && aligned16(c);
}

template <typename T>
hipError_t cg_update_r(int64_t n, int k, const T *q, T *r, int64_t ld, T *part, int *nparts, CgState<T> cs,
                       hipStream_t st) {
    if (k > 128) return hipErrorInvalidValue;
    constexpr int V = 16 / sizeof(T);
    if (cg_vec_ok<T>(k, ld, q, r, r) && ld <= 64 * V) {
        const int ldv = (int)(ld / V);
        const int64_t units = (n + 4 * (256 / ldv) - 1) / (4 * (256 / ldv));
        GCGE_ROW_GO((k_cg_update_r_pk<T, V, 4>), units, nparts, n, ldv, k, q, r, part, cs);
        return hipGetLastError();
    }
    if (cg_vec_ok<T>(k, ld, q, r, r)) {
        const int lanes = (k + V - 1) / V;
        const int G = lanes <= 4 ? 4 : lanes <= 8 ? 8 : lanes <= 16 ? 16 : lanes <= 32 ? 32 : 64;
        const int64_t units = (n + 256 / G - 1) / (256 / G);
#define GCGE_UR(Gv) \
    if (G == Gv) { GCGE_ROW_GO((k_cg_update_r_v<T, Gv, V>), units, nparts, n, k, q, r, ld, part, 0, (int64_t)0, cs); }
        GCGE_UR(4) else GCGE_UR(8) else GCGE_UR(16) else GCGE_UR(32) else GCGE_UR(64)
#undef GCGE_UR
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t cg_beta(const T *part, int nparts, int k, double rel_tol, CgState<T> cs, hipStream_t st) {
    const T tol2 = (T)(rel_tol * rel_tol);
    if (cs.done != nullptr && k > 0)
        hipLaunchKernelGGL(k_cg_beta_c<T>, dim3(k), dim3(256), 0, st, part, nparts, k, tol2, cs);
    else hipLaunchKernelGGL(k_cg_beta<T>, dim3(1), dim3(1024), 0, st, part, nparts, k, tol2, cs);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_update_xp(int64_t n, int k, T *x, T *p, const T *r, int64_t ld, CgState<T> cs, hipStream_t st) {
    if (k > 128) return hipErrorInvalidValue;
    constexpr int V = 16 / sizeof(T);
    if (cg_vec_ok<T>(k, ld, x, p, r) && ld <= 128) {
        const int64_t nvec = n * (ld / V);
        const int64_t blocks = (nvec + 255) / 256;
        if (blocks < (int64_t)1 << 31) {
            hipLaunchKernelGGL((k_cg_update_xp_flat<T, V>), dim3((unsigned)blocks), dim3(256), 0, st, nvec,
                               (int)(ld / V), k, x, p, r, cs);
            return hipGetLastError();
        }
    }
    if (cg_vec_ok<T>(k, ld, x, p, r)) {
        const int lanes = (k + V - 1) / V;
        const int G = lanes <= 4 ? 4 : lanes <= 8 ? 8 : lanes <= 16 ? 16 : lanes <= 32 ? 32 : 64;
        const int64_t units = (n + 256 / G - 1) / (256 / G);
        int *none = nullptr;
#define GCGE_UX(Gv) \
    if (G == Gv) { GCGE_ROW_GO((k_cg_update_xp_v<T, Gv, V>), units, none, n, k, x, p, r, ld, (int64_t)0, cs); }
        GCGE_UX(4) else GCGE_UX(8) else GCGE_UX(16) else GCGE_UX(32) else GCGE_UX(64)
#undef GCGE_UX
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

template <typename T>
bool cg_hist_ok(int64_t n, int k, int64_t ld, int H) {
    constexpr int V = 16 / sizeof(T);
    const int kp = (k + V - 1) / V * V;
    return H >= 2 && H <= CG_HIST_MAX && k <= 128 && ld % V == 0 && kp <= ld && ld <= 128 &&
           n * (ld / V) < ((int64_t)1 << 31) * 256;
}

template <typename T>
hipError_t cg_update_p(int64_t n, int k, const T *p, T *pn, const T *s, int64_t ld, CgState<T> cs,
                       hipStream_t st) {
    constexpr int V = 16 / sizeof(T);
    if (!cg_hist_ok<T>(n, k, ld, 2) || !aligned16(p) || !aligned16(pn) || !aligned16(s)) return hipErrorInvalidValue;
    if (n == 0 || k == 0) return hipSuccess;
    const int64_t nvec = n * (ld / V);
    hipLaunchKernelGGL((k_cg_update_p_flat<T, V>), dim3((unsigned)((nvec + 255) / 256)), dim3(256), 0, st, nvec,
                       (int)(ld / V), k, p, pn, s, cs);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_fold(int64_t n, int k, T *x, int64_t ld, const T *hist, int64_t sstride, int H, const T *ar,
                   int astride, int first, int count, bool init, hipStream_t st) {
    constexpr int V = 16 / sizeof(T);
    if (!cg_hist_ok<T>(n, k, ld, H) || count < 0 || count > H || astride < k || sstride < n * ld || !aligned16(x) ||
        !aligned16(hist) || sstride % V != 0)
        return hipErrorInvalidValue;
    if (n == 0 || k == 0 || (count == 0 && !init)) return hipSuccess;
    const int ldv = (int)(ld / V);
    const int64_t units = (n + 4 * (256 / ldv) - 1) / (4 * (256 / ldv));
    int *none = nullptr;
    GCGE_ROW_GO((k_cg_fold<T, V, 4>), units, none, n, ldv, k, x, hist, sstride, H, ar, astride, first, count,
                init ? 1 : 0);
    return hipGetLastError();
}

template <typename T>
hipError_t pcg_rz(const T *part, int nparts, int k, bool init, CgState<T> cs, hipStream_t st) {
    if (k > 128 || cs.rz == nullptr) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pcg_rz<T>, dim3(1), dim3(1024), 0, st, part, nparts, k, init ? 1 : 0, cs);
    return hipGetLastError();
}
template hipError_t pcg_rz<double>(const double *, int, int, bool, CgState<double>, hipStream_t);
template hipError_t pcg_rz<float>(const float *, int, int, bool, CgState<float>, hipStream_t);

template <typename T>
hipError_t coldot_part(int64_t n, int k, const T *X, int64_t ldx, const T *Y, int64_t ldy, T *part, int *nparts,
                       hipStream_t st) {
    if (k < 1 || k > 128 || n < 1) return hipErrorInvalidValue;
    const int g = (int)std::min<int64_t>((n + 3) / 4, (int64_t)max_row_parts());
    hipLaunchKernelGGL(k_coldot_part<T>, dim3(g), dim3(256), 0, st, n, k, X, ldx, Y, ldy, part);
    *nparts = g;
    return hipGetLastError();
}
template hipError_t coldot_part<double>(int64_t, int, const double *, int64_t, const double *, int64_t, double *,
                                        int *, hipStream_t);
template hipError_t coldot_part<float>(int64_t, int, const float *, int64_t, const float *, int64_t, float *, int *,
                                       hipStream_t);

#define GCGE_CG_INST(T)                                                                                          \
    template hipError_t cg_init<T>(const double *, int64_t, const double *, int, int64_t, T *, T *, T *, int64_t, \
                                   T *, int *, CgState<T>, hipStream_t);                                          \
    template hipError_t cg_init_finish<T>(const T *, int, int, CgState<T>, hipStream_t);                          \
    template hipError_t cg_alpha<T>(const T *, int, int, CgState<T>, hipStream_t);                                \
    template hipError_t cg_update_r<T>(int64_t, int, const T *, T *, int64_t, T *, int *, CgState<T>, hipStream_t); \
    template hipError_t cg_beta<T>(const T *, int, int, double, CgState<T>, hipStream_t);                         \
    template hipError_t cg_update_xp<T>(int64_t, int, T *, T *, const T *, int64_t, CgState<T>, hipStream_t);       \
    template bool cg_hist_ok<T>(int64_t, int, int64_t, int);                                                     \
    template hipError_t cg_update_p<T>(int64_t, int, const T *, T *, const T *, int64_t, CgState<T>, hipStream_t); \
    template hipError_t cg_fold<T>(int64_t, int, T *, int64_t, const T *, int64_t, int, const T *, int, int, int,   \
                                   bool, hipStream_t);
GCGE_CG_INST(double)
GCGE_CG_INST(float)
#undef GCGE_CG_INST

// ---------------------------------------------------------------------------
// Block inner product C = X^T diag(d) Y on the FP64 matrix cores.
// A work-group (4 waves) owns one (TM x TN) output tile over one chunk of
// rows; each wave streams every 4th group of 4 NS rows (NS = 1 for 16 x 16
// tiles, 2 for 32 x 32: the fastest measured) and feeds them straight from
// global memory into v_mfma_f64_16x16x4f64 (the 16 consecutive columns of a
// row that one MFMA operand needs are one 128-byte load).  The loads of the
// next group are in flight while the current one is consumed (NS MFMA
// steps), with clamped addresses and masked values.  When the Y tile is the X
// strip itself (X^T D X), Y is not loaded again.  The four waves' tiles are
// summed in LDS in a fixed order and written as one partial; a second kernel
// sums the partials over the chunks.
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
    const int *go;   // device flag: nothing is done when go != nullptr and *go == 0
};

template <int MB, int NB, int NS = MB == 1 ? 1 : 2>   // NS MFMA steps (4 rows each) per group
__global__ __launch_bounds__(256) void k_gram(GramParams P) {
    if (P.go != nullptr && *P.go == 0) return;
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
        xv[a] = (a * 16 + li) < tl.ncol;
        xc[a] = xv[a] ? tl.xcol0 + a * 16 + li : 0;   // clamped: loads carry no branch
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        yv[b] = yt * TN + b * 16 + li < P.k;
        yc[b] = yv[b] ? yt * TN + b * 16 + li : 0;
    }
    // Y is the X strip itself: same address, stride and valid columns
    const bool same = MB == NB && tl.xp + tl.xcol0 == P.Y + yt * TN && tl.ldx == P.ldy &&
                      tl.ncol == min(TN, P.k - yt * TN);
    double av[NS][MB], bv[NS][NB], an[NS][MB], bn[NS][NB];
    auto load = [&](int64_t rb, double (&ao)[NS][MB], double (&bo)[NS][NB]) {
        double xr[NS][MB], yr[NS][NB], dw[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int64_t row = min(rb + 4 * q + lk, r1 - 1);
#pragma unroll
            for (int a = 0; a < MB; ++a) xr[q][a] = tl.xp[row * tl.ldx + xc[a]];
            if (!same) {
#pragma unroll
                for (int b = 0; b < NB; ++b) yr[q][b] = P.Y[row * P.ldy + yc[b]];
            }
            dw[q] = P.d != nullptr ? P.d[row] : 1.0;
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const bool rv = rb + 4 * q + lk < r1;
#pragma unroll
            for (int a = 0; a < MB; ++a) ao[q][a] = (rv && xv[a]) ? xr[q][a] : 0.0;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const double y = same ? xr[q][b < MB ? b : 0] : yr[q][b];
                bo[q][b] = (rv && yv[b]) ? y * dw[q] : 0.0;
            }
        }
    };
    int64_t rb = r0 + wave * 4 * NS;
    load(rb, av, bv);
    for (; rb < r1; rb += 16 * NS) {
        load(rb + 16 * NS, an, bn);   // past the chunk end: clamped addresses, masked to zero
#pragma unroll
        for (int q = 0; q < NS; ++q)
#pragma unroll
            for (int a = 0; a < MB; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q][a], bv[q][b], acc[a][b], 0, 0, 0);
#pragma unroll
        for (int q = 0; q < NS; ++q) {
#pragma unroll
            for (int a = 0; a < MB; ++a) av[q][a] = an[q][a];
#pragma unroll
            for (int b = 0; b < NB; ++b) bv[q][b] = bn[q][b];
        }
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

// Fixed-order sums of the per-chunk partial tiles: element e of tile tp is
// the sum over c of part[(tp * nchunk + c) * TE + e].  A work-group of 16 waves
// covers 64 consecutive elements; wave w sums the w-th of 16 contiguous chunk
// ranges with 8 independent loads in flight, then the 16 range sums are added
// in range order.  The order depends only on nchunk, so results are
// reproducible.
__global__ __launch_bounds__(1024) void k_tile_reduce(GramParams P, int TN, int TE, double *C, int64_t ldc) {
    if (P.go != nullptr && *P.go == 0) return;
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int epb = (TE + 63) / 64;
    const int tp = blockIdx.x / epb, e = (blockIdx.x % epb) * 64 + lane;
    const int cs = (P.nchunk + 15) / 16;
    const int c_lo = min(P.nchunk, w * cs), c_hi = min(P.nchunk, c_lo + cs);
    const double *src = P.part + (size_t)tp * P.nchunk * TE + min(e, TE - 1);
    double s = 0.0;
    int c = c_lo;
    for (; c + 8 <= c_hi; c += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[(size_t)(c + u) * TE];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < c_hi; ++c) s += src[(size_t)c * TE];
    __shared__ double red[16][64];
    red[w][lane] = s;
    __syncthreads();
    if (w != 0 || e >= TE) return;
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) t += red[i][lane];
    const int ti = tp / P.nyt, yt = tp % P.nyt;
    const GTile tl = P.t[ti];
    const int i = e / TN, j = e % TN, cj = yt * TN + j;
    if (i < tl.ncol && cj < P.k) C[(int64_t)(tl.crow0 + i) * ldc + cj] = t;
}

// Large block inner products: a 64 x 64 tile of C per work-group over one
// chunk of rows, 4 waves of 32 x 32.  Rows are staged through LDS 32 at a
// time (X strip and the d-weighted Y strip); the next 32 rows are loaded into
// registers while the MFMAs consume the current ones.  Each work-group writes
// its partial tile; k_tile_reduce sums the partials.
template <bool HAS_D>
__global__ __launch_bounds__(512) void k_gram_lds(GramParams P) {
    if (P.go != nullptr && *P.go == 0) return;
    constexpr int T = 64, KR = 32, NT = 512;
    __shared__ double sbuf[2 * KR * T];   // X and Y stages; at the end, one wave group's tile
    double(*Xs)[T] = reinterpret_cast<double(*)[T]>(sbuf);
    double(*Ys)[T] = reinterpret_cast<double(*)[T]>(sbuf + KR * T);
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int per_chunk = P.ntile * P.nyt;
    const int chunk = lid / per_chunk, rem = lid % per_chunk;
    const int ti = rem / P.nyt, yt = rem % P.nyt;
    const GTile tl = P.t[ti];
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, li = lane % 16, lk = lane / 16;
    // waves 0-3 take rows 0-15 of each stage, waves 4-7 rows 16-31; within a
    // group, 2 x 2 waves of 32 x 32
    const int wk = wave / 4, wr = (wave % 4) / 2, wc = wave % 2;
    const int64_t r0 = (int64_t)chunk * P.rows_per, r1 = min(P.n, r0 + P.rows_per);
    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    // staging: thread t holds column t % 64 of rows t / 64 + 8 q (q = 0..3), so
    // each load instruction of a wave reads 64 consecutive doubles of one row.
    // Addresses are clamped to valid elements and the values masked, so the
    // loads carry no branches.
    const int lc = tid % 64, lr = tid / 64;
    const bool xcv = lc < tl.ncol, ycv = yt * T + lc < P.k;
    const double *xbase = tl.xp + tl.xcol0 + (xcv ? lc : 0);
    const double *ybase = P.Y + yt * T + (ycv ? lc : 0);
    constexpr int Q = KR * T / NT;
    double xr[Q], yr[Q];
    auto load = [&](int64_t rb) {
        double xv[Q], yv[Q], dv[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int64_t row = min(rb + lr + 8 * q, r1 - 1);
            xv[q] = xbase[row * tl.ldx];
            yv[q] = ybase[row * P.ldy];
            dv[q] = HAS_D ? P.d[row] : 1.0;
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const bool rv = rb + lr + 8 * q < r1;
            xr[q] = (rv && xcv) ? xv[q] : 0.0;
            yr[q] = (rv && ycv) ? yv[q] * dv[q] : 0.0;
        }
    };
    int64_t rb = r0;
    if (rb < r1) load(rb);
    for (; rb < r1; rb += KR) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            Xs[lr + 8 * q][lc] = xr[q];
            Ys[lr + 8 * q][lc] = yr[q];
        }
        __syncthreads();
        load(rb + KR);   // past the chunk end: clamped addresses, masked to zero
#pragma unroll
        for (int ks = 0; ks < KR / 2; ks += 4) {
            const int kr = wk * (KR / 2) + ks + lk;
            double av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = Xs[kr][wr * 32 + a * 16 + li];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Ys[kr][wc * 32 + b * 16 + li];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    // the second row group's tile through LDS, added to the first's (fixed order)
    if (wk == 1) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    sbuf[(wr * 32 + a * 16 + lk + 4 * r) * T + wc * 32 + b * 16 + li] = acc[a][b][r];
    }
    __syncthreads();
    if (wk == 1) return;
    double *dst = P.part + ((size_t)(ti * P.nyt + yt) * P.nchunk + chunk) * (T * T);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = wr * 32 + a * 16 + lk + 4 * r, j = wc * 32 + b * 16 + li;
                dst[i * T + j] = acc[a][b][r] + sbuf[i * T + j];
            }
}

hipError_t gram_into(int64_t n, const Segs &X, const double *Y, int64_t ldy, int k, const double *d, double *C,
                     int64_t ldc, double *part, size_t part_bytes, size_t *need, hipStream_t st, const int *go) {
    if (need) *need = 0;
    const int m = X.total();
    if (m == 0 || k == 0) return hipSuccess;
    int MB, NB;
    const bool lds = !(m <= 32 && k <= 32);
    if (m <= 16 && k <= 16) { MB = 1; NB = 1; }
    else if (m <= 32 && k <= 32) { MB = 2; NB = 2; }
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
    const size_t tile_bytes = (size_t)TM * TN * sizeof(double);
    // one residency wave of work-groups for the large-tile kernel
    const int cap = lds ? resident_grid((const void *)k_gram_lds<false>, 1 << 30, 512) : 2048;
    int nchunk = std::max(1, cap / tiles);
    nchunk = (int)std::min<int64_t>(nchunk, std::max<int64_t>(1, (n + 255) / 256));
    // a caller-sized partial buffer may hold fewer chunks (longer chunks, same kernels)
    const size_t fit = part_bytes / ((size_t)tiles * tile_bytes);
    if (fit < 1) return hipErrorInvalidValue;
    if ((size_t)nchunk > fit) nchunk = (int)fit;
    int64_t rp = (n + nchunk - 1) / nchunk;
    rp = (rp + 31) / 32 * 32;
    nchunk = (int)((n + rp - 1) / rp);
    P.nchunk = nchunk;
    P.rows_per = rp;
    if (need) {
        *need = (size_t)tiles * nchunk * tile_bytes;
        if (part == nullptr) return hipSuccess;
    }
    if (part == nullptr) return hipErrorInvalidValue;
    P.part = part;
    P.go = go;
    dim3 grid(tiles * nchunk), block(256);
    if (lds) {
        if (d != nullptr) hipLaunchKernelGGL(k_gram_lds<true>, grid, dim3(512), 0, st, P);
        else hipLaunchKernelGGL(k_gram_lds<false>, grid, dim3(512), 0, st, P);
        hipLaunchKernelGGL(k_tile_reduce, dim3(tiles * (TM * TN / 64)), dim3(1024), 0, st, P, TN, TM * TN, C, ldc);
        return hipGetLastError();
    }
#define GCGE_GRAM(MBv, NBv)                                                                     \
    if (MB == MBv && NB == NBv) {                                                               \
        hipLaunchKernelGGL((k_gram<MBv, NBv>), grid, block, 0, st, P);                          \
        hipLaunchKernelGGL(k_tile_reduce, dim3(tiles * (TM * TN / 64)), dim3(1024), 0, st, P, TN, TM * TN, C, ldc); \
    }
    GCGE_GRAM(1, 1)
    GCGE_GRAM(2, 2)
#undef GCGE_GRAM
    return hipGetLastError();
}

// gram_into keeps tiles * chunks within one residency wave of the large-tile
// kernel (64 x 64 tiles) or within 2048 work-groups of the small ones (at
// most 32 x 32 tiles).
size_t gram_part_bytes_max() {
    const size_t lds = (size_t)resident_grid((const void *)k_gram_lds<false>, 1 << 30, 512) * 64 * 64 * sizeof(double);
    const size_t small = (size_t)2048 * 32 * 32 * sizeof(double);
    return std::max(lds, small);
}

hipError_t gram(int64_t n, const Segs &X, const double *Y, int64_t ldy, int k, const double *d, double *C,
                int64_t ldc, Workspace &ws, hipStream_t st, const int *go) {
    size_t need = 0;
    hipError_t e = gram_into(n, X, Y, ldy, k, d, C, ldc, nullptr, SIZE_MAX, &need, st);
    if (e != hipSuccess || need == 0) return e;
    e = ws.ensure_part(need);
    if (e != hipSuccess) return e;
    return gram_into(n, X, Y, ldy, k, d, C, ldc, ws.part, ws.part_bytes, nullptr, st, go);
}

// ---------------------------------------------------------------------------
// Y = alpha * X S + beta * Y on the FP64 matrix cores, X read as up to
// MAX_SEG column segments, X and S tiles staged through LDS.
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
    const int *go;   // device flag: nothing is done when go != nullptr and *go == 0
};

// BM x BN output tile per work-group, WM x WN waves of (BM/WM) x (BN/WN);
// K walked in chunks of BK columns, segment by segment.  The next chunk's
// global loads are held in registers (clamped addresses, masked values, no
// branches) while the MFMAs consume the current chunk from LDS.
template <int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm(GemmParams P) {
    if (P.go != nullptr && *P.go == 0) return;
    constexpr int T = 64 * WM * WN;
    constexpr int TM = BM / WM, TN = BN / WN, MB = TM / 16, NB = TN / 16;
    constexpr int VPT = BM * BK / T, SPT = BK * BN / T;
    constexpr int VRS = T / BK, SRS = T / BN;
    static_assert(VPT * T == BM * BK && SPT * T == BK * BN, "tile / thread mismatch");
    __shared__ double Vt[BM][BK + 1];
    __shared__ double St[BK][BN];
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int rt = lid / P.nct, ct = lid % P.nct;
    const int64_t row0 = (int64_t)rt * BM;
    const int col0 = ct * BN;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, li = lane % 16, lk = lane / 16;
    const int wr = wave / WN, wc = wave % WN;
    d4 acc[MB][NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    const int vc = tid % BK, vr = tid / BK;
    const int sc = tid % BN, sr = tid / BN;
    const bool scv = col0 + sc < P.k;
    const int64_t rmax = P.n - 1;
    double vreg[VPT], sreg[SPT];
    auto load_chunk = [&](int sgi, int kc) {
        const double *xp = P.s[sgi].p;
        const int64_t xld = P.s[sgi].ld;
        const int ncol = P.s[sgi].ncol;
        const bool cv = kc + vc < ncol;
        const double *vb = xp + (cv ? kc + vc : 0);
#pragma unroll
        for (int q = 0; q < VPT; ++q) vreg[q] = vb[min(row0 + vr + VRS * q, rmax) * xld];
#pragma unroll
        for (int q = 0; q < VPT; ++q) vreg[q] = (cv && row0 + vr + VRS * q <= rmax) ? vreg[q] : 0.0;
        const double *sb = P.S + (int64_t)P.soff[sgi] * P.lds + (scv ? col0 + sc : 0);
#pragma unroll
        for (int q = 0; q < SPT; ++q) sreg[q] = sb[(int64_t)min(kc + sr + SRS * q, ncol - 1) * P.lds];
#pragma unroll
        for (int q = 0; q < SPT; ++q) sreg[q] = (scv && kc + sr + SRS * q < ncol) ? sreg[q] : 0.0;
    };
    int sgi = 0, kc = 0;
    while (sgi < P.nseg && P.s[sgi].ncol <= 0) ++sgi;
    if (sgi < P.nseg) load_chunk(sgi, 0);
    while (sgi < P.nseg) {
#pragma unroll
        for (int q = 0; q < VPT; ++q) Vt[vr + VRS * q][vc] = vreg[q];
#pragma unroll
        for (int q = 0; q < SPT; ++q) St[sr + SRS * q][sc] = sreg[q];
        __syncthreads();
        int nsgi = sgi, nkc = kc + BK;
        if (nkc >= P.s[nsgi].ncol) {
            ++nsgi;
            nkc = 0;
            while (nsgi < P.nseg && P.s[nsgi].ncol <= 0) ++nsgi;
        }
        if (nsgi < P.nseg) load_chunk(nsgi, nkc);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            double av[MB], bv[NB];
#pragma unroll
            for (int a = 0; a < MB; ++a) av[a] = Vt[wr * TM + a * 16 + li][ks + lk];
#pragma unroll
            for (int b = 0; b < NB; ++b) bv[b] = St[ks + lk][wc * TN + b * 16 + li];
#pragma unroll
            for (int a = 0; a < MB; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
        sgi = nsgi;
        kc = nkc;
    }
    // epilogue: Y = alpha acc + beta Y; stores masked
    const bool addy = P.beta != 0.0;
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int col = col0 + wc * TN + b * 16 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + wr * TM + a * 16 + lk + 4 * r;
                if (row < P.n && col < P.k) {
                    double *y = P.Y + row * P.ldy + col;
                    *y = addy ? fma(P.beta, *y, P.alpha * acc[a][b][r]) : P.alpha * acc[a][b][r];
                }
            }
        }
}

// Narrow products (at most 32 input and 32 output columns, one X segment):
// a group of G lanes per row, lane l holding input column l and output
// column l; the input row is broadcast across the group by shuffles and S is
// read from LDS.  Each row depends only on itself, so Y may alias X.
template <int G>
__global__ __launch_bounds__(256) void k_gemm_rows(int64_t n, const double *X, int64_t ldx, int m,
                                                   const double *__restrict__ S, int64_t lds, int k, double alpha,
                                                   double beta, double *Y, int64_t ldy, const int *go) {
    if (go != nullptr && *go == 0) return;
    __shared__ double Ss[32 * 32];
    for (int i = threadIdx.x; i < m * k; i += 256) Ss[i] = S[(int64_t)(i / k) * lds + i % k];
    __syncthreads();
    constexpr int NGR = 256 / G, RU = 4;   // RU rows per group and step: RU loads in flight per lane
    const int grp = threadIdx.x / G, l = threadIdx.x % G;
    const int lx = l < m ? l : 0, ly = l < k ? l : 0;   // clamped columns: loads carry no branch
    for (int64_t rb = ((int64_t)blockIdx.x * NGR + grp) * RU; rb < n; rb += (int64_t)gridDim.x * NGR * RU) {
        // every row of the step is read before any is written (Y may be X):
        // rows past n read row n - 1 and are not stored
        double xv[RU], yo[RU], acc[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t rc = min(rb + u, n - 1);
            xv[u] = X[rc * ldx + lx];
            yo[u] = (beta != 0.0) ? Y[rc * ldy + ly] : 0.0;
            acc[u] = 0.0;
        }
        for (int j = 0; j < m; ++j) {
            const double sv = Ss[j * k + ly];
#pragma unroll
            for (int u = 0; u < RU; ++u) acc[u] = fma(__shfl(xv[u], j, G), sv, acc[u]);
        }
#pragma unroll
        for (int u = 0; u < RU; ++u)
            if (l < k && rb + u < n)
                Y[(rb + u) * ldy + l] = (beta != 0.0) ? fma(beta, yo[u], alpha * acc[u]) : alpha * acc[u];
    }
}

// Narrow products with at most 16 input and 16 output columns (the leaves of
// Algorithm 3): a row per 16-lane DPP row.  Lane l holds X[row][l] and column
// l of S in registers (rows of S past m are zero), and X[row][j] reaches every
// lane of the row by a DPP row broadcast (a VALU move, no LDS).  The next rows
// are loaded before the current ones are combined and stored; rows belong to
// one group, so Y may alias X.
template <int J>
__device__ __forceinline__ double row_bcast(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x150 + J, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x150 + J, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// acc[u] += sum over j = J..15 of X[row u][j] S[j][l], j in order.  The
// empty asm makes the next broadcast of each row wait for its FMA, so that at
// most RU broadcasts are live (the compiler would otherwise hoist all of them).
template <int J, int RU>
__device__ __forceinline__ void row_bcast_fma(double (&xv)[RU], const double (&sv)[16], double (&acc)[RU]) {
    if constexpr (J < 16) {
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            acc[u] = fma(row_bcast<J>(xv[u]), sv[J], acc[u]);
            asm volatile("" : "+v"(xv[u]) : "v"(acc[u]));
        }
        row_bcast_fma<J + 1, RU>(xv, sv, acc);
    }
}

__global__ __launch_bounds__(256) void k_gemm_rows16(int64_t n, const double *X, int64_t ldx, int m,
                                                     const double *__restrict__ S, int64_t lds, int k, double alpha,
                                                     double beta, double *Y, int64_t ldy, const int *go) {
    if (go != nullptr && *go == 0) return;
    constexpr int NGR = 16, RU = 4;   // 16 row groups of 16 lanes; RU rows per group and step
    const int grp = threadIdx.x / 16, l = threadIdx.x % 16;
    const int lx = l < m ? l : 0, ly = l < k ? l : 0;   // clamped columns: loads carry no branch
    double sv[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) sv[j] = (j < m && l < k) ? S[(int64_t)j * lds + l] : 0.0;
    const int64_t step = (int64_t)gridDim.x * NGR * RU;
    double xn[RU], yn[RU];
    auto load = [&](int64_t rb) {   // rows past n read row n - 1 and are not stored
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t rc = min(rb + u, n - 1);
            xn[u] = X[rc * ldx + lx];
            yn[u] = (beta != 0.0) ? Y[rc * ldy + ly] : 0.0;
        }
    };
    int64_t rb = ((int64_t)blockIdx.x * NGR + grp) * RU;
    if (rb < n) load(rb);
    for (; rb < n; rb += step) {
        double xv[RU], yo[RU], acc[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            xv[u] = xn[u];
            yo[u] = yn[u];
            acc[u] = 0.0;
        }
        if (rb + step < n) load(rb + step);
        row_bcast_fma<0, RU>(xv, sv, acc);
#pragma unroll
        for (int u = 0; u < RU; ++u)
            if (l < k && rb + u < n)
                Y[(rb + u) * ldy + l] = (beta != 0.0) ? fma(beta, yo[u], alpha * acc[u]) : alpha * acc[u];
    }
}

hipError_t gemm(int64_t n, const Segs &X, const double *S, int64_t lds, int k, double alpha, double beta,
                double *Y, int64_t ldy, hipStream_t st, const int *go) {
    if (n == 0 || k == 0) return hipSuccess;
    if (X.nseg == 1 && X.s[0].ncol <= 32 && k <= 32) {
        const int m = X.s[0].ncol, w = std::max(m, k);
        const int G = w <= 8 ? 8 : w <= 16 ? 16 : 32;
        const int64_t rows_per_wg = 256 / G * 4;
        const int64_t nb = std::min<int64_t>((n + rows_per_wg - 1) / rows_per_wg, (int64_t)num_cu() * 16);
        if (G == 16)
            hipLaunchKernelGGL(k_gemm_rows16, dim3((unsigned)nb), dim3(256), 0, st, n, X.s[0].p, X.s[0].ld, m, S, lds,
                               k, alpha, beta, Y, ldy, go);
#define GCGE_GR(Gv)                                                                                          \
    if (G == Gv) hipLaunchKernelGGL(k_gemm_rows<Gv>, dim3((unsigned)nb), dim3(256), 0, st, n, X.s[0].p, X.s[0].ld, m, \
                                    S, lds, k, alpha, beta, Y, ldy, go);
        GCGE_GR(8) GCGE_GR(32)
#undef GCGE_GR
        return hipGetLastError();
    }
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
    P.go = go;
    // up to 64 output columns: 128 x 64 tiles; wider: 128 x 128 tiles; K
    // chunks of 16 and 8 waves (4 x 2) for both (a K chunk of 32 for the
    // narrow tile measured 8 % slower at 400 -> 50 columns: it holds two
    // work-groups per CU instead of three)
    const int BN = (k <= 64) ? 64 : 128;
    P.nct = (k + BN - 1) / BN;
    const int64_t nrt = (n + 127) / 128;
    const int64_t nb = nrt * P.nct;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    if (BN == 64) hipLaunchKernelGGL((k_gemm<128, 64, 16, 4, 2>), dim3((unsigned)nb), dim3(512), 0, st, P);
    else hipLaunchKernelGGL((k_gemm<128, 128, 16, 4, 2>), dim3((unsigned)nb), dim3(512), 0, st, P);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// STEP 2 decisions on the device: the "repeat until small" tests and the drop
// decisions of Algorithms 2 and 3, written to flags that gate the launches the
// host has already enqueued (one work-group each; the blocks are small).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_orth_init(int *ints, int k, int nloops) {
    const int total = ORTH_ALIVE + k + 2 * nloops;
    for (int i = threadIdx.x; i < total; i += 256) ints[i] = (i < 2) ? 0 : 1;
}

hipError_t orth_init(int *ints, int k, int nloops, hipStream_t st) {
    hipLaunchKernelGGL(k_orth_init, dim3(1), dim3(256), 0, st, ints, k, nloops);
    return hipGetLastError();
}

__global__ __launch_bounds__(128) void k_orth_norm_scale(const double *__restrict__ G, int ldg, int k, double thr,
                                                         int *ints, double *scale, const int *go) {
    if (go != nullptr && *go == 0) return;
    for (int j = threadIdx.x; j < k; j += 128) {
        const double nu2 = G[(int64_t)j * ldg + j];
        int *alive = ints + ORTH_ALIVE + j;
        const bool keep = *alive != 0 && nu2 > thr && isfinite(nu2);
        scale[j] = keep ? 1.0 / sqrt(nu2) : 0.0;
        if (*alive && !keep) {
            *alive = 0;
            ints[1] = 1;
        }
    }
}

hipError_t orth_norm_scale(const double *G, int ldg, int k, double thr, int *ints, double *scale, const int *go,
                           hipStream_t st) {
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_orth_norm_scale, dim3(1), dim3(128), 0, st, G, ldg, k, thr, ints, scale, go);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_orth_pass_test(const double *__restrict__ R, int rows, int cols, int ldr,
                                                        double tol, int allow_skip, int allow_break, int *loop) {
    __shared__ double red[256];
    if (loop[0] == 0) {
        if (threadIdx.x == 0) loop[1] = 0;
        return;
    }
    double m = 0.0;
    for (int64_t e = threadIdx.x; e < (int64_t)rows * cols; e += 256) {
        const double v = fabs(R[(e / cols) * ldr + e % cols]);
        m = (v > m || v != v) ? v : m;   // a NaN makes the block "not small"
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            const double a = red[threadIdx.x], b = red[threadIdx.x + h];
            red[threadIdx.x] = (b > a || b != b) ? b : a;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool small = red[0] <= tol;
        loop[1] = (allow_skip && small) ? 0 : 1;
        if (allow_break && small) loop[0] = 0;
    }
}

hipError_t orth_pass_test(const double *R, int rows, int cols, int ldr, double tol, int allow_skip, int allow_break,
                          int *loop, hipStream_t st) {
    hipLaunchKernelGGL(k_orth_pass_test, dim3(1), dim3(256), 0, st, R, rows, cols, ldr, tol, allow_skip, allow_break,
                       loop);
    return hipGetLastError();
}

// Leaf pass of Algorithm 3 in one wave.  The symmetric kl x kl Gram is
// diagonalized by cyclic Jacobi rotations (Golub & Van Loan, "Matrix
// Computations", section 8.5): a rotation in the (p, q) plane with
// tau = (a_qq - a_pp) / (2 a_pq), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
// c = 1 / sqrt(1 + t^2), s = t c annihilates a_pq.  The pairs of one round
// are a perfect matching of the indices (round-robin tournament, index 0
// fixed, the others rotating), so their rotations commute: all row updates,
// then all column updates (and the eigenvector updates V <- V J).  A rotation
// is skipped when |a_pq| <= eps sqrt(|a_pp a_qq|); the sweeps end after one
// with no rotation.
constexpr int LEAF_MAX = 16;
__device__ __forceinline__ int rr_player(int pos, int round, int np) {
    return pos == 0 ? 0 : 1 + (pos - 1 + round) % (np - 1);
}

__global__ __launch_bounds__(64) void k_orth_leaf(const double *__restrict__ M, int kl, double drop_tol,
                                                  double orth_tol, int skip_final, int *ints, int s0, double *S,
                                                  int *loop) {
    constexpr int L = LEAF_MAX;
    __shared__ double a[L][L + 1], v[L][L + 1];
    __shared__ double cs[L / 2], sn[L / 2];
    __shared__ int pp[L / 2], qq[L / 2];
    __shared__ int rot;
    __shared__ double lam[L];
    __shared__ int rank[L];
    const int t = threadIdx.x;
    if (loop[0] == 0) {
        if (t == 0) loop[1] = 0;
        return;
    }
    for (int e = t; e < L * L; e += 64) {
        const int i = e / L, j = e % L;
        a[i][j] = (i < kl && j < kl) ? 0.5 * (M[i * kl + j] + M[j * kl + i]) : 0.0;
        v[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int np = (kl + 1) & ~1;   // an odd kl plays against a dummy index kl
    const int npair = np / 2;
    const double eps = 2.220446049250313e-16;
    for (int sweep = 0; sweep < 50 && kl > 1; ++sweep) {
        if (t == 0) rot = 0;
        __syncthreads();
        for (int round = 0; round < np - 1; ++round) {
            if (t < npair) {
                int p = rr_player(t, round, np), q = rr_player(np - 1 - t, round, np);
                if (p > q) {
                    const int x = p;
                    p = q;
                    q = x;
                }
                double c = 1.0, sv = 0.0;
                if (q < kl) {
                    const double apq = a[p][q], app = a[p][p], aqq = a[q][q];
                    if (apq != 0.0 && fabs(apq) > eps * sqrt(fabs(app * aqq))) {
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        sv = tt * c;
                        rot = 1;
                    }
                }
                pp[t] = p;
                qq[t] = q < kl ? q : -1;
                cs[t] = c;
                sn[t] = sv;
            }
            __syncthreads();
            for (int e = t; e < npair * L; e += 64) {   // rows p, q of J^T A
                const int i = e / L, j = e % L, p = pp[i], q = qq[i];
                if (q < 0 || j >= kl) continue;
                const double x = a[p][j], y = a[q][j];
                a[p][j] = cs[i] * x - sn[i] * y;
                a[q][j] = sn[i] * x + cs[i] * y;
            }
            __syncthreads();
            for (int e = t; e < npair * L; e += 64) {   // columns p, q of (J^T A) J and of V J
                const int i = e / L, j = e % L, p = pp[i], q = qq[i];
                if (q < 0 || j >= kl) continue;
                const double x = a[j][p], y = a[j][q];
                a[j][p] = cs[i] * x - sn[i] * y;
                a[j][q] = sn[i] * x + cs[i] * y;
                const double xv = v[j][p], yv = v[j][q];
                v[j][p] = cs[i] * xv - sn[i] * yv;
                v[j][q] = sn[i] * xv + cs[i] * yv;
            }
            __syncthreads();
        }
        if (rot == 0) break;
        __syncthreads();
    }
    // eigenvalues, their ascending order (ties by index) and the drop test
    int *alive = ints + ORTH_ALIVE + s0;
    if (t < kl) lam[t] = a[t][t];
    __syncthreads();
    if (t < kl) {
        int r = 0;
        for (int i = 0; i < kl; ++i) r += (lam[i] < lam[t] || (lam[i] == lam[t] && i < t)) ? 1 : 0;
        rank[r] = t;   // rank[r] = index of the r-th smallest eigenvalue
    }
    __syncthreads();
    if (t == 0) {
        int kk = 0, nz = 0;
        double dev = 0.0;
        for (int r = 0; r < kl; ++r) {
            const double l = lam[rank[r]];
            if (l > drop_tol && isfinite(l)) {
                ++kk;
                dev = fmax(dev, fabs(l - 1.0));
            }
        }
        for (int j = 0; j < kl; ++j) nz += alive[j] != 0;
        rot = kk;   // reuse: number kept
        const bool skip = skip_final && kk == nz && dev <= orth_tol;
        loop[1] = skip ? 0 : 1;
        if (skip || dev <= orth_tol || kk == 0) loop[0] = 0;
        if (!skip) {
            if (kk < nz) ints[1] = 1;
            for (int j = 0; j < kl; ++j) alive[j] = j < kk ? 1 : 0;
        }
    }
    __syncthreads();
    // S[:, col] = Q[:, j] / sqrt(lam_j) for the kept j in ascending order, zero after
    if (loop[1] != 0) {
        for (int e = t; e < kl * kl; e += 64) {
            const int i = e / kl, col = e % kl;
            double val = 0.0;
            if (col < rot) {
                // the col-th kept eigenvalue in ascending order
                int seen = 0, j = -1;
                for (int r = 0; r < kl; ++r) {
                    const double l = lam[rank[r]];
                    if (l > drop_tol && isfinite(l)) {
                        if (seen == col) {
                            j = rank[r];
                            break;
                        }
                        ++seen;
                    }
                }
                val = v[i][j] / sqrt(lam[j]);
            }
            S[i * kl + col] = val;
        }
    }
}

hipError_t orth_leaf(const double *M, int kl, double drop_tol, double orth_tol, int skip_final, int *ints, int s,
                     double *S, int *loop, hipStream_t st) {
    if (kl < 1 || kl > LEAF_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_orth_leaf, dim3(1), dim3(64), 0, st, M, kl, drop_tol, orth_tol, skip_final, ints, s, S,
                       loop);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_orth_mbo_coef(const double *__restrict__ c, int nu, int pass,
                                                       double *state) {
    __shared__ double red[256];
    double ss = 0.0;
    for (int i = threadIdx.x; i < nu; i += 256) ss += c[i] * c[i];
    red[threadIdx.x] = ss;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (pass == 0) state[0] = c[nu];
        state[1] = c[nu] - red[0];
    }
}

hipError_t orth_mbo_coef(const double *c, int nu, int pass, double *state, hipStream_t st) {
    hipLaunchKernelGGL(k_orth_mbo_coef, dim3(1), dim3(256), 0, st, c, nu, pass, state);
    return hipGetLastError();
}

__global__ void k_orth_mbo_keep(const double *__restrict__ state, double drop_tol, int *ints, int j, double *scale) {
    if (threadIdx.x != 0) return;
    const double n0 = state[0], n1 = state[1];
    const bool keep = ints[ORTH_ALIVE + j] != 0 && n0 > 0.0 && isfinite(n1) && n1 > drop_tol;
    scale[0] = keep ? 1.0 / sqrt(n1) : 0.0;
    if (ints[ORTH_ALIVE + j] && !keep) {
        ints[ORTH_ALIVE + j] = 0;
        ints[1] = 1;
    }
}

hipError_t orth_mbo_keep(const double *state, double drop_tol, int *ints, int j, double *scale, hipStream_t st) {
    hipLaunchKernelGGL(k_orth_mbo_keep, dim3(1), dim3(64), 0, st, state, drop_tol, ints, j, scale);
    return hipGetLastError();
}

// Kept count, and (only when something was dropped) the in-place compaction
// of every row: one wave per row walks the row in chunks of 64 columns, in
// order.  A kept column j moves to pos[j] <= j, a position that the wave has
// already read (in an earlier chunk, or in this chunk, whose loads all come
// before its stores), and a row belongs to one wave, so the move is safe in
// place.  The column map is built in LDS by each work-group.
constexpr int ORTH_FINISH_MAXK = 4096;
__global__ __launch_bounds__(256) void k_orth_finish(int64_t n, double *W, int64_t ldw, int k, int *ints) {
    __shared__ int pos[ORTH_FINISH_MAXK];
    __shared__ int kept;
    const int *alive = ints + ORTH_ALIVE;
    if (threadIdx.x == 0) {
        int c = 0;
        for (int j = 0; j < k; ++j) {
            pos[j] = alive[j] ? c : -1;
            c += alive[j] != 0;
        }
        kept = c;
        if (blockIdx.x == 0) ints[0] = c;
    }
    __syncthreads();
    if (ints[1] == 0 || kept == k) return;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int64_t row = (int64_t)blockIdx.x * 4 + wave; row < n; row += (int64_t)gridDim.x * 4) {
        double *w = W + row * ldw;
        for (int c0 = 0; c0 < k; c0 += 64) {
            const int j = c0 + lane;
            const double v = j < k ? w[j] : 0.0;
            __builtin_amdgcn_wave_barrier();
            if (j < k && pos[j] >= 0) w[pos[j]] = v;
            __builtin_amdgcn_wave_barrier();
        }
    }
}

hipError_t orth_finish(int64_t n, double *W, int64_t ldw, int k, int *ints, hipStream_t st) {
    if (k > ORTH_FINISH_MAXK) return hipErrorInvalidValue;
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>((n + 3) / 4, (int64_t)num_cu() * 8));
    hipLaunchKernelGGL(k_orth_finish, dim3((unsigned)nb), dim3(256), 0, st, n, W, ldw, k, ints);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// STEP 5 and the STEP 3 assembly on the device (the Rayleigh-Ritz quantities
// stay in device memory: xhat, Abar, phat, alpha0).
// ---------------------------------------------------------------------------
// ptilde = columns shift .. shift + nn - 1 of xhat (dim x nx, ld nx) with rows
// 0 .. n_old - 1 zeroed (eq. CP_tilde), and the norm of each of its columns.
// One work-group per column.
__global__ __launch_bounds__(256) void k_phat_init(int dim, int nx, const double *__restrict__ xhat, int shift,
                                                   int n_old, int nn, double *__restrict__ pt,
                                                   double *__restrict__ nrm0) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    double ss = 0.0;
    for (int i = threadIdx.x; i < dim; i += 256) {
        const double v = i < n_old ? 0.0 : xhat[(int64_t)i * nx + shift + j];
        pt[(int64_t)i * nn + j] = v;
        ss += v * v;
    }
    red[threadIdx.x] = ss;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) nrm0[j] = sqrt(red[0]);
}

hipError_t phat_init(int dim, int nx, const double *xhat, int shift, int n_old, int nn, double *pt, double *nrm0,
                     hipStream_t st) {
    if (nn <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_phat_init, dim3(nn), dim3(256), 0, st, dim, nx, xhat, shift, n_old, nn, pt, nrm0);
    return hipGetLastError();
}

// Gram-Schmidt among the columns of pt (dim x nn, ld nn) in one work-group:
// column j is orthogonalized against the columns kept so far (twice; each
// pass takes all coefficients against the kept columns at once), then kept
// (normalized, at the next free column of phat) when its norm exceeds
// drop_tol times its norm before the projections against xhat, nrm0[j].
// Columns of phat (dim x n_new, ld n_new) past the kept ones are zeroed; *np
// receives the kept count.  The column being processed sits in LDS (dim
// doubles, dynamic), the kept columns in phat (global, cache-resident).
constexpr int PHAT_MAXDIM = 16384, PHAT_T = 1024;
__global__ __launch_bounds__(PHAT_T) void k_phat_mgs(int dim, int nn, const double *__restrict__ pt,
                                                     const double *__restrict__ nrm0, double drop_tol,
                                                     double *__restrict__ phat, int n_new, int *np_out) {
    extern __shared__ double v[];
    __shared__ double cf[128];
    __shared__ double red[PHAT_T / 64];
    __shared__ int s_np;
    const int t = threadIdx.x, wave = t / 64, lane = t % 64, nw = PHAT_T / 64;
    if (t == 0) s_np = 0;
    __syncthreads();
    for (int j = 0; j < nn; ++j) {
        for (int i = t; i < dim; i += PHAT_T) v[i] = pt[(int64_t)i * nn + j];
        __syncthreads();
        const int np = s_np;
        for (int pass = 0; pass < 2 && np > 0; ++pass) {
            for (int q = wave; q < np; q += nw) {   // cf[q] = phat[:, q] . v, one wave per coefficient
                double s = 0.0;
                for (int i = lane; i < dim; i += 64) s += phat[(int64_t)i * n_new + q] * v[i];
                s = wave_sum(s);
                if (lane == 0) cf[q] = s;
            }
            __syncthreads();
            for (int i = t; i < dim; i += PHAT_T) {
                double x = v[i];
                for (int q = 0; q < np; ++q) x -= cf[q] * phat[(int64_t)i * n_new + q];
                v[i] = x;
            }
            __syncthreads();
        }
        double s = 0.0;
        for (int i = t; i < dim; i += PHAT_T) s += v[i] * v[i];
        s = wave_sum(s);
        if (lane == 0) red[wave] = s;
        __syncthreads();
        double nrm = 0.0;
        for (int w = 0; w < nw; ++w) nrm += red[w];
        nrm = sqrt(nrm);
        const bool keep = nrm0[j] > 0.0 && nrm > drop_tol * nrm0[j];
        if (keep)
            for (int i = t; i < dim; i += PHAT_T) phat[(int64_t)i * n_new + np] = v[i] / nrm;
        __syncthreads();
        if (t == 0 && keep) s_np = np + 1;
        __syncthreads();
    }
    const int np = s_np;
    for (int e = t; e < dim * (n_new - np); e += PHAT_T) {
        const int i = e / (n_new - np), q = np + e % (n_new - np);
        phat[(int64_t)i * n_new + q] = 0.0;
    }
    if (t == 0) np_out[0] = np;
}

hipError_t phat_mgs(int dim, int nn, const double *pt, const double *nrm0, double drop_tol, double *phat, int n_new,
                    int *np, hipStream_t st) {
    if (dim > PHAT_MAXDIM || nn > 128 || n_new > 128 || nn > n_new) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_phat_mgs, dim3(1), dim3(PHAT_T), sizeof(double) * dim, st, dim, nn, pt, nrm0, drop_tol, phat,
                       n_new, np);
    return hipGetLastError();
}

// Abar over V_u = [X_u, P, W] (dim = nx + np + nw) with the structure of
// Section 3.2: X_u^T A X_u = diag(lam), X_u^T A P = 0, P^T A P = alpha0
// (symmetrized), and the last block column [X_u, P, W]^T A W = G (dim x nw,
// ld nw), mirrored below the diagonal, its W block symmetrized.
__global__ __launch_bounds__(256) void k_assemble_abar(int dim, int nx, int np, int nw, const double *__restrict__ lam,
                                                       const double *__restrict__ a0, int lda0,
                                                       const double *__restrict__ G, double *__restrict__ Ab) {
    const int64_t total = (int64_t)dim * dim;
    const int wb = nx + np;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int i = (int)(e / dim), j = (int)(e % dim);
        double v = 0.0;
        if (i >= wb && j >= wb) {
            v = 0.5 * (G[(int64_t)i * nw + (j - wb)] + G[(int64_t)j * nw + (i - wb)]);
        } else if (j >= wb) {
            v = G[(int64_t)i * nw + (j - wb)];
        } else if (i >= wb) {
            v = G[(int64_t)j * nw + (i - wb)];
        } else if (i < nx && j < nx) {
            v = (i == j) ? lam[i] : 0.0;
        } else if (i >= nx && j >= nx) {
            const int a = i - nx, b = j - nx;
            v = 0.5 * (a0[(int64_t)a * lda0 + b] + a0[(int64_t)b * lda0 + a]);
        }
        Ab[e] = v;
    }
}

hipError_t assemble_abar(int dim, int nx, int np, int nw, const double *lam, const double *a0, int lda0,
                         const double *G, double *Ab, hipStream_t st) {
    if (dim <= 0) return hipSuccess;
    const int64_t total = (int64_t)dim * dim;
    hipLaunchKernelGGL(k_assemble_abar, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 4096)), dim3(256), 0,
                       st, dim, nx, np, nw, lam, a0, lda0, G, Ab);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small elementwise kernels
// ---------------------------------------------------------------------------
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_copy_cols(int64_t n, int k, const TI *X, int64_t ldx, TO *Y, int64_t ldy,
                                                   const double *__restrict__ scale, const int *go) {
    if (go != nullptr && *go == 0) return;
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
                     hipStream_t st, const int *go) {
    if (n == 0 || k == 0) return hipSuccess;
    hipLaunchKernelGGL((k_copy_cols<TI, TO>), dim3(ew_grid(n * k)), dim3(256), 0, st, n, k, X, ldx, Y, ldy, scale, go);
    return hipGetLastError();
}
template hipError_t copy_cols<double, double>(int64_t, int, const double *, int64_t, double *, int64_t,
                                                const double *, hipStream_t, const int *);
template hipError_t copy_cols<float, double>(int64_t, int, const float *, int64_t, double *, int64_t,
                                                const double *, hipStream_t, const int *);
template hipError_t copy_cols<double, float>(int64_t, int, const double *, int64_t, float *, int64_t,
                                                const double *, hipStream_t, const int *);
template hipError_t copy_cols<float, float>(int64_t, int, const float *, int64_t, float *, int64_t,
                                                const double *, hipStream_t, const int *);

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

// One work-group scans all rows (a one-off check at set-up) and keeps the
// smallest offending row in LDS; thread 0 writes it.
__global__ __launch_bounds__(1024) void k_first_bad_diag(int64_t n, const int32_t *__restrict__ dpos,
                                                         const double *__restrict__ b, const double *__restrict__ dg,
                                                         int *out) {
    __shared__ int64_t lo[1024];
    int64_t best = n;
    for (int64_t i = threadIdx.x; i < n && i < best; i += 1024) {
        double v;
        if (dg != nullptr) v = dg[i];
        else v = dpos[i] >= 0 ? b[dpos[i]] : 0.0;
        if (!(v > 0.0) || !isfinite(v)) best = i;
    }
    lo[threadIdx.x] = best;
    __syncthreads();
    for (int h = 512; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) lo[threadIdx.x] = min(lo[threadIdx.x], lo[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (int)lo[0];
}

hipError_t first_nonpositive_diag(int64_t n, const int32_t *dpos, const double *b, const double *dg, int *out,
                                  hipStream_t st) {
    if (n > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_first_bad_diag, dim3(1), dim3(1024), 0, st, n, dpos, b, dg, out);
    return hipGetLastError();
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

template <typename T>
__global__ __launch_bounds__(256) void k_scale_rows(int64_t n, int k, const T *__restrict__ d, const T *__restrict__ X,
                                                    int64_t ldx, T *__restrict__ Y, int64_t ldy) {
    const int64_t total = n * k;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
        const int64_t i = t / k;
        const int j = (int)(t % k);
        Y[i * ldy + j] = d[i] * X[i * ldx + j];
    }
}

template <typename T>
hipError_t scale_rows(int64_t n, int k, const T *d, const T *X, int64_t ldx, T *Y, int64_t ldy, hipStream_t st) {
    if (n == 0 || k == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_rows<T>, dim3(ew_grid(n * k)), dim3(256), 0, st, n, k, d, X, ldx, Y, ldy);
    return hipGetLastError();
}
template hipError_t scale_rows<double>(int64_t, int, const double *, const double *, int64_t, double *, int64_t,
                                       hipStream_t);
template hipError_t scale_rows<float>(int64_t, int, const float *, const float *, int64_t, float *, int64_t,
                                      hipStream_t);

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
hipError_t Workspace::ensure_orth(size_t bytes) { return grow((void **)&orth, &orth_bytes, bytes); }
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
