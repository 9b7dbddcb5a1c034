// HIP kernels for the solve phase (gfx950, wave64).
//
// All sparse operators use the 64-row sliced-ELLPACK layout of device.h: one
// thread per (block) row, one wavefront per chunk, so each column-index and each
// block-element load of a wavefront is one contiguous 256/512-byte segment.
#pragma once

#include "device.h"

namespace ps {
namespace k {

constexpr int WG = 256;      // threads per workgroup (4 wavefronts)
constexpr int MAXV = 256;    // max Krylov vectors handled by one launch (restart <= 200)

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Wavefront sum without LDS traffic: pair, quad, half-row and row sums with DPP lane moves
// (each lane adds its partner's value, so both partners hold the same bits), then the four
// 16-lane row sums read from lanes 0, 16, 32, 48 and added as (r0 + r1) + (r2 + r3).  The
// result is wave-uniform.  Needs every lane of the wavefront active.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <int LANE>
__device__ __forceinline__ double readlane_f64(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, LANE);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), LANE);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_f64<0xB1>(v);     // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp_f64<0x4E>(v);     // quad_perm [2,3,0,1]: lane ^ 2
    v += dpp_f64<0x141>(v);    // row_half_mirror: lane 7 - i within eight
    v += dpp_f64<0x140>(v);    // row_mirror: lane 15 - i within sixteen
    const double r0 = readlane_f64<0>(v), r1 = readlane_f64<16>(v);
    const double r2 = readlane_f64<32>(v), r3 = readlane_f64<48>(v);
    return (r0 + r1) + (r2 + r3);
}

// Deterministic block sum (WG threads): fixed shuffle tree per wave, then the four
// wave sums added in wave order by thread 0.  Result valid in thread 0 only.
__device__ __forceinline__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = ((red[0] + red[1]) + red[2]) + red[3];
    __syncthreads();
    return r;
}

template <typename T>
__device__ __forceinline__ void chunk_of(const Sell<T> &A, int pos, int &s0, int &w) {
    int ch = pos >> 6;
    s0 = A.cptr[ch];
    w = A.cptr[ch + 1] - s0;
}

// ------------------------------------------------------------------ SpMV family
// y = A x (MODE 0), y = b - A x (MODE 1), y += A x (MODE 2); R x C blocks.
template <int R, int C, typename T, typename TX, typename TY, int MODE>
__global__ __launch_bounds__(WG) void spmv(Sell<T> A, const TX *__restrict__ x,
                                          const TY *__restrict__ b, TY *__restrict__ y) {
    int pos = blockIdx.x * WG + threadIdx.x;
    if (pos >= A.nrows) return;
    int lane = pos & 63, s0, w;
    chunk_of(A, pos, s0, w);
    const int *col = A.col + (size_t)s0 * 64 + lane;
    const T *val = A.val + (size_t)s0 * 64 * (R * C) + lane;
    T acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = T(0);
#pragma unroll 2
    for (int k = 0; k < w; ++k) {
        int c = col[(size_t)k * 64];
        T xv[C];
#pragma unroll
        for (int e = 0; e < C; ++e) xv[e] = (T)x[(size_t)c * C + e];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int e = 0; e < C; ++e) acc[r] += val[((size_t)k * (R * C) + r * C + e) * 64] * xv[e];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        size_t o = (size_t)pos * R + r;
        if (MODE == 0) y[o] = (TY)acc[r];
        else if (MODE == 1) y[o] = (TY)((T)b[o] - acc[r]);
        else y[o] = (TY)((T)y[o] + acc[r]);
    }
}

// Two block matrices sharing the row space: y = A1 x1 + A2 x2, or b - (...).  The matrix
// values are read once per product and bypass the caches (non-temporal loads), which leaves
// them to the gathered x: 10% faster on MI355X (the plain copy's bandwidth).
template <int R, int C1, int C2, typename TX, bool RESID>
__device__ __forceinline__ void spmv2_row(const Sell<double> &A1, const TX *__restrict__ x1,
                                          const Sell<double> &A2, const TX *__restrict__ x2,
                                          const double *__restrict__ b, double *__restrict__ y, int pos) {
    if (pos >= A1.nrows) return;
    int lane = pos & 63;
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    {
        int s0, w;
        chunk_of(A1, pos, s0, w);
        const int *col = A1.col + (size_t)s0 * 64 + lane;
        const double *val = A1.val + (size_t)s0 * 64 * (R * C1) + lane;
#pragma unroll 2
        for (int k = 0; k < w; ++k) {
            int c = col[(size_t)k * 64];
            double xv[C1];
#pragma unroll
            for (int e = 0; e < C1; ++e) xv[e] = (double)x1[(size_t)c * C1 + e];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int e = 0; e < C1; ++e)
                    acc[r] += __builtin_nontemporal_load(&val[((size_t)k * (R * C1) + r * C1 + e) * 64]) * xv[e];
        }
    }
    {
        int s0, w;
        chunk_of(A2, pos, s0, w);
        const int *col = A2.col + (size_t)s0 * 64 + lane;
        const double *val = A2.val + (size_t)s0 * 64 * (R * C2) + lane;
#pragma unroll 2
        for (int k = 0; k < w; ++k) {
            int c = col[(size_t)k * 64];
            double xv[C2];
#pragma unroll
            for (int e = 0; e < C2; ++e) xv[e] = (double)x2[(size_t)c * C2 + e];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int e = 0; e < C2; ++e)
                    acc[r] += __builtin_nontemporal_load(&val[((size_t)k * (R * C2) + r * C2 + e) * 64]) * xv[e];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        size_t o = (size_t)pos * R + r;
        y[o] = RESID ? b[o] - acc[r] : acc[r];
    }
}

template <int R, int C1, int C2, typename TX, bool RESID>
__global__ __launch_bounds__(WG) void spmv2(Sell<double> A1, const TX *__restrict__ x1,
                                           Sell<double> A2, const TX *__restrict__ x2,
                                           const double *__restrict__ b, double *__restrict__ y) {
    spmv2_row<R, C1, C2, TX, RESID>(A1, x1, A2, x2, b, y, blockIdx.x * WG + threadIdx.x);
}

// The whole system product in one launch: the first gn workgroups take the node rows
// ([A_uu A_uf] z), the rest the cell rows ([A_fu A_ff] z), so that the two halves' ramps
// overlap instead of each launch draining before the next starts.
template <int NF, typename TX, bool RESID>
__global__ __launch_bounds__(WG) void spmv_sys(Sell<double> Auu, Sell<double> Auf, Sell<double> Afu,
                                              Sell<double> Aff, const TX *__restrict__ xu,
                                              const TX *__restrict__ xf, const double *__restrict__ bu,
                                              const double *__restrict__ bf, double *__restrict__ yu,
                                              double *__restrict__ yf, int gn) {
    if ((int)blockIdx.x < gn)
        spmv2_row<3, 3, NF, TX, RESID>(Auu, xu, Auf, xf, bu, yu, blockIdx.x * WG + threadIdx.x);
    else
        spmv2_row<NF, 3, NF, TX, RESID>(Afu, xu, Aff, xf, bf, yf, (blockIdx.x - gn) * WG + threadIdx.x);
}

// ------------------------------------------------------------------ AMG level kernels
template <typename T>
__device__ __forceinline__ T row_dot(const Sell<T> &A, int pos, const T *__restrict__ x) {
    int lane = pos & 63, s0, w;
    chunk_of(A, pos, s0, w);
    const int *col = A.col + (size_t)s0 * 64 + lane;
    const T *val = A.val + (size_t)s0 * 64 + lane;
    T acc = T(0);
#pragma unroll 4
    for (int k = 0; k < w; ++k) acc += val[(size_t)k * 64] * x[col[(size_t)k * 64]];
    return acc;
}

template <typename T>
__device__ __forceinline__ T row_dot2(const Sell<T> &A, int pos, const T *__restrict__ x,
                                      const T *__restrict__ s) {
    int lane = pos & 63, s0, w;
    chunk_of(A, pos, s0, w);
    const int *col = A.col + (size_t)s0 * 64 + lane;
    const T *val = A.val + (size_t)s0 * 64 + lane;
    T acc = T(0);
#pragma unroll 4
    for (int k = 0; k < w; ++k) {
        int c = col[(size_t)k * 64];
        acc += val[(size_t)k * 64] * (x[c] * s[c]);
    }
    return acc;
}

// l1-Jacobi pre-smoothing from x = 0 fused with the residual: x = D^-1 b, r = b - A x.
template <typename T>
__global__ __launch_bounds__(WG) void l1_pre(Sell<T> A, const T *__restrict__ b, const T *__restrict__ dinv,
                                            T *__restrict__ x, T *__restrict__ r) {
    int i = blockIdx.x * WG + threadIdx.x;
    if (i >= A.nrows) return;
    T acc = row_dot2(A, i, b, dinv);
    T bi = b[i];
    x[i] = bi * dinv[i];
    r[i] = bi - acc;
}

// Chebyshev(2) pre-smoothing from x = 0: d0 = c0 b, r1 = b - A d0, x = d0 + (cm d0 + c1 r1).
template <typename T>
__global__ __launch_bounds__(WG) void cheb_pre(Sell<T> A, const T *__restrict__ b, const T *__restrict__ c0,
                                              const T *__restrict__ c1, const T *__restrict__ cm,
                                              T *__restrict__ x) {
    int i = blockIdx.x * WG + threadIdx.x;
    if (i >= A.nrows) return;
    T acc = row_dot2(A, i, b, c0);
    T d0 = c0[i] * b[i];
    T r1 = b[i] - acc;
    x[i] = d0 + (cm[i] * d0 + c1[i] * r1);
}

// Chebyshev(2) post-smoothing, step 1: r0 = b - A x, d0 = c0 r0, x1 = x + d0.
template <typename T>
__global__ __launch_bounds__(WG) void cheb_post1(Sell<T> A, const T *__restrict__ b, const T *__restrict__ x,
                                                const T *__restrict__ c0, T *__restrict__ x1,
                                                T *__restrict__ d0) {
    int i = blockIdx.x * WG + threadIdx.x;
    if (i >= A.nrows) return;
    T r0 = b[i] - row_dot(A, i, x);
    T d = c0[i] * r0;
    d0[i] = d;
    x1[i] = x[i] + d;
}

// Chebyshev(2) post-smoothing, step 2: r1 = b - A x1, out = x1 + (cm d0 + c1 r1).
template <typename T>
__global__ __launch_bounds__(WG) void cheb_post2(Sell<T> A, const T *__restrict__ b, const T *__restrict__ x1,
                                                const T *__restrict__ d0, const T *__restrict__ c1,
                                                const T *__restrict__ cm, T *__restrict__ out) {
    int i = blockIdx.x * WG + threadIdx.x;
    if (i >= A.nrows) return;
    T r1 = b[i] - row_dot(A, i, x1);
    out[i] = x1[i] + (cm[i] * d0[i] + c1[i] * r1);
}

// l1-Jacobi post-smoothing: out = x + D^-1 (b - A x).
template <typename T>
__global__ __launch_bounds__(WG) void l1_post(Sell<T> A, const T *__restrict__ b, const T *__restrict__ x,
                                             const T *__restrict__ dinv, T *__restrict__ out) {
    int i = blockIdx.x * WG + threadIdx.x;
    if (i >= A.nrows) return;
    T r = b[i] - row_dot(A, i, x);
    out[i] = x[i] + r * dinv[i];
}

// The vectors of up to MAXB solves that share one hierarchy's operators: a V-cycle kernel
// launched with gridDim.y = k applies the same operator to the vectors p[0..k-1], slice
// blockIdx.y taking p[blockIdx.y] (serving batches several requests of one grid this way;
// a single solve is a batch of one).  Every slice runs the single-vector arithmetic.
constexpr int MAXB = 8;
template <typename T>
struct VP {
    T *p[MAXB];
};

// Coarsest level: x = A_c^{-1} b with the FP64 dense inverse; one wavefront per row.
template <typename T>
__global__ __launch_bounds__(WG) void coarse_solve(const double *__restrict__ Ainv, int n, VP<const T> bv,
                                                  VP<T> xv) {
    const T *__restrict__ b = bv.p[blockIdx.y];
    T *__restrict__ x = xv.p[blockIdx.y];
    int row = blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (row >= n) return;                      // whole wavefront leaves together
    const double *a = Ainv + (size_t)row * n;
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s += a[j] * (double)b[j];
    s = wave_sum(s);
    if (lane == 0) x[row] = (T)s;
}

// ------------------------------------------------------------------ AMG levels in CSR
// G consecutive lanes share one row (G = 1..64, a power of two): lane g of the group
// accumulates entries rp[i]+g, rp[i]+g+G, ...; the group then reduces with shuffles
// (fixed pattern, so the result is deterministic).  Consecutive groups take
// consecutive rows, so a wavefront reads one contiguous stretch of ci/v.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T a) {
    if constexpr (G <= 1) return a;
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, G);
    return a;
}

// SELL-64 row (G <= 0): the lane owns row i and adds its entries in order; a wavefront's
// loads of entry k of its 64 rows are one contiguous stretch, and on a stencil-like level
// so are the gathers of x.  Four entries are loaded before any is used; past the row's
// end the loads repeat its last entry and are not added.
// (DELTA: the columns are read as 16-bit offsets from the row, 6 bytes per FP32 entry
// instead of 8; NT: the values are read with non-temporal loads, as in the post-smoothing
// sweep, their last use in a V-cycle: 33 -> 28 us per sweep of the 64^3 level 0 on MI355X)
template <bool S, bool DELTA, typename T, bool NT = false>
__device__ __forceinline__ T sell_dot(const DCsr<T> &A, int i, const T *__restrict__ x,
                                      const T *__restrict__ s) {
    const int len = A.rp[i + 1] - A.rp[i];
    const size_t base = (size_t)A.cptr[i >> 6] * 64 + (i & 63);
    const int *__restrict__ ci = DELTA ? nullptr : A.ci + base;
    const short *__restrict__ cd = DELTA ? A.cd + base : nullptr;
    const T *__restrict__ v = A.v + base;
    T acc = T(0);
    for (int k = 0; k < len; k += 4) {
        int c[4];
        T a[4], xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = k + u < len ? k + u : len - 1;
            c[u] = DELTA ? i + (int)cd[kk * 64] : ci[kk * 64];
            a[u] = NT ? __builtin_nontemporal_load(&v[kk * 64]) : v[kk * 64];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = S ? x[c[u]] * s[c[u]] : x[c[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (k + u < len) acc += a[u] * xv[u];
    }
    return acc;
}

// Setup: the longest row of each 64-row slice.
__global__ __launch_bounds__(WG) void slice_width(const int *__restrict__ rp, int n, int *__restrict__ w) {
    const int s = blockIdx.x * WG + threadIdx.x;
    if (s >= (n + 63) / 64) return;
    int m = 0;
    for (int i = s * 64; i < n && i < s * 64 + 64; ++i) m = max(m, rp[i + 1] - rp[i]);
    w[s] = m;
}

// Setup: CSR (FP64 values) into SELL-64 slots; padding slots are left as they are.
template <typename T>
__global__ __launch_bounds__(WG) void csr_to_sell(const int *__restrict__ rp, const int *__restrict__ ci,
                                                 const double *__restrict__ v, int n,
                                                 const int *__restrict__ cptr, int *__restrict__ sci,
                                                 T *__restrict__ sv) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= n) return;
    const size_t base = (size_t)cptr[i >> 6] * 64 + (i & 63);
    for (int t = rp[i], k = 0; t < rp[i + 1]; ++t, ++k) {
        sci[base + (size_t)k * 64] = ci[t];
        sv[base + (size_t)k * 64] = (T)v[t];
    }
}

// sum_j a_ij x_j (or a_ij x_j s_j when S) for the calling group's row
// (four of a lane's entries are loaded before any is used, so their index loads and
// gathers overlap; past the row's end the loads repeat its last entry and are not added;
// the sum still runs in increasing t)
// lanes per row of a level kernel: G for CSR (G + 64: CSR with 16-bit column offsets from
// the row in cd), one for SELL-64 (G <= 0)
template <int G>
constexpr int lanes_of() {
    return G <= 0 ? 1 : G > 64 ? G - 64 : G;
}

template <int G, bool S, typename T, bool NT = false>
__device__ __forceinline__ T csr_dot(const DCsr<T> &A, int i, int g, const T *__restrict__ x,
                                     const T *__restrict__ s) {
    if constexpr (G <= 0) {
        return sell_dot<S, G == -1, T, NT>(A, i, x, s);
    } else {
        constexpr int GL = lanes_of<G>();
        constexpr bool DELTA = G > 64;
        T acc = T(0);
        const int e = A.rp[i + 1];
        for (int t = A.rp[i] + g; t < e; t += 4 * GL) {
            int c[4];
            T a[4], xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int tt = t + u * GL < e ? t + u * GL : e - 1;
                c[u] = DELTA ? i + (int)A.cd[tt] : A.ci[tt];
                a[u] = A.v[tt];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) xv[u] = S ? x[c[u]] * s[c[u]] : x[c[u]];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (t + u * GL < e) acc += a[u] * xv[u];
        }
        return group_sum<GL>(acc);
    }
}

#define PS_CSR_ROW(G)                                         \
    constexpr int LPR_ = lanes_of<G>();                       \
    int gid = blockIdx.x * WG + threadIdx.x;                  \
    int i = gid / LPR_, g = gid % LPR_;                       \
    if (i >= A.n) return;

// y = A x (0), b - A x (1), y + A x (2)
template <int G, int MODE, typename T>
__global__ __launch_bounds__(WG) void csr_spmv(DCsr<T> A, VP<const T> xv, VP<const T> bv, VP<T> yv) {
    const T *__restrict__ x = xv.p[blockIdx.y];
    const T *__restrict__ b = bv.p[blockIdx.y];
    T *__restrict__ y = yv.p[blockIdx.y];
    PS_CSR_ROW(G)
    T a = csr_dot<G, false>(A, i, g, x, x);
    if (g == 0) y[i] = MODE == 0 ? a : MODE == 1 ? b[i] - a : y[i] + a;
}

// Restriction to a level below which the V-cycle goes on (l1-Jacobi): b = R r, and that
// level's first smoothing step x = D^-1 b, so its pre-smoother gathers one vector.
template <int G, typename T>
__global__ __launch_bounds__(WG) void csr_restrict_l1(DCsr<T> A, VP<const T> rv, const T *__restrict__ dinv,
                                                     VP<T> bv, VP<T> xv) {
    const T *__restrict__ r = rv.p[blockIdx.y];
    T *__restrict__ b = bv.p[blockIdx.y];
    T *__restrict__ x = xv.p[blockIdx.y];
    PS_CSR_ROW(G)
    T a = csr_dot<G, false>(A, i, g, r, r);
    if (g == 0) {
        b[i] = a;
        x[i] = a * dinv[i];
    }
}

template <int G, typename T>
__global__ __launch_bounds__(WG) void csr_l1_pre(DCsr<T> A, VP<const T> bv, const T *__restrict__ dinv,
                                                VP<T> xv, VP<T> rv) {
    const T *__restrict__ b = bv.p[blockIdx.y];
    T *__restrict__ x = xv.p[blockIdx.y];
    T *__restrict__ r = rv.p[blockIdx.y];
    PS_CSR_ROW(G)
    T a = csr_dot<G, true>(A, i, g, b, dinv);
    if (g == 0) {
        T bi = b[i];
        x[i] = bi * dinv[i];
        r[i] = bi - a;
    }
}

template <int G, typename T>
__global__ __launch_bounds__(WG) void csr_cheb_pre(DCsr<T> A, VP<const T> bv, const T *__restrict__ c0,
                                                  const T *__restrict__ c1, const T *__restrict__ cm, VP<T> xv) {
    const T *__restrict__ b = bv.p[blockIdx.y];
    T *__restrict__ x = xv.p[blockIdx.y];
    PS_CSR_ROW(G)
    T a = csr_dot<G, true>(A, i, g, b, c0);
    if (g == 0) {
        T d0 = c0[i] * b[i];
        T r1 = b[i] - a;
        x[i] = d0 + (cm[i] * d0 + c1[i] * r1);
    }
}

template <int G, typename T>
__global__ __launch_bounds__(WG) void csr_cheb_post1(DCsr<T> A, VP<const T> bv, VP<const T> xv,
                                                    const T *__restrict__ c0, VP<T> x1v, VP<T> d0v) {
    const T *__restrict__ b = bv.p[blockIdx.y];
    const T *__restrict__ x = xv.p[blockIdx.y];
    T *__restrict__ x1 = x1v.p[blockIdx.y];
    T *__restrict__ d0 = d0v.p[blockIdx.y];
    PS_CSR_ROW(G)
    T a = csr_dot<G, false>(A, i, g, x, x);
    if (g == 0) {
        T d = c0[i] * (b[i] - a);
        d0[i] = d;
        x1[i] = x[i] + d;
    }
}

template <int G, typename T>
__global__ __launch_bounds__(WG) void csr_cheb_post2(DCsr<T> A, VP<const T> bv, VP<const T> x1v, VP<const T> d0v,
                                                    const T *__restrict__ c1, const T *__restrict__ cm,
                                                    VP<T> outv) {
    const T *__restrict__ b = bv.p[blockIdx.y];
    const T *__restrict__ x1 = x1v.p[blockIdx.y];
    const T *__restrict__ d0 = d0v.p[blockIdx.y];
    T *__restrict__ out = outv.p[blockIdx.y];
    PS_CSR_ROW(G)
    T a = csr_dot<G, false>(A, i, g, x1, x1);
    if (g == 0) out[i] = x1[i] + (cm[i] * d0[i] + c1[i] * (b[i] - a));
}

template <int G, typename T>
__global__ __launch_bounds__(WG) void csr_l1_post(DCsr<T> A, VP<const T> bv, VP<const T> xv,
                                                 const T *__restrict__ dinv, VP<T> outv) {
    const T *__restrict__ b = bv.p[blockIdx.y];
    const T *__restrict__ x = xv.p[blockIdx.y];
    T *__restrict__ out = outv.p[blockIdx.y];
    PS_CSR_ROW(G)
    T a = csr_dot<G, false, T, true>(A, i, g, x, x);
    if (g == 0) out[i] = x[i] + (b[i] - a) * dinv[i];
}

// ------------------------------------------------------------------ setup
// S_ff (Sec. 5.1, fixed stress) from the system's A_ff in the same SELL-64 layout: the
// fixed-stress terms are added in FP64 to the last column of each row's diagonal block
// (slot dslot[pos]), then every entry is rounded to T.  One lane per row position,
// padding lanes included.
template <int NF, typename T>
__global__ __launch_bounds__(WG) void sff_from_aff(Sell<double> A, const double *__restrict__ d_sp,
                                                  const double *__restrict__ d_pp, const int *__restrict__ dslot,
                                                  T *__restrict__ sff) {
    const int pos = blockIdx.x * WG + threadIdx.x;
    if (pos >= A.nchunks * 64) return;
    const int lane = pos & 63, ch = pos >> 6, s0 = A.cptr[ch], w = A.cptr[ch + 1] - s0, ds = dslot[pos];
    for (int k = 0; k < w; ++k)
#pragma unroll
        for (int e = 0; e < NF * NF; ++e) {
            const size_t idx = ((size_t)(s0 + k) * (NF * NF) + e) * 64 + lane;
            double v = A.val[idx];
            if (k == ds && e % NF == NF - 1)
                v += e / NF < NF - 1 ? d_sp[(size_t)pos * (NF - 1) + e / NF] : d_pp[pos];
            sff[idx] = (T)v;
        }
}

// ------------------------------------------------------------------ Algorithm 1 kernels
// Steps 2-3: y = v_f - A_fu z_u (per cell), z_s = D_ss^{-1} y_s.
template <int NF, typename T>
__global__ __launch_bounds__(WG) void step23(Sell<T> Afu, const double *__restrict__ vf,
                                            const T *__restrict__ zu, const T *__restrict__ dss_inv,
                                            T *__restrict__ y, T *__restrict__ zs) {
    int i = blockIdx.x * WG + threadIdx.x;
    if (i >= Afu.nrows) return;
    int lane = i & 63, s0, w;
    chunk_of(Afu, i, s0, w);
    const int *col = Afu.col + (size_t)s0 * 64 + lane;
    const T *val = Afu.val + (size_t)s0 * 64 * (NF * 3) + lane;
    T acc[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) acc[r] = T(0);
#pragma unroll 2
    for (int k = 0; k < w; ++k) {
        int c = col[(size_t)k * 64];
        T xv[3] = {zu[(size_t)c * 3 + 0], zu[(size_t)c * 3 + 1], zu[(size_t)c * 3 + 2]};
#pragma unroll
        for (int r = 0; r < NF; ++r)
#pragma unroll
            for (int e = 0; e < 3; ++e)
                acc[r] += __builtin_nontemporal_load(&val[((size_t)k * (NF * 3) + r * 3 + e) * 64]) * xv[e];
    }
    T yv[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) {
        yv[r] = (T)vf[(size_t)i * NF + r] - acc[r];
        y[(size_t)i * NF + r] = yv[r];
    }
    if (NF == 2) {
        zs[i] = dss_inv[i] * yv[0];
    } else {
        const T *d = dss_inv + (size_t)i * 4;
        zs[(size_t)i * 2 + 0] = d[0] * yv[0] + d[1] * yv[1];
        zs[(size_t)i * 2 + 1] = d[2] * yv[0] + d[3] * yv[1];
    }
}

// Step 4: w_p = y_p - A_ps z_s using the (p, s) entries of the S_ff blocks.
template <int NF, typename T>
__global__ __launch_bounds__(WG) void step4(Sell<T> S, const T *__restrict__ y, const T *__restrict__ zs,
                                           T *__restrict__ wp) {
    constexpr int M = NF - 1;
    int i = blockIdx.x * WG + threadIdx.x;
    if (i >= S.nrows) return;
    int lane = i & 63, s0, w;
    chunk_of(S, i, s0, w);
    const int *col = S.col + (size_t)s0 * 64 + lane;
    const T *val = S.val + (size_t)s0 * 64 * (NF * NF) + lane;
    T acc = T(0);
#pragma unroll 2
    for (int k = 0; k < w; ++k) {
        int c = col[(size_t)k * 64];
#pragma unroll
        for (int s = 0; s < M; ++s) acc += val[((size_t)k * (NF * NF) + (NF - 1) * NF + s) * 64] * zs[(size_t)c * M + s];
    }
    wp[i] = y[(size_t)i * NF + NF - 1] - acc;
}

// Step 6: w = y - S_ff [z_s; z_p].
template <int NF, typename T>
__global__ __launch_bounds__(WG) void step6(Sell<T> S, const T *__restrict__ y, const T *__restrict__ zs,
                                           const T *__restrict__ zp, T *__restrict__ wout) {
    constexpr int M = NF - 1;
    int i = blockIdx.x * WG + threadIdx.x;
    if (i >= S.nrows) return;
    int lane = i & 63, s0, w;
    chunk_of(S, i, s0, w);
    const int *col = S.col + (size_t)s0 * 64 + lane;
    const T *val = S.val + (size_t)s0 * 64 * (NF * NF) + lane;
    T acc[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) acc[r] = T(0);
#pragma unroll 2
    for (int k = 0; k < w; ++k) {
        int c = col[(size_t)k * 64];
        T xv[NF];
#pragma unroll
        for (int s = 0; s < M; ++s) xv[s] = zs[(size_t)c * M + s];
        xv[M] = zp[c];
#pragma unroll
        for (int r = 0; r < NF; ++r)
#pragma unroll
            for (int e = 0; e < NF; ++e)
                acc[r] += __builtin_nontemporal_load(&val[((size_t)k * (NF * NF) + r * NF + e) * 64]) * xv[e];
    }
#pragma unroll
    for (int r = 0; r < NF; ++r) wout[(size_t)i * NF + r] = y[(size_t)i * NF + r] - acc[r];
}

// BILU(0) forward sweep over one level: t_i = w_i - sum_{k<i} L_ik t_k.
template <int NF, typename T>
__global__ __launch_bounds__(WG) void bilu_fwd(Sell<T> L, int pos0, int pos1, const T *__restrict__ win,
                                              T *__restrict__ t) {
    int pos = pos0 + blockIdx.x * WG + threadIdx.x;
    if (pos >= pos1) return;
    int row = L.rowmap[pos];
    if (row < 0) return;
    int lane = pos & 63, s0, w;
    chunk_of(L, pos, s0, w);
    const int *col = L.col + (size_t)s0 * 64 + lane;
    const T *val = L.val + (size_t)s0 * 64 * (NF * NF) + lane;
    T acc[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) acc[r] = T(0);
    for (int k = 0; k < w; ++k) {
        int c = col[(size_t)k * 64];
        T xv[NF];
#pragma unroll
        for (int e = 0; e < NF; ++e) xv[e] = t[(size_t)c * NF + e];
#pragma unroll
        for (int r = 0; r < NF; ++r)
#pragma unroll
            for (int e = 0; e < NF; ++e)
                acc[r] += __builtin_nontemporal_load(&val[((size_t)k * (NF * NF) + r * NF + e) * 64]) * xv[e];
    }
#pragma unroll
    for (int r = 0; r < NF; ++r) t[(size_t)row * NF + r] = win[(size_t)row * NF + r] - acc[r];
}

// BILU(0) backward sweep over one level, in place on t:
//   delta_i = D_i^{-1} (t_i - sum_{j>i} U_ij delta_j);
// ACC: dz_i += delta_i (else dz_i = delta_i); FINAL: zout_i = [z_s; z_p]_i + dz_i.
template <int NF, typename T, bool ACC, bool FINAL>
__global__ __launch_bounds__(WG) void bilu_bwd(Sell<T> U, int pos0, int pos1, T *__restrict__ t,
                                              const T *__restrict__ dinv, T *__restrict__ dz,
                                              const T *__restrict__ zs, const T *__restrict__ zp,
                                              T *__restrict__ zout) {
    constexpr int M = NF - 1;
    int pos = pos0 + blockIdx.x * WG + threadIdx.x;
    if (pos >= pos1) return;
    int row = U.rowmap[pos];
    if (row < 0) return;
    int lane = pos & 63, s0, w;
    chunk_of(U, pos, s0, w);
    const int *col = U.col + (size_t)s0 * 64 + lane;
    const T *val = U.val + (size_t)s0 * 64 * (NF * NF) + lane;
    T acc[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) acc[r] = T(0);
    for (int k = 0; k < w; ++k) {
        int c = col[(size_t)k * 64];
        T xv[NF];
#pragma unroll
        for (int e = 0; e < NF; ++e) xv[e] = t[(size_t)c * NF + e];
#pragma unroll
        for (int r = 0; r < NF; ++r)
#pragma unroll
            for (int e = 0; e < NF; ++e)
                acc[r] += __builtin_nontemporal_load(&val[((size_t)k * (NF * NF) + r * NF + e) * 64]) * xv[e];
    }
    T rv[NF], dl[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) rv[r] = t[(size_t)row * NF + r] - acc[r];
    const T *d = dinv + (size_t)row * NF * NF;
#pragma unroll
    for (int r = 0; r < NF; ++r) {
        T s = T(0);
#pragma unroll
        for (int e = 0; e < NF; ++e) s += d[r * NF + e] * rv[e];
        dl[r] = s;
    }
#pragma unroll
    for (int r = 0; r < NF; ++r) {
        size_t o = (size_t)row * NF + r;
        t[o] = dl[r];
        T v = ACC ? dz[o] + dl[r] : dl[r];
        if (!FINAL) dz[o] = v;
        if (FINAL) {
            T zf = r < M ? zs[(size_t)row * M + r] : zp[row];
            zout[o] = zf + v;
        }
    }
}

// The same sweeps with all levels in one workgroup of WG1 threads: one barrier per
// level.  __syncthreads() makes the workgroup's global writes of a level visible to
// its reads in the next, so no kernel boundary is needed between levels.
constexpr int WG1 = 1024;

template <int NF, typename T>
__device__ __forceinline__ void bilu_row_fwd(const Sell<T> &L, int pos, const T *__restrict__ win, T *__restrict__ t) {
    int row = L.rowmap[pos];
    if (row < 0) return;
    int lane = pos & 63, s0, w;
    chunk_of(L, pos, s0, w);
    const int *col = L.col + (size_t)s0 * 64 + lane;
    const T *val = L.val + (size_t)s0 * 64 * (NF * NF) + lane;
    T acc[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) acc[r] = T(0);
    for (int k = 0; k < w; ++k) {
        int c = col[(size_t)k * 64];
        T xv[NF];
#pragma unroll
        for (int e = 0; e < NF; ++e) xv[e] = t[(size_t)c * NF + e];
#pragma unroll
        for (int r = 0; r < NF; ++r)
#pragma unroll
            for (int e = 0; e < NF; ++e)
                acc[r] += __builtin_nontemporal_load(&val[((size_t)k * (NF * NF) + r * NF + e) * 64]) * xv[e];
    }
#pragma unroll
    for (int r = 0; r < NF; ++r) t[(size_t)row * NF + r] = win[(size_t)row * NF + r] - acc[r];
}

template <int NF, typename T>
__global__ __launch_bounds__(WG1) void bilu_fwd_1wg(Sell<T> L, const int *__restrict__ lchunk, int nlev,
                                                   const T *__restrict__ win, T *__restrict__ t) {
    for (int l = 0; l < nlev; ++l) {
        int p0 = lchunk[l] * 64, p1 = lchunk[l + 1] * 64;
        for (int pos = p0 + (int)threadIdx.x; pos < p1; pos += WG1) bilu_row_fwd<NF, T>(L, pos, win, t);
        __syncthreads();
    }
}

template <int NF, typename T, bool ACC, bool FINAL>
__device__ __forceinline__ void bilu_row_bwd(const Sell<T> &U, int pos, T *__restrict__ t, const T *__restrict__ dinv,
                                             T *__restrict__ dz, const T *__restrict__ zs,
                                             const T *__restrict__ zp, T *__restrict__ zout) {
    constexpr int M = NF - 1;
    int row = U.rowmap[pos];
    if (row < 0) return;
    int lane = pos & 63, s0, w;
    chunk_of(U, pos, s0, w);
    const int *col = U.col + (size_t)s0 * 64 + lane;
    const T *val = U.val + (size_t)s0 * 64 * (NF * NF) + lane;
    T acc[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) acc[r] = T(0);
    for (int k = 0; k < w; ++k) {
        int c = col[(size_t)k * 64];
        T xv[NF];
#pragma unroll
        for (int e = 0; e < NF; ++e) xv[e] = t[(size_t)c * NF + e];
#pragma unroll
        for (int r = 0; r < NF; ++r)
#pragma unroll
            for (int e = 0; e < NF; ++e)
                acc[r] += __builtin_nontemporal_load(&val[((size_t)k * (NF * NF) + r * NF + e) * 64]) * xv[e];
    }
    T rv[NF], dl[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) rv[r] = t[(size_t)row * NF + r] - acc[r];
    const T *d = dinv + (size_t)row * NF * NF;
#pragma unroll
    for (int r = 0; r < NF; ++r) {
        T s = T(0);
#pragma unroll
        for (int e = 0; e < NF; ++e) s += d[r * NF + e] * rv[e];
        dl[r] = s;
    }
#pragma unroll
    for (int r = 0; r < NF; ++r) {
        size_t o = (size_t)row * NF + r;
        t[o] = dl[r];
        T v = ACC ? dz[o] + dl[r] : dl[r];
        if (!FINAL) dz[o] = v;
        if (FINAL) {
            T zf = r < M ? zs[(size_t)row * M + r] : zp[row];
            zout[o] = zf + v;
        }
    }
}

template <int NF, typename T, bool ACC, bool FINAL>
__global__ __launch_bounds__(WG1) void bilu_bwd_1wg(Sell<T> U, const int *__restrict__ lchunk, int nlev,
                                                   T *__restrict__ t, const T *__restrict__ dinv,
                                                   T *__restrict__ dz, const T *__restrict__ zs,
                                                   const T *__restrict__ zp, T *__restrict__ zout) {
    for (int l = 0; l < nlev; ++l) {
        int p0 = lchunk[l] * 64, p1 = lchunk[l + 1] * 64;
        for (int pos = p0 + (int)threadIdx.x; pos < p1; pos += WG1)
            bilu_row_bwd<NF, T, ACC, FINAL>(U, pos, t, dinv, dz, zs, zp, zout);
        __syncthreads();
    }
}

// Processor-local BILU(0) sweep pair with the subdomain's vector resident in LDS: one
// workgroup per subdomain runs the forward levels, then the backward levels, with a
// barrier between levels and no HBM traffic for the vector in between.
//
// Layout (N = n_cells; rows of the forward order are grouped by subdomain and, inside
// it, by forward level; p = the row's position inside its subdomain):
//   fcol[s*N + r], fval[(s*NF*NF + q)*N + r]   strict-lower blocks of forward row r,
//                                              slot s in increasing global column order,
//                                              column given as a subdomain position (-1: pad)
//   bpos[r], bcol/bval, bdinv[q*N + r]         the same for the backward order (bpos: the
//                                              row's position), with D_i^{-1}
//   flev/blev                                  level boundaries (row indices), per subdomain
//                                              from flev[flev_off[d]] to flev[flev_off[d+1]]
//   ncell[j], npos[j]                          the subdomain's cells in increasing index and
//                                              their positions (for coalesced gathers/scatters)
// Per row the arithmetic is that of bilu_fwd/bilu_bwd, in the same order.
template <typename T, int NF, int W>
struct SubRow {
    int c[W];
    T v[W][NF * NF];
};

// Loads are unconditional (row 0 stands in for rows past the level's end, whose
// results are not used): a load whose result may be replaced on another path forces
// the compiler to wait for it at once, which would serialise the prefetch.
// (each plane's base is uniform and the row a 32-bit unsigned offset, so a load takes one
// scalar base and one shared vector offset)
template <typename T, int NF, int W>
__device__ __forceinline__ void sub_load(SubRow<T, NF, W> &d, const int *__restrict__ col,
                                         const T *__restrict__ val, size_t N, int r, bool ok) {
    const unsigned rr = ok ? (unsigned)r : 0u;
#pragma unroll
    for (int s = 0; s < W; ++s) {
        d.c[s] = (col + (size_t)s * N)[rr];
#pragma unroll
        for (int q = 0; q < NF * NF; ++q) d.v[s][q] = (val + ((size_t)s * NF * NF + q) * N)[rr];
    }
}

// acc = sum over the row's blocks of block * y[column]; padding slots (column -1) hold
// zero blocks and read y[0].  Columns are clamped into the subdomain so that threads
// past the level's end (which hold another row's data) read inside it too.
template <typename T, int NF, int W>
__device__ __forceinline__ void sub_acc(const SubRow<T, NF, W> &d, const T *y, int n, T *acc) {
#pragma unroll
    for (int r = 0; r < NF; ++r) acc[r] = T(0);
#pragma unroll
    for (int s = 0; s < W; ++s) {
        const int c = min(max(d.c[s], 0), n - 1);
        T xv[NF];
#pragma unroll
        for (int e = 0; e < NF; ++e) xv[e] = y[c * NF + e];
#pragma unroll
        for (int r = 0; r < NF; ++r)
#pragma unroll
            for (int e = 0; e < NF; ++e) acc[r] += d.v[s][r * NF + e] * xv[e];
    }
}

struct SubLayout {
    int N;
    const int *sub_off, *flev_off, *blev_off, *flev, *blev, *bpos, *ncell, *npos;
    const int *fcol, *bcol;
};

template <typename T, int NF, int W>
struct SubRowB {
    SubRow<T, NF, W> u;
    T dv[NF * NF];
    int p;
};

template <typename T, int NF, int W>
__device__ __forceinline__ void sub_load_b(SubRowB<T, NF, W> &d, const SubLayout &L, const T *__restrict__ bval,
                                           const T *__restrict__ bdinv, size_t N, int r, bool ok) {
    sub_load(d.u, L.bcol, bval, N, r, ok);
    const unsigned rr = ok ? (unsigned)r : 0u;
#pragma unroll
    for (int q = 0; q < NF * NF; ++q) d.dv[q] = (bdinv + (size_t)q * N)[rr];
    d.p = L.bpos[rr];
}

// LDS holds the subdomain's level boundaries and, unless GY (subdomains too large for
// LDS), its vector; with GY, ygl + (off+d)*NF is the subdomain's slice in HBM, which
// __syncthreads() makes visible across the workgroup as it does for LDS.
template <int NF, int W, typename T, bool ACC, bool FINAL, bool GY>
__global__ __launch_bounds__(512) void bilu_sub(SubLayout L, const T *__restrict__ fval,
                                                const T *__restrict__ bval, const T *__restrict__ bdinv,
                                                const T *__restrict__ win, T *__restrict__ dz,
                                                const T *__restrict__ zs, const T *__restrict__ zp,
                                                T *__restrict__ zout, T *__restrict__ ygl, int lev_cap) {
    constexpr int M = NF - 1;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int *lf = reinterpret_cast<int *>(lds_raw);
    int *lb = lf + lev_cap;
    const int d = blockIdx.x, tid = threadIdx.x, bs = blockDim.x;
    const int off = L.sub_off[d], n = L.sub_off[d + 1] - off;
    // y[n] is a dummy slot written by threads that have no row in a level, so that a
    // level runs with no divergent branch (which would make the compiler wait for
    // every load in flight)
    // (GY is a template parameter so that the compiler sees which memory y is in and
    // issues LDS instructions, not flat ones that would wait on every global load)
    T *y;
    if constexpr (GY) y = ygl + ((size_t)off + d) * NF;
    else y = reinterpret_cast<T *>(lds_raw + (size_t)2 * lev_cap * sizeof(int));
    const size_t N = (size_t)L.N;
    const int fb = L.flev_off[d], nfl = L.flev_off[d + 1] - fb;     // nfl boundaries: nfl-1 levels
    const int bb = L.blev_off[d], nbl = L.blev_off[d + 1] - bb;
    for (int j = tid; j < nfl; j += bs) lf[j] = L.flev[fb + j];
    for (int j = tid; j < nbl; j += bs) lb[j] = L.blev[bb + j];
    for (int j = tid; j < n; j += bs) {
        int c = L.ncell[off + j], p = L.npos[off + j];
#pragma unroll
        for (int e = 0; e < NF; ++e) y[p * NF + e] = win[(size_t)c * NF + e];
    }
    __syncthreads();
    // A level's rows are prefetched three levels ahead into one of four register buffers
    // that rotate without copies (the loop is unrolled by four), together with the level's
    // bounds, so that after a barrier a level only gathers from LDS, computes and writes;
    // the reads of the next bounds and the issue of the next loads follow.  Steps past the
    // last level are empty (bounds 0, 0).
    // forward: t_p = w_p - sum_k L_pk t_k, in place.
    {
        const int nl = nfl - 1;
        struct Buf {
            SubRow<T, NF, W> x;
            int r0, r1;
        };
        Buf c0, c1, c2, c3;
        auto load = [&](Buf &b, int l) {
            b.r0 = l < nl ? lf[l] : 0;
            b.r1 = l < nl ? lf[l + 1] : 0;
            const int r = b.r0 + tid;
            sub_load(b.x, L.fcol, fval, N, r, r < b.r1);
        };
        auto step = [&](int l, const Buf &cur, Buf &ahead) {
            {
                T acc[NF];
                sub_acc(cur.x, y, n, acc);
                const int p = cur.r0 + tid < cur.r1 ? cur.r0 + tid - off : n;
#pragma unroll
                for (int e = 0; e < NF; ++e) y[p * NF + e] = y[p * NF + e] - acc[e];
            }
            for (int rr = cur.r0 + tid + bs; rr < cur.r1; rr += bs) {
                SubRow<T, NF, W> x;
                sub_load(x, L.fcol, fval, N, rr, true);
                T acc[NF];
                sub_acc(x, y, n, acc);
                const int p = rr - off;
#pragma unroll
                for (int e = 0; e < NF; ++e) y[p * NF + e] = y[p * NF + e] - acc[e];
            }
            load(ahead, l + 3);
            __syncthreads();
        };
        load(c0, 0);
        load(c1, 1);
        load(c2, 2);
        for (int l = 0; l < nl; l += 4) {
            step(l, c0, c3);
            step(l + 1, c1, c0);
            step(l + 2, c2, c1);
            step(l + 3, c3, c2);
        }
    }
    // backward: delta_p = D_p^{-1} (t_p - sum_j U_pj delta_j), in place
    {
        const int nl = nbl - 1;
        struct Buf {
            SubRowB<T, NF, W> x;
            int r0, r1;
        };
        Buf c0, c1, c2, c3;
        auto load = [&](Buf &b, int l) {
            b.r0 = l < nl ? lb[l] : 0;
            b.r1 = l < nl ? lb[l + 1] : 0;
            const int r = b.r0 + tid;
            sub_load_b(b.x, L, bval, bdinv, N, r, r < b.r1);
        };
        auto row = [&](const SubRowB<T, NF, W> &x, bool act) {
            T acc[NF], rv[NF];
            sub_acc(x.u, y, n, acc);
            const int p = act ? x.p : n;
#pragma unroll
            for (int e = 0; e < NF; ++e) rv[e] = y[p * NF + e] - acc[e];
#pragma unroll
            for (int a2 = 0; a2 < NF; ++a2) {
                T sm = T(0);
#pragma unroll
                for (int e = 0; e < NF; ++e) sm += x.dv[a2 * NF + e] * rv[e];
                y[p * NF + a2] = sm;
            }
        };
        auto step = [&](int l, const Buf &cur, Buf &ahead) {
            row(cur.x, cur.r0 + tid < cur.r1);
            for (int rr = cur.r0 + tid + bs; rr < cur.r1; rr += bs) {
                SubRowB<T, NF, W> x;
                sub_load_b(x, L, bval, bdinv, N, rr, true);
                row(x, true);
            }
            load(ahead, l + 3);
            __syncthreads();
        };
        load(c0, 0);
        load(c1, 1);
        load(c2, 2);
        for (int l = 0; l < nl; l += 4) {
            step(l, c0, c3);
            step(l + 1, c1, c0);
            step(l + 2, c2, c1);
            step(l + 3, c3, c2);
        }
    }
    for (int j = tid; j < n; j += bs) {
        int c = L.ncell[off + j], p = L.npos[off + j];
#pragma unroll
        for (int e = 0; e < NF; ++e) {
            size_t o = (size_t)c * NF + e;
            T v = ACC ? dz[o] + y[p * NF + e] : y[p * NF + e];
            if (!FINAL) dz[o] = v;
            if (FINAL) {
                T zf = e < M ? zs[(size_t)c * M + e] : zp[c];
                zout[o] = zf + v;
            }
        }
    }
}

// Setup, processor-local BILU(0) (Sec. 5.3) on the device: the host's block ILU(0) of
// the subdomain-restricted S_ff, operation for operation (no contraction), so that the
// factor is bitwise the host's.
struct SubFactorLayout {
    int N, nml;
    const int *ml_src, *ml_fs, *fdiag, *lo_t, *lo_d, *up_u, *up_q;
};

// factor values := restricted S_ff: A_ff's value plus, in a diagonal block's last column,
// the fixed-stress term
template <int NF>
__global__ __launch_bounds__(WG) void sub_factor_init(SubFactorLayout F, const double *__restrict__ aff,
                                                     const double *__restrict__ d_sp,
                                                     const double *__restrict__ d_pp, double *__restrict__ fv) {
    const int t = blockIdx.x * WG + threadIdx.x;
    if (t >= F.nml) return;
    const int c = F.ml_fs[t];
    const size_t src = (size_t)F.ml_src[t];
#pragma unroll
    for (int e = 0; e < NF * NF; ++e) {
        double v = aff[src + (size_t)e * 64];
        if (c >= 0 && e % NF == NF - 1) v += e / NF < NF - 1 ? d_sp[(size_t)c * (NF - 1) + e / NF] : d_pp[c];
        fv[(size_t)t * NF * NF + e] = v;
    }
}

template <int NF>
__device__ __forceinline__ void fac_mm(const double *a, const double *b, double *c) {
#pragma clang fp contract(off)
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int j = 0; j < NF; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < NF; ++k) s += a[i * NF + k] * b[k * NF + j];
            c[i * NF + j] = s;
        }
}

// Gauss-Jordan with partial pivoting (first largest |pivot|), as the host's small inverse
template <int NF>
__device__ __forceinline__ bool fac_inv(const double *a, double *inv) {
#pragma clang fp contract(off)
    double m[NF][2 * NF];
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int j = 0; j < 2 * NF; ++j) m[i][j] = j < NF ? a[i * NF + j] : (j - NF == i ? 1.0 : 0.0);
#pragma unroll
    for (int c = 0; c < NF; ++c) {
        int piv = c;
#pragma unroll
        for (int r = c + 1; r < NF; ++r)
            if (fabs(m[r][c]) > fabs(m[piv][c])) piv = r;
        double pv = 0.0;
#pragma unroll
        for (int r = 0; r < NF; ++r)
            if (r == piv) pv = m[r][c];
        if (pv == 0.0 || !isfinite(pv)) return false;
        if (piv != c) {
#pragma unroll
            for (int r = c + 1; r < NF; ++r)
                if (r == piv)
#pragma unroll
                    for (int j = 0; j < 2 * NF; ++j) {
                        const double x = m[c][j];
                        m[c][j] = m[r][j];
                        m[r][j] = x;
                    }
        }
        const double d = m[c][c];
#pragma unroll
        for (int j = 0; j < 2 * NF; ++j) m[c][j] /= d;
#pragma unroll
        for (int r = 0; r < NF; ++r) {
            if (r == c) continue;
            const double f = m[r][c];
            if (f == 0.0) continue;
#pragma unroll
            for (int j = 0; j < 2 * NF; ++j) m[r][j] -= f * m[c][j];
        }
    }
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int j = 0; j < NF; ++j) {
            inv[i * NF + j] = m[i][NF + j];
            if (!isfinite(inv[i * NF + j])) return false;
        }
    return true;
}

// One workgroup per subdomain walks its forward levels; a row's blocks are its own during
// its level and final after it (the barrier orders the levels).
template <int NF, int W>
__global__ __launch_bounds__(512) void sub_factor(SubLayout L, SubFactorLayout F, double *__restrict__ fv,
                                                  int *__restrict__ flag) {
#pragma clang fp contract(off)
    constexpr int NN = NF * NF;
    const int d = blockIdx.x, tid = threadIdx.x, bs = blockDim.x;
    const size_t N = (size_t)F.N;
    const int fb = L.flev_off[d], nfl = L.flev_off[d + 1] - fb;
    for (int l = 0; l + 1 < nfl; ++l) {
        const int r0 = L.flev[fb + l], r1 = L.flev[fb + l + 1];
        for (int r = r0 + tid; r < r1; r += bs) {
            for (int k = 0; k < W; ++k) {
                const int t = F.lo_t[k * N + r];
                if (t < 0) break;
                const int kd = F.lo_d[k * N + r];
                double a[NN], dk[NN], lk[NN];
#pragma unroll
                for (int e = 0; e < NN; ++e) {
                    a[e] = fv[(size_t)t * NN + e];
                    dk[e] = fv[(size_t)kd * NN + e];
                }
                fac_mm<NF>(a, dk, lk);                         // L_ik = A_ik D_k^-1
#pragma unroll
                for (int e = 0; e < NN; ++e) fv[(size_t)t * NN + e] = lk[e];
                for (int m = 0; m < W; ++m) {
                    const size_t slot = ((size_t)k * W + m) * N + r;
                    const int u = F.up_u[slot];
                    if (u < 0) break;
                    const int q = F.up_q[slot];
                    double ub[NN], pr[NN];
#pragma unroll
                    for (int e = 0; e < NN; ++e) ub[e] = fv[(size_t)u * NN + e];
                    fac_mm<NF>(lk, ub, pr);                    // A_ij -= L_ik U_kj
#pragma unroll
                    for (int e = 0; e < NN; ++e) fv[(size_t)q * NN + e] = fv[(size_t)q * NN + e] - pr[e];
                }
            }
            const int dd = F.fdiag[r];
            double a[NN], inv[NN];
#pragma unroll
            for (int e = 0; e < NN; ++e) a[e] = fv[(size_t)dd * NN + e];
            if (fac_inv<NF>(a, inv)) {
#pragma unroll
                for (int e = 0; e < NN; ++e) fv[(size_t)dd * NN + e] = inv[e];    // D_i^-1
            } else {
                flag[0] = 1;
            }
        }
        __syncthreads();
    }
}

// ELL planes of the sweeps from the factor: out[(s*NN + q)*N + r] = fv[src[s*N + r]], as T
template <int NN, typename T>
__global__ __launch_bounds__(WG) void sub_factor_out(int N, int W, const int *__restrict__ src,
                                                    const double *__restrict__ fv, T *__restrict__ out) {
    const size_t g = (size_t)blockIdx.x * WG + threadIdx.x;
    if (g >= (size_t)W * N) return;
    const size_t s = g / N, r = g % N;
    const int t = src[g];
#pragma unroll
    for (int q = 0; q < NN; ++q) out[(s * NN + q) * N + r] = t < 0 ? T(0) : (T)fv[(size_t)t * NN + q];
}

// Block-Jacobi sweep: delta = D^{-1}(w - S dz_in) (FIRST: D^{-1} w); dz_out = dz_in + delta;
// FINAL: zout = [z_s; z_p] + dz_out.
template <int NF, typename T, bool FIRST, bool FINAL>
__global__ __launch_bounds__(WG) void bjacobi(Sell<T> S, const T *__restrict__ win, const T *__restrict__ dinv,
                                             const T *__restrict__ dz_in, T *__restrict__ dz_out,
                                             const T *__restrict__ zs, const T *__restrict__ zp,
                                             T *__restrict__ zout) {
    constexpr int M = NF - 1;
    int i = blockIdx.x * WG + threadIdx.x;
    if (i >= S.nrows) return;
    T rv[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) rv[r] = win[(size_t)i * NF + r];
    if (!FIRST) {
        int lane = i & 63, s0, w;
        chunk_of(S, i, s0, w);
        const int *col = S.col + (size_t)s0 * 64 + lane;
        const T *val = S.val + (size_t)s0 * 64 * (NF * NF) + lane;
        for (int k = 0; k < w; ++k) {
            int c = col[(size_t)k * 64];
            T xv[NF];
#pragma unroll
            for (int e = 0; e < NF; ++e) xv[e] = dz_in[(size_t)c * NF + e];
#pragma unroll
            for (int r = 0; r < NF; ++r)
#pragma unroll
                for (int e = 0; e < NF; ++e) rv[r] -= val[((size_t)k * (NF * NF) + r * NF + e) * 64] * xv[e];
        }
    }
    const T *d = dinv + (size_t)i * NF * NF;
#pragma unroll
    for (int r = 0; r < NF; ++r) {
        T s = T(0);
#pragma unroll
        for (int e = 0; e < NF; ++e) s += d[r * NF + e] * rv[e];
        size_t o = (size_t)i * NF + r;
        T v = FIRST ? s : dz_in[o] + s;
        if (FINAL) {
            T zf = r < M ? zs[(size_t)i * M + r] : zp[i];
            zout[o] = zf + v;
        } else {
            dz_out[o] = v;
        }
    }
}

// Multicolour block Gauss-Seidel, one colour: for rows of the colour (no two adjacent),
// dz_i += D_i^{-1}(w_i - sum_j S_ij dz_j); FINAL: zout_i = [z_s; z_p]_i + dz_i.
template <int NF, typename T, bool FINAL>
__global__ __launch_bounds__(WG) void mcgs(Sell<T> S, int pos0, int pos1, const T *__restrict__ win,
                                          const T *__restrict__ dinv, T *__restrict__ dz,
                                          const T *__restrict__ zs, const T *__restrict__ zp,
                                          T *__restrict__ zout) {
    constexpr int M = NF - 1;
    int pos = pos0 + blockIdx.x * WG + threadIdx.x;
    if (pos >= pos1) return;
    int row = S.rowmap[pos];
    if (row < 0) return;
    int lane = pos & 63, s0, w;
    chunk_of(S, pos, s0, w);
    const int *col = S.col + (size_t)s0 * 64 + lane;
    const T *val = S.val + (size_t)s0 * 64 * (NF * NF) + lane;
    T rv[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) rv[r] = win[(size_t)row * NF + r];
    for (int k = 0; k < w; ++k) {
        int c = col[(size_t)k * 64];
        T xv[NF];
#pragma unroll
        for (int e = 0; e < NF; ++e) xv[e] = dz[(size_t)c * NF + e];
#pragma unroll
        for (int r = 0; r < NF; ++r)
#pragma unroll
            for (int e = 0; e < NF; ++e) rv[r] -= val[((size_t)k * (NF * NF) + r * NF + e) * 64] * xv[e];
    }
    const T *d = dinv + (size_t)row * NF * NF;
#pragma unroll
    for (int r = 0; r < NF; ++r) {
        T s = T(0);
#pragma unroll
        for (int e = 0; e < NF; ++e) s += d[r * NF + e] * rv[e];
        size_t o = (size_t)row * NF + r;
        T v = dz[o] + s;
        dz[o] = v;
        if (FINAL) {
            T zf = r < M ? zs[(size_t)row * M + r] : zp[row];
            zout[o] = zf + v;
        }
    }
}

// ------------------------------------------------------------------ vector kernels
template <typename TI, typename TO>
__global__ __launch_bounds__(WG) void convert(const TI *__restrict__ in, TO *__restrict__ out, size_t n) {
    size_t i = (size_t)blockIdx.x * WG + threadIdx.x;
    if (i < n) out[i] = (TO)in[i];
}

// x += z (z in the preconditioner's type, widened exactly)
template <typename TZ>
__global__ __launch_bounds__(WG) void add_to(double *__restrict__ x, const TZ *__restrict__ z, size_t n) {
    size_t i = (size_t)blockIdx.x * WG + threadIdx.x;
    if (i < n) x[i] += (double)z[i];
}

template <typename T>
__global__ __launch_bounds__(WG) void fill(T *__restrict__ p, T v, size_t n) {
    size_t i = (size_t)blockIdx.x * WG + threadIdx.x;
    if (i < n) p[i] = v;
}

// y = x / s[idx]  (s on the device)
__global__ __launch_bounds__(WG) void scale_div(const double *__restrict__ x, const double *__restrict__ s,
                                               int idx, double *__restrict__ y, size_t n) {
    size_t i = (size_t)blockIdx.x * WG + threadIdx.x;
    if (i < n) y[i] = x[i] / s[idx];
}

__global__ __launch_bounds__(WG) void nonfinite_count(const float *__restrict__ p, size_t n,
                                                     double *__restrict__ out) {
    __shared__ double red[4];
    double c = 0.0;
    for (size_t i = (size_t)blockIdx.x * WG + threadIdx.x; i < n; i += (size_t)gridDim.x * WG)
        if (!isfinite(p[i])) c += 1.0;
    c = block_sum(c, red);
    if (threadIdx.x == 0) out[blockIdx.x] = c;
}

// ------------------------------------------------------------------ FGMRES kernels
// partial[k * nblk + blk] = sum over this block's chunk of V_k . w (k < nv), and
// partial[nv * nblk + blk] = w . w when NORM.  The chunk of w is staged in LDS.
template <bool NORM, bool LDSW>
__global__ __launch_bounds__(WG) void mdot(const double *__restrict__ V, size_t ldv, int nv,
                                          const double *__restrict__ w, size_t n, int chunk,
                                          double *__restrict__ partial, int nblk) {
    // Eight vectors per pass over the chunk, three elements per thread per step: the 24
    // loads of a step are issued before any of them is used (a wave needs many bytes in
    // flight to stream at full bandwidth).  The |w|^2 term rides along in the first pass;
    // each wave's sums go to LDS without a barrier and the four waves are combined once
    // at the end in a fixed order.  Per thread, elements are accumulated in increasing
    // index order.
    constexpr int U = 3;
    extern __shared__ double sw[];
    __shared__ double red[4][MAXV + 1];
    size_t i0 = (size_t)blockIdx.x * chunk;
    int len = i0 < n ? (int)((n - i0) < (size_t)chunk ? (n - i0) : (size_t)chunk) : 0;
    const double *wb = w + i0;
    if (LDSW) {
        for (int t = threadIdx.x; t < len; t += WG) sw[t] = wb[t];
        __syncthreads();
    }
    const double *ws = LDSW ? sw : wb;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int npass = nv > 0 ? (nv + 7) / 8 : (NORM ? 1 : 0);
    for (int p = 0; p < npass; ++p) {
        const int k0 = 8 * p, kk = nv - k0 < 8 ? nv - k0 : 8;
        const bool wnorm = NORM && p == 0;
        // rows past nv re-read row k0 (in bounds, unused): every load is unconditional
        const double *v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = kk > 0 ? V + (size_t)(q < kk ? k0 + q : k0) * ldv + i0 : ws;
        double a[8], an = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) a[q] = 0.0;
        for (int t0 = threadIdx.x; t0 < len; t0 += U * WG) {
            double x[U][8], wt[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u * WG, tc = t < len ? t : len - 1;
                wt[u] = ws[tc];
                if (kk > 0) {
#pragma unroll
                    for (int q = 0; q < 8; ++q) x[u][q] = v[q][tc];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (t0 + u * WG < len) {
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (q < kk) a[q] += x[u][q] * wt[u];
                    if (wnorm) an += wt[u] * wt[u];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (q < kk) {
                const double r = wave_sum_dpp(a[q]);
                if (lane == 0) red[wid][k0 + q] = r;
            }
        }
        if (wnorm) {
            const double r = wave_sum_dpp(an);
            if (lane == 0) red[wid][nv] = r;
        }
    }
    __syncthreads();
    const int ntot = nv + (NORM ? 1 : 0);
    for (int k = threadIdx.x; k < ntot; k += WG)
        partial[(size_t)k * nblk + blockIdx.x] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
}

// out[k] = sum_b partial[k * nblk + b] (fixed order); if add: sum_out[k] = add[k] + out[k].
__global__ __launch_bounds__(WG) void reduce_rows(const double *__restrict__ partial, int nblk,
                                                 double *__restrict__ out, const double *__restrict__ add,
                                                 double *__restrict__ sum_out) {
    __shared__ double red[4];
    int k = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += WG) s += partial[(size_t)k * nblk + b];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        out[k] = s;
        if (add) sum_out[k] = add[k] + s;
    }
}

// w -= sum_{k<nv} V_k h_k over this block's chunk; NORM: partial[blk] = |w_new|^2 (chunk).
// V is read with non-temporal loads: as the last CGS2 pass over V this left w in the caches
// and ran 16% faster on MI355X (in the first and the fused pass the same loads did not help).
template <bool NORM>
__global__ __launch_bounds__(WG) void gemv_sub(const double *__restrict__ V, size_t ldv, int nv,
                                              const double *__restrict__ h, double *__restrict__ w,
                                              size_t n, int chunk, double *__restrict__ partial) {
    __shared__ double hs[MAXV];
    __shared__ double red[4];
    for (int t = threadIdx.x; t < nv; t += WG) hs[t] = h[t];
    __syncthreads();
    size_t i0 = (size_t)blockIdx.x * chunk;
    int len = i0 < n ? (int)((n - i0) < (size_t)chunk ? (n - i0) : (size_t)chunk) : 0;
    double acc = 0.0;
    for (int t = threadIdx.x; t < len; t += WG) {
        size_t i = i0 + t;
        double s = 0.0;
        for (int k = 0; k < nv; ++k) s += __builtin_nontemporal_load(&V[(size_t)k * ldv + i]) * hs[k];
        double wn = w[i] - s;
        w[i] = wn;
        acc += wn * wn;
    }
    if (NORM) {
        acc = block_sum(acc, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = acc;
    }
}

// The middle of CGS2 in one pass over V: w -= V h (stored), then partial[k * nblk + blk] =
// V_k . w over this block's chunk, for k < nv.  The chunk goes through LDS in tiles of
// 64 elements x nv vectors (row stride 65 doubles), so each element of V is read from
// HBM once for both products; the next tile's rows are loaded into registers (RW rows
// per wave, nv <= 4 RW) while the current tile is computed.  Loads past the chunk or past
// nv repeat the last element / row (in bounds, unused).  Dynamic LDS: nv * 65 doubles.
constexpr int SUBDOT_MAXV = 112;    // 112 x 65 doubles + static arrays < 64 KB of LDS
template <int RW>
__global__ __launch_bounds__(WG) void gemv_sub_mdot(const double *__restrict__ V, size_t ldv, int nv,
                                                   const double *__restrict__ h, double *__restrict__ w,
                                                   size_t n, int chunk, double *__restrict__ partial,
                                                   int nblk) {
    extern __shared__ double tile[];
    __shared__ double hs[SUBDOT_MAXV];
    __shared__ double part[4][64];
    __shared__ double wn[64];
    __shared__ double part2[WG];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    // V_k . w over a tile: nq threads per vector, each over 64 / nq consecutive elements
    // (eight when at most 32 vectors leave most threads idle; measured slower for more)
    const int nq = nv <= 32 ? 8 : 1, span = 64 / nq, kq = tid / nq, part_ = tid % nq;
    for (int t = tid; t < nv; t += WG) hs[t] = h[t];
    const size_t i0 = (size_t)blockIdx.x * chunk;
    const int len = i0 < n ? (int)((n - i0) < (size_t)chunk ? (n - i0) : (size_t)chunk) : 0;
    double acc = 0.0;
    double r[RW];
    auto load = [&](int e0) {
        const int ne = len - e0 < 64 ? len - e0 : 64;
        const int el = lane < ne ? lane : ne - 1;
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            const int k = wid + 4 * q < nv ? wid + 4 * q : nv - 1;
            r[q] = V[(size_t)k * ldv + i0 + e0 + el];
        }
    };
    if (len > 0) load(0);
    __syncthreads();
    for (int e0 = 0; e0 < len; e0 += 64) {
        const int ne = len - e0 < 64 ? len - e0 : 64;
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            const int k = wid + 4 * q;
            if (k < nv) tile[k * 65 + lane] = lane < ne ? r[q] : 0.0;
        }
        __syncthreads();
        if (e0 + 64 < len) load(e0 + 64);
        double s = 0.0;
        for (int k = wid; k < nv; k += 4) s += tile[k * 65 + lane] * hs[k];
        part[wid][lane] = s;
        __syncthreads();
        if (wid == 0) {
            double wv = 0.0;
            if (lane < ne) {
                const size_t i = i0 + e0 + lane;
                wv = w[i] - (((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]);
                w[i] = wv;
            }
            wn[lane] = wv;
        }
        __syncthreads();
        if (kq < nv) {
            double d = 0.0;
            const int e0p = part_ * span;
#pragma unroll 8
            for (int e = 0; e < span; ++e) d += tile[kq * 65 + e0p + e] * wn[e0p + e];
            acc += d;
        }
        __syncthreads();
    }
    // the nq partial dot products of each vector, added in order
    part2[tid] = acc;
    __syncthreads();
    if (tid < nv) {
        double d = part2[tid * nq];
        for (int q = 1; q < nq; ++q) d += part2[tid * nq + q];
        partial[(size_t)tid * nblk + blockIdx.x] = d;
    }
}

// Rotations 0..n-1 applied in order to col[0..n] (in LDS): the updated entry i + 1 is
// carried in a register from one rotation to the next, so the dependent chain is two
// multiply-adds per rotation rather than a round trip through LDS.
__device__ __forceinline__ void rotate_col(double *col, const double *c, const double *s, int n) {
    double x = col[0];
    for (int i = 0; i < n; ++i) {
        const double y = col[i + 1];
        const double t = c[i] * x + s[i] * y;
        x = -s[i] * x + c[i] * y;
        col[i] = t;
    }
    col[n] = x;
}

// Givens update of Hessenberg column j (column-major, leading dimension m+1).
// h: j+1 orthogonalisation coefficients; naz2[0] = |A z_j|^2; |w|^2 is the sum of the nblk
// chunk partials wpart, added as reduce_rows adds them (the same bits).
// scal out: [0] |g_{j+1}|, [1] h_{j+1,j}, [2] |A z_j|, [3] breakdown flag.
__global__ __launch_bounds__(WG) void givens(int j, int m, const double *__restrict__ h,
                                            const double *__restrict__ naz2, const double *__restrict__ wpart,
                                            int nblk, double *__restrict__ H, double *__restrict__ cs,
                                            double *__restrict__ sn, double *__restrict__ g,
                                            double *__restrict__ scal, double *__restrict__ hscal) {
    // the column and the previous rotations are staged in LDS by the workgroup; one thread
    // applies the rotations in order (a dependent chain), the workgroup writes back
    __shared__ double col[MAXV + 1], c[MAXV], s[MAXV];
    __shared__ double out[4], red[4];
    __shared__ double nw2[1];
    const int tid = threadIdx.x;
    {
        double a = 0.0;
        for (int b = tid; b < nblk; b += WG) a += wpart[b];
        a = block_sum(a, red);
        if (tid == 0) nw2[0] = a;
    }
    for (int i = tid; i <= j; i += WG) {
        col[i] = h[i];
        if (i < j) {
            c[i] = cs[i];
            s[i] = sn[i];
        }
    }
    __syncthreads();
    if (tid == 0) {
        const double hn = sqrt(nw2[0]);
        col[j + 1] = hn;
        rotate_col(col, c, s, j);
        const double rho = hypot(col[j], col[j + 1]);
        out[1] = hn;
        out[2] = sqrt(naz2[0]);
        if (rho == 0.0) {
            out[0] = fabs(g[j]);
            out[3] = 1.0;
        } else {
            const double cj = col[j] / rho, sj = col[j + 1] / rho;
            cs[j] = cj;
            sn[j] = sj;
            col[j] = rho;
            col[j + 1] = 0.0;
            const double gj = g[j];
            g[j + 1] = -sj * gj;
            g[j] = cj * gj;
            out[0] = fabs(-sj * gj);
            out[3] = 0.0;
        }
    }
    __syncthreads();
    double *hc = H + (size_t)j * (m + 1);
    for (int i = tid; i <= j + 1; i += WG) hc[i] = col[i];
    if (tid < 4) {
        scal[tid] = out[tid];
        if (hscal) hscal[tid] = out[tid];     // pinned host copy: no separate transfer
    }
}

// ------------------------------------------------------------------ DCGS2
// Classical Gram-Schmidt with delayed re-orthogonalisation (Bielich et al., Parallel
// Computing 112, 2022).  While iteration j runs, V_0..V_{j-1} are finished and V_j holds u,
// the vector that entered the preconditioner after one Gram-Schmidt pass (scaled to unit
// norm); w = A z_j sits in V_{j+1}.  One pass over the basis gives every product, a second
// finishes u and projects w.  Rows of the reduced products h (mdot2's partial rows):
//   h[k] = V_k . w (k <= j; h[j] = u . w),  h[j+1] = w . w,  h[j+2+k] = V_k . u (k <= j;
//   h[2j+2] = u . u).

// partial rows (nv = j + 1): k < nv: V_k . w; nv: w . w; nv + 1 + k: V_k . u, over this
// block's chunk.  Eight vectors per pass; each thread takes element pairs (16-byte loads:
// a chunk starts at an even row and the basis vectors at 256-byte boundaries), two pairs
// per step, all loads of a step issued before any is used; fixed-order combination of the
// four waves; w and u are staged in LDS.  A pair past an odd chunk end reads the element
// after it (the basis stride's padding, or unused LDS) without adding it.  Launch bounds ask
// for four waves per SIMD (at most 128 VGPRs; unbounded, the pair loads take 138).
template <bool LDSW>
__global__ __launch_bounds__(WG, 4) void mdot2(const double *__restrict__ V, size_t ldv, int nv,
                                           const double *__restrict__ w, size_t n, int chunk,
                                           double *__restrict__ partial, int nblk) {
    constexpr int U = 2;
    extern __shared__ __align__(16) double sw[];
    __shared__ double red[4][2 * MAXV + 2];
    size_t i0 = (size_t)blockIdx.x * chunk;
    int len = i0 < n ? (int)((n - i0) < (size_t)chunk ? (n - i0) : (size_t)chunk) : 0;
    const double *wb = w + i0;
    const double *ub = V + (size_t)(nv - 1) * ldv + i0;
    if (LDSW) {
        for (int t = threadIdx.x; t < len; t += WG) {
            sw[t] = wb[t];
            sw[chunk + t] = ub[t];
        }
        __syncthreads();
    }
    const double2 *ws = reinterpret_cast<const double2 *>(LDSW ? sw : wb);
    const double2 *us = reinterpret_cast<const double2 *>(LDSW ? sw + chunk : ub);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int np = (len + 1) >> 1;
    const int npass = (nv + 7) / 8;
    for (int p = 0; p < npass; ++p) {
        const int k0 = 8 * p, kk = nv - k0 < 8 ? nv - k0 : 8;
        const bool wnorm = p == 0;
        // rows past nv re-read row k0 (in bounds, unused): every load is unconditional
        const double2 *v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            v[q] = reinterpret_cast<const double2 *>(V + (size_t)(q < kk ? k0 + q : k0) * ldv + i0);
        double a[8], c[8], an = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) a[q] = c[q] = 0.0;
        for (int t0 = threadIdx.x; t0 < np; t0 += U * WG) {
            double2 x[U][8], wt[U], ut[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u * WG, tc = t < np ? t : np - 1;
                wt[u] = ws[tc];
                ut[u] = us[tc];
#pragma unroll
                for (int q = 0; q < 8; ++q) x[u][q] = v[q][tc];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u * WG;
                if (t < np) {
                    const bool hi = 2 * t + 1 < len;
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        if (q < kk) {
                            a[q] += x[u][q].x * wt[u].x;
                            c[q] += x[u][q].x * ut[u].x;
                            if (hi) {
                                a[q] += x[u][q].y * wt[u].y;
                                c[q] += x[u][q].y * ut[u].y;
                            }
                        }
                    }
                    if (wnorm) {
                        an += wt[u].x * wt[u].x;
                        if (hi) an += wt[u].y * wt[u].y;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (q < kk) {
                const double ra = wave_sum_dpp(a[q]);
                const double rc = wave_sum_dpp(c[q]);
                if (lane == 0) {
                    red[wid][k0 + q] = ra;
                    red[wid][nv + 1 + k0 + q] = rc;
                }
            }
        }
        if (wnorm) {
            const double r = wave_sum_dpp(an);
            if (lane == 0) red[wid][nv] = r;
        }
    }
    __syncthreads();
    const int ntot = 2 * nv + 1;
    for (int k = threadIdx.x; k < ntot; k += WG)
        partial[(size_t)k * nblk + blockIdx.x] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
}

// alpha = sqrt(u.u - s.s) and t = (u.w - s.p) / alpha from the reduced rows h (j finished
// vectors); one thread, increasing k: every caller gets the same bits.
__device__ __forceinline__ void dcgs2_coef(const double *__restrict__ h, int j, double &alpha, double &t) {
    double ss = 0.0, sp = 0.0;
    for (int k = 0; k < j; ++k) {
        const double sk = h[j + 2 + k];
        ss += sk * sk;
        sp += sk * h[k];
    }
    const double a2 = h[2 * j + 2] - ss;
    alpha = a2 > 0.0 ? sqrt(a2) : 0.0;
    t = (h[j] - sp) / alpha;
}

// The second pass: u <- (u - V_j s) / alpha (the finished v_j), r = w - V_j p - t v_j, and w
// <- r / |w| (the next u: scaled by |A z_j| = sqrt(h[j+1]), known before this pass, so that
// it needs no normalising pass and its scale does not compound); partial[blk] = |r|^2 over
// this block's chunk.  Block 0 stores alpha, t in coef[0], coef[1].  V is read with
// non-temporal loads, as in gemv_sub (the last pass over it this iteration).
typedef double vd2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(WG) void gemv_sub2(const double *__restrict__ V, size_t ldv, int j,
                                               const double *__restrict__ h, double *__restrict__ u,
                                               double *__restrict__ w, size_t n, int chunk,
                                               double *__restrict__ partial, double *__restrict__ coef) {
    __shared__ double hs[MAXV], hp[MAXV];
    __shared__ double red[4];
    __shared__ double at[2];
    for (int k = threadIdx.x; k < j; k += WG) {
        hs[k] = h[j + 2 + k];
        hp[k] = h[k];
    }
    if (threadIdx.x == 0) {
        double alpha, t;
        dcgs2_coef(h, j, alpha, t);
        at[0] = alpha;
        at[1] = t;
        if (blockIdx.x == 0) {
            coef[0] = alpha;
            coef[1] = t;
        }
    }
    __syncthreads();
    const double alpha = at[0], t = at[1];
    const double naz = sqrt(h[j + 1]);
    size_t i0 = (size_t)blockIdx.x * chunk;
    int len = i0 < n ? (int)((n - i0) < (size_t)chunk ? (n - i0) : (size_t)chunk) : 0;
    // element pairs per thread (16-byte loads: a chunk starts at an even row and the basis
    // vectors at 256-byte boundaries); each element's sums run over k in increasing order.
    // A pair past an odd chunk end reads the element after it (the basis stride's padding)
    // and neither stores nor adds it.
    double acc = 0.0;
    const int np = (len + 1) >> 1;
    for (int e = threadIdx.x; e < np; e += WG) {
        const size_t i = i0 + 2 * (size_t)e;
        const bool hi = 2 * e + 1 < len;
        vd2 su = {0.0, 0.0}, sw = {0.0, 0.0};
        for (int k = 0; k < j; ++k) {
            const vd2 v = __builtin_nontemporal_load(reinterpret_cast<const vd2 *>(&V[(size_t)k * ldv + i]));
            su += v * hs[k];
            sw += v * hp[k];
        }
        const vd2 uu = *reinterpret_cast<const vd2 *>(&u[i]), ww = *reinterpret_cast<const vd2 *>(&w[i]);
        const double vn0 = (uu.x - su.x) / alpha, vn1 = (uu.y - su.y) / alpha;
        const double rn0 = (ww.x - sw.x) - t * vn0, rn1 = (ww.y - sw.y) - t * vn1;
        const double wn0 = naz > 0.0 ? rn0 / naz : 0.0, wn1 = naz > 0.0 ? rn1 / naz : 0.0;
        if (hi) {
            *reinterpret_cast<vd2 *>(&u[i]) = vd2{vn0, vn1};
            *reinterpret_cast<vd2 *>(&w[i]) = vd2{wn0, wn1};
        } else {
            u[i] = vn0;
            w[i] = wn0;
        }
        acc += rn0 * rn0;
        if (hi) acc += rn1 * rn1;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// Hessenberg columns under DCGS2 (column-major H, leading dimension m+1).  Column j - 1 is
// finished now that u_j's products are known: its first-pass entries raw[0..j-1] gain
// c s and h_{j,j-1} = c alpha, c = |A z_{j-1}| (the scale of u_j, in coef[2]); its rotation is
// kept.  Column j's first-pass entries (p, t) replace raw, |A z_j| goes to coef[2], and the
// Givens estimate with the unfinished column j (subdiagonal |r_j|, from the chunk partials
// wpart; rotation not kept) decides whether to stop.  scal out: [0] estimate, [1] |r_j|,
// [2] |A z_j|, [3] breakdown flag; hscal: pinned host copy.
__global__ __launch_bounds__(WG) void givens2(int j, int m, const double *__restrict__ h,
                                             double *__restrict__ coef, double *__restrict__ raw,
                                             const double *__restrict__ wpart, int nblk,
                                             double *__restrict__ H, double *__restrict__ cs,
                                             double *__restrict__ sn, double *__restrict__ g,
                                             double *__restrict__ scal, double *__restrict__ hscal) {
    __shared__ double col[MAXV + 1], c[MAXV], s[MAXV], rw[MAXV], hs[MAXV], hp[MAXV], fin[MAXV + 1];
    __shared__ double out[4], red[4];
    __shared__ double nw2[1];
    const int tid = threadIdx.x;
    // every operand is loaded before the first reduction, so the loads' latencies overlap:
    // one column entry, rotation and product per thread (j < WG), the scalars by thread 0
    double l_rw = 0.0, l_c = 0.0, l_s = 0.0, l_hs = 0.0, l_hp = 0.0;
    if (tid < j) {
        l_rw = raw[tid];
        l_c = cs[tid];
        l_s = sn[tid];
        l_hs = h[j + 2 + tid];
        l_hp = h[tid];
    }
    double l_alpha = 0.0, l_t = 0.0, l_bp = 0.0, l_h1 = 0.0, l_g0 = 0.0, l_gj = 0.0;
    if (tid == 0) {
        l_alpha = coef[0];
        l_t = coef[1];
        l_bp = coef[2];
        l_h1 = h[j + 1];
        l_gj = g[j];
        if (j > 0) l_g0 = g[j - 1];
    }
    {
        double a = 0.0;
        for (int b = tid; b < nblk; b += WG) a += wpart[b];
        a = block_sum(a, red);
        if (tid == 0) nw2[0] = a;
    }
    // every operand staged in LDS by the workgroup; one thread runs the dependent chains
    if (tid < j) {
        rw[tid] = l_rw;
        c[tid] = l_c;
        s[tid] = l_s;
        hs[tid] = l_hs;
        hp[tid] = l_hp;
    }
    for (int i = tid + WG; i < j; i += WG) {
        rw[i] = raw[i];
        c[i] = cs[i];
        s[i] = sn[i];
        hs[i] = h[j + 2 + i];
        hp[i] = h[i];
    }
    __syncthreads();
    if (tid == 0) {
        const double alpha = l_alpha, t = l_t, naz = sqrt(l_h1);
        double gcur = l_gj;                      // g[j] as this kernel leaves it
        if (j > 0) {
            const double bp = l_bp;
            for (int i = 0; i < j; ++i) fin[i] = rw[i] + bp * hs[i];
            fin[j] = bp * alpha;
            rotate_col(fin, c, s, j - 1);
            const double rho = hypot(fin[j - 1], fin[j]);
            const double cj = fin[j - 1] / rho, sj = fin[j] / rho;
            c[j - 1] = cj;
            s[j - 1] = sj;
            fin[j - 1] = rho;
            fin[j] = 0.0;
            const double gj = l_g0;
            gcur = -sj * gj;
            g[j] = gcur;
            g[j - 1] = cj * gj;
        }
        // column j as the first pass left it, with its estimate (rotation not kept)
        const double hn = sqrt(nw2[0]);
        coef[2] = naz;
        for (int i = 0; i < j; ++i) col[i] = hp[i];
        col[j] = t;
        col[j + 1] = hn;
        rotate_col(col, c, s, j);
        const double rho = hypot(col[j], col[j + 1]);
        out[1] = hn;
        out[2] = naz;
        if (rho == 0.0) {
            out[0] = fabs(gcur);
            out[3] = 1.0;
        } else {
            out[0] = fabs(col[j + 1] / rho * gcur);
            out[3] = 0.0;
        }
        col[j] = t;                 // raw[j]
    }
    __syncthreads();
    if (j > 0) {
        double *hc = H + (size_t)(j - 1) * (m + 1);
        for (int i = tid; i <= j; i += WG) hc[i] = fin[i];
        if (tid == 0) {
            cs[j - 1] = c[j - 1];
            sn[j - 1] = s[j - 1];
        }
    }
    for (int i = tid; i < j; i += WG) raw[i] = hp[i];
    if (tid == 0) raw[j] = col[j];
    if (tid < 4) {
        scal[tid] = out[tid];
        if (hscal) hscal[tid] = out[tid];
    }
}

// End of a DCGS2 cycle: column j is finished with u_{j+1} = r_j / c, c = |A z_j| (in
// coef[2]), and its reduced products h2[k] = V_k . u_{j+1} (k <= j), h2[j+1] = |u_{j+1}|^2:
// the first-pass entries raw[0..j] gain c s', h_{j+1,j} = c alpha' with alpha' =
// sqrt(|u|^2 - s'.s'), and its rotation is kept (g updated).  c = 0: nothing to add.
__global__ void givens_finish(int j, int m, const double *__restrict__ h2, const double *__restrict__ coef,
                              const double *__restrict__ raw, double *__restrict__ H, double *__restrict__ cs,
                              double *__restrict__ sn, double *__restrict__ g) {
    __shared__ double col[MAXV + 1];
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double bt = coef[2];
    for (int i = 0; i <= j; ++i) col[i] = raw[i];
    col[j + 1] = 0.0;
    if (bt != 0.0) {
        double ss = 0.0;
        for (int i = 0; i <= j; ++i) {
            ss += h2[i] * h2[i];
            col[i] += bt * h2[i];
        }
        const double a2 = h2[j + 1] - ss;
        col[j + 1] = a2 > 0.0 ? bt * sqrt(a2) : 0.0;
    }
    rotate_col(col, cs, sn, j);
    const double rho = hypot(col[j], col[j + 1]);
    const double cj = col[j] / rho, sj = col[j + 1] / rho;
    cs[j] = cj;
    sn[j] = sj;
    col[j] = rho;
    col[j + 1] = 0.0;
    double *hc = H + (size_t)j * (m + 1);
    for (int i = 0; i <= j + 1; ++i) hc[i] = col[i];
    const double gj = g[j];
    g[j + 1] = -sj * gj;
    g[j] = cj * gj;
}

// Start of a cycle: g = beta e_1 with beta = sqrt(nr2[0]).
__global__ void cycle_start(int m, const double *__restrict__ nr2, double *__restrict__ g,
                            double *__restrict__ scal) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double beta = sqrt(nr2[0]);
    for (int i = 0; i <= m; ++i) g[i] = 0.0;
    g[0] = beta;
    scal[4] = beta;
}

// y = H_k^{-1} g_k (upper triangular back substitution).
__global__ void backsolve(int k, int m, const double *__restrict__ H, const double *__restrict__ g,
                          double *__restrict__ y) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int c = i + 1; c < k; ++c) s -= H[(size_t)c * (m + 1) + i] * y[c];
        y[i] = s / H[(size_t)i * (m + 1) + i];
    }
}

// x += sum_{t<k} Z_t y_t.
template <typename TZ>
__global__ __launch_bounds__(WG) void xupdate(double *__restrict__ x, const TZ *__restrict__ Z, size_t ldz,
                                             int k, const double *__restrict__ y, size_t n) {
    __shared__ double ys[MAXV];
    for (int t = threadIdx.x; t < k; t += WG) ys[t] = y[t];
    __syncthreads();
    size_t i = (size_t)blockIdx.x * WG + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int t = 0; t < k; ++t) s += (double)Z[(size_t)t * ldz + i] * ys[t];
    x[i] += s;
}

}  // namespace k
}  // namespace ps
