// Galerkin coarse operators of the pressure AMG on the device (Sec. 5.3, M_pp = amg(S_pp);
// the coarse operator of each level is R (A P) with R = P^T).
//
// C = A B is formed by expansion, stable sort and ordered segmented sums: every product
// a_il b_lk is written in row-major order of A (increasing l inside a row, then the
// entries of row l of B), a stable radix sort on (i, k) keeps that order inside each
// key, and each key's products are added one after another from 0.0.  That is exactly
// the sequence of roundings of a row-by-row Gustavson product that accumulates in
// increasing inner index, so the coarse operators equal the host build bit for bit.
// Entries that sum to exactly zero are dropped; columns come out sorted.
#include <cstring>
#include <mutex>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "device.h"

namespace ps {
namespace {

constexpr int TB = 256;

inline unsigned blocks(long long n) { return (unsigned)((n + TB - 1) / TB); }

__global__ void fill_int(int *p, int v, long long n) {
    long long i = (long long)blockIdx.x * TB + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void row_ids(const int *__restrict__ rp, int n, int *__restrict__ rid) {
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    for (int t = rp[i]; t < rp[i + 1]; ++t) rid[t] = i;
}

__global__ void product_counts(const int *__restrict__ aci, int nnz, const int *__restrict__ brp,
                               long long *__restrict__ cnt) {
    int t = blockIdx.x * TB + threadIdx.x;
    if (t < nnz) cnt[t] = brp[aci[t] + 1] - brp[aci[t]];
    if (t == nnz) cnt[t] = 0;
}

__global__ void expand(const int *__restrict__ rid, const int *__restrict__ aci, const double *__restrict__ av,
                       int nnz, const int *__restrict__ brp, const int *__restrict__ bci,
                       const double *__restrict__ bv, const long long *__restrict__ off, int cbits,
                       unsigned long long *__restrict__ keys, double *__restrict__ vals) {
    int t = blockIdx.x * TB + threadIdx.x;
    if (t >= nnz) return;
    const unsigned long long row = (unsigned long long)rid[t] << cbits;
    const int l = aci[t];
    const double a = av[t];
    long long o = off[t];
    for (int u = brp[l]; u < brp[l + 1]; ++u, ++o) {
        keys[o] = row | (unsigned long long)bci[u];
        vals[o] = __dmul_rn(a, bv[u]);
    }
}

__global__ void heads(const unsigned long long *__restrict__ k, long long n, long long *__restrict__ h) {
    long long p = (long long)blockIdx.x * TB + threadIdx.x;
    if (p < n) h[p] = (p == 0 || k[p] != k[p - 1]) ? 1 : 0;
}

// sid: inclusive scan of the head flags (segment number + 1)
__global__ void segment_starts(const long long *__restrict__ h, const long long *__restrict__ sid, long long n,
                               long long *__restrict__ start) {
    long long p = (long long)blockIdx.x * TB + threadIdx.x;
    if (p < n && h[p]) start[sid[p] - 1] = p;
    if (p == 0) start[sid[n - 1]] = n;
}

// (S, the number of segments, is read from the device; nz is defined on 0..P, zero from S
// on, so that its scan over P + 1 entries ends with the number of nonzero sums)
__global__ void segment_sums(const long long *__restrict__ start, const long long *__restrict__ Sp, long long P,
                             const double *__restrict__ vals, double *__restrict__ sum, long long *__restrict__ nz) {
    long long s = (long long)blockIdx.x * TB + threadIdx.x;
    const long long S = *Sp;
    if (s > P) return;
    if (s >= S) {
        nz[s] = 0;
        return;
    }
    double acc = 0.0;
    for (long long p = start[s]; p < start[s + 1]; ++p) acc = __dadd_rn(acc, vals[p]);
    sum[s] = acc;
    nz[s] = acc != 0.0 ? 1 : 0;
}

__global__ void scatter(const long long *__restrict__ start, const long long *__restrict__ Sp,
                        const unsigned long long *__restrict__ keys, const double *__restrict__ sum,
                        const long long *__restrict__ nz, const long long *__restrict__ pos, int cbits,
                        int *__restrict__ ci, double *__restrict__ v, int *__restrict__ rowcnt) {
    long long s = (long long)blockIdx.x * TB + threadIdx.x;
    if (s >= *Sp || !nz[s]) return;
    const unsigned long long key = keys[start[s]];
    const long long q = pos[s];
    ci[q] = (int)(key & ((1ull << cbits) - 1));
    v[q] = sum[s];
    atomicAdd(&rowcnt[key >> cbits], 1);
}

int bits_for(long long n) {           // bits to hold 0 .. n-1 (at least 1)
    int b = 1;
    while ((1ll << b) < n) ++b;
    return b;
}

template <typename T>
void exclusive_scan(Arena &tmp, const T *in, T *out, size_t n, hipStream_t st) {
    size_t bytes = 0;
    PS_HIP(rocprim::exclusive_scan(nullptr, bytes, in, out, T(0), n, rocprim::plus<T>(), st));
    void *w = tmp.alloc<char>(bytes);
    PS_HIP(rocprim::exclusive_scan(w, bytes, in, out, T(0), n, rocprim::plus<T>(), st));
}

int g_round_trips = 0;              // host-device round trips of the current level (tracing)

// A pinned word per thread for the size and count read-backs of the build (a copy into
// pageable memory would be staged through a bounce buffer), kept until the process ends.
void *pinned_word() {
    static thread_local void *p = nullptr;
    if (!p) PS_HIP(hipHostMalloc(&p, 64, hipHostMallocDefault));
    return p;
}

template <typename T>
T read_back(const T *d, hipStream_t st) {
    ++g_round_trips;
    void *pin = pinned_word();
    PS_HIP(hipMemcpyAsync(pin, d, sizeof(T), hipMemcpyDeviceToHost, st));
    PS_HIP(hipStreamSynchronize(st));
    T h;
    std::memcpy(&h, pin, sizeof(T));
    return h;
}

// ---------------------------------------------------------------- coarsening on the device
// The steps of coarsen_level (host) with the same definitions and, where floating point
// is involved, the same operations in the same order, so that C/F splittings and
// interpolation weights equal the host's bit for bit.

__device__ __forceinline__ double unit_hash_dev(unsigned long long i) {
    // SplitMix64 (Steele, Lea, Flood 2014) of the row index, top 53 bits as a double in [0, 1)
    unsigned long long z = i + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * 0x1.0p-53;
}

// strength: j in S_i iff j != i and -a_ij >= theta * max_{k != i}(-a_ik) > 0; per-row
// counts of S_i and of S^T (how many rows depend on j)
__global__ void strength_k(const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ v,
                           int n, double theta, signed char *__restrict__ smask, int *__restrict__ scount,
                           int *__restrict__ lam) {
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    double m = -INFINITY;
    for (int t = rp[i]; t < rp[i + 1]; ++t) {
        if (ci[t] == i) continue;
        const double x = -v[t];
        m = m < x ? x : m;
    }
    int c = 0;
    if (m > 0.0) {
        const double thr = __dmul_rn(theta, m);
        for (int t = rp[i]; t < rp[i + 1]; ++t) {
            const bool s = ci[t] != i && -v[t] >= thr;
            smask[t] = s;
            if (s) {
                ++c;
                atomicAdd(&lam[ci[t]], 1);
            }
        }
    } else {
        for (int t = rp[i]; t < rp[i + 1]; ++t) smask[t] = 0;
    }
    scount[i] = c;
}

__global__ void fill_s_k(const int *__restrict__ rp, const int *__restrict__ ci, const signed char *__restrict__ smask,
                         int n, const int *__restrict__ srp, int *__restrict__ sci) {
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    int k = srp[i];
    for (int t = rp[i]; t < rp[i + 1]; ++t)
        if (smask[t]) sci[k++] = ci[t];
}

// S^T rows (order inside a row is irrelevant: PMIS only asks whether some neighbour wins)
__global__ void fill_st_k(const int *__restrict__ srp, const int *__restrict__ sci, int n, int *__restrict__ cur,
                          int *__restrict__ tci) {
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    for (int k = srp[i]; k < srp[i + 1]; ++k) tci[atomicAdd(&cur[sci[k]], 1)] = i;
}

// weights w_i = |S^T_i| + u_i; points nobody depends on start as F
__global__ void pmis_init_k(const int *__restrict__ trp, int n, double *__restrict__ w, signed char *__restrict__ st,
                            int *__restrict__ undecided) {
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    const int lam = trp[i + 1] - trp[i];
    w[i] = (double)lam + unit_hash_dev((unsigned long long)i);
    st[i] = lam == 0 ? -1 : 0;
    if (lam != 0) atomicAdd(undecided, 1);
}

__device__ __forceinline__ bool beats(const double *w, int j, int i) { return w[j] > w[i] || (w[j] == w[i] && j > i); }

// one PMIS round, part 1: an undecided point becomes C if no undecided neighbour in
// S_i u S^T_i beats it (reads the states at the start of the round only)
__global__ void pmis_select_k(const signed char *__restrict__ st, const double *__restrict__ w,
                              const int *__restrict__ srp, const int *__restrict__ sci, const int *__restrict__ trp,
                              const int *__restrict__ tci, int n, signed char *__restrict__ newc) {
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    if (st[i] != 0) {
        newc[i] = 0;
        return;
    }
    bool beaten = false;
    for (int k = srp[i]; k < srp[i + 1] && !beaten; ++k) {
        const int j = sci[k];
        if (st[j] == 0 && beats(w, j, i)) beaten = true;
    }
    for (int k = trp[i]; k < trp[i + 1] && !beaten; ++k) {
        const int j = tci[k];
        if (st[j] == 0 && beats(w, j, i)) beaten = true;
    }
    newc[i] = !beaten;
}

// part 2: new C points are set; an undecided point strongly depending on one becomes F
__global__ void pmis_mark_k(signed char *__restrict__ st, const signed char *__restrict__ newc,
                            const int *__restrict__ srp, const int *__restrict__ sci, int n,
                            int *__restrict__ undecided) {
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    if (newc[i]) {
        st[i] = 1;
        return;
    }
    if (st[i] != 0) return;
    for (int k = srp[i]; k < srp[i + 1]; ++k)
        if (newc[sci[k]]) {
            st[i] = -1;
            return;
        }
    atomicAdd(undecided, 1);
}

// C-promotion, equal to the sequential rule "in increasing i, an F point with S_i
// non-empty and no C point in S_i becomes C": candidates are the F points whose S_i has
// no PMIS C point; a candidate is promoted iff no candidate j < i in S_i was promoted,
// decided in rounds once every candidate j < i in S_i is decided (cs: 0 not a candidate
// / decided F, 1 undecided, 2 promoted)
__global__ void promo_init_k(const signed char *__restrict__ st, const int *__restrict__ srp,
                             const int *__restrict__ sci, int n, signed char *__restrict__ cs,
                             int *__restrict__ count) {
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    signed char c = 0;
    if (st[i] == -1 && srp[i + 1] > srp[i]) {
        c = 1;
        for (int k = srp[i]; k < srp[i + 1]; ++k)
            if (st[sci[k]] == 1) {
                c = 0;
                break;
            }
    }
    cs[i] = c;
    if (c) atomicAdd(count, 1);
}

__global__ void promo_round_k(signed char *cs, const int *__restrict__ srp, const int *__restrict__ sci, int n,
                              int *__restrict__ undecided) {
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    if (__hip_atomic_load(&cs[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 1) return;
    bool wait = false;
    for (int k = srp[i]; k < srp[i + 1]; ++k) {
        const int j = sci[k];
        if (j >= i) continue;
        const signed char c = __hip_atomic_load(&cs[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (c == 2) {                          // an earlier promoted point: stays F
            __hip_atomic_store(&cs[i], (signed char)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        if (c == 1) wait = true;
    }
    if (wait) {
        atomicAdd(undecided, 1);
        return;
    }
    __hip_atomic_store(&cs[i], (signed char)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void promo_apply_k(signed char *__restrict__ st, const signed char *__restrict__ cs, int n,
                              int *__restrict__ cflag) {
    int i = blockIdx.x * TB + threadIdx.x;
    if (i > n) return;
    if (i == n) {
        cflag[n] = 0;
        return;
    }
    if (cs[i] == 2) st[i] = 1;
    cflag[i] = st[i] == 1;
}

// direct interpolation (Stueben): C rows identity; F row i:
// P_ij = -(alpha_i a_ij) / atil_ii for j in S_i n C, alpha_i = sum_{a_ij<0} a_ij / sum_{j in S_i n C} a_ij,
// atil_ii = a_ii + sum_{j != i, a_ij > 0} a_ij, all sums in increasing column order from 0
__global__ void interp_count_k(const int *__restrict__ rp, const int *__restrict__ ci,
                               const signed char *__restrict__ smask, const signed char *__restrict__ st, int n,
                               int *__restrict__ plen) {
    int i = blockIdx.x * TB + threadIdx.x;
    if (i > n) return;
    if (i == n) {
        plen[n] = 0;
        return;
    }
    if (st[i] == 1) {
        plen[i] = 1;
        return;
    }
    int c = 0;
    for (int t = rp[i]; t < rp[i + 1]; ++t) c += ci[t] != i && smask[t] && st[ci[t]] == 1;
    plen[i] = c;
}

__global__ void interp_fill_k(const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ v,
                              const signed char *__restrict__ smask, const signed char *__restrict__ st,
                              const int *__restrict__ cidx, int n, const int *__restrict__ prp,
                              int *__restrict__ pci, double *__restrict__ pv) {
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    int o = prp[i];
    if (st[i] == 1) {
        pci[o] = cidx[i];
        pv[o] = 1.0;
        return;
    }
    double diag = 0.0, pos = 0.0, negs = 0.0, den = 0.0;
    for (int t = rp[i]; t < rp[i + 1]; ++t) {
        const int j = ci[t];
        const double a = v[t];
        if (j == i) {
            diag = a;
            continue;
        }
        if (a > 0.0) pos = __dadd_rn(pos, a);
        if (a < 0.0) negs = __dadd_rn(negs, a);
        if (smask[t] && st[j] == 1) den = __dadd_rn(den, a);
    }
    const double atil = __dadd_rn(diag, pos);
    const double alpha = den != 0.0 ? __ddiv_rn(negs, den) : 0.0;
    for (int t = rp[i]; t < rp[i + 1]; ++t) {
        const int j = ci[t];
        if (j != i && smask[t] && st[j] == 1) {
            pci[o] = cidx[j];
            pv[o] = __ddiv_rn(-__dmul_rn(alpha, v[t]), atil);
            ++o;
        }
    }
}

// R = P^T: column counts, unordered fill, then each row sorted by fine index
__global__ void col_count_k(const int *__restrict__ ci, int nnz, int *__restrict__ cnt) {
    int t = blockIdx.x * TB + threadIdx.x;
    if (t < nnz) atomicAdd(&cnt[ci[t]], 1);
}

__global__ void transpose_fill_k(const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ v,
                                 int n, int *__restrict__ cur, int *__restrict__ tci, double *__restrict__ tv) {
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    for (int t = rp[i]; t < rp[i + 1]; ++t) {
        const int k = atomicAdd(&cur[ci[t]], 1);
        tci[k] = i;
        tv[k] = v[t];
    }
}

// Each row's entries in increasing column order (stable), one wavefront per row: a row of
// at most 64 entries is held one entry per lane and each lane's rank is counted with
// shuffles; a longer row is insertion-sorted by its first lane.
__global__ void sort_rows_k(const int *__restrict__ rp, int n, int *__restrict__ ci, double *__restrict__ v) {
    const int r = (int)(((long long)blockIdx.x * TB + threadIdx.x) >> 6), lane = threadIdx.x & 63;
    if (r >= n) return;                      // uniform over the wavefront
    const int r0 = rp[r], len = rp[r + 1] - r0;
    if (len <= 64) {
        const int c = lane < len ? ci[r0 + lane] : 0x7fffffff;
        const double x = lane < len ? v[r0 + lane] : 0.0;
        int rank = 0;
        for (int k = 0; k < len; ++k) {
            const int ck = __shfl(c, k, 64);
            rank += ck < c || (ck == c && k < lane);
        }
        if (lane < len) {
            ci[r0 + rank] = c;
            v[r0 + rank] = x;
        }
        return;
    }
    if (lane != 0) return;
    for (int a = r0 + 1; a < r0 + len; ++a) {
        const int c = ci[a];
        const double x = v[a];
        int b = a - 1;
        while (b >= r0 && ci[b] > c) {
            ci[b + 1] = ci[b];
            v[b + 1] = v[b];
            --b;
        }
        ci[b + 1] = c;
        v[b + 1] = x;
    }
}

// l1-Jacobi: dinv_i = 1 / (a_ii + sum_{j != i} |a_ij|), the sum in column order from 0
__global__ void l1_inv_k(const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ v, int n,
                         double *__restrict__ dinv, int *__restrict__ zero_diag) {
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    double diag = 0.0, s = 0.0;
    for (int t = rp[i]; t < rp[i + 1]; ++t) {
        if (ci[t] == i) {
            diag = v[t];
            continue;
        }
        s = __dadd_rn(s, fabs(v[t]));
    }
    if (diag == 0.0) atomicAdd(zero_diag, 1);
    dinv[i] = __ddiv_rn(1.0, __dadd_rn(diag, s));
}


// ---------------------------------------------------------------- coarsest level
// Dense inverse of the coarsest operator on the device, operation for operation the host's
// invert_dense (LU with partial pivoting, ties to the lowest row, rows swapped whole; then
// the identity's columns solved forward and backward; products and differences rounded
// separately, as the host compiles them), so that the inverse is bitwise the host's.  One
// workgroup of DI_WG threads; n <= DI_WG.  With LDS_A the factor and the columns being
// solved live in LDS (2 n^2 doubles), else in `ga` and inv; inv (row-major) receives the
// inverse.  flag[0] = 1: singular or not finite, as on the host.
constexpr int DI_WG = 1024;

// The best (largest value, then lowest index) of a wavefront's (val, idx) pairs, in every
// lane: DPP moves within rows of 16 lanes (pair, quad, half-row, row), then the four rows'
// bests read from lanes 0, 16, 32, 48.  The rule is a total order on distinct indices, so
// the order of the steps cannot change the result.  Needs every lane active.
__device__ __forceinline__ bool di_better(double v1, int i1, double v0, int i0) {
    return v1 > v0 || (v1 == v0 && i1 < i0);
}

template <int CTRL>
__device__ __forceinline__ void di_step(double &val, int &idx) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, val);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    const double ov = __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
    const int oi = __builtin_amdgcn_mov_dpp(idx, CTRL, 0xF, 0xF, false);
    if (di_better(ov, oi, val, idx)) {
        val = ov;
        idx = oi;
    }
}

__device__ __forceinline__ void di_wave_best(double &val, int &idx) {
    di_step<0xB1>(val, idx);     // lane ^ 1
    di_step<0x4E>(val, idx);     // lane ^ 2
    di_step<0x141>(val, idx);    // 7 - i within eight
    di_step<0x140>(val, idx);    // 15 - i within sixteen
    const unsigned long long b = __builtin_bit_cast(unsigned long long, val);
    double bv = val;
    int bi = idx;
    auto lane_of = [&](int l, double &v, int &i) {
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
        v = __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
        i = __builtin_amdgcn_readlane(idx, l);
    };
    lane_of(0, bv, bi);
    for (int l = 16; l < 64; l += 16) {
        double v;
        int i;
        lane_of(l, v, i);
        if (di_better(v, i, bv, bi)) {
            bv = v;
            bi = i;
        }
    }
    val = bv;
    idx = bi;
}

template <bool LDS_A>
__global__ __launch_bounds__(DI_WG) void dense_inverse_k(const int *__restrict__ rp, const int *__restrict__ ci,
                                                        const double *__restrict__ v, int n, double *ga,
                                                        double *__restrict__ inv, int *__restrict__ piv,
                                                        int *__restrict__ flag) {
    extern __shared__ double lds_a[];
    double *a = LDS_A ? lds_a : ga;
    double *X = LDS_A ? lds_a + (size_t)n * n : inv;
    __shared__ double rv[DI_WG / 64];
    __shared__ int ri[DI_WG / 64];
    __shared__ int bad, pc;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const size_t nn = (size_t)n * n;
    for (size_t e = tid; e < nn; e += DI_WG) a[e] = 0.0;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int i = tid; i < n; i += DI_WG)
        for (int t = rp[i]; t < rp[i + 1]; ++t) a[(size_t)i * n + ci[t]] = v[t];
    __syncthreads();
    for (int c = 0; c < n; ++c) {
        // pivot: the first row r >= c with the largest |a_rc| (NaN entries below the
        // diagonal never win; a NaN on the diagonal makes the matrix singular); only the
        // wavefronts holding rows c..n-1 search
        const int r = c + tid, nwv = (n - c + 63) / 64;
        if (wid < nwv) {
            double val = -1.0;
            if (r < n) {
                const double x = fabs(a[(size_t)r * n + c]);
                val = (r == c || x == x) ? x : -1.0;
            }
            int idx = r < n ? r : n;
            di_wave_best(val, idx);
            if (lane == 0) {
                rv[wid] = val;
                ri[wid] = idx;
            }
        }
        __syncthreads();
        if (tid == 0) {
            double best = rv[0];
            int p = ri[0];
            for (int w = 1; w < nwv; ++w)
                if (rv[w] > best || (rv[w] == best && ri[w] < p)) {
                    best = rv[w];
                    p = ri[w];
                }
            const double dgl = fabs(a[(size_t)c * n + c]);
            if (dgl != dgl) best = dgl;
            if (best == 0.0 || !isfinite(best)) bad = 1;
            pc = p;
            piv[c] = p;
        }
        __syncthreads();
        if (bad) break;
        const int p = pc;
        if (p != c)
            for (int j = tid; j < n; j += DI_WG) {
                const double t = a[(size_t)c * n + j];
                a[(size_t)c * n + j] = a[(size_t)p * n + j];
                a[(size_t)p * n + j] = t;
            }
        __syncthreads();
        const double d = a[(size_t)c * n + c];
        for (int rr = c + 1 + tid; rr < n; rr += DI_WG) a[(size_t)rr * n + c] = __ddiv_rn(a[(size_t)rr * n + c], d);
        __syncthreads();
        // trailing update on a 32 x 32 thread layout (rows tid / 32 + 32 k, columns tid % 32
        // + 32 l): no index division; each element gets the one update of this step
        for (int rr = c + 1 + (tid >> 5); rr < n; rr += DI_WG / 32) {
            const double f = a[(size_t)rr * n + c];
            if (f != 0.0)
                for (int j = c + 1 + (tid & 31); j < n; j += 32)
                    a[(size_t)rr * n + j] = __dsub_rn(a[(size_t)rr * n + j], __dmul_rn(f, a[(size_t)c * n + j]));
        }
        __syncthreads();
    }
    if (bad) {
        if (tid == 0) flag[0] = 1;
        return;
    }
    // column k of the inverse: P e_k, then L y = P e_k, then U x = y (thread k)
    // the sums in the host's order (increasing c), their operands loaded eight at a time
    const int k = tid;
    if (k < n) {
        for (int r = 0; r < n; ++r) X[(size_t)r * n + k] = r == k ? 1.0 : 0.0;
        for (int c = 0; c < n; ++c) {
            const int p = piv[c];
            const double t = X[(size_t)c * n + k];
            X[(size_t)c * n + k] = X[(size_t)p * n + k];
            X[(size_t)p * n + k] = t;
        }
        auto dot_sub = [&](double s, const double *ar, int c0, int c1) {
            int c = c0;
            for (; c + 8 <= c1; c += 8) {
                double av[8], xv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    av[u] = ar[c + u];
                    xv[u] = X[(size_t)(c + u) * n + k];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) s = __dsub_rn(s, __dmul_rn(av[u], xv[u]));
            }
            for (; c < c1; ++c) s = __dsub_rn(s, __dmul_rn(ar[c], X[(size_t)c * n + k]));
            return s;
        };
        for (int r = 1; r < n; ++r)                                  // L y = P e_k
            X[(size_t)r * n + k] = dot_sub(X[(size_t)r * n + k], a + (size_t)r * n, 0, r);
        bool fin = true;
        for (int r = n - 1; r >= 0; --r) {                           // U x = y
            const double sr = dot_sub(X[(size_t)r * n + k], a + (size_t)r * n, r + 1, n);
            const double x = __ddiv_rn(sr, a[(size_t)r * n + r]);
            X[(size_t)r * n + k] = x;
            fin = fin && isfinite(x);
        }
        if (LDS_A)
            for (int r = 0; r < n; ++r) inv[(size_t)r * n + k] = X[(size_t)r * n + k];
        if (!fin) atomicOr(flag, 1);
    }
}

}  // namespace

void spgemm_device(const DevCsr &A, const DevCsr &B, DevCsr &C, Arena &out, Arena &tmp, hipStream_t st) {
    C.n = A.n;
    C.m = B.m;
    C.rp = out.alloc<int>((size_t)A.n + 1);
    int *rowcnt = tmp.alloc<int>((size_t)A.n + 1);
    hipLaunchKernelGGL(fill_int, dim3(blocks(A.n + 1)), dim3(TB), 0, st, rowcnt, 0, (long long)A.n + 1);
    const int cbits = bits_for(B.m), rbits = bits_for(A.n);
    if (rbits + cbits > 64) throw Error(PS_EINVAL, "Galerkin product too large for 64-bit keys");
    // products per entry of A and their offsets in row-major order
    long long P = 0;
    int *rid = nullptr;
    long long *off = nullptr;
    if (A.nnz > 0 && B.nnz > 0) {
        rid = tmp.alloc<int>(A.nnz);
        hipLaunchKernelGGL(row_ids, dim3(blocks(A.n)), dim3(TB), 0, st, A.rp, A.n, rid);
        long long *cnt = tmp.alloc<long long>((size_t)A.nnz + 1);
        off = tmp.alloc<long long>((size_t)A.nnz + 1);
        hipLaunchKernelGGL(product_counts, dim3(blocks(A.nnz + 1)), dim3(TB), 0, st, A.ci, A.nnz, B.rp, cnt);
        exclusive_scan(tmp, cnt, off, (size_t)A.nnz + 1, st);
        P = read_back(off + A.nnz, st);
    }
    long long *start = nullptr, *nz = nullptr, *pos = nullptr, *Sp = nullptr;
    unsigned long long *kout = nullptr;
    double *sum = nullptr;
    if (P > 0) {
        unsigned long long *kin = tmp.alloc<unsigned long long>(P);
        kout = tmp.alloc<unsigned long long>(P);
        double *vin = tmp.alloc<double>(P), *vout = tmp.alloc<double>(P);
        hipLaunchKernelGGL(expand, dim3(blocks(A.nnz)), dim3(TB), 0, st, rid, A.ci, A.v, A.nnz, B.rp, B.ci, B.v,
                           off, cbits, kin, vin);
        size_t bytes = 0;
        PS_HIP(rocprim::radix_sort_pairs(nullptr, bytes, kin, kout, vin, vout, (size_t)P, 0u,
                                         (unsigned)(rbits + cbits), st));
        void *w = tmp.alloc<char>(bytes);
        PS_HIP(rocprim::radix_sort_pairs(w, bytes, kin, kout, vin, vout, (size_t)P, 0u,
                                         (unsigned)(rbits + cbits), st));
        // segments of equal keys, summed in order
        long long *h = tmp.alloc<long long>(P), *sid = tmp.alloc<long long>(P);
        hipLaunchKernelGGL(heads, dim3(blocks(P)), dim3(TB), 0, st, kout, P, h);
        size_t sb = 0;
        PS_HIP(rocprim::inclusive_scan(nullptr, sb, h, sid, (size_t)P, rocprim::plus<long long>(), st));
        void *w2 = tmp.alloc<char>(sb);
        PS_HIP(rocprim::inclusive_scan(w2, sb, h, sid, (size_t)P, rocprim::plus<long long>(), st));
        // the segment count S = sid[P-1] stays on the device: the segment arrays are sized P
        Sp = sid + P - 1;
        start = tmp.alloc<long long>((size_t)P + 1);
        hipLaunchKernelGGL(segment_starts, dim3(blocks(P)), dim3(TB), 0, st, h, sid, P, start);
        sum = tmp.alloc<double>(P);
        nz = tmp.alloc<long long>((size_t)P + 1);
        pos = tmp.alloc<long long>((size_t)P + 1);
        hipLaunchKernelGGL(segment_sums, dim3(blocks(P + 1)), dim3(TB), 0, st, start, (const long long *)Sp, P, vout,
                           sum, nz);
        exclusive_scan(tmp, nz, pos, (size_t)P + 1, st);
    }
    const long long nnz = P > 0 ? read_back(pos + P, st) : 0;
    if (nnz >= (1ll << 31)) throw Error(PS_EINVAL, "Galerkin product exceeds 2^31 entries");
    C.nnz = (int)nnz;
    C.ci = out.alloc<int>((size_t)nnz);
    C.v = out.alloc<double>((size_t)nnz);
    if (nnz > 0)
        hipLaunchKernelGGL(scatter, dim3(blocks(P)), dim3(TB), 0, st, start, (const long long *)Sp, kout, sum, nz, pos,
                           cbits, C.ci, C.v, rowcnt);
    exclusive_scan(tmp, rowcnt, C.rp, (size_t)A.n + 1, st);
    PS_HIP(hipStreamSynchronize(st));
}

// Quasi-IMPES reduction (Sec. 5.2) from the system's A_ff in SELL-64 (one lane per cell
// row) and the fixed-stress terms: the same operations as the host's, without contraction.
// D_ss^{-1} into dss (if given); S_pp's values, on A_ff's block pattern (rp), into spp (if
// given): the pressure-row, pressure-column entry of each S_ff block less t_i times its
// saturation-row entries, t_i = D_ps,i D_ss,i^{-1}.  flag (if given) is set for a singular D_ss.
template <int NF, typename TD>
__global__ void qimpes_k(Sell<double> A, const int *__restrict__ rp, const int *__restrict__ dslot,
                         const double *__restrict__ d_sp, const double *__restrict__ d_pp, int n,
                         double *__restrict__ spp, TD *__restrict__ dss, int *__restrict__ flag) {
#pragma clang fp contract(off)
    constexpr int NN = NF * NF;
    const int i = blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    const int lane = i & 63, s0 = A.cptr[i >> 6], ds = dslot[i];
    auto val = [&](int k, int e) { return A.val[((size_t)(s0 + k) * NN + e) * 64 + lane]; };
    double t0 = 0.0, t1 = 0.0;
    if (NF == 2) {
        const double dss_ = val(ds, 0), dps = val(ds, NF * (NF - 1) + 0);
        if (dss_ == 0.0) {
            if (flag) flag[0] = 1;
            return;
        }
        t0 = dps / dss_;
        if (dss) dss[i] = (TD)(1.0 / dss_);
    } else {
        const double a = val(ds, 0 * NF + 0), b = val(ds, 0 * NF + 1), c = val(ds, 1 * NF + 0), d = val(ds, 1 * NF + 1);
        const double det = a * d - b * c;
        if (det == 0.0 || !isfinite(det)) {
            if (flag) flag[0] = 1;
            return;
        }
        const double i00 = d / det, i01 = -b / det, i10 = -c / det, i11 = a / det;
        const double p0 = val(ds, (NF - 1) * NF + 0), p1 = val(ds, (NF - 1) * NF + 1);
        t0 = p0 * i00 + p1 * i10;
        t1 = p0 * i01 + p1 * i11;
        if (dss) {
            dss[(size_t)i * 4 + 0] = (TD)i00;
            dss[(size_t)i * 4 + 1] = (TD)i01;
            dss[(size_t)i * 4 + 2] = (TD)i10;
            dss[(size_t)i * 4 + 3] = (TD)i11;
        }
    }
    if (!spp) return;
    const int r0 = rp[i], len = rp[i + 1] - r0;
    for (int k = 0; k < len; ++k) {
        double app = val(k, (NF - 1) * NF + NF - 1), sp0 = val(k, 0 * NF + NF - 1);
        double sp1 = NF == 3 ? val(k, 1 * NF + NF - 1) : 0.0;
        if (k == ds) {                      // fixed-stress terms of the diagonal block
            sp0 += d_sp[(size_t)i * (NF - 1) + 0];
            if (NF == 3) sp1 += d_sp[(size_t)i * (NF - 1) + 1];
            app += d_pp[i];
        }
        if (NF == 2) {
            spp[r0 + k] = app - t0 * sp0;
        } else {
            const double s0v = t0 * sp0, s1v = t1 * sp1;
            spp[r0 + k] = app - (s0v + s1v);
        }
    }
}

static DevCsr upload(Arena &ar, const Csr &A) {
    DevCsr d;
    d.n = A.n;
    d.m = A.m;
    d.nnz = A.nnz();
    d.rp = ar.upload(A.rp.data(), A.rp.size());
    d.ci = ar.upload(A.ci.data(), A.ci.size());
    d.v = ar.upload(A.v.data(), A.v.size());
    return d;
}

static Csr download(const DevCsr &d) {
    Csr A;
    A.n = d.n;
    A.m = d.m;
    A.rp.resize((size_t)d.n + 1);
    A.ci.resize(d.nnz);
    A.v.resize(d.nnz);
    PS_HIP(hipMemcpy(A.rp.data(), d.rp, sizeof(int) * A.rp.size(), hipMemcpyDeviceToHost));
    if (d.nnz) {
        PS_HIP(hipMemcpy(A.ci.data(), d.ci, sizeof(int) * A.ci.size(), hipMemcpyDeviceToHost));
        PS_HIP(hipMemcpy(A.v.data(), d.v, sizeof(double) * A.v.size(), hipMemcpyDeviceToHost));
    }
    return A;
}

// The pressure AMG of amg_build with each Galerkin product R (A P) formed on the device:
// the host coarsens level l (strength, PMIS, interpolation) from its copy of A_l, the
// device forms A_{l+1}, and the host copy of A_{l+1} comes back for the next level.
// (Used with Chebyshev smoothing, whose eigenvalue estimate is taken on the host.)
static void build_pressure_hybrid(const Csr &Spp, const Options &o, Hierarchy &H, PresStore &S) {
    const hipStream_t st = 0;
    Csr A = Spp;
    DevCsr Ad = upload(S.arena, A);
    while (A.n > o.coarse_max && (int)H.lev.size() + 1 < o.max_levels) {
        Level L;
        if (!coarsen_level(A, o, L)) break;
        DevCsr Pd = upload(S.arena, L.P), Rd = upload(S.arena, L.R), APd, Acd;
        S.work.recycle();
        S.tmp.recycle();
        spgemm_device(Ad, Pd, APd, S.work, S.tmp, st);
        S.tmp.recycle();
        spgemm_device(Rd, APd, Acd, S.arena, S.tmp, st);
        Csr Ac = download(Acd);
        L.A = std::move(A);
        finish_level(L, o.smoother);
        H.lev.push_back(std::move(L));
        S.A.push_back(Ad);
        S.P.push_back(Pd);
        S.R.push_back(Rd);
        A = std::move(Ac);
        Ad = Acd;
    }
    S.A.push_back(Ad);
    coarse_level(std::move(A), H);
}

// The whole pressure AMG on the device (l1-Jacobi smoothing): strength, PMIS, C-promotion,
// direct interpolation, R = P^T, the Galerkin product and the smoother diagonal, with the
// same results as the host build; only counts come back per step, and the coarsest
// operator at the end for its dense inverse.  H holds the level sizes and the coarse
// inverse; the operators, splittings and smoother data stay in S.
// Levels of the l1-Jacobi hierarchy from the level-0 operator A, all on the device.
static void build_pressure_levels(DevCsr A, const Options &o, Hierarchy &H, PresStore &S) {
    const hipStream_t st = 0;
    auto zero = [&](int *p, long long n) {
        hipLaunchKernelGGL(fill_int, dim3(blocks(n)), dim3(TB), 0, st, p, 0, n);
    };
    int *ctr = S.arena.alloc<int>(4);
    int *zdiag = ctr + 1;                 // a zero diagonal on some level (checked once, at the end)
    zero(zdiag, 1);
    while (A.n > o.coarse_max && (int)H.lev.size() + 1 < o.max_levels) {
        const int n = A.n, nnz = A.nnz;
        TraceTick lt("pressure level");
        g_round_trips = 0;
        struct Note {
            TraceTick &t;
            ~Note() { t.note = g_round_trips; }
        } note{lt};
        S.work.recycle();
        S.tmp.recycle();
        // strength and S, S^T
        signed char *smask = S.work.alloc<signed char>(nnz);
        int *scount = S.work.alloc<int>((size_t)n + 1), *lam = S.work.alloc<int>((size_t)n + 1);
        zero(scount, n + 1);
        zero(lam, n + 1);
        hipLaunchKernelGGL(strength_k, dim3(blocks(n)), dim3(TB), 0, st, A.rp, A.ci, A.v, n, o.theta, smask, scount,
                           lam);
        int *srp = S.work.alloc<int>((size_t)n + 1), *trp = S.work.alloc<int>((size_t)n + 1);
        exclusive_scan(S.tmp, scount, srp, (size_t)n + 1, st);
        exclusive_scan(S.tmp, lam, trp, (size_t)n + 1, st);
        // S and S^T hold at most nnz entries (no read-back of the exact count)
        int *sci = S.work.alloc<int>(nnz), *tci = S.work.alloc<int>(nnz), *cur = S.work.alloc<int>(n);
        hipLaunchKernelGGL(fill_s_k, dim3(blocks(n)), dim3(TB), 0, st, A.rp, A.ci, smask, n, srp, sci);
        PS_HIP(hipMemcpyAsync(cur, trp, sizeof(int) * n, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(fill_st_k, dim3(blocks(n)), dim3(TB), 0, st, srp, sci, n, cur, tci);
        // PMIS rounds
        double *w = S.work.alloc<double>(n);
        signed char *cf = S.arena.alloc<signed char>(n), *newc = S.work.alloc<signed char>(n);
        zero(ctr, 1);
        hipLaunchKernelGGL(pmis_init_k, dim3(blocks(n)), dim3(TB), 0, st, trp, n, w, cf, ctr);
        // two rounds per read-back of the undecided count, the first two before any (a round
        // with nothing undecided changes nothing)
        int rounds = 0;
        for (int und = n > 0 ? 1 : 0; und > 0; und = read_back(ctr, st)) {
            for (int k = 0; k < 2; ++k) {
                if (++rounds > n + 1) throw Error(PS_EDEVICE, "PMIS did not terminate");   // each round decides >= 1 point
                hipLaunchKernelGGL(pmis_select_k, dim3(blocks(n)), dim3(TB), 0, st, cf, w, srp, sci, trp, tci, n, newc);
                zero(ctr, 1);
                hipLaunchKernelGGL(pmis_mark_k, dim3(blocks(n)), dim3(TB), 0, st, cf, newc, srp, sci, n, ctr);
            }
        }
        // C-promotion
        signed char *cs = S.work.alloc<signed char>(n);
        zero(ctr, 1);
        hipLaunchKernelGGL(promo_init_k, dim3(blocks(n)), dim3(TB), 0, st, cf, srp, sci, n, cs, ctr);
        rounds = 0;
        for (int und = n > 0 ? 1 : 0; und > 0; und = read_back(ctr, st)) {
            for (int k = 0; k < 2; ++k) {
                if (++rounds > n + 1) throw Error(PS_EDEVICE, "C-promotion did not terminate");
                zero(ctr, 1);
                hipLaunchKernelGGL(promo_round_k, dim3(blocks(n)), dim3(TB), 0, st, cs, srp, sci, n, ctr);
            }
        }
        int *cflag = S.work.alloc<int>((size_t)n + 1), *cidx = S.work.alloc<int>((size_t)n + 1);
        hipLaunchKernelGGL(promo_apply_k, dim3(blocks(n + 1)), dim3(TB), 0, st, cf, cs, n, cflag);
        exclusive_scan(S.tmp, cflag, cidx, (size_t)n + 1, st);
        const int nc = read_back(cidx + n, st);
        if (nc == 0 || (double)nc > 0.9 * (double)n) break;
        // direct interpolation and R = P^T
        int *plen = S.work.alloc<int>((size_t)n + 1);
        hipLaunchKernelGGL(interp_count_k, dim3(blocks(n + 1)), dim3(TB), 0, st, A.rp, A.ci, smask, cf, n, plen);
        DevCsr P;
        P.n = n;
        P.m = nc;
        P.rp = S.arena.alloc<int>((size_t)n + 1);
        exclusive_scan(S.tmp, plen, P.rp, (size_t)n + 1, st);
        P.nnz = read_back(P.rp + n, st);
        P.ci = S.arena.alloc<int>(P.nnz);
        P.v = S.arena.alloc<double>(P.nnz);
        hipLaunchKernelGGL(interp_fill_k, dim3(blocks(n)), dim3(TB), 0, st, A.rp, A.ci, A.v, smask, cf, cidx, n, P.rp,
                           P.ci, P.v);
        DevCsr R;
        R.n = nc;
        R.m = n;
        R.nnz = P.nnz;
        int *rcnt = S.work.alloc<int>((size_t)nc + 1), *rcur = S.work.alloc<int>(nc);
        zero(rcnt, nc + 1);
        hipLaunchKernelGGL(col_count_k, dim3(blocks(P.nnz)), dim3(TB), 0, st, P.ci, P.nnz, rcnt);
        R.rp = S.arena.alloc<int>((size_t)nc + 1);
        exclusive_scan(S.tmp, rcnt, R.rp, (size_t)nc + 1, st);
        R.ci = S.arena.alloc<int>(R.nnz);
        R.v = S.arena.alloc<double>(R.nnz);
        PS_HIP(hipMemcpyAsync(rcur, R.rp, sizeof(int) * nc, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(transpose_fill_k, dim3(blocks(n)), dim3(TB), 0, st, P.rp, P.ci, P.v, n, rcur, R.ci, R.v);
        hipLaunchKernelGGL(sort_rows_k, dim3(blocks((long long)nc * 64)), dim3(TB), 0, st, R.rp, nc, R.ci, R.v);
        // smoother diagonal
        double *dinv = S.arena.alloc<double>(n);
        hipLaunchKernelGGL(l1_inv_k, dim3(blocks(n)), dim3(TB), 0, st, A.rp, A.ci, A.v, n, dinv, zdiag);
        // Galerkin product
        DevCsr AP, Ac;
        S.tmp.recycle();
        spgemm_device(A, P, AP, S.work, S.tmp, st);
        S.tmp.recycle();
        spgemm_device(R, AP, Ac, S.arena, S.tmp, st);
        Level L;
        L.A.n = L.A.m = n;
        H.lev.push_back(std::move(L));
        S.A.push_back(A);
        S.P.push_back(P);
        S.R.push_back(R);
        S.cf.push_back(cf);
        S.dinv.push_back(dinv);
        A = Ac;
    }
    S.A.push_back(A);
    if (A.n > DI_WG) {                    // dense inverse on the host (beyond one workgroup)
        if (read_back(zdiag, st) != 0) throw Error(PS_ESINGULAR, "zero diagonal in an AMG level");
        coarse_level(download(A), H);
        return;
    }
    // the coarsest level's dense inverse on the device (bitwise the host's); one read-back
    // brings the zero-diagonal flag and the inverse's singularity flag together
    int *iflag = ctr + 2;
    zero(iflag, 1);
    const size_t an = (size_t)A.n * A.n;
    S.cinv = S.arena.alloc<double>(an);
    int *piv = S.work.alloc<int>((size_t)A.n + 1);
    if (2 * an * sizeof(double) <= (size_t)150 * 1024) {
        // the factor and the solved columns in LDS: allow up to 150 KB (once per process)
        static std::once_flag raised;
        std::call_once(raised, [] {
            PS_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&dense_inverse_k<true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
        });
        hipLaunchKernelGGL((dense_inverse_k<true>), dim3(1), dim3(DI_WG), 2 * an * sizeof(double), st, A.rp, A.ci,
                           A.v, A.n, (double *)nullptr, S.cinv, piv, iflag);
    } else {
        double *ga = S.work.alloc<double>(an);
        hipLaunchKernelGGL((dense_inverse_k<false>), dim3(1), dim3(DI_WG), 0, st, A.rp, A.ci, A.v, A.n, ga, S.cinv, piv,
                           iflag);
    }
    PS_HIP(hipGetLastError());
    struct Flags {
        int zdiag, singular;
    };
    const Flags fl = read_back(reinterpret_cast<const Flags *>(zdiag), st);
    if (fl.zdiag != 0) throw Error(PS_ESINGULAR, "zero diagonal in an AMG level");
    if (fl.singular != 0) throw Error(PS_ESINGULAR, "singular coarsest AMG matrix");
    Level C;
    C.A.n = C.A.m = A.n;
    C.cf.assign(A.n, 0);
    H.coarse_n = A.n;
    H.lev.push_back(std::move(C));
}

static void clear_store(Hierarchy &H, PresStore &S) {
    H = Hierarchy();
    S.cinv = nullptr;
    S.arena.recycle();
    S.A.clear();
    S.P.clear();
    S.R.clear();
    S.cf.clear();
    S.dinv.clear();
}

void build_pressure(const Csr &Spp, const Options &o, Hierarchy &H, PresStore &S) {
    clear_store(H, S);
    S.on_device = o.smoother == PS_L1JAC;
    if (S.on_device) build_pressure_levels(upload(S.arena, Spp), o, H, S);
    else build_pressure_hybrid(Spp, o, H, S);
    S.arena.trim();          // blocks of an earlier, larger hierarchy that were not reused
}

void layout_pressure_operator(const System &s, PresStore &S) {
    const Bsr &A = s.Aff;
    const int n = A.nbr;
    std::vector<int> dslot(n, -1);
    for (int i = 0; i < n; ++i)
        for (int t = A.rp[i]; t < A.rp[i + 1]; ++t)
            if (A.ci[t] == i) dslot[i] = t - A.rp[i];
    for (int i = 0; i < n; ++i)
        if (dslot[i] < 0) throw Error(PS_EINVAL, "A_ff row without a diagonal block");
    S.pat.release();
    S.spp_rp = S.pat.upload(A.rp.data(), A.rp.size());
    S.spp_ci = S.pat.upload(A.ci.data(), A.ci.size());
    S.aff_dslot = S.pat.upload(dslot.data(), dslot.size());
    S.fs = S.pat.alloc<double>((size_t)n * s.nf);
    S.flag = S.pat.alloc<int>(1);
    S.nnzpat = A.rp[n];
    S.npat = n;
}

void build_pressure_from_system(const System &s, const DSystem &D, const Options &o, Hierarchy &H, PresStore &S) {
    if (S.npat != s.n_cells || o.smoother != PS_L1JAC) throw Error(PS_EDEVICE, "pressure operator not laid out");
    clear_store(H, S);
    S.on_device = true;
    const int n = s.n_cells, nf = s.nf;
    const size_t nsp = (size_t)n * (nf - 1);
    double *h = static_cast<double *>(S.stg.get((size_t)n * nf * sizeof(double)));
    std::memcpy(h, s.d_sp.data(), nsp * sizeof(double));
    std::memcpy(h + nsp, s.d_pp.data(), (size_t)n * sizeof(double));
    S.stg.copy_to_device(S.fs, h, (size_t)n * nf * sizeof(double));
    DevCsr A;
    A.n = A.m = n;
    A.nnz = S.nnzpat;
    A.rp = S.spp_rp;
    A.ci = S.spp_ci;
    A.v = S.arena.alloc<double>(S.nnzpat);
    const hipStream_t st = 0;
    hipLaunchKernelGGL(fill_int, dim3(1), dim3(TB), 0, st, S.flag, 0, 1ll);
    if (nf == 2)
        hipLaunchKernelGGL((qimpes_k<2, double>), dim3(blocks(n)), dim3(TB), 0, st, D.Aff, (const int *)S.spp_rp,
                           (const int *)S.aff_dslot, (const double *)S.fs, (const double *)S.fs + nsp, n, A.v,
                           (double *)nullptr, S.flag);
    else
        hipLaunchKernelGGL((qimpes_k<3, double>), dim3(blocks(n)), dim3(TB), 0, st, D.Aff, (const int *)S.spp_rp,
                           (const int *)S.aff_dslot, (const double *)S.fs, (const double *)S.fs + nsp, n, A.v,
                           (double *)nullptr, S.flag);
    if (read_back(S.flag, st)) throw Error(PS_ESINGULAR, nf == 2 ? "zero D_ss entry" : "singular D_ss block");
    build_pressure_levels(A, o, H, S);
    S.arena.trim();
}

template <typename T>
void dss_inverse_device(const DSystem &D, const int *dslot, T *dss_inv, hipStream_t st) {
    const int n = D.n_cells;
    if (D.nf == 2)
        hipLaunchKernelGGL((qimpes_k<2, T>), dim3(blocks(n)), dim3(TB), 0, st, D.Aff, (const int *)nullptr, dslot,
                           (const double *)nullptr, (const double *)nullptr, n, (double *)nullptr, dss_inv,
                           (int *)nullptr);
    else
        hipLaunchKernelGGL((qimpes_k<3, T>), dim3(blocks(n)), dim3(TB), 0, st, D.Aff, (const int *)nullptr, dslot,
                           (const double *)nullptr, (const double *)nullptr, n, (double *)nullptr, dss_inv,
                           (int *)nullptr);
    PS_HIP(hipGetLastError());
}

template void dss_inverse_device<double>(const DSystem &, const int *, double *, hipStream_t);
template void dss_inverse_device<float>(const DSystem &, const int *, float *, hipStream_t);

void download_level(const PresStore &S, int lvl, Csr &A, std::vector<int8_t> &cf) {
    A = download(S.A.at(lvl));
    cf.assign(A.n, 0);
    if (lvl < (int)S.cf.size() && A.n)
        PS_HIP(hipMemcpy(cf.data(), S.cf[lvl], (size_t)A.n, hipMemcpyDeviceToHost));
}

}  // namespace ps
