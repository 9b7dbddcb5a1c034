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

__global__ void segment_sums(const long long *__restrict__ start, long long S, const double *__restrict__ vals,
                             double *__restrict__ sum, long long *__restrict__ nz) {
    long long s = (long long)blockIdx.x * TB + threadIdx.x;
    if (s > S) return;
    if (s == S) {
        nz[s] = 0;
        return;
    }
    double acc = 0.0;
    for (long long p = start[s]; p < start[s + 1]; ++p) acc = __dadd_rn(acc, vals[p]);
    sum[s] = acc;
    nz[s] = acc != 0.0 ? 1 : 0;
}

__global__ void scatter(const long long *__restrict__ start, long long S, const unsigned long long *__restrict__ keys,
                        const double *__restrict__ sum, const long long *__restrict__ nz,
                        const long long *__restrict__ pos, int cbits, int *__restrict__ ci,
                        double *__restrict__ v, int *__restrict__ rowcnt) {
    long long s = (long long)blockIdx.x * TB + threadIdx.x;
    if (s >= S || !nz[s]) return;
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

template <typename T>
T read_back(const T *d, hipStream_t st) {
    T h;
    PS_HIP(hipMemcpyAsync(&h, d, sizeof(T), hipMemcpyDeviceToHost, st));
    PS_HIP(hipStreamSynchronize(st));
    return h;
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
    long long S = 0, *start = nullptr, *nz = nullptr, *pos = nullptr;
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
        S = read_back(sid + P - 1, st);
        start = tmp.alloc<long long>((size_t)S + 1);
        hipLaunchKernelGGL(segment_starts, dim3(blocks(P)), dim3(TB), 0, st, h, sid, P, start);
        sum = tmp.alloc<double>(S);
        nz = tmp.alloc<long long>((size_t)S + 1);
        pos = tmp.alloc<long long>((size_t)S + 1);
        hipLaunchKernelGGL(segment_sums, dim3(blocks(S + 1)), dim3(TB), 0, st, start, S, vout, sum, nz);
        exclusive_scan(tmp, nz, pos, (size_t)S + 1, st);
    }
    const long long nnz = S > 0 ? read_back(pos + S, st) : 0;
    if (nnz >= (1ll << 31)) throw Error(PS_EINVAL, "Galerkin product exceeds 2^31 entries");
    C.nnz = (int)nnz;
    C.ci = out.alloc<int>((size_t)nnz);
    C.v = out.alloc<double>((size_t)nnz);
    if (nnz > 0)
        hipLaunchKernelGGL(scatter, dim3(blocks(S)), dim3(TB), 0, st, start, S, kout, sum, nz, pos, cbits, C.ci,
                           C.v, rowcnt);
    exclusive_scan(tmp, rowcnt, C.rp, (size_t)A.n + 1, st);
    PS_HIP(hipStreamSynchronize(st));
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
void build_pressure(const Csr &Spp, const Options &o, Hierarchy &H, PresStore &S) {
    H = Hierarchy();
    S.arena.recycle();
    S.A.clear();
    S.P.clear();
    S.R.clear();
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
    S.arena.trim();          // blocks of an earlier, larger hierarchy that were not reused
}

}  // namespace ps
