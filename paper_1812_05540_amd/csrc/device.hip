// Device data layout, uploads and the solve-phase drivers (Algorithm 1, FGMRES).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <optional>
#include <string>

#include "kernels.h"

namespace ps {

using k::WG;

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(PS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
}

static inline unsigned grid_for(size_t n) { return (unsigned)((n + WG - 1) / WG); }

#define LAUNCH(kernel, grid, shm, st, ...)                                             \
    do {                                                                               \
        if ((grid) > 0) hipLaunchKernelGGL(kernel, dim3(grid), dim3(WG), shm, st, __VA_ARGS__); \
    } while (0)

// ------------------------------------------------------------------ kernel timing
namespace ktime {
namespace {
std::atomic<unsigned> g_mask{0u};          // bit i: kernel id i is bracketed
std::mutex g_mu;
struct Rec {
    int id;
    hipEvent_t e0, e1;
    double bytes;
};
std::vector<Rec> g_pending;
std::vector<hipEvent_t> g_pool;
long long g_launches[NUM];
double g_seconds[NUM], g_bytes[NUM];

hipEvent_t get_event() {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    PS_HIP(hipEventCreate(&e));
    return e;
}

void drain_locked() {
    for (Rec &r : g_pending) {
        PS_HIP(hipEventSynchronize(r.e1));
        float ms = 0.f;
        PS_HIP(hipEventElapsedTime(&ms, r.e0, r.e1));
        g_launches[r.id] += 1;
        g_seconds[r.id] += ms * 1e-3;
        g_bytes[r.id] += r.bytes;
        g_pool.push_back(r.e0);
        g_pool.push_back(r.e1);
    }
    g_pending.clear();
}
}  // namespace

const char *name(int id) {
    static const char *n[NUM] = {"system_spmv", "cgs2_project", "cgs2_subtract_project", "cgs2_subtract_norm",
                                 "bilu_subdomain", "sdc_l0_presmooth", "sdc_l0_restrict", "sdc_l0_prolong",
                                 "sdc_l0_postsmooth", "pres_l0_presmooth", "pres_l0_restrict",
                                 "pres_l0_prolong", "pres_l0_postsmooth", "dcgs2_project", "dcgs2_subtract"};
    return id >= 0 && id < NUM ? n[id] : "";
}

bool enabled() { return g_mask.load(std::memory_order_relaxed) != 0u; }

bool enabled(int id) { return id >= 0 && id < NUM && ((g_mask.load(std::memory_order_relaxed) >> id) & 1u); }

void set_mask(unsigned mask) {
    std::lock_guard<std::mutex> lk(g_mu);
    drain_locked();
    for (int i = 0; i < NUM; ++i) {
        g_launches[i] = 0;
        g_seconds[i] = g_bytes[i] = 0.0;
    }
    g_mask.store(mask & ((1u << NUM) - 1u));
}

Scope::Scope(int i, hipStream_t s, double b) : id(i), st(s), bytes(b) {
    if (!enabled(id)) return;
    e0 = get_event();
    PS_HIP(hipEventRecord(e0, st));
}

Scope::~Scope() {
    if (!e0) return;
    hipEvent_t e1 = get_event();
    if (hipEventRecord(e1, st) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_pending.size() >= 4096) drain_locked();    // bound the events in flight
    g_pending.push_back({id, e0, e1, bytes});
}

void totals(int id, long long &launches, double &seconds, double &bytes) {
    std::lock_guard<std::mutex> lk(g_mu);
    drain_locked();
    launches = g_launches[id];
    seconds = g_seconds[id];
    bytes = g_bytes[id];
}
}  // namespace ktime

// ------------------------------------------------------------------ setup tracing
static bool trace_setup() {
    static const bool on = [] {
        const char *e = std::getenv("PS_TRACE");
        return e && *e && *e != '0';
    }();
    return on;
}

static double wall_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

TraceTick::TraceTick(const char *w) : what(w), t0(wall_s()) {}

TraceTick::~TraceTick() {
    if (!trace_setup()) return;
    if (note >= 0) std::fprintf(stderr, "[ps]     %-24s %8.2f ms  (%d)\n", what, 1e3 * (wall_s() - t0), note);
    else std::fprintf(stderr, "[ps]     %-24s %8.2f ms\n", what, 1e3 * (wall_s() - t0));
}

// ------------------------------------------------------------------ SELL
HostSell sell_from_bsr(const std::vector<int> &rp, const std::vector<int> &ci, const std::vector<double> &v,
                       int nbr, int br, int bc, const std::vector<int> *row_order,
                       bool (*keep)(int, int), bool values) {
    HostSell h;
    h.br = br;
    h.bc = bc;
    const int rc = br * bc;
    std::vector<int> order;
    if (row_order) {
        order = *row_order;
    } else {
        order.resize(nbr);
        std::iota(order.begin(), order.end(), 0);
    }
    h.nrows = (int)order.size();
    h.nchunks = (h.nrows + 63) / 64;
    auto count = [&](int row) {
        if (row < 0) return 0;
        if (!keep) return rp[row + 1] - rp[row];
        int c = 0;
        for (int t = rp[row]; t < rp[row + 1]; ++t) c += keep(row, ci[t]);
        return c;
    };
    h.cptr.assign(h.nchunks + 1, 0);
    for (int ch = 0; ch < h.nchunks; ++ch) {
        int w = 0;
        for (int l = 0; l < 64; ++l) {
            int pos = ch * 64 + l;
            if (pos < h.nrows) w = std::max(w, count(order[pos]));
        }
        h.cptr[ch + 1] = h.cptr[ch] + w;
    }
    size_t nslots = (size_t)h.cptr[h.nchunks];
    h.col.assign(nslots * 64, 0);
    h.src.assign(nslots * 64, -1);
    if (values) h.val.assign(nslots * 64 * rc, 0.0);
    for (int pos = 0; pos < h.nrows; ++pos) {
        int row = order[pos];
        if (row < 0) continue;
        int ch = pos >> 6, lane = pos & 63;
        size_t s0 = (size_t)h.cptr[ch];
        int kk = 0;
        for (int t = rp[row]; t < rp[row + 1]; ++t) {
            if (keep && !keep(row, ci[t])) continue;
            h.col[(s0 + kk) * 64 + lane] = ci[t];
            h.src[(s0 + kk) * 64 + lane] = t;
            if (values)
                for (int e = 0; e < rc; ++e) h.val[((s0 + kk) * rc + e) * 64 + lane] = v[(size_t)t * rc + e];
            ++kk;
        }
    }
    if (row_order) h.rowmap = order;
    return h;
}

HostSell sell_from_csr(const Csr &A) { return sell_from_bsr(A.rp, A.ci, A.v, A.n, 1, 1); }

template <typename T>
Sell<T> upload_sell(Arena &ar, const HostSell &h) {
    Sell<T> s;
    s.nrows = h.nrows;
    s.nchunks = h.nchunks;
    s.br = h.br;
    s.bc = h.bc;
    s.nslots = h.cptr.empty() ? 0 : (size_t)h.cptr.back();
    s.cptr = ar.upload(h.cptr.data(), h.cptr.size());
    s.col = ar.upload(h.col.data(), h.col.size());
    std::vector<T> vt(h.val.begin(), h.val.end());
    s.val = ar.upload(vt.data(), vt.size());
    if (!h.rowmap.empty()) s.rowmap = ar.upload(h.rowmap.data(), h.rowmap.size());
    return s;
}

// An operator takes the SELL-64 form (one lane per row, coalesced loads) when its 64-row
// slices pad it to at most 1.5 stored slots per entry, its rows average at most 128 entries
// and it has at least 2^17 rows (2048 wavefronts); otherwise one lane per row leaves too
// few wavefronts with too long a chain of loads each, and CSR with G lanes per row is
// faster on MI355X (measured on grf64: the SDC operator's second level, 227k rows of 67
// entries on average, is 12 us per V-cycle faster in SELL-64; its third, 44k rows, slower).
// PS_SELL=all puts every operator in SELL-64, PS_SELL=off none.
static int sell_mode() {                 // 0 by the rule above, 1 all, -1 none
    const char *e = std::getenv("PS_SELL");
    if (!e) return 0;
    if (std::string(e) == "all") return 1;
    if (std::string(e) == "off") return -1;
    return 0;
}

// Stored slots per entry of the SELL-64 form of an n-row matrix with nnz entries whose
// slices have widths w.
static double sell_padding(const int *w, int n, size_t nnz) {
    size_t slots = 0;
    for (int s = 0; s < (n + 63) / 64; ++s) slots += (size_t)w[s] * 64;
    return nnz ? (double)slots / nnz : 1e30;
}

static bool take_sell(double pad, int n, size_t nnz) {
    const int mode = sell_mode();
    if (mode < 0 || pad * nnz >= 2e9) return false;
    return mode > 0 || (pad <= 1.5 && n >= (1 << 17) && nnz <= (size_t)128 * n);
}

static int lanes_per_row(int n, size_t nnz) {
    double avg = n ? (double)nnz / n : 1.0;
    int G = 1;
    while (G < 32 && G * 3 < avg) G *= 2;
    return G;
}

// sell: an operator A, which may take SELL-64 (P and R stay CSR)
template <typename T>
static DCsr<T> upload_csr(Arena &ar, const Csr &A, bool sell) {
    DCsr<T> d;
    d.n = A.n;
    d.nnz = A.nnz();
    d.G = lanes_per_row(A.n, A.nnz());
    d.rp = ar.upload(A.rp.data(), A.rp.size());
    std::vector<int> w((A.n + 63) / 64, 0);
    for (int i = 0; i < A.n; ++i) w[i >> 6] = std::max(w[i >> 6], A.rp[i + 1] - A.rp[i]);
    if (sell && A.n && take_sell(sell_padding(w.data(), A.n, A.nnz()), A.n, A.nnz())) {
        HostSell h = sell_from_bsr(A.rp, A.ci, A.v, A.n, 1, 1);
        d.G = 0;
        d.cptr = ar.upload(h.cptr.data(), h.cptr.size());
        // columns as 16-bit offsets from the row when every one fits (stencil-like levels)
        std::vector<short> cd(h.col.size(), 0);
        bool fits = true;
        for (int i = 0; i < A.n && fits; ++i) {
            const int ch = i >> 6, lane = i & 63;
            for (int k = 0; k < A.rp[i + 1] - A.rp[i]; ++k) {
                const size_t q = ((size_t)h.cptr[ch] + k) * 64 + lane;
                const int dlt = h.col[q] - i;
                if (dlt < -32768 || dlt > 32767) {
                    fits = false;
                    break;
                }
                cd[q] = (short)dlt;
            }
        }
        if (fits) {
            d.G = -1;
            d.cd = ar.upload(cd.data(), cd.size());
        } else {
            d.ci = ar.upload(h.col.data(), h.col.size());
        }
        std::vector<T> v(h.val.begin(), h.val.end());
        d.v = ar.upload(v.data(), v.size());
        return d;
    }
    // an operator's columns as 16-bit offsets from the row when every one fits
    bool fits = sell && A.n > 0;
    std::vector<short> cd;
    if (fits) {
        cd.resize(A.ci.size());
        for (int i = 0; i < A.n && fits; ++i)
            for (int t = A.rp[i]; t < A.rp[i + 1]; ++t) {
                const int dlt = A.ci[t] - i;
                if (dlt < -32768 || dlt > 32767) {
                    fits = false;
                    break;
                }
                cd[t] = (short)dlt;
            }
    }
    if (fits) {
        d.G += 64;
        d.cd = ar.upload(cd.data(), cd.size());
    } else {
        d.ci = ar.upload(A.ci.data(), A.ci.size());
    }
    std::vector<T> v(A.v.begin(), A.v.end());
    d.v = ar.upload(v.data(), v.size());
    return d;
}

template <typename T>
static const T *upload_vec(Arena &ar, const std::vector<double> &v) {
    std::vector<T> t(v.begin(), v.end());
    return ar.upload(t.data(), t.size());
}

// Level 0 of the separate-displacement-component hierarchy is stored in the
// interleaved (node-major) order of z_u: component-major index c*nn + i -> 3 i + c.
static void interleave_level0(Csr &A, Csr &P, Csr &R, std::vector<std::vector<double> *> vecs) {
    int n = A.n, nn = n / 3;
    auto il = [nn](int a) { return 3 * (a % nn) + a / nn; };
    auto permute_rows = [&](const Csr &M, bool map_cols) {
        Csr out;
        out.n = M.n;
        out.m = M.m;
        out.rp.assign(M.n + 1, 0);
        std::vector<int> src(M.n);
        for (int a = 0; a < M.n; ++a) src[il(a)] = a;
        std::vector<std::pair<int, double>> row;
        for (int r = 0; r < M.n; ++r) {
            int a = src[r];
            row.clear();
            for (int t = M.rp[a]; t < M.rp[a + 1]; ++t)
                row.push_back({map_cols ? il(M.ci[t]) : M.ci[t], M.v[t]});
            std::sort(row.begin(), row.end(), [](auto &x, auto &y) { return x.first < y.first; });
            for (auto &e : row) {
                out.ci.push_back(e.first);
                out.v.push_back(e.second);
            }
            out.rp[r + 1] = (int)out.ci.size();
        }
        return out;
    };
    A = permute_rows(A, true);
    P = permute_rows(P, false);
    Csr Rn = R;
    for (int r = 0; r < R.n; ++r) {
        std::vector<std::pair<int, double>> row;
        for (int t = R.rp[r]; t < R.rp[r + 1]; ++t) row.push_back({il(R.ci[t]), R.v[t]});
        std::sort(row.begin(), row.end(), [](auto &x, auto &y) { return x.first < y.first; });
        for (size_t q = 0; q < row.size(); ++q) {
            Rn.ci[R.rp[r] + q] = row[q].first;
            Rn.v[R.rp[r] + q] = row[q].second;
        }
    }
    R = std::move(Rn);
    for (auto *v : vecs) {
        if (v->empty()) continue;
        std::vector<double> o(v->size());
        for (int a = 0; a < n; ++a) o[il(a)] = (*v)[a];
        *v = std::move(o);
    }
}

template <typename T>
void upload_hierarchy_into(DHierarchy<T> &dh, const Hierarchy &H, int smoother, bool interleave3) {
    DHierarchy<T> *d = &dh;
    d->arena.recycle();
    d->smoother = smoother;
    int nl = (int)H.lev.size();
    d->lev.assign(nl, DLevel<T>());
    for (int l = 0; l + 1 < nl; ++l) {
        const Level &L = H.lev[l];
        DLevel<T> &D = d->lev[l];
        if (l == 0 && interleave3) {
            Csr A = L.A, P = L.P, R = L.R;
            std::vector<double> dl1 = L.dl1, c0 = L.c0, c1 = L.c1, cm = L.cm;
            interleave_level0(A, P, R, {&dl1, &c0, &c1, &cm});
            D.n = A.n;
            D.A = upload_csr<T>(d->arena, A, true);
            D.P = upload_csr<T>(d->arena, P, false);
            D.R = upload_csr<T>(d->arena, R, false);
            if (smoother == PS_L1JAC) {
                std::vector<double> inv(dl1.size());
                for (size_t i = 0; i < dl1.size(); ++i) inv[i] = 1.0 / dl1[i];
                D.dinv = upload_vec<T>(d->arena, inv);
            } else {
                D.c0 = upload_vec<T>(d->arena, c0);
                D.c1 = upload_vec<T>(d->arena, c1);
                D.cm = upload_vec<T>(d->arena, cm);
            }
            continue;
        }
        D.n = L.A.n;
        D.A = upload_csr<T>(d->arena, L.A, true);
        D.P = upload_csr<T>(d->arena, L.P, false);
        D.R = upload_csr<T>(d->arena, L.R, false);
        if (smoother == PS_L1JAC) {
            std::vector<double> inv(L.dl1.size());
            for (size_t i = 0; i < L.dl1.size(); ++i) inv[i] = 1.0 / L.dl1[i];
            D.dinv = upload_vec<T>(d->arena, inv);
        } else {
            D.c0 = upload_vec<T>(d->arena, L.c0);
            D.c1 = upload_vec<T>(d->arena, L.c1);
            D.cm = upload_vec<T>(d->arena, L.cm);
        }
    }
    d->lev[nl - 1].n = H.coarse_n;
    d->cn = H.coarse_n;
    d->cinv = d->arena.upload(H.coarse_inv.data(), H.coarse_inv.size());
}

template <typename T>
std::unique_ptr<DHierarchy<T>> upload_hierarchy(const Hierarchy &H, int smoother, bool interleave3) {
    auto d = std::make_unique<DHierarchy<T>>();
    upload_hierarchy_into(*d, H, smoother, interleave3);
    return d;
}

static bool keep_lower(int row, int col) { return col < row; }
static bool keep_upper(int row, int col) { return col > row; }

void *Staging::get(size_t n) {
    if (n > bytes) {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        PS_HIP(hipHostMalloc(&p, n, hipHostMallocDefault));
        bytes = n;
    }
    return p;
}

hipStream_t Staging::stream() {
    if (!st) PS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    return st;
}

void Staging::copy_async(void *dev, const void *host, size_t n) {
    if (n) PS_HIP(hipMemcpyAsync(dev, host, n, hipMemcpyHostToDevice, stream()));
}

void Staging::wait() {
    if (st) PS_HIP(hipStreamSynchronize(st));
}

void Staging::copy_to_device(void *dev, const void *host, size_t n) {
    copy_async(dev, host, n);
    wait();
}

Staging::~Staging() {
    if (st) (void)hipStreamDestroy(st);
    if (p) (void)hipHostFree(p);
}

// Scatter block values into the SELL slot layout (src: source block per slot lane),
// converting to T, in a pinned buffer, then copy to the device array.
template <typename T>
static void upload_values(T *dev, const std::vector<int> &src, int rc, const std::vector<double> &v,
                          Staging &stg) {
    size_t nslots = src.size() / 64;
    if (nslots == 0) return;
    T *out = static_cast<T *>(stg.get(nslots * 64 * rc * sizeof(T)));
    parallel_for((int)nslots, [&](int b, int e, int) {
        for (int s = b; s < e; ++s)
            for (int l = 0; l < 64; ++l) {
                int t = src[(size_t)s * 64 + l];
                for (int q = 0; q < rc; ++q)
                    out[((size_t)s * rc + q) * 64 + l] = t < 0 ? T(0) : (T)v[(size_t)t * rc + q];
            }
    });
    stg.copy_to_device(dev, out, nslots * 64 * rc * sizeof(T));
}

template <typename T>
static void upload_dense(T *dev, const std::vector<double> &v, Staging &stg) {
    if (v.empty()) return;
    T *out = static_cast<T *>(stg.get(v.size() * sizeof(T)));
    parallel_for((int)v.size(), [&](int b, int e, int) {
        for (int i = b; i < e; ++i) out[i] = (T)v[i];
    });
    stg.copy_to_device(dev, out, v.size() * sizeof(T));
}

template <typename T>
static Sell<T> layout_sell(Arena &ar, const HostSell &h, T *&val, std::vector<int> &src) {
    Sell<T> s;
    s.nrows = h.nrows;
    s.nchunks = h.nchunks;
    s.br = h.br;
    s.bc = h.bc;
    s.nslots = h.cptr.empty() ? 0 : (size_t)h.cptr.back();
    s.cptr = ar.upload(h.cptr.data(), h.cptr.size());
    s.col = ar.upload(h.col.data(), h.col.size());
    if (!h.rowmap.empty()) s.rowmap = ar.upload(h.rowmap.data(), h.rowmap.size());
    val = ar.template alloc<T>(s.nslots * 64 * h.br * h.bc);
    s.val = val;
    src = h.src;
    return s;
}

// Scatter block values into an ELL layout val[(s*rc + q)*N + r] (src[s*N + r]: source block).
template <typename T>
static void scatter_ell(T *out, const std::vector<int> &src, int W, int N, int rc, const std::vector<double> &v) {
    parallel_for(N, [&](int b, int e, int) {
        for (int r = b; r < e; ++r)             // a block's rc values are read together
            for (int s = 0; s < W; ++s) {
                const int t = src[(size_t)s * N + r];
                for (int q = 0; q < rc; ++q)
                    out[((size_t)s * rc + q) * N + r] = t < 0 ? T(0) : (T)v[(size_t)t * rc + q];
            }
    });
}

// PS_BILU_FACTOR=host keeps the local-stage factorization on the host at every setup.
static bool device_factor_off() {
    const char *e = std::getenv("PS_BILU_FACTOR");
    return e && std::string(e) == "host";
}

static bool bilu_levels_forced() {
    const char *e = std::getenv("PS_BILU_LAUNCH");
    return e && (std::string(e) == "levels" || std::string(e) == "1wg");
}

// Layout of the subdomain-resident BILU(0) kernel, built once per handle from the
// factor's pattern (restricted to subdomains) and its level schedule.  Returns false
// (and the per-level kernels are used) when a subdomain's vector does not fit in LDS
// or a row has more than 8 blocks on one side of the diagonal.
template <typename T>
static bool layout_sub_bilu(DFlow<T> &d, const FlowSetup &f, const System &s) {
    if (s.ml_part.empty() || bilu_levels_forced()) return false;
    const int N = s.n_cells, nf = s.nf;
    const Bsr &F = f.ml;
    const BiluSchedule &sc = f.sched;
    // dense subdomain ids in increasing order of the caller's ids
    std::vector<int> ids(s.ml_part.begin(), s.ml_part.end());
    std::sort(ids.begin(), ids.end());
    ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
    const int D = (int)ids.size();
    std::vector<int> sid(N);
    for (int i = 0; i < N; ++i) sid[i] = (int)(std::lower_bound(ids.begin(), ids.end(), s.ml_part[i]) - ids.begin());
    std::vector<int> size(D, 0);
    for (int i = 0; i < N; ++i) ++size[sid[i]];
    int nmax = *std::max_element(size.begin(), size.end());
    int dev = 0, lds_max = 0;
    PS_HIP(hipGetDevice(&dev));
    PS_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // per-subdomain rows in level order, with level boundaries
    auto group = [&](const std::vector<int> &ptr, const std::vector<int> &rows, std::vector<int> &order,
                     std::vector<int> &lev, std::vector<int> &lev_off, int &maxw) {
        std::vector<std::vector<int>> r(D), b(D);
        std::vector<int> last(D, -1);
        for (size_t l = 0; l + 1 < ptr.size(); ++l)
            for (int q = ptr[l]; q < ptr[l + 1]; ++q) {
                int i = rows[q], g = sid[i];
                if (last[g] != (int)l) {
                    b[g].push_back((int)r[g].size());
                    last[g] = (int)l;
                }
                r[g].push_back(i);
            }
        order.clear();
        lev.clear();
        lev_off.assign(D + 1, 0);
        maxw = 0;
        for (int g = 0; g < D; ++g) {
            int base = (int)order.size();
            b[g].push_back((int)r[g].size());
            for (size_t k = 0; k < b[g].size(); ++k) {
                lev.push_back(base + b[g][k]);
                if (k + 1 < b[g].size()) maxw = std::max(maxw, b[g][k + 1] - b[g][k]);
            }
            lev_off[g + 1] = (int)lev.size();
            order.insert(order.end(), r[g].begin(), r[g].end());
        }
    };
    std::vector<int> ford, flev, flev_off, bord, blev, blev_off;
    int wf = 0, wb = 0;
    group(sc.fwd_ptr, sc.fwd_rows, ford, flev, flev_off, wf);
    group(sc.bwd_ptr, sc.bwd_rows, bord, blev, blev_off, wb);
    std::vector<int> sub_off(D + 1, 0);
    for (int g = 0; g < D; ++g) sub_off[g + 1] = sub_off[g] + size[g];
    std::vector<int> lpos(N);
    for (int r = 0; r < N; ++r) lpos[ford[r]] = r - sub_off[sid[ford[r]]];
    int W = 0;
    for (int i = 0; i < N; ++i) {
        int lo = 0, hi = 0;
        for (int t = F.rp[i]; t < F.rp[i + 1]; ++t) {
            if (F.ci[t] < i) ++lo;
            if (F.ci[t] > i) ++hi;
        }
        W = std::max(W, std::max(lo, hi));
    }
    if (W > 8) return false;
    W = W <= 3 ? 3 : 8;        // 3: seven-point cell stencil
    int lev_cap = 0;
    for (int g = 0; g < D; ++g)
        lev_cap = std::max(lev_cap, std::max(flev_off[g + 1] - flev_off[g], blev_off[g + 1] - blev_off[g]));
    lev_cap = (lev_cap + 3) / 4 * 4;
    size_t lds_lev = (size_t)2 * lev_cap * sizeof(int);
    size_t lds_vec = (size_t)(nmax + 1) * nf * sizeof(T);        // + one dummy row
    if (lds_lev > (size_t)lds_max / 2) return false;
    const bool vec_in_lds = lds_lev + lds_vec <= (size_t)lds_max;
    SubBilu<T> &b = d.sb;
    b.N = N;
    b.nsub = D;
    b.W = W;
    b.lev_cap = lev_cap;
    b.lds = lds_lev + (vec_in_lds ? lds_vec : 0);
    b.bs = std::min(512, std::max(256, (std::max(wf, wb) + 63) / 64 * 64));
    std::vector<int> fcol((size_t)W * N, -1), bcol((size_t)W * N, -1), bpos(N), dsrc(N, -1);
    b.fsrc.assign((size_t)W * N, -1);
    b.bsrc.assign((size_t)W * N, -1);
    for (int r = 0; r < N; ++r) {
        int i = ford[r], k = 0;
        for (int t = F.rp[i]; t < F.rp[i + 1] && F.ci[t] < i; ++t, ++k) {
            fcol[(size_t)k * N + r] = lpos[F.ci[t]];
            b.fsrc[(size_t)k * N + r] = t;
        }
        i = bord[r];
        bpos[r] = lpos[i];
        k = 0;
        for (int t = F.rp[i]; t < F.rp[i + 1]; ++t) {
            if (F.ci[t] == i) dsrc[r] = t;
            if (F.ci[t] <= i) continue;
            bcol[(size_t)k * N + r] = lpos[F.ci[t]];
            b.bsrc[(size_t)k * N + r] = t;
            ++k;
        }
    }
    b.dsrc = dsrc;
    b.ford = ford;
    {
        // stored blocks (values + column) of both sweeps, D^{-1}, and the vectors
        // (rhs read, z_s/z_p read, z written)
        size_t nblk = 0;
        for (int v : b.fsrc) nblk += v >= 0;
        for (int v : b.bsrc) nblk += v >= 0;
        b.bytes = (double)nblk * (nf * nf * sizeof(T) + 4) + (double)N * nf * nf * sizeof(T) + 3.0 * N * nf * sizeof(T);
    }
    std::vector<int> ncell(N), npos(N);
    for (int g = 0; g < D; ++g) {
        std::vector<int> cells(ford.begin() + sub_off[g], ford.begin() + sub_off[g + 1]);
        std::sort(cells.begin(), cells.end());
        for (int j = 0; j < size[g]; ++j) {
            ncell[sub_off[g] + j] = cells[j];
            npos[sub_off[g] + j] = lpos[cells[j]];
        }
    }
    // every index the kernel forms must stay inside its subdomain and its arrays
    auto check = [](bool ok, const char *what) {
        if (!ok) throw Error(PS_EDEVICE, std::string("subdomain BILU layout: ") + what);
    };
    check((int)flev_off.size() == D + 1 && (int)blev_off.size() == D + 1, "offset arrays");
    for (int g = 0; g < D; ++g) {
        for (auto *lv : {&flev_off, &blev_off}) {
            const std::vector<int> &lev = lv == &flev_off ? flev : blev;
            int a = (*lv)[g], z = (*lv)[g + 1];
            check(z > a && z <= (int)lev.size(), "level offsets");
            check(lev[a] == sub_off[g] && lev[z - 1] == sub_off[g + 1], "level bounds");
            for (int l = a; l + 1 < z; ++l) check(lev[l] < lev[l + 1], "empty level");
        }
        for (int r = sub_off[g]; r < sub_off[g + 1]; ++r) {
            check(bpos[r] >= 0 && bpos[r] < size[g], "bpos");
            check(ncell[r] >= 0 && ncell[r] < N && npos[r] >= 0 && npos[r] < size[g], "cell maps");
            for (int k = 0; k < W; ++k) {
                int fc = fcol[(size_t)k * N + r], bc = bcol[(size_t)k * N + r];
                check(fc >= -1 && fc < size[g] && bc >= -1 && bc < size[g], "column positions");
            }
        }
    }
    Arena &ar = d.arena;
    b.sub_off = ar.upload(sub_off.data(), sub_off.size());
    b.flev_off = ar.upload(flev_off.data(), flev_off.size());
    b.blev_off = ar.upload(blev_off.data(), blev_off.size());
    b.flev = ar.upload(flev.data(), flev.size());
    b.blev = ar.upload(blev.data(), blev.size());
    b.bpos = ar.upload(bpos.data(), bpos.size());
    b.ncell = ar.upload(ncell.data(), ncell.size());
    b.npos = ar.upload(npos.data(), npos.size());
    b.fcol = ar.upload(fcol.data(), fcol.size());
    b.bcol = ar.upload(bcol.data(), bcol.size());
    b.fval = ar.template alloc<T>((size_t)W * nf * nf * N);
    b.bval = ar.template alloc<T>((size_t)W * nf * nf * N);
    b.bdinv = ar.template alloc<T>((size_t)nf * nf * N);
    b.ygl = vec_in_lds ? nullptr : ar.template alloc<T>((size_t)nf * (N + D));   // + one dummy row each
    return true;
}

// Tables of the device BILU(0) factorization (pattern only, built once): hs is the SELL
// layout shared by S_ff and the system's A_ff.  Returns false (the host factors) when a
// factor block has no A_ff position or a table would not fit 32-bit indices.
template <typename T>
static bool layout_sub_factor(DFlow<T> &d, const FlowSetup &f, const HostSell &hs) {
    SubBilu<T> &b = d.sb;
    const Bsr &F = f.ml, &S = f.Sff;
    const int N = F.nbr, nn = F.br * F.bc, W = b.W;
    const int nml = F.rp[N];
    if ((size_t)hs.cptr.back() * nn * 64 >= (size_t)1 << 31 || (size_t)W * W * N >= (size_t)1 << 31) return false;
    std::vector<int> ml_src(nml, -1), ml_fs(nml, -1), dpos(N, -1);
    for (int i = 0; i < N; ++i) {
        const int ch = i >> 6, lane = i & 63;
        int tm = F.rp[i];
        for (int ts = S.rp[i]; ts < S.rp[i + 1] && tm < F.rp[i + 1]; ++ts) {
            if (F.ci[tm] != S.ci[ts]) continue;                  // dropped: another subdomain
            const size_t slot = (size_t)hs.cptr[ch] + (ts - S.rp[i]);
            ml_src[tm] = (int)(slot * nn * 64 + lane);
            if (F.ci[tm] == i) {
                ml_fs[tm] = i;
                dpos[i] = tm;
            }
            ++tm;
        }
        if (tm != F.rp[i + 1] || dpos[i] < 0) return false;
    }
    std::vector<int> fdiag(N), lo_t((size_t)W * N, -1), lo_d((size_t)W * N, -1), up_u((size_t)W * W * N, -1),
        up_q((size_t)W * W * N, -1);
    for (int r = 0; r < N; ++r) {
        const int i = b.ford[r];
        fdiag[r] = dpos[i];
        int k = 0;
        for (int t = F.rp[i]; t < F.rp[i + 1] && F.ci[t] < i; ++t, ++k) {
            if (k >= W) return false;
            const int kc = F.ci[t];
            lo_t[(size_t)k * N + r] = t;
            lo_d[(size_t)k * N + r] = dpos[kc];
            int m = 0;
            for (int u = dpos[kc] + 1; u < F.rp[kc + 1]; ++u) {
                int q = -1;
                for (int x = F.rp[i]; x < F.rp[i + 1]; ++x)
                    if (F.ci[x] == F.ci[u]) q = x;
                if (q < 0) continue;
                if (m >= W) return false;
                up_u[((size_t)k * W + m) * N + r] = u;
                up_q[((size_t)k * W + m) * N + r] = q;
                ++m;
            }
        }
    }
    Arena &ar = d.arena;
    b.nml = nml;
    b.ml_src = ar.upload(ml_src.data(), ml_src.size());
    b.ml_fs = ar.upload(ml_fs.data(), ml_fs.size());
    b.fdiag = ar.upload(fdiag.data(), fdiag.size());
    b.lo_t = ar.upload(lo_t.data(), lo_t.size());
    b.lo_d = ar.upload(lo_d.data(), lo_d.size());
    b.up_u = ar.upload(up_u.data(), up_u.size());
    b.up_q = ar.upload(up_q.data(), up_q.size());
    b.d_fsrc = ar.upload(b.fsrc.data(), b.fsrc.size());
    b.d_bsrc = ar.upload(b.bsrc.data(), b.bsrc.size());
    b.d_dsrc = ar.upload(b.dsrc.data(), b.dsrc.size());
    b.fv = ar.template alloc<double>((size_t)nml * nn);
    b.flag = ar.template alloc<int>(1);
    b.dev_factor = true;
    return true;
}

// The local-stage factor on st from A_ff and the fixed-stress terms in d.d_fs (uploaded on
// st before), then the sweeps' value planes in T.
template <int NF, int W, typename T>
static void factor_sub_device(DFlow<T> &d, const DSystem &S, Staging &stg) {
    SubBilu<T> &b = d.sb;
    constexpr int NN = NF * NF;
    const hipStream_t st = stg.stream();
    const size_t nsp = (size_t)d.nc * (NF - 1);
    k::SubFactorLayout F{b.N, b.nml, b.ml_src, b.ml_fs, b.fdiag, b.lo_t, b.lo_d, b.up_u, b.up_q};
    k::SubLayout L{b.N, b.sub_off, b.flev_off, b.blev_off, b.flev, b.blev, b.bpos, b.ncell, b.npos, b.fcol, b.bcol};
    LAUNCH((k::fill<int>), 1, 0, st, b.flag, 0, (size_t)1);
    LAUNCH((k::sub_factor_init<NF>), grid_for((size_t)b.nml), 0, st, F, (const double *)S.Aff.val,
           (const double *)d.d_fs, (const double *)d.d_fs + nsp, b.fv);
    hipLaunchKernelGGL((k::sub_factor<NF, W>), dim3(b.nsub), dim3(b.bs), 0, st, L, F, b.fv, b.flag);
    PS_HIP(hipGetLastError());
    LAUNCH((k::sub_factor_out<NN, T>), grid_for((size_t)W * b.N), 0, st, b.N, W, b.d_fsrc, (const double *)b.fv, b.fval);
    LAUNCH((k::sub_factor_out<NN, T>), grid_for((size_t)W * b.N), 0, st, b.N, W, b.d_bsrc, (const double *)b.fv, b.bval);
    LAUNCH((k::sub_factor_out<NN, T>), grid_for((size_t)b.N), 0, st, b.N, 1, b.d_dsrc, (const double *)b.fv, b.bdinv);
    int *h = static_cast<int *>(stg.get(sizeof(int)));
    PS_HIP(hipMemcpyAsync(h, b.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    PS_HIP(hipStreamSynchronize(st));
    if (*h) throw Error(PS_ESINGULAR, "singular BILU(0) pivot block");
}

// A level matrix of the device-built pressure hierarchy as a kernel operand: index arrays
// shared, values shared (FP64) or converted (FP32).
// w: slice widths of an operator A (which may then take SELL-64, built on the device), or
// null for P and R.
template <typename T>
static DCsr<T> adopt_csr(Arena &ar, const DevCsr &c, const int *w) {
    DCsr<T> d;
    d.n = c.n;
    d.nnz = c.nnz;
    d.G = lanes_per_row(c.n, c.nnz);
    d.rp = c.rp;
    if (w && c.n && take_sell(sell_padding(w, c.n, c.nnz), c.n, c.nnz)) {
        const int ns = (c.n + 63) / 64;
        std::vector<int> cptr(ns + 1, 0);
        for (int s = 0; s < ns; ++s) cptr[s + 1] = cptr[s] + w[s];
        const size_t slots = (size_t)cptr[ns] * 64;
        int *sci = ar.template alloc<int>(slots);
        T *sv = ar.template alloc<T>(slots);
        const int *dcp = ar.upload(cptr.data(), cptr.size());
        LAUNCH((k::csr_to_sell<T>), grid_for((size_t)c.n), 0, 0, c.rp, c.ci, c.v, c.n, dcp, sci, sv);
        d.G = 0;
        d.cptr = dcp;
        d.ci = sci;
        d.v = sv;
        return d;
    }
    d.ci = c.ci;
    if constexpr (sizeof(T) == 8) {
        d.v = c.v;
    } else {
        T *v = ar.template alloc<T>(c.nnz);
        LAUNCH((k::convert<double, T>), grid_for((size_t)c.nnz), 0, 0, c.v, v, (size_t)c.nnz);
        d.v = v;
    }
    return d;
}

template <typename T>
static void adopt_hierarchy(DHierarchy<T> &d, const Hierarchy &H, const PresStore &S, int smoother) {
    d.arena.recycle();
    d.smoother = smoother;
    const int nl = (int)H.lev.size();
    if ((int)S.A.size() != nl || (int)S.P.size() != nl - 1) throw Error(PS_EDEVICE, "pressure hierarchy mismatch");
    d.lev.assign(nl, DLevel<T>());
    // slice widths of every level operator, in one copy to the host
    std::vector<size_t> woff(nl, 0);
    size_t nw = 0;
    for (int l = 0; l + 1 < nl; ++l) {
        woff[l] = nw;
        nw += ((size_t)S.A[l].n + 63) / 64;
    }
    std::vector<int> hw(nw);
    if (nw) {
        int *dw = d.arena.template alloc<int>(nw);
        for (int l = 0; l + 1 < nl; ++l)
            LAUNCH(k::slice_width, grid_for(((size_t)S.A[l].n + 63) / 64), 0, 0, S.A[l].rp, S.A[l].n, dw + woff[l]);
        PS_HIP(hipMemcpy(hw.data(), dw, nw * sizeof(int), hipMemcpyDeviceToHost));
    }
    for (int l = 0; l + 1 < nl; ++l) {
        const Level &L = H.lev[l];
        DLevel<T> &D = d.lev[l];
        D.n = L.A.n;
        D.A = adopt_csr<T>(d.arena, S.A[l], hw.data() + woff[l]);
        D.P = adopt_csr<T>(d.arena, S.P[l], nullptr);
        D.R = adopt_csr<T>(d.arena, S.R[l], nullptr);
        if (S.on_device) {
            if constexpr (sizeof(T) == 8) {
                D.dinv = S.dinv[l];
            } else {
                T *v = d.arena.template alloc<T>(D.n);
                LAUNCH((k::convert<double, T>), grid_for((size_t)D.n), 0, 0, (const double *)S.dinv[l], v,
                       (size_t)D.n);
                D.dinv = v;
            }
        } else if (smoother == PS_L1JAC) {
            std::vector<double> inv(L.dl1.size());
            for (size_t i = 0; i < L.dl1.size(); ++i) inv[i] = 1.0 / L.dl1[i];
            D.dinv = upload_vec<T>(d.arena, inv);
        } else {
            D.c0 = upload_vec<T>(d.arena, L.c0);
            D.c1 = upload_vec<T>(d.arena, L.c1);
            D.cm = upload_vec<T>(d.arena, L.cm);
        }
    }
    d.lev[nl - 1].n = H.coarse_n;
    d.cn = H.coarse_n;
    d.cinv = S.cinv ? S.cinv : d.arena.upload(H.coarse_inv.data(), H.coarse_inv.size());
    PS_HIP(hipStreamSynchronize(0));
}

template <typename T>
void update_flow_values(DFlow<T> &d, const FlowSetup &f, const System &s, const DSystem &S, const Options &o,
                        Staging &stg, bool afu_changed, bool factor_on_device, bool operators_on_device) {
    const int nf = s.nf, nc = s.n_cells, nn = nf * nf;
    static const std::vector<double> none;
    if (!d.layout) {
        d.nc = nc;
        d.nf = nf;
        d.ml_kind = o.ml_kind;
        d.ml_sweeps = o.ml_sweeps;
        d.Afu = layout_sell<T>(d.arena, sell_from_bsr(s.Afu.rp, s.Afu.ci, none, nc, nf, 3, nullptr, nullptr, false),
                               d.afu_val, d.src_afu);
        {
            HostSell hs = sell_from_bsr(f.Sff.rp, f.Sff.ci, none, nc, nf, nf, nullptr, nullptr, false);
            d.Sff = layout_sell<T>(d.arena, hs, d.sff_val, d.src_sff);
            // S_ff is formed on the device from A_ff when both have the same SELL layout
            if (S.Aff.nchunks == hs.nchunks && S.Aff.nslots == d.Sff.nslots && f.Sff.rp == s.Aff.rp &&
                f.Sff.ci == s.Aff.ci) {
                std::vector<int> dslot((size_t)hs.nchunks * 64, -1);
                for (int i = 0; i < nc; ++i) {
                    const int ch = i >> 6, lane = i & 63;
                    for (int k = hs.cptr[ch]; k < hs.cptr[ch + 1]; ++k) {
                        const int t = hs.src[(size_t)k * 64 + lane];
                        if (t >= 0 && f.Sff.ci[t] == i) {
                            dslot[i] = k - hs.cptr[ch];
                            break;
                        }
                    }
                }
                d.sff_dslot = d.arena.upload(dslot.data(), dslot.size());
                d.d_fs = d.arena.template alloc<double>((size_t)nc * nf);
            }
        }
        auto order = [&](const std::vector<int> &ptr, const std::vector<int> &rows, std::vector<int> &lchunk) {
            std::vector<int> ord;
            lchunk.assign(1, 0);
            for (size_t l = 0; l + 1 < ptr.size(); ++l) {
                for (int p = ptr[l]; p < ptr[l + 1]; ++p) ord.push_back(rows[p]);
                while (ord.size() % 64) ord.push_back(-1);
                lchunk.push_back((int)(ord.size() / 64));
            }
            return ord;
        };
        if (o.ml_kind == PS_BILU0 && layout_sub_bilu(d, f, s)) {
            d.sub = true;
            if (d.sff_dslot && !device_factor_off()) {
                HostSell hs = sell_from_bsr(f.Sff.rp, f.Sff.ci, none, nc, nf, nf, nullptr, nullptr, false);
                layout_sub_factor(d, f, hs);
            }
        } else if (o.ml_kind == PS_BILU0) {
            std::vector<int> of = order(f.sched.fwd_ptr, f.sched.fwd_rows, d.lchunk_f);
            std::vector<int> ob = order(f.sched.bwd_ptr, f.sched.bwd_rows, d.lchunk_b);
            d.Lf = layout_sell<T>(d.arena, sell_from_bsr(f.ml.rp, f.ml.ci, none, nc, nf, nf, &of, keep_lower, false),
                                  d.lf_val, d.src_lf);
            d.Ub = layout_sell<T>(d.arena, sell_from_bsr(f.ml.rp, f.ml.ci, none, nc, nf, nf, &ob, keep_upper, false),
                                  d.ub_val, d.src_ub);
            d.d_lchunk_f = d.arena.upload(d.lchunk_f.data(), d.lchunk_f.size());
            d.d_lchunk_b = d.arena.upload(d.lchunk_b.data(), d.lchunk_b.size());
        } else if (o.ml_kind == PS_MCGS) {
            std::vector<int> oc = order(f.sched.fwd_ptr, f.sched.fwd_rows, d.lchunk_f);
            d.Lf = layout_sell<T>(d.arena, sell_from_bsr(f.Sff.rp, f.Sff.ci, none, nc, nf, nf, &oc, nullptr, false),
                                  d.lf_val, d.src_lf);
        }
        d.dss_inv = d.arena.template alloc<T>(f.dss_inv.size());
        d.dinv = d.arena.template alloc<T>((size_t)nc * nn);
        d.pres = std::make_unique<DHierarchy<T>>();
        d.pres->ktag = ktime::PRES_PRE;
        d.layout = true;
        afu_changed = true;
    }
    {
        TraceTick tt("values A_fu, S_ff, D_ss");
        if (afu_changed) upload_values(d.afu_val, d.src_afu, nf * 3, s.Afu.v, stg);
        if (d.sff_dslot) {
            const size_t nsp = (size_t)nc * (nf - 1);
            double *h = static_cast<double *>(stg.get((size_t)nc * nf * sizeof(double)));
            std::memcpy(h, s.d_sp.data(), nsp * sizeof(double));
            std::memcpy(h + nsp, s.d_pp.data(), (size_t)nc * sizeof(double));
            stg.copy_to_device(d.d_fs, h, (size_t)nc * nf * sizeof(double));
            const unsigned g = grid_for((size_t)S.Aff.nchunks * 64);
            if (nf == 2)
                LAUNCH((k::sff_from_aff<2, T>), g, 0, stg.stream(), S.Aff, (const double *)d.d_fs,
                       (const double *)d.d_fs + nsp, d.sff_dslot, d.sff_val);
            else
                LAUNCH((k::sff_from_aff<3, T>), g, 0, stg.stream(), S.Aff, (const double *)d.d_fs,
                       (const double *)d.d_fs + nsp, d.sff_dslot, d.sff_val);
            stg.wait();
        } else {
            upload_values(d.sff_val, d.src_sff, nn, f.Sff.v, stg);
        }
        if (operators_on_device) {
            if (!d.sff_dslot) throw Error(PS_EDEVICE, "no device S_ff layout");
            dss_inverse_device<T>(S, d.sff_dslot, d.dss_inv, stg.stream());
            stg.wait();
        } else {
            upload_dense(d.dss_inv, f.dss_inv, stg);
        }
    }
    std::vector<double> dinv((size_t)nc * nn);
    if (d.sub) {
        const SubBilu<T> &b = d.sb;
        if (factor_on_device) {
            if (!b.dev_factor) throw Error(PS_EDEVICE, "no device BILU(0) layout");
            TraceTick tt("factor subdomain BILU");
            if (nf == 2 && b.W == 3) factor_sub_device<2, 3, T>(d, S, stg);
            else if (nf == 2) factor_sub_device<2, 8, T>(d, S, stg);
            else if (b.W == 3) factor_sub_device<3, 3, T>(d, S, stg);
            else factor_sub_device<3, 8, T>(d, S, stg);
        } else {
            // each array is copied while the next one is scattered
            TraceTick tt("values subdomain BILU");
            const size_t ne = (size_t)b.W * nn * nc, nd = (size_t)nn * nc;
            T *out = static_cast<T *>(stg.get((2 * ne + nd) * sizeof(T)));
            scatter_ell(out, b.fsrc, b.W, nc, nn, f.ml.v);
            stg.copy_async(b.fval, out, ne * sizeof(T));
            scatter_ell(out + ne, b.bsrc, b.W, nc, nn, f.ml.v);
            stg.copy_async(b.bval, out + ne, ne * sizeof(T));
            scatter_ell(out + 2 * ne, b.dsrc, 1, nc, nn, f.ml.v);
            stg.copy_async(b.bdinv, out + 2 * ne, nd * sizeof(T));
            stg.wait();
        }
        dinv.clear();
    } else if (o.ml_kind == PS_BILU0) {
        upload_values(d.lf_val, d.src_lf, nn, f.ml.v, stg);
        upload_values(d.ub_val, d.src_ub, nn, f.ml.v, stg);
        parallel_for(nc, [&](int b, int e, int) {
            for (int i = b; i < e; ++i)
                for (int t = f.ml.rp[i]; t < f.ml.rp[i + 1]; ++t)
                    if (f.ml.ci[t] == i) std::memcpy(&dinv[(size_t)i * nn], &f.ml.v[(size_t)t * nn], sizeof(double) * nn);
        });
    } else {
        if (o.ml_kind == PS_MCGS) upload_values(d.lf_val, d.src_lf, nn, f.Sff.v, stg);
        dinv = f.ml.v;
    }
    if (!dinv.empty()) upload_dense(d.dinv, dinv, stg);
}

template <typename T>
void update_flow_pressure(DFlow<T> &d, const FlowSetup &f, const Options &o, const PresStore *ps) {
    TraceTick tt("pressure levels");
    if (ps) adopt_hierarchy(*d.pres, f.pres, *ps, o.smoother);
    else upload_hierarchy_into(*d.pres, f.pres, o.smoother, false);
}

void upload_system(const System &s, DSystem &d) {
    d.n_nodes = s.n_nodes;
    d.n_cells = s.n_cells;
    d.nf = s.nf;
    d.Auu = upload_sell<double>(d.arena, sell_from_bsr(s.Auu.rp, s.Auu.ci, s.Auu.v, s.n_nodes, 3, 3));
    {
        HostSell h = sell_from_bsr(s.Auf.rp, s.Auf.ci, s.Auf.v, s.n_nodes, 3, s.nf);
        d.Auf = upload_sell<double>(d.arena, h);
        d.src_auf = std::move(h.src);
    }
    {
        HostSell h = sell_from_bsr(s.Afu.rp, s.Afu.ci, s.Afu.v, s.n_cells, s.nf, 3);
        d.Afu = upload_sell<double>(d.arena, h);
        d.src_afu = std::move(h.src);
    }
    {
        HostSell h = sell_from_bsr(s.Aff.rp, s.Aff.ci, s.Aff.v, s.n_cells, s.nf, s.nf);
        d.Aff = upload_sell<double>(d.arena, h);
        d.src_aff = std::move(h.src);
    }
    auto blk = [](const Bsr &b) { return (double)b.nb() * (b.br * b.bc * 8 + 4) + 4.0 * b.rp.size(); };
    d.mat_bytes = blk(s.Auu) + blk(s.Auf) + blk(s.Afu) + blk(s.Aff);
}

void update_system_flow_values(const System &s, DSystem &d, Staging &stg, bool auf) {
    if (auf) upload_values(const_cast<double *>(d.Auf.val), d.src_auf, 3 * s.nf, s.Auf.v, stg);
    upload_values(const_cast<double *>(d.Afu.val), d.src_afu, s.nf * 3, s.Afu.v, stg);
    upload_values(const_cast<double *>(d.Aff.val), d.src_aff, s.nf * s.nf, s.Aff.v, stg);
}

template <typename T>
static void alloc_hier_work(HierWork<T> &w, const DHierarchy<T> &H, Arena &ar) {
    int nl = (int)H.lev.size();
    w.x.assign(nl, nullptr);
    w.x1.assign(nl, nullptr);
    w.d.assign(nl, nullptr);
    w.r.assign(nl, nullptr);
    w.b.assign(nl, nullptr);
    w.e.assign(nl, nullptr);
    for (int l = 0; l < nl; ++l) {
        size_t n = H.lev[l].n;
        if (l + 1 < nl) {
            w.x[l] = ar.template alloc<T>(n);
            w.x1[l] = ar.template alloc<T>(n);
            w.d[l] = ar.template alloc<T>(n);
            w.r[l] = ar.template alloc<T>(n);
        }
        if (l > 0) {
            w.b[l] = ar.template alloc<T>(n);
            w.e[l] = ar.template alloc<T>(n);
        }
    }
}

template <typename T>
void alloc_prec_work(PrecWork<T> &w, const DHierarchy<T> &sdc, const DFlow<T> &fl, int n_nodes) {
    if (!w.fixed) {
        alloc_hier_work(w.sdc, sdc, w.arena);
        size_t nfl = (size_t)fl.nc * fl.nf;
        if (sizeof(T) == 4) w.vconv = w.arena.template alloc<T>((size_t)3 * n_nodes);
        w.y = w.arena.template alloc<T>(nfl);
        w.zs = w.arena.template alloc<T>((size_t)fl.nc * (fl.nf - 1));
        w.wp = w.arena.template alloc<T>(fl.nc);
        w.zp = w.arena.template alloc<T>(fl.nc);
        w.w = w.arena.template alloc<T>(nfl);
        w.t = w.arena.template alloc<T>(nfl);
        w.dz = w.arena.template alloc<T>(nfl);
        w.r2 = w.arena.template alloc<T>(nfl);
        w.fixed = true;
    }
    w.pres_arena.recycle();
    alloc_hier_work(w.pres, *fl.pres, w.pres_arena);
}

// ------------------------------------------------------------------ V-cycle
// Calls f with a compile-time group width equal to G.
template <typename F>
static void with_G(int G, F &&f) {
    switch (G) {
    case -1: f(std::integral_constant<int, -1>{}); break;
    case 0: f(std::integral_constant<int, 0>{}); break;
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    case 32: f(std::integral_constant<int, 32>{}); break;
    case 65: f(std::integral_constant<int, 65>{}); break;
    case 66: f(std::integral_constant<int, 66>{}); break;
    case 68: f(std::integral_constant<int, 68>{}); break;
    case 72: f(std::integral_constant<int, 72>{}); break;
    case 80: f(std::integral_constant<int, 80>{}); break;
    case 96: f(std::integral_constant<int, 96>{}); break;
    default: throw Error(PS_EDEVICE, "level matrix layout");
    }
}

#define LAUNCHB(kernel, grid, nb, shm, st, ...)                                          \
    do {                                                                                 \
        if ((grid) > 0) hipLaunchKernelGGL(kernel, dim3(grid, nb), dim3(WG), shm, st, __VA_ARGS__); \
    } while (0)

// The solves whose V-cycles run in one sequence of launches on a shared hierarchy: their
// per-level work vectors.  A single solve is a batch of one.
template <typename T>
struct VBatch {
    int k = 1;
    HierWork<T> *W[k::MAXB] = {};
};

template <typename T>
static k::VP<T> one(T *p) {
    k::VP<T> v{};
    v.p[0] = p;
    return v;
}

// level l's vector `field` of every solve of the batch
template <typename T>
static k::VP<T> level_vec(const VBatch<T> &B, std::vector<T *> HierWork<T>::*field, int l) {
    k::VP<T> v{};
    for (int i = 0; i < B.k; ++i) v.p[i] = (B.W[i]->*field)[l];
    return v;
}

template <typename T>
static k::VP<const T> cvp(const k::VP<T> &v) {
    k::VP<const T> c{};
    for (int i = 0; i < k::MAXB; ++i) c.p[i] = v.p[i];
    return c;
}

template <int MODE, typename T>
static void csr_spmv(const DCsr<T> &A, k::VP<const T> x, k::VP<const T> b, k::VP<T> y, int nb, hipStream_t st) {
    with_G(A.G, [&](auto Gc) {
        constexpr int G = decltype(Gc)::value;
        LAUNCHB((k::csr_spmv<G, MODE, T>), grid_for((size_t)A.n * k::lanes_of<G>()), nb, 0, st, A, x, b, y);
    });
}

// Algorithmic bytes of one pass over a level operator: values and column indices of the
// stored entries (16-bit columns count 2 bytes), row pointers, and `vecs` vectors of the
// operator's row count (read or written once each; gathers counted once).
template <typename T>
static double op_bytes(const DCsr<T> &A, double vecs_rows, double vecs_cols = 0.0, double ncols = 0.0) {
    const double cb = A.cd ? 2.0 : 4.0;
    return (double)A.nnz * (sizeof(T) + cb) + 4.0 * (A.n + 1) + vecs_rows * A.n * sizeof(T) +
           vecs_cols * ncols * sizeof(T);
}

// One V(1,1)-cycle from level l for every solve of the batch B (right-hand sides b, results
// out): each launch covers the batch (gridDim.y = B.k), reading the level's operator once
// per slice and computing every slice with the single-solve arithmetic.
template <typename T>
static void vcycle(const DHierarchy<T> &H, const VBatch<T> &B, int l, k::VP<const T> b, k::VP<T> out,
                   hipStream_t st) {
    const int nb = B.k;
    const int last = (int)H.lev.size() - 1;
    if (l == last) {
        unsigned g = (unsigned)((H.cn + (WG / 64) - 1) / (WG / 64));
        LAUNCHB(k::coarse_solve<T>, g, nb, 0, st, H.cinv, H.cn, b, out);
        return;
    }
    const DLevel<T> &L = H.lev[l];
    const bool cheb = H.smoother == PS_CHEB2;
    const k::VP<T> x = level_vec(B, &HierWork<T>::x, l), r = level_vec(B, &HierWork<T>::r, l);
    // level 0 of a single solve is timed when kernel timing is on (ktag: the hierarchy's
    // first phase id)
    const int tag = l == 0 && nb == 1 ? H.ktag : -1;
    auto scope = [&](std::optional<ktime::Scope> &o, int phase, double bytes) {
        if (tag >= 0 && ktime::enabled()) o.emplace(tag + phase, st, bytes);
    };
    const int nc = H.lev[l + 1].n;
    {
        // l1-Jacobi: b, D^-1 (gathered) in, x and r out; Chebyshev: the first step (b, c0
        // gathered, c1, cm in, x out) and the residual (x, b in, r out)
        std::optional<ktime::Scope> ts;
        scope(ts, 0, cheb ? op_bytes(L.A, 5) + op_bytes(L.A, 3) : op_bytes(L.A, l > 0 ? 3 : 4));
        with_G(L.A.G, [&](auto Gc) {
            constexpr int G = decltype(Gc)::value;
            unsigned g = grid_for((size_t)L.n * k::lanes_of<G>());
            if (cheb) {
                LAUNCHB((k::csr_cheb_pre<G, T>), g, nb, 0, st, L.A, b, L.c0, L.c1, L.cm, x);
                LAUNCHB((k::csr_spmv<G, 1, T>), g, nb, 0, st, L.A, cvp(x), b, r);
            } else if (l > 0) {                 // x = D^-1 b was written with b by the restriction
                LAUNCHB((k::csr_spmv<G, 1, T>), g, nb, 0, st, L.A, cvp(x), b, r);
            } else {
                LAUNCHB((k::csr_l1_pre<G, T>), g, nb, 0, st, L.A, b, L.dinv, x, r);
            }
        });
    }
    const k::VP<T> bc = level_vec(B, &HierWork<T>::b, l + 1), ec = level_vec(B, &HierWork<T>::e, l + 1);
    if (!cheb && l + 1 < last) {
        // R r (r gathered) with the coarse level's D^-1 in, b and x = D^-1 b out
        std::optional<ktime::Scope> ts;
        scope(ts, 1, op_bytes(L.R, 3, 1, L.n));
        const k::VP<T> xc = level_vec(B, &HierWork<T>::x, l + 1);
        with_G(L.R.G, [&](auto Gc) {
            constexpr int G = decltype(Gc)::value;
            LAUNCHB((k::csr_restrict_l1<G, T>), grid_for((size_t)L.R.n * k::lanes_of<G>()), nb, 0, st, L.R, cvp(r),
                    H.lev[l + 1].dinv, bc, xc);
        });
    } else {
        std::optional<ktime::Scope> ts;
        scope(ts, 1, op_bytes(L.R, 1, 1, L.n));
        csr_spmv<0, T>(L.R, cvp(r), k::VP<const T>{}, bc, nb, st);
    }
    vcycle(H, B, l + 1, cvp(bc), ec, st);
    {
        std::optional<ktime::Scope> ts;
        scope(ts, 2, op_bytes(L.P, 2, 1, nc));             // e (gathered) in, x read and written
        csr_spmv<2, T>(L.P, cvp(ec), k::VP<const T>{}, x, nb, st);
    }
    // l1-Jacobi: b, x (gathered), D^-1 in, out written; Chebyshev: two sweeps (x, b, c0 in,
    // x1, d0 out; x1, b, d0, c1, cm in, out written)
    std::optional<ktime::Scope> ts;
    scope(ts, 3, cheb ? op_bytes(L.A, 5) + op_bytes(L.A, 6) : op_bytes(L.A, 4));
    with_G(L.A.G, [&](auto Gc) {
        constexpr int G = decltype(Gc)::value;
        unsigned g = grid_for((size_t)L.n * k::lanes_of<G>());
        if (cheb) {
            const k::VP<T> x1 = level_vec(B, &HierWork<T>::x1, l), d = level_vec(B, &HierWork<T>::d, l);
            LAUNCHB((k::csr_cheb_post1<G, T>), g, nb, 0, st, L.A, b, cvp(x), L.c0, x1, d);
            LAUNCHB((k::csr_cheb_post2<G, T>), g, nb, 0, st, L.A, b, cvp(x1), cvp(d), L.c1, L.cm, out);
        } else {
            LAUNCHB((k::csr_l1_post<G, T>), g, nb, 0, st, L.A, b, cvp(x), L.dinv, out);
        }
    });
}

template <typename T>
static void vcycle(const DHierarchy<T> &H, HierWork<T> &W, int l, const T *b, T *out, hipStream_t st) {
    VBatch<T> B;
    B.W[0] = &W;
    vcycle(H, B, l, one(b), one(out), st);
}

// ------------------------------------------------------------------ Algorithm 1
// BILU sweeps: one launch per level (default), or one workgroup walking all levels
// (PS_BILU_LAUNCH=1wg; measured slower on MI355X, kept for comparison).
static bool bilu_one_workgroup() {
    static const bool v = [] {
        const char *e = std::getenv("PS_BILU_LAUNCH");
        return e && std::string(e) == "1wg";
    }();
    return v;
}

template <int NF, int W, typename T, bool ACC, bool FINAL, bool GY>
static void launch_sub_y(const SubBilu<T> &b, const T *src, PrecWork<T> &w, T *zf, hipStream_t st) {
    auto kern = k::bilu_sub<NF, W, T, ACC, FINAL, GY>;
    if (b.lds > 65536) {
        // once per instantiation, also when several threads launch: allow the device's LDS maximum
        static std::once_flag raised;
        std::call_once(raised, [&] {
            int dev = 0, mx = 0;
            PS_HIP(hipGetDevice(&dev));
            PS_HIP(hipDeviceGetAttribute(&mx, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
            PS_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, mx));
        });
    }
    k::SubLayout L{b.N, b.sub_off, b.flev_off, b.blev_off, b.flev, b.blev, b.bpos, b.ncell, b.npos, b.fcol, b.bcol};
    ktime::Scope ts(ktime::BILU_SUB, st, b.bytes);
    hipLaunchKernelGGL(kern, dim3(b.nsub), dim3(b.bs), b.lds, st, L, (const T *)b.fval, (const T *)b.bval,
                       (const T *)b.bdinv, src, w.dz, (const T *)w.zs, (const T *)w.zp, zf, b.ygl, b.lev_cap);
}

template <int NF, int W, typename T, bool ACC, bool FINAL>
static void launch_sub(const SubBilu<T> &b, const T *src, PrecWork<T> &w, T *zf, hipStream_t st) {
    if (b.ygl) launch_sub_y<NF, W, T, ACC, FINAL, true>(b, src, w, zf, st);
    else launch_sub_y<NF, W, T, ACC, FINAL, false>(b, src, w, zf, st);
}

template <int NF, typename T>
static void local_stage(const DFlow<T> &fl, PrecWork<T> &w, T *zf, hipStream_t st) {
    const int sweeps = fl.ml_sweeps;
    unsigned g = grid_for(fl.nc);
    if (fl.ml_kind == PS_BJACOBI) {
        T *bufs[2] = {w.dz, w.r2};
        for (int s = 0; s < sweeps; ++s) {
            bool first = s == 0, final = s == sweeps - 1;
            const T *din = bufs[s & 1];
            T *dout = bufs[(s + 1) & 1];
            if (first && final)
                LAUNCH((k::bjacobi<NF, T, true, true>), g, 0, st, fl.Sff, w.w, fl.dinv, din, dout, w.zs, w.zp, zf);
            else if (first)
                LAUNCH((k::bjacobi<NF, T, true, false>), g, 0, st, fl.Sff, w.w, fl.dinv, din, dout, w.zs, w.zp, zf);
            else if (final)
                LAUNCH((k::bjacobi<NF, T, false, true>), g, 0, st, fl.Sff, w.w, fl.dinv, din, dout, w.zs, w.zp, zf);
            else
                LAUNCH((k::bjacobi<NF, T, false, false>), g, 0, st, fl.Sff, w.w, fl.dinv, din, dout, w.zs, w.zp, zf);
        }
        return;
    }
    if (fl.ml_kind == PS_MCGS) {
        LAUNCH((k::fill<T>), grid_for((size_t)fl.nc * NF), 0, st, w.dz, T(0), (size_t)fl.nc * NF);
        for (int s = 0; s < sweeps; ++s) {
            bool final = s == sweeps - 1;
            for (size_t c = 0; c + 1 < fl.lchunk_f.size(); ++c) {
                int p0 = fl.lchunk_f[c] * 64, p1 = fl.lchunk_f[c + 1] * 64;
                if (final)
                    LAUNCH((k::mcgs<NF, T, true>), grid_for(p1 - p0), 0, st, fl.Lf, p0, p1, (const T *)w.w,
                           fl.dinv, w.dz, w.zs, w.zp, zf);
                else
                    LAUNCH((k::mcgs<NF, T, false>), grid_for(p1 - p0), 0, st, fl.Lf, p0, p1, (const T *)w.w,
                           fl.dinv, w.dz, w.zs, w.zp, zf);
            }
        }
        return;
    }
    const bool one_wg = bilu_one_workgroup();
    for (int s = 0; s < sweeps; ++s) {
        const T *src = w.w;
        if (s > 0) {
            LAUNCH((k::spmv<NF, NF, T, T, T, 1>), g, 0, st, fl.Sff, (const T *)w.dz, (const T *)w.w, w.r2);
            src = w.r2;
        }
        if (fl.sub) {
            bool first = s == 0, final = s == sweeps - 1;
            if (fl.sb.W == 3) {
                if (first && final) launch_sub<NF, 3, T, false, true>(fl.sb, src, w, zf, st);
                else if (first) launch_sub<NF, 3, T, false, false>(fl.sb, src, w, zf, st);
                else if (final) launch_sub<NF, 3, T, true, true>(fl.sb, src, w, zf, st);
                else launch_sub<NF, 3, T, true, false>(fl.sb, src, w, zf, st);
            } else {
                if (first && final) launch_sub<NF, 8, T, false, true>(fl.sb, src, w, zf, st);
                else if (first) launch_sub<NF, 8, T, false, false>(fl.sb, src, w, zf, st);
                else if (final) launch_sub<NF, 8, T, true, true>(fl.sb, src, w, zf, st);
                else launch_sub<NF, 8, T, true, false>(fl.sb, src, w, zf, st);
            }
            continue;
        }
        if (one_wg) {
            bool final = s == sweeps - 1;
            int nlf = (int)fl.lchunk_f.size() - 1, nlb = (int)fl.lchunk_b.size() - 1;
            hipLaunchKernelGGL((k::bilu_fwd_1wg<NF, T>), dim3(1), dim3(k::WG1), 0, st, fl.Lf, fl.d_lchunk_f, nlf,
                               src, w.t);
            if (s == 0 && final)
                hipLaunchKernelGGL((k::bilu_bwd_1wg<NF, T, false, true>), dim3(1), dim3(k::WG1), 0, st, fl.Ub,
                                   fl.d_lchunk_b, nlb, w.t, fl.dinv, w.dz, w.zs, w.zp, zf);
            else if (s == 0)
                hipLaunchKernelGGL((k::bilu_bwd_1wg<NF, T, false, false>), dim3(1), dim3(k::WG1), 0, st, fl.Ub,
                                   fl.d_lchunk_b, nlb, w.t, fl.dinv, w.dz, w.zs, w.zp, zf);
            else if (final)
                hipLaunchKernelGGL((k::bilu_bwd_1wg<NF, T, true, true>), dim3(1), dim3(k::WG1), 0, st, fl.Ub,
                                   fl.d_lchunk_b, nlb, w.t, fl.dinv, w.dz, w.zs, w.zp, zf);
            else
                hipLaunchKernelGGL((k::bilu_bwd_1wg<NF, T, true, false>), dim3(1), dim3(k::WG1), 0, st, fl.Ub,
                                   fl.d_lchunk_b, nlb, w.t, fl.dinv, w.dz, w.zs, w.zp, zf);
            continue;
        }
        for (size_t l = 0; l + 1 < fl.lchunk_f.size(); ++l) {
            int p0 = fl.lchunk_f[l] * 64, p1 = fl.lchunk_f[l + 1] * 64;
            LAUNCH((k::bilu_fwd<NF, T>), grid_for(p1 - p0), 0, st, fl.Lf, p0, p1, src, w.t);
        }
        bool final = s == sweeps - 1;
        for (size_t l = 0; l + 1 < fl.lchunk_b.size(); ++l) {
            int p0 = fl.lchunk_b[l] * 64, p1 = fl.lchunk_b[l + 1] * 64;
            unsigned gl = grid_for(p1 - p0);
            if (s == 0 && final)
                LAUNCH((k::bilu_bwd<NF, T, false, true>), gl, 0, st, fl.Ub, p0, p1, w.t, fl.dinv, w.dz, w.zs, w.zp, zf);
            else if (s == 0)
                LAUNCH((k::bilu_bwd<NF, T, false, false>), gl, 0, st, fl.Ub, p0, p1, w.t, fl.dinv, w.dz, w.zs, w.zp, zf);
            else if (final)
                LAUNCH((k::bilu_bwd<NF, T, true, true>), gl, 0, st, fl.Ub, p0, p1, w.t, fl.dinv, w.dz, w.zs, w.zp, zf);
            else
                LAUNCH((k::bilu_bwd<NF, T, true, false>), gl, 0, st, fl.Ub, p0, p1, w.t, fl.dinv, w.dz, w.zs, w.zp, zf);
        }
    }
}

template <int NF, typename T>
static void flow_stage(const DFlow<T> &fl, PrecWork<T> &w, const double *vf, const T *zu, T *zf,
                       hipStream_t st) {
    unsigned g = grid_for(fl.nc);
    LAUNCH((k::step23<NF, T>), g, 0, st, fl.Afu, vf, zu, fl.dss_inv, w.y, w.zs);     // steps 2-3
    LAUNCH((k::step4<NF, T>), g, 0, st, fl.Sff, (const T *)w.y, (const T *)w.zs, w.wp); // step 4
    vcycle(*fl.pres, w.pres, 0, (const T *)w.wp, w.zp, st);                             // step 5
    LAUNCH((k::step6<NF, T>), g, 0, st, fl.Sff, (const T *)w.y, (const T *)w.zs, (const T *)w.zp, w.w);  // step 6
    local_stage<NF, T>(fl, w, zf, st);                                                 // steps 7-8
}

template <typename T>
const T *precond_pre(PrecWork<T> &w, int n_nodes, const double *v, hipStream_t st) {
    size_t nu = (size_t)3 * n_nodes;
    if constexpr (sizeof(T) == 4) {
        LAUNCH((k::convert<double, T>), grid_for(nu), 0, st, v, w.vconv, nu);
        return w.vconv;
    } else {
        return reinterpret_cast<const T *>(v);
    }
}

template <typename T>
void precond_post(const DFlow<T> &fl, PrecWork<T> &w, int n_nodes, const double *v, T *z, hipStream_t st) {
    size_t nu = (size_t)3 * n_nodes;
    if (fl.nf == 2) flow_stage<2, T>(fl, w, v + nu, z, z + nu, st);
    else flow_stage<3, T>(fl, w, v + nu, z, z + nu, st);
}

template <typename T>
void apply_precond(const DHierarchy<T> &sdc, const DFlow<T> &fl, PrecWork<T> &w, int n_nodes,
                   const double *v, T *z, hipStream_t st) {
    const T *vu = precond_pre(w, n_nodes, v, st);
    vcycle(sdc, w.sdc, 0, vu, z, st);                                                  // step 1
    precond_post(fl, w, n_nodes, v, z, st);                                            // steps 2-8
}

static_assert(kBatchMax == k::MAXB, "batch bound of the V-cycle kernels");

template <typename T>
void step1_batch(const DHierarchy<T> &sdc, PrecWork<T> *const *w, const T *const *vu, T *const *zu, int nb,
                 hipStream_t st) {
    if (nb < 1 || nb > k::MAXB) throw Error(PS_EINVAL, "batch size");
    VBatch<T> B;
    B.k = nb;
    k::VP<const T> b{};
    k::VP<T> out{};
    for (int i = 0; i < nb; ++i) {
        B.W[i] = &w[i]->sdc;
        b.p[i] = vu[i];
        out.p[i] = zu[i];
    }
    vcycle(sdc, B, 0, b, out, st);
}

// ------------------------------------------------------------------ system SpMV
template <int NF, typename TX>
static void spmv_full_nf(const DSystem &S, const TX *x, const double *b, double *y, hipStream_t st) {
    size_t nu = (size_t)3 * S.n_nodes;
    const double N = (double)nu + (double)NF * S.n_cells;
    ktime::Scope ts(ktime::SPMV, st, S.mat_bytes + N * sizeof(TX) + N * 8 * (b ? 2 : 1));
    const unsigned gn = grid_for(S.n_nodes), g = gn + grid_for(S.n_cells);
    if (b)
        LAUNCH((k::spmv_sys<NF, TX, true>), g, 0, st, S.Auu, S.Auf, S.Afu, S.Aff, x, x + nu, b, b + nu, y, y + nu,
               (int)gn);
    else
        LAUNCH((k::spmv_sys<NF, TX, false>), g, 0, st, S.Auu, S.Auf, S.Afu, S.Aff, x, x + nu, b, b, y, y + nu,
               (int)gn);
}

template <typename TX>
void spmv_full(const DSystem &S, const TX *x, const double *b, double *y, hipStream_t st) {
    if (S.nf == 2) spmv_full_nf<2, TX>(S, x, b, y, st);
    else spmv_full_nf<3, TX>(S, x, b, y, st);
}

// ------------------------------------------------------------------ Krylov workspace
Krylov::~Krylov() {
    if (hostscal && own_hostscal) (void)hipHostFree(hostscal);
}

// The workspace's arrays in one fixed order, each 256-byte aligned; `take(bytes)` hands
// out the memory (an arena, or a bump pointer in caller-provided memory).
template <typename Take>
static void layout_krylov(Krylov &K, size_t N, int m, bool z_fp32, Take take) {
    K.m = m;
    K.N = N;
    K.z_fp32 = z_fp32;
    // three workgroups per compute unit (256 on MI355X) for the passes over the basis: on a
    // 1.35M-row basis 768 took the DCGS2 passes from 102 / 89 us to 98 / 86 us against 1024
    // (four per unit) and 512
    K.nblk = (int)std::min<size_t>(3 * 256, std::max<size_t>(1, (N + 255) / 256));
    size_t chunk = (N + K.nblk - 1) / K.nblk;
    K.chunk = (int)((chunk + 63) / 64 * 64);
    auto d = [&](size_t n) { return static_cast<double *>(take(n * sizeof(double))); };
    K.ldv = (N + 31) / 32 * 32;
    K.V = d((size_t)(m + 1) * K.ldv);
    K.Z = take((size_t)m * N * (z_fp32 ? sizeof(float) : sizeof(double)));
    K.H = d((size_t)(m + 1) * m);
    K.cs = d(m);
    K.sn = d(m);
    K.g = d(m + 1);
    K.y = d(m);
    K.h1 = d(2 * (size_t)m + 4);         // CGS2: m + 2 rows; DCGS2: 2 (m + 1) + 1
    K.h2 = d(m + 2);
    K.hsum = d(m + 2);
    K.nw2 = d(2);
    K.scal = d(8);
    K.partial = d((2 * (size_t)m + 4) * K.nblk);
    K.raw = d(m + 2);
    K.coef = d(4);
    K.r = d(N);
}

static size_t round256(size_t b) { return ((b ? b : 1) + 255) / 256 * 256; }

void alloc_krylov(Krylov &K, size_t N, int m, bool z_fp32) {
    K.arena.release();
    if (K.hostscal && K.own_hostscal) (void)hipHostFree(K.hostscal);
    K.hostscal = nullptr;
    layout_krylov(K, N, m, z_fp32, [&](size_t bytes) { return (void *)K.arena.alloc<char>(round256(bytes)); });
    PS_HIP(hipHostMalloc((void **)&K.hostscal, 8 * sizeof(double), hipHostMallocDefault));
    K.own_hostscal = true;
}

size_t krylov_bytes(size_t N, int m, bool z_fp32) {
    Krylov K;
    size_t used = 0;
    layout_krylov(K, N, m, z_fp32, [&](size_t bytes) {
        used += round256(bytes);
        return (void *)nullptr;
    });
    return used;
}

void carve_krylov(Krylov &K, void *base, size_t cap, size_t N, int m, bool z_fp32, double *hostscal) {
    const size_t need = krylov_bytes(N, m, z_fp32);
    if (need > cap)
        throw Error(PS_EINVAL, "the Krylov workspace needs " + std::to_string(need) + " bytes; the static scratch holds " +
                                   std::to_string(cap));
    char *p = static_cast<char *>(base);
    layout_krylov(K, N, m, z_fp32, [&](size_t bytes) {
        void *q = p;
        p += round256(bytes);
        return q;
    });
    K.hostscal = hostscal;
    K.own_hostscal = false;
}

// partial[...] <- chunk sums; rows = nv (+1 for |w|^2)
static void launch_mdot(const Krylov &K, const double *V, int nv, const double *w, bool norm, hipStream_t st) {
    bool lds = K.chunk <= 7680;          // <= 60 KB of LDS per workgroup
    size_t shm = lds ? (size_t)K.chunk * sizeof(double) : 0;
    if (norm && lds)
        LAUNCH((k::mdot<true, true>), K.nblk, shm, st, V, K.ldv, nv, w, K.N, K.chunk, K.partial, K.nblk);
    else if (norm)
        LAUNCH((k::mdot<true, false>), K.nblk, shm, st, V, K.ldv, nv, w, K.N, K.chunk, K.partial, K.nblk);
    else if (lds)
        LAUNCH((k::mdot<false, true>), K.nblk, shm, st, V, K.ldv, nv, w, K.N, K.chunk, K.partial, K.nblk);
    else
        LAUNCH((k::mdot<false, false>), K.nblk, shm, st, V, K.ldv, nv, w, K.N, K.chunk, K.partial, K.nblk);
}

// out[0] <- |w|^2 (deterministic)
static void norm2_dev(const Krylov &K, const double *w, double *out, hipStream_t st) {
    launch_mdot(K, nullptr, 0, w, true, st);
    LAUNCH(k::reduce_rows, 1, 0, st, (const double *)K.partial, K.nblk, out, (const double *)nullptr,
           (double *)nullptr);
}

void fill_zero(double *p, size_t n, hipStream_t st) {
    LAUNCH((k::fill<double>), grid_for(n), 0, st, p, 0.0, n);
}

void widen_f32(const float *in, double *out, size_t n, hipStream_t st) {
    LAUNCH((k::convert<float, double>), grid_for(n), 0, st, in, out, n);
}

// ------------------------------------------------------------------ FGMRES
Fgmres::Fgmres(const DSystem &S, Krylov &K, PrecFn &M, const double *b, double *x, double rtol, int maxit,
               hipStream_t st, int orth)
    : S_(S), K_(K), M_(M), b_(b), x_(x), rtol_(rtol), maxit_(maxit), st_(st), orth_(orth) {}

void Fgmres::copy_scal() {
    PS_HIP(hipMemcpyAsync(K_.hostscal, K_.scal, 8 * sizeof(double), hipMemcpyDeviceToHost, st_));
}

void Fgmres::start() {
    // |b|^2 -> scal[5]
    norm2_dev(K_, b_, K_.scal + 5, st_);
    copy_scal();
    phase_ = START;
}

void Fgmres::begin_cycle(const double *r) {
    // g = beta e_1, V_0 = r / beta with beta = sqrt(scal[5])
    LAUNCH(k::cycle_start, 1, 0, st_, K_.m, (const double *)(K_.scal + 5), K_.g, K_.scal);
    LAUNCH(k::scale_div, grid_for(K_.N), 0, st_, r, (const double *)K_.scal, 4, K_.V, K_.N);
    j_ = 0;
    breakdown_ = false;
    open_col_ = false;
    enqueue_iteration();
}

void Fgmres::enqueue_iteration() {
    const size_t N = K_.N;
    double *Vj = K_.V + (size_t)j_ * K_.ldv;
    size_t esz = K_.z_fp32 ? sizeof(float) : sizeof(double);
    void *zj = (char *)K_.Z + (size_t)j_ * N * esz;
    if (defer_ && M_.can_split()) {                                     // step 1 by the caller
        s1_rhs_ = M_.pre(Vj, st_);
        s1_z_ = zj;
        pending_ = true;
        return;
    }
    M_(Vj, zj, st_);                                                    // z_j = M^{-1} v_j
    rest_of_iteration();
}

void Fgmres::finish_iteration() {
    if (!pending_) return;
    const size_t N = K_.N;
    M_.post(K_.V + (size_t)j_ * K_.ldv, s1_z_, st_);                    // steps 2-8
    pending_ = false;
    rest_of_iteration();
}

void Fgmres::rest_of_iteration() {
    const int j = j_, m = K_.m, nv = j + 1;
    const size_t N = K_.N;
    double *w = K_.V + (size_t)(j + 1) * K_.ldv;
    size_t esz = K_.z_fp32 ? sizeof(float) : sizeof(double);
    void *zj = (char *)K_.Z + (size_t)j * N * esz;
    if (K_.z_fp32) spmv_full<float>(S_, (const float *)zj, nullptr, w, st_);   // w = A z_j
    else spmv_full<double>(S_, (const double *)zj, nullptr, w, st_);
    if (orth_ == PS_DCGS2) {
        rest_dcgs2();
        return;
    }
    // CGS2: h1 = V^T w (+ |w|^2), w -= V h1, h2 = V^T w, w -= V h2, h = h1 + h2, |w|^2
    const double vb = (double)N * 8;                  // bytes of one basis vector
    {
        ktime::Scope ts(ktime::CGS2_PROJECT, st_, (nv + 1) * vb);
        launch_mdot(K_, K_.V, nv, w, true, st_);
    }
    LAUNCH(k::reduce_rows, nv + 1, 0, st_, (const double *)K_.partial, K_.nblk, K_.h1, (const double *)nullptr,
           (double *)nullptr);
    if (nv >= 16 && nv <= k::SUBDOT_MAXV) {          // below ~16 vectors two passes are as fast
        ktime::Scope ts(ktime::CGS2_FUSED, st_, (nv + 2) * vb);
        const size_t shm = (size_t)nv * 65 * sizeof(double);
        // RW rows per wavefront: above 32 vectors the next even number of at least nv / 4, so
        // that few loads repeat a row past nv (measured: 4% faster for 33..64 vectors, the same
        // above; at most 32 vectors RW = 8 throughout is as fast as the finer choice)
        auto fused = [&](auto rwc) {
            constexpr int RW = decltype(rwc)::value;
            LAUNCH((k::gemv_sub_mdot<RW>), K_.nblk, shm, st_, (const double *)K_.V, K_.ldv, nv,
                   (const double *)K_.h1, w, N, K_.chunk, K_.partial, K_.nblk);
        };
        switch ((nv + 7) / 8) {
        case 2:
        case 3:
        case 4: fused(std::integral_constant<int, 8>{}); break;
        case 5: fused(std::integral_constant<int, 10>{}); break;
        case 6: fused(std::integral_constant<int, 12>{}); break;
        case 7: fused(std::integral_constant<int, 14>{}); break;
        case 8: fused(std::integral_constant<int, 16>{}); break;
        case 9: fused(std::integral_constant<int, 18>{}); break;
        case 10: fused(std::integral_constant<int, 20>{}); break;
        case 11: fused(std::integral_constant<int, 22>{}); break;
        case 12: fused(std::integral_constant<int, 24>{}); break;
        case 13: fused(std::integral_constant<int, 26>{}); break;
        default: fused(std::integral_constant<int, 28>{}); break;
        }
    } else {
        LAUNCH((k::gemv_sub<false>), K_.nblk, 0, st_, (const double *)K_.V, K_.ldv, nv, (const double *)K_.h1, w,
               N, K_.chunk, K_.partial);
        launch_mdot(K_, K_.V, nv, w, false, st_);
    }
    LAUNCH(k::reduce_rows, nv, 0, st_, (const double *)K_.partial, K_.nblk, K_.h2, (const double *)K_.h1, K_.hsum);
    {
        ktime::Scope ts(ktime::CGS2_SUBTRACT, st_, (nv + 2) * vb);
        LAUNCH((k::gemv_sub<true>), K_.nblk, 0, st_, (const double *)K_.V, K_.ldv, nv, (const double *)K_.h2, w,
               N, K_.chunk, K_.partial);
    }
    LAUNCH(k::givens, 1, 0, st_, j, m, (const double *)K_.hsum, (const double *)(K_.h1 + nv),
           (const double *)K_.partial, K_.nblk, K_.H, K_.cs, K_.sn, K_.g, K_.scal, K_.hostscal);
    phase_ = ITER;
}

// DCGS2 (j = j_): one pass over V_0..V_j = u for every product (mdot2), their sums, the
// second pass (u finished as v_j, w projected; gemv_sub2), then column j - 1 finished and
// the estimate from the unfinished column j (givens2).
void Fgmres::rest_dcgs2() {
    const int j = j_, m = K_.m, nv = j + 1;
    const size_t N = K_.N;
    double *u = K_.V + (size_t)j * K_.ldv, *w = u + K_.ldv;
    const double vb = (double)N * 8;
    {
        ktime::Scope ts(ktime::DCGS2_PROJECT, st_, (nv + 1) * vb);
        const bool lds = K_.chunk <= 3840;           // w and u: <= 60 KB of LDS
        const size_t shm = lds ? 2 * (size_t)K_.chunk * sizeof(double) : 0;
        if (lds)
            LAUNCH((k::mdot2<true>), K_.nblk, shm, st_, (const double *)K_.V, K_.ldv, nv, (const double *)w, N,
                   K_.chunk, K_.partial, K_.nblk);
        else
            LAUNCH((k::mdot2<false>), K_.nblk, shm, st_, (const double *)K_.V, K_.ldv, nv, (const double *)w, N,
                   K_.chunk, K_.partial, K_.nblk);
    }
    LAUNCH(k::reduce_rows, 2 * nv + 1, 0, st_, (const double *)K_.partial, K_.nblk, K_.h1,
           (const double *)nullptr, (double *)nullptr);
    {
        ktime::Scope ts(ktime::DCGS2_SUBTRACT, st_, (nv + 3) * vb);
        LAUNCH(k::gemv_sub2, K_.nblk, 0, st_, (const double *)K_.V, K_.ldv, j, (const double *)K_.h1, u, w, N,
               K_.chunk, K_.partial, K_.coef);
    }
    LAUNCH(k::givens2, 1, 0, st_, j, m, (const double *)K_.h1, K_.coef, K_.raw, (const double *)K_.partial,
           K_.nblk, K_.H, K_.cs, K_.sn, K_.g, K_.scal, K_.hostscal);
    open_col_ = true;
    phase_ = ITER;
}

// DCGS2 at the end of a cycle of k columns: the products of u_k (in V_k) with V_0..V_{k-1}
// and its norm, then column k - 1 finished and its rotation kept.
void Fgmres::finish_last_column(int k) {
    const size_t N = K_.N;
    double *w = K_.V + (size_t)k * K_.ldv;
    launch_mdot(K_, K_.V, k, w, true, st_);
    LAUNCH(k::reduce_rows, k + 1, 0, st_, (const double *)K_.partial, K_.nblk, K_.h2, (const double *)nullptr,
           (double *)nullptr);
    LAUNCH(k::givens_finish, 1, 0, st_, k - 1, K_.m, (const double *)K_.h2, (const double *)K_.coef,
           (const double *)K_.raw, K_.H, K_.cs, K_.sn, K_.g);
    open_col_ = false;
}

void Fgmres::end_cycle(int k) {
    if (k > 0 && open_col_) finish_last_column(k);
    open_col_ = false;
    if (k > 0) {
        LAUNCH(k::backsolve, 1, 0, st_, k, K_.m, (const double *)K_.H, (const double *)K_.g, K_.y);
        if (K_.z_fp32)
            LAUNCH((k::xupdate<float>), grid_for(K_.N), 0, st_, x_, (const float *)K_.Z, K_.N, k,
                   (const double *)K_.y, K_.N);
        else
            LAUNCH((k::xupdate<double>), grid_for(K_.N), 0, st_, x_, (const double *)K_.Z, K_.N, k,
                   (const double *)K_.y, K_.N);
    }
    spmv_full<double>(S_, x_, b_, K_.r, st_);                           // r = b - A x
    norm2_dev(K_, K_.r, K_.scal + 5, st_);
    copy_scal();
    phase_ = CYCLE_END;
}

bool Fgmres::advance() {
    const double *hs = K_.hostscal;
    switch (phase_) {
    case START: {
        beta_b_ = std::sqrt(hs[5]);
        if (!std::isfinite(beta_b_)) {
            out.status = PS_EINVAL;
            phase_ = DONE;
            return false;
        }
        fill_zero(x_, K_.N, st_);
        if (beta_b_ == 0.0) {
            phase_ = DONE;
            return false;
        }
        begin_cycle(b_);
        return true;
    }
    case ITER: {
        double est = hs[0], hn = hs[1], naz = hs[2];
        bool brk = hs[3] != 0.0;
        ++its_;
        int k = j_ + 1;
        if (!std::isfinite(est) || !std::isfinite(hn) || !std::isfinite(naz)) {
            out.status = K_.z_fp32 ? PS_EPRECISION : PS_EBREAKDOWN;
            out.iterations = its_;
            phase_ = DONE;
            return false;
        }
        if (brk) {
            breakdown_ = true;
            open_col_ = false;                // column k - 1 is dropped; k - 2 is finished
            end_cycle(k - 1);
            return true;
        }
        if (est <= rtol_ * beta_b_ || hn <= 1e-14 * naz || its_ >= maxit_ || k == K_.m) {
            end_cycle(k);
            return true;
        }
        double *w = K_.V + (size_t)k * K_.ldv;
        if (orth_ != PS_DCGS2)                       // DCGS2: gemv_sub2 wrote u_k already scaled
            LAUNCH(k::scale_div, grid_for(K_.N), 0, st_, (const double *)w, (const double *)K_.scal, 1, w, K_.N);
        j_ = k;
        enqueue_iteration();
        return true;
    }
    case CYCLE_END: {
        double rel = std::sqrt(hs[5]) / beta_b_;
        out.iterations = its_;
        out.restarts = cycles_;
        out.rel_residual = rel;
        if (rel <= rtol_) {
            out.status = PS_OK;
        } else if (breakdown_) {
            out.status = PS_EBREAKDOWN;
        } else if (its_ >= maxit_) {
            out.status = PS_EMAXIT;
        } else if (!std::isfinite(rel)) {
            out.status = K_.z_fp32 ? PS_EPRECISION : PS_EBREAKDOWN;
        } else {
            ++cycles_;
            begin_cycle(K_.r);
            return true;
        }
        phase_ = DONE;
        return false;
    }
    default:
        return false;
    }
}

void rsl_diagonals(const DSystem &S, const DHierarchy<double> &sdc, RslWork &w, int iters,
                   std::vector<double> &d_sp, std::vector<double> &d_pp, hipStream_t st) {
    const int nf = S.nf, nc = S.n_cells;
    const size_t nu = (size_t)3 * S.n_nodes, N = nu + (size_t)nf * nc;
    if (!w.ready) {
        std::vector<double> e(N, 0.0);                       // 1 on the pressure unknowns
        for (int i = 0; i < nc; ++i) e[nu + (size_t)i * nf + nf - 1] = 1.0;
        w.e = w.arena.upload(e.data(), N);
        w.y = w.arena.alloc<double>(N);
        w.g = w.arena.alloc<double>(N);
        w.t = w.arena.alloc<double>(N);
        w.z = w.arena.alloc<double>(nu);
        alloc_hier_work(w.hw, sdc, w.arena);
        w.ready = true;
    }
    fill_zero(w.y, N, st);                                   // y = 0 (its flow part stays 0)
    fill_zero(w.g, N, st);
    spmv_full<double>(S, w.e, nullptr, w.t, st);             // node rows: A_uu 0 + A_up e
    PS_HIP(hipMemcpyAsync(w.g, w.t, nu * sizeof(double), hipMemcpyDeviceToDevice, st));
    for (int it = 0; it < iters; ++it) {
        spmv_full<double>(S, w.y, w.g, w.t, st);             // node rows: g - A_uu y
        vcycle(sdc, w.hw, 0, (const double *)w.t, w.z, st);   // z = M_uu^{-1} (g - A_uu y)
        LAUNCH((k::add_to<double>), grid_for(nu), 0, st, w.y, (const double *)w.z, nu);
    }
    spmv_full<double>(S, w.y, nullptr, w.t, st);             // cell rows: A_fu y
    std::vector<double> h((size_t)nf * nc);
    PS_HIP(hipMemcpyAsync(h.data(), w.t + nu, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    PS_HIP(hipStreamSynchronize(st));
    d_sp.assign((size_t)nc * (nf - 1), 0.0);
    d_pp.assign(nc, 0.0);
    for (int i = 0; i < nc; ++i) {
        for (int l = 0; l < nf - 1; ++l) d_sp[(size_t)i * (nf - 1) + l] = -h[(size_t)i * nf + l];
        d_pp[i] = -h[(size_t)i * nf + nf - 1];
    }
}

// Preconditioned Richardson iteration x_{k+1} = x_k + M^{-1}(b - A x_k) from x_0 = 0: the
// two-stage preconditioner as a sequential (fixed-point) scheme, steps 1 and 2-8 of
// Algorithm 1 alternating mechanics and flow updates (remark after Algorithm 1).  Stops when
// |b - A x_k| <= rtol |b| (FP64 residual, checked every iteration) or after maxit steps.
// Uses K.r (residual), the first column of K.Z (the correction) and K.scal.
SolveOut richardson_blocking(const DSystem &S, Krylov &K, PrecFn &M, const double *b, double *x, double rtol,
                             int maxit, hipStream_t st) {
    SolveOut o;
    const size_t N = K.N;
    auto read_norm = [&](const double *v) {
        norm2_dev(K, v, K.scal + 5, st);
        PS_HIP(hipMemcpyAsync(K.hostscal, K.scal, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
        PS_HIP(hipStreamSynchronize(st));
        return std::sqrt(K.hostscal[5]);
    };
    const double beta_b = read_norm(b);
    fill_zero(x, N, st);
    if (!std::isfinite(beta_b)) {
        o.status = PS_EINVAL;
        return o;
    }
    if (beta_b == 0.0) {
        PS_HIP(hipStreamSynchronize(st));
        return o;
    }
    const double *r = b;                      // r_0 = b (x_0 = 0)
    for (;;) {
        M(r, K.Z, st);                        // z = M^-1 r
        if (K.z_fp32) LAUNCH((k::add_to<float>), grid_for(N), 0, st, x, (const float *)K.Z, N);
        else LAUNCH((k::add_to<double>), grid_for(N), 0, st, x, (const double *)K.Z, N);
        spmv_full<double>(S, x, b, K.r, st);  // r = b - A x
        r = K.r;
        ++o.iterations;
        const double rel = read_norm(K.r) / beta_b;
        o.rel_residual = rel;
        if (!std::isfinite(rel)) {
            o.status = K.z_fp32 ? PS_EPRECISION : PS_EBREAKDOWN;
            return o;
        }
        if (rel <= rtol) {
            o.status = PS_OK;
            return o;
        }
        if (o.iterations >= maxit) {
            o.status = PS_EMAXIT;
            return o;
        }
    }
}

SolveOut fgmres_blocking(Fgmres &run, hipStream_t st) {
    run.start();
    do {
        PS_HIP(hipStreamSynchronize(st));
    } while (run.advance());
    PS_HIP(hipStreamSynchronize(st));
    return run.out;
}

// ------------------------------------------------------------------ explicit instantiations
template Sell<double> upload_sell<double>(Arena &, const HostSell &);
template Sell<float> upload_sell<float>(Arena &, const HostSell &);
template std::unique_ptr<DHierarchy<double>> upload_hierarchy<double>(const Hierarchy &, int, bool);
template std::unique_ptr<DHierarchy<float>> upload_hierarchy<float>(const Hierarchy &, int, bool);
template void update_flow_values<double>(DFlow<double> &, const FlowSetup &, const System &, const DSystem &,
                                         const Options &, Staging &, bool, bool, bool);
template void update_flow_values<float>(DFlow<float> &, const FlowSetup &, const System &, const DSystem &,
                                        const Options &, Staging &, bool, bool, bool);
template void update_flow_pressure<double>(DFlow<double> &, const FlowSetup &, const Options &, const PresStore *);
template void update_flow_pressure<float>(DFlow<float> &, const FlowSetup &, const Options &, const PresStore *);
template void alloc_prec_work<double>(PrecWork<double> &, const DHierarchy<double> &, const DFlow<double> &, int);
template void alloc_prec_work<float>(PrecWork<float> &, const DHierarchy<float> &, const DFlow<float> &, int);
template void apply_precond<double>(const DHierarchy<double> &, const DFlow<double> &, PrecWork<double> &, int,
                                    const double *, double *, hipStream_t);
template void apply_precond<float>(const DHierarchy<float> &, const DFlow<float> &, PrecWork<float> &, int,
                                   const double *, float *, hipStream_t);
template const double *precond_pre<double>(PrecWork<double> &, int, const double *, hipStream_t);
template const float *precond_pre<float>(PrecWork<float> &, int, const double *, hipStream_t);
template void precond_post<double>(const DFlow<double> &, PrecWork<double> &, int, const double *, double *,
                                   hipStream_t);
template void precond_post<float>(const DFlow<float> &, PrecWork<float> &, int, const double *, float *,
                                  hipStream_t);
template void step1_batch<double>(const DHierarchy<double> &, PrecWork<double> *const *, const double *const *,
                                  double *const *, int, hipStream_t);
template void step1_batch<float>(const DHierarchy<float> &, PrecWork<float> *const *, const float *const *,
                                 float *const *, int, hipStream_t);
template void spmv_full<double>(const DSystem &, const double *, const double *, double *, hipStream_t);
template void spmv_full<float>(const DSystem &, const float *, const double *, double *, hipStream_t);

}  // namespace ps
