// C ABI of the solver (include/ps.h, include/ps_host.h) and the serving scheduler.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <exception>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>

#include "../../include/ps.h"
#include "../../include/ps_host.h"
#include "device.h"

using namespace ps;

namespace {

thread_local std::string g_last_error;

template <typename F>
int guard(F &&f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const Error &e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return PS_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return PS_EDEVICE;
    } catch (...) {
        g_last_error = "unknown error";
        return PS_EDEVICE;
    }
}

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// PS_TRACE=1 in the environment prints setup phase timings to stderr.
bool tracing() {
    static const bool on = [] {
        const char *e = std::getenv("PS_TRACE");
        return e && *e && *e != '0';
    }();
    return on;
}

struct PhaseTimer {
    const char *what;
    double t0;
    explicit PhaseTimer(const char *w) : what(w), t0(now_s()) {}
    ~PhaseTimer() {
        if (tracing()) std::fprintf(stderr, "[ps] %-28s %8.2f ms\n", what, 1e3 * (now_s() - t0));
    }
};

// Mechanics (separate displacement component) hierarchy, built once and shared by
// handles with the same mech_key (Sec. 5.2: the elasticity AMG is set up once).
struct Mech {
    std::mutex mu;
    // what the hierarchy was built for: a handle that shares the key must match it
    int n_nodes = 0, nblocks = 0;
    uint64_t pattern_hash = 0;
    Hierarchy host;
    bool built = false;
    std::unique_ptr<DHierarchy<double>> d64;
    std::unique_ptr<DHierarchy<float>> d32;
    size_t bytes() const { return (d64 ? d64->bytes() : 0) + (d32 ? d32->bytes() : 0); }
};

struct Request;

}  // namespace

struct ps_ctx {
    int device = 0;
    size_t budget = 0;
    std::mutex mu;
    // key: (mech_key, smoother, theta, coarse_max, max_levels) -- the options that shape
    // the hierarchy, so that handles with other options build their own
    std::map<std::tuple<uint64_t, int, double, int, int>, std::weak_ptr<Mech>> mech_cache;
    // Set-up handles released by ps_destroy, kept for a later ps_create of a system with the
    // same mech_key, options and block patterns: it takes the handle's device layouts and
    // workspaces, uploads only its own values, and its first ps_setup runs the device path.
    // key -> handles (most recent last); at most kMaxParked per key, parked_bytes <= budget / 4.
    std::map<std::string, std::vector<ps_handle *>> parked;
    size_t parked_bytes = 0;
    // serving
    std::condition_variable cv, done_cv;
    std::deque<Request *> queue;
    std::vector<Request *> active;
    std::map<uint64_t, std::unique_ptr<Request>> requests;
    std::atomic<uint64_t> next_ticket{1};
    size_t used = 0;
    bool stop = false;
    std::thread worker;
    // batched step 1 (requests on one mechanics hierarchy in one sequence of launches)
    std::atomic<uint64_t> batch_launches{0}, batch_requests{0};
    void scheduler();
};

struct ps_handle {
    ps_ctx *ctx = nullptr;
    System sys;
    Options opt;
    DSystem dsys;
    std::shared_ptr<Mech> mech;
    FlowSetup flow;
    std::unique_ptr<DFlow<double>> fl64;
    std::unique_ptr<DFlow<float>> fl32;
    Staging staging;
    PresStore pstore;                 // device copies of the pressure hierarchy (device RAP)
    bool afu_changed = true;          // A_fu values changed since the last upload
    PrecWork<double> w64;
    PrecWork<float> w32;
    RslWork rsl;                      // fixed_stress = PS_FS_RSL: vectors of the lumping
    std::unique_ptr<Krylov> K;
    double *ztmp = nullptr;           // FP32 z -> FP64 staging for ps_apply_precond
    Arena aux;
    bool ready = false;
    std::atomic<bool> busy{false};
    double setup_s = 0.0;
    std::string park_key;             // non-empty: reusable by a later ps_create (mech_key set)
    size_t parked_bytes = 0;
    size_t krylov_bytes(bool z32) const {
        size_t N = sys.N(), m = opt.restart;
        return (m + 1) * N * 8 + m * N * (z32 ? 4 : 8) + N * 8 + (m + 2) * 1024 * 8;
    }
    size_t bytes() const {
        return dsys.arena.bytes() + (mech ? mech->bytes() : 0) + (fl64 ? fl64->bytes() : 0) +
               (fl32 ? fl32->bytes() : 0) + w64.arena.bytes() + w32.arena.bytes() +
               (K ? K->arena.bytes() : 0) + aux.bytes() + pstore.arena.bytes() + pstore.work.bytes() +
               pstore.tmp.bytes() + rsl.arena.bytes();
    }
};

namespace {

struct Prec64 : PrecFn {
    ps_handle *h;
    explicit Prec64(ps_handle *hh) : h(hh) {}
    void operator()(const double *v, void *z, hipStream_t st) override {
        apply_precond<double>(*h->mech->d64, *h->fl64, h->w64, h->sys.n_nodes, v, (double *)z, st);
    }
    bool can_split() const override { return true; }
    const void *pre(const double *v, hipStream_t st) override {
        return precond_pre<double>(h->w64, h->sys.n_nodes, v, st);
    }
    void post(const double *v, void *z, hipStream_t st) override {
        precond_post<double>(*h->fl64, h->w64, h->sys.n_nodes, v, (double *)z, st);
    }
};

struct Prec32 : PrecFn {
    ps_handle *h;
    explicit Prec32(ps_handle *hh) : h(hh) {}
    void operator()(const double *v, void *z, hipStream_t st) override {
        apply_precond<float>(*h->mech->d32, *h->fl32, h->w32, h->sys.n_nodes, v, (float *)z, st);
    }
    bool can_split() const override { return true; }
    const void *pre(const double *v, hipStream_t st) override {
        return precond_pre<float>(h->w32, h->sys.n_nodes, v, st);
    }
    void post(const double *v, void *z, hipStream_t st) override {
        precond_post<float>(*h->fl32, h->w32, h->sys.n_nodes, v, (float *)z, st);
    }
};

struct Request {
    uint64_t ticket = 0;
    ps_handle *h = nullptr;
    const double *rhs = nullptr;
    double *x = nullptr;
    double rtol = 0.0;
    int status = PS_PENDING;
    ps_result res{};
    size_t bytes = 0;
    double t_submit = 0.0, t_start = 0.0;
    hipStream_t st = nullptr;
    hipEvent_t ready = nullptr;       // recorded on the caller's stream at submit
    hipEvent_t mark = nullptr;        // orders the request's stream against a batched step 1
    std::unique_ptr<Krylov> K;
    std::unique_ptr<PrecFn> M;
    std::unique_ptr<Fgmres> run;
};

void set_device(int dev) { PS_HIP(hipSetDevice(dev)); }

// Galerkin products of the pressure AMG on the device (default) or on host threads
// (PS_GALERKIN=host); both give the same hierarchy bit for bit.
bool galerkin_on_device() {
    const char *e = std::getenv("PS_GALERKIN");
    return !(e && std::string(e) == "host");
}

bool use_fp32(const ps_handle *h) { return h->opt.precision == PS_FP32_PREC; }

bool host_operators_forced() {
    const char *e = std::getenv("PS_OPERATORS");
    return e && std::string(e) == "host";
}

// FNV-1a over A_uu's row pointers and column indices: handles sharing a mechanics
// hierarchy must agree on the pattern it was built for.
uint64_t pattern_hash(const Bsr &U) {
    uint64_t x = 1469598103934665603ull;
    auto mix = [&x](const std::vector<int> &a) {
        for (int v : a) {
            x ^= (uint32_t)v;
            x *= 1099511628211ull;
        }
    };
    mix(U.rp);
    mix(U.ci);
    return x;
}

constexpr size_t kMaxParked = 4;

// What a parked handle must share with a new system to be reused: the mechanics key, every
// option, the sizes, and the four block patterns and the subdomain partition.
std::string park_key(const System &s, const Options &o) {
    uint64_t part = 1469598103934665603ull;
    for (int v : s.ml_part) {
        part ^= (uint32_t)v;
        part *= 1099511628211ull;
    }
    char buf[512];
    std::snprintf(buf, sizeof buf,
                  "%llu|%d,%d,%d,%d,%d,%d,%d,%d,%d,%.17g,%d,%d,%d,%d,%d|%d,%d,%d|%llx,%llx,%llx,%llx,%llx",
                  (unsigned long long)s.mech_key, o.precision, o.restart, o.maxit, o.smoother, o.ml_kind,
                  o.ml_sweeps, o.coarse_max, o.max_levels, o.fp32_fallback, o.theta, o.method, o.reduction,
                  o.fixed_stress, o.fs_iters, o.orth, s.n_nodes, s.n_cells, s.nf, (unsigned long long)pattern_hash(s.Auu),
                  (unsigned long long)pattern_hash(s.Auf), (unsigned long long)pattern_hash(s.Afu),
                  (unsigned long long)pattern_hash(s.Aff), (unsigned long long)part);
    return buf;
}

std::shared_ptr<Mech> new_mech(int n_nodes, int nblocks, uint64_t phash) {
    auto m = std::make_shared<Mech>();
    m->n_nodes = n_nodes;
    m->nblocks = nblocks;
    m->pattern_hash = phash;
    return m;
}

void ensure_mech_device(ps_handle *h, bool need64, bool need32) {
    std::lock_guard<std::mutex> lk(h->mech->mu);
    if (!h->mech->built) {
        h->mech->host = amg_build(sdc_matrix(h->sys), h->opt);
        h->mech->built = true;
    }
    if (need64 && !h->mech->d64) {
        h->mech->d64 = upload_hierarchy<double>(h->mech->host, h->opt.smoother, true);
        h->mech->d64->ktag = ktime::SDC_PRE;
    }
    if (need32 && !h->mech->d32) {
        h->mech->d32 = upload_hierarchy<float>(h->mech->host, h->opt.smoother, true);
        h->mech->d32->ktag = ktime::SDC_PRE;
    }
}

// ---------------------------------------------------------------- no-allocation solves
// Static device memory for ps_solve_noalloc: the Krylov workspace of one solve at a time
// per device.  Host code never uses the array's name as an address (it is a host-side
// stand-in); the device address comes from hipGetSymbolAddress, looked up once per device
// with that device current, at ps_ctx_create.
__device__ __align__(256) unsigned char scratch[PS_NOALLOC_SCRATCH_BYTES];

struct NoAllocDev {
    std::once_flag once;
    void *ptr = nullptr;                // this device's copy of `scratch`
    double *hostscal = nullptr;         // pinned scalar mirror used by the solve's driver
    std::mutex mu;                      // one ps_solve_noalloc at a time on this device
};
constexpr int kMaxDevices = 64;
NoAllocDev g_noalloc[kMaxDevices];

// Called with `dev` current (ps_ctx_create).
void noalloc_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) throw Error(PS_EINVAL, "device index beyond the no-allocation table");
    NoAllocDev &d = g_noalloc[dev];
    std::call_once(d.once, [&] {
        void *p = nullptr;
        PS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        double *hs = nullptr;
        PS_HIP(hipHostMalloc((void **)&hs, 8 * sizeof(double), hipHostMallocDefault));
        d.ptr = p;
        d.hostscal = hs;
    });
    if (!d.ptr || !d.hostscal) throw Error(PS_EDEVICE, "no-allocation scratch not set up for this device");
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char *ps_last_error(void) { return g_last_error.c_str(); }

const char *ps_strerror(int s) {
    switch (s) {
    case PS_OK: return "ok";
    case PS_PENDING: return "pending";
    case PS_EINVAL: return "invalid argument";
    case PS_ENOMEM: return "out of memory";
    case PS_EDEVICE: return "device error";
    case PS_ENOTSETUP: return "handle not set up";
    case PS_ESINGULAR: return "singular block or coarse matrix";
    case PS_EMAXIT: return "maximum iterations reached";
    case PS_EPRECISION: return "non-finite value in the FP32 preconditioner";
    case PS_EBUSY: return "busy";
    case PS_EBREAKDOWN: return "Krylov breakdown";
    default: return "unknown status";
    }
}

void ps_default_options(ps_options *o) {
    if (!o) return;
    o->precision = PS_FP64;
    o->restart = 100;
    o->maxit = 1000;
    o->smoother = PS_CHEB2;
    o->ml_kind = PS_BILU0;
    o->ml_sweeps = 1;
    o->coarse_max = 256;
    o->max_levels = 25;
    o->fp32_fallback = 0;
    o->theta = 0.25;
    o->method = PS_FGMRES;
    o->reduction = PS_QUASI_IMPES;
    o->fixed_stress = PS_FS_GIVEN;
    o->fs_iters = 10;
    o->orth = PS_CGS2;
}

int ps_ctx_create(int device, size_t budget, ps_ctx **out) {
    return guard([&] {
        if (!out) throw Error(PS_EINVAL, "out is NULL");
        *out = nullptr;
        int n = 0;
        PS_HIP(hipGetDeviceCount(&n));
        if (device < 0 || device >= n) throw Error(PS_EINVAL, "no such device");
        set_device(device);
        noalloc_init(device);
        auto c = std::make_unique<ps_ctx>();
        c->device = device;
        if (budget == 0) {
            size_t fr = 0, tot = 0;
            PS_HIP(hipMemGetInfo(&fr, &tot));
            budget = (size_t)(0.9 * (double)fr);
        }
        c->budget = budget;
        ps_ctx *raw = c.get();
        c->worker = std::thread([raw] { raw->scheduler(); });
        *out = c.release();
        return PS_OK;
    });
}

void ps_ctx_destroy(ps_ctx *c) {
    if (!c) return;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        c->stop = true;
    }
    c->cv.notify_all();
    if (c->worker.joinable()) c->worker.join();
    (void)hipSetDevice(c->device);
    for (auto &kv : c->parked)
        for (ps_handle *h : kv.second) delete h;
    c->parked.clear();
    delete c;
}

int ps_create(ps_ctx *ctx, const ps_system *sys, const ps_options *opts, ps_handle **out) {
    return guard([&] {
        if (!ctx || !out) throw Error(PS_EINVAL, "ctx/out is NULL");
        *out = nullptr;
        ps_options def;
        ps_default_options(&def);
        Options opt = options_from(opts ? opts : &def);
        System vs;
        validate_and_copy(sys, vs);
        std::string key;
        if (vs.mech_key != 0) {
            key = park_key(vs, opt);
            ps_handle *reuse = nullptr;
            {
                std::lock_guard<std::mutex> lk(ctx->mu);
                auto it = ctx->parked.find(key);
                if (it != ctx->parked.end() && !it->second.empty()) {
                    reuse = it->second.back();
                    it->second.pop_back();
                    ctx->parked_bytes -= reuse->parked_bytes;
                    reuse->parked_bytes = 0;
                }
            }
            if (reuse) {
                // same patterns and options: keep the layouts, take this system's values (A_uu
                // is the shared one by the mech_key contract)
                std::unique_ptr<ps_handle> h(reuse);
                h->sys = std::move(vs);
                set_device(ctx->device);
                update_system_flow_values(h->sys, h->dsys, h->staging, true);
                h->afu_changed = true;
                h->ready = false;
                h->setup_s = 0.0;
                *out = h.release();
                return PS_OK;
            }
        }
        auto h = std::make_unique<ps_handle>();
        h->ctx = ctx;
        h->opt = opt;
        h->sys = std::move(vs);
        h->park_key = key;
        set_device(ctx->device);
        upload_system(h->sys, h->dsys);
        const Bsr &U = h->sys.Auu;
        const uint64_t phash = pattern_hash(U);
        if (h->sys.mech_key != 0) {
            std::lock_guard<std::mutex> lk(ctx->mu);
            auto key = std::make_tuple(h->sys.mech_key, (int)h->opt.smoother, h->opt.theta,
                                       (int)h->opt.coarse_max, (int)h->opt.max_levels);
            auto it = ctx->mech_cache.find(key);
            if (it != ctx->mech_cache.end()) h->mech = it->second.lock();
            if (h->mech && (h->mech->n_nodes != h->sys.n_nodes || h->mech->nblocks != U.nb() ||
                            h->mech->pattern_hash != phash))
                throw Error(PS_EINVAL, "mech_key names a mechanics hierarchy built for another A_uu pattern");
            if (!h->mech) {
                h->mech = new_mech(h->sys.n_nodes, U.nb(), phash);
                ctx->mech_cache[key] = h->mech;
            }
        } else {
            h->mech = new_mech(h->sys.n_nodes, U.nb(), phash);
        }
        *out = h.release();
        return PS_OK;
    });
}

int ps_update_flow(ps_handle *h, const double *afu, const double *aff, const double *d_sp, const double *d_pp,
                   const double *auf) {
    return guard([&] {
        if (!h) throw Error(PS_EINVAL, "handle is NULL");
        if (h->busy) throw Error(PS_EBUSY, "handle has a request in flight");
        System &s = h->sys;
        auto take = [](std::vector<double> &dst, const double *src) {
            if (!src) return;
            for (size_t i = 0; i < dst.size(); ++i)
                if (!std::isfinite(src[i])) throw Error(PS_EINVAL, "non-finite value");
            std::memcpy(dst.data(), src, dst.size() * sizeof(double));
        };
        take(s.Auf.v, auf);
        take(s.Afu.v, afu);
        if (afu) h->afu_changed = true;
        take(s.Aff.v, aff);
        take(s.d_sp, d_sp);
        take(s.d_pp, d_pp);
        set_device(h->ctx->device);
        // only the flow blocks' values cross PCIe, into the resident layout
        update_system_flow_values(s, h->dsys, h->staging, auf != nullptr);
        h->ready = false;
        return PS_OK;
    });
}

int ps_setup(ps_handle *h) {
    return guard([&] {
        if (!h) throw Error(PS_EINVAL, "handle is NULL");
        if (h->busy) throw Error(PS_EBUSY, "handle has a request in flight");
        double t0 = now_s();
        set_device(h->ctx->device);
        h->ready = false;
        bool f32 = use_fp32(h);
        bool f64 = !f32 || h->opt.fp32_fallback;
        const bool rsl = h->opt.fixed_stress == PS_FS_RSL;
        {
            PhaseTimer pt("mechanics (if not built)");
            ensure_mech_device(h, f64 || rsl, f32);      // RSL runs the FP64 mechanics V-cycle
        }
        if (rsl) {
            PhaseTimer pt("RSL fixed-stress diagonals");
            rsl_diagonals(h->dsys, *h->mech->d64, h->rsl, h->opt.fs_iters, h->sys.d_sp, h->sys.d_pp, nullptr);
        }
        const bool dev_rap = galerkin_on_device();
        // after the first setup has laid out the subdomain BILU(0), its factorization runs on
        // the device from S_ff's values (the host keeps the pattern only)
        auto dev_factor_ready = [](const auto &fl) { return fl && fl->sub && fl->sb.dev_factor; };
        const bool dev_factor = (!f64 || dev_factor_ready(h->fl64)) && (!f32 || dev_factor_ready(h->fl32));
        // and S_pp, D_ss (quasi-IMPES) and the pressure hierarchy come from the system on the
        // device, with no host work in front of the pressure hierarchy (PS_OPERATORS=host:
        // fixed stress and quasi-IMPES on the host at every setup)
        // (quasi-IMPES only: the true-IMPES column sums are formed on the host)
        const bool dev_ops = dev_factor && dev_rap && h->opt.smoother == PS_L1JAC &&
                             h->opt.reduction == PS_QUASI_IMPES && h->pstore.npat == h->sys.n_cells &&
                             !host_operators_forced();
        // layouts (first call) and values of the flow stage that do not depend on the
        // pressure hierarchy, for the precisions in use
        auto flow_values = [&] {
            PhaseTimer pt("flow values upload");
            if (f64) {
                if (!h->fl64) h->fl64 = std::make_unique<DFlow<double>>();
                update_flow_values<double>(*h->fl64, h->flow, h->sys, h->dsys, h->opt, h->staging, h->afu_changed,
                                           dev_factor, dev_ops);
            }
            if (f32) {
                if (!h->fl32) h->fl32 = std::make_unique<DFlow<float>>();
                update_flow_values<float>(*h->fl32, h->flow, h->sys, h->dsys, h->opt, h->staging, h->afu_changed,
                                          dev_factor, dev_ops);
            }
        };
        {
            PhaseTimer pt("flow setup");
            if (!dev_ops) build_flow_operators(h->sys, h->opt, h->flow);
            if (dev_rap) {
                // local-stage factors and the flow-stage value uploads on a host thread
                // while the pressure hierarchy is built (its own copies run on the null
                // stream, the uploads on the staging buffer's stream)
                std::exception_ptr err;
                const int dev = h->ctx->device;
                std::thread local([&] {
                    try {
                        set_device(dev);
                        build_flow_local(h->sys, h->opt, h->flow, dev_factor);
                        flow_values();
                    } catch (...) {
                        err = std::current_exception();
                    }
                });
                try {
                    PhaseTimer pt2("pressure AMG (device)");
                    if (dev_ops) {
                        build_pressure_from_system(h->sys, h->dsys, h->opt, h->flow.pres, h->pstore);
                    } else {
                        build_pressure(h->flow.Spp, h->opt, h->flow.pres, h->pstore);
                        if (h->opt.smoother == PS_L1JAC && h->pstore.npat == 0)
                            layout_pressure_operator(h->sys, h->pstore);
                    }
                } catch (...) {
                    local.join();
                    throw;
                }
                local.join();
                if (err) std::rethrow_exception(err);
            } else {
                h->pstore.on_device = false;
                {
                    PhaseTimer pt2("pressure AMG (host)");
                    h->flow.pres = amg_build(h->flow.Spp, h->opt);
                }
                build_flow_local(h->sys, h->opt, h->flow, dev_factor);
                flow_values();
            }
        }
        const PresStore *ps = dev_rap ? &h->pstore : nullptr;
        PhaseTimer pt("pressure levels + work");
        if (f64) {
            update_flow_pressure<double>(*h->fl64, h->flow, h->opt, ps);
            alloc_prec_work(h->w64, *h->mech->d64, *h->fl64, h->sys.n_nodes);
        }
        if (f32) {
            update_flow_pressure<float>(*h->fl32, h->flow, h->opt, ps);
            alloc_prec_work(h->w32, *h->mech->d32, *h->fl32, h->sys.n_nodes);
        }
        h->afu_changed = false;
        PS_HIP(hipDeviceSynchronize());
        h->setup_s = now_s() - t0;
        h->ready = true;
        return PS_OK;
    });
}

// Krylov workspace columns an outer iteration needs: the restart length for FGMRES, one
// correction vector for Richardson.
static int workspace_m(const ps_handle *h) { return h->opt.method == PS_RICHARDSON ? 1 : h->opt.restart; }

static SolveOut run_solve(ps_handle *h, Krylov &K, bool fp32, const double *rhs, double *x, double rtol,
                          hipStream_t st) {
    Prec32 m32(h);
    Prec64 m64(h);
    PrecFn &M = fp32 ? static_cast<PrecFn &>(m32) : static_cast<PrecFn &>(m64);
    if (h->opt.method == PS_RICHARDSON) return richardson_blocking(h->dsys, K, M, rhs, x, rtol, h->opt.maxit, st);
    Fgmres run(h->dsys, K, M, rhs, x, rtol, h->opt.maxit, st, h->opt.orth);
    return fgmres_blocking(run, st);
}

static void check_solve_args(ps_handle *h, const double *rhs, const double *x, double rtol) {
    if (!h) throw Error(PS_EINVAL, "handle is NULL");
    if (!rhs || !x) throw Error(PS_EINVAL, "rhs/x is NULL");
    if (!(rtol > 0.0) || !std::isfinite(rtol)) throw Error(PS_EINVAL, "rtol must be positive and finite");
    if (!h->ready) throw Error(PS_ENOTSETUP, "ps_setup has not been called");
}

int ps_solve(ps_handle *h, const double *rhs, double *x, double rtol, void *stream, ps_result *res) {
    int code = guard([&] {
        check_solve_args(h, rhs, x, rtol);
        bool expected = false;
        if (!h->busy.compare_exchange_strong(expected, true)) throw Error(PS_EBUSY, "handle has a request in flight");
        struct Unbusy {
            ps_handle *h;
            ~Unbusy() { h->busy = false; }
        } ub{h};
        set_device(h->ctx->device);
        hipStream_t st = (hipStream_t)stream;
        double t0 = now_s();
        bool f32 = use_fp32(h);
        const int m = workspace_m(h);
        if (!h->K || h->K->z_fp32 != f32 || h->K->m != m) {
            h->K = std::make_unique<Krylov>();
            alloc_krylov(*h->K, h->sys.N(), m, f32);
        }
        SolveOut o = run_solve(h, *h->K, f32, rhs, x, rtol, st);
        if (o.status == PS_EPRECISION && f32 && h->opt.fp32_fallback) {
            Krylov K64;
            alloc_krylov(K64, h->sys.N(), m, false);
            o = run_solve(h, K64, false, rhs, x, rtol, st);
        }
        if (res) {
            res->status = o.status;
            res->iterations = o.iterations;
            res->restarts = o.restarts;
            res->rel_residual = o.rel_residual;
            res->setup_s = h->setup_s;
            res->solve_s = now_s() - t0;
        }
        return o.status;
    });
    if (code != PS_OK && res && code != PS_EMAXIT && code != PS_EPRECISION && code != PS_EBREAKDOWN)
        res->status = code;
    return code;
}

int ps_solve_noalloc(ps_handle *h, const double *rhs, double *x, double rtol, void *stream, ps_result *res) {
    int code = guard([&] {
        check_solve_args(h, rhs, x, rtol);
        const int dev = h->ctx->device;
        NoAllocDev &d = g_noalloc[dev];
        if (!d.ptr) throw Error(PS_EDEVICE, "no-allocation scratch not set up for this device");
        const bool f32 = use_fp32(h);
        const int m = workspace_m(h);
        const size_t need = krylov_bytes(h->sys.N(), m, f32);
        if (need > (size_t)PS_NOALLOC_SCRATCH_BYTES)
            throw Error(PS_EINVAL, "ps_solve_noalloc: N = " + std::to_string(h->sys.N()) + " with restart " +
                                       std::to_string(h->opt.restart) + " needs " + std::to_string(need) +
                                       " bytes of scratch; the maximum is " +
                                       std::to_string((size_t)PS_NOALLOC_SCRATCH_BYTES));
        bool expected = false;
        if (!h->busy.compare_exchange_strong(expected, true)) throw Error(PS_EBUSY, "handle has a request in flight");
        struct Unbusy {
            ps_handle *h;
            ~Unbusy() { h->busy = false; }
        } ub{h};
        std::lock_guard<std::mutex> lk(d.mu);
        set_device(dev);
        hipStream_t st = (hipStream_t)stream;
        double t0 = now_s();
        Krylov K;
        carve_krylov(K, d.ptr, (size_t)PS_NOALLOC_SCRATCH_BYTES, h->sys.N(), m, f32, d.hostscal);
        SolveOut o = run_solve(h, K, f32, rhs, x, rtol, st);
        if (res) {
            res->status = o.status;
            res->iterations = o.iterations;
            res->restarts = o.restarts;
            res->rel_residual = o.rel_residual;
            res->setup_s = h->setup_s;
            res->solve_s = now_s() - t0;
        }
        return o.status;
    });
    if (code != PS_OK && res && code != PS_EMAXIT && code != PS_EPRECISION && code != PS_EBREAKDOWN)
        res->status = code;
    return code;
}

int ps_apply_precond(ps_handle *h, const double *v, double *z, void *stream) {
    return guard([&] {
        if (!h || !v || !z) throw Error(PS_EINVAL, "NULL argument");
        if (!h->ready) throw Error(PS_ENOTSETUP, "ps_setup has not been called");
        set_device(h->ctx->device);
        hipStream_t st = (hipStream_t)stream;
        if (use_fp32(h)) {
            size_t N = h->sys.N();
            if (!h->ztmp) h->ztmp = (double *)h->aux.alloc<float>(N);
            Prec32 M(h);
            M(v, h->ztmp, st);
            widen_f32((const float *)h->ztmp, z, N, st);
        } else {
            Prec64 M(h);
            M(v, z, st);
        }
        PS_HIP(hipGetLastError());
        return PS_OK;
    });
}

int ps_spmv(ps_handle *h, const double *x, double *y, void *stream) {
    return guard([&] {
        if (!h || !x || !y) throw Error(PS_EINVAL, "NULL argument");
        set_device(h->ctx->device);
        hipStream_t st = (hipStream_t)stream;
        spmv_full<double>(h->dsys, x, nullptr, y, st);
        PS_HIP(hipGetLastError());
        return PS_OK;
    });
}

int ps_footprint(ps_handle *h, size_t *bytes) {
    return guard([&] {
        if (!h || !bytes) throw Error(PS_EINVAL, "NULL argument");
        *bytes = h->bytes();
        return PS_OK;
    });
}

void ps_destroy(ps_handle *h) {
    if (!h) return;
    ps_ctx *c = h->ctx;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    if (!h->park_key.empty() && h->ready && !h->busy) {
        const size_t b = h->bytes();
        std::lock_guard<std::mutex> lk(c->mu);
        auto &v = c->parked[h->park_key];
        if (!c->stop && v.size() < kMaxParked && c->parked_bytes + b <= c->budget / 4) {
            h->parked_bytes = b;
            c->parked_bytes += b;
            v.push_back(h);
            return;
        }
    }
    delete h;
}

// ---------------------------------------------------------------- serving
int ps_submit(ps_handle *h, const double *rhs, double *x, double rtol, void *stream, uint64_t *ticket) {
    return guard([&] {
        check_solve_args(h, rhs, x, rtol);
        if (!ticket) throw Error(PS_EINVAL, "ticket is NULL");
        if (h->opt.method != PS_FGMRES) throw Error(PS_EINVAL, "ps_submit runs FGMRES only (method PS_FGMRES)");
        bool expected = false;
        if (!h->busy.compare_exchange_strong(expected, true)) throw Error(PS_EBUSY, "handle has a request in flight");
        ps_ctx *c = h->ctx;
        auto r = std::make_unique<Request>();
        try {
            set_device(c->device);
            PS_HIP(hipEventCreateWithFlags(&r->ready, hipEventDisableTiming));
            PS_HIP(hipEventRecord(r->ready, (hipStream_t)stream));
        } catch (...) {
            h->busy = false;
            throw;
        }
        r->ticket = c->next_ticket++;
        r->h = h;
        r->rhs = rhs;
        r->x = x;
        r->rtol = rtol;
        r->t_submit = now_s();
        r->bytes = h->krylov_bytes(use_fp32(h));
        *ticket = r->ticket;
        {
            std::lock_guard<std::mutex> lk(c->mu);
            if (c->stop) {
                h->busy = false;
                throw Error(PS_EBUSY, "context is shutting down");
            }
            c->queue.push_back(r.get());
            c->requests[r->ticket] = std::move(r);
        }
        c->cv.notify_all();
        return PS_OK;
    });
}

static int take_result(ps_ctx *c, uint64_t ticket, ps_result *res, bool wait) {
    std::unique_lock<std::mutex> lk(c->mu);
    auto it = c->requests.find(ticket);
    if (it == c->requests.end()) throw Error(PS_EINVAL, "unknown ticket");
    if (wait) c->done_cv.wait(lk, [&] { return it->second->status != PS_PENDING; });
    Request *r = it->second.get();
    if (r->status == PS_PENDING) return PS_PENDING;
    if (res) *res = r->res;
    int s = r->status;
    c->requests.erase(it);
    return s;
}

int ps_poll(ps_ctx *c, uint64_t ticket, ps_result *res) {
    return guard([&] {
        if (!c) throw Error(PS_EINVAL, "ctx is NULL");
        return take_result(c, ticket, res, false);
    });
}

int ps_kernel_timing(int enable) {
    return guard([&] {
        ktime::set_mask(enable == PS_KT_ALL ? ~0u : (unsigned)enable);
        return PS_OK;
    });
}

int ps_kernel_stats(int idx, char *name, size_t len, int64_t *launches, double *seconds, double *bytes) {
    return guard([&] {
        if (idx < 0 || idx >= ktime::NUM) throw Error(PS_EINVAL, "kernel index out of range");
        long long l = 0;
        double sec = 0.0, b = 0.0;
        ktime::totals(idx, l, sec, b);
        if (name && len) {
            std::strncpy(name, ktime::name(idx), len - 1);
            name[len - 1] = 0;
        }
        if (launches) *launches = l;
        if (seconds) *seconds = sec;
        if (bytes) *bytes = b;
        return PS_OK;
    });
}

int ps_pressure_level(ps_handle *h, int lvl, int32_t *nlevels, int32_t *n, int32_t *nnz, int32_t *rowptr,
                      int32_t *colind, double *vals, int8_t *cf) {
    return guard([&] {
        if (!h) throw Error(PS_EINVAL, "handle is NULL");
        if (!h->ready) throw Error(PS_ENOTSETUP, "ps_setup has not run");
        const Hierarchy &H = h->flow.pres;
        if (nlevels) *nlevels = (int32_t)H.lev.size();
        if (lvl < 0 || lvl >= (int)H.lev.size()) throw Error(PS_EINVAL, "level out of range");
        Csr dA;
        std::vector<int8_t> dcf;
        const bool dev = h->pstore.on_device;
        if (dev) download_level(h->pstore, lvl, dA, dcf);      // built on the device: copy back
        const Csr &A = dev ? dA : H.lev[lvl].A;
        const std::vector<int8_t> &c = dev ? dcf : H.lev[lvl].cf;
        if (n) *n = A.n;
        if (nnz) *nnz = A.nnz();
        if (rowptr) std::memcpy(rowptr, A.rp.data(), A.rp.size() * sizeof(int32_t));
        if (colind) std::memcpy(colind, A.ci.data(), A.ci.size() * sizeof(int32_t));
        if (vals) std::memcpy(vals, A.v.data(), A.v.size() * sizeof(double));
        if (cf && !c.empty()) std::memcpy(cf, c.data(), c.size());
        return PS_OK;
    });
}

int ps_ctx_batches(ps_ctx *c, uint64_t *launches, uint64_t *requests) {
    return guard([&] {
        if (!c) throw Error(PS_EINVAL, "ctx is NULL");
        if (launches) *launches = c->batch_launches.load();
        if (requests) *requests = c->batch_requests.load();
        return PS_OK;
    });
}

int ps_wait(ps_ctx *c, uint64_t ticket, ps_result *res) {
    return guard([&] {
        if (!c) throw Error(PS_EINVAL, "ctx is NULL");
        return take_result(c, ticket, res, true);
    });
}

}  // extern "C"

// Iteration-level continuous batching: every admitted request advances by one piece of
// FGMRES work (one iteration or one cycle end) on its own stream as soon as its previous
// piece has completed, so the device overlaps requests; queued requests are admitted
// whenever their device footprint fits the budget, and finished ones leave at once.
void ps_ctx::scheduler() {
    (void)hipSetDevice(device);
    // step 1 of requests that share a mechanics hierarchy runs as one batch (gridDim.y = the
    // requests) on this stream, ordered by events against each request's own stream
    const bool batching = [] {
        const char *e = std::getenv("PS_SERVING_BATCH");
        return !(e && std::string(e) == "0");
    }();
    hipStream_t bst = nullptr;
    hipEvent_t bev = nullptr;
    if (batching) {
        if (hipStreamCreateWithFlags(&bst, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&bev, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            bst = nullptr;
        }
    }
    auto finish = [this](Request *r, int status, const SolveOut *o) {
        r->res.status = status;
        if (o) {
            r->res.iterations = o->iterations;
            r->res.restarts = o->restarts;
            r->res.rel_residual = o->rel_residual;
        }
        r->res.setup_s = r->h->setup_s;
        r->res.solve_s = now_s() - r->t_submit;
        if (r->st) {                      // work still queued (after an error) ends first
            (void)hipStreamSynchronize(r->st);
            (void)hipStreamDestroy(r->st);
        }
        r->st = nullptr;
        if (r->ready) (void)hipEventDestroy(r->ready);
        r->ready = nullptr;
        if (r->mark) (void)hipEventDestroy(r->mark);
        r->mark = nullptr;
        r->run.reset();
        r->M.reset();
        r->K.reset();
        r->h->busy = false;
        std::lock_guard<std::mutex> lk(mu);
        used -= r->bytes;
        r->status = status;
        done_cv.notify_all();
    };
    for (;;) {
        std::vector<Request *> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
            if (stop && active.empty()) {
                if (bev) (void)hipEventDestroy(bev);
                if (bst) (void)hipStreamDestroy(bst);
                bev = nullptr;
                bst = nullptr;
                for (Request *r : queue) {
                    r->status = PS_EBUSY;
                    r->res.status = PS_EBUSY;
                    r->h->busy = false;
                    if (r->ready) (void)hipEventDestroy(r->ready);
                    r->ready = nullptr;
                }
                queue.clear();
                done_cv.notify_all();
                return;
            }
            while (!queue.empty() && !stop) {
                Request *r = queue.front();
                if (!active.empty() && used + r->bytes > budget) break;
                queue.pop_front();
                used += r->bytes;
                admitted.push_back(r);
            }
        }
        for (Request *r : admitted) {
            int code = guard([&] {
                bool f32 = use_fp32(r->h);
                PS_HIP(hipStreamCreateWithFlags(&r->st, hipStreamNonBlocking));
                PS_HIP(hipStreamWaitEvent(r->st, r->ready, 0));
                PS_HIP(hipEventCreateWithFlags(&r->mark, hipEventDisableTiming));
                r->K = std::make_unique<Krylov>();
                alloc_krylov(*r->K, r->h->sys.N(), r->h->opt.restart, f32);
                if (f32) r->M = std::make_unique<Prec32>(r->h);
                else r->M = std::make_unique<Prec64>(r->h);
                r->run = std::make_unique<Fgmres>(r->h->dsys, *r->K, *r->M, r->rhs, r->x, r->rtol,
                                                  r->h->opt.maxit, r->st, r->h->opt.orth);
                r->t_start = now_s();
                r->run->start();
                return PS_OK;
            });
            if (code != PS_OK) finish(r, code, nullptr);
            else active.push_back(r);
        }
        // Completion-driven: a request whose stream has drained (its scalars are on the
        // host) advances by one piece of work; the others keep running, so a small request
        // is not held to the pace of a large one.  When nothing was ready the loop waits a
        // few microseconds (or for a new submission) instead of spinning.
        std::vector<Request *> still;
        std::vector<Request *> step1;          // ready requests whose next iteration waits for step 1
        bool progressed = false;
        for (Request *r : active) {
            const hipError_t q = hipStreamQuery(r->st);
            if (q == hipErrorNotReady) {
                still.push_back(r);
                continue;
            }
            progressed = true;
            bool more = false;
            int code = guard([&] {
                if (q != hipSuccess) PS_HIP(q);
                r->run->set_defer(bst != nullptr);
                more = r->run->advance();
                if (more && r->run->step1_pending()) step1.push_back(r);
                return PS_OK;
            });
            if (code != PS_OK) {
                finish(r, code, nullptr);
            } else if (!more) {
                (void)hipStreamSynchronize(r->st);
                SolveOut o = r->run->out;
                finish(r, o.status, &o);
            } else {
                still.push_back(r);
            }
        }
        // step 1 of the deferred iterations: requests on one mechanics hierarchy (same grid and
        // precision) in batches of up to kBatchMax, each slice computing what it would alone
        std::vector<bool> done(step1.size(), false);
        for (size_t a = 0; a < step1.size(); ++a) {
            if (done[a]) continue;
            const bool f32 = use_fp32(step1[a]->h);
            const void *hier = f32 ? (const void *)step1[a]->h->mech->d32.get()
                                   : (const void *)step1[a]->h->mech->d64.get();
            std::vector<Request *> grp;
            for (size_t c = a; c < step1.size() && (int)grp.size() < kBatchMax; ++c) {
                if (done[c] || use_fp32(step1[c]->h) != f32) continue;
                const void *hc = f32 ? (const void *)step1[c]->h->mech->d32.get()
                                     : (const void *)step1[c]->h->mech->d64.get();
                if (hc != hier) continue;
                grp.push_back(step1[c]);
                done[c] = true;
            }
            int code = guard([&] {
                const int nb = (int)grp.size();
                if (nb > 1) {
                    for (Request *r : grp) {
                        PS_HIP(hipEventRecord(r->mark, r->st));
                        PS_HIP(hipStreamWaitEvent(bst, r->mark, 0));
                    }
                }
                hipStream_t s1 = nb > 1 ? bst : grp[0]->st;
                if (f32) {
                    PrecWork<float> *w[kBatchMax];
                    const float *vu[kBatchMax];
                    float *zu[kBatchMax];
                    for (int i = 0; i < nb; ++i) {
                        w[i] = &grp[i]->h->w32;
                        vu[i] = (const float *)grp[i]->run->step1_rhs();
                        zu[i] = (float *)grp[i]->run->step1_out();
                    }
                    step1_batch<float>(*grp[0]->h->mech->d32, w, vu, zu, nb, s1);
                } else {
                    PrecWork<double> *w[kBatchMax];
                    const double *vu[kBatchMax];
                    double *zu[kBatchMax];
                    for (int i = 0; i < nb; ++i) {
                        w[i] = &grp[i]->h->w64;
                        vu[i] = (const double *)grp[i]->run->step1_rhs();
                        zu[i] = (double *)grp[i]->run->step1_out();
                    }
                    step1_batch<double>(*grp[0]->h->mech->d64, w, vu, zu, nb, s1);
                }
                if (nb > 1) {
                    PS_HIP(hipEventRecord(bev, bst));
                    for (Request *r : grp) PS_HIP(hipStreamWaitEvent(r->st, bev, 0));
                    batch_launches += 1;
                    batch_requests += nb;
                }
                for (Request *r : grp) r->run->finish_iteration();
                return PS_OK;
            });
            if (code != PS_OK) {
                // the group's requests end with the error; they leave the active set
                for (Request *r : grp) {
                    still.erase(std::remove(still.begin(), still.end(), r), still.end());
                    finish(r, code, nullptr);
                }
            }
        }
        active.swap(still);
        if (!progressed && !admitted.size()) {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait_for(lk, std::chrono::microseconds(20), [&] { return stop || !queue.empty(); });
        }
    }
}

// ====================================================================== host setup ABI
struct ps_host_setup {
    System sys;
    Options opt;
    Hierarchy sdc;
    FlowSetup flow;
};

extern "C" {

int ps_host_setup_create(const ps_system *sys, const ps_options *opts, ps_host_setup **out) {
    return guard([&] {
        if (!out) throw Error(PS_EINVAL, "out is NULL");
        *out = nullptr;
        auto s = std::make_unique<ps_host_setup>();
        ps_options def;
        ps_default_options(&def);
        s->opt = options_from(opts ? opts : &def);
        validate_and_copy(sys, s->sys);
        s->sdc = amg_build(sdc_matrix(s->sys), s->opt);
        build_flow(s->sys, s->opt, s->flow);
        *out = s.release();
        return PS_OK;
    });
}

void ps_host_setup_destroy(ps_host_setup *s) { delete s; }

static const Hierarchy &pick(const ps_host_setup *s, int which) {
    if (which == PS_H_SDC) return s->sdc;
    if (which == PS_H_PRES) return s->flow.pres;
    throw Error(PS_EINVAL, "which must be PS_H_SDC or PS_H_PRES");
}

int ps_host_levels(const ps_host_setup *s, int which, int32_t *nlevels) {
    return guard([&] {
        if (!s || !nlevels) throw Error(PS_EINVAL, "NULL argument");
        *nlevels = (int32_t)pick(s, which).lev.size();
        return PS_OK;
    });
}

int ps_host_level(const ps_host_setup *s, int which, int lvl, int32_t *n, int32_t *nnz, int32_t *rowptr,
                  int32_t *colind, double *vals, int8_t *cf, int32_t *nc, int32_t *p_nnz, int32_t *p_rowptr,
                  int32_t *p_colind, double *p_vals) {
    return guard([&] {
        if (!s) throw Error(PS_EINVAL, "NULL argument");
        const Hierarchy &H = pick(s, which);
        if (lvl < 0 || lvl >= (int)H.lev.size()) throw Error(PS_EINVAL, "level out of range");
        const Level &L = H.lev[lvl];
        if (n) *n = L.A.n;
        if (nnz) *nnz = L.A.nnz();
        if (rowptr) std::memcpy(rowptr, L.A.rp.data(), L.A.rp.size() * sizeof(int32_t));
        if (colind) std::memcpy(colind, L.A.ci.data(), L.A.ci.size() * sizeof(int32_t));
        if (vals) std::memcpy(vals, L.A.v.data(), L.A.v.size() * sizeof(double));
        if (cf) std::memcpy(cf, L.cf.data(), L.cf.size());
        if (nc) *nc = L.P.m;
        if (p_nnz) *p_nnz = L.P.nnz();
        if (p_rowptr && !L.P.rp.empty()) std::memcpy(p_rowptr, L.P.rp.data(), L.P.rp.size() * sizeof(int32_t));
        if (p_colind) std::memcpy(p_colind, L.P.ci.data(), L.P.ci.size() * sizeof(int32_t));
        if (p_vals) std::memcpy(p_vals, L.P.v.data(), L.P.v.size() * sizeof(double));
        return PS_OK;
    });
}

int ps_host_level_lambda(const ps_host_setup *s, int which, int lvl, double *lam) {
    return guard([&] {
        if (!s || !lam) throw Error(PS_EINVAL, "NULL argument");
        const Hierarchy &H = pick(s, which);
        if (lvl < 0 || lvl >= (int)H.lev.size()) throw Error(PS_EINVAL, "level out of range");
        *lam = H.lev[lvl].lam;
        return PS_OK;
    });
}

int ps_host_spp(const ps_host_setup *s, double *vals) {
    return guard([&] {
        if (!s || !vals) throw Error(PS_EINVAL, "NULL argument");
        std::memcpy(vals, s->flow.Spp.v.data(), s->flow.Spp.v.size() * sizeof(double));
        return PS_OK;
    });
}

int ps_host_bilu(const ps_host_setup *s, double *vals) {
    return guard([&] {
        if (!s || !vals) throw Error(PS_EINVAL, "NULL argument");
        if (s->opt.ml_kind != PS_BILU0) throw Error(PS_EINVAL, "setup was not built with PS_BILU0");
        std::memcpy(vals, s->flow.ml.v.data(), s->flow.ml.v.size() * sizeof(double));
        return PS_OK;
    });
}

int ps_host_bilu_levels(const ps_host_setup *s, int32_t *fwd, int32_t *bwd) {
    return guard([&] {
        if (!s || !fwd || !bwd) throw Error(PS_EINVAL, "NULL argument");
        *fwd = s->flow.sched.fwd_ptr.empty() ? 0 : (int32_t)s->flow.sched.fwd_ptr.size() - 1;
        *bwd = s->flow.sched.bwd_ptr.empty() ? 0 : (int32_t)s->flow.sched.bwd_ptr.size() - 1;
        return PS_OK;
    });
}

}  // extern "C"
