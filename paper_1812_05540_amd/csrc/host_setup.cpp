// Setup phase of the two-stage preconditioner on the host (paper Sec. 5.4).
//
// Floating-point expressions here are evaluated in a fixed order with no fused
// multiply-add contraction (built with -ffp-contract=off): every sum runs in
// increasing column order from 0.0, so the hierarchy is reproducible bit for bit.
#include "host_setup.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <mutex>
#include <functional>
#include <condition_variable>
#include <numeric>
#include <thread>

namespace ps {

namespace {
bool trace_on() {
    static const bool on = [] {
        const char *e = std::getenv("PS_TRACE");
        return e && *e && *e != '0';
    }();
    return on;
}
struct Tick {
    const char *what;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    explicit Tick(const char *w) : what(w) {}
    ~Tick() {
        if (!trace_on()) return;
        double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        std::fprintf(stderr, "[ps]   %-26s %8.2f ms\n", what, ms);
    }
};
// Row-range parallelism for the setup: each row's arithmetic is independent of the
// split, so results do not depend on the thread count.
int setup_threads() {
    static const int n = [] {
        const char *e = std::getenv("PS_THREADS");
        int v = e ? std::atoi(e) : (int)std::thread::hardware_concurrency();
        return std::max(1, std::min(v, 16));
    }();
    return n;
}

// Persistent worker threads for parallel_rows: starting 16 threads per parallel loop
// costs about as much as the loops of the setup themselves.  Workers spin briefly on a
// generation counter, then sleep on a condition variable.  One loop at a time uses the
// pool; a loop started while it is busy (the local-stage factorisation runs beside the
// pressure AMG) starts its own threads.
class Pool {
  public:
    explicit Pool(int n) : n_(n) {
        for (int t = 1; t < n_; ++t) th_.emplace_back([this, t] { worker(t); });
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            gen_.fetch_add(1);
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    int size() const { return n_; }
    std::mutex busy;
    // run job(p) for p = 0 .. parts-1 (parts <= size()); the caller runs part 0
    void run(int parts, const std::function<void(int)> &job) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            job_ = &job;
            parts_ = parts;
            left_.store(parts - 1);
            gen_.fetch_add(1);
        }
        cv_.notify_all();
        job(0);
        while (left_.load(std::memory_order_acquire) > 0) std::this_thread::yield();
    }

  private:
    void worker(int t) {
        unsigned long long seen = 0;
        for (;;) {
            unsigned long long g;
            for (int spin = 0; (g = gen_.load(std::memory_order_acquire)) == seen && spin < 20000; ++spin) {
            }
            if (g == seen) {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return gen_.load() != seen; });
            }
            // generation, job and part count are read together under the lock, so a
            // worker runs each generation's part at most once (a run cannot start
            // before every part of the previous one has finished)
            const std::function<void(int)> *job;
            int parts;
            {
                std::lock_guard<std::mutex> lk(mu_);
                if (stop_) return;
                seen = gen_.load();
                job = job_;
                parts = parts_;
            }
            if (t < parts) {
                (*job)(t);
                left_.fetch_sub(1, std::memory_order_acq_rel);
            }
        }
    }
    int n_;
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::atomic<unsigned long long> gen_{0};
    std::atomic<int> left_{0};
    const std::function<void(int)> *job_ = nullptr;
    int parts_ = 0;
    bool stop_ = false;
};

Pool &pool() {
    static Pool p(setup_threads());
    return p;
}

template <class F>
void parallel_rows(int n, F &&f) {           // f(begin, end, part)
    int parts = std::min(setup_threads(), std::max(1, n / 8192));
    if (parts <= 1) {
        f(0, n, 0);
        return;
    }
    auto range = [n, parts](int p, int &b, int &e) {
        b = (int)((long long)n * p / parts);
        e = (int)((long long)n * (p + 1) / parts);
    };
    Pool &P = pool();
    std::unique_lock<std::mutex> lk(P.busy, std::try_to_lock);
    if (lk.owns_lock()) {
        std::function<void(int)> job = [&](int p) {
            int b, e;
            range(p, b, e);
            f(b, e, p);
        };
        P.run(parts, job);
        return;
    }
    std::vector<std::thread> th;
    for (int p = 1; p < parts; ++p) {
        int b, e;
        range(p, b, e);
        th.emplace_back([&f, b, e, p] { f(b, e, p); });
    }
    int b, e;
    range(0, b, e);
    f(b, e, 0);
    for (auto &t : th) t.join();
}

// A team of host threads that runs f(tid, nthreads, team) once per thread; team.sync()
// is a barrier (spins briefly, then yields).  Used for level-by-level work where the
// levels are too small to pay for a thread launch each.
class Team {
    std::atomic<int> count_{0}, phase_{0};
    int n_;

public:
    explicit Team(int n) : n_(n) {}
    void sync() {
        int ph = phase_.load(std::memory_order_acquire);
        if (count_.fetch_add(1, std::memory_order_acq_rel) + 1 == n_) {
            count_.store(0, std::memory_order_relaxed);
            phase_.store(ph + 1, std::memory_order_release);
            return;
        }
        for (int spin = 0; phase_.load(std::memory_order_acquire) == ph; ++spin)
            if (spin > 256) std::this_thread::yield();
    }
    template <class F>
    static void run(int n, F &&f) {
        Team team(n);
        if (n <= 1) {
            f(0, 1, team);
            return;
        }
        std::vector<std::thread> th;
        for (int t = 1; t < n; ++t) th.emplace_back([&f, &team, t, n] { f(t, n, team); });
        f(0, n, team);
        for (auto &x : th) x.join();
    }
};

// Copy a vector of trivially copyable values on the setup threads.
template <class T>
void parallel_copy(const std::vector<T> &src, std::vector<T> &dst) {
    dst.resize(src.size());
    parallel_rows((int)std::min<size_t>(src.size(), 1u << 30), [&](int b, int e, int) {
        std::memcpy(dst.data() + b, src.data() + b, sizeof(T) * (size_t)(e - b));
    });
}

}  // namespace

void parallel_for(int n, const std::function<void(int, int, int)> &f) { parallel_rows(n, f); }
int setup_thread_count() { return setup_threads(); }

namespace {
// Concatenate per-part CSR pieces (row ranges in order) into one matrix.
struct CsrPart {
    std::vector<int> len, ci;
    std::vector<double> v;
};
void concat_parts(std::vector<CsrPart> &parts, Csr &C) {
    size_t nnz = 0;
    for (auto &p : parts) nnz += p.ci.size();
    C.ci.resize(nnz);
    C.v.resize(nnz);
    size_t off = 0;
    int row = 0;
    C.rp[0] = 0;
    for (auto &p : parts) {
        std::copy(p.ci.begin(), p.ci.end(), C.ci.begin() + off);
        std::copy(p.v.begin(), p.v.end(), C.v.begin() + off);
        off += p.ci.size();
        for (int l : p.len) {
            C.rp[row + 1] = C.rp[row] + l;
            ++row;
        }
    }
}
}  // namespace

Options options_from(const ps_options *o) {
    Options r;
    if (!o) return r;
    r.precision = o->precision;
    r.restart = o->restart;
    r.maxit = o->maxit;
    r.smoother = o->smoother;
    r.ml_kind = o->ml_kind;
    r.ml_sweeps = o->ml_sweeps;
    r.coarse_max = o->coarse_max;
    r.max_levels = o->max_levels;
    r.fp32_fallback = o->fp32_fallback;
    r.theta = o->theta;
    r.method = o->method;
    r.reduction = o->reduction;
    r.fixed_stress = o->fixed_stress;
    r.fs_iters = o->fs_iters;
    r.orth = o->orth;
    if (r.precision != PS_FP64 && r.precision != PS_FP32_PREC) throw Error(PS_EINVAL, "precision");
    if (r.method != PS_FGMRES && r.method != PS_RICHARDSON) throw Error(PS_EINVAL, "method");
    if (r.reduction != PS_QUASI_IMPES && r.reduction != PS_TRUE_IMPES) throw Error(PS_EINVAL, "reduction");
    if (r.fixed_stress != PS_FS_GIVEN && r.fixed_stress != PS_FS_RSL) throw Error(PS_EINVAL, "fixed_stress");
    if (r.fs_iters < 1 || r.fs_iters > 100) throw Error(PS_EINVAL, "fs_iters must be in 1..100");
    if (r.orth != PS_CGS2 && r.orth != PS_DCGS2) throw Error(PS_EINVAL, "orth must be PS_CGS2 or PS_DCGS2");
    if (r.restart < 1 || r.restart > 200) throw Error(PS_EINVAL, "restart must be in 1..200");
    if (r.maxit < 1) throw Error(PS_EINVAL, "maxit must be positive");
    if (r.smoother != PS_CHEB2 && r.smoother != PS_L1JAC) throw Error(PS_EINVAL, "smoother");
    if (r.ml_kind != PS_BILU0 && r.ml_kind != PS_BJACOBI && r.ml_kind != PS_MCGS)
        throw Error(PS_EINVAL, "ml_kind");
    if (r.ml_sweeps < 1 || r.ml_sweeps > 16) throw Error(PS_EINVAL, "ml_sweeps must be in 1..16");
    if (r.coarse_max < 1 || r.coarse_max > 6000) throw Error(PS_EINVAL, "coarse_max must be in 1..6000");
    if (r.max_levels < 1 || r.max_levels > 40) throw Error(PS_EINVAL, "max_levels must be in 1..40");
    if (!(r.theta > 0.0 && r.theta <= 1.0)) throw Error(PS_EINVAL, "theta must be in (0, 1]");
    return r;
}

// ---------------------------------------------------------------- validation
static void copy_bsr(const ps_bsr &b, int nbr, int nbc, int br, int bc, bool need_diag,
                     const char *name, Bsr &out) {
    auto fail = [&](const std::string &m) { throw Error(PS_EINVAL, std::string(name) + ": " + m); };
    if (b.nbrows != nbr || b.nbcols != nbc) fail("wrong block dimensions");
    if (b.br != br || b.bc != bc) fail("wrong block size");
    if (b.nblocks < 0) fail("negative nblocks");
    if (!b.rowptr) fail("rowptr is NULL");
    if (b.nblocks > 0 && (!b.colind || !b.vals)) fail("colind/vals is NULL");
    out.nbr = nbr;
    out.nbc = nbc;
    out.br = br;
    out.bc = bc;
    out.rp.assign(b.rowptr, b.rowptr + nbr + 1);
    if (out.rp[0] != 0 || out.rp[nbr] != b.nblocks) fail("rowptr must start at 0 and end at nblocks");
    for (int i = 0; i < nbr; ++i)
        if (out.rp[i + 1] < out.rp[i]) fail("rowptr not non-decreasing");
    out.ci.assign(b.colind, b.colind + b.nblocks);
    size_t nv = (size_t)b.nblocks * br * bc;
    out.v.assign(b.vals, b.vals + nv);
    for (int i = 0; i < nbr; ++i) {
        bool has_diag = false;
        for (int t = out.rp[i]; t < out.rp[i + 1]; ++t) {
            int c = out.ci[t];
            if (c < 0 || c >= nbc) fail("column index out of range");
            if (t > out.rp[i] && c <= out.ci[t - 1]) fail("columns not sorted/unique");
            if (c == i) has_diag = true;
        }
        if (need_diag && !has_diag) fail("missing diagonal block");
    }
    for (size_t k = 0; k < nv; ++k)
        if (!std::isfinite(out.v[k])) fail("non-finite value");
}

void validate_and_copy(const ps_system *s, System &out) {
    if (!s) throw Error(PS_EINVAL, "system is NULL");
    if (s->nf != 2 && s->nf != 3) throw Error(PS_EINVAL, "nf must be 2 or 3");
    if (s->p_index != s->nf - 1) throw Error(PS_EINVAL, "p_index must be nf-1");
    if (s->n_nodes <= 0 || s->n_cells <= 0) throw Error(PS_EINVAL, "empty system");
    if ((int64_t)3 * s->n_nodes + (int64_t)s->nf * s->n_cells > INT32_MAX / 2)
        throw Error(PS_EINVAL, "system too large for 32-bit indices");
    out.n_nodes = s->n_nodes;
    out.n_cells = s->n_cells;
    out.nf = s->nf;
    out.mech_key = s->mech_key;
    int nf = s->nf;
    copy_bsr(s->Auu, s->n_nodes, s->n_nodes, 3, 3, true, "Auu", out.Auu);
    copy_bsr(s->Auf, s->n_nodes, s->n_cells, 3, nf, false, "Auf", out.Auf);
    copy_bsr(s->Afu, s->n_cells, s->n_nodes, nf, 3, false, "Afu", out.Afu);
    copy_bsr(s->Aff, s->n_cells, s->n_cells, nf, nf, true, "Aff", out.Aff);
    if (!s->d_sp || !s->d_pp) throw Error(PS_EINVAL, "d_sp/d_pp is NULL");
    out.d_sp.assign(s->d_sp, s->d_sp + (size_t)s->n_cells * (nf - 1));
    out.d_pp.assign(s->d_pp, s->d_pp + s->n_cells);
    for (double v : out.d_sp)
        if (!std::isfinite(v)) throw Error(PS_EINVAL, "d_sp: non-finite value");
    for (double v : out.d_pp)
        if (!std::isfinite(v)) throw Error(PS_EINVAL, "d_pp: non-finite value");
    out.ml_part.clear();
    if (s->ml_part) {
        out.ml_part.assign(s->ml_part, s->ml_part + s->n_cells);
        for (int v : out.ml_part)
            if (v < 0) throw Error(PS_EINVAL, "ml_part: negative subdomain id");
    }
}

// ---------------------------------------------------------------- small dense
bool invert_small(const double *a, double *inv, int n) {
    double m[3][6];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j) m[i][j] = j < n ? a[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(m[r][c]) > std::fabs(m[piv][c])) piv = r;
        if (m[piv][c] == 0.0 || !std::isfinite(m[piv][c])) return false;
        if (piv != c)
            for (int j = 0; j < 2 * n; ++j) std::swap(m[c][j], m[piv][j]);
        double d = m[c][c];
        for (int j = 0; j < 2 * n; ++j) m[c][j] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = m[r][c];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * n; ++j) m[r][j] -= f * m[c][j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            inv[i * n + j] = m[i][n + j];
            if (!std::isfinite(inv[i * n + j])) return false;
        }
    return true;
}

bool invert_dense(std::vector<double> a, std::vector<double> &inv, int n) {
    // LU with partial pivoting (ties -> lowest row), then solve for the identity.
    std::vector<int> piv(n);
    for (int c = 0; c < n; ++c) {
        int p = c;
        double best = std::fabs(a[(size_t)c * n + c]);
        for (int r = c + 1; r < n; ++r) {
            double v = std::fabs(a[(size_t)r * n + c]);
            if (v > best) { best = v; p = r; }
        }
        piv[c] = p;
        if (best == 0.0 || !std::isfinite(best)) return false;
        if (p != c)
            for (int j = 0; j < n; ++j) std::swap(a[(size_t)c * n + j], a[(size_t)p * n + j]);
        double d = a[(size_t)c * n + c];
        for (int r = c + 1; r < n; ++r) {
            double f = a[(size_t)r * n + c] / d;
            a[(size_t)r * n + c] = f;
            if (f == 0.0) continue;
            for (int j = c + 1; j < n; ++j) a[(size_t)r * n + j] -= f * a[(size_t)c * n + j];
        }
    }
    inv.assign((size_t)n * n, 0.0);
    std::vector<double> col(n);
    for (int k = 0; k < n; ++k) {
        std::fill(col.begin(), col.end(), 0.0);
        col[k] = 1.0;
        for (int c = 0; c < n; ++c) std::swap(col[c], col[piv[c]]);   // apply P
        for (int r = 1; r < n; ++r) {                                 // L y = P e_k
            double s = col[r];
            for (int c = 0; c < r; ++c) s -= a[(size_t)r * n + c] * col[c];
            col[r] = s;
        }
        for (int r = n - 1; r >= 0; --r) {                            // U x = y
            double s = col[r];
            for (int c = r + 1; c < n; ++c) s -= a[(size_t)r * n + c] * col[c];
            col[r] = s / a[(size_t)r * n + r];
        }
        for (int r = 0; r < n; ++r) inv[(size_t)r * n + k] = col[r];
    }
    for (double v : inv)
        if (!std::isfinite(v)) return false;
    return true;
}

// ---------------------------------------------------------------- operators
static std::vector<int> diag_positions(const Bsr &b) {
    std::vector<int> d(b.nbr, -1);
    parallel_rows(b.nbr, [&](int lo, int hi, int) {
        for (int i = lo; i < hi; ++i)
            for (int t = b.rp[i]; t < b.rp[i + 1]; ++t)
                if (b.ci[t] == i) d[i] = t;
    });
    return d;
}

void fixed_stress(const System &s, Bsr &S) {
    S.nbr = s.Aff.nbr;
    S.nbc = s.Aff.nbc;
    S.br = s.Aff.br;
    S.bc = s.Aff.bc;
    if (S.rp != s.Aff.rp) S.rp = s.Aff.rp;
    if (S.ci != s.Aff.ci) S.ci = s.Aff.ci;
    parallel_copy(s.Aff.v, S.v);
    int nf = s.nf, nn = nf * nf;
    std::vector<int> dpos = diag_positions(S);
    parallel_rows(s.n_cells, [&](int b, int e, int) {
        for (int i = b; i < e; ++i) {
            double *blk = &S.v[(size_t)dpos[i] * nn];
            for (int l = 0; l < nf - 1; ++l) blk[l * nf + nf - 1] += s.d_sp[(size_t)i * (nf - 1) + l];
            blk[(nf - 1) * nf + nf - 1] += s.d_pp[i];
        }
    });
}

Bsr fixed_stress(const System &s) {
    Bsr S;
    fixed_stress(s, S);
    return S;
}

void quasi_impes(const System &s, const Bsr &Sff, Csr &Spp, std::vector<double> &dss_inv, int reduction) {
    int nf = s.nf, nn = nf * nf, m = nf - 1, nc = s.n_cells;
    std::vector<int> dpos = diag_positions(s.Aff);
    // true-IMPES (eq. CPR_CSL): the cell blocks summed down each block column of A_ff, rows
    // in increasing order; quasi-IMPES: the diagonal cell blocks
    std::vector<double> csum;
    if (reduction == PS_TRUE_IMPES) {
        csum.assign((size_t)nc * nn, 0.0);
        for (int k = 0; k < nc; ++k)
            for (int t = s.Aff.rp[k]; t < s.Aff.rp[k + 1]; ++t) {
                double *o = &csum[(size_t)s.Aff.ci[t] * nn];
                const double *a = &s.Aff.v[(size_t)t * nn];
                for (int e = 0; e < nn; ++e) o[e] += a[e];
            }
    }
    std::vector<double> t((size_t)nc * m);
    dss_inv.assign((size_t)nc * m * m, 0.0);
    std::atomic<int> singular{0};
    parallel_rows(nc, [&](int lo, int hi, int) {
        for (int i = lo; i < hi; ++i) {
            // original A_ff (A_ss, A_ps unmodified by fixed stress)
            const double *blk = reduction == PS_TRUE_IMPES ? &csum[(size_t)i * nn] : &s.Aff.v[(size_t)dpos[i] * nn];
            if (nf == 2) {
                double dss = blk[0], dps = blk[nf * (nf - 1) + 0];
                if (dss == 0.0) { singular = 1; continue; }
                t[i] = dps / dss;
                dss_inv[i] = 1.0 / dss;
            } else {
                double a = blk[0 * nf + 0], b = blk[0 * nf + 1], c = blk[1 * nf + 0], d = blk[1 * nf + 1];
                double det = a * d - b * c;
                if (det == 0.0 || !std::isfinite(det)) { singular = 1; continue; }
                double i00 = d / det, i01 = -b / det, i10 = -c / det, i11 = a / det;
                double p0 = blk[(nf - 1) * nf + 0], p1 = blk[(nf - 1) * nf + 1];
                t[(size_t)i * 2 + 0] = p0 * i00 + p1 * i10;
                t[(size_t)i * 2 + 1] = p0 * i01 + p1 * i11;
                double *o = &dss_inv[(size_t)i * 4];
                o[0] = i00; o[1] = i01; o[2] = i10; o[3] = i11;
            }
        }
    });
    if (singular) throw Error(PS_ESINGULAR, nf == 2 ? "zero D_ss entry" : "singular D_ss block");
    Spp.n = Spp.m = nc;
    if (Spp.rp != Sff.rp) Spp.rp = Sff.rp;
    if (Spp.ci != Sff.ci) Spp.ci = Sff.ci;
    Spp.v.resize(Sff.ci.size());
    parallel_rows(nc, [&](int lo, int hi, int) {
        for (int i = lo; i < hi; ++i)
            for (int k = Sff.rp[i]; k < Sff.rp[i + 1]; ++k) {
                const double *blk = &Sff.v[(size_t)k * nn];
                double app = blk[(nf - 1) * nf + nf - 1];
                if (nf == 2) {
                    Spp.v[k] = app - t[i] * blk[0 * nf + nf - 1];
                } else {
                    double s0 = t[(size_t)i * 2 + 0] * blk[0 * nf + nf - 1];
                    double s1 = t[(size_t)i * 2 + 1] * blk[1 * nf + nf - 1];
                    Spp.v[k] = app - (s0 + s1);
                }
            }
    });
}

Csr sdc_matrix(const System &s) {
    int nn = s.n_nodes;
    const Bsr &A = s.Auu;
    Csr r;
    r.n = r.m = 3 * nn;
    r.rp.resize((size_t)3 * nn + 1);
    r.ci.reserve((size_t)3 * A.nb());
    r.v.reserve((size_t)3 * A.nb());
    r.rp[0] = 0;
    for (int c = 0; c < 3; ++c)
        for (int i = 0; i < nn; ++i) {
            for (int t = A.rp[i]; t < A.rp[i + 1]; ++t) {
                r.ci.push_back(c * nn + A.ci[t]);
                r.v.push_back(A.v[(size_t)t * 9 + c * 3 + c]);
            }
            r.rp[(size_t)c * nn + i + 1] = (int)r.ci.size();
        }
    return r;
}

// ---------------------------------------------------------------- AMG
static inline double unit_hash(uint64_t i) {
    // SplitMix64 (Steele, Lea, Flood 2014; Vigna's finaliser constants) seeded with i.
    uint64_t z = i + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * 0x1.0p-53;
}

static std::vector<char> strength(const Csr &A, double theta) {
    std::vector<char> s(A.ci.size(), 0);
    parallel_rows(A.n, [&](int b, int e, int) {
        for (int i = b; i < e; ++i) {
            double m = -INFINITY;
            for (int t = A.rp[i]; t < A.rp[i + 1]; ++t)
                if (A.ci[t] != i) m = std::max(m, -A.v[t]);
            if (!(m > 0.0)) continue;
            double thr = theta * m;
            for (int t = A.rp[i]; t < A.rp[i + 1]; ++t)
                if (A.ci[t] != i && -A.v[t] >= thr) s[t] = 1;
        }
    });
    return s;
}

static Csr transpose(const Csr &P);

static std::vector<int8_t> pmis(const Csr &A, const std::vector<char> &smask) {
    const int n = A.n;
    // S rows (i depends on j) and their transpose
    Csr S;
    S.n = S.m = n;
    S.rp.assign(n + 1, 0);
    parallel_rows(n, [&](int b, int e, int) {
        for (int i = b; i < e; ++i) {
            int c = 0;
            for (int t = A.rp[i]; t < A.rp[i + 1]; ++t) c += smask[t] != 0;
            S.rp[i + 1] = c;
        }
    });
    for (int i = 0; i < n; ++i) S.rp[i + 1] += S.rp[i];
    S.ci.resize(S.rp[n]);
    S.v.assign(S.rp[n], 0.0);
    parallel_rows(n, [&](int b, int e, int) {
        for (int i = b; i < e; ++i)
            for (int t = A.rp[i], k = S.rp[i]; t < A.rp[i + 1]; ++t)
                if (smask[t]) S.ci[k++] = A.ci[t];
    });
    Csr T = transpose(S);
    const std::vector<int> &srp = S.rp, &sci = S.ci, &trp = T.rp, &tci = T.ci;
    std::vector<int> lam(n);
    std::vector<double> w(n);
    parallel_rows(n, [&](int b, int e, int) {
        for (int i = b; i < e; ++i) {
            lam[i] = trp[i + 1] - trp[i];
            w[i] = (double)lam[i] + unit_hash((uint64_t)i);
        }
    });
    std::vector<int8_t> st(n, 0);
    size_t undecided = 0;
    for (int i = 0; i < n; ++i) {
        if (lam[i] == 0) st[i] = -1;
        else ++undecided;
    }
    std::vector<char> newc(n, 0);
    std::vector<int> und;
    und.reserve(n);
    for (int i = 0; i < n; ++i)
        if (st[i] == 0) und.push_back(i);
    auto beats = [&](int j, int i) { return w[j] > w[i] || (w[j] == w[i] && j > i); };
    // Each round reads the state at its start only, so rows are independent within
    // a round and the result does not depend on the split.
    while (!und.empty()) {
        const int nu = (int)und.size();
        parallel_rows(nu, [&](int b, int e, int) {
            for (int q = b; q < e; ++q) {
                int i = und[q];
                bool beaten = false;
                for (int k = srp[i]; k < srp[i + 1] && !beaten; ++k) {
                    int j = sci[k];
                    if (st[j] == 0 && beats(j, i)) beaten = true;
                }
                for (int k = trp[i]; k < trp[i + 1] && !beaten; ++k) {
                    int j = tci[k];
                    if (st[j] == 0 && beats(j, i)) beaten = true;
                }
                newc[i] = !beaten;
            }
        });
        for (int i : und)
            if (newc[i]) st[i] = 1;
        parallel_rows(nu, [&](int b, int e, int) {
            for (int q = b; q < e; ++q) {
                int i = und[q];
                if (st[i] != 0) continue;
                for (int k = srp[i]; k < srp[i + 1]; ++k)
                    if (newc[sci[k]]) { st[i] = -1; break; }
            }
        });
        for (int i : und) newc[i] = 0;
        std::vector<int> next;
        next.reserve(und.size());
        for (int i : und)
            if (st[i] == 0) next.push_back(i);
        und.swap(next);
    }
    // C-promotion, sequential in increasing i
    for (int i = 0; i < n; ++i) {
        if (st[i] != -1 || srp[i + 1] == srp[i]) continue;
        bool hasc = false;
        for (int k = srp[i]; k < srp[i + 1]; ++k)
            if (st[sci[k]] == 1) { hasc = true; break; }
        if (!hasc) st[i] = 1;
    }
    return st;
}

static Csr direct_interpolation(const Csr &A, const std::vector<char> &smask,
                                const std::vector<int8_t> &cf, int &nc) {
    const int n = A.n;
    std::vector<int> cidx(n, -1);
    nc = 0;
    for (int i = 0; i < n; ++i)
        if (cf[i] == 1) cidx[i] = nc++;
    Csr P;
    P.n = n;
    P.m = nc;
    P.rp.assign(n + 1, 0);
    int nparts = std::min(setup_threads(), std::max(1, n / 8192));
    std::vector<CsrPart> parts(nparts);
    parallel_rows(n, [&](int b, int e, int part) {
    CsrPart &out = parts[part];
    for (int i = b; i < e; ++i) {
        int before = (int)out.ci.size();
        if (cf[i] == 1) {
            out.ci.push_back(cidx[i]);
            out.v.push_back(1.0);
        } else {
            double diag = 0.0, pos = 0.0, negs = 0.0, den = 0.0;
            for (int t = A.rp[i]; t < A.rp[i + 1]; ++t) {
                int j = A.ci[t];
                double a = A.v[t];
                if (j == i) { diag = a; continue; }
                if (a > 0.0) pos += a;
                if (a < 0.0) negs += a;
                if (smask[t] && cf[j] == 1) den += a;
            }
            double atil = diag + pos;
            double alpha = den != 0.0 ? negs / den : 0.0;
            for (int t = A.rp[i]; t < A.rp[i + 1]; ++t) {
                int j = A.ci[t];
                if (j != i && smask[t] && cf[j] == 1) {
                    out.ci.push_back(cidx[j]);
                    out.v.push_back(-(alpha * A.v[t]) / atil);
                }
            }
        }
        out.len.push_back((int)out.ci.size() - before);
    }
    });
    concat_parts(parts, P);
    return P;
}

static Csr transpose(const Csr &P) {
    Csr R;
    R.n = P.m;
    R.m = P.n;
    R.rp.assign(R.n + 1, 0);
    R.ci.resize(P.ci.size());
    R.v.resize(P.ci.size());
    const int parts = std::min(setup_threads(), std::max(1, P.n / 8192));
    // cnt[p][c]: entries of column c in row range p; prefix over (c, p) gives each
    // part its write position, so rows stay in increasing order within each column
    std::vector<std::vector<int>> cnt(parts, std::vector<int>(R.n, 0));
    auto range = [&](int p, int &b, int &e) {
        b = (int)((long long)P.n * p / parts);
        e = (int)((long long)P.n * (p + 1) / parts);
    };
    std::vector<std::thread> th;
    auto count = [&](int p) {
        int b, e;
        range(p, b, e);
        for (int t = P.rp[b]; t < P.rp[e]; ++t) ++cnt[p][P.ci[t]];
    };
    for (int p = 1; p < parts; ++p) th.emplace_back(count, p);
    count(0);
    for (auto &x : th) x.join();
    th.clear();
    int off = 0;
    for (int c = 0; c < R.n; ++c) {
        R.rp[c] = off;
        for (int p = 0; p < parts; ++p) {
            int k = cnt[p][c];
            cnt[p][c] = off;
            off += k;
        }
    }
    R.rp[R.n] = off;
    auto fill = [&](int p) {
        int b, e;
        range(p, b, e);
        std::vector<int> &pos = cnt[p];
        for (int i = b; i < e; ++i)
            for (int t = P.rp[i]; t < P.rp[i + 1]; ++t) {
                int k = pos[P.ci[t]]++;
                R.ci[k] = i;
                R.v[k] = P.v[t];
            }
    };
    for (int p = 1; p < parts; ++p) th.emplace_back(fill, p);
    fill(0);
    for (auto &x : th) x.join();
    return R;
}

// C = A B; each entry accumulated in increasing order of the inner index starting
// from 0.0; exact zeros dropped; columns sorted.
static Csr spgemm(const Csr &A, const Csr &B) {
    Csr C;
    C.n = A.n;
    C.m = B.m;
    C.rp.assign(A.n + 1, 0);
    int nparts = std::min(setup_threads(), std::max(1, A.n / 8192));
    std::vector<CsrPart> parts(nparts);
    parallel_rows(A.n, [&](int b, int e, int p) {
        CsrPart &out = parts[p];
        std::vector<double> acc(B.m, 0.0);
        std::vector<int> mark(B.m, -1), cols;
        out.len.reserve(e - b);
        for (int i = b; i < e; ++i) {
            cols.clear();
            for (int t = A.rp[i]; t < A.rp[i + 1]; ++t) {
                int l = A.ci[t];
                double a = A.v[t];
                for (int u = B.rp[l]; u < B.rp[l + 1]; ++u) {
                    int k = B.ci[u];
                    if (mark[k] != i) { mark[k] = i; acc[k] = 0.0; cols.push_back(k); }
                    acc[k] += a * B.v[u];
                }
            }
            std::sort(cols.begin(), cols.end());
            int c = 0;
            for (int k : cols)
                if (acc[k] != 0.0) { out.ci.push_back(k); out.v.push_back(acc[k]); ++c; }
            out.len.push_back(c);
        }
    });
    concat_parts(parts, C);
    return C;
}

static double norm2(const std::vector<double> &v) {
    double s = 0.0;
    for (double x : v) s += x * x;
    return std::sqrt(s);
}

static void smoother_setup(Level &L, int kind) {
    const Csr &A = L.A;
    const int n = A.n;
    L.diag.assign(n, 0.0);
    L.dl1.assign(n, 0.0);
    std::vector<char> iso(n, 1);
    std::atomic<int> zero{0};
    parallel_rows(n, [&](int b, int e, int) {
        for (int i = b; i < e; ++i) {
            double s = 0.0;
            for (int t = A.rp[i]; t < A.rp[i + 1]; ++t) {
                if (A.ci[t] == i) { L.diag[i] = A.v[t]; continue; }
                s += std::fabs(A.v[t]);
                if (A.v[t] != 0.0) iso[i] = 0;
            }
            L.dl1[i] = L.diag[i] + s;
            if (L.diag[i] == 0.0) zero = 1;
        }
    });
    if (zero) throw Error(PS_ESINGULAR, "zero diagonal in an AMG level");
    if (kind == PS_L1JAC) return;
    // power iteration for the largest eigenvalue of D^-1 A
    std::vector<double> v(n), wv(n);
    for (int i = 0; i < n; ++i) v[i] = 1.0 + unit_hash((uint64_t)i);
    double nv = norm2(v);
    for (int i = 0; i < n; ++i) v[i] = v[i] / nv;
    double lam = 0.0;
    for (int it = 0; it < 10; ++it) {
        parallel_rows(n, [&](int b, int e, int) {
            for (int i = b; i < e; ++i) {
                double s = 0.0;
                for (int t = A.rp[i]; t < A.rp[i + 1]; ++t) s += A.v[t] * v[A.ci[t]];
                wv[i] = s / L.diag[i];
            }
        });
        lam = norm2(wv);
        for (int i = 0; i < n; ++i) v[i] = wv[i] / lam;
    }
    lam = 1.1 * lam;
    double lo = 0.3 * lam, hi = lam;
    double theta = (hi + lo) / 2.0, delta = (hi - lo) / 2.0;
    double sigma = theta / delta;
    double rho0 = 1.0 / sigma;
    double rho1 = 1.0 / (2.0 * sigma - rho0);
    L.lam = lam;
    L.c0.resize(n);
    L.c1.resize(n);
    L.cm.resize(n);
    for (int i = 0; i < n; ++i) {
        double d = L.diag[i];
        if (iso[i]) {
            L.c0[i] = 1.0 / d;
            L.cm[i] = 0.0;
            L.c1[i] = 0.0;
        } else {
            L.c0[i] = 1.0 / (theta * d);
            L.cm[i] = rho1 * rho0;
            L.c1[i] = 2.0 * rho1 / (delta * d);
        }
    }
}

bool coarsen_level(const Csr &A, const Options &o, Level &L) {
    std::vector<char> smask;
    {
        Tick t("strength + PMIS");
        smask = strength(A, o.theta);
        L.cf = pmis(A, smask);
    }
    int nc = 0;
    for (int8_t c : L.cf) nc += (c == 1);
    if (nc == 0 || (double)nc > 0.9 * (double)A.n) return false;
    Tick t("interpolation");
    L.P = direct_interpolation(A, smask, L.cf, nc);
    L.R = transpose(L.P);
    return true;
}

Csr galerkin(const Level &L, const Csr &A) { return spgemm(L.R, spgemm(A, L.P)); }

void finish_level(Level &L, int smoother) {
    Tick t("smoother setup");
    smoother_setup(L, smoother);
}

void coarse_level(Csr A, Hierarchy &H) {
    if (A.n > 6000) throw Error(PS_ESINGULAR, "AMG coarsening stagnated above the dense-solve limit");
    Level C;
    C.cf.assign(A.n, 0);
    std::vector<double> dense((size_t)A.n * A.n, 0.0);
    for (int i = 0; i < A.n; ++i)
        for (int t = A.rp[i]; t < A.rp[i + 1]; ++t) dense[(size_t)i * A.n + A.ci[t]] = A.v[t];
    if (!invert_dense(dense, H.coarse_inv, A.n)) throw Error(PS_ESINGULAR, "singular coarsest AMG matrix");
    H.coarse_n = A.n;
    C.A = std::move(A);
    H.lev.push_back(std::move(C));
}

Hierarchy amg_build(const Csr &A0, const Options &o) {
    Hierarchy H;
    Csr A = A0;
    while (A.n > o.coarse_max && (int)H.lev.size() + 1 < o.max_levels) {
        Level L;
        if (!coarsen_level(A, o, L)) break;
        Csr Ac;
        {
            Tick t("Galerkin RAP (host)");
            Ac = galerkin(L, A);
        }
        L.A = std::move(A);
        finish_level(L, o.smoother);
        H.lev.push_back(std::move(L));
        A = std::move(Ac);
    }
    coarse_level(std::move(A), H);
    return H;
}

// ---------------------------------------------------------------- local stage
static inline void mm(const double *a, const double *b, double *c, int n) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += a[i * n + k] * b[k * n + j];
            c[i * n + j] = s;
        }
}

// IKJ block ILU(0) of F in place.  A row of one forward level depends only on rows of
// earlier levels, so each level is factored by the whole thread team; the arithmetic
// of every row is the same as in row-by-row order.
void bilu0_factor_inplace(Bsr &F, const BiluSchedule &sc) {
    const int n = F.nbr, nf = F.br, nn = nf * nf;
    std::vector<int> dpos = diag_positions(F);
    std::atomic<int> singular{0};
    const int nt = std::min(setup_threads(), std::max(1, n / 4096));
    Team::run(nt, [&](int tid, int nthr, Team &team) {
        std::vector<int> pos(n, -1);
        double tmp[9], prod[9];
        for (size_t l = 0; l + 1 < sc.fwd_ptr.size(); ++l) {
            const int lb = sc.fwd_ptr[l], le = sc.fwd_ptr[l + 1];
            const int b = lb + (int)((long long)(le - lb) * tid / nthr);
            const int e = lb + (int)((long long)(le - lb) * (tid + 1) / nthr);
            for (int q = b; q < e; ++q) {
                const int i = sc.fwd_rows[q];
                for (int t = F.rp[i]; t < F.rp[i + 1]; ++t) pos[F.ci[t]] = t;
                for (int t = F.rp[i]; t < F.rp[i + 1]; ++t) {
                    int k = F.ci[t];
                    if (k >= i) break;
                    double *lik = &F.v[(size_t)t * nn];
                    mm(lik, &F.v[(size_t)dpos[k] * nn], tmp, nf);       // L_ik = A_ik D_k^-1
                    std::memcpy(lik, tmp, sizeof(double) * nn);
                    for (int u = dpos[k] + 1; u < F.rp[k + 1]; ++u) {
                        int qq = pos[F.ci[u]];
                        if (qq < 0) continue;
                        mm(lik, &F.v[(size_t)u * nn], prod, nf);          // A_ij -= L_ik U_kj
                        double *aij = &F.v[(size_t)qq * nn];
                        for (int x = 0; x < nn; ++x) aij[x] -= prod[x];
                    }
                }
                double *dblk = &F.v[(size_t)dpos[i] * nn];
                if (!invert_small(dblk, tmp, nf)) singular = 1;
                else std::memcpy(dblk, tmp, sizeof(double) * nn);     // store D_i^-1
                for (int t = F.rp[i]; t < F.rp[i + 1]; ++t) pos[F.ci[t]] = -1;
            }
            team.sync();
        }
    });
    if (singular) throw Error(PS_ESINGULAR, "singular BILU(0) pivot block");
}

void bilu0_factor(const Bsr &S, Bsr &F) {
    F = S;
    bilu0_factor_inplace(F, bilu_schedule(S));
}

void block_jacobi_factor(const Bsr &S, Bsr &F) {
    const int n = S.nbr, nf = S.br, nn = nf * nf;
    std::vector<int> dpos = diag_positions(S);
    F.nbr = F.nbc = n;
    F.br = F.bc = nf;
    F.rp.resize(n + 1);
    F.ci.resize(n);
    F.v.resize((size_t)n * nn);
    std::atomic<int> singular{0};
    parallel_rows(n, [&](int b, int e, int) {
        for (int i = b; i < e; ++i) {
            F.rp[i] = i;
            F.ci[i] = i;
            if (!invert_small(&S.v[(size_t)dpos[i] * nn], &F.v[(size_t)i * nn], nf)) singular = 1;
        }
    });
    if (singular) throw Error(PS_ESINGULAR, "singular diagonal cell block");
    F.rp[n] = n;
}

void restrict_to_parts(const Bsr &S, const std::vector<int> &part, Bsr &R) {
    R.nbr = S.nbr;
    R.nbc = S.nbc;
    R.br = S.br;
    R.bc = S.bc;
    const size_t nn = (size_t)S.br * S.bc;
    R.rp.assign(S.nbr + 1, 0);
    parallel_rows(S.nbr, [&](int b, int e, int) {
        for (int i = b; i < e; ++i) {
            int c = 0;
            for (int t = S.rp[i]; t < S.rp[i + 1]; ++t) c += part[S.ci[t]] == part[i];
            R.rp[i + 1] = c;
        }
    });
    for (int i = 0; i < S.nbr; ++i) R.rp[i + 1] += R.rp[i];
    R.ci.resize(R.rp[S.nbr]);
    R.v.resize(R.ci.size() * nn);
    parallel_rows(S.nbr, [&](int b, int e, int) {
        for (int i = b; i < e; ++i) {
            int o = R.rp[i];
            for (int t = S.rp[i]; t < S.rp[i + 1]; ++t) {
                if (part[S.ci[t]] != part[i]) continue;
                R.ci[o] = S.ci[t];
                std::memcpy(&R.v[(size_t)o * nn], &S.v[(size_t)t * nn], sizeof(double) * nn);
                ++o;
            }
        }
    });
}

Bsr restrict_to_parts(const Bsr &S, const std::vector<int> &part) {
    Bsr R;
    restrict_to_parts(S, part, R);
    return R;
}

BiluSchedule bilu_schedule(const Bsr &S) {
    const int n = S.nbr;
    std::vector<int> lf(n, 0), lb(n, 0);
    int maxf = 0, maxb = 0;
    for (int i = 0; i < n; ++i) {
        int l = 0;
        for (int t = S.rp[i]; t < S.rp[i + 1]; ++t)
            if (S.ci[t] < i) l = std::max(l, lf[S.ci[t]] + 1);
        lf[i] = l;
        maxf = std::max(maxf, l);
    }
    for (int i = n - 1; i >= 0; --i) {
        int l = 0;
        for (int t = S.rp[i]; t < S.rp[i + 1]; ++t)
            if (S.ci[t] > i) l = std::max(l, lb[S.ci[t]] + 1);
        lb[i] = l;
        maxb = std::max(maxb, l);
    }
    BiluSchedule sc;
    auto group = [n](const std::vector<int> &lv, int nl, std::vector<int> &ptr, std::vector<int> &rows) {
        ptr.assign(nl + 2, 0);
        for (int i = 0; i < n; ++i) ++ptr[lv[i] + 1];
        for (int l = 0; l <= nl; ++l) ptr[l + 1] += ptr[l];
        rows.resize(n);
        std::vector<int> fill(ptr.begin(), ptr.end() - 1);
        for (int i = 0; i < n; ++i) rows[fill[lv[i]]++] = i;
        ptr.resize(nl + 2);
    };
    group(lf, maxf, sc.fwd_ptr, sc.fwd_rows);
    group(lb, maxb, sc.bwd_ptr, sc.bwd_rows);
    return sc;
}

// Greedy colouring in increasing row order: each row takes the smallest colour not
// used by a lower-index neighbour; rows grouped by colour, increasing index within.
BiluSchedule color_schedule(const Bsr &S) {
    const int n = S.nbr;
    std::vector<int> col(n, -1), used;
    int ncol = 0;
    for (int i = 0; i < n; ++i) {
        used.clear();
        for (int t = S.rp[i]; t < S.rp[i + 1]; ++t)
            if (S.ci[t] < i) used.push_back(col[S.ci[t]]);
        int c = 0;
        while (std::find(used.begin(), used.end(), c) != used.end()) ++c;
        col[i] = c;
        ncol = std::max(ncol, c + 1);
    }
    BiluSchedule sc;
    sc.fwd_ptr.assign(ncol + 1, 0);
    for (int i = 0; i < n; ++i) ++sc.fwd_ptr[col[i] + 1];
    for (int c = 0; c < ncol; ++c) sc.fwd_ptr[c + 1] += sc.fwd_ptr[c];
    sc.fwd_rows.resize(n);
    std::vector<int> fill(sc.fwd_ptr.begin(), sc.fwd_ptr.end() - 1);
    for (int i = 0; i < n; ++i) sc.fwd_rows[fill[col[i]]++] = i;
    return sc;
}

void build_flow_operators(const System &s, const Options &o, FlowSetup &f) {
    Tick t("fixed stress + IMPES reduction");
    fixed_stress(s, f.Sff);
    quasi_impes(s, f.Sff, f.Spp, f.dss_inv, o.reduction);
}

void build_flow_local(const System &s, const Options &o, FlowSetup &f, bool pattern_only) {
    Tick t("local stage factor");
    if (o.ml_kind == PS_BILU0 && pattern_only && !f.sched.fwd_ptr.empty() && !f.ml.rp.empty()) return;
    if (o.ml_kind == PS_BILU0) {
        if (!s.ml_part.empty()) {
            restrict_to_parts(f.Sff, s.ml_part, f.ml);
        } else {
            f.ml.nbr = f.Sff.nbr;
            f.ml.nbc = f.Sff.nbc;
            f.ml.br = f.Sff.br;
            f.ml.bc = f.Sff.bc;
            if (f.ml.rp != f.Sff.rp) f.ml.rp = f.Sff.rp;
            if (f.ml.ci != f.Sff.ci) f.ml.ci = f.Sff.ci;
            parallel_copy(f.Sff.v, f.ml.v);
        }
        if (f.sched.fwd_ptr.empty()) f.sched = bilu_schedule(f.ml);    // pattern-only, kept across setups
        Tick t2("BILU(0) factor");
        bilu0_factor_inplace(f.ml, f.sched);
    } else if (o.ml_kind == PS_MCGS) {
        block_jacobi_factor(f.Sff, f.ml);
        if (f.sched.fwd_ptr.empty()) f.sched = color_schedule(f.Sff);
    } else {
        block_jacobi_factor(f.Sff, f.ml);
        f.sched = BiluSchedule();
    }
}

void build_flow(const System &s, const Options &o, FlowSetup &f) {
    build_flow_operators(s, o, f);
    {
        Tick t("pressure AMG");
        f.pres = amg_build(f.Spp, o);
    }
    build_flow_local(s, o, f);
}

}  // namespace ps
