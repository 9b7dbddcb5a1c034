// Device-side data of a handle and the solve-phase drivers (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "host_setup.h"

namespace ps {

void hip_check(hipError_t e, const char *what);
#define PS_HIP(x) ::ps::hip_check((x), #x)

// Device allocations owned by one object; freed together.  recycle() keeps the
// blocks for reuse by later alloc() calls of the same or slightly smaller size, so a
// setup that is repeated with new values does not go back to hipMalloc/hipFree.
class Arena {
  public:
    Arena() = default;
    Arena(const Arena &) = delete;
    Arena &operator=(const Arena &) = delete;
    Arena(Arena &&o) noexcept : used_(std::move(o.used_)), free_(std::move(o.free_)) {}
    Arena &operator=(Arena &&o) noexcept {
        if (this != &o) {
            release();
            used_ = std::move(o.used_);
            free_ = std::move(o.free_);
        }
        return *this;
    }
    ~Arena() { release(); }
    template <typename T>
    T *alloc(size_t n) {
        size_t bytes = ((n ? n : 1) * sizeof(T) + 255) / 256 * 256;
        size_t best = free_.size();
        for (size_t i = 0; i < free_.size(); ++i)
            if (free_[i].bytes >= bytes && free_[i].bytes <= 2 * bytes &&
                (best == free_.size() || free_[i].bytes < free_[best].bytes))
                best = i;
        if (best != free_.size()) {
            used_.push_back(free_[best]);
            free_.erase(free_.begin() + best);
            return static_cast<T *>(used_.back().p);
        }
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(PS_ENOMEM, "hipMalloc failed");
        }
        used_.push_back({p, bytes});
        return static_cast<T *>(p);
    }
    template <typename T>
    T *upload(const T *h, size_t n) {
        T *d = alloc<T>(n);
        if (n) PS_HIP(hipMemcpy(d, h, n * sizeof(T), hipMemcpyHostToDevice));
        return d;
    }
    void trim() {                                  // free the blocks not reused since recycle()
        for (auto &b : free_) (void)hipFree(b.p);
        free_.clear();
    }
    void recycle() {
        free_.insert(free_.end(), used_.begin(), used_.end());
        used_.clear();
    }
    void release() {
        for (auto &b : used_) (void)hipFree(b.p);
        for (auto &b : free_) (void)hipFree(b.p);
        used_.clear();
        free_.clear();
    }
    size_t bytes() const {
        size_t t = 0;
        for (auto &b : used_) t += b.bytes;
        for (auto &b : free_) t += b.bytes;
        return t;
    }

  private:
    struct Blk {
        void *p;
        size_t bytes;
    };
    std::vector<Blk> used_, free_;
};

// Sliced ELLPACK with 64-row chunks (one wavefront per chunk) over br x bc blocks.
// Chunk c holds slots [cptr[c], cptr[c+1]); slot k of row lane l stores its column
// at col[k*64 + l] and block element e at val[(k*br*bc + e)*64 + l], so every load
// instruction of a wavefront reads 64 consecutive words.  Padding slots have
// column 0 and zero values.  rowmap (optional) maps the sliced row position to
// the matrix row (-1 for padding rows); without it position == row.
template <typename T>
struct Sell {
    int nrows = 0, nchunks = 0, br = 1, bc = 1;
    const int *cptr = nullptr;
    const int *col = nullptr;
    const T *val = nullptr;
    const int *rowmap = nullptr;
    size_t nslots = 0;
};

struct HostSell {                 // host image of a Sell before upload
    int nrows = 0, nchunks = 0, br = 1, bc = 1;
    std::vector<int> cptr, col, rowmap;
    std::vector<double> val;
    std::vector<int> src;         // per slot and lane: source block index, -1 = padding
};

HostSell sell_from_bsr(const std::vector<int> &rp, const std::vector<int> &ci,
                       const std::vector<double> &v, int nbr, int br, int bc,
                       const std::vector<int> *row_order = nullptr,
                       bool (*keep)(int row, int col) = nullptr, bool values = true);
HostSell sell_from_csr(const Csr &A);
template <typename T>
Sell<T> upload_sell(Arena &ar, const HostSell &h);

// ---- preconditioner device data ------------------------------------------------
// FP64 CSR in device memory (the Galerkin builder's matrices).
struct DevCsr {
    int n = 0, m = 0, nnz = 0;
    int *rp = nullptr, *ci = nullptr;
    double *v = nullptr;
};

// C = A B on the device, bitwise equal to the host product (galerkin.hip).
void spgemm_device(const DevCsr &A, const DevCsr &B, DevCsr &C, Arena &out, Arena &tmp, hipStream_t st);

// Pinned host buffer for value uploads, and the (non-blocking) stream its copies use, so
// that uploads from a setup thread do not wait on work queued on the null stream.
struct Staging {
    void *p = nullptr;
    size_t bytes = 0;
    hipStream_t st = nullptr;
    void *get(size_t n);
    void copy_to_device(void *dev, const void *host, size_t n);   // returns when done
    void copy_async(void *dev, const void *host, size_t n);       // queued; see wait()
    void wait();
    hipStream_t stream();                                          // created on first use
    ~Staging();
};

// Pressure hierarchy whose Galerkin products are formed on the device: host levels in H
// (operators copied back for the next coarsening and for inspection), FP64 device copies of
// every A_l, P_l, R_l here, shared by the FP64 and FP32 preconditioners.
struct PresStore {
    Arena arena, work, tmp;
    std::vector<DevCsr> A, P, R;
    bool on_device = false;            // whole build on the device (l1-Jacobi): the host levels
                                       // in H carry sizes only; cf and dinv are here
    std::vector<signed char *> cf;     // C/F splitting per level (1 C, -1 F)
    std::vector<double *> dinv;        // l1-Jacobi 1 / (a_ii + sum |a_ij|) per level
    double *cinv = nullptr;            // dense inverse of the coarsest operator, when formed here
    // S_pp formed on the device (quasi-IMPES from the system's A_ff and the fixed-stress
    // terms) once its pattern, A_ff's block pattern, is laid out here (npat rows)
    Arena pat;                         // kept across setups
    int npat = 0, nnzpat = 0;
    int *spp_rp = nullptr, *spp_ci = nullptr, *aff_dslot = nullptr, *flag = nullptr;
    double *fs = nullptr;              // d_sp (n * (nf-1)) then d_pp (n)
    Staging stg;
};
void build_pressure(const Csr &Spp, const Options &o, Hierarchy &H, PresStore &S);
// operator and splitting of level lvl copied to the host (zeros on the coarsest level)
void download_level(const PresStore &S, int lvl, Csr &A, std::vector<int8_t> &cf);

// A level matrix on the device.  G >= 1: CSR processed by groups of G lanes per row (G a
// power of two chosen from the mean row length).  G <= 0: SELL-64, one lane per row; entry
// k of row i at (cptr[i / 64] + k) * 64 + i % 64 of ci and v (padding never read), the
// row's length from rp; G == -1: the columns stored as 16-bit offsets from the row (cd)
// instead of ci.  G > 64: CSR with G - 64 lanes per row and 16-bit column offsets (cd).  An
// operator A takes SELL-64 when its slices pad it little.
template <typename T>
struct DCsr {
    int n = 0, G = 1;
    long long nnz = 0;            // stored entries (padding excluded)
    const int *rp = nullptr, *ci = nullptr;
    const T *v = nullptr;
    const int *cptr = nullptr;    // SELL-64 only: first slot of each 64-row slice
    const short *cd = nullptr;    // G == -1 or G > 64: column - row per stored entry
};

template <typename T>
struct DLevel {                   // matrices and per-row constants of one AMG level
    int n = 0;
    DCsr<T> A, P, R;
    const T *dinv = nullptr;      // l1-Jacobi: 1 / (a_ii + sum |a_ij|)
    const T *c0 = nullptr, *c1 = nullptr, *cm = nullptr;   // Chebyshev
};

template <typename T>
struct DHierarchy {
    std::vector<DLevel<T>> lev;   // coarsest last (only n used there)
    const double *cinv = nullptr; // dense inverse of the coarsest operator (FP64)
    int cn = 0;
    int smoother = PS_CHEB2;
    int ktag = -1;                // ktime id of level 0's first phase (SDC_PRE / PRES_PRE), -1: none
    Arena arena;
    size_t bytes() const { return arena.bytes(); }
};

template <typename T>
struct HierWork {                 // per-handle vectors of one hierarchy
    std::vector<T *> x, x1, d, r; // smoother iterate, temp, Chebyshev step, residual
    std::vector<T *> b, e;        // right-hand side and result of level l >= 1
};

// Processor-local BILU(0) with each subdomain's vector resident in LDS (one workgroup per
// subdomain; see the bilu_sub kernel for the layout).
template <typename T>
struct SubBilu {
    int N = 0, nsub = 0, W = 0, bs = 0, lev_cap = 0;
    double bytes = 0.0;                   // algorithmic bytes of one application
    size_t lds = 0;
    T *ygl = nullptr;                     // vectors in HBM when a subdomain's does not fit in LDS
    const int *sub_off = nullptr, *flev_off = nullptr, *blev_off = nullptr, *flev = nullptr, *blev = nullptr,
              *bpos = nullptr, *ncell = nullptr, *npos = nullptr, *fcol = nullptr, *bcol = nullptr;
    T *fval = nullptr, *bval = nullptr, *bdinv = nullptr;
    std::vector<int> fsrc, bsrc, dsrc;    // value source blocks (host), -1 = padding
    std::vector<int> ford;                // cell of each forward position (host)
    // The factorization on the device (when S_ff's values are formed there): per factor
    // block its A_ff SELL position and, for a diagonal block, its cell (else -1); per
    // forward position r, the diagonal block, and for each strict-lower block k (slot
    // k*N + r, -1 past the row's end) the diagonal block of its column row and the matched
    // updates (slot (k*W + m)*N + r): block u of that row's upper part and block q of row r.
    bool dev_factor = false;
    int nml = 0;
    const int *ml_src = nullptr, *ml_fs = nullptr, *fdiag = nullptr, *lo_t = nullptr, *lo_d = nullptr,
              *up_u = nullptr, *up_q = nullptr, *d_fsrc = nullptr, *d_bsrc = nullptr, *d_dsrc = nullptr;
    double *fv = nullptr;                 // FP64 factor values, nml blocks
    int *flag = nullptr;                  // set when a pivot block is singular
};

template <typename T>
struct DFlow {                    // flow stage of Algorithm 1 on the device
    int nc = 0, nf = 0, ml_kind = PS_BILU0, ml_sweeps = 1;
    bool layout = false;          // patterns fixed for the life of a handle
    Sell<T> Afu, Sff;             // nf x 3 and nf x nf
    Sell<T> Lf, Ub;               // BILU strict lower / upper blocks in level order (block GS:
                                  // Lf = all S_ff blocks in colour order)
    T *afu_val = nullptr, *sff_val = nullptr, *lf_val = nullptr, *ub_val = nullptr;
    std::vector<int> src_afu, src_sff, src_lf, src_ub;   // value source maps (host)
    std::vector<int> lchunk_f, lchunk_b;                 // chunk ranges per level / colour
    const int *d_lchunk_f = nullptr, *d_lchunk_b = nullptr;
    const int *sff_dslot = nullptr;   // slot of each row's diagonal block in Sff (-1: padding lane)
    double *d_fs = nullptr;       // fixed-stress terms d_sp (nc * (nf-1)) then d_pp (nc)
    T *dss_inv = nullptr;         // nc * (nf-1)^2
    T *dinv = nullptr;            // BILU D_i^{-1} or block-diagonal inverse, nc * nf * nf
    bool sub = false;             // BILU applied by the subdomain-resident kernel
    SubBilu<T> sb;
    std::unique_ptr<DHierarchy<T>> pres;
    Arena arena;                  // fixed-layout arrays
    size_t bytes() const { return arena.bytes() + (pres ? pres->bytes() : 0); }
};

// PS_TRACE=1: a setup phase prints its wall time (and a note) to stderr when it ends.
struct TraceTick {
    const char *what;
    double t0;
    int note = -1;                // printed when >= 0 (e.g. host-device round trips)
    explicit TraceTick(const char *w);
    ~TraceTick();
};


template <typename T>
struct PrecWork {                 // per-handle work vectors for Algorithm 1
    bool fixed = false;           // sizes of everything but the pressure levels are fixed
    Arena pres_arena;             // pressure-level vectors (sizes change with each setup)
    HierWork<T> sdc, pres;
    T *vconv = nullptr;           // v_u rounded to T (FP32 path)
    T *y = nullptr, *zs = nullptr, *wp = nullptr, *zp = nullptr;   // steps 2-5
    T *w = nullptr, *t = nullptr, *dz = nullptr, *r2 = nullptr;    // steps 6-8
    Arena arena;
};

struct DSystem;
// S_pp's pattern and A_ff's diagonal slots (the first setup, after build_pressure)
void layout_pressure_operator(const System &s, PresStore &S);
// S_pp on the device from the system (S.npat > 0), then the hierarchy as build_pressure
// (l1-Jacobi smoothing)
void build_pressure_from_system(const System &s, const DSystem &D, const Options &o, Hierarchy &H, PresStore &S);
// D_ss^{-1} of the quasi-IMPES reduction (Sec. 5.2) on the device, as T: dslot[i] is the
// slot of row i's diagonal block in the SELL A_ff
template <typename T>
void dss_inverse_device(const DSystem &D, const int *dslot, T *dss_inv, hipStream_t st);

struct DSystem {                  // FP64 system matrix for A z and the true residual
    int n_nodes = 0, n_cells = 0, nf = 0;
    Sell<double> Auu, Auf, Afu, Aff;
    double mat_bytes = 0.0;       // algorithmic bytes of the four blocks (values, columns, row pointers)
    std::vector<int> src_auf, src_afu, src_aff;   // SELL slot -> block of A_uf, A_fu, A_ff (host), for new values
    Arena arena;
};

// Optional HIP-event timing of the hot kernels (ps_kernel_timing / ps_kernel_stats): an
// instrumented launch records an event before and after it on the stream it runs on and
// adds its algorithmic bytes.  Off by default; a launch then costs one atomic load.
namespace ktime {
enum Id {
    SPMV, CGS2_PROJECT, CGS2_FUSED, CGS2_SUBTRACT, BILU_SUB,
    // level 0 of the two V-cycles: pre-smoothing sweep (with the residual), restriction,
    // prolongation (x += P e), post-smoothing sweep
    SDC_PRE, SDC_RESTRICT, SDC_PROLONG, SDC_POST,
    PRES_PRE, PRES_RESTRICT, PRES_PROLONG, PRES_POST,
    // the two passes of delayed re-orthogonalisation
    DCGS2_PROJECT, DCGS2_SUBTRACT,
    NUM
};
// first id of the four level-0 V-cycle phases of a hierarchy: SDC_PRE or PRES_PRE
const char *name(int id);
bool enabled();                     // any kernel bracketed
bool enabled(int id);
void set_mask(unsigned mask);       // bit i brackets kernel id i; clears the totals
struct Scope {
    Scope(int id, hipStream_t st, double bytes);
    ~Scope();
    int id;
    hipStream_t st;
    double bytes;
    hipEvent_t e0 = nullptr;
};
// totals of kernel id (waits for recorded events)
void totals(int id, long long &launches, double &seconds, double &bytes);
}  // namespace ktime

struct Krylov {                   // FGMRES workspace (FP64 basis, Z in the precond type)
    int m = 0, nblk = 0, chunk = 0;
    size_t N = 0;
    size_t ldv = 0;               // basis stride: N rounded up to 32 (256-byte aligned vectors)
    bool z_fp32 = false;
    double *V = nullptr;          // (m+1) x ldv
    void *Z = nullptr;            // m x N (double or float)
    double *H = nullptr;          // (m+1) x m, column-major, Givens-rotated
    double *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr;
    double *h1 = nullptr, *h2 = nullptr, *hsum = nullptr, *nw2 = nullptr;
    double *scal = nullptr;       // [|g_j+1|, h_j+1,j, |A z_j|, breakdown, beta, |r|^2, -, -]
    double *partial = nullptr;    // (2m+4) x nblk reduction partials
    double *raw = nullptr;        // DCGS2: first-pass entries of the unfinished column (m+2)
    double *coef = nullptr;       // DCGS2: [alpha, t, beta of the unfinished column, -]
    double *r = nullptr;          // true residual
    double *hostscal = nullptr;   // pinned host mirror of scal
    bool own_hostscal = true;     // false: hostscal belongs to the caller
    Arena arena;
    ~Krylov();
};

template <typename T>
std::unique_ptr<DHierarchy<T>> upload_hierarchy(const Hierarchy &H, int smoother, bool interleave3);
template <typename T>
void upload_hierarchy_into(DHierarchy<T> &d, const Hierarchy &H, int smoother, bool interleave3);
// Flow stage of a setup in two parts: the layouts (first call) and values of A_fu, S_ff,
// D_ss and the local-stage factors, which do not depend on the pressure hierarchy (S: the
// system on the device, whose A_ff gives S_ff's values); then the pressure levels (ps:
// device copies of the pressure hierarchy, adopted rather than uploaded, or nullptr).
// factor_on_device: the local-stage BILU(0) factor is computed on the device from S_ff's
// values (f.ml holds the pattern only); possible once d.sb.dev_factor is set.
// operators_on_device: S_pp and D_ss are formed on the device too (f.Sff, f.dss_inv are not
// recomputed on the host).
template <typename T>
void update_flow_values(DFlow<T> &d, const FlowSetup &f, const System &s, const DSystem &S, const Options &o,
                        Staging &stg, bool afu_changed, bool factor_on_device = false,
                        bool operators_on_device = false);
template <typename T>
void update_flow_pressure(DFlow<T> &d, const FlowSetup &f, const Options &o, const PresStore *ps);
void upload_system(const System &s, DSystem &d);
// new values of A_fu and A_ff (and A_uf when `auf`; same patterns) into d's layout, through stg
void update_system_flow_values(const System &s, DSystem &d, Staging &stg, bool auf = false);
template <typename T>
void alloc_prec_work(PrecWork<T> &w, const DHierarchy<T> &sdc, const DFlow<T> &fl, int n_nodes);
void alloc_krylov(Krylov &k, size_t N, int m, bool z_fp32);
// bytes of device memory a Krylov workspace takes (arrays 256-byte aligned)
size_t krylov_bytes(size_t N, int m, bool z_fp32);
// The same workspace laid out inside caller-provided device memory [base, base + cap),
// with a caller-owned pinned scalar mirror: allocates nothing.  Throws Error(PS_EINVAL)
// when the workspace does not fit.
void carve_krylov(Krylov &k, void *base, size_t cap, size_t N, int m, bool z_fp32, double *hostscal);

// y = A x (FP64), or y = b - A x when b != nullptr; x of type TX.
template <typename TX>
void spmv_full(const DSystem &S, const TX *x, const double *b, double *y, hipStream_t st);

// z = M^{-1} v (Algorithm 1); v FP64, z of type T (length N).
template <typename T>
void apply_precond(const DHierarchy<T> &sdc, const DFlow<T> &fl, PrecWork<T> &w, int n_nodes,
                   const double *v, T *z, hipStream_t st);
// The same in three parts, so that step 1 of several solves sharing one mechanics hierarchy
// can run as one batch: precond_pre returns step 1's right-hand side (v_u in T), step 1 writes
// z_u = z[0 .. 3 n_nodes), precond_post runs steps 2-8.
template <typename T>
const T *precond_pre(PrecWork<T> &w, int n_nodes, const double *v, hipStream_t st);
template <typename T>
void precond_post(const DFlow<T> &fl, PrecWork<T> &w, int n_nodes, const double *v, T *z, hipStream_t st);
constexpr int kBatchMax = 8;       // solves in one batched step 1
// Step 1 (one V-cycle of the shared hierarchy) for nb <= kBatchMax solves in one sequence of launches:
// w[i], vu[i], zu[i] of solve i.  Each solve's z_u is bitwise what apply_precond computes.
template <typename T>
void step1_batch(const DHierarchy<T> &sdc, PrecWork<T> *const *w, const T *const *vu, T *const *zu, int nb,
                 hipStream_t st);

struct SolveOut {
    int status = PS_OK, iterations = 0, restarts = 0;
    double rel_residual = 0.0;
};

// Preconditioner callback: z (double or float, per Krylov::z_fp32) = M^{-1} v.
struct PrecFn {
    virtual void operator()(const double *v, void *z, hipStream_t st) = 0;
    // The application in parts around step 1 (precond_pre / precond_post), for callers that
    // run step 1 of several solves together; can_split() = false: whole applications only.
    virtual bool can_split() const { return false; }
    virtual const void *pre(const double *v, hipStream_t st) { return nullptr; }
    virtual void post(const double *v, void *z, hipStream_t st) {}
    virtual ~PrecFn() = default;
};

// Right-preconditioned flexible GMRES(m) with CGS2 and Givens rotations (paper
// Sec. 4), as a resumable state machine: start() enqueues the first work, and
// after each stream synchronisation advance() consumes the 64-byte scalar
// read-back and enqueues the next piece (one iteration, or the end of a cycle).
// advance() returns false once `out` is final.  The serving scheduler interleaves
// many of these, one per request and stream.
class Fgmres {
  public:
    // orth: PS_CGS2 or PS_DCGS2 (Arnoldi step)
    Fgmres(const DSystem &S, Krylov &K, PrecFn &M, const double *b, double *x, double rtol, int maxit,
           hipStream_t st, int orth = PS_CGS2);
    void start();
    bool advance();
    SolveOut out;
    // With defer set (and a splittable preconditioner), an iteration that advance() starts
    // stops before step 1: step1_pending() is then true, step1_rhs() / step1_out() are step
    // 1's operands (in the preconditioner's type), and after the caller has enqueued step 1
    // -- ordered after this solve's stream and before its next work -- finish_iteration()
    // enqueues the rest of the iteration on the solve's stream.
    void set_defer(bool d) { defer_ = d; }
    bool step1_pending() const { return pending_; }
    const void *step1_rhs() const { return s1_rhs_; }
    void *step1_out() const { return s1_z_; }
    void finish_iteration();

  private:
    enum Phase { START, ITER, CYCLE_END, DONE };
    void copy_scal();
    void begin_cycle(const double *r);
    void enqueue_iteration();
    void rest_of_iteration();
    void rest_dcgs2();
    void finish_last_column(int k);
    void end_cycle(int k);
    bool defer_ = false, pending_ = false;
    const void *s1_rhs_ = nullptr;
    void *s1_z_ = nullptr;
    const DSystem &S_;
    Krylov &K_;
    PrecFn &M_;
    const double *b_;
    double *x_;
    double rtol_;
    int maxit_;
    hipStream_t st_;
    int orth_;
    bool open_col_ = false;       // DCGS2: the newest column still lacks its second pass
    Phase phase_ = START;
    int j_ = 0, its_ = 0, cycles_ = 0;
    double beta_b_ = 0.0;
    bool breakdown_ = false;
};
SolveOut fgmres_blocking(Fgmres &run, hipStream_t st);
// Fixed-stress diagonals by row-sum lumping (eq. FS_RSL): d_sp = -(A_su y), d_pp = -(A_pu y)
// with y ~ A_uu^{-1} A_up e from `iters` Richardson steps y += M_uu^{-1}(A_up e - A_uu y)
// preconditioned by the FP64 mechanics V-cycle; all products with the device system.
// Results (host, n_cells x (nf-1) and n_cells) are written into d_sp, d_pp.
struct RslWork {
    Arena arena;
    double *e = nullptr, *y = nullptr, *g = nullptr, *t = nullptr, *z = nullptr;
    HierWork<double> hw;
    bool ready = false;
};
void rsl_diagonals(const DSystem &S, const DHierarchy<double> &sdc, RslWork &w, int iters,
                   std::vector<double> &d_sp, std::vector<double> &d_pp, hipStream_t st);

// Preconditioned Richardson iteration (blocking); K needs restart >= 1.
SolveOut richardson_blocking(const DSystem &S, Krylov &K, PrecFn &M, const double *b, double *x, double rtol,
                             int maxit, hipStream_t st);

void fill_zero(double *p, size_t n, hipStream_t st);
void widen_f32(const float *in, double *out, size_t n, hipStream_t st);

}  // namespace ps
