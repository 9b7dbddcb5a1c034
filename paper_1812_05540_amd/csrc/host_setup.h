// Host-side data structures and the setup phase of the two-stage preconditioner.
#pragma once

#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ps.h"

namespace ps {

// Error carrying a ps.h status code across C++ frames; caught at the C boundary.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

struct Csr {                      // scalar CSR, sorted columns
    int n = 0, m = 0;
    std::vector<int> rp, ci;
    std::vector<double> v;
    int nnz() const { return (int)ci.size(); }
};

struct Bsr {                      // block CSR, row-major blocks, sorted columns
    int nbr = 0, nbc = 0, br = 0, bc = 0;
    std::vector<int> rp, ci;
    std::vector<double> v;        // nblocks * br * bc
    int nb() const { return (int)ci.size(); }
};

struct Level {                    // one AMG level
    Csr A, P, R;                  // P, R empty on the coarsest level
    std::vector<int8_t> cf;       // 1 = C, -1 = F
    std::vector<double> diag, dl1;// diagonal, l1 row sums
    std::vector<double> c0, c1, cm;  // Chebyshev per-row coefficients
    double lam = 0.0;             // 1.1 x power-iteration estimate of rho(D^-1 A)
};

struct Hierarchy {
    std::vector<Level> lev;       // coarsest last
    std::vector<double> coarse_inv;  // dense inverse of the coarsest operator, row-major
    int coarse_n = 0;
};

struct Options {
    int precision = PS_FP64, restart = 100, maxit = 1000, smoother = PS_CHEB2;
    int ml_kind = PS_BILU0, ml_sweeps = 1, coarse_max = 256, max_levels = 25;
    int fp32_fallback = 0;
    double theta = 0.25;
    int method = PS_FGMRES, reduction = PS_QUASI_IMPES, fixed_stress = PS_FS_GIVEN, fs_iters = 10;
    int orth = PS_CGS2;
};

Options options_from(const ps_options *o);

struct System {                   // validated host copy of a ps_system
    int n_nodes = 0, n_cells = 0, nf = 0;
    Bsr Auu, Auf, Afu, Aff;
    std::vector<double> d_sp, d_pp;
    std::vector<int> ml_part;     // empty: global BILU(0)
    uint64_t mech_key = 0;
    size_t N() const { return (size_t)3 * n_nodes + (size_t)nf * n_cells; }
};

void validate_and_copy(const ps_system *s, System &out);   // throws Error(PS_EINVAL)

struct BiluSchedule {             // level sets of the BILU sweeps (or colour groups)
    std::vector<int> fwd_ptr, fwd_rows, bwd_ptr, bwd_rows;
};

struct FlowSetup {                // recomputed at every ps_setup (Sec. 5.4)
    Bsr Sff;                      // S_ff^(fs) values on the A_ff pattern
    Csr Spp;                      // quasi-IMPES pressure operator on the cell pattern
    std::vector<double> dss_inv;  // n_cells * (nf-1)^2
    Hierarchy pres;
    Bsr ml;                       // BILU(0) factors (diag blocks = D_i^{-1}) or block-Jacobi D^{-1}
    BiluSchedule sched;
};

// --- setup steps ------------------------------------------------------------
Bsr fixed_stress(const System &s);
void fixed_stress(const System &s, Bsr &S);              // into S, reusing its storage
// reduction: PS_QUASI_IMPES (diagonal cell blocks) or PS_TRUE_IMPES (column sums)
void quasi_impes(const System &s, const Bsr &Sff, Csr &Spp, std::vector<double> &dss_inv,
                 int reduction = PS_QUASI_IMPES);
Csr sdc_matrix(const System &s);                         // component-major
Hierarchy amg_build(const Csr &A, const Options &o);
// The steps of amg_build, for builders that form the Galerkin product elsewhere:
bool coarsen_level(const Csr &A, const Options &o, Level &L);  // cf, P, R; false: stop coarsening
Csr galerkin(const Level &L, const Csr &A);                   // R (A P), exact zeros dropped
void finish_level(Level &L, int smoother);                    // smoother data of L (L.A set)
void coarse_level(Csr A, Hierarchy &H);                       // dense inverse of the last level
void bilu0_factor(const Bsr &S, Bsr &F);                 // throws Error(PS_ESINGULAR)
void bilu0_factor_inplace(Bsr &F, const BiluSchedule &sc);  // sc: forward levels of F's pattern
Bsr restrict_to_parts(const Bsr &S, const std::vector<int> &part);   // drop inter-part blocks
void restrict_to_parts(const Bsr &S, const std::vector<int> &part, Bsr &R);
void block_jacobi_factor(const Bsr &S, Bsr &F);
BiluSchedule bilu_schedule(const Bsr &S);
BiluSchedule color_schedule(const Bsr &S);             // colour groups in fwd_ptr/fwd_rows
void build_flow(const System &s, const Options &o, FlowSetup &f);
void build_flow_operators(const System &s, const Options &o, FlowSetup &f);   // S_ff^(fs), S_pp, D_ss^{-1}
// local-stage factors; pattern_only: a BILU(0) factor whose pattern and schedule exist
// is left to the device (f.ml keeps its pattern, its values are not recomputed)
void build_flow_local(const System &s, const Options &o, FlowSetup &f, bool pattern_only = false);

// Run f(begin, end, part) over [0, n) split into contiguous parts on host threads.
void parallel_for(int n, const std::function<void(int, int, int)> &f);
int setup_thread_count();

// --- small dense helpers ----------------------------------------------------
bool invert_small(const double *a, double *inv, int n);  // Gauss-Jordan, partial pivoting
bool invert_dense(std::vector<double> a, std::vector<double> &inv, int n);

}  // namespace ps
