/*
 * ps_host.h -- host-side setup phase of the two-stage preconditioner, callable
 * without a GPU.  ps_setup runs exactly this code before uploading to the device;
 * it is exported so that the setup can be inspected and checked on a CPU.
 *
 * Operations (paper Sec. 5):
 *   - fixed-stress Schur approximation S_ff^(fs) (eq. Schur_1_FS, eq. FS_Dps_Dpp);
 *   - quasi-IMPES pressure operator S_pp = A_pp^(fs) - D_ps D_ss^{-1} A_sp^(fs)
 *     (Sec. 5.3, eq. S1_LDU and the Quasi-IMPES reduction);
 *   - separate-displacement-component operator blockdiag(A_xx, A_yy, A_zz) in
 *     component-major order (Sec. 5.2);
 *   - one AMG hierarchy per scalar operator (strength, PMIS, C-promotion, direct
 *     interpolation, Galerkin product, dense coarsest level);
 *   - BILU(0) factors of S_ff^(fs) (Sec. 5.3, ILU(0) on the interleaved system).
 * Same status codes and ownership rules as ps.h; exported arrays are copied into
 * caller buffers (pass NULL to query sizes first).
 */
#ifndef PS_HOST_H
#define PS_HOST_H

#include "ps.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ps_host_setup ps_host_setup;

#define PS_H_SDC 0       /* mechanics (separate displacement component) hierarchy */
#define PS_H_PRES 1      /* quasi-IMPES pressure hierarchy */

/* Run the whole host setup on a validated copy of sys. */
int  ps_host_setup_create(const ps_system *sys, const ps_options *opts, ps_host_setup **out);
void ps_host_setup_destroy(ps_host_setup *s);

/* Number of levels (coarsest level included) of hierarchy `which`. */
int  ps_host_levels(const ps_host_setup *s, int which, int32_t *nlevels);

/* Level `lvl` of hierarchy `which`: operator A (n x n, nnz entries, CSR with sorted
 * columns), C/F splitting cf[n] (1 = C, -1 = F; all zero on the coarsest level), and
 * for non-coarsest levels the prolongation P (n x nc, p_nnz entries).  Any output
 * pointer may be NULL; sizes are always written. */
int  ps_host_level(const ps_host_setup *s, int which, int lvl, int32_t *n, int32_t *nnz,
                   int32_t *rowptr, int32_t *colind, double *vals, int8_t *cf,
                   int32_t *nc, int32_t *p_nnz, int32_t *p_rowptr, int32_t *p_colind,
                   double *p_vals);

/* Smoother constants of level lvl: Chebyshev eigenvalue bound (lambda' = 1.1 x the
 * power-iteration estimate; 0 for l1-Jacobi). */
int  ps_host_level_lambda(const ps_host_setup *s, int which, int lvl, double *lam);

/* Quasi-IMPES pressure matrix values on the A_ff block pattern (Aff.nblocks values). */
int  ps_host_spp(const ps_host_setup *s, double *vals);

/* BILU(0) factor values on the factor's block pattern -- the A_ff pattern, or its
 * restriction to same-subdomain blocks when ml_part is given -- (nblocks * nf * nf;
 * strictly lower blocks hold L_ik, upper blocks U_ij, diagonal blocks D_i^{-1}). */
int  ps_host_bilu(const ps_host_setup *s, double *vals);

/* Level schedule of the BILU(0) forward sweep: number of levels (nf x nf block rows
 * with all dependencies in earlier levels). */
int  ps_host_bilu_levels(const ps_host_setup *s, int32_t *fwd_levels, int32_t *bwd_levels);

#ifdef __cplusplus
}
#endif
#endif /* PS_HOST_H */
