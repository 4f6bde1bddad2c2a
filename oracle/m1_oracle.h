/*
 * m1_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU oracle of the implicit M1 radiative-transfer
 * multigrid method of Bloch, Tremblin, Gonzalez & Audit, "Towards a multigrid
 * method for the M1 model for radiative transfer" (arXiv 2208.14703).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The GPU product path never includes this
 * header, never links this code and shares no helper with it.
 *
 * Layout conventions (the oracle's own):
 *   a state is one contiguous double array of 4*nx*ny values holding the
 *   fields E, Fx, Fy, T one after the other, each row-major with x fastest;
 *   an opacity array holds sigma_a then sigma_s (2*nx*ny values).
 * In one dimension ny == 1 and the Fy field stays identically zero.
 */
#ifndef M1_ORACLE_H
#define M1_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_BC_PERIODIC = 0, OR_BC_REFLECTIVE = 1, OR_BC_NEUMANN = 2, OR_BC_DIRICHLET = 3, OR_BC_INFLOW = 4 };
enum { OR_DTAU_SIGNED = 0, OR_DTAU_LITERAL = 1 };
enum { OR_SMOOTH_JACOBI = 0, OR_SMOOTH_RBGS = 1 };
enum { OR_CYCLE_V = 0, OR_CYCLE_W = 1, OR_CYCLE_F = 2 };
enum { OR_TRANSFER_FULL = 0, OR_TRANSFER_MEAN = 1 };

typedef struct {
    int32_t dim, nx, ny, pad_;
    double hx, hy, dt, c, a_r, c_v;
    int32_t bc_kind[4];              /* sides x-, x+, y-, y+ */
    double bc_E[4], bc_Fx[4], bc_Fy[4]; /* Dirichlet / inflow ghost state per side */
    double bc_lo[4], bc_hi[4];          /* inflow segment of each side, as fractions of its length */
    double bc_Eo[4];                    /* inflow sides: energy of the isotropic ghost outside the segment */
} or_grid;

typedef struct {
    int32_t levels;        /* total number of levels incl. the finest; 0 = down to side 4 */
    int32_t nu0;           /* Jacobi sweeps before and after the correction, finest level */
    int32_t nu_l;          /* Jacobi sweeps per implicit pseudo-time step, coarse levels */
    int32_t pseudo_steps;  /* pseudo-time steps per coarse smoothing */
    int32_t sub_steps;     /* max explicit sub-steps per pseudo-time step */
    int32_t max_cycles;
    int32_t dtau_rule;     /* OR_DTAU_SIGNED or OR_DTAU_LITERAL */
    int32_t pseudo_local;  /* 1: implicit pseudo-time step uses each cell's own tau_i; 0: dtau_im everywhere */
    int32_t smoother;      /* finest-level sweeps: OR_SMOOTH_JACOBI or OR_SMOOTH_RBGS (red-black Gauss-Seidel) */
    int32_t cycle;         /* OR_CYCLE_V, OR_CYCLE_W or OR_CYCLE_F */
    int32_t transfer;      /* OR_TRANSFER_FULL (full weighting, Sect. 4.2) or OR_TRANSFER_MEAN (2^d-cell mean,
                              piecewise-constant prolongation) */
    int32_t dtau_carry;    /* 1: dtau_im runs on from one time step to the next (the overall algorithm of
                              Appendix A does not set it at the start of a step; Sect. 5 gives its initial
                              value); 0: reset to dtau_im0 at the start of every time step */
    double dtau_im0, eps_inc, eps_dec, eta, rtol, dtau_min, dtau_max;
    double omega;          /* relaxation weight of the finest-level Jacobi sweeps (1 = Algorithm 1) */
} or_params;

typedef struct {
    int32_t cycles, status, levels, pad_;
    double r0, rel_residual, dtau;
} or_info;

/* single-cell pieces */
double or_chi(double f);
void   or_closure(double E, double Fx, double Fy, double c, double P[3]);
void   or_local_solve(double beta, double gamma, double a, double ka, double ks, double cv, double ar,
                      const double B[4], double out[4]);
double or_ray(double c, const double w[4], const double s[4]);
int    or_admissible(double c, const double w[4]);

/* grid operators (one level, spacing taken from g) */
void   or_apply_A(const or_grid* g, const double* sigma, const double* v, double* out);
void   or_residual(const or_grid* g, const double* sigma, const double* b, const double* v, double* r);
double or_norm(const or_grid* g, const double* r);
void   or_jacobi(const or_grid* g, const double* sigma, double beta, double gamma, const double* gamma_cell,
                 const double* rhs, const double* v_in, double* v_out);
void   or_sweep(const or_grid* g, const double* sigma, double omega, const double* b, const double* v_in,
                double* v_out);
void   or_rb_sweep(const or_grid* g, const double* sigma, double omega, const double* b, const double* v_in,
                   double* v_out);
void   or_restrict(const or_grid* fine, const double* x_fine, int32_t nfields, double* x_coarse);
void   or_prolong(const or_grid* fine, const double* x_coarse, int32_t nfields, double* x_fine);
void   or_restrict_t(const or_grid* fine, const double* x_fine, int32_t nfields, double* x_coarse, int32_t transfer);
void   or_prolong_t(const or_grid* fine, const double* x_coarse, int32_t nfields, double* x_fine, int32_t transfer);
void   or_pseudo_time(const or_grid* g, const or_params* p, double dtau, const double* f, const double* u_in,
                      double* taus, double* u_tilde);
void   or_pseudo_step(const or_grid* g, const double* sigma, const or_params* p, double dtau,
                      const double* f, const double* u_in, double* u_out);
void   or_project(const or_grid* g, const or_params* p, const double* u, const double* w, double* out);
or_grid or_coarse_grid(const or_grid* g);

/* whole method */
int32_t or_num_levels(const or_grid* g, const or_params* p);
void   or_vcycle(const or_grid* g, const double* sigma, const or_params* p, double dtau,
                 const double* b, const double* v, double* out);
void   or_cycle(const or_grid* g, const double* sigma, const or_params* p, int32_t kind, double dtau,
                const double* b, const double* v, double* out);
int32_t or_step(const or_grid* g, const double* sigma, const or_params* p, double* v, int32_t nsteps,
                or_info* info, double* history, int32_t history_len);
int32_t or_threads(void);

/* explicit reference of the homogeneous system (HLL with the M1 wave speeds, or Rusanov) */
void   or_wave_speeds(double c, const double U[3], int axis, double* lm, double* lp);
void   or_explicit_step(const or_grid* g, int hll, const double* v, double* out);
int32_t or_explicit_run(const or_grid* g, int hll, double* v, int32_t max_steps, double tol);
void   or_set_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
