/*
 * m1_oracle3.h -- TEST INFRASTRUCTURE ONLY: the plain FP64 CPU oracle of the
 * three-dimensional method (arXiv 2208.14703 with d = 3: the 7-point form of
 * the implicit Rusanov system, R = 2^-3 P^T of Sect. 4.2).
 *
 * State layout: five fields (E, Fx, Fy, Fz, T), each nx*ny*nz doubles with x
 * fastest: v[q*n + (k*ny + j)*nx + i].  Sides: 0 x-, 1 x+, 2 y-, 3 y+, 4 z-,
 * 5 z+; kinds as in the 2-D oracle (periodic, reflective, Neumann, Dirichlet).
 */
#ifndef M1_ORACLE3_H
#define M1_ORACLE3_H

#include <stdint.h>

#include "m1_oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz, pad_;
    double hx, hy, hz, dt, c, a_r, c_v;
    int32_t bc_kind[6];
    double bc_E[6], bc_Fx[6], bc_Fy[6], bc_Fz[6];
} or3_grid;

void    or3_closure(double E, double Fx, double Fy, double Fz, double c, double P[6]);
int     or3_admissible(double c, const double w[5]);
double  or3_ray(double c, const double w[5], const double s[5]);
void    or3_apply_A(const or3_grid* g, const double* sigma, const double* v, double* out);
void    or3_residual(const or3_grid* g, const double* sigma, const double* b, const double* v, double* r);
double  or3_norm(const or3_grid* g, const double* r);
void    or3_sweep(const or3_grid* g, const double* sigma, double omega, const double* b, const double* v_in,
                  double* v_out);
void    or3_pseudo_step(const or3_grid* g, const double* sigma, const or_params* p, double dtau, const double* f,
                        const double* u_in, double* u_out);
void    or3_project(const or3_grid* g, const or_params* p, const double* u, const double* w, double* out);
or3_grid or3_coarse_grid(const or3_grid* g);
void    or3_restrict(const or3_grid* fine, const double* x_fine, int32_t nfields, double* x_coarse);
void    or3_prolong(const or3_grid* fine, const double* x_coarse, int32_t nfields, double* x_fine);
int32_t or3_num_levels(const or3_grid* g, const or_params* p);
void    or3_vcycle(const or3_grid* g, const double* sigma, const or_params* p, double dtau, const double* b,
                   const double* v, double* out);
void    or3_cycle(const or3_grid* g, const double* sigma, const or_params* p, int32_t kind, double dtau,
                  const double* b, const double* v, double* out);
int32_t or3_step(const or3_grid* g, const double* sigma, const or_params* p, double* v, int32_t nsteps,
                 or_info* info);

#ifdef __cplusplus
}
#endif
#endif
