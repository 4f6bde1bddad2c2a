/*
 * m1_oracle.c -- TEST INFRASTRUCTURE ONLY: the plain FP64 CPU oracle.
 *
 * What it computes is the method of Bloch, Tremblin, Gonzalez & Audit,
 * "Towards a multigrid method for the M1 model for radiative transfer"
 * (arXiv 2208.14703), with the readings recorded in the design notes where
 * the paper is silent (sources and gas coupling, 2-D form, boundary ghosts,
 * sub-cycling rule, projection step, pseudo-time step adaptation).
 *
 * Written for obviousness, not speed: straight loops, one cell at a time, the
 * paper's formulas in the paper's order.  The only concession is an OpenMP
 * loop over rows, which does not change any result (every cell is computed
 * independently and the norm is summed row by row in a fixed order).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include "m1_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NFIELD 4 /* E, Fx, Fy, T */

static size_t ncell(const or_grid* g) { return (size_t)g->nx * (size_t)g->ny; }

static double* dalloc(size_t n)
{
    double* p = (double*)calloc(n ? n : 1, sizeof(double));
    if (!p) abort();
    return p;
}

int32_t or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the oracle's parallel row loops from now on (n >= 1). */
void or_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------- */
/* M1 closure, Sect. 2.1 (closure relation): P = ((1-chi)/2 I + (3chi-1)/2 n n) E,
 * chi(f) = (3 + 4 f^2) / (5 + 2 sqrt(4 - 3 f^2)), n = F/|F|, f = |F|/(cE).     */
double or_chi(double f) { return (3.0 + 4.0 * f * f) / (5.0 + 2.0 * sqrt(4.0 - 3.0 * f * f)); }

void or_closure(double E, double Fx, double Fy, double c, double P[3])
{
    double normF = sqrt(Fx * Fx + Fy * Fy);
    double f = normF / (c * E);
    if (f > 1.0) f = 1.0; /* rounding guard on the boundary |F| = cE */
    double chi = or_chi(f);
    double nx = 0.0, ny = 0.0; /* F = 0: n is irrelevant since (3chi-1)/2 = 0 */
    if (normF > 0.0) {
        nx = Fx / normF;
        ny = Fy / normF;
    }
    double iso = 0.5 * (1.0 - chi);
    double dir = 0.5 * (3.0 * chi - 1.0);
    P[0] = (iso + dir * nx * nx) * E; /* Pxx */
    P[1] = (dir * nx * ny) * E;       /* Pxy */
    P[2] = (iso + dir * ny * ny) * E; /* Pyy */
}

/* Admissible set of Sect. 3.1, extended with the gas temperature:
 * E > 0, |F| <= cE, T > 0.                                                   */
int or_admissible(double c, const double w[4])
{
    return w[0] > 0.0 && w[3] > 0.0 && (w[1] * w[1] + w[2] * w[2]) <= c * c * w[0] * w[0];
}

/* ------------------------------------------------------------------------- */
/* Ghost / neighbour state (E, Fx, Fy) of cell (i,j) in direction (di,dj).
 * Periodic: wrap; reflective: the cell itself with the normal flux negated;
 * Neumann: the cell itself; Dirichlet: the fixed wall state of that side;
 * inflow: the wall state for the boundary cells whose centres lie in the
 * side's [lo, hi] (fractions of its length), the isotropic state (Eo, F = 0)
 * elsewhere.                                                                 */
static void neighbour(const or_grid* g, const double* v, int i, int j, int di, int dj, double U[3])
{
    const size_t n = ncell(g);
    int ni = i + di, nj = j + dj, side = -1;
    if (ni < 0) side = 0;
    else if (ni >= g->nx) side = 1;
    else if (nj < 0) side = 2;
    else if (nj >= g->ny) side = 3;
    if (side >= 0) {
        switch (g->bc_kind[side]) {
        case OR_BC_PERIODIC:
            ni = (ni + g->nx) % g->nx;
            nj = (nj + g->ny) % g->ny;
            break;
        case OR_BC_REFLECTIVE: {
            size_t k = (size_t)j * g->nx + i;
            U[0] = v[k];
            U[1] = v[n + k];
            U[2] = v[2 * n + k];
            if (side < 2) U[1] = -U[1];
            else U[2] = -U[2];
            return;
        }
        case OR_BC_INFLOW: {
            const int along = side < 2 ? j : i, len = side < 2 ? g->ny : g->nx;
            const double centre = along + 0.5;
            if (centre >= g->bc_lo[side] * len && centre <= g->bc_hi[side] * len) {
                U[0] = g->bc_E[side];
                U[1] = g->bc_Fx[side];
                U[2] = g->bc_Fy[side];
            } else {
                U[0] = g->bc_Eo[side];
                U[1] = 0.0;
                U[2] = 0.0;
            }
            return;
        }
        case OR_BC_NEUMANN: {
            size_t k = (size_t)j * g->nx + i;
            U[0] = v[k];
            U[1] = v[n + k];
            U[2] = v[2 * n + k];
            return;
        }
        default: /* OR_BC_DIRICHLET */
            U[0] = g->bc_E[side];
            U[1] = g->bc_Fx[side];
            U[2] = g->bc_Fy[side];
            return;
        }
    }
    size_t k = (size_t)nj * g->nx + ni;
    U[0] = v[k];
    U[1] = v[n + k];
    U[2] = v[2 * n + k];
}

/* Left (sign=+1) and right (sign=-1) operators of Sect. 3.1 along one axis:
 * L(U) = dt/(2h) (c U + G(U)),  R(U) = dt/(2h) (c U - G(U)),
 * with the directional physical flux G_x = (Fx, c^2 Pxx, c^2 Pxy) or
 * G_y = (Fy, c^2 Pxy, c^2 Pyy).  In 1-D this is exactly the printed L and R. */
static void op_LR(const or_grid* g, int axis, double sign, const double U[3], double out[3])
{
    const double c = g->c;
    double P[3], G[3];
    or_closure(U[0], U[1], U[2], c, P);
    if (axis == 0) {
        G[0] = U[1];
        G[1] = c * c * P[0];
        G[2] = c * c * P[1];
    } else {
        G[0] = U[2];
        G[1] = c * c * P[1];
        G[2] = c * c * P[2];
    }
    const double h = (axis == 0) ? g->hx : g->hy;
    const double k = g->dt / (2.0 * h);
    for (int m = 0; m < 3; ++m) out[m] = k * (c * U[m] + sign * G[m]);
}

/* Off-diagonal part of row (i,j): L_x(v_{i-1,j}) + R_x(v_{i+1,j}) [+ L_y(v_{i,j-1}) + R_y(v_{i,j+1})]. */
static void offdiag(const or_grid* g, const double* v, int i, int j, double S[3])
{
    double U[3], t[3];
    S[0] = S[1] = S[2] = 0.0;
    neighbour(g, v, i, j, -1, 0, U);
    op_LR(g, 0, +1.0, U, t);
    for (int m = 0; m < 3; ++m) S[m] += t[m];
    neighbour(g, v, i, j, +1, 0, U);
    op_LR(g, 0, -1.0, U, t);
    for (int m = 0; m < 3; ++m) S[m] += t[m];
    if (g->dim == 2) {
        neighbour(g, v, i, j, 0, -1, U);
        op_LR(g, 1, +1.0, U, t);
        for (int m = 0; m < 3; ++m) S[m] += t[m];
        neighbour(g, v, i, j, 0, +1, U);
        op_LR(g, 1, -1.0, U, t);
        for (int m = 0; m < 3; ++m) S[m] += t[m];
    }
}

/* Diagonal coefficient of the transport part: 1 + c dt/hx (+ c dt/hy). */
static double diag_a(const or_grid* g)
{
    double a = 1.0 + g->c * g->dt / g->hx;
    if (g->dim == 2) a += g->c * g->dt / g->hy;
    return a;
}

/* ------------------------------------------------------------------------- */
/* Nonlinear operator A of Sect. 3.1 (its rows: D(v_i) - L(v_{i-1}) - R(v_{i+1})),
 * with the source terms of eq. (m1) taken implicitly and the gas energy row
 * C_v T + c dt sigma_a (a_r T^4 - E):
 *   A_E  = a E  - S_E  + ka (E - a_r T^4)
 *   A_F  = a F  - S_F  + (ka + ks) F
 *   A_T  = C_v T + ka (a_r T^4 - E)          (ka = c dt sigma_a, ks = c dt sigma_s) */
void or_apply_A(const or_grid* g, const double* sigma, const double* v, double* out)
{
    const size_t n = ncell(g);
    const double a = diag_a(g);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < g->ny; ++j) {
        for (int i = 0; i < g->nx; ++i) {
            size_t k = (size_t)j * g->nx + i;
            double S[3];
            offdiag(g, v, i, j, S);
            double ka = g->c * g->dt * sigma[k];
            double ks = g->c * g->dt * sigma[n + k];
            double E = v[k], Fx = v[n + k], Fy = v[2 * n + k], T = v[3 * n + k];
            double T4 = T * T * T * T;
            out[k] = a * E - S[0] + ka * (E - g->a_r * T4);
            out[n + k] = a * Fx - S[1] + (ka + ks) * Fx;
            out[2 * n + k] = (g->dim == 2) ? a * Fy - S[2] + (ka + ks) * Fy : 0.0;
            out[3 * n + k] = g->c_v * T + ka * (g->a_r * T4 - E);
        }
    }
}

/* Residual, eq. (defResidual): r = b - A(v). */
void or_residual(const or_grid* g, const double* sigma, const double* b, const double* v, double* r)
{
    const size_t n = ncell(g);
    or_apply_A(g, sigma, v, r);
    for (size_t k = 0; k < NFIELD * n; ++k) r[k] = b[k] - r[k];
}

/* Discrete L2 norm of (r_E, r_Fx/c, r_Fy/c, r_T) over all cells, summed row by
 * row in a fixed order.                                                      */
double or_norm(const or_grid* g, const double* r)
{
    const size_t n = ncell(g);
    double* rows = dalloc((size_t)g->ny);
    const double ic = 1.0 / g->c;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < g->ny; ++j) {
        double s = 0.0;
        for (int i = 0; i < g->nx; ++i) {
            size_t k = (size_t)j * g->nx + i;
            double e = r[k], fx = r[n + k] * ic, fy = r[2 * n + k] * ic, t = r[3 * n + k];
            s += e * e + fx * fx + fy * fy + t * t;
        }
        rows[j] = s;
    }
    double s = 0.0;
    for (int j = 0; j < g->ny; ++j) s += rows[j];
    free(rows);
    return sqrt(s);
}

/* ------------------------------------------------------------------------- */
/* Local inverse of the (scaled) diagonal operator: solve for one cell
 *   beta*E  + gamma*((a + ka) E - ka a_r T^4)           = B_E
 *   beta*F  + gamma*(a + ka + ks) F                     = B_F
 *   beta*Cv T + gamma*(Cv T + ka (a_r T^4 - E))         = B_T
 * (beta, gamma) = (0, 1) is D^{-1} of Algorithm 1; (1, dtau) is the implicit
 * pseudo-time step of Algorithm 3 with the mass matrix diag(1, 1, 1, C_v).
 * E is eliminated, leaving an increasing convex quartic in T that is solved by
 * Newton's method from an upper bound of its root (monotone convergence).   */
void or_local_solve(double beta, double gamma, double a, double ka, double ks, double cv, double ar,
                    const double B[4], double out[4])
{
    const double dE = beta + gamma * (a + ka);
    const double dF = beta + gamma * (a + ka + ks);
    const double k = gamma * ka;
    const double cT = (beta + gamma) * cv;
    /* cT T + K T^4 = Q,  K = k a_r (dE - k)/dE,  Q = B_T + k B_E / dE */
    const double K = k * ar * (beta + gamma * a) / dE;
    const double Q = B[3] + k * B[0] / dE;
    double T;
    if (K == 0.0) {
        T = Q / cT;
    } else {
        double t1 = Q / cT, t2 = sqrt(sqrt(Q / K));
        T = t1 < t2 ? t1 : t2; /* each term alone bounds the root from above */
        for (int it = 0; it < 200; ++it) {
            double g = cT * T + K * T * T * T * T - Q;
            double dg = cT + 4.0 * K * T * T * T;
            double dT = g / dg;
            T -= dT;
            if (fabs(dT) <= 1e-15 * T) break;
        }
    }
    out[0] = (B[0] + k * ar * T * T * T * T) / dE;
    out[1] = B[1] / dF;
    out[2] = B[2] / dF;
    out[3] = T;
}

/* One sweep of the nonlinear Jacobi method (Algorithm 1) on
 *   (beta M + gamma A)(u) = rhs:
 *   u_i^{k+1} = local_solve(rhs_i + gamma (L(u_{i-1}^k) + R(u_{i+1}^k) + ...)).
 * gamma_cell, when given, replaces gamma by a per-cell value (the local
 * pseudo-time steps of Algorithm 3).  Out of place: only iterate k is read.  */
void or_jacobi(const or_grid* g, const double* sigma, double beta, double gamma0, const double* gamma_cell,
               const double* rhs, const double* v_in, double* v_out)
{
    const size_t n = ncell(g);
    const double a = diag_a(g);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < g->ny; ++j) {
        for (int i = 0; i < g->nx; ++i) {
            size_t k = (size_t)j * g->nx + i;
            double S[3], B[4], o[4];
            double gamma = gamma_cell ? gamma_cell[k] : gamma0;
            offdiag(g, v_in, i, j, S);
            B[0] = rhs[k] + gamma * S[0];
            B[1] = rhs[n + k] + gamma * S[1];
            B[2] = (g->dim == 2) ? rhs[2 * n + k] + gamma * S[2] : 0.0;
            B[3] = rhs[3 * n + k];
            double ka = g->c * g->dt * sigma[k];
            double ks = g->c * g->dt * sigma[n + k];
            or_local_solve(beta, gamma, a, ka, ks, g->c_v, g->a_r, B, o);
            v_out[k] = o[0];
            v_out[n + k] = o[1];
            v_out[2 * n + k] = o[2];
            v_out[3 * n + k] = o[3];
        }
    }
}

/* Finest-level smoothing sweep: one Jacobi sweep of A(u) = b (Algorithm 1),
 * blended with the previous iterate, u_new = (1 - omega) u + omega J(u).
 * omega = 1 is Algorithm 1 itself; 0 < omega < 1 keeps u_new admissible (a
 * convex combination of admissible states) and has the same fixed point.    */
void or_sweep(const or_grid* g, const double* sigma, double omega, const double* b, const double* v_in,
              double* v_out)
{
    const size_t n = ncell(g);
    or_jacobi(g, sigma, 0.0, 1.0, NULL, b, v_in, v_out);
    if (omega != 1.0)
        for (size_t k = 0; k < NFIELD * n; ++k) v_out[k] = (1.0 - omega) * v_in[k] + omega * v_out[k];
}

/* Red-black nonlinear Gauss-Seidel sweep, the alternative to the Jacobi
 * smoother of Sect. 6.3: the "red" cells (i + j even) take the relaxed Jacobi
 * update of v_in, then the "black" cells (i + j odd) take the relaxed Jacobi
 * update of that intermediate state.  Where every neighbour of a cell has the
 * other colour (sides of even length or not periodic), each half is the
 * Gauss-Seidel update of one colour.  Each cell's update is the local solve
 * of a Jacobi sweep with admissible neighbours, so the argument of Prop. 1
 * keeps every state admissible.                                              */
void or_rb_sweep(const or_grid* g, const double* sigma, double omega, const double* b, const double* v_in,
                 double* v_out)
{
    const size_t n = ncell(g);
    double* J = dalloc(NFIELD * n);
    double* mid = dalloc(NFIELD * n);
    or_sweep(g, sigma, omega, b, v_in, J);
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
            const size_t k = (size_t)j * g->nx + i;
            for (int m = 0; m < NFIELD; ++m) mid[m * n + k] = ((i + j) % 2 == 0) ? J[m * n + k] : v_in[m * n + k];
        }
    or_sweep(g, sigma, omega, b, mid, J);
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
            const size_t k = (size_t)j * g->nx + i;
            for (int m = 0; m < NFIELD; ++m) v_out[m * n + k] = ((i + j) % 2 == 1) ? J[m * n + k] : mid[m * n + k];
        }
    free(J);
    free(mid);
}

/* ------------------------------------------------------------------------- */
/* Grid transfer, Sect. 4.2.  Fine cell 2I coincides with coarse cell I; odd
 * fine cells interpolate linearly (eq. prolongationOperator1D); restriction is
 * full weighting 1/4, 1/2, 1/4 (= 2^-d P^T, eq. restrictionOperator in 2-D as
 * the tensor product).  Periodic axes wrap; on other axes a stencil point
 * outside the domain is dropped and the remaining weights renormalised to 1.  */
static int prolong_w1d(int i, int nc, int periodic, int idx[2], double w[2])
{
    if (i % 2 == 0) {
        idx[0] = i / 2;
        w[0] = 1.0;
        return 1;
    }
    int I0 = (i - 1) / 2, I1 = (i + 1) / 2;
    if (I1 >= nc) {
        if (periodic) {
            I1 -= nc;
        } else {
            idx[0] = I0;
            w[0] = 1.0;
            return 1;
        }
    }
    idx[0] = I0;
    idx[1] = I1;
    w[0] = 0.5;
    w[1] = 0.5;
    return 2;
}

static int restrict_w1d(int I, int nf, int periodic, int idx[3], double w[3])
{
    static const int off[3] = {-1, 0, 1};
    static const double base[3] = {0.25, 0.5, 0.25};
    int cnt = 0;
    double sum = 0.0;
    for (int m = 0; m < 3; ++m) {
        int f = 2 * I + off[m];
        if (f < 0 || f >= nf) {
            if (!periodic) continue;
            f = (f + nf) % nf;
        }
        idx[cnt] = f;
        w[cnt] = base[m];
        sum += base[m];
        ++cnt;
    }
    for (int m = 0; m < cnt; ++m) w[m] /= sum;
    return cnt;
}

or_grid or_coarse_grid(const or_grid* g)
{
    or_grid c = *g;
    c.nx = g->nx / 2;
    c.hx = g->hx * 2.0;
    if (g->dim == 2) {
        c.ny = g->ny / 2;
        c.hy = g->hy * 2.0;
    }
    return c;
}

/* The alternative pair of Sect. 6.3 (the transfer operators are named there as
 * a choice that changes the speed, not the solution): coarse cell I is the
 * union of fine cells 2I and 2I+1 along each axis; the prolongation gives both
 * the coarse value (piecewise constant), and R = 2^-d P^T is the mean of the
 * 2^d fine cells.                                                             */
static int mean_w1d(int I, int idx[3], double w[3])
{
    idx[0] = 2 * I;
    idx[1] = 2 * I + 1;
    w[0] = w[1] = 0.5;
    return 2;
}

static int const_w1d(int i, int idx[2], double w[2])
{
    idx[0] = i / 2;
    w[0] = 1.0;
    return 1;
}

void or_restrict_t(const or_grid* fine, const double* x_fine, int32_t nfields, double* x_coarse, int32_t transfer)
{
    or_grid cg = or_coarse_grid(fine);
    const size_t nf = ncell(fine), nc = ncell(&cg);
    const int px = fine->bc_kind[0] == OR_BC_PERIODIC, py = fine->bc_kind[2] == OR_BC_PERIODIC;
#pragma omp parallel for schedule(static)
    for (int J = 0; J < cg.ny; ++J) {
        for (int I = 0; I < cg.nx; ++I) {
            int ix[3], iy[3];
            double wx[3], wy[3];
            int cx, cy;
            if (transfer == OR_TRANSFER_MEAN) cx = mean_w1d(I, ix, wx);
            else cx = restrict_w1d(I, fine->nx, px, ix, wx);
            if (fine->dim == 2) {
                if (transfer == OR_TRANSFER_MEAN) cy = mean_w1d(J, iy, wy);
                else cy = restrict_w1d(J, fine->ny, py, iy, wy);
            } else {
                cy = 1;
                iy[0] = 0;
                wy[0] = 1.0;
            }
            for (int q = 0; q < nfields; ++q) {
                double s = 0.0;
                for (int b = 0; b < cy; ++b)
                    for (int a = 0; a < cx; ++a)
                        s += wx[a] * wy[b] * x_fine[q * nf + (size_t)iy[b] * fine->nx + ix[a]];
                x_coarse[q * nc + (size_t)J * cg.nx + I] = s;
            }
        }
    }
}

void or_prolong_t(const or_grid* fine, const double* x_coarse, int32_t nfields, double* x_fine, int32_t transfer)
{
    or_grid cg = or_coarse_grid(fine);
    const size_t nf = ncell(fine), nc = ncell(&cg);
    const int px = fine->bc_kind[0] == OR_BC_PERIODIC, py = fine->bc_kind[2] == OR_BC_PERIODIC;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < fine->ny; ++j) {
        for (int i = 0; i < fine->nx; ++i) {
            int ix[2], iy[2];
            double wx[2], wy[2];
            int cx, cy;
            if (transfer == OR_TRANSFER_MEAN) cx = const_w1d(i, ix, wx);
            else cx = prolong_w1d(i, cg.nx, px, ix, wx);
            if (fine->dim == 2) {
                if (transfer == OR_TRANSFER_MEAN) cy = const_w1d(j, iy, wy);
                else cy = prolong_w1d(j, cg.ny, py, iy, wy);
            } else {
                cy = 1;
                iy[0] = 0;
                wy[0] = 1.0;
            }
            for (int q = 0; q < nfields; ++q) {
                double s = 0.0;
                for (int b = 0; b < cy; ++b)
                    for (int a = 0; a < cx; ++a)
                        s += wx[a] * wy[b] * x_coarse[q * nc + (size_t)iy[b] * cg.nx + ix[a]];
                x_fine[q * nf + (size_t)j * fine->nx + i] = s;
            }
        }
    }
}

void or_restrict(const or_grid* fine, const double* x_fine, int32_t nfields, double* x_coarse)
{
    or_restrict_t(fine, x_fine, nfields, x_coarse, OR_TRANSFER_FULL);
}

void or_prolong(const or_grid* fine, const double* x_coarse, int32_t nfields, double* x_fine)
{
    or_prolong_t(fine, x_coarse, nfields, x_fine, OR_TRANSFER_FULL);
}

/* ------------------------------------------------------------------------- */
/* Largest step along a ray that stays admissible:
 *   tau*(w, s) = sup{tau >= 0 : w + tau s in S'}  (w admissible),
 * the smallest of -E/s_E (s_E < 0), -T/s_T (s_T < 0) and the first positive
 * root of q(tau) = c^2 (E + tau s_E)^2 - |F + tau s_F|^2 = A tau^2 + 2B tau + C.
 * Returns +inf when the whole ray is admissible.                             */
double or_ray(double c, const double w[4], const double s[4])
{
    double tau = INFINITY;
    if (s[0] < 0.0) tau = fmin(tau, -w[0] / s[0]);
    if (s[3] < 0.0) tau = fmin(tau, -w[3] / s[3]);
    const double c2 = c * c;
    const double A = c2 * s[0] * s[0] - (s[1] * s[1] + s[2] * s[2]);
    const double B = c2 * w[0] * s[0] - (w[1] * s[1] + w[2] * s[2]);
    double C = c2 * w[0] * w[0] - (w[1] * w[1] + w[2] * w[2]);
    if (C < 0.0) C = 0.0;
    double r = INFINITY;
    if (A == 0.0) {
        if (B < 0.0) r = C / (-2.0 * B);
    } else {
        double disc = B * B - A * C;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            if (B < 0.0) r = C / (-B + sq); /* smaller positive root, no cancellation */
            else if (A < 0.0) r = (B + sq) / (-A);
        }
    }
    return fmin(tau, r);
}

/* The explicit part of one pseudo-time step (Algorithm 3): per cell, sub-steps
 * u~ <- u~ + dtau_ex M^{-1} f from u, each eta times the admissible length of
 * the ray left (or_ray), never past dtau in total, at most sub_steps of them.
 * Writes each cell's pseudo time tau_i <= dtau and u~.                        */
void or_pseudo_time(const or_grid* g, const or_params* p, double dtau, const double* f, const double* u_in,
                    double* taus, double* u_tilde)
{
    const size_t n = ncell(g);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < g->ny; ++j) {
        for (int i = 0; i < g->nx; ++i) {
            size_t k = (size_t)j * g->nx + i;
            double s[4] = {f[k], f[n + k], f[2 * n + k], f[3 * n + k] / g->c_v};
            double w[4] = {u_in[k], u_in[n + k], u_in[2 * n + k], u_in[3 * n + k]};
            double tau_ex = 0.0;
            for (int it = 0; it < p->sub_steps && tau_ex < dtau; ++it) {
                double ts = or_ray(g->c, w, s);
                double d = fmin(dtau - tau_ex, p->eta * ts);
                for (int m = 0; m < 4; ++m) w[m] += d * s[m];
                tau_ex += d;
            }
            taus[k] = tau_ex;
            for (int m = 0; m < 4; ++m) u_tilde[m * n + k] = w[m];
        }
    }
}

/* One pseudo-time step of Algorithm 3 for  M du/dtau + A(u) = f :
 * per cell, explicit sub-steps u~ <- u~ + dtau_ex M^{-1} f, each as long as
 * eta times the admissible length of the ray and never past dtau_im in total,
 * at most sub_steps of them, reaching the pseudo-time tau_i <= dtau_im; then
 * the implicit step (M + tau A)(u) = M u~ with nu_l Jacobi sweeps started from
 * u, where tau is each cell's own tau_i (pseudo_local = 1: the split step of
 * eq. (splitting) with a local step, whose steady state is A(u) = f in every
 * cell with tau_i > 0) or dtau_im everywhere (pseudo_local = 0, as printed).  */
void or_pseudo_step(const or_grid* g, const double* sigma, const or_params* p, double dtau,
                    const double* f, const double* u_in, double* u_out)
{
    const size_t n = ncell(g);
    double* rhs = dalloc(NFIELD * n);
    double* taus = dalloc(n);
    or_pseudo_time(g, p, dtau, f, u_in, taus, rhs);
    for (size_t k = 0; k < n; ++k) rhs[3 * n + k] *= g->c_v; /* M u~ */
    double* cur = dalloc(NFIELD * n);
    double* nxt = dalloc(NFIELD * n);
    memcpy(cur, u_in, NFIELD * n * sizeof(double));
    for (int s = 0; s < p->nu_l; ++s) {
        or_jacobi(g, sigma, 1.0, dtau, p->pseudo_local ? taus : NULL, rhs, cur, nxt);
        double* t = cur;
        cur = nxt;
        nxt = t;
    }
    memcpy(u_out, cur, NFIELD * n * sizeof(double));
    free(cur);
    free(nxt);
    free(rhs);
    free(taus);
}

/* Correction with admissibility, eq. (prolongatedSol): where the corrected
 * state w = u + P(e) is not admissible, take one implicit pseudo-time step of
 * d u/d taubar + u = w from u, u_new = (u + dtaubar w)/(1 + dtaubar), with
 * dtaubar/(1 + dtaubar) = eta tau*(u, w - u) so that u_new is admissible.      */
void or_project(const or_grid* g, const or_params* p, const double* u, const double* w, double* out)
{
    const size_t n = ncell(g);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < g->ny; ++j) {
        for (int i = 0; i < g->nx; ++i) {
            size_t k = (size_t)j * g->nx + i;
            double uu[4], ww[4], s[4];
            for (int m = 0; m < 4; ++m) {
                uu[m] = u[m * n + k];
                ww[m] = w[m * n + k];
                s[m] = ww[m] - uu[m];
            }
            if (or_admissible(g->c, ww)) {
                for (int m = 0; m < 4; ++m) out[m * n + k] = ww[m];
                continue;
            }
            double ts = or_ray(g->c, uu, s);
            if (ts > 1.0) ts = 1.0;
            double theta = p->eta * ts;
            double dtb = theta / (1.0 - theta);
            for (int m = 0; m < 4; ++m) out[m * n + k] = (uu[m] + dtb * ww[m]) / (1.0 + dtb);
        }
    }
}

/* ------------------------------------------------------------------------- */
int32_t or_num_levels(const or_grid* g, const or_params* p)
{
    int L = 1, nx = g->nx, ny = g->ny;
    for (;;) {
        if (p->levels > 0 && L >= p->levels) break;
        int ok = (nx % 2 == 0) && nx / 2 >= 4;
        if (g->dim == 2) ok = ok && (ny % 2 == 0) && ny / 2 >= 4;
        if (!ok) break;
        nx /= 2;
        if (g->dim == 2) ny /= 2;
        ++L;
    }
    return L;
}

static void sweeps(const or_grid* g, const double* sigma, double omega, int smoother, const double* b,
                   const double* v0, int nu, double* out)
{
    const size_t n = ncell(g);
    double* cur = dalloc(NFIELD * n);
    double* nxt = dalloc(NFIELD * n);
    memcpy(cur, v0, NFIELD * n * sizeof(double));
    for (int s = 0; s < nu; ++s) {
        if (smoother == OR_SMOOTH_RBGS) or_rb_sweep(g, sigma, omega, b, cur, nxt);
        else or_sweep(g, sigma, omega, b, cur, nxt);
        double* t = cur;
        cur = nxt;
        nxt = t;
    }
    memcpy(out, cur, NFIELD * n * sizeof(double));
    free(cur);
    free(nxt);
}

static void pseudo_smooth(const or_grid* g, const double* sigma, const or_params* p, double dtau, const double* f,
                          const double* u0, double* out)
{
    const size_t n = ncell(g);
    double* cur = dalloc(NFIELD * n);
    double* nxt = dalloc(NFIELD * n);
    memcpy(cur, u0, NFIELD * n * sizeof(double));
    for (int m = 0; m < p->pseudo_steps; ++m) {
        or_pseudo_step(g, sigma, p, dtau, f, cur, nxt);
        double* t = cur;
        cur = nxt;
        nxt = t;
    }
    memcpy(out, cur, NFIELD * n * sizeof(double));
    free(cur);
    free(nxt);
}

/* One V-cycle of the overall algorithm (Appendix A) with the FAS coarse
 * problems of Sect. 4.2 solved in pseudo-time (Sect. 4.3):
 *   finest: nu0 (relaxed) Jacobi sweeps, residual rbar = b - A_0(u_0);
 *   level l: v_l = R(u_{l-1}), f_l = A_l(v_l) + R(rbar_{l-1}), m pseudo-time
 *            steps from v_l, rbar_l = f_l - A_l(u_l);
 *   upward:  u_l <- projected(u_l + P(u_{l+1} - v_{l+1})), then the same
 *            smoothing again (nu0 sweeps on the finest level).              */
static void vcycle_loop(const or_grid* g, const double* sigma, const or_params* p, double dtau, const double* b,
                        const double* v, double* out)
{
    const int L = or_num_levels(g, p);
    or_grid* G = (or_grid*)malloc(sizeof(or_grid) * L);
    double **U = (double**)calloc(L, sizeof(double*)), **V = (double**)calloc(L, sizeof(double*));
    double **Fr = (double**)calloc(L, sizeof(double*)), **S = (double**)calloc(L, sizeof(double*));
    G[0] = *g;
    for (int l = 1; l < L; ++l) G[l] = or_coarse_grid(&G[l - 1]);
    S[0] = (double*)sigma;
    for (int l = 1; l < L; ++l) {
        S[l] = dalloc(2 * ncell(&G[l]));
        or_restrict_t(&G[l - 1], S[l - 1], 2, S[l], p->transfer); /* coarse opacity by the same restriction */
    }
    for (int l = 0; l < L; ++l) {
        U[l] = dalloc(NFIELD * ncell(&G[l]));
        if (l > 0) {
            V[l] = dalloc(NFIELD * ncell(&G[l]));
            Fr[l] = dalloc(NFIELD * ncell(&G[l]));
        }
    }

    sweeps(&G[0], S[0], p->omega, p->smoother, b, v, p->nu0, U[0]);
    if (L > 1) {
        double* rbar = dalloc(NFIELD * ncell(&G[0]));
        or_residual(&G[0], S[0], b, U[0], rbar);
        for (int l = 1; l < L; ++l) {
            const size_t n = ncell(&G[l]);
            double* rr = dalloc(NFIELD * n);
            or_restrict_t(&G[l - 1], U[l - 1], NFIELD, V[l], p->transfer);
            or_restrict_t(&G[l - 1], rbar, NFIELD, rr, p->transfer);
            or_apply_A(&G[l], S[l], V[l], Fr[l]);
            for (size_t k = 0; k < NFIELD * n; ++k) Fr[l][k] += rr[k];
            free(rr);
            pseudo_smooth(&G[l], S[l], p, dtau, Fr[l], V[l], U[l]);
            free(rbar);
            rbar = NULL;
            if (l < L - 1) {
                rbar = dalloc(NFIELD * n);
                or_apply_A(&G[l], S[l], U[l], rbar);
                for (size_t k = 0; k < NFIELD * n; ++k) rbar[k] = Fr[l][k] - rbar[k];
            }
        }
        free(rbar);
        for (int l = L - 2; l >= 0; --l) {
            const size_t n = ncell(&G[l]), nc = ncell(&G[l + 1]);
            double* e = dalloc(NFIELD * nc);
            double* w = dalloc(NFIELD * n);
            for (size_t k = 0; k < NFIELD * nc; ++k) e[k] = U[l + 1][k] - V[l + 1][k];
            or_prolong_t(&G[l], e, NFIELD, w, p->transfer);
            for (size_t k = 0; k < NFIELD * n; ++k) w[k] += U[l][k];
            or_project(&G[l], p, U[l], w, U[l]);
            free(e);
            free(w);
            double* t = dalloc(NFIELD * n);
            if (l == 0) sweeps(&G[0], S[0], p->omega, p->smoother, b, U[0], p->nu0, t);
            else pseudo_smooth(&G[l], S[l], p, dtau, Fr[l], U[l], t);
            memcpy(U[l], t, NFIELD * n * sizeof(double));
            free(t);
        }
    }
    memcpy(out, U[0], NFIELD * ncell(g) * sizeof(double));
    for (int l = 0; l < L; ++l) {
        free(U[l]);
        free(V[l]);
        free(Fr[l]);
        if (l > 0) free(S[l]);
    }
    free(U);
    free(V);
    free(Fr);
    free(S);
    free(G);
}

/* The cycle of Sect. 4 written recursively over the coarse problems, for the
 * other cycle shapes Sect. 6.3 names.  coarse_visit(l) takes the FAS problem
 * A_l(u) = f_l of level l from u: m pseudo-time steps (Algorithm 3); above the
 * coarsest level, the residual and the iterate restricted to level l+1, its
 * problem visited once (V), twice (W), or by an F-cycle then a V-cycle (F),
 * the correction with admissibility (eq. prolongatedSol) and m pseudo-time
 * steps again.  The finest level is the same with nu0 Jacobi sweeps in place
 * of the pseudo-time steps.  With kind V this is or_vcycle's cycle.          */
typedef struct {
    int L, transfer;
    or_grid* G;
    double **S, **U, **V, **F;
} cyc_levels;

static void coarse_visit(const cyc_levels* c, const or_params* p, double dtau, int l, int kind);

/* restrict u_l and its residual rhs_l - A_l(u_l) to level l+1: v_{l+1}, f_{l+1} = A(v_{l+1}) + R(residual) */
static void descend(const cyc_levels* c, int l, const double* rhs)
{
    const size_t n = ncell(&c->G[l]), nc = ncell(&c->G[l + 1]);
    double* rb = dalloc(NFIELD * n);
    double* rr = dalloc(NFIELD * nc);
    or_apply_A(&c->G[l], c->S[l], c->U[l], rb);
    for (size_t k = 0; k < NFIELD * n; ++k) rb[k] = rhs[k] - rb[k];
    or_restrict_t(&c->G[l], c->U[l], NFIELD, c->V[l + 1], c->transfer);
    or_restrict_t(&c->G[l], rb, NFIELD, rr, c->transfer);
    or_apply_A(&c->G[l + 1], c->S[l + 1], c->V[l + 1], c->F[l + 1]);
    for (size_t k = 0; k < NFIELD * nc; ++k) c->F[l + 1][k] += rr[k];
    memcpy(c->U[l + 1], c->V[l + 1], NFIELD * nc * sizeof(double));
    free(rb);
    free(rr);
}

/* visit level l+1 as `kind` prescribes, then correct u_l */
static void visit_and_correct(const cyc_levels* c, const or_params* p, double dtau, int l, int kind)
{
    if (kind == OR_CYCLE_F) {
        coarse_visit(c, p, dtau, l + 1, OR_CYCLE_F);
        coarse_visit(c, p, dtau, l + 1, OR_CYCLE_V);
    } else {
        const int times = (kind == OR_CYCLE_W) ? 2 : 1;
        for (int t = 0; t < times; ++t) coarse_visit(c, p, dtau, l + 1, kind);
    }
    const size_t n = ncell(&c->G[l]), nc = ncell(&c->G[l + 1]);
    double* e = dalloc(NFIELD * nc);
    double* w = dalloc(NFIELD * n);
    for (size_t k = 0; k < NFIELD * nc; ++k) e[k] = c->U[l + 1][k] - c->V[l + 1][k];
    or_prolong_t(&c->G[l], e, NFIELD, w, c->transfer);
    for (size_t k = 0; k < NFIELD * n; ++k) w[k] += c->U[l][k];
    or_project(&c->G[l], p, c->U[l], w, c->U[l]);
    free(e);
    free(w);
}

static void coarse_visit(const cyc_levels* c, const or_params* p, double dtau, int l, int kind)
{
    const size_t n = ncell(&c->G[l]);
    double* t = dalloc(NFIELD * n);
    pseudo_smooth(&c->G[l], c->S[l], p, dtau, c->F[l], c->U[l], t);
    memcpy(c->U[l], t, NFIELD * n * sizeof(double));
    if (l < c->L - 1) {
        descend(c, l, c->F[l]);
        visit_and_correct(c, p, dtau, l, kind);
        pseudo_smooth(&c->G[l], c->S[l], p, dtau, c->F[l], c->U[l], t);
        memcpy(c->U[l], t, NFIELD * n * sizeof(double));
    }
    free(t);
}

void or_cycle(const or_grid* g, const double* sigma, const or_params* p, int32_t kind, double dtau, const double* b,
              const double* v, double* out)
{
    cyc_levels c;
    c.L = or_num_levels(g, p);
    c.transfer = p->transfer;
    c.G = (or_grid*)malloc(sizeof(or_grid) * c.L);
    c.S = (double**)calloc(c.L, sizeof(double*));
    c.U = (double**)calloc(c.L, sizeof(double*));
    c.V = (double**)calloc(c.L, sizeof(double*));
    c.F = (double**)calloc(c.L, sizeof(double*));
    c.G[0] = *g;
    c.S[0] = (double*)sigma;
    for (int l = 1; l < c.L; ++l) {
        c.G[l] = or_coarse_grid(&c.G[l - 1]);
        c.S[l] = dalloc(2 * ncell(&c.G[l]));
        or_restrict_t(&c.G[l - 1], c.S[l - 1], 2, c.S[l], p->transfer); /* coarse opacity by the same restriction */
    }
    for (int l = 0; l < c.L; ++l) {
        c.U[l] = dalloc(NFIELD * ncell(&c.G[l]));
        c.V[l] = dalloc(NFIELD * ncell(&c.G[l]));
        c.F[l] = dalloc(NFIELD * ncell(&c.G[l]));
    }
    sweeps(&c.G[0], c.S[0], p->omega, p->smoother, b, v, p->nu0, c.U[0]);
    if (c.L > 1) {
        double* t = dalloc(NFIELD * ncell(g));
        descend(&c, 0, b);
        visit_and_correct(&c, p, dtau, 0, kind);
        sweeps(&c.G[0], c.S[0], p->omega, p->smoother, b, c.U[0], p->nu0, t);
        memcpy(c.U[0], t, NFIELD * ncell(g) * sizeof(double));
        free(t);
    }
    memcpy(out, c.U[0], NFIELD * ncell(g) * sizeof(double));
    for (int l = 0; l < c.L; ++l) {
        free(c.U[l]);
        free(c.V[l]);
        free(c.F[l]);
        if (l > 0) free(c.S[l]);
    }
    free(c.G);
    free(c.S);
    free(c.U);
    free(c.V);
    free(c.F);
}

/* One cycle of the shape p->cycle (V: the loop form above). */
void or_vcycle(const or_grid* g, const double* sigma, const or_params* p, double dtau, const double* b,
               const double* v, double* out)
{
    if (p->cycle == OR_CYCLE_V) vcycle_loop(g, sigma, p, dtau, b, v, out);
    else or_cycle(g, sigma, p, p->cycle, dtau, b, v, out);
}

/* Pseudo-time step adaptation after each cycle (Appendix A): grow by 1.1 when
 * the residual changed by more than eps_inc, halve it when less than eps_dec.
 * OR_DTAU_LITERAL measures the change as |r_k - r_{k-1}| / r_0 as printed;
 * OR_DTAU_SIGNED uses the signed relative decrease (r_{k-1} - r_k) / r_{k-1}. */
static double adapt_dtau(const or_params* p, double dtau, double r0, double rprev, double r)
{
    double d;
    if (p->dtau_rule == OR_DTAU_LITERAL) d = fabs(r - rprev) / r0;
    else d = (rprev - r) / rprev;
    if (d > p->eps_inc) dtau *= 1.1;
    if (d < p->eps_dec) dtau *= 0.5;
    if (dtau < p->dtau_min) dtau = p->dtau_min;
    if (dtau > p->dtau_max) dtau = p->dtau_max;
    return dtau;
}

/* Implicit Euler time steps, each solved by cycles until
 * |b - A(v)| <= rtol |b - A(v^n)| (relative residual of Sect. 5), with
 * b = (E^n, F^n, C_v T^n) and the initial guess v^n.  A residual at the
 * rounding level of evaluating A, 16 eps a |b| (a = 1 + c dt/hx + c dt/hy),
 * also counts as converged, so an exact solution takes zero cycles.  The
 * pseudo-time step dtau_im starts at dtau_im0 and is adapted after every cycle;
 * the overall algorithm of Appendix A (one time step) does not set it among its
 * first steps and Sect. 5 gives only its initial value, so with dtau_carry it
 * runs on into the next time step (dtau_carry 0 restarts it at dtau_im0).
 * Returns 0 on success, 3 when max_cycles was reached (v then holds the last
 * iterate).                                                                 */
int32_t or_step(const or_grid* g, const double* sigma, const or_params* p, double* v, int32_t nsteps, or_info* info,
                double* history, int32_t history_len)
{
    const size_t n = ncell(g);
    double* b = dalloc(NFIELD * n);
    double* r = dalloc(NFIELD * n);
    double* nv = dalloc(NFIELD * n);
    int32_t status = 0, hpos = 0, total = 0;
    double r0 = 0.0, rel = 0.0, dtau = p->dtau_im0;
    for (int step = 0; step < nsteps; ++step) {
        memcpy(b, v, NFIELD * n * sizeof(double));
        for (size_t k = 0; k < n; ++k) b[3 * n + k] = g->c_v * v[3 * n + k];
        if (!p->dtau_carry) dtau = p->dtau_im0;
        or_residual(g, sigma, b, v, r);
        r0 = or_norm(g, r);
        const double floor_r = 16.0 * DBL_EPSILON * diag_a(g) * or_norm(g, b);
        rel = 0.0;
        if (r0 <= floor_r) continue;
        double rprev = r0;
        int conv = 0;
        for (int kc = 1; kc <= p->max_cycles; ++kc) {
            or_vcycle(g, sigma, p, dtau, b, v, nv);
            memcpy(v, nv, NFIELD * n * sizeof(double));
            or_residual(g, sigma, b, v, r);
            double rk = or_norm(g, r);
            ++total;
            rel = rk / r0;
            if (history && hpos < history_len) history[hpos++] = rel;
            dtau = adapt_dtau(p, dtau, r0, rprev, rk);
            rprev = rk;
            if (rel <= p->rtol || rk <= floor_r) {
                conv = 1;
                break;
            }
        }
        if (!conv) {
            status = 3;
            break;
        }
    }
    if (info) {
        info->cycles = total;
        info->status = status;
        info->levels = or_num_levels(g, p);
        info->r0 = r0;
        info->rel_residual = rel;
        info->dtau = dtau;
    }
    free(b);
    free(r);
    free(nv);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Explicit reference solver of the homogeneous M1 system (Sect. 2.2 with no
 * sources; the explicit HLL scheme the paper compares against in Sect. 5).  */

/* Smallest and largest eigenvalue of the Jacobian of the directional flux
 * (axis 0: x, 1: y) of the M1 system at U = (E, F): with f = |F|/(cE),
 * s = sqrt(4 - 3 f^2) and mu the cosine between F and the axis,
 *   lambda = c (f mu -+ sqrt(2/3 (4 - 3 f^2 - s) + 2 mu^2 (2 - f^2 - s))) / s,
 * the wave speeds of the M1 model in closed form (the eigenvalues the HLL
 * speeds of Sect. 2.2 come from; they lie in [-c, c]).                       */
void or_wave_speeds(double c, const double U[3], int axis, double* lm, double* lp)
{
    const double normF = sqrt(U[1] * U[1] + U[2] * U[2]);
    double f = normF / (c * U[0]);
    if (f > 1.0) f = 1.0;
    const double mu = normF > 0.0 ? (axis == 0 ? U[1] : U[2]) / normF : 0.0;
    const double s = sqrt(4.0 - 3.0 * f * f);
    double rad = 2.0 / 3.0 * (4.0 - 3.0 * f * f - s) + 2.0 * mu * mu * (2.0 - f * f - s);
    if (rad < 0.0) rad = 0.0; /* rounding at f = 1 */
    const double r = sqrt(rad);
    *lm = c * (f * mu - r) / s;
    *lp = c * (f * mu + r) / s;
}

/* Directional physical flux G_axis(U). */
static void phys_flux(double c, const double U[3], int axis, double G[3])
{
    double P[3];
    or_closure(U[0], U[1], U[2], c, P);
    if (axis == 0) {
        G[0] = U[1];
        G[1] = c * c * P[0];
        G[2] = c * c * P[1];
    } else {
        G[0] = U[2];
        G[1] = c * c * P[1];
        G[2] = c * c * P[2];
    }
}

/* Numerical flux between the states UL (low side) and UR (high side) along
 * `axis`: HLL with speeds lm = min(lambda-(UL), lambda-(UR)) and
 * lp = max(lambda+(UL), lambda+(UR)) (hll = 1), or the speeds -c and c, the
 * Rusanov flux the implicit scheme uses (hll = 0).                            */
static void num_flux(double c, const double UL[3], const double UR[3], int axis, int hll, double H[3])
{
    double GL[3], GR[3], lm = -c, lp = c;
    phys_flux(c, UL, axis, GL);
    phys_flux(c, UR, axis, GR);
    if (hll) {
        double a, b, a2, b2;
        or_wave_speeds(c, UL, axis, &a, &b);
        or_wave_speeds(c, UR, axis, &a2, &b2);
        lm = fmin(a, a2);
        lp = fmax(b, b2);
    }
    if (lm >= 0.0) {
        for (int m = 0; m < 3; ++m) H[m] = GL[m];
    } else if (lp <= 0.0) {
        for (int m = 0; m < 3; ++m) H[m] = GR[m];
    } else {
        for (int m = 0; m < 3; ++m) H[m] = (lp * GL[m] - lm * GR[m] + lp * lm * (UR[m] - UL[m])) / (lp - lm);
    }
}

/* One explicit Euler step of dU/dt + div G(U) = 0 (E and F; T is left as it
 * is) with the grid's dt, from v into out: finite volumes with the numerical
 * flux above at every face, boundary faces taking the ghost state of the
 * boundary rule (periodic, reflective, Neumann, Dirichlet, inflow).  Stable
 * and admissible for c dt (1/hx + 1/hy) <= 1.                                */
void or_explicit_step(const or_grid* g, int hll, const double* v, double* out)
{
    const size_t n = ncell(g);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < g->ny; ++j) {
        for (int i = 0; i < g->nx; ++i) {
            const size_t k = (size_t)j * g->nx + i;
            double U[3] = {v[k], v[n + k], v[2 * n + k]}, N[3], H[3], d[3] = {0.0, 0.0, 0.0};
            neighbour(g, v, i, j, -1, 0, N); /* face i-1/2 */
            num_flux(g->c, N, U, 0, hll, H);
            for (int m = 0; m < 3; ++m) d[m] += H[m] / g->hx;
            neighbour(g, v, i, j, +1, 0, N); /* face i+1/2 */
            num_flux(g->c, U, N, 0, hll, H);
            for (int m = 0; m < 3; ++m) d[m] -= H[m] / g->hx;
            if (g->dim == 2) {
                neighbour(g, v, i, j, 0, -1, N);
                num_flux(g->c, N, U, 1, hll, H);
                for (int m = 0; m < 3; ++m) d[m] += H[m] / g->hy;
                neighbour(g, v, i, j, 0, +1, N);
                num_flux(g->c, U, N, 1, hll, H);
                for (int m = 0; m < 3; ++m) d[m] -= H[m] / g->hy;
            }
            for (int m = 0; m < 3; ++m) out[m * n + k] = U[m] + g->dt * d[m];
            out[3 * n + k] = v[3 * n + k];
        }
    }
}

/* Explicit steps from v (updated in place) until the largest change of E in a
 * step is at most tol times the largest E, or max_steps.  Returns the steps. */
int32_t or_explicit_run(const or_grid* g, int hll, double* v, int32_t max_steps, double tol)
{
    const size_t n = ncell(g);
    double* nv = dalloc(NFIELD * n);
    int32_t s = 0;
    while (s < max_steps) {
        or_explicit_step(g, hll, v, nv);
        ++s;
        double dmax = 0.0, emax = 0.0;
        for (size_t k = 0; k < n; ++k) {
            dmax = fmax(dmax, fabs(nv[k] - v[k]));
            emax = fmax(emax, fabs(nv[k]));
        }
        memcpy(v, nv, NFIELD * n * sizeof(double));
        if (dmax <= tol * emax) break;
    }
    free(nv);
    return s;
}
