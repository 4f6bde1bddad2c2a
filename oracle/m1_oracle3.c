/*
 * m1_oracle3.c -- TEST INFRASTRUCTURE ONLY: the plain FP64 CPU oracle of the
 * method in three dimensions.
 *
 * The paper writes its scheme in 1-D, says the extension to more dimensions
 * is direct (Sect. 2.2), and defines the restriction for d = 1, 2, 3 as
 * R = 2^-d P^T (Sect. 4.2).  This file is that extension, written out like the
 * 2-D oracle: per axis the Rusanov left/right operators of Sect. 3.1 with the
 * directional flux (F_axis, c^2 P[:, axis]), the sources of eq. (m1) taken
 * implicitly, the nonlinear Jacobi sweep (Algorithm 1), the pseudo-time steps
 * of Algorithm 3, the admissible correction of eq. (prolongatedSol), trilinear
 * prolongation and its scaled transpose, and the V-cycle (with the W and F
 * shapes of Sect. 6.3) / time-step driver of
 * Appendix A with the same readings as the 2-D oracle.  The single-cell
 * gas-radiation solve is the 2-D oracle's (the flux components decouple from
 * it and share one divisor).
 */
#include "m1_oracle3.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NF3 5 /* E, Fx, Fy, Fz, T */

static size_t ncell3(const or3_grid* g) { return (size_t)g->nx * (size_t)g->ny * (size_t)g->nz; }

static double* dalloc3(size_t n)
{
    double* p = (double*)calloc(n ? n : 1, sizeof(double));
    if (!p) abort();
    return p;
}

static size_t at(const or3_grid* g, int i, int j, int k) { return ((size_t)k * g->ny + j) * g->nx + i; }

/* Sect. 2.1 closure in 3-D: P = ((1-chi)/2 I + (3chi-1)/2 n n) E, stored
 * (Pxx, Pxy, Pxz, Pyy, Pyz, Pzz).                                            */
void or3_closure(double E, double Fx, double Fy, double Fz, double c, double P[6])
{
    const double normF = sqrt(Fx * Fx + Fy * Fy + Fz * Fz);
    double f = normF / (c * E);
    if (f > 1.0) f = 1.0;
    const double chi = or_chi(f);
    double n[3] = {0.0, 0.0, 0.0};
    if (normF > 0.0) {
        n[0] = Fx / normF;
        n[1] = Fy / normF;
        n[2] = Fz / normF;
    }
    const double iso = 0.5 * (1.0 - chi), dir = 0.5 * (3.0 * chi - 1.0);
    P[0] = (iso + dir * n[0] * n[0]) * E;
    P[1] = (dir * n[0] * n[1]) * E;
    P[2] = (dir * n[0] * n[2]) * E;
    P[3] = (iso + dir * n[1] * n[1]) * E;
    P[4] = (dir * n[1] * n[2]) * E;
    P[5] = (iso + dir * n[2] * n[2]) * E;
}

int or3_admissible(double c, const double w[5])
{
    return w[0] > 0.0 && w[4] > 0.0 && (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) <= c * c * w[0] * w[0];
}

/* Largest tau with w + tau s admissible (as or_ray, with three flux components). */
double or3_ray(double c, const double w[5], const double s[5])
{
    double tau = INFINITY;
    if (s[0] < 0.0) tau = fmin(tau, -w[0] / s[0]);
    if (s[4] < 0.0) tau = fmin(tau, -w[4] / s[4]);
    const double c2 = c * c;
    const double A = c2 * s[0] * s[0] - (s[1] * s[1] + s[2] * s[2] + s[3] * s[3]);
    const double B = c2 * w[0] * s[0] - (w[1] * s[1] + w[2] * s[2] + w[3] * s[3]);
    double C = c2 * w[0] * w[0] - (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
    if (C < 0.0) C = 0.0;
    double r = INFINITY;
    if (A == 0.0) {
        if (B < 0.0) r = C / (-2.0 * B);
    } else {
        const double disc = B * B - A * C;
        if (disc >= 0.0) {
            const double sq = sqrt(disc);
            if (B < 0.0) r = C / (-B + sq);
            else if (A < 0.0) r = (B + sq) / (-A);
        }
    }
    return fmin(tau, r);
}

/* (E, Fx, Fy, Fz) of the neighbour of (i,j,k) in direction `dir` (0..5 = x-, x+, y-, y+, z-, z+):
 * periodic wrap; reflective: the cell with its normal flux negated; Neumann: the cell; Dirichlet: the wall state. */
static void neighbour3(const or3_grid* g, const double* v, int i, int j, int k, int dir, double U[4])
{
    const size_t n = ncell3(g);
    int ni = i, nj = j, nk = k;
    const int axis = dir / 2, step = (dir % 2) ? 1 : -1;
    if (axis == 0) ni += step;
    else if (axis == 1) nj += step;
    else nk += step;
    const int len = axis == 0 ? g->nx : axis == 1 ? g->ny : g->nz;
    const int pos = axis == 0 ? ni : axis == 1 ? nj : nk;
    if (pos < 0 || pos >= len) {
        switch (g->bc_kind[dir]) {
        case OR_BC_PERIODIC: {
            const int w = (pos + len) % len;
            if (axis == 0) ni = w;
            else if (axis == 1) nj = w;
            else nk = w;
            break;
        }
        case OR_BC_REFLECTIVE:
        case OR_BC_NEUMANN: {
            const size_t c = at(g, i, j, k);
            for (int q = 0; q < 4; ++q) U[q] = v[q * n + c];
            if (g->bc_kind[dir] == OR_BC_REFLECTIVE) U[1 + axis] = -U[1 + axis];
            return;
        }
        default:
            U[0] = g->bc_E[dir];
            U[1] = g->bc_Fx[dir];
            U[2] = g->bc_Fy[dir];
            U[3] = g->bc_Fz[dir];
            return;
        }
    }
    const size_t c = at(g, ni, nj, nk);
    for (int q = 0; q < 4; ++q) U[q] = v[q * n + c];
}

/* L (sign +1) / R (sign -1) operator of Sect. 3.1 along `axis`: dt/(2h) (c U + sign G_axis(U)),
 * G_axis = (F_axis, c^2 P[x][axis], c^2 P[y][axis], c^2 P[z][axis]).                            */
static void op_LR3(const or3_grid* g, int axis, double sign, const double U[4], double out[4])
{
    static const int col[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}}; /* P[row][axis] in the packed storage */
    const double c = g->c;
    double P[6], G[4];
    or3_closure(U[0], U[1], U[2], U[3], c, P);
    G[0] = U[1 + axis];
    for (int m = 0; m < 3; ++m) G[1 + m] = c * c * P[col[m][axis]];
    const double h = axis == 0 ? g->hx : axis == 1 ? g->hy : g->hz;
    const double kk = g->dt / (2.0 * h);
    for (int m = 0; m < 4; ++m) out[m] = kk * (c * U[m] + sign * G[m]);
}

/* Sum of the six off-diagonal operators of row (i,j,k), x then y then z, lower neighbour first. */
static void offdiag3(const or3_grid* g, const double* v, int i, int j, int k, double S[4])
{
    double U[4], t[4];
    S[0] = S[1] = S[2] = S[3] = 0.0;
    for (int dir = 0; dir < 6; ++dir) {
        neighbour3(g, v, i, j, k, dir, U);
        op_LR3(g, dir / 2, (dir % 2) ? -1.0 : 1.0, U, t);
        for (int m = 0; m < 4; ++m) S[m] += t[m];
    }
}

static double diag_a3(const or3_grid* g) { return 1.0 + g->c * g->dt / g->hx + g->c * g->dt / g->hy + g->c * g->dt / g->hz; }

/* A of Sect. 3.1 with the implicit sources (the 2-D oracle's rows with a third flux component):
 *   A_E = a E - S_E + ka (E - a_r T^4),  A_F = a F - S_F + (ka + ks) F,  A_T = C_v T + ka (a_r T^4 - E). */
void or3_apply_A(const or3_grid* g, const double* sigma, const double* v, double* out)
{
    const size_t n = ncell3(g);
    const double a = diag_a3(g);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                const size_t c = at(g, i, j, k);
                double S[4];
                offdiag3(g, v, i, j, k, S);
                const double ka = g->c * g->dt * sigma[c], ks = g->c * g->dt * sigma[n + c];
                const double E = v[c], T = v[4 * n + c], T4 = T * T * T * T;
                out[c] = a * E - S[0] + ka * (E - g->a_r * T4);
                for (int m = 1; m <= 3; ++m) out[m * n + c] = a * v[m * n + c] - S[m] + (ka + ks) * v[m * n + c];
                out[4 * n + c] = g->c_v * T + ka * (g->a_r * T4 - E);
            }
}

void or3_residual(const or3_grid* g, const double* sigma, const double* b, const double* v, double* r)
{
    const size_t n = ncell3(g);
    or3_apply_A(g, sigma, v, r);
    for (size_t c = 0; c < NF3 * n; ++c) r[c] = b[c] - r[c];
}

/* L2 norm of (r_E, r_F/c, r_T), summed plane by plane, row by row, in a fixed order. */
double or3_norm(const or3_grid* g, const double* r)
{
    const size_t n = ncell3(g);
    const double ic = 1.0 / g->c;
    double s = 0.0;
    for (size_t c = 0; c < n; ++c) {
        const double e = r[c], fx = r[n + c] * ic, fy = r[2 * n + c] * ic, fz = r[3 * n + c] * ic, t = r[4 * n + c];
        s += e * e + fx * fx + fy * fy + fz * fz + t * t;
    }
    return sqrt(s);
}

/* One Jacobi sweep of (beta M + gamma A)(u) = rhs (Algorithm 1; the implicit pseudo-time step with
 * (beta, gamma) = (1, tau)): the cell's (E, Fx, Fy, T) by the 2-D oracle's local solve, Fz with the
 * same divisor as the other flux components.                                                        */
static void jacobi3(const or3_grid* g, const double* sigma, double beta, double gamma0, const double* gamma_cell,
                    const double* rhs, const double* v_in, double* v_out)
{
    const size_t n = ncell3(g);
    const double a = diag_a3(g);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                const size_t c = at(g, i, j, k);
                const double gamma = gamma_cell ? gamma_cell[c] : gamma0;
                double S[4], B[4], o[4];
                offdiag3(g, v_in, i, j, k, S);
                const double ka = g->c * g->dt * sigma[c], ks = g->c * g->dt * sigma[n + c];
                B[0] = rhs[c] + gamma * S[0];
                B[1] = rhs[n + c] + gamma * S[1];
                B[2] = rhs[2 * n + c] + gamma * S[2];
                B[3] = rhs[4 * n + c];
                or_local_solve(beta, gamma, a, ka, ks, g->c_v, g->a_r, B, o);
                const double BFz = rhs[3 * n + c] + gamma * S[3];
                v_out[c] = o[0];
                v_out[n + c] = o[1];
                v_out[2 * n + c] = o[2];
                v_out[3 * n + c] = BFz / (beta + gamma * (a + ka + ks));
                v_out[4 * n + c] = o[3];
            }
}

/* Finest-level sweep: u_new = (1 - omega) u + omega J(u). */
void or3_sweep(const or3_grid* g, const double* sigma, double omega, const double* b, const double* v_in,
               double* v_out)
{
    const size_t n = ncell3(g);
    jacobi3(g, sigma, 0.0, 1.0, NULL, b, v_in, v_out);
    if (omega != 1.0)
        for (size_t c = 0; c < NF3 * n; ++c) v_out[c] = (1.0 - omega) * v_in[c] + omega * v_out[c];
}

/* One pseudo-time step of Algorithm 3 (as or_pseudo_step): per cell explicit sub-steps along
 * M^{-1} f, each eta times the admissible length left, at most sub_steps of them and never past dtau,
 * reaching tau_i; then nu_l Jacobi sweeps of (M + tau A)(u) = M u~ from u (tau = tau_i when
 * pseudo_local, else dtau).                                                                          */
void or3_pseudo_step(const or3_grid* g, const double* sigma, const or_params* p, double dtau, const double* f,
                     const double* u_in, double* u_out)
{
    const size_t n = ncell3(g);
    double* rhs = dalloc3(NF3 * n);
    double* taus = dalloc3(n);
    for (size_t c = 0; c < n; ++c) {
        double s[5] = {f[c], f[n + c], f[2 * n + c], f[3 * n + c], f[4 * n + c] / g->c_v};
        double w[5] = {u_in[c], u_in[n + c], u_in[2 * n + c], u_in[3 * n + c], u_in[4 * n + c]};
        double tau_ex = 0.0;
        for (int it = 0; it < p->sub_steps && tau_ex < dtau; ++it) {
            const double d = fmin(dtau - tau_ex, p->eta * or3_ray(g->c, w, s));
            for (int m = 0; m < 5; ++m) w[m] += d * s[m];
            tau_ex += d;
        }
        taus[c] = tau_ex;
        for (int m = 0; m < 4; ++m) rhs[m * n + c] = w[m];
        rhs[4 * n + c] = g->c_v * w[4]; /* M u~ */
    }
    double* cur = dalloc3(NF3 * n);
    double* nxt = dalloc3(NF3 * n);
    memcpy(cur, u_in, NF3 * n * sizeof(double));
    for (int s = 0; s < p->nu_l; ++s) {
        jacobi3(g, sigma, 1.0, dtau, p->pseudo_local ? taus : NULL, rhs, cur, nxt);
        double* t = cur;
        cur = nxt;
        nxt = t;
    }
    memcpy(u_out, cur, NF3 * n * sizeof(double));
    free(cur);
    free(nxt);
    free(rhs);
    free(taus);
}

/* eq. (prolongatedSol): w where admissible, else (u + dtb w)/(1 + dtb) with dtb/(1+dtb) = eta min(tau*, 1). */
void or3_project(const or3_grid* g, const or_params* p, const double* u, const double* w, double* out)
{
    const size_t n = ncell3(g);
    for (size_t c = 0; c < n; ++c) {
        double uu[5], ww[5], s[5];
        for (int m = 0; m < 5; ++m) {
            uu[m] = u[m * n + c];
            ww[m] = w[m * n + c];
            s[m] = ww[m] - uu[m];
        }
        if (or3_admissible(g->c, ww)) {
            for (int m = 0; m < 5; ++m) out[m * n + c] = ww[m];
            continue;
        }
        double ts = or3_ray(g->c, uu, s);
        if (ts > 1.0) ts = 1.0;
        const double theta = p->eta * ts, dtb = theta / (1.0 - theta);
        for (int m = 0; m < 5; ++m) out[m * n + c] = (uu[m] + dtb * ww[m]) / (1.0 + dtb);
    }
}

/* ------------------------------------------------------------------------- */
/* Transfer (Sect. 4.2, d = 3): fine cell 2I coincides with coarse cell I, odd fine cells interpolate
 * linearly along each axis (trilinear as the tensor product); R = 2^-3 P^T, i.e. the tensor product of
 * 1/4, 1/2, 1/4.  Periodic axes wrap; on other axes a point outside is dropped and the remaining
 * weights renormalised, as in the 2-D oracle.                                                         */
static int pw1(int i, int nc, int periodic, int idx[2], double w[2])
{
    if (i % 2 == 0) {
        idx[0] = i / 2;
        w[0] = 1.0;
        return 1;
    }
    int I1 = i / 2 + 1;
    if (I1 >= nc) {
        if (!periodic) {
            idx[0] = i / 2;
            w[0] = 1.0;
            return 1;
        }
        I1 -= nc;
    }
    idx[0] = i / 2;
    idx[1] = I1;
    w[0] = w[1] = 0.5;
    return 2;
}

static int rw1(int I, int nf, int periodic, int idx[3], double w[3])
{
    static const double base[3] = {0.25, 0.5, 0.25};
    int cnt = 0;
    double sum = 0.0;
    for (int m = 0; m < 3; ++m) {
        int f = 2 * I - 1 + m;
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

or3_grid or3_coarse_grid(const or3_grid* g)
{
    or3_grid c = *g;
    c.nx = g->nx / 2;
    c.ny = g->ny / 2;
    c.nz = g->nz / 2;
    c.hx = 2.0 * g->hx;
    c.hy = 2.0 * g->hy;
    c.hz = 2.0 * g->hz;
    return c;
}

void or3_restrict(const or3_grid* fine, const double* x, int32_t nfields, double* xc)
{
    const or3_grid cg = or3_coarse_grid(fine);
    const size_t nf = ncell3(fine), nc = ncell3(&cg);
    const int px = fine->bc_kind[0] == OR_BC_PERIODIC, py = fine->bc_kind[2] == OR_BC_PERIODIC,
              pz = fine->bc_kind[4] == OR_BC_PERIODIC;
#pragma omp parallel for schedule(static)
    for (int K = 0; K < cg.nz; ++K)
        for (int J = 0; J < cg.ny; ++J)
            for (int I = 0; I < cg.nx; ++I) {
                int ix[3], iy[3], iz[3];
                double wx[3], wy[3], wz[3];
                const int cx = rw1(I, fine->nx, px, ix, wx), cy = rw1(J, fine->ny, py, iy, wy),
                          cz = rw1(K, fine->nz, pz, iz, wz);
                for (int q = 0; q < nfields; ++q) {
                    double s = 0.0;
                    for (int c3 = 0; c3 < cz; ++c3)
                        for (int b = 0; b < cy; ++b)
                            for (int a = 0; a < cx; ++a)
                                s += wx[a] * wy[b] * wz[c3] * x[q * nf + at(fine, ix[a], iy[b], iz[c3])];
                    xc[q * nc + at(&cg, I, J, K)] = s;
                }
            }
}

void or3_prolong(const or3_grid* fine, const double* xc, int32_t nfields, double* x)
{
    const or3_grid cg = or3_coarse_grid(fine);
    const size_t nf = ncell3(fine), nc = ncell3(&cg);
    const int px = fine->bc_kind[0] == OR_BC_PERIODIC, py = fine->bc_kind[2] == OR_BC_PERIODIC,
              pz = fine->bc_kind[4] == OR_BC_PERIODIC;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < fine->nz; ++k)
        for (int j = 0; j < fine->ny; ++j)
            for (int i = 0; i < fine->nx; ++i) {
                int ix[2], iy[2], iz[2];
                double wx[2], wy[2], wz[2];
                const int cx = pw1(i, cg.nx, px, ix, wx), cy = pw1(j, cg.ny, py, iy, wy),
                          cz = pw1(k, cg.nz, pz, iz, wz);
                for (int q = 0; q < nfields; ++q) {
                    double s = 0.0;
                    for (int c3 = 0; c3 < cz; ++c3)
                        for (int b = 0; b < cy; ++b)
                            for (int a = 0; a < cx; ++a)
                                s += wx[a] * wy[b] * wz[c3] * xc[q * nc + at(&cg, ix[a], iy[b], iz[c3])];
                    x[q * nf + at(fine, i, j, k)] = s;
                }
            }
}

int32_t or3_num_levels(const or3_grid* g, const or_params* p)
{
    int L = 1, nx = g->nx, ny = g->ny, nz = g->nz;
    for (;;) {
        if (p->levels > 0 && L >= p->levels) break;
        if (nx % 2 || ny % 2 || nz % 2 || nx / 2 < 4 || ny / 2 < 4 || nz / 2 < 4) break;
        nx /= 2;
        ny /= 2;
        nz /= 2;
        ++L;
    }
    return L;
}

static void sweeps3(const or3_grid* g, const double* sigma, double omega, const double* b, const double* v0, int nu,
                    double* out)
{
    const size_t n = ncell3(g);
    double* cur = dalloc3(NF3 * n);
    double* nxt = dalloc3(NF3 * n);
    memcpy(cur, v0, NF3 * n * sizeof(double));
    for (int s = 0; s < nu; ++s) {
        or3_sweep(g, sigma, omega, b, cur, nxt);
        double* t = cur;
        cur = nxt;
        nxt = t;
    }
    memcpy(out, cur, NF3 * n * sizeof(double));
    free(cur);
    free(nxt);
}

static void smooth3(const or3_grid* g, const double* sigma, const or_params* p, double dtau, const double* f,
                    const double* u0, double* out)
{
    const size_t n = ncell3(g);
    double* cur = dalloc3(NF3 * n);
    double* nxt = dalloc3(NF3 * n);
    memcpy(cur, u0, NF3 * n * sizeof(double));
    for (int m = 0; m < p->pseudo_steps; ++m) {
        or3_pseudo_step(g, sigma, p, dtau, f, cur, nxt);
        double* t = cur;
        cur = nxt;
        nxt = t;
    }
    memcpy(out, cur, NF3 * n * sizeof(double));
    free(cur);
    free(nxt);
}

/* W- and F-cycles (Sect. 6.3; the shapes of or_cycle): the recursion over the
 * coarse problems.  A visit of level l smooths its FAS problem (Algorithm 3),
 * restricts the iterate and its residual to level l+1, visits that level once
 * (V), twice (W) or by an F-visit then a V-visit (F), corrects with the
 * projection of eq. (prolongatedSol) and smooths again; the coarsest level is
 * smoothed once per visit.  Same steps as or3_vcycle below for kind V. */
typedef struct {
    int L;
    or3_grid* G;
    double **S, **U, **V, **F;
} cyc3;

static void visit3(const cyc3* c, const or_params* p, double dtau, int l, int kind);

static void descend3(const cyc3* c, int l, const double* rhs)
{
    const size_t nc = ncell3(&c->G[l + 1]);
    double* rb = dalloc3(NF3 * ncell3(&c->G[l]));
    double* rr = dalloc3(NF3 * nc);
    or3_residual(&c->G[l], c->S[l], rhs, c->U[l], rb);
    or3_restrict(&c->G[l], c->U[l], NF3, c->V[l + 1]);
    or3_restrict(&c->G[l], rb, NF3, rr);
    or3_apply_A(&c->G[l + 1], c->S[l + 1], c->V[l + 1], c->F[l + 1]);
    for (size_t k = 0; k < NF3 * nc; ++k) c->F[l + 1][k] += rr[k];
    memcpy(c->U[l + 1], c->V[l + 1], NF3 * nc * sizeof(double));
    free(rb);
    free(rr);
}

static void below_and_correct3(const cyc3* c, const or_params* p, double dtau, int l, int kind)
{
    if (kind == OR_CYCLE_F) {
        visit3(c, p, dtau, l + 1, OR_CYCLE_F);
        visit3(c, p, dtau, l + 1, OR_CYCLE_V);
    } else {
        for (int t = 0; t < ((kind == OR_CYCLE_W) ? 2 : 1); ++t) visit3(c, p, dtau, l + 1, kind);
    }
    const size_t n = ncell3(&c->G[l]), nc = ncell3(&c->G[l + 1]);
    double* e = dalloc3(NF3 * nc);
    double* w = dalloc3(NF3 * n);
    for (size_t k = 0; k < NF3 * nc; ++k) e[k] = c->U[l + 1][k] - c->V[l + 1][k];
    or3_prolong(&c->G[l], e, NF3, w);
    for (size_t k = 0; k < NF3 * n; ++k) w[k] += c->U[l][k];
    or3_project(&c->G[l], p, c->U[l], w, c->U[l]);
    free(e);
    free(w);
}

static void visit3(const cyc3* c, const or_params* p, double dtau, int l, int kind)
{
    const size_t n = ncell3(&c->G[l]);
    double* t = dalloc3(NF3 * n);
    smooth3(&c->G[l], c->S[l], p, dtau, c->F[l], c->U[l], t);
    memcpy(c->U[l], t, NF3 * n * sizeof(double));
    if (l < c->L - 1) {
        descend3(c, l, c->F[l]);
        below_and_correct3(c, p, dtau, l, kind);
        smooth3(&c->G[l], c->S[l], p, dtau, c->F[l], c->U[l], t);
        memcpy(c->U[l], t, NF3 * n * sizeof(double));
    }
    free(t);
}

void or3_cycle(const or3_grid* g, const double* sigma, const or_params* p, int32_t kind, double dtau, const double* b,
               const double* v, double* out)
{
    cyc3 c;
    c.L = or3_num_levels(g, p);
    c.G = (or3_grid*)malloc(sizeof(or3_grid) * c.L);
    c.S = (double**)calloc(c.L, sizeof(double*));
    c.U = (double**)calloc(c.L, sizeof(double*));
    c.V = (double**)calloc(c.L, sizeof(double*));
    c.F = (double**)calloc(c.L, sizeof(double*));
    c.G[0] = *g;
    c.S[0] = (double*)sigma;
    for (int l = 1; l < c.L; ++l) {
        c.G[l] = or3_coarse_grid(&c.G[l - 1]);
        c.S[l] = dalloc3(2 * ncell3(&c.G[l]));
        or3_restrict(&c.G[l - 1], c.S[l - 1], 2, c.S[l]);
    }
    for (int l = 0; l < c.L; ++l) {
        c.U[l] = dalloc3(NF3 * ncell3(&c.G[l]));
        c.V[l] = dalloc3(NF3 * ncell3(&c.G[l]));
        c.F[l] = dalloc3(NF3 * ncell3(&c.G[l]));
    }
    sweeps3(&c.G[0], c.S[0], p->omega, b, v, p->nu0, c.U[0]);
    if (c.L > 1) {
        double* t = dalloc3(NF3 * ncell3(g));
        descend3(&c, 0, b);
        below_and_correct3(&c, p, dtau, 0, kind);
        sweeps3(&c.G[0], c.S[0], p->omega, b, c.U[0], p->nu0, t);
        memcpy(c.U[0], t, NF3 * ncell3(g) * sizeof(double));
        free(t);
    }
    memcpy(out, c.U[0], NF3 * ncell3(g) * sizeof(double));
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

/* One cycle of the parameters' shape: the V-cycle's loop form below, W and F by or3_cycle. */
static void vcycle3_loop(const or3_grid* g, const double* sigma, const or_params* p, double dtau, const double* b,
                         const double* v, double* out);

void or3_vcycle(const or3_grid* g, const double* sigma, const or_params* p, double dtau, const double* b,
                const double* v, double* out)
{
    if (p->cycle == OR_CYCLE_V) vcycle3_loop(g, sigma, p, dtau, b, v, out);
    else or3_cycle(g, sigma, p, p->cycle, dtau, b, v, out);
}

/* One V-cycle (Appendix A) with the FAS coarse problems of Sect. 4.2, as the 2-D oracle's loop form. */
static void vcycle3_loop(const or3_grid* g, const double* sigma, const or_params* p, double dtau, const double* b,
                const double* v, double* out)
{
    const int L = or3_num_levels(g, p);
    or3_grid* G = (or3_grid*)malloc(sizeof(or3_grid) * L);
    double **U = (double**)calloc(L, sizeof(double*)), **V = (double**)calloc(L, sizeof(double*));
    double **Fr = (double**)calloc(L, sizeof(double*)), **S = (double**)calloc(L, sizeof(double*));
    G[0] = *g;
    S[0] = (double*)sigma;
    for (int l = 1; l < L; ++l) {
        G[l] = or3_coarse_grid(&G[l - 1]);
        S[l] = dalloc3(2 * ncell3(&G[l]));
        or3_restrict(&G[l - 1], S[l - 1], 2, S[l]);
    }
    for (int l = 0; l < L; ++l) {
        U[l] = dalloc3(NF3 * ncell3(&G[l]));
        V[l] = dalloc3(NF3 * ncell3(&G[l]));
        Fr[l] = dalloc3(NF3 * ncell3(&G[l]));
    }
    sweeps3(&G[0], S[0], p->omega, b, v, p->nu0, U[0]);
    if (L > 1) {
        double* rbar = dalloc3(NF3 * ncell3(&G[0]));
        or3_residual(&G[0], S[0], b, U[0], rbar);
        for (int l = 1; l < L; ++l) {
            const size_t n = ncell3(&G[l]);
            double* rr = dalloc3(NF3 * n);
            or3_restrict(&G[l - 1], U[l - 1], NF3, V[l]);
            or3_restrict(&G[l - 1], rbar, NF3, rr);
            or3_apply_A(&G[l], S[l], V[l], Fr[l]);
            for (size_t c = 0; c < NF3 * n; ++c) Fr[l][c] += rr[c];
            free(rr);
            smooth3(&G[l], S[l], p, dtau, Fr[l], V[l], U[l]);
            free(rbar);
            rbar = NULL;
            if (l < L - 1) {
                rbar = dalloc3(NF3 * n);
                or3_residual(&G[l], S[l], Fr[l], U[l], rbar);
            }
        }
        free(rbar);
        for (int l = L - 2; l >= 0; --l) {
            const size_t n = ncell3(&G[l]), nc = ncell3(&G[l + 1]);
            double* e = dalloc3(NF3 * nc);
            double* w = dalloc3(NF3 * n);
            double* t = dalloc3(NF3 * n);
            for (size_t c = 0; c < NF3 * nc; ++c) e[c] = U[l + 1][c] - V[l + 1][c];
            or3_prolong(&G[l], e, NF3, w);
            for (size_t c = 0; c < NF3 * n; ++c) w[c] += U[l][c];
            or3_project(&G[l], p, U[l], w, U[l]);
            if (l == 0) sweeps3(&G[0], S[0], p->omega, b, U[0], p->nu0, t);
            else smooth3(&G[l], S[l], p, dtau, Fr[l], U[l], t);
            memcpy(U[l], t, NF3 * n * sizeof(double));
            free(e);
            free(w);
            free(t);
        }
    }
    memcpy(out, U[0], NF3 * ncell3(g) * sizeof(double));
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

/* Time steps as or_step: b = (E^n, F^n, C_v T^n), cycles until rtol or the rounding floor
 * 16 eps a |b|, dtau starting from dtau_im0 (on every step when dtau_carry is 0) and adapted after each
 * cycle (Appendix A). */
int32_t or3_step(const or3_grid* g, const double* sigma, const or_params* p, double* v, int32_t nsteps, or_info* info)
{
    const size_t n = ncell3(g);
    double* b = dalloc3(NF3 * n);
    double* r = dalloc3(NF3 * n);
    double* nv = dalloc3(NF3 * n);
    int32_t status = 0, total = 0;
    double r0 = 0.0, rel = 0.0, dtau = p->dtau_im0;
    for (int step = 0; step < nsteps; ++step) {
        memcpy(b, v, NF3 * n * sizeof(double));
        for (size_t c = 0; c < n; ++c) b[4 * n + c] = g->c_v * v[4 * n + c];
        if (!p->dtau_carry) dtau = p->dtau_im0;
        or3_residual(g, sigma, b, v, r);
        r0 = or3_norm(g, r);
        const double floor_r = 16.0 * DBL_EPSILON * diag_a3(g) * or3_norm(g, b);
        rel = 0.0;
        if (r0 <= floor_r) continue;
        double rprev = r0;
        int conv = 0;
        for (int kc = 1; kc <= p->max_cycles; ++kc) {
            or3_vcycle(g, sigma, p, dtau, b, v, nv);
            memcpy(v, nv, NF3 * n * sizeof(double));
            or3_residual(g, sigma, b, v, r);
            const double rk = or3_norm(g, r);
            ++total;
            rel = rk / r0;
            double d = (p->dtau_rule == OR_DTAU_LITERAL) ? fabs(rk - rprev) / r0 : (rprev - rk) / rprev;
            if (d > p->eps_inc) dtau *= 1.1;
            if (d < p->eps_dec) dtau *= 0.5;
            dtau = fmin(fmax(dtau, p->dtau_min), p->dtau_max);
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
        info->levels = or3_num_levels(g, p);
        info->r0 = r0;
        info->rel_residual = rel;
        info->dtau = dtau;
    }
    free(b);
    free(r);
    free(nv);
    return status;
}
