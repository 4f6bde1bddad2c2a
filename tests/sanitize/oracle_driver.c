/* A host program that runs the oracle's code paths on small problems, built by
 * tests/test_oracle_sanitized.py with AddressSanitizer and UndefinedBehavior-
 * Sanitizer: every out-of-bounds access, use after free, leak or undefined
 * operation in the oracle ends the run with an error.  Exit status 0 when all
 * solves converged. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/m1_oracle.h"
#include "../../oracle/m1_oracle3.h"

static unsigned long long rng_state = 88172645463325252ull;
static double uniform(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static or_params params(int cycle, int transfer, int smoother)
{
    or_params p;
    memset(&p, 0, sizeof p);
    p.nu0 = 3;
    p.nu_l = 1;
    p.pseudo_steps = 3;
    p.sub_steps = 4;
    p.max_cycles = 5000;
    p.pseudo_local = 1;
    p.smoother = smoother;
    p.cycle = cycle;
    p.transfer = transfer;
    p.dtau_im0 = 1e-3;
    p.eps_inc = 0.05;
    p.eta = 0.9;
    p.rtol = 1e-10;
    p.dtau_min = 1e-6;
    p.dtau_max = 1e6;
    p.omega = 0.8;
    return p;
}

/* random admissible state and opacities on an nx x ny grid (4 fields) */
static void fill2(int n, double* v, double* sig, double c)
{
    for (int k = 0; k < n; ++k) {
        const double E = 0.5 + uniform(), f = 0.9 * uniform(), th = 6.283185307179586 * uniform();
        v[k] = E;
        v[n + k] = f * c * E * cos(th);
        v[2 * n + k] = f * c * E * sin(th);
        v[3 * n + k] = 0.5 + uniform();
        sig[k] = pow(10.0, -2.0 + 3.0 * uniform());
        sig[n + k] = uniform();
    }
}

static int run2d(int nx, int ny, const int kinds[4], int cycle, int transfer, int smoother)
{
    or_grid g;
    memset(&g, 0, sizeof g);
    g.dim = 2;
    g.nx = nx;
    g.ny = ny;
    g.hx = 1.0 / nx;
    g.hy = 1.0 / ny;
    g.c = 1.0;
    g.dt = 20.0 * g.hx;
    g.a_r = 1.0;
    g.c_v = 1.0;
    for (int s = 0; s < 4; ++s) {
        g.bc_kind[s] = kinds[s];
        g.bc_E[s] = 3.0;
        g.bc_Fx[s] = 1.0;
        g.bc_lo[s] = 0.25;
        g.bc_hi[s] = 0.6;
        g.bc_Eo[s] = 0.5;
    }
    const int n = nx * ny;
    double* v = calloc(4 * (size_t)n, sizeof(double));
    double* sig = calloc(2 * (size_t)n, sizeof(double));
    fill2(n, v, sig, g.c);
    or_params p = params(cycle, transfer, smoother);
    or_info info;
    double hist[64];
    const int st = or_step(&g, sig, &p, v, 2, &info, hist, 64);
    double* w = calloc(4 * (size_t)n, sizeof(double));
    memcpy(w, v, 4 * (size_t)n * sizeof(double));
    const int ex = or_explicit_run(&g, 1, w, 20, 1e-30);
    printf("2-D %dx%d cycle %d transfer %d smoother %d: status %d, %d cycles, explicit %d steps\n", nx, ny, cycle,
           transfer, smoother, st, info.cycles, ex);
    free(v);
    free(sig);
    free(w);
    return st;
}

static int run3d(int nx, int ny, int nz, const int kinds[6])
{
    or3_grid g;
    memset(&g, 0, sizeof g);
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.hx = 1.0 / nx;
    g.hy = 1.0 / ny;
    g.hz = 1.0 / nz;
    g.c = 1.0;
    g.dt = 10.0 * g.hx;
    g.a_r = 1.0;
    g.c_v = 1.0;
    for (int s = 0; s < 6; ++s) {
        g.bc_kind[s] = kinds[s];
        g.bc_E[s] = 3.0;
        g.bc_Fx[s] = 1.0;
    }
    const int n = nx * ny * nz;
    double* v = calloc(5 * (size_t)n, sizeof(double));
    double* sig = calloc(2 * (size_t)n, sizeof(double));
    for (int k = 0; k < n; ++k) {
        const double E = 0.5 + uniform(), f = 0.9 * uniform();
        v[k] = E;
        v[n + k] = f * E * 0.6;
        v[2 * n + k] = -f * E * 0.48;
        v[3 * n + k] = f * E * 0.64;
        v[4 * n + k] = 0.5 + uniform();
        sig[k] = pow(10.0, -2.0 + 3.0 * uniform());
        sig[n + k] = uniform();
    }
    or_params p = params(0, 0, 0);
    or_info info;
    const int st = or3_step(&g, sig, &p, v, 1, &info);
    printf("3-D %dx%dx%d: status %d, %d cycles\n", nx, ny, nz, st, info.cycles);
    free(v);
    free(sig);
    return st;
}

int main(void)
{
    or_set_threads(1);
    const int mixed[4] = {OR_BC_INFLOW, OR_BC_NEUMANN, OR_BC_REFLECTIVE, OR_BC_DIRICHLET};
    const int periodic[4] = {OR_BC_PERIODIC, OR_BC_PERIODIC, OR_BC_PERIODIC, OR_BC_PERIODIC};
    int bad = 0;
    bad |= run2d(16, 12, mixed, OR_CYCLE_V, OR_TRANSFER_FULL, OR_SMOOTH_JACOBI);
    bad |= run2d(16, 16, periodic, OR_CYCLE_W, OR_TRANSFER_MEAN, OR_SMOOTH_JACOBI);
    bad |= run2d(24, 8, mixed, OR_CYCLE_F, OR_TRANSFER_FULL, OR_SMOOTH_RBGS);
    bad |= run2d(13, 7, mixed, OR_CYCLE_V, OR_TRANSFER_FULL, OR_SMOOTH_JACOBI);
    const int k3[6] = {OR_BC_DIRICHLET, OR_BC_NEUMANN, OR_BC_REFLECTIVE, OR_BC_REFLECTIVE, OR_BC_PERIODIC,
                       OR_BC_PERIODIC};
    bad |= run3d(8, 8, 8, k3);
    bad |= run3d(10, 6, 4, k3);
    return bad ? 1 : 0;
}
