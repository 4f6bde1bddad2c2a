// m1_kernels3.hip -- grid kernels of the three-dimensional cycle.
//
// One thread per cell over a 1-D launch in the XCD-aware block order of
// m1::xcd_block() (each XCD walks a contiguous band of z-planes, so the
// neighbouring planes a stencil reads stay in its own L2).  Per cell the 7-point
// form of the implicit Rusanov system (Sect. 3.1 along each of the three axes:
// L/R = dt/(2h) (c U +- G_axis(U)), G_axis = (F_axis, c^2 P[., axis])), the
// sources of eq. (m1) taken implicitly, and the single-cell gas-radiation
// solve of the 2-D kernels (the three flux components share one divisor).
// The stop flag `active` is read with the data and gates the stores, as in
// the 2-D grid kernels.
#include "m1_3d.hpp"
#include "m1_cells.hpp"

namespace m1 {

namespace {

constexpr int kB3 = 256;

unsigned blocks3(int64_t n) { return (unsigned)((n + kB3 - 1) / kB3); }

// 0 in a vector register: keeps the flag read an ordinary vector load (see the 2-D kernels).
__device__ __forceinline__ uint32_t vzero3()
{
    uint32_t z = 0;
    asm("" : "+v"(z));
    return z;
}

__device__ __forceinline__ bool cell3(const Lvl3& L, uint32_t& k, int& i, int& j, int& l)
{
    k = (uint32_t)xcd_block() * kB3 + threadIdx.x;
    const uint32_t nxy = (uint32_t)L.nx * (uint32_t)L.ny;
    if (k >= nxy * (uint32_t)L.nz) return false;
    l = (int)(k / nxy);
    const uint32_t r = k - (uint32_t)l * nxy;
    j = (int)(r / (uint32_t)L.nx);
    i = (int)(r - (uint32_t)j * (uint32_t)L.nx);
    return true;
}

// Admissible length of the ray w + tau s with three flux components (as ray_len).
__device__ __forceinline__ double ray3(double c2, double E, double Fx, double Fy, double Fz, double T, double sE,
                                       double sFx, double sFy, double sFz, double sT)
{
    double tau = INFINITY;
    if (sE < 0.0) tau = -E * rcp_nr(sE);
    if (sT < 0.0) tau = fmin(tau, -T * rcp_nr(sT));
    const double A = c2 * sE * sE - fma(sFx, sFx, fma(sFy, sFy, sFz * sFz));
    const double B = c2 * E * sE - fma(Fx, sFx, fma(Fy, sFy, Fz * sFz));
    const double C = fmax(c2 * E * E - fma(Fx, Fx, fma(Fy, Fy, Fz * Fz)), 0.0);
    double r = INFINITY;
    if (A == 0.0) {
        if (B < 0.0) r = C * rcp_nr(-2.0 * B);
    } else {
        const double disc = B * B - A * C;
        if (disc >= 0.0) {
            const double sq = disc > 0.0 ? sqrt_nr(disc) : 0.0;
            if (B < 0.0) r = C * rcp_nr(sq - B);
            else if (A < 0.0) r = (B + sq) * rcp_nr(-A);
        }
    }
    return fmin(tau, r);
}

__device__ __forceinline__ bool admissible3(double c2, double E, double Fx, double Fy, double Fz, double T)
{
    return E > 0.0 && T > 0.0 && fma(Fx, Fx, fma(Fy, Fy, Fz * Fz)) <= c2 * E * E;
}

// (E, Fx, Fy, Fz) of the neighbour of cell k = (i, j, l) in direction dir (0..5: x-, x+, y-, y+, z-, z+):
// a cell of the grid, the wrapped cell (periodic), the cell itself with the normal flux negated
// (reflective) or not (Neumann), or the side's wall state (Dirichlet).
__device__ __forceinline__ void nb3(const Phys3& ph, const Lvl3& L, const CSoa3& v, int i, int j, int l, uint32_t k,
                                    int dir, double& E, double& Fx, double& Fy, double& Fz)
{
    const int axis = dir >> 1;
    const bool up = dir & 1;
    const int pos = axis == 0 ? i : (axis == 1 ? j : l);
    const int len = axis == 0 ? L.nx : (axis == 1 ? L.ny : L.nz);
    const uint32_t stride = axis == 0 ? 1u : (axis == 1 ? (uint32_t)L.nx : (uint32_t)L.nx * (uint32_t)L.ny);
    const bool inside = up ? pos + 1 < len : pos > 0;
    uint32_t kn = up ? k + stride : k - stride;
    const int kind = ph.bc[dir];
    if (!inside) {
        if (kind == BC_DIRICHLET) {
            E = ph.bcE[dir];
            Fx = ph.bcFx[dir];
            Fy = ph.bcFy[dir];
            Fz = ph.bcFz[dir];
            return;
        }
        kn = kind == BC_PERIODIC ? (up ? k - (uint32_t)(len - 1) * stride : k + (uint32_t)(len - 1) * stride) : k;
    }
    E = ld(v.E, kn);
    Fx = ld(v.Fx, kn);
    Fy = ld(v.Fy, kn);
    Fz = ld(v.Fz, kn);
    if (!inside && kind == BC_REFLECTIVE) {
        if (axis == 0) Fx = -Fx;
        else if (axis == 1) Fy = -Fy;
        else Fz = -Fz;
    }
}

// Sum of the six off-diagonal operators of row k: x-, x+, y-, y+, z-, z+ (lower neighbour: L = k (cU + G),
// upper: R = k (cU - G)), with c^2 P_ab = iso delta_ab + 3 r F_a F_b from the closure of the 2-D kernels.
__device__ __forceinline__ void offdiag3(const Phys3& ph, const Lvl3& L, const CSoa3& v, int i, int j, int l,
                                         uint32_t k, double S[4])
{
    S[0] = S[1] = S[2] = S[3] = 0.0;
#pragma unroll
    for (int dir = 0; dir < 6; ++dir) {
        double E, F[3];
        nb3(ph, L, v, i, j, l, k, dir, E, F[0], F[1], F[2]);
        const int axis = dir >> 1;
        const double sgn = (dir & 1) ? -1.0 : 1.0;
        const double kk = axis == 0 ? L.kx : (axis == 1 ? L.ky : L.kz);
        const double F2 = fma(F[0], F[0], fma(F[1], F[1], F[2] * F[2]));
        const double c2E2 = ph.c2 * E * E;
        const double root = sqrt_nr(fmax(fma(4.0, c2E2, -3.0 * F2), c2E2));
        const double r = ph.c * rcp_nr(fma(2.0 * ph.c, E, root));
        const double iso = fma(-F2, r, ph.c2 * E * (1.0 / 3.0)), r3 = 3.0 * r;
        const double Fa = F[axis];
        S[0] = fma(kk, fma(sgn, Fa, ph.c * E), S[0]);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const double G = fma(r3 * F[m], Fa, m == axis ? iso : 0.0);
            S[1 + m] = fma(kk, fma(sgn, G, ph.c * F[m]), S[1 + m]);
        }
    }
}

// (E, Fx, Fy, T) by the 2-D kernels' local solve, Fz with the divisor the flux components share.
__device__ __forceinline__ void local_solve3(double beta, double g, double a, double ka, double ks, double cv,
                                             double ar, double BE, double BFx, double BFy, double BFz, double BT,
                                             double Tg, double& E, double& Fx, double& Fy, double& Fz, double& T)
{
    local_solve(beta, g, a, ka, ks, cv, ar, BE, BFx, BFy, BT, Tg, E, Fx, Fy, T);
    Fz = BFz * rcp_nr(fma(g, ks, fma(g, a + ka, beta)));
}

}  // namespace

__global__ __launch_bounds__(kB3) void k3_apply(Phys3 ph, Lvl3 L, CSoa3 v, CSoa3 x, double sgn, Soa3 out,
                                                double* __restrict__ partials, const int* __restrict__ active)
{
    const bool live = active[vzero3()] != 0;
    uint32_t k;
    int i, j, l;
    double q = 0.0;
    if (cell3(L, k, i, j, l)) {
        double S[4];
        offdiag3(ph, L, v, i, j, l, k, S);
        const double E = ld(v.E, k), Fx = ld(v.Fx, k), Fy = ld(v.Fy, k), Fz = ld(v.Fz, k), T = ld(v.T, k);
        const double ka = L.cdt * ld(L.sa, k), ks = L.cdt * ld(L.ss, k);
        const double T2 = T * T;
        const double ex = ka * fma(-ph.a_r * T2, T2, E);  // ka (E - a_r T^4)
        const double dF = L.a + ka + ks;
        double rE = sgn * (fma(L.a, E, ex) - S[0]);
        double rFx = sgn * fma(dF, Fx, -S[1]);
        double rFy = sgn * fma(dF, Fy, -S[2]);
        double rFz = sgn * fma(dF, Fz, -S[3]);
        double rT = sgn * fma(ph.c_v, T, -ex);
        if (x.E) {
            rE += ld(x.E, k);
            rFx += ld(x.Fx, k);
            rFy += ld(x.Fy, k);
            rFz += ld(x.Fz, k);
            rT += ld(x.T, k);
        }
        if (partials) {
            const double ic = 1.0 / ph.c;
            const double a = rFx * ic, b = rFy * ic, c = rFz * ic;
            q = fma(rE, rE, fma(a, a, fma(b, b, fma(c, c, rT * rT))));
        }
        if (live && out.E) {
            st(out.E, k, rE);
            st(out.Fx, k, rFx);
            st(out.Fy, k, rFy);
            st(out.Fz, k, rFz);
            st(out.T, k, rT);
        }
    }
    if (partials) block_partial(q, partials + blockIdx.x);
}

__global__ __launch_bounds__(kB3) void k3_relax(Phys3 ph, Lvl3 L, CSoa3 b, double omega, CSoa3 u, Soa3 out,
                                                const int* __restrict__ active)
{
    const bool live = active[vzero3()] != 0;
    uint32_t k;
    int i, j, l;
    if (!cell3(L, k, i, j, l)) return;
    double S[4];
    offdiag3(ph, L, u, i, j, l, k, S);
    const double ka = L.cdt * ld(L.sa, k), ks = L.cdt * ld(L.ss, k);
    const double uE = ld(u.E, k), uFx = ld(u.Fx, k), uFy = ld(u.Fy, k), uFz = ld(u.Fz, k), uT = ld(u.T, k);
    double E, Fx, Fy, Fz, T;
    local_solve3(0.0, 1.0, L.a, ka, ks, ph.c_v, ph.a_r, ld(b.E, k) + S[0], ld(b.Fx, k) + S[1], ld(b.Fy, k) + S[2],
                 ld(b.Fz, k) + S[3], ld(b.T, k), uT, E, Fx, Fy, Fz, T);
    if (omega != 1.0) {
        E = fma(omega, E - uE, uE);
        Fx = fma(omega, Fx - uFx, uFx);
        Fy = fma(omega, Fy - uFy, uFy);
        Fz = fma(omega, Fz - uFz, uFz);
        T = fma(omega, T - uT, uT);
    }
    if (!live) return;
    st(out.E, k, E);
    st(out.Fx, k, Fx);
    st(out.Fy, k, Fy);
    st(out.Fz, k, Fz);
    st(out.T, k, T);
}

// Pseudo-time step: s = M^{-1} f; tau_i = min(dtau, tau*(u, s) reach) (the pseudo time the explicit sub-steps
// reach); u~ = u + tau_i s; one Jacobi sweep of (M + g A)(u) = M u~ from u, g = tau_i (local) or dtau.
__global__ __launch_bounds__(kB3) void k3_pseudo(Phys3 ph, Lvl3 L, CSoa3 f, CSoa3 u, Soa3 out, double dtau_h,
                                                 const double* __restrict__ dtau_dev, double reach, int local,
                                                 const int* __restrict__ active)
{
    const bool live = active[vzero3()] != 0;
    const double dtau = dtau_dev ? dtau_dev[vzero3()] : dtau_h;
    uint32_t k;
    int i, j, l;
    if (!cell3(L, k, i, j, l)) return;
    double S[4];
    offdiag3(ph, L, u, i, j, l, k, S);
    const double ka = L.cdt * ld(L.sa, k), ks = L.cdt * ld(L.ss, k);
    const double uE = ld(u.E, k), uFx = ld(u.Fx, k), uFy = ld(u.Fy, k), uFz = ld(u.Fz, k), uT = ld(u.T, k);
    const double sE = ld(f.E, k), sFx = ld(f.Fx, k), sFy = ld(f.Fy, k), sFz = ld(f.Fz, k);
    const double sT = ld(f.T, k) * rcp_nr(ph.c_v);
    const double ts = ray3(ph.c2, uE, uFx, uFy, uFz, uT, sE, sFx, sFy, sFz, sT);
    const double tau = fmin(dtau, ts * reach);
    const double g = local ? tau : dtau;
    double E, Fx, Fy, Fz, T;
    local_solve3(1.0, g, L.a, ka, ks, ph.c_v, ph.a_r, fma(g, S[0], fma(tau, sE, uE)), fma(g, S[1], fma(tau, sFx, uFx)),
                 fma(g, S[2], fma(tau, sFy, uFy)), fma(g, S[3], fma(tau, sFz, uFz)), ph.c_v * fma(tau, sT, uT), uT, E,
                 Fx, Fy, Fz, T);
    if (!live) return;
    st(out.E, k, E);
    st(out.Fx, k, Fx);
    st(out.Fy, k, Fy);
    st(out.Fz, k, Fz);
    st(out.T, k, T);
}

namespace {

// Full-weighting weights of coarse index I along an axis of nf fine cells: fine 2I-1, 2I, 2I+1 with
// 1/4, 1/2, 1/4; periodic wrap, else a point outside gets weight 0 (and reads the clamped cell) and the
// others are renormalised.
__device__ __forceinline__ void rw3(int I, int nf, bool per, int idx[3], double w[3])
{
    double sum = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        int f = 2 * I - 1 + m;
        double wm = m == 1 ? 0.5 : 0.25;
        if (f < 0 || f >= nf) {
            if (per) {
                f = f < 0 ? f + nf : f - nf;
            } else {
                f = f < 0 ? 0 : nf - 1;
                wm = 0.0;
            }
        }
        idx[m] = f;
        w[m] = wm;
        sum += wm;
    }
    if (sum != 1.0) {
#pragma unroll
        for (int m = 0; m < 3; ++m) w[m] /= sum;
    }
}

// Linear prolongation weights of fine index i from nc coarse cells: even i <- coarse i/2; odd i averages
// i/2 and i/2 + 1 (periodic wrap, else the missing one gets weight 0).
__device__ __forceinline__ void pw3(int i, int nc, bool per, int idx[2], double w[2])
{
    const int I0 = i >> 1;
    idx[0] = idx[1] = I0;
    w[0] = 1.0;
    w[1] = 0.0;
    if ((i & 1) == 0) return;
    int I1 = I0 + 1;
    if (I1 >= nc) {
        if (!per) return;
        I1 -= nc;
    }
    idx[1] = I1;
    w[0] = w[1] = 0.5;
}

}  // namespace

template <int NF>
__global__ __launch_bounds__(kB3) void k3_restrict(int nxf, int nyf, int nzf, int px, int py, int pz, Fields F,
                                                   const int* __restrict__ active)
{
    const bool live = active[vzero3()] != 0;
    const int nxc = nxf / 2, nyc = nyf / 2, nzc = nzf / 2;
    const uint32_t nxy = (uint32_t)nxc * (uint32_t)nyc;
    const uint32_t k = (uint32_t)xcd_block() * kB3 + threadIdx.x;
    if (k >= nxy * (uint32_t)nzc) return;
    const int K = (int)(k / nxy);
    const uint32_t r = k - (uint32_t)K * nxy;
    const int J = (int)(r / (uint32_t)nxc), I = (int)(r - (uint32_t)J * (uint32_t)nxc);
    int ix[3], iy[3], iz[3];
    double wx[3], wy[3], wz[3];
    rw3(I, nxf, px != 0, ix, wx);
    rw3(J, nyf, py != 0, iy, wy);
    rw3(K, nzf, pz != 0, iz, wz);
    double s[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) s[q] = 0.0;
    for (int c = 0; c < 3; ++c) {
        for (int b = 0; b < 3; ++b) {
            const uint32_t row = ((uint32_t)iz[c] * (uint32_t)nyf + (uint32_t)iy[b]) * (uint32_t)nxf;
            const double wyz = wy[b] * wz[c];
#pragma unroll
            for (int q = 0; q < NF; ++q) {
                const double t = fma(wx[2], ld(F.in[q], row + ix[2]),
                                     fma(wx[1], ld(F.in[q], row + ix[1]), wx[0] * ld(F.in[q], row + ix[0])));
                s[q] = fma(wyz, t, s[q]);
            }
        }
    }
    if (!live) return;
#pragma unroll
    for (int q = 0; q < NF; ++q) st(F.out[q], k, s[q]);
}

__global__ __launch_bounds__(kB3) void k3_prolong_project(Phys3 ph, int nx, int ny, int nz, int px, int py, int pz,
                                                          double eta, CSoa3 u, CSoa3 uc, CSoa3 vc, Soa3 out,
                                                          const int* __restrict__ active)
{
    const bool live = active[vzero3()] != 0;
    const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
    const uint32_t k = (uint32_t)xcd_block() * kB3 + threadIdx.x;
    if (k >= nxy * (uint32_t)nz) return;
    const int l = (int)(k / nxy);
    const uint32_t r = k - (uint32_t)l * nxy;
    const int j = (int)(r / (uint32_t)nx), i = (int)(r - (uint32_t)j * (uint32_t)nx);
    const int nxc = nx / 2, nyc = ny / 2, nzc = nz / 2;
    int ix[2], iy[2], iz[2];
    double wx[2], wy[2], wz[2];
    pw3(i, nxc, px != 0, ix, wx);
    pw3(j, nyc, py != 0, iy, wy);
    pw3(l, nzc, pz != 0, iz, wz);
    double e[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const double w = wx[a] * wy[b] * wz[c];
                if (w == 0.0) continue;
                const uint32_t kc = ((uint32_t)iz[c] * (uint32_t)nyc + (uint32_t)iy[b]) * (uint32_t)nxc + (uint32_t)ix[a];
                e[0] = fma(w, ld(uc.E, kc) - ld(vc.E, kc), e[0]);
                e[1] = fma(w, ld(uc.Fx, kc) - ld(vc.Fx, kc), e[1]);
                e[2] = fma(w, ld(uc.Fy, kc) - ld(vc.Fy, kc), e[2]);
                e[3] = fma(w, ld(uc.Fz, kc) - ld(vc.Fz, kc), e[3]);
                e[4] = fma(w, ld(uc.T, kc) - ld(vc.T, kc), e[4]);
            }
    const double uE = ld(u.E, k), uFx = ld(u.Fx, k), uFy = ld(u.Fy, k), uFz = ld(u.Fz, k), uT = ld(u.T, k);
    double wE = uE + e[0], wFx = uFx + e[1], wFy = uFy + e[2], wFz = uFz + e[3], wT = uT + e[4];
    if (!admissible3(ph.c2, wE, wFx, wFy, wFz, wT)) {  // eq. prolongatedSol
        const double th = eta * fmin(ray3(ph.c2, uE, uFx, uFy, uFz, uT, e[0], e[1], e[2], e[3], e[4]), 1.0);
        wE = fma(th, e[0], uE);
        wFx = fma(th, e[1], uFx);
        wFy = fma(th, e[2], uFy);
        wFz = fma(th, e[3], uFz);
        wT = fma(th, e[4], uT);
    }
    if (!live) return;
    st(out.E, k, wE);
    st(out.Fx, k, wFx);
    st(out.Fy, k, wFy);
    st(out.Fz, k, wFz);
    st(out.T, k, wT);
}

__global__ __launch_bounds__(kB3) void k3_make_rhs(int64_t n, double cv, CSoa3 v, Soa3 b)
{
    const int64_t k = (int64_t)blockIdx.x * kB3 + threadIdx.x;
    if (k >= n) return;
    b.E[k] = v.E[k];
    b.Fx[k] = v.Fx[k];
    b.Fy[k] = v.Fy[k];
    b.Fz[k] = v.Fz[k];
    b.T[k] = cv * v.T[k];
}

__global__ __launch_bounds__(kB3) void k3_copy(int64_t n, CSoa3 a, Soa3 b)
{
    const int64_t k = (int64_t)blockIdx.x * kB3 + threadIdx.x;
    if (k >= n) return;
    b.E[k] = a.E[k];
    b.Fx[k] = a.Fx[k];
    b.Fy[k] = a.Fy[k];
    b.Fz[k] = a.Fz[k];
    b.T[k] = a.T[k];
}

__global__ __launch_bounds__(kB3) void k3_check_state(int64_t n, double c, CSoa3 v, unsigned long long* bad)
{
    const int64_t k = (int64_t)blockIdx.x * kB3 + threadIdx.x;
    if (k >= n) return;
    const double E = v.E[k], Fx = v.Fx[k], Fy = v.Fy[k], Fz = v.Fz[k], T = v.T[k];
    const bool ok = isfinite(E) && isfinite(Fx) && isfinite(Fy) && isfinite(Fz) && isfinite(T) && E > 0.0 &&
                    T > 0.0 && sqrt(fma(Fx, Fx, fma(Fy, Fy, Fz * Fz))) <= c * E * (1.0 + 1e-12);
    if (!ok) atomicMin(bad, (unsigned long long)k);
}

// ---- launchers ----------------------------------------------------------------
void launch3_apply(hipStream_t st, const Phys3& ph, const Lvl3& L, CSoa3 v, CSoa3 x, double sgn, Soa3 out,
                   double* partials, const int* active)
{
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(k3_apply, dim3(blocks3(n)), dim3(kB3), 0, st, ph, L, v, x, sgn, out, partials, active);
}

void launch3_relax(hipStream_t st, const Phys3& ph, const Lvl3& L, CSoa3 b, double omega, CSoa3 in, Soa3 out,
                   const int* active)
{
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(k3_relax, dim3(blocks3(n)), dim3(kB3), 0, st, ph, L, b, omega, in, out, active);
}

void launch3_pseudo(hipStream_t st, const Phys3& ph, const Lvl3& L, CSoa3 f, CSoa3 in, Soa3 out, double dtau,
                    const double* dtau_dev, double reach, int local, const int* active)
{
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(k3_pseudo, dim3(blocks3(n)), dim3(kB3), 0, st, ph, L, f, in, out, dtau, dtau_dev, reach, local,
                       active);
}

void launch3_restrict(hipStream_t st, int nxf, int nyf, int nzf, int px, int py, int pz, const Fields& F,
                      const int* active)
{
    const int64_t nc = (int64_t)(nxf / 2) * (nyf / 2) * (nzf / 2);
    const dim3 g(blocks3(nc)), b(kB3);
    switch (F.n) {
    case 2: hipLaunchKernelGGL((k3_restrict<2>), g, b, 0, st, nxf, nyf, nzf, px, py, pz, F, active); break;
    case 5: hipLaunchKernelGGL((k3_restrict<5>), g, b, 0, st, nxf, nyf, nzf, px, py, pz, F, active); break;
    default: hipLaunchKernelGGL((k3_restrict<10>), g, b, 0, st, nxf, nyf, nzf, px, py, pz, F, active); break;
    }
}

void launch3_prolong_project(hipStream_t st, const Phys3& ph, int nx, int ny, int nz, int px, int py, int pz,
                             double eta, CSoa3 u, CSoa3 uc, CSoa3 vc, Soa3 out, const int* active)
{
    const int64_t n = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL(k3_prolong_project, dim3(blocks3(n)), dim3(kB3), 0, st, ph, nx, ny, nz, px, py, pz, eta, u, uc,
                       vc, out, active);
}

void launch3_make_rhs(hipStream_t st, int64_t n, double cv, CSoa3 v, Soa3 b)
{
    hipLaunchKernelGGL(k3_make_rhs, dim3(blocks3(n)), dim3(kB3), 0, st, n, cv, v, b);
}

void launch3_check_state(hipStream_t st, int64_t n, double c, CSoa3 v, unsigned long long* bad)
{
    hipLaunchKernelGGL(k3_check_state, dim3(blocks3(n)), dim3(kB3), 0, st, n, c, v, bad);
}

void launch3_copy(hipStream_t st, int64_t n, CSoa3 a, Soa3 b)
{
    hipLaunchKernelGGL(k3_copy, dim3(blocks3(n)), dim3(kB3), 0, st, n, a, b);
}

}  // namespace m1
