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

#include <atomic>

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

// The closure of one state as the directional fluxes use it: c^2 P_ab = iso delta_ab + r3 F_a F_b (the
// arrangement of the 2-D kernels' closure).
struct Rec3 {
    double E, F[3], iso, r3;
};

__device__ __forceinline__ Rec3 rec3(const Phys3& ph, double E, double Fx, double Fy, double Fz)
{
    Rec3 R;
    R.E = E;
    R.F[0] = Fx;
    R.F[1] = Fy;
    R.F[2] = Fz;
    const double F2 = fma(Fx, Fx, fma(Fy, Fy, Fz * Fz));
    const double c2E2 = ph.c2 * E * E;
    const double root = sqrt_nr(fmax(fma(4.0, c2E2, -3.0 * F2), c2E2));
    const double r = ph.c * rcp_nr(fma(2.0 * ph.c, E, root));
    R.iso = fma(-F2, r, ph.c2 * E * (1.0 / 3.0));
    R.r3 = 3.0 * r;
    return R;
}

// Add a neighbour's operator along `axis`: sgn = +1 for the lower neighbour (L = kk (cU + G)), -1 for the
// upper one (R = kk (cU - G)), G = (F_axis, c^2 P[., axis]).
__device__ __forceinline__ void add3(const Phys3& ph, double kk, double sgn, int axis, const Rec3& R, double S[4])
{
    const double Fa = R.F[axis];
    S[0] = fma(kk, fma(sgn, Fa, ph.c * R.E), S[0]);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const double G = fma(R.r3 * R.F[m], Fa, m == axis ? R.iso : 0.0);
        S[1 + m] = fma(kk, fma(sgn, G, ph.c * R.F[m]), S[1 + m]);
    }
}

// Sum of the six off-diagonal operators of row k in the order x-, x+, y-, y+, z-, z+.
__device__ __forceinline__ void offdiag3(const Phys3& ph, const Lvl3& L, const CSoa3& v, int i, int j, int l,
                                         uint32_t k, double S[4])
{
    S[0] = S[1] = S[2] = S[3] = 0.0;
#pragma unroll
    for (int dir = 0; dir < 6; ++dir) {
        double E, Fx, Fy, Fz;
        nb3(ph, L, v, i, j, l, k, dir, E, Fx, Fy, Fz);
        const int axis = dir >> 1;
        add3(ph, axis == 0 ? L.kx : (axis == 1 ? L.ky : L.kz), (dir & 1) ? -1.0 : 1.0, axis,
             rec3(ph, E, Fx, Fy, Fz), S);
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

// ---- per-cell ends of the three operations, from the cell's state u and its off-diagonal sum S ----------
// x + sgn A(u) (x.E null: sgn A(u)) into o; returns r_E^2 + |r_F/c|^2 + r_T^2 of o.
__device__ __forceinline__ double fin_apply(const Phys3& ph, const Lvl3& L, const double u[5], const double S[4],
                                            const CSoa3& x, double sgn, uint32_t k, double o[5])
{
    const double ka = L.cdt * ld(L.sa, k), ks = L.cdt * ld(L.ss, k);
    const double T2 = u[4] * u[4];
    const double ex = ka * fma(-ph.a_r * T2, T2, u[0]);  // ka (E - a_r T^4)
    const double dF = L.a + ka + ks;
    o[0] = sgn * (fma(L.a, u[0], ex) - S[0]);
    o[1] = sgn * fma(dF, u[1], -S[1]);
    o[2] = sgn * fma(dF, u[2], -S[2]);
    o[3] = sgn * fma(dF, u[3], -S[3]);
    o[4] = sgn * fma(ph.c_v, u[4], -ex);
    if (x.E) {
        o[0] += ld(x.E, k);
        o[1] += ld(x.Fx, k);
        o[2] += ld(x.Fy, k);
        o[3] += ld(x.Fz, k);
        o[4] += ld(x.T, k);
    }
    const double ic = 1.0 / ph.c;
    const double a = o[1] * ic, b = o[2] * ic, c = o[3] * ic;
    return fma(o[0], o[0], fma(a, a, fma(b, b, fma(c, c, o[4] * o[4]))));
}

// Relaxed Jacobi update of A(u) = b: u + omega (local_solve(b + S) - u).
__device__ __forceinline__ void fin_relax(const Phys3& ph, const Lvl3& L, const double u[5], const double S[4],
                                          const CSoa3& b, double omega, uint32_t k, double o[5])
{
    const double ka = L.cdt * ld(L.sa, k), ks = L.cdt * ld(L.ss, k);
    local_solve3(0.0, 1.0, L.a, ka, ks, ph.c_v, ph.a_r, ld(b.E, k) + S[0], ld(b.Fx, k) + S[1], ld(b.Fy, k) + S[2],
                 ld(b.Fz, k) + S[3], ld(b.T, k), u[4], o[0], o[1], o[2], o[3], o[4]);
    if (omega != 1.0) {
#pragma unroll
        for (int q = 0; q < 5; ++q) o[q] = fma(omega, o[q] - u[q], u[q]);
    }
}

// Pseudo-time step: s = M^{-1} f; tau_i = min(dtau, tau*(u, s) reach) (the pseudo time the explicit sub-steps
// reach); u~ = u + tau_i s; one Jacobi sweep of (M + g A)(u) = M u~ from u, g = tau_i (local) or dtau.
__device__ __forceinline__ void fin_pseudo(const Phys3& ph, const Lvl3& L, const double u[5], const double S[4],
                                           const CSoa3& f, double dtau, double reach, int local, uint32_t k,
                                           double o[5], bool& stall)
{
    const double ka = L.cdt * ld(L.sa, k), ks = L.cdt * ld(L.ss, k);
    const double sE = ld(f.E, k), sFx = ld(f.Fx, k), sFy = ld(f.Fy, k), sFz = ld(f.Fz, k);
    const double sT = ld(f.T, k) * rcp_nr(ph.c_v);
    const double ts = ray3(ph.c2, u[0], u[1], u[2], u[3], u[4], sE, sFx, sFy, sFz, sT);
    stall = ts == 0.0;
    const double tau = fmin(dtau, ts * reach);
    const double g = local ? tau : dtau;
    local_solve3(1.0, g, L.a, ka, ks, ph.c_v, ph.a_r, fma(g, S[0], fma(tau, sE, u[0])),
                 fma(g, S[1], fma(tau, sFx, u[1])), fma(g, S[2], fma(tau, sFy, u[2])),
                 fma(g, S[3], fma(tau, sFz, u[3])), ph.c_v * fma(tau, sT, u[4]), u[4], o[0], o[1], o[2], o[3], o[4]);
}

__device__ __forceinline__ void st5(const Soa3& out, uint32_t k, const double o[5])
{
    st(out.E, k, o[0]);
    st(out.Fx, k, o[1]);
    st(out.Fy, k, o[2]);
    st(out.Fz, k, o[3]);
    st(out.T, k, o[4]);
}

__device__ __forceinline__ void load5(const CSoa3& v, uint32_t k, double u[5])
{
    u[0] = ld(v.E, k);
    u[1] = ld(v.Fx, k);
    u[2] = ld(v.Fy, k);
    u[3] = ld(v.Fz, k);
    u[4] = ld(v.T, k);
}

}  // namespace

__global__ __launch_bounds__(kB3) void k3_apply(Phys3 ph, Lvl3 L, CSoa3 v, CSoa3 x, double sgn, Soa3 out,
                                                double* __restrict__ partials, const int* __restrict__ active)
{
    const bool live = active[vzero3()] != 0;
    if (!live) return;  // a cycle enqueued after the stop: nothing to compute (the flag is uniform)
    uint32_t k;
    int i, j, l;
    double q = 0.0;
    if (cell3(L, k, i, j, l)) {
        double S[4], u[5], o[5];
        offdiag3(ph, L, v, i, j, l, k, S);
        load5(v, k, u);
        q = fin_apply(ph, L, u, S, x, sgn, k, o);
        if (live && out.E) st5(out, k, o);
    }
    if (partials) block_partial(q, partials + blockIdx.x);
}

// NORM: also the norm partials of the input's residual b - A(u) (per cell fin_apply's value, as k3_apply).
template <bool NORM>
__global__ __launch_bounds__(kB3) void k3_relax(Phys3 ph, Lvl3 L, CSoa3 b, double omega, CSoa3 u, Soa3 out,
                                                double* __restrict__ partials, const int* __restrict__ active)
{
    const bool live = active[vzero3()] != 0;
    if (!live) return;  // a cycle enqueued after the stop: nothing to compute (the flag is uniform)
    uint32_t k;
    int i, j, l;
    double q = 0.0;
    if (cell3(L, k, i, j, l)) {
        double S[4], uc[5], o[5];
        offdiag3(ph, L, u, i, j, l, k, S);
        load5(u, k, uc);
        if (NORM) q = fin_apply(ph, L, uc, S, b, -1.0, k, o);
        fin_relax(ph, L, uc, S, b, omega, k, o);
        if (live) st5(out, k, o);
    }
    if (NORM) block_partial(q, partials + blockIdx.x);
}

__global__ __launch_bounds__(kB3) void k3_pseudo(Phys3 ph, Lvl3 L, CSoa3 f, CSoa3 u, Soa3 out, double dtau_h,
                                                 const double* __restrict__ dtau_dev, double reach, int local,
                                                 const int* __restrict__ active)
{
    const bool live = active[vzero3()] != 0;
    if (!live) return;  // a cycle enqueued after the stop: nothing to compute (the flag is uniform)
    const double dtau = dtau_dev ? dtau_dev[vzero3()] : dtau_h;
    uint32_t k;
    int i, j, l;
    if (!cell3(L, k, i, j, l)) return;
    double S[4], uc[5], o[5];
    offdiag3(ph, L, u, i, j, l, k, S);
    load5(u, k, uc);
    bool stall;
    fin_pseudo(ph, L, uc, S, f, dtau, reach, local, k, o, stall);
    if (!live) return;
    if (stall && ph.stalls) note_stall(ph.stalls);
    st5(out, k, o);
}

// ---- the same three operations staged: 2.5-D blocking ---------------------------------------------------
// A block owns a 64 x 4 column of cells in x-y and marches through kSZ z-planes.  For each plane the
// closures of the tile and of its one-cell ring (with the ghost rules at the sides) are evaluated once into
// LDS; each thread keeps the closures of its own column's planes below and above in registers.  Every cell's
// off-diagonal sum then adds the same six terms in the same order as the one-cell kernels, from the same
// closure values, so the results are bitwise those of k3_apply / k3_relax / k3_pseudo.  About 1.5 closure
// evaluations per cell instead of 6.
namespace {

// 8 planes per block: about 2 % less time per sweep than 16 and 1.5 % less than 4 at 256^3 (more blocks to balance
// against the two extra column closures a block evaluates to start its march)
constexpr int kSX = 64, kSY = 4, kSZ = 8, kSW = kSX + 2, kSH = kSY + 2, kSN = kSW * kSH, kRing = kSN - kSX * kSY;

// Closure record of the neighbour position (gx, gy) of plane z: a cell, the ghost beyond an x or y side (by the
// side's rule, as nb3), or (never read) a placeholder.
__device__ __forceinline__ Rec3 plane_rec(const Phys3& ph, const Lvl3& L, const CSoa3& v, int gx, int gy, int z)
{
    const bool inX = gx >= 0 && gx < L.nx, inY = gy >= 0 && gy < L.ny;
    int side = -1;
    if (inX && inY) {
        const uint32_t k = ((uint32_t)z * (uint32_t)L.ny + (uint32_t)gy) * (uint32_t)L.nx + (uint32_t)gx;
        return rec3(ph, ld(v.E, k), ld(v.Fx, k), ld(v.Fy, k), ld(v.Fz, k));
    }
    if (inY && (gx == -1 || gx == L.nx)) side = gx < 0 ? 0 : 1;
    else if (inX && (gy == -1 || gy == L.ny)) side = gy < 0 ? 2 : 3;
    if (side < 0) {
        Rec3 R{};
        R.E = 1.0;
        return R;
    }
    const int kind = ph.bc[side];
    if (kind == BC_DIRICHLET) return rec3(ph, ph.bcE[side], ph.bcFx[side], ph.bcFy[side], ph.bcFz[side]);
    int sx = gx, sy = gy;
    if (side < 2) sx = kind == BC_PERIODIC ? (gx < 0 ? L.nx - 1 : 0) : (gx < 0 ? 0 : L.nx - 1);
    else sy = kind == BC_PERIODIC ? (gy < 0 ? L.ny - 1 : 0) : (gy < 0 ? 0 : L.ny - 1);
    const uint32_t k = ((uint32_t)z * (uint32_t)L.ny + (uint32_t)sy) * (uint32_t)L.nx + (uint32_t)sx;
    Rec3 R = rec3(ph, ld(v.E, k), ld(v.Fx, k), ld(v.Fy, k), ld(v.Fz, k));
    if (kind == BC_REFLECTIVE) {  // the normal component (constant indices: no private array in memory)
        if (side < 2) R.F[0] = -R.F[0];
        else R.F[1] = -R.F[1];
    }
    return R;
}

// Closure record of cell (i, j) in plane zz of its own column, or the ghost below z = 0 / above z = nz - 1.
__device__ __forceinline__ Rec3 column_rec(const Phys3& ph, const Lvl3& L, const CSoa3& v, int i, int j, int zz)
{
    int z = zz, kind = -1;
    if (zz < 0 || zz >= L.nz) {
        const int side = zz < 0 ? 4 : 5;
        kind = ph.bc[side];
        if (kind == BC_DIRICHLET) return rec3(ph, ph.bcE[side], ph.bcFx[side], ph.bcFy[side], ph.bcFz[side]);
        z = kind == BC_PERIODIC ? (zz < 0 ? L.nz - 1 : 0) : (zz < 0 ? 0 : L.nz - 1);
    }
    const uint32_t k = ((uint32_t)z * (uint32_t)L.ny + (uint32_t)j) * (uint32_t)L.nx + (uint32_t)i;
    Rec3 R = rec3(ph, ld(v.E, k), ld(v.Fx, k), ld(v.Fy, k), ld(v.Fz, k));
    if (kind == BC_REFLECTIVE) R.F[2] = -R.F[2];
    return R;
}

}  // namespace

struct StageArgs3 {
    CSoa3 rhs;      // apply: x (nullable); relax: b; pseudo: f
    double* partials;  // relax with the norm: per block
    double omega;   // relax
    double sgn;     // apply
    Soa3 out;
    double dtau;    // pseudo (dtau_dev when set)
    const double* dtau_dev;
    double reach;
    int local;
};

// MODE 0: out = x + sgn A(u); 1: relaxed Jacobi sweep; 2: pseudo-time step; 3: the sweep with the norm
// partials of its input's residual b - A(u) (per cell fin_apply's value, as k3_apply)
template <int MODE>
__global__ __launch_bounds__(kB3) void k3_staged(Phys3 ph, Lvl3 L, CSoa3 u, StageArgs3 A,
                                                 const int* __restrict__ active)
{
    __shared__ double sE[kSN], sF0[kSN], sF1[kSN], sF2[kSN], sI[kSN], sR[kSN];
    const bool live = active[vzero3()] != 0;
    if (!live) return;  // a cycle enqueued after the stop: nothing to compute (the flag is uniform)
    const double dtau = (MODE == 2 && A.dtau_dev) ? A.dtau_dev[vzero3()] : A.dtau;
    const int ntx = (L.nx + kSX - 1) / kSX, nty = (L.ny + kSY - 1) / kSY;
    const int b = (int)xcd_block();
    const int tz = b / (ntx * nty), rem = b - tz * ntx * nty, tyb = rem / ntx, txb = rem - tyb * ntx;
    const int x0 = txb * kSX, y0 = tyb * kSY, z0 = tz * kSZ, z1 = min(z0 + kSZ, L.nz);
    const int tx = threadIdx.x & (kSX - 1), ty = threadIdx.x / kSX;
    const int i = x0 + tx, j = y0 + ty;
    const bool own = i < L.nx && j < L.ny;
    auto put = [&](int p, const Rec3& R) {
        sE[p] = R.E;
        sF0[p] = R.F[0];
        sF1[p] = R.F[1];
        sF2[p] = R.F[2];
        sI[p] = R.iso;
        sR[p] = R.r3;
    };
    auto get = [&](int p) {
        Rec3 R;
        R.E = sE[p];
        R.F[0] = sF0[p];
        R.F[1] = sF1[p];
        R.F[2] = sF2[p];
        R.iso = sI[p];
        R.r3 = sR[p];
        return R;
    };
    // the ring position this thread fills: rows above and below the tile, then the columns left and right
    int rx = 0, ry = 0;
    const int r = threadIdx.x;
    if (r < kRing) {
        if (r < 2 * kSX) {
            rx = 1 + (r & (kSX - 1));
            ry = r < kSX ? 0 : kSH - 1;
        } else {
            rx = ((r - 2 * kSX) & 1) ? kSW - 1 : 0;
            ry = (r - 2 * kSX) >> 1;
        }
    }
    Rec3 prev{}, cur{}, next{};
    if (own) {
        prev = column_rec(ph, L, u, i, j, z0 - 1);
        cur = column_rec(ph, L, u, i, j, z0);
    }
    const int slot = (ty + 1) * kSW + tx + 1;
    double q = 0.0;
    for (int z = z0; z < z1; ++z) {
        if (own) next = column_rec(ph, L, u, i, j, z + 1);
        __syncthreads();  // the previous plane's reads are done
        put(slot, own ? cur : plane_rec(ph, L, u, i, j, z));
        if (r < kRing) put(ry * kSW + rx, plane_rec(ph, L, u, x0 - 1 + rx, y0 - 1 + ry, z));
        __syncthreads();
        if (own) {
            double S[4] = {0.0, 0.0, 0.0, 0.0};
            add3(ph, L.kx, 1.0, 0, get(slot - 1), S);
            add3(ph, L.kx, -1.0, 0, get(slot + 1), S);
            add3(ph, L.ky, 1.0, 1, get(slot - kSW), S);
            add3(ph, L.ky, -1.0, 1, get(slot + kSW), S);
            add3(ph, L.kz, 1.0, 2, prev, S);
            add3(ph, L.kz, -1.0, 2, next, S);
            const uint32_t k = ((uint32_t)z * (uint32_t)L.ny + (uint32_t)j) * (uint32_t)L.nx + (uint32_t)i;
            double uc[5] = {cur.E, cur.F[0], cur.F[1], cur.F[2], ld(u.T, k)}, o[5];
            bool stall = false;
            if (MODE == 3) q += fin_apply(ph, L, uc, S, A.rhs, -1.0, k, o);
            if (MODE == 0) (void)fin_apply(ph, L, uc, S, A.rhs, A.sgn, k, o);
            else if (MODE == 1 || MODE == 3) fin_relax(ph, L, uc, S, A.rhs, A.omega, k, o);
            else fin_pseudo(ph, L, uc, S, A.rhs, dtau, A.reach, A.local, k, o, stall);
            if (live && stall && ph.stalls) note_stall(ph.stalls);
            if (live && A.out.E) st5(A.out, k, o);
        }
        prev = cur;
        cur = next;
    }
    if (MODE == 3) block_partial(q, A.partials + blockIdx.x);  // every thread of the block gets here
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
    if (!live) return;  // a cycle enqueued after the stop: nothing to compute (the flag is uniform)
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

// u + e at fine cell k with the admissibility correction of eq. prolongatedSol, stored when live.
__device__ __forceinline__ void project_store3(const Phys3& ph, double eta, const CSoa3& u, const double e[5],
                                               const Soa3& out, uint32_t k, bool live)
{
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

__global__ __launch_bounds__(kB3) void k3_prolong_project(Phys3 ph, int nx, int ny, int nz, int px, int py, int pz,
                                                          double eta, CSoa3 u, CSoa3 uc, CSoa3 vc, Soa3 out,
                                                          const int* __restrict__ active)
{
    const bool live = active[vzero3()] != 0;
    if (!live) return;  // a cycle enqueued after the stop: nothing to compute (the flag is uniform)
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
    project_store3(ph, eta, u, e, out, k, live);
}

// The same correction with the coarse differences staged: a block owns a 32 x 4 x 2 tile of coarse cells
// (its 64 x 8 x 4 fine cells); the differences uc - vc of the tile and of the next coarse cell along each axis
// go to LDS once (about 1.9 loads per coarse value instead of 27 per fine cell's eight), then each thread
// corrects eight fine cells, x fastest.  Each fine cell sums its coarse differences with pw3's weights in
// k3_prolong_project's order, so the results are bitwise that kernel's.  Fine sides even (twice the coarse).
namespace {
constexpr int kPX = 32, kPY = 4, kPZ = 2, kPW = kPX + 1, kPH = kPY + 1, kPD = kPZ + 1, kPN = kPW * kPH * kPD;
}  // namespace

__global__ __launch_bounds__(kB3) void k3_prolong_project_lds(Phys3 ph, int nx, int ny, int nz, int px, int py,
                                                              int pz, double eta, CSoa3 u, CSoa3 uc, CSoa3 vc,
                                                              Soa3 out, const int* __restrict__ active)
{
    __shared__ double dq[5][kPN];
    const bool live = active[vzero3()] != 0;
    if (!live) return;  // a cycle enqueued after the stop: nothing to compute (the flag is uniform)
    const int nxc = nx / 2, nyc = ny / 2, nzc = nz / 2;
    const int tbx = (nxc + kPX - 1) / kPX, tby = (nyc + kPY - 1) / kPY;
    const int blk = (int)xcd_block();
    const int tz = blk / (tbx * tby), rem = blk - tz * tbx * tby, ty = rem / tbx, tx = rem - ty * tbx;
    const int I0 = tx * kPX, J0 = ty * kPY, K0 = tz * kPZ;
    // coarse index of tile offset a along an axis: past the end wraps when periodic, else clamps (such a
    // cell has weight 0 wherever it is read, or belongs to no fine cell of the grid)
    const auto cidx = [](int I, int nc, int per) {
        if (I >= nc) I = per ? I - nc : nc - 1;
        return I < nc ? I : nc - 1;
    };
    for (int t = threadIdx.x; t < kPN; t += kB3) {
        const int c = t / (kPW * kPH), r = t - c * kPW * kPH, b = r / kPW, a = r - b * kPW;
        const uint32_t kc = ((uint32_t)cidx(K0 + c, nzc, pz) * (uint32_t)nyc + (uint32_t)cidx(J0 + b, nyc, py)) *
                                (uint32_t)nxc + (uint32_t)cidx(I0 + a, nxc, px);
        dq[0][t] = ld(uc.E, kc) - ld(vc.E, kc);
        dq[1][t] = ld(uc.Fx, kc) - ld(vc.Fx, kc);
        dq[2][t] = ld(uc.Fy, kc) - ld(vc.Fy, kc);
        dq[3][t] = ld(uc.Fz, kc) - ld(vc.Fz, kc);
        dq[4][t] = ld(uc.T, kc) - ld(vc.T, kc);
    }
    __syncthreads();
    // pw3 along one axis for fine offset f of the tile: local coarse slots and weights
    const auto weights = [](int f, int C0, int nc, int per, int s[2], double w[2]) {
        const int Il = f >> 1;
        s[0] = s[1] = Il;
        w[0] = 1.0;
        w[1] = 0.0;
        if ((f & 1) == 0 || (C0 + Il + 1 >= nc && !per)) return;
        s[1] = Il + 1;
        w[0] = w[1] = 0.5;
    };
#pragma unroll 1
    for (int m = 0; m < 8; ++m) {
        const int q = (int)threadIdx.x + kB3 * m;  // fine offset in the 64 x 8 x 4 tile, x fastest
        const int fz = q / (2 * kPX * 2 * kPY), r = q - fz * (2 * kPX * 2 * kPY), fy = r / (2 * kPX),
                  fx = r - fy * (2 * kPX);
        const int i = 2 * I0 + fx, j = 2 * J0 + fy, l = 2 * K0 + fz;
        if (i >= nx || j >= ny || l >= nz) continue;
        int sx[2], sy[2], sz[2];
        double wx[2], wy[2], wz[2];
        weights(fx, I0, nxc, px, sx, wx);
        weights(fy, J0, nyc, py, sy, wy);
        weights(fz, K0, nzc, pz, sz, wz);
        double e[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    const double w = wx[a] * wy[b] * wz[c];
                    if (w == 0.0) continue;
                    const int t = (sz[c] * kPH + sy[b]) * kPW + sx[a];
#pragma unroll
                    for (int f = 0; f < 5; ++f) e[f] = fma(w, dq[f][t], e[f]);
                }
        const uint32_t k = ((uint32_t)l * (uint32_t)ny + (uint32_t)j) * (uint32_t)nx + (uint32_t)i;
        project_store3(ph, eta, u, e, out, k, live);
    }
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

unsigned launch3_relax(hipStream_t st, const Phys3& ph, const Lvl3& L, CSoa3 b, double omega, CSoa3 in, Soa3 out,
                       const int* active, double* partials)
{
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    const unsigned g = blocks3(n);
    if (partials)
        hipLaunchKernelGGL(k3_relax<true>, dim3(g), dim3(kB3), 0, st, ph, L, b, omega, in, out, partials, active);
    else
        hipLaunchKernelGGL(k3_relax<false>, dim3(g), dim3(kB3), 0, st, ph, L, b, omega, in, out, nullptr, active);
    return g;
}

void launch3_pseudo(hipStream_t st, const Phys3& ph, const Lvl3& L, CSoa3 f, CSoa3 in, Soa3 out, double dtau,
                    const double* dtau_dev, double reach, int local, const int* active)
{
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(k3_pseudo, dim3(blocks3(n)), dim3(kB3), 0, st, ph, L, f, in, out, dtau, dtau_dev, reach, local,
                       active);
}

namespace {
std::atomic<int> g_stage3{1};
std::atomic<int> g_prolong_lds{1};

unsigned staged_blocks(const Lvl3& L) { return (unsigned)staged3_blocks(L.nx, L.ny, L.nz); }
}  // namespace

int64_t staged3_blocks(int nx, int ny, int nz)
{
    return (int64_t)((nx + kSX - 1) / kSX) * ((ny + kSY - 1) / kSY) * ((nz + kSZ - 1) / kSZ);
}

void set_stage3(int mode) { g_stage3 = mode < 0 ? 0 : (mode > 2 ? 2 : mode); }
int stage3() { return g_stage3.load(); }
void set_prolong3_lds(int on) { g_prolong_lds = on != 0; }
int prolong3_lds() { return g_prolong_lds.load(); }
bool stage3_fits(const Lvl3& L, bool sweep)
{
    const int m = g_stage3.load();
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    return L.nx >= kStage3MinNx && (m == 2 || (m == 1 && sweep && n >= kStage3MinCells));
}

void launch3_apply_staged(hipStream_t st, const Phys3& ph, const Lvl3& L, CSoa3 v, CSoa3 x, double sgn, Soa3 out,
                          const int* active)
{
    StageArgs3 A{};
    A.rhs = x;
    A.sgn = sgn;
    A.out = out;
    hipLaunchKernelGGL(k3_staged<0>, dim3(staged_blocks(L)), dim3(kB3), 0, st, ph, L, v, A, active);
}

unsigned launch3_relax_staged(hipStream_t st, const Phys3& ph, const Lvl3& L, CSoa3 b, double omega, CSoa3 in,
                              Soa3 out, const int* active, double* partials)
{
    StageArgs3 A{};
    A.rhs = b;
    A.omega = omega;
    A.out = out;
    A.partials = partials;
    const unsigned g = staged_blocks(L);
    if (partials) hipLaunchKernelGGL(k3_staged<3>, dim3(g), dim3(kB3), 0, st, ph, L, in, A, active);
    else hipLaunchKernelGGL(k3_staged<1>, dim3(g), dim3(kB3), 0, st, ph, L, in, A, active);
    return g;
}

void launch3_pseudo_staged(hipStream_t st, const Phys3& ph, const Lvl3& L, CSoa3 f, CSoa3 in, Soa3 out,
                           double dtau, const double* dtau_dev, double reach, int local, const int* active)
{
    StageArgs3 A{};
    A.rhs = f;
    A.out = out;
    A.dtau = dtau;
    A.dtau_dev = dtau_dev;
    A.reach = reach;
    A.local = local;
    hipLaunchKernelGGL(k3_staged<2>, dim3(staged_blocks(L)), dim3(kB3), 0, st, ph, L, in, A, active);
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
    if (g_prolong_lds.load() && nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0) {
        const int nxc = nx / 2, nyc = ny / 2, nzc = nz / 2;
        const unsigned g = (unsigned)(((nxc + kPX - 1) / kPX) * ((nyc + kPY - 1) / kPY) * ((nzc + kPZ - 1) / kPZ));
        hipLaunchKernelGGL(k3_prolong_project_lds, dim3(g), dim3(kB3), 0, st, ph, nx, ny, nz, px, py, pz, eta, u, uc,
                           vc, out, active);
    }
    else
        hipLaunchKernelGGL(k3_prolong_project, dim3(blocks3(n)), dim3(kB3), 0, st, ph, nx, ny, nz, px, py, pz, eta,
                           u, uc, vc, out, active);
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
