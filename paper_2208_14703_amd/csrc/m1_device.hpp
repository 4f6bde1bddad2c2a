// m1_device.hpp -- per-cell device math of the implicit M1 solver (gfx950, wave64).
//
// Everything here is FP64 and register-only; the kernels in m1_kernels.hip
// compose these pieces into stencil sweeps.  Formulas follow the paper
// (arXiv 2208.14703) but are arranged for the GPU: the closure is written
// through one square root and one division with no 0/0 at F = 0, and the
// local source solve warm-starts Newton's method from the previous T.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace m1 {

enum BcKind : int { BC_PERIODIC = 0, BC_REFLECTIVE = 1, BC_NEUMANN = 2, BC_DIRICHLET = 3, BC_INFLOW = 4 };

// Physics and boundary data shared by every level.
struct Phys {
    double c, c2, a_r, c_v;
    int bc[4];  // x-, x+, y-, y+
    double bcE[4], bcFx[4], bcFy[4];
    double bcEo[4];  // inflow sides: energy of the isotropic ghost outside the segment
    unsigned long long* stalls;  // count of pseudo-time stalls (device counter; may be null)
};

// A pseudo-time stall: a cell whose explicit sub-steps cannot move (tau* = 0: the state is on the boundary of
// the admissible set and the source points out of it), so its pseudo-time step leaves it unchanged.  Counted
// with one vector atomic (the address goes through a per-lane zero offset).
__device__ __forceinline__ void note_stall(unsigned long long* stalls)
{
    uint32_t z = 0;
    asm("" : "+v"(z));
    atomicAdd(stalls + z, 1ull);
}

// One grid level as seen by a kernel.  Cells are numbered k = j nx + i in
// 32 bits (a level holds at most 2^29 cells, so byte offsets fit too).
struct Lvl {
    int nx, ny;
    int sh;         // log2(nx) when nx is a power of two, else -1
    double kx, ky;  // dt / (2 hx), dt / (2 hy); ky = 0 in 1-D
    double a;       // 1 + c dt/hx + c dt/hy
    double cdt;     // c dt  (kappa = c dt sigma)
    const double* sa;
    const double* ss;
    int sg0[4], sg1[4];  // inflow sides: boundary cells sg0 <= along < sg1 take the wall state (else empty)
};

struct Soa {
    double* E;
    double* Fx;
    double* Fy;
    double* T;
};
struct CSoa {
    const double* E;
    const double* Fx;
    const double* Fy;
    const double* T;
};
__host__ __device__ inline CSoa cs(const Soa& s) { return CSoa{s.E, s.Fx, s.Fy, s.T}; }

// Field element k as the field's (wave-uniform) base plus a 32-bit byte
// offset: the scalar-base addressing form of the global loads and stores, one
// offset register shared by every field at the same cell.
__device__ __forceinline__ double ld(const double* p, uint32_t k)
{
    return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(p) + (k << 3));
}
__device__ __forceinline__ void st(double* p, uint32_t k, double x)
{
    *reinterpret_cast<double*>(reinterpret_cast<char*>(p) + (k << 3)) = x;
}

// (i, j) of cell k: shift and mask for power-of-two rows, else a 32-bit divide.
__device__ __forceinline__ void ij_of(int nx, int sh, uint32_t k, int& i, int& j)
{
    if (sh >= 0) {
        j = (int)(k >> sh);
        i = (int)(k & (uint32_t)(nx - 1));
    } else {
        const uint32_t q = k / (uint32_t)nx;
        j = (int)q;
        i = (int)(k - q * (uint32_t)nx);
    }
}

// Reciprocal and square root (x > 0) from the hardware approximations
// (relative error < 6e-8 on gfx950) with one Newton correction each: a few
// ulp (~4e-15 relative), at a fraction of the correctly rounded sequences'
// latency on a cell's dependent chain.
__device__ __forceinline__ double rcp_nr(double x)
{
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}
__device__ __forceinline__ double sqrt_nr(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double h = x * y;
    return fma(fma(-h, h, x), 0.5 * y, h);
}

// ---------------------------------------------------------------------------
// M1 closure (Sect. 2.1) arranged for the directional fluxes.  With
//   r = 1 / ((2 + s) E),  s = sqrt(4 - 3 f^2),  f = |F| / (cE),
// one has (1 - chi)/2 E = E/3 - (|F|^2/c^2) r and (3 chi - 1)/2 E n_i n_j =
// 3 r F_i F_j / c^2, so c^2 P_ij = (c^2 E/3 - |F|^2 r) delta_ij + 3 r F_i F_j
// and r = c / (2cE + sqrt(4 c^2 E^2 - 3 |F|^2)).  The radicand is clamped to
// c^2 E^2 (f <= 1) against rounding on the free-streaming boundary.
struct C2P {
    double iso;  // c^2 E/3 - |F|^2 r
    double r3;   // 3 r
};
__device__ __forceinline__ C2P closure(double c, double c2, double E, double Fx, double Fy)
{
    const double F2 = fma(Fx, Fx, Fy * Fy);
    const double c2E2 = c2 * E * E;
    const double root = sqrt_nr(fmax(fma(4.0, c2E2, -3.0 * F2), c2E2));
    const double r = c * rcp_nr(fma(2.0 * c, E, root));
    C2P o;
    o.iso = fma(-F2, r, c2 * E * (1.0 / 3.0));
    o.r3 = 3.0 * r;
    return o;
}

// The rows of c^2 P of a state: Gxx = c^2 Pxx, Gxy = c^2 Pxy, Gyy = c^2 Pyy.
__device__ __forceinline__ double p_xx(const C2P& p, double Fx) { return fma(p.r3 * Fx, Fx, p.iso); }
__device__ __forceinline__ double p_xy(const C2P& p, double Fx, double Fy) { return p.r3 * Fx * Fy; }
__device__ __forceinline__ double p_yy(const C2P& p, double Fy) { return fma(p.r3 * Fy, Fy, p.iso); }

// Add sgn-side x contribution of a neighbour whose c^2 P row is (Gxx, Gxy):
// sgn = +1 for L_x (left neighbour), -1 for R_x (right):
//   k (cE + sgn Fx,  c Fx + sgn c^2 Pxx,  c Fy + sgn c^2 Pxy)
__device__ __forceinline__ void acc_x(double k, double c, double sgn, double E, double Fx, double Fy, double Gxx,
                                      double Gxy, double& S0, double& S1, double& S2)
{
    S0 = fma(k, fma(sgn, Fx, c * E), S0);
    S1 = fma(k, fma(sgn, Gxx, c * Fx), S1);
    S2 = fma(k, fma(sgn, Gxy, c * Fy), S2);
}
// y contribution: k (cE + sgn Fy,  c Fx + sgn c^2 Pxy,  c Fy + sgn c^2 Pyy)
__device__ __forceinline__ void acc_y(double k, double c, double sgn, double E, double Fx, double Fy, double Gxy,
                                      double Gyy, double& S0, double& S1, double& S2)
{
    S0 = fma(k, fma(sgn, Fy, c * E), S0);
    S1 = fma(k, fma(sgn, Gxy, c * Fx), S1);
    S2 = fma(k, fma(sgn, Gyy, c * Fy), S2);
}
__device__ __forceinline__ void add_x(double k, double c, double c2, double sgn, double E, double Fx, double Fy,
                                      double& S0, double& S1, double& S2)
{
    const C2P p = closure(c, c2, E, Fx, Fy);
    acc_x(k, c, sgn, E, Fx, Fy, p_xx(p, Fx), p_xy(p, Fx, Fy), S0, S1, S2);
}
__device__ __forceinline__ void add_y(double k, double c, double c2, double sgn, double E, double Fx, double Fy,
                                      double& S0, double& S1, double& S2)
{
    const C2P p = closure(c, c2, E, Fx, Fy);
    acc_y(k, c, sgn, E, Fx, Fy, p_xy(p, Fx, Fy), p_yy(p, Fy), S0, S1, S2);
}

// ---------------------------------------------------------------------------
// Boundary rule of side `side` (0 x-, 1 x+, 2 y-, 3 y+) applied to the values
// loaded for that neighbour: inside the domain (or across a periodic side) they
// are the neighbour's own; at another side they were loaded from the cell
// itself and become its ghost (Neumann copy, reflective mirror of the normal
// flux, Dirichlet wall state; on an inflow side the wall state on the cells
// of its segment, `seg`, and the isotropic state (Eo, 0) elsewhere).  Exact arithmetic
// selects (x 1, x 0 of a finite value, x -1), so that callers can load
// unconditionally.
__device__ __forceinline__ bool is_ghost(const Phys& ph, int side, bool inside)
{
    return !inside && ph.bc[side] != BC_PERIODIC;
}
// Whether boundary cell number `along` (counted along side `side`) lies in the side's inflow segment.
template <class LV>
__device__ __forceinline__ bool in_seg(const LV& L, int side, int along)
{
    return along >= L.sg0[side] && along < L.sg1[side];
}
__device__ __forceinline__ void ghost_rule(const Phys& ph, int side, bool inside, bool seg, double le, double lfx,
                                           double lfy, double& e, double& fx, double& fy)
{
    const int kind = ph.bc[side];
    const bool ghost = is_ghost(ph, side, inside);
    const bool amb = ghost && kind == BC_INFLOW && !seg;
    const bool dir = ghost && (kind == BC_DIRICHLET || (kind == BC_INFLOW && seg));
    const bool flip = ghost && kind == BC_REFLECTIVE;
    const double keep = (dir || amb) ? 0.0 : 1.0;
    const double sx = (flip && side < 2) ? -keep : keep, sy = (flip && side >= 2) ? -keep : keep;
    e = fma(keep, le, dir ? ph.bcE[side] : (amb ? ph.bcEo[side] : 0.0));
    fx = fma(sx, lfx, dir ? ph.bcFx[side] : 0.0);
    fy = fma(sy, lfy, dir ? ph.bcFy[side] : 0.0);
}

// Neighbour state for side `side`: kn is the neighbour's index (the periodic
// wrap across a domain side), kc the cell's own.  The loads always happen, so
// the four neighbours' loads are in flight at once.
template <int DIM>
__device__ __forceinline__ void nb_state(const Phys& ph, int side, bool inside, bool seg, uint32_t kn, uint32_t kc,
                                         const CSoa& v, double& e, double& fx, double& fy)
{
    const uint32_t k = is_ghost(ph, side, inside) ? kc : kn;
    const double le = ld(v.E, k), lfx = ld(v.Fx, k), lfy = (DIM == 2) ? ld(v.Fy, k) : 0.0;
    ghost_rule(ph, side, inside, seg, le, lfx, lfy, e, fx, fy);
}

// Off-diagonal sum S = L_x(v_{i-1}) + R_x(v_{i+1}) [+ L_y(v_{j-1}) + R_y(v_{j+1})] of cell (i,j).
template <int DIM>
__device__ __forceinline__ void offdiag(const Phys& ph, const Lvl& L, const CSoa& v, int i, int j, uint32_t k,
                                        double& S0, double& S1, double& S2)
{
    double e, fx, fy;
    S0 = S1 = S2 = 0.0;
    const uint32_t wx = (uint32_t)(L.nx - 1);
    nb_state<DIM>(ph, 0, i > 0, in_seg(L, 0, j), i > 0 ? k - 1 : k + wx, k, v, e, fx, fy);
    add_x(L.kx, ph.c, ph.c2, +1.0, e, fx, fy, S0, S1, S2);
    nb_state<DIM>(ph, 1, i < L.nx - 1, in_seg(L, 1, j), i < L.nx - 1 ? k + 1 : k - wx, k, v, e, fx, fy);
    add_x(L.kx, ph.c, ph.c2, -1.0, e, fx, fy, S0, S1, S2);
    if (DIM == 2) {
        const uint32_t nx = (uint32_t)L.nx, wrap = (uint32_t)(L.ny - 1) * nx;
        nb_state<DIM>(ph, 2, j > 0, in_seg(L, 2, i), j > 0 ? k - nx : k + wrap, k, v, e, fx, fy);
        add_y(L.ky, ph.c, ph.c2, +1.0, e, fx, fy, S0, S1, S2);
        nb_state<DIM>(ph, 3, j < L.ny - 1, in_seg(L, 3, i), j < L.ny - 1 ? k + nx : k - wrap, k, v, e, fx, fy);
        add_y(L.ky, ph.c, ph.c2, -1.0, e, fx, fy, S0, S1, S2);
    }
}

// ---------------------------------------------------------------------------
// Local solve of one cell (the inverse of the diagonal block, sources included):
//   beta E  + gamma ((a + ka) E - ka a_r T^4)      = BE
//   beta F  + gamma (a + ka + ks) F                = BF
//   (beta + gamma) C_v T + gamma ka (a_r T^4 - E)  = BT
// E is eliminated; C_v' T + K T^4 = Q (convex, increasing) is solved by Newton
// from the previous temperature Tg, clamped to the upper bound of the root
// min(Q/C_v', (Q/K)^(1/4)) so that every iterate after the first lies above
// the root and the sequence decreases monotonically.
__device__ __forceinline__ void local_solve(double beta, double gamma, double a, double ka, double ks, double cv,
                                            double ar, double BE, double BFx, double BFy, double BT, double Tg,
                                            double& E, double& Fx, double& Fy, double& T)
{
    const double dE = fma(gamma, a + ka, beta);
    const double iF = rcp_nr(fma(gamma, ks, dE));
    Fx = BFx * iF;
    Fy = BFy * iF;
    const double k = gamma * ka;
    const double cT = (beta + gamma) * cv;
    const double idE = rcp_nr(dE);
    if (k == 0.0) {
        T = BT / cT;
        E = BE * idE;
        return;
    }
    const double K = k * ar * fma(gamma, a, beta) * idE;
    const double Q = fma(k * BE, idE, BT);
    // Newton on g(t) = K t^4 + cT t - Q (convex, increasing for t > 0) from the
    // guess Tg, clamped to an upper bound of the root, which is also the start
    // when Tg is not below it.  The root is below both Q / cT and (Q / K)^(1/4);
    // the bound takes them from the hardware reciprocal and reciprocal square
    // root (measured relative error below 6e-8 each on gfx950) raised by 2^-12,
    // which keeps it above the root, off the cell's dependent chain of exact
    // divisions and square roots.  Newton reaches the same root from any upper
    // bound; only the last bits of the stopping iterate may differ.
    const double Tup = (1.0 + 0x1p-12) * fmin(Q * __builtin_amdgcn_rcp(cT),
                                              __builtin_amdgcn_rsq(__builtin_amdgcn_rsq(Q * __builtin_amdgcn_rcp(K))));
    double t = (Tg > 0.0 && Tg < Tup) ? Tg : Tup;
    for (int it = 0; it < 64; ++it) {
        const double t2 = t * t;
        const double g = fma(K * t2, t2, fma(cT, t, -Q));
        const double dg = fma(4.0 * K * t2, t, cT);
        // the step uses the hardware reciprocal of g' unrefined: Newton corrects
        // its relative error (< 6e-8) in the next iterate and converges to the
        // same root, quadratically until that error dominates
        const double tn = fmin(fma(-g, __builtin_amdgcn_rcp(dg), t), Tup);
        // converged once a step is below 1e-7 of the iterate: near the root the
        // error after a step s is about (g'' / 2g') s^2 <= 1.5 s^2 / t, so the
        // returned iterate is within ~2e-14 relative of the root (one more
        // iterate would only confirm it)
        const bool done = fabs(tn - t) <= 1e-7 * tn;
        t = tn;
        if (done) break;
    }
    T = t;
    const double t2 = t * t;
    E = fma(k * ar * t2, t2, BE) * idE;
}

// ---------------------------------------------------------------------------
// Admissible length of the ray w + tau s (w admissible): the smallest of
// -E/sE, -T/sT and the first positive root of
//   q(tau) = c^2 (E + tau sE)^2 - |F + tau sF|^2 = A tau^2 + 2 B tau + C.
__device__ __forceinline__ double ray_len(double c2, double E, double Fx, double Fy, double T, double sE, double sFx,
                                          double sFy, double sT)
{
    double tau = INFINITY;
    if (sE < 0.0) tau = -E * rcp_nr(sE);
    if (sT < 0.0) tau = fmin(tau, -T * rcp_nr(sT));
    const double A = c2 * sE * sE - fma(sFx, sFx, sFy * sFy);
    const double B = c2 * E * sE - fma(Fx, sFx, Fy * sFy);
    const double C = fmax(c2 * E * E - fma(Fx, Fx, Fy * Fy), 0.0);
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

__device__ __forceinline__ bool admissible(double c2, double E, double Fx, double Fy, double T)
{
    return E > 0.0 && T > 0.0 && fma(Fx, Fx, Fy * Fy) <= c2 * E * E;
}

// Fine coordinate g on an axis of n cells: the cell read (src), whether the
// point is the ghost beyond a non-periodic side, whether it is used at all.
__device__ __forceinline__ void rc_axis(int g, int n, bool per, int& src, bool& ghost, bool& need)
{
    src = g;
    ghost = false;
    need = true;
    if (g >= 0 && g < n) return;
    if (per) {
        src = ((g % n) + n) % n;
    } else if (g == -1 || g == n) {
        src = g < 0 ? 0 : n - 1;
        ghost = true;
    } else {
        need = false;
    }
}

// XCD-aware block order: hardware hands consecutive blocks to the 8 XCDs round
// robin; remap so that each XCD walks one contiguous band of the grid and the
// stencil halo rows it needs stay in its own L2.
__device__ __forceinline__ int64_t xcd_block()
{
    const int64_t nb = gridDim.x, b = blockIdx.x;
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

}  // namespace m1
