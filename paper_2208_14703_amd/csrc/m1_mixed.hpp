// m1_mixed.hpp -- FP32 delta-form pieces of the mixed-precision solver.
//
// Mixed precision keeps the finest-level state v in FP64 and solves, once per
// V-cycle, for a correction d with the FP64 residual r = b - A(v) as data:
//   N_v(d) = A(v + d) - A(v) = r.
// Smoothing sweeps and every coarse level work in FP32 on corrections around
// FP32 copies of their base states.  N_v and all its pieces are evaluated in
// increment form, free of cancellation (every term is a product of a base value
// and a correction), so FP32 rounding scales with |d| and not with |v|; the
// outer FP64 defect correction then converges to the FP64 solution.  The gas
// temperature update (the increment of a_r T^4) is solved in FP64.
#pragma once

#include "m1_device.hpp"

namespace m1 {

struct Soa32 {
    float* E;
    float* Fx;
    float* Fy;
    float* T;
};
struct CSoa32 {
    const float* E;
    const float* Fx;
    const float* Fy;
    const float* T;
};
__host__ __device__ inline CSoa32 cs(const Soa32& s) { return CSoa32{s.E, s.Fx, s.Fy, s.T}; }

// FP32 field element k: base plus 32-bit byte offset (as ld/st for FP64).
__device__ __forceinline__ float ldf(const float* p, uint32_t k)
{
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(p) + (k << 2));
}
__device__ __forceinline__ void stf(float* p, uint32_t k, float x)
{
    *reinterpret_cast<float*>(reinterpret_cast<char*>(p) + (k << 2)) = x;
}

// One level in the FP32 path: spacing data as for FP64, opacities in FP32.
struct Lvl32 {
    int nx, ny;
    int sh;  // log2(nx) when nx is a power of two, else -1
    float kx, ky, a, cdt;
    const float* sa;
    const float* ss;
    int sg0[4], sg1[4];  // inflow segments, as in Lvl
};

// Increment of the closure, c^2 dP = c^2 (P(U + dU) - P(U)), for a base
// (E, Fx, Fy) and a correction (e, gx, gy).  With q = |F|^2,
// X = 4 c^2 E^2 - 3 q, den = 2cE + sqrt(X), r = c/den (so that
// c^2 P_ij = (c^2 E/3 - q r) delta_ij + 3 r F_i F_j):
//   dq = g.(2F + g),  dX = 4 c^2 e (2E + e) - 3 dq  (X' clamped to c^2 E'^2),
//   dsqrt = dX / (sqrt(X') + sqrt(X)),  dden = 2 c e + dsqrt,
//   dr = -r dden / den',  diso = c^2 e/3 - (dq r' + q dr),
//   d(r F_i F_j) = dr F'_i F'_j + r (g_i F'_j + F_i g_j).
struct DP {
    float xx, xy, yy;
};
// FP32 reciprocal and square root from the hardware instructions (about 1 ulp):
// FP32 is only used for corrections, whose relative accuracy this does not
// limit, and the correctly rounded sequences cost several times more.
__device__ __forceinline__ float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt32(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ DP closure_inc(float c, float c2, float E, float Fx, float Fy, float e, float gx, float gy)
{
    const float q = fmaf(Fx, Fx, Fy * Fy);
    const float dq = fmaf(gx, 2.0f * Fx + gx, gy * (2.0f * Fy + gy));
    const float c2E2 = c2 * E * E;
    const float X = fmaxf(fmaf(4.0f, c2E2, -3.0f * q), c2E2);
    const float m = fmaxf(c2E2 - q, 0.0f);
    const float ee = e * (2.0f * E + e);
    float dX = fmaf(4.0f * c2, ee, -3.0f * dq);
    dX = fmaxf(dX, fmaf(c2, ee, -3.0f * m));
    const float sX = sqrt32(X);
    const float sXn = sqrt32(fmaxf(X + dX, 0.0f));
    const float dsq = (sXn + sX) > 0.0f ? dX * rcp32(sXn + sX) : 0.0f;
    const float den = fmaf(2.0f * c, E, sX);
    const float dden = fmaf(2.0f * c, e, dsq);
    const float denn = den + dden;
    const float iden = rcp32(den), idenn = rcp32(denn);
    const float r = c * iden;
    const float rn = c * idenn;
    const float dr = -r * dden * idenn;
    const float diso = fmaf(c2 * (1.0f / 3.0f), e, -fmaf(dq, rn, q * dr));
    const float Fxn = Fx + gx, Fyn = Fy + gy;
    DP o;
    o.xx = fmaf(3.0f, fmaf(dr * Fxn, Fxn, r * gx * (Fxn + Fx)), diso);
    o.xy = 3.0f * fmaf(dr * Fxn, Fyn, r * fmaf(gx, Fyn, Fx * gy));
    o.yy = fmaf(3.0f, fmaf(dr * Fyn, Fyn, r * gy * (Fyn + Fy)), diso);
    return o;
}

// Add the sgn-side contribution of a neighbour with correction (e, gx, gy) and
// c^2 P increment p to the increment of the off-diagonal sum (x or y side).
__device__ __forceinline__ void acc_inc(float kk, float sgn, bool xdir, float c, float e, float gx, float gy,
                                        const DP& p, float& S0, float& S1, float& S2)
{
    const float G0 = xdir ? gx : gy;
    const float G1 = xdir ? p.xx : p.xy;
    const float G2 = xdir ? p.xy : p.yy;
    S0 = fmaf(kk, fmaf(sgn, G0, c * e), S0);
    S1 = fmaf(kk, fmaf(sgn, G1, c * gx), S1);
    S2 = fmaf(kk, fmaf(sgn, G2, c * gy), S2);
}

// The boundary rule of side `side` in increment form, applied to loaded values
// (identity inside the domain and across periodic sides).
__device__ __forceinline__ void ghost_inc(const Phys& ph, int side, bool inside, bool seg, float lE, float lFx,
                                          float lFy, float le, float lgx, float lgy, float& E, float& Fx, float& Fy,
                                          float& e, float& gx, float& gy)
{
    const int kind = ph.bc[side];
    const bool ghost = !inside && kind != BC_PERIODIC;
    const bool amb = ghost && kind == BC_INFLOW && !seg;
    const bool dir = ghost && (kind == BC_DIRICHLET || (kind == BC_INFLOW && seg));
    const bool flip = ghost && kind == BC_REFLECTIVE;
    const float keep = (dir || amb) ? 0.0f : 1.0f;
    const float sx = (flip && side < 2) ? -keep : keep, sy = (flip && side >= 2) ? -keep : keep;
    E = fmaf(keep, lE, dir ? (float)ph.bcE[side] : (amb ? (float)ph.bcEo[side] : 0.0f));
    Fx = fmaf(sx, lFx, dir ? (float)ph.bcFx[side] : 0.0f);
    Fy = fmaf(sy, lFy, dir ? (float)ph.bcFy[side] : 0.0f);
    e = keep * le;
    gx = sx * lgx;
    gy = sy * lgy;
}

// Ghost of a neighbour in increment form: the base ghost follows the boundary
// rule of the side; the correction ghost is its linear part (0 for Dirichlet).
// Branch-free like nb_state: unconditional loads, exact arithmetic selects.
template <int DIM>
__device__ __forceinline__ void nb_inc(const Phys& ph, int side, bool inside, bool seg, uint32_t kn, uint32_t kc,
                                       const CSoa32& w, const CSoa32& d, float& E, float& Fx, float& Fy, float& e,
                                       float& gx, float& gy)
{
    const bool ghost = !inside && ph.bc[side] != BC_PERIODIC;
    const uint32_t k = ghost ? kc : kn;
    const float lE = ldf(w.E, k), lFx = ldf(w.Fx, k), lFy = (DIM == 2) ? ldf(w.Fy, k) : 0.0f;
    const float le = ldf(d.E, k), lgx = ldf(d.Fx, k), lgy = (DIM == 2) ? ldf(d.Fy, k) : 0.0f;
    ghost_inc(ph, side, inside, seg, lE, lFx, lFy, le, lgx, lgy, E, Fx, Fy, e, gx, gy);
}


// Increment of the off-diagonal sum, dS = S(w + d) - S(w).
template <int DIM>
__device__ __forceinline__ void offdiag_inc(const Phys& ph, const Lvl32& L, const CSoa32& w, const CSoa32& d, int i,
                                            int j, uint32_t k, float& S0, float& S1, float& S2)
{
    const float c = (float)ph.c, c2 = (float)ph.c2;
    float E, Fx, Fy, e, gx, gy;
    S0 = S1 = S2 = 0.0f;
    auto add = [&](float kk, float sgn, bool xdir) {
        acc_inc(kk, sgn, xdir, c, e, gx, gy, closure_inc(c, c2, E, Fx, Fy, e, gx, gy), S0, S1, S2);
    };
    const uint32_t wx = (uint32_t)(L.nx - 1);
    nb_inc<DIM>(ph, 0, i > 0, in_seg(L, 0, j), i > 0 ? k - 1 : k + wx, k, w, d, E, Fx, Fy, e, gx, gy);
    add(L.kx, +1.0f, true);
    nb_inc<DIM>(ph, 1, i < L.nx - 1, in_seg(L, 1, j), i < L.nx - 1 ? k + 1 : k - wx, k, w, d, E, Fx, Fy, e, gx, gy);
    add(L.kx, -1.0f, true);
    if (DIM == 2) {
        const uint32_t nx = (uint32_t)L.nx, wrap = (uint32_t)(L.ny - 1) * nx;
        nb_inc<DIM>(ph, 2, j > 0, in_seg(L, 2, i), j > 0 ? k - nx : k + wrap, k, w, d, E, Fx, Fy, e, gx, gy);
        add(L.ky, +1.0f, false);
        nb_inc<DIM>(ph, 3, j < L.ny - 1, in_seg(L, 3, i), j < L.ny - 1 ? k + nx : k - wrap, k, w, d, E, Fx, Fy, e, gx, gy);
        add(L.ky, -1.0f, false);
    }
}

// (T + t)^4 - T^4 without cancellation, FP64.
__device__ __forceinline__ double quartic_inc(double T, double t)
{
    return t * fma(t, fma(t, 4.0 * T + t, 6.0 * T * T), 4.0 * T * T * T);
}

// Increment of the diagonal block: D(w + d) - D(w) for one cell (FP64 T^4 part).
__device__ __forceinline__ void diag_inc(double a, double ka, double ks, double cv, double ar, float T, float e,
                                         float gx, float gy, float t, float& DE, float& DFx, float& DFy, float& DT)
{
    const double q4 = ar * quartic_inc((double)T, (double)t);
    DE = (float)(fma(a + ka, (double)e, -ka * q4));
    const float dF = (float)(a + ka + ks);
    DFx = dF * gx;
    DFy = dF * gy;
    DT = (float)(fma(cv, (double)t, ka * (q4 - (double)e)));
}

// Local solve in increment form (FP64 inside):
//   beta x + gamma (D(w + x) - D(w)) = Q    with  M = diag(1,1,1,C_v) on the T row:
//   (beta + gamma (a + ka)) xE - gamma ka a_r dq4(xT)              = QE
//   (beta + gamma (a + ka + ks)) xF                                = QF
//   (beta + gamma) C_v xT + gamma ka (a_r dq4(xT) - xE)            = QT
// dq4(x) = (T + x)^4 - T^4; Newton on the convex increasing scalar equation in
// xT from the guess tg, clamped to an upper bound of the root.
__device__ __forceinline__ void local_solve_inc(double beta, double gamma, double a, double ka, double ks, double cv,
                                                double ar, double QE, double QFx, double QFy, double QT, double T,
                                                double tg, float& xE, float& xFx, float& xFy, float& xT)
{
    const double dE = fma(gamma, a + ka, beta);
    const double iF = rcp_nr(fma(gamma, ks, dE));
    xFx = (float)(QFx * iF);
    xFy = (float)(QFy * iF);
    const double k = gamma * ka;
    const double cT = (beta + gamma) * cv;
    const double idE = rcp_nr(dE);
    if (k == 0.0) {
        xT = (float)(QT / cT);
        xE = (float)(QE * idE);
        return;
    }
    const double K = k * ar * fma(gamma, a, beta) * idE;
    const double Q = fma(k * QE, idE, QT);
    // upper bound of the increment's root, min(Q / cT, (T^4 + Q / K)^(1/4) - T),
    // from the hardware reciprocal and reciprocal square root raised by 2^-12
    // (still above the root; as in local_solve)
    double up = 0.0;
    if (Q > 0.0) {
        const double T2 = T * T;
        constexpr double raise = 1.0 + 0x1p-12;
        const double r4 = __builtin_amdgcn_rsq(__builtin_amdgcn_rsq(fma(T2, T2, Q * __builtin_amdgcn_rcp(K))));
        up = fmin(raise * (Q * __builtin_amdgcn_rcp(cT)), raise * r4 - T);
    }
    double x = (tg < up && T + tg > 0.0) ? tg : up;
    for (int it = 0; it < 64; ++it) {
        const double Tx = T + x;
        const double g = fma(K, quartic_inc(T, x), fma(cT, x, -Q));
        const double dg = fma(4.0 * K * Tx * Tx, Tx, cT);
        const double xn = fmin(fma(-g, __builtin_amdgcn_rcp(dg), x), up);  // unrefined, as in local_solve
        // converged once the step is below 1e-7 of the increment or 1e-8 of T:
        // the error left after it is ~1.5 s^2 / (T + x), far below FP32 rounding
        const bool done = fabs(xn - x) <= 1e-7 * fmax(fabs(xn), 1e-30 * T) || fabs(xn - x) <= 1e-8 * T;
        x = xn;
        if (done) break;
    }
    xT = (float)x;
    xE = (float)(fma(k * ar, quartic_inc(T, x), QE) * idE);
}

__device__ __forceinline__ float ray_len32(float c2, float E, float Fx, float Fy, float T, float sE, float sFx,
                                           float sFy, float sT)
{
    float tau = INFINITY;
    if (sE < 0.0f) tau = -E / sE;
    if (sT < 0.0f) tau = fminf(tau, -T / sT);
    const float A = c2 * sE * sE - fmaf(sFx, sFx, sFy * sFy);
    const float B = c2 * E * sE - fmaf(Fx, sFx, Fy * sFy);
    const float C = fmaxf(c2 * E * E - fmaf(Fx, Fx, Fy * Fy), 0.0f);
    float r = INFINITY;
    if (A == 0.0f) {
        if (B < 0.0f) r = C / (-2.0f * B);
    } else {
        const float disc = B * B - A * C;
        if (disc >= 0.0f) {
            const float sq = sqrtf(disc);
            if (B < 0.0f) r = C / (sq - B);
            else if (A < 0.0f) r = (B + sq) / (-A);
        }
    }
    return fminf(tau, r);
}

__device__ __forceinline__ bool admissible32(float c2, float E, float Fx, float Fy, float T)
{
    return E > 0.0f && T > 0.0f && fmaf(Fx, Fx, Fy * Fy) <= c2 * E * E;
}

}  // namespace m1
