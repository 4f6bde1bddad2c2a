// m1_cells.hpp -- per-cell bodies of the FP64 cycle operations, shared by the
// single-problem grid kernels (m1_kernels.hip) and the batched kernels
// (same file), plus the body of the single-workgroup tail.
#pragma once

#include "m1_internal.hpp"

namespace m1 {

// ===========================================================================
// Per-cell bodies
// ===========================================================================

// Jacobi sweep of (beta M + gamma A)(u) = rhs, M = diag(1,1,1,C_v):
//   out = u + omega (local_solve(rhs + gamma S(u)) - u);  gcell: per-cell gamma.
// With NORM (only for the finest-level sweep, beta = 0, gamma = 1) the cell's
// share of |b - A(u)|^2 of the INPUT u is returned: b - A(u) = B - D(u), where
// B = b + S(u) is formed for the update anyway.
// The update of relax_cell from the cell's off-diagonal sum S and its own
// state: u.T is Tin, the other components come from cen(0..2) (E, Fx, Fy),
// called only where needed.  relax_values returns the new state, relax_update
// stores it at k of out.  Shared by every form of the sweep.
template <int DIM, bool NORM, class Cen>
__device__ __forceinline__ double relax_values(const Phys& ph, const Lvl& L, const CSoa& rhs, double g, double beta,
                                               double omega, double S0, double S1, double S2, double Tin, Cen cen,
                                               uint32_t k, double& E, double& Fx, double& Fy, double& T)
{
    const double BE = fma(g, S0, ld(rhs.E, k));
    const double BFx = fma(g, S1, ld(rhs.Fx, k));
    const double BFy = (DIM == 2) ? fma(g, S2, ld(rhs.Fy, k)) : 0.0;
    const double BT = ld(rhs.T, k);
    const double ka = L.cdt * ld(L.sa, k), ks = L.cdt * ld(L.ss, k);
    double q = 0.0;
    if (NORM) {
        const double Ein = cen(0), Fxin = cen(1), Fyin = (DIM == 2) ? cen(2) : 0.0;
        const double T2 = Tin * Tin;
        const double ex = ka * fma(-ph.a_r * T2, T2, Ein);  // ka (E - a_r T^4)
        const double dF = L.a + ka + ks;
        const double rE = BE - fma(L.a, Ein, ex);
        const double ic = 1.0 / ph.c;
        const double rFx = (BFx - dF * Fxin) * ic, rFy = (BFy - dF * Fyin) * ic;
        const double rT = BT - fma(ph.c_v, Tin, -ex);
        q = fma(rE, rE, fma(rFx, rFx, fma(rFy, rFy, rT * rT)));
    }
    local_solve(beta, g, L.a, ka, ks, ph.c_v, ph.a_r, BE, BFx, BFy, BT, Tin, E, Fx, Fy, T);
    if (omega != 1.0) {
        const double Ein = cen(0), Fxin = cen(1);
        E = fma(omega, E - Ein, Ein);
        Fx = fma(omega, Fx - Fxin, Fxin);
        if (DIM == 2) {
            const double Fyin = cen(2);
            Fy = fma(omega, Fy - Fyin, Fyin);
        }
        T = fma(omega, T - Tin, Tin);
    }
    return q;
}

template <int DIM, bool NORM, class Cen>
__device__ __forceinline__ double relax_update(const Phys& ph, const Lvl& L, const CSoa& rhs, double g, double beta,
                                               double omega, double S0, double S1, double S2, double Tin, Cen cen,
                                               const Soa& out, uint32_t k)
{
    double E, Fx, Fy, T;
    const double q = relax_values<DIM, NORM>(ph, L, rhs, g, beta, omega, S0, S1, S2, Tin, cen, k, E, Fx, Fy, T);
    st(out.E, k, E);
    st(out.Fx, k, Fx);
    if (DIM == 2) st(out.Fy, k, Fy);
    st(out.T, k, T);
    return q;
}

template <int DIM, bool NORM = false>
__device__ __forceinline__ double relax_cell(const Phys& ph, const Lvl& L, const CSoa& rhs, const double* gcell,
                                             double beta, double gamma, double omega, const CSoa& u, const Soa& out,
                                             uint32_t k, int i, int j)
{
    double S0, S1, S2;
    offdiag<DIM>(ph, L, u, i, j, k, S0, S1, S2);
    const double g = gcell ? ld(gcell, k) : gamma;
    const double Tin = ld(u.T, k);
    auto cen = [&](int f) { return ld(f == 0 ? u.E : (f == 1 ? u.Fx : u.Fy), k); };
    return relax_update<DIM, NORM>(ph, L, rhs, g, beta, omega, S0, S1, S2, Tin, cen, out, k);
}

// One pseudo-time step (Algorithm 3) of M du/dtau + A(u) = f, fused:
//   s = M^{-1} f;  tau_i = min(dtau, tau*(u, s) (1 - (1-eta)^K)) -- the pseudo
//   time reached by K explicit sub-steps, each eta of the remaining admissible
//   ray;  u~ = u + tau_i s;  one Jacobi sweep of (M + g A)(u) = M u~ from u,
//   with g = tau_i (local) or dtau.  rs/gs (nullable) keep M u~ and g for
//   further sweeps.  With FIRST (the first step of the pre-smoothing, u = v_l)
//   f holds the restricted residual on entry and the FAS right-hand side
//   f = A(v_l) + R(rbar) is formed here and written back (A(v) = D(v) - S(v),
//   S(v) being needed for the sweep anyway).
// The arithmetic of one pseudo-time step for one cell, from its values: u,
// the off-diagonal sum S(u), kappa_a/s, and f (with FIRST: R(rbar) on entry,
// the FAS right-hand side on return).  Returns the new u and, for further
// sweeps, M u~ (t) and g.
template <int DIM, bool FIRST>
__device__ __forceinline__ void pseudo_core(const Phys& ph, const Lvl& L, double uE, double uFx, double uFy, double uT,
                                            double S0, double S1, double S2, double ka, double ks, double& fE,
                                            double& fFx, double& fFy, double& fT, double dtau, double reach,
                                            int local, double& E, double& Fx, double& Fy, double& T, double& tE,
                                            double& tFx, double& tFy, double& tT, double& g, bool& stall)
{
    if (FIRST) {
        const double T2 = uT * uT;
        const double ex = ka * fma(-ph.a_r * T2, T2, uE);
        const double dF = L.a + ka + ks;
        fE += fma(L.a, uE, ex) - S0;
        fFx += fma(dF, uFx, -S1);
        fFy += fma(dF, uFy, -S2);
        fT += fma(ph.c_v, uT, -ex);
    }
    const double sE = fE, sFx = fFx, sFy = fFy, sT = fT * rcp_nr(ph.c_v);
    const double ts = ray_len(ph.c2, uE, uFx, uFy, uT, sE, sFx, sFy, sT);
    stall = ts == 0.0;
    const double tau = fmin(dtau, ts * reach);
    tE = fma(tau, sE, uE);
    tFx = fma(tau, sFx, uFx);
    tFy = fma(tau, sFy, uFy);
    tT = ph.c_v * fma(tau, sT, uT);
    g = local ? tau : dtau;
    local_solve(1.0, g, L.a, ka, ks, ph.c_v, ph.a_r, fma(g, S0, tE), fma(g, S1, tFx), fma(g, S2, tFy), tT, uT, E, Fx,
                Fy, T);
}

// The rest of a pseudo-time step of one cell from its state and its
// off-diagonal sum S: stores (gated on `live`) the new state, with FIRST the
// FAS right-hand side, and with gs the values further sweeps need.
template <int DIM, bool FIRST>
__device__ __forceinline__ void pseudo_update(const Phys& ph, const Lvl& L, const CSoa& fin, const Soa& fout,
                                              double uE, double uFx, double uFy, double uT, double S0, double S1,
                                              double S2, const Soa& out, double dtau, double reach, int local,
                                              const Soa& rs, double* gs, uint32_t k, bool live)
{
    const double ka = L.cdt * ld(L.sa, k), ks = L.cdt * ld(L.ss, k);
    double fE = ld(fin.E, k), fFx = ld(fin.Fx, k), fFy = (DIM == 2) ? ld(fin.Fy, k) : 0.0, fT = ld(fin.T, k);
    double E, Fx, Fy, T, tE, tFx, tFy, tT, g;
    bool stall;
    pseudo_core<DIM, FIRST>(ph, L, uE, uFx, uFy, uT, S0, S1, S2, ka, ks, fE, fFx, fFy, fT, dtau, reach, local, E, Fx,
                            Fy, T, tE, tFx, tFy, tT, g, stall);
    if (!live) return;
    if (stall && ph.stalls) note_stall(ph.stalls);
    if (FIRST) {
        st(fout.E, k, fE);
        st(fout.Fx, k, fFx);
        if (DIM == 2) st(fout.Fy, k, fFy);
        st(fout.T, k, fT);
    }
    st(out.E, k, E);
    st(out.Fx, k, Fx);
    if (DIM == 2) st(out.Fy, k, Fy);
    st(out.T, k, T);
    if (gs) {
        st(rs.E, k, tE);
        st(rs.Fx, k, tFx);
        if (DIM == 2) st(rs.Fy, k, tFy);
        st(rs.T, k, tT);
        st(gs, k, g);
    }
}

template <int DIM, bool FIRST = false>
__device__ __forceinline__ void pseudo_cell(const Phys& ph, const Lvl& L, const CSoa& fin, const Soa& fout,
                                            const CSoa& u, const Soa& out, double dtau, double reach, int local,
                                            const Soa& rs, double* gs, uint32_t k, int i, int j, bool live = true)
{
    const double uE = ld(u.E, k), uFx = ld(u.Fx, k), uFy = (DIM == 2) ? ld(u.Fy, k) : 0.0, uT = ld(u.T, k);
    double S0, S1, S2;
    offdiag<DIM>(ph, L, u, i, j, k, S0, S1, S2);
    pseudo_update<DIM, FIRST>(ph, L, fin, fout, uE, uFx, uFy, uT, S0, S1, S2, out, dtau, reach, local, rs, gs, k,
                              live);
}

// out = X + sgn A(v) (X.E == nullptr: out = sgn A(v)); out stored when out.E
// is set.  Returns r_E^2 + (r_F/c)^2 + r_T^2 of the result (norm contribution).
// X + sgn A(v) of one cell from its state and off-diagonal sum S (X.E null: sgn A(v)).
// The same from the cell's opacities (sa, ss) and X (x: null when X.E is null), loaded by the caller.
template <int DIM>
__device__ __forceinline__ void apply_values_from(const Phys& ph, const Lvl& L, double E, double Fx, double Fy,
                                                  double T, double S0, double S1, double S2, double sa, double ss,
                                                  const double* x, double sgn, double& rE, double& rFx, double& rFy,
                                                  double& rT)
{
    const double ka = L.cdt * sa, ks = L.cdt * ss;
    const double T2 = T * T;
    const double ex = ka * fma(-ph.a_r * T2, T2, E);  // ka (E - a_r T^4)
    const double dF = L.a + ka + ks;
    rE = sgn * (fma(L.a, E, ex) - S0);
    rFx = sgn * fma(dF, Fx, -S1);
    rFy = sgn * fma(dF, Fy, -S2);
    rT = sgn * fma(ph.c_v, T, -ex);
    if (x) {
        rE += x[0];
        rFx += x[1];
        if (DIM == 2) rFy += x[2];
        rT += x[3];
    }
}

template <int DIM>
__device__ __forceinline__ void apply_values(const Phys& ph, const Lvl& L, double E, double Fx, double Fy, double T,
                                             double S0, double S1, double S2, const CSoa& X, double sgn, uint32_t k,
                                             double& rE, double& rFx, double& rFy, double& rT)
{
    double x[4] = {0.0, 0.0, 0.0, 0.0};
    if (X.E) {
        x[0] = ld(X.E, k);
        x[1] = ld(X.Fx, k);
        if (DIM == 2) x[2] = ld(X.Fy, k);
        x[3] = ld(X.T, k);
    }
    apply_values_from<DIM>(ph, L, E, Fx, Fy, T, S0, S1, S2, ld(L.sa, k), ld(L.ss, k), X.E ? x : nullptr, sgn, rE, rFx,
                           rFy, rT);
}

// The rest of apply_cell from the cell's state and off-diagonal sum S.
template <int DIM>
__device__ __forceinline__ double apply_update(const Phys& ph, const Lvl& L, double E, double Fx, double Fy, double T,
                                               double S0, double S1, double S2, const CSoa& X, double sgn,
                                               const Soa& out, uint32_t k, bool live)
{
    double rE, rFx, rFy, rT;
    apply_values<DIM>(ph, L, E, Fx, Fy, T, S0, S1, S2, X, sgn, k, rE, rFx, rFy, rT);
    if (out.E && live) {
        st(out.E, k, rE);
        st(out.Fx, k, rFx);
        if (DIM == 2) st(out.Fy, k, rFy);
        st(out.T, k, rT);
    }
    const double ic = 1.0 / ph.c;
    const double fx = rFx * ic, fy = (DIM == 2) ? rFy * ic : 0.0;
    return fma(rE, rE, fma(fx, fx, fma(fy, fy, rT * rT)));
}

template <int DIM>
__device__ __forceinline__ double apply_cell(const Phys& ph, const Lvl& L, const CSoa& v, const CSoa& X, double sgn,
                                             const Soa& out, uint32_t k, int i, int j, bool live = true)
{
    double S0, S1, S2;
    offdiag<DIM>(ph, L, v, i, j, k, S0, S1, S2);
    const double E = ld(v.E, k), Fx = ld(v.Fx, k), Fy = (DIM == 2) ? ld(v.Fy, k) : 0.0, T = ld(v.T, k);
    return apply_update<DIM>(ph, L, E, Fx, Fy, T, S0, S1, S2, X, sgn, out, k, live);
}

// Full-weighting weights along one axis (1/4, 1/2, 1/4 on fine 2I-1, 2I, 2I+1):
// periodic axes wrap, otherwise outside points get weight 0 (index clamped to a
// valid cell) and the others are renormalised to sum 1.  Always 3 entries so
// that every load is issued unconditionally.
__device__ __forceinline__ void rweights(int I, int nf, bool periodic, int idx[3], double w[3])
{
    double sum = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const double base = (m == 1) ? 0.5 : 0.25;
        int f = 2 * I - 1 + m;
        double wm = base;
        if (f < 0 || f >= nf) {
            if (periodic) {
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

// Restriction of NF fields for coarse cell k.  All 3x3 x NF values are
// gathered first (32-bit offsets from the per-field bases) so that every load
// is in flight before the first use, then summed.
template <int DIM, int NF>
__device__ __forceinline__ void restrict_cell(int nxf, int nyf, int shf, int px, int py, const double* const* in,
                                              double* const* out, uint32_t k, bool live = true)
{
    const int nxc = nxf / 2;
    int I, J;
    ij_of(nxc, shf > 0 ? shf - 1 : -1, k, I, J);
    int ix[3], iy[3] = {0, 0, 0};
    double wx[3], wy[3] = {1.0, 0.0, 0.0};
    rweights(I, nxf, px != 0, ix, wx);
    if (DIM == 2) rweights(J, nyf, py != 0, iy, wy);
    constexpr int NB = (DIM == 2) ? 3 : 1;
    uint32_t off[NB * 3];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) off[b * 3 + a] = (uint32_t)iy[b] * (uint32_t)nxf + (uint32_t)ix[a];
    double val[NF][NB * 3];
#pragma unroll
    for (int q = 0; q < NF; ++q)
#pragma unroll
        for (int m = 0; m < NB * 3; ++m) val[q][m] = ld(in[q], off[m]);
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const double t = fma(wx[2], val[q][b * 3 + 2], fma(wx[1], val[q][b * 3 + 1], wx[0] * val[q][b * 3]));
            s = fma(wy[b], t, s);
        }
        if (live) st(out[q], k, s);
    }
}

// Linear prolongation weights along one axis: fine 2I <- coarse I; odd fine
// cells average coarse I and I+1 (periodic wrap, else the missing one gets
// weight 0 and the other 1).  Always 2 entries.
__device__ __forceinline__ void pweights(int i, int nc, bool periodic, int idx[2], double w[2])
{
    const int I0 = i >> 1;
    idx[0] = I0;
    if ((i & 1) == 0) {
        idx[1] = I0;
        w[0] = 1.0;
        w[1] = 0.0;
        return;
    }
    int I1 = I0 + 1;
    if (I1 >= nc) {
        if (!periodic) {
            idx[1] = I0;
            w[0] = 1.0;
            w[1] = 0.0;
            return;
        }
        I1 -= nc;
    }
    idx[1] = I1;
    w[0] = 0.5;
    w[1] = 0.5;
}

// Correction with admissibility (eq. prolongatedSol) of fine cell (i, j) with
// state u:  w = u + P(uc - vc); w if admissible, else
// u + eta min(tau*(u, w - u), 1) (w - u).
template <int DIM>
__device__ __forceinline__ void prolong_value(const Phys& ph, int nx, int ny, int px, int py, double eta, int i, int j,
                                              double uE, double uFx, double uFy, double uT, const CSoa& uc,
                                              const CSoa& vc, double& wE, double& wFx, double& wFy, double& wT)
{
    const int nxc = nx / 2, nyc = (DIM == 2) ? ny / 2 : 1;
    int ix[2], iy[2] = {0, 0};
    double wx[2], wy[2] = {1.0, 0.0};
    pweights(i, nxc, px != 0, ix, wx);
    if (DIM == 2) pweights(j, nyc, py != 0, iy, wy);
    constexpr int NB = (DIM == 2) ? 2 : 1;
    double e0 = 0.0, e1 = 0.0, e2 = 0.0, e3 = 0.0;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const uint32_t kc = (uint32_t)iy[b] * (uint32_t)nxc + (uint32_t)ix[a];
            const double w = wx[a] * wy[b];
            e0 = fma(w, ld(uc.E, kc) - ld(vc.E, kc), e0);
            e1 = fma(w, ld(uc.Fx, kc) - ld(vc.Fx, kc), e1);
            if (DIM == 2) e2 = fma(w, ld(uc.Fy, kc) - ld(vc.Fy, kc), e2);
            e3 = fma(w, ld(uc.T, kc) - ld(vc.T, kc), e3);
        }
    }
    wE = uE + e0;
    wFx = uFx + e1;
    wFy = uFy + e2;
    wT = uT + e3;
    if (!admissible(ph.c2, wE, wFx, wFy, wT)) {
        const double th = eta * fmin(ray_len(ph.c2, uE, uFx, uFy, uT, e0, e1, e2, e3), 1.0);
        wE = fma(th, e0, uE);
        wFx = fma(th, e1, uFx);
        wFy = fma(th, e2, uFy);
        wT = fma(th, e3, uT);
    }
}

// prolong_value of a fine cell (i, j) of a level of nx x ny cells whose coarse
// corrections uc - vc are staged: c?[(Jc - Jc0) cw + Ic - Ic0] for the coarse
// cells it reads, none of them across a side (no wrap, no clamp).  The same
// weights, differences and order as prolong_value, so the same result.
__device__ __forceinline__ void prolong_value_staged(const Phys& ph, int nx, int ny, double eta, int i, int j,
                                                     double uE, double uFx, double uFy, double uT, const double* cE,
                                                     const double* cFx, const double* cFy, const double* cT, int Ic0,
                                                     int Jc0, int cw, double& wE, double& wFx, double& wFy,
                                                     double& wT)
{
    int ix[2], iy[2];
    double wx[2], wy[2];
    pweights(i, nx / 2, false, ix, wx);
    pweights(j, ny / 2, false, iy, wy);
    double e0 = 0.0, e1 = 0.0, e2 = 0.0, e3 = 0.0;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int c = (iy[b] - Jc0) * cw + ix[a] - Ic0;
            const double w = wx[a] * wy[b];
            e0 = fma(w, cE[c], e0);
            e1 = fma(w, cFx[c], e1);
            e2 = fma(w, cFy[c], e2);
            e3 = fma(w, cT[c], e3);
        }
    }
    wE = uE + e0;
    wFx = uFx + e1;
    wFy = uFy + e2;
    wT = uT + e3;
    if (!admissible(ph.c2, wE, wFx, wFy, wT)) {
        const double th = eta * fmin(ray_len(ph.c2, uE, uFx, uFy, uT, e0, e1, e2, e3), 1.0);
        wE = fma(th, e0, uE);
        wFx = fma(th, e1, uFx);
        wFy = fma(th, e2, uFy);
        wT = fma(th, e3, uT);
    }
}

template <int DIM>
__device__ __forceinline__ void prolong_cell(const Phys& ph, int nx, int ny, int sh, int px, int py, double eta,
                                             const CSoa& u, const CSoa& uc, const CSoa& vc, const Soa& out, uint32_t k,
                                             bool live = true)
{
    int i, j;
    ij_of(nx, sh, k, i, j);
    const double uE = ld(u.E, k), uFx = ld(u.Fx, k), uFy = (DIM == 2) ? ld(u.Fy, k) : 0.0, uT = ld(u.T, k);
    double wE, wFx, wFy, wT;
    prolong_value<DIM>(ph, nx, ny, px, py, eta, i, j, uE, uFx, uFy, uT, uc, vc, wE, wFx, wFy, wT);
    if (!live) return;
    st(out.E, k, wE);
    st(out.Fx, k, wFx);
    if (DIM == 2) st(out.Fy, k, wFy);
    st(out.T, k, wT);
}


// Cycle control update of one time step from the residual norm r (one thread):
// the first call records r0; later calls adapt dtau (x1.1 above eps_inc,
// /2 below eps_dec) and stop on rtol, the rounding floor or max_cycles.
__device__ __forceinline__ void ctrl_update(Ctrl* ctrl, double r)
{
    if (ctrl->cycles < 0) {  // first call of a time step: the residual of v^n itself, no adaptation
        ctrl->cycles = 0;
        ctrl->r0 = r;
        ctrl->rprev = r;
        ctrl->rel = 1.0;
        if (r <= ctrl->floor_r) {
            ctrl->conv = 1;
            ctrl->active = 0;
        }
        return;
    }
    ctrl->cycles += 1;
    const double rel = r / ctrl->r0;
    ctrl->rel = rel;
    const double d = ctrl->literal ? fabs(r - ctrl->rprev) / ctrl->r0 : (ctrl->rprev - r) / ctrl->rprev;
    double dt = ctrl->dtau;
    if (d > ctrl->eps_inc) dt *= 1.1;
    if (d < ctrl->eps_dec) dt *= 0.5;
    ctrl->dtau = fmin(fmax(dt, ctrl->dtau_min), ctrl->dtau_max);
    ctrl->rprev = r;
    if (rel <= ctrl->rtol || r <= ctrl->floor_r) {
        ctrl->conv = 1;
        ctrl->active = 0;
    } else if (!isfinite(rel) || ctrl->cycles >= ctrl->max_cycles) {
        ctrl->active = 0;
    }
}

// Fixed-order sum over a block of n partial values (any block size <= 1024).
__device__ __forceinline__ double block_sum(const double* __restrict__ partials, int n)
{
    __shared__ double red_sum[16];
    double s = 0.0;
    for (int m = threadIdx.x; m < n; m += blockDim.x) s += partials[m];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red_sum[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red_sum[w];
    __syncthreads();
    return t;
}

// Fixed-order reduction of q over a 256-thread block into *dst (thread 0).
__device__ __forceinline__ void block_partial(double q, double* dst)
{
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) *dst = (red[0] + red[1]) + (red[2] + red[3]);
}
// ---------------------------------------------------------------------------
// Bottom of the V-cycle in one workgroup: levels lt..L-1 (all small), entered
// with v_lt = R(u_{lt-1}) and f_lt = R(rbar_{lt-1}) already in place; leaves
// the smoothed, corrected u_lt in lev[lt].u.  Same per-cell bodies and the same
// order of operations as the grid path, with __syncthreads between phases.
template <int DIM>
__device__ __forceinline__ Soa tail_pseudo(const TailArgs& A, const TailLevel& T, double dtau, Soa in, bool first)
{
    const uint32_t n = (uint32_t)T.L.nx * (uint32_t)T.L.ny;
    for (int m = 0; m < A.pseudo_steps; ++m) {
        const Soa out = (in.E == T.u.E) ? T.u2 : T.u;
        for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) {
            int i, j;
            ij_of(T.L.nx, T.L.sh, k, i, j);
            if (first && m == 0)
                pseudo_cell<DIM, true>(A.ph, T.L, cs(T.f), T.f, cs(in), out, dtau, A.reach, A.local, Soa{}, nullptr,
                                       k, i, j);
            else
                pseudo_cell<DIM, false>(A.ph, T.L, cs(T.f), T.f, cs(in), out, dtau, A.reach, A.local, Soa{},
                                        nullptr, k, i, j);
        }
        __syncthreads();
        in = out;
    }
    return in;
}

template <int DIM>
__device__ __forceinline__ void tail_body(const TailArgs& A, double dt)
{
    unsigned in_u2 = 0;  // bit l set: the current iterate of level l is in u2 (else u)
    auto cur = [&](int l) { return ((in_u2 >> l) & 1u) ? A.lev[l].u2 : A.lev[l].u; };
    auto set = [&](int l, const Soa& s) {
        if (s.E == A.lev[l].u2.E) in_u2 |= 1u << l;
        else in_u2 &= ~(1u << l);
    };
    for (int l = A.lt; l < A.L; ++l) {
        const TailLevel& T = A.lev[l];
        const uint32_t n = (uint32_t)T.L.nx * (uint32_t)T.L.ny;
        if (l > A.lt) {
            const TailLevel& F = A.lev[l - 1];
            const Soa uf = cur(l - 1);
            const double* in[8] = {uf.E, uf.Fx, uf.Fy, uf.T, F.rb.E, F.rb.Fx, F.rb.Fy, F.rb.T};
            double* out[8] = {T.v.E, T.v.Fx, T.v.Fy, T.v.T, T.f.E, T.f.Fx, T.f.Fy, T.f.T};
            if (DIM == 1) {  // no Fy planes: (E, Fx, T) of u then of rbar
                in[2] = in[3];
                in[3] = in[4];
                in[4] = in[5];
                in[5] = in[7];
                out[2] = out[3];
                out[3] = out[4];
                out[4] = out[5];
                out[5] = out[7];
            }
            for (uint32_t k = threadIdx.x; k < n; k += blockDim.x)
                restrict_cell<DIM, DIM == 2 ? 8 : 6>(F.L.nx, F.L.ny, F.L.sh, A.px, A.py, in, out, k);
            __syncthreads();
        }
        set(l, tail_pseudo<DIM>(A, T, dt, T.v, true));  // forms f = A(v) + R(rbar) on the way
        if (l < A.L - 1) {
            const Soa u = cur(l);
            for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) {  // rbar = f - A(u)
                int i, j;
                ij_of(T.L.nx, T.L.sh, k, i, j);
                apply_cell<DIM>(A.ph, T.L, cs(u), cs(T.f), -1.0, T.rb, k, i, j);
            }
            __syncthreads();
        }
    }
    for (int l = A.L - 2; l >= A.lt; --l) {
        const TailLevel& T = A.lev[l];
        const TailLevel& C = A.lev[l + 1];
        const uint32_t n = (uint32_t)T.L.nx * (uint32_t)T.L.ny;
        const Soa u = cur(l), uc = cur(l + 1);
        for (uint32_t k = threadIdx.x; k < n; k += blockDim.x)
            prolong_cell<DIM>(A.ph, T.L.nx, T.L.ny, T.L.sh, A.px, A.py, A.eta, cs(u), cs(uc), cs(C.v), u, k);
        __syncthreads();
        set(l, tail_pseudo<DIM>(A, T, dt, u, false));
    }
    const TailLevel& T = A.lev[A.lt];
    const Soa res = cur(A.lt);
    if (res.E != T.u.E) {
        const uint32_t n = (uint32_t)T.L.nx * (uint32_t)T.L.ny;
        for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) {
            st(T.u.E, k, ld(res.E, k));
            st(T.u.Fx, k, ld(res.Fx, k));
            if (DIM == 2) st(T.u.Fy, k, ld(res.Fy, k));
            st(T.u.T, k, ld(res.T, k));
        }
    }
}


}  // namespace m1
