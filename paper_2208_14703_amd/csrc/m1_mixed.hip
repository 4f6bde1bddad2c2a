// m1_mixed.hip -- kernels of the mixed-precision (FP32 delta-form) cycle.
//
// Per V-cycle on the finest level:
//   k_mx_resid   apply the pending FP32 correction to the FP64 state with the
//                FP64 admissibility projection, then r = b - A(v) in FP64 (the
//                stopping norm), FP32 copies of the new base state and of r;
//   k_mx_sweep   relaxed Jacobi sweeps on the correction d: D(v+d') - D(v) =
//                r + S(v+d) - S(v);
//   k_mx_apply   residual of the correction equation, rho = r - N_v(d);
//   k_mx_prolong_fine  d += P(e - d_c) with the admissibility test of v + d in FP64.
// Coarse levels carry a base w_l = R(w_{l-1}), a correction e_l and the
// right-hand side g_l = N_w(R d) + R(rho) of the FAS correction equation
// N_w(e) = g, smoothed by pseudo-time steps in increment form (k_mx_pseudo).
#include "m1_internal.hpp"
#include "m1_mixed.hpp"

namespace m1 {

constexpr int kBlock32 = 256;

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock32 - 1) / kBlock32); }

__device__ __forceinline__ bool mx_inactive(const int* active) { return active && *active == 0; }

__device__ __forceinline__ bool mx_cell(int nx, int ny, int64_t& k, int& i, int& j)
{
    k = xcd_block() * kBlock32 + threadIdx.x;
    if (k >= (int64_t)nx * ny) return false;
    j = (int)(k / nx);
    i = (int)(k - (int64_t)j * nx);
    return true;
}

// ---------------------------------------------------------------------------
// FP64 state update with admissibility projection: w = v + d where admissible,
// else v + eta min(tau*(v, d), 1) d.
template <int DIM>
__device__ __forceinline__ void upd64(const Phys& ph, double eta, const CSoa& v, const CSoa32& d, int64_t k,
                                      double& E, double& Fx, double& Fy, double& T)
{
    E = v.E[k];
    Fx = v.Fx[k];
    Fy = (DIM == 2) ? v.Fy[k] : 0.0;
    T = v.T[k];
    if (!d.E) return;
    const double e = d.E[k], gx = d.Fx[k], gy = (DIM == 2) ? (double)d.Fy[k] : 0.0, t = d.T[k];
    const double wE = E + e, wFx = Fx + gx, wFy = Fy + gy, wT = T + t;
    if (admissible(ph.c2, wE, wFx, wFy, wT)) {
        E = wE;
        Fx = wFx;
        Fy = wFy;
        T = wT;
        return;
    }
    const double th = eta * fmin(ray_len(ph.c2, E, Fx, Fy, T, e, gx, gy, t), 1.0);
    E = fma(th, e, E);
    Fx = fma(th, gx, Fx);
    Fy = fma(th, gy, Fy);
    T = fma(th, t, T);
}

template <int DIM>
__device__ __forceinline__ void nb_upd64(const Phys& ph, double eta, int side, bool inside, int64_t kn, int64_t kc,
                                         const CSoa& v, const CSoa32& d, double& E, double& Fx, double& Fy)
{
    const int kind = inside ? BC_PERIODIC : ph.bc[side];
    if (kind == BC_DIRICHLET) {
        E = ph.bcE[side];
        Fx = ph.bcFx[side];
        Fy = ph.bcFy[side];
        return;
    }
    double T;
    upd64<DIM>(ph, eta, v, d, kind == BC_PERIODIC ? kn : kc, E, Fx, Fy, T);
    if (kind == BC_REFLECTIVE) {
        if (side < 2) Fx = -Fx;
        else Fy = -Fy;
    }
}

// v_new = proj(v + d); r = b - A(v_new) (FP64); base32 = (float) v_new; r32 = (float) r;
// optional block partials of |r|^2.  v and v_new must not alias (neighbours read v).
template <int DIM>
__global__ __launch_bounds__(kBlock32) void k_mx_resid(Phys ph, Lvl L, double eta, CSoa v, CSoa32 d, CSoa b,
                                                       Soa vnew, Soa32 base, Soa32 r32, double* __restrict__ partials,
                                                       const int* __restrict__ active)
{
    if (mx_inactive(active)) return;
    __shared__ double red[kBlock32 / 64];
    int64_t k;
    int i, j;
    double q = 0.0;
    if (mx_cell(L.nx, L.ny, k, i, j)) {
        double S0 = 0.0, S1 = 0.0, S2 = 0.0, e, fx, fy;
        nb_upd64<DIM>(ph, eta, 0, i > 0, i > 0 ? k - 1 : k + (L.nx - 1), k, v, d, e, fx, fy);
        add_x(L.kx, ph.c, ph.c2, +1.0, e, fx, fy, S0, S1, S2);
        nb_upd64<DIM>(ph, eta, 1, i < L.nx - 1, i < L.nx - 1 ? k + 1 : k - (L.nx - 1), k, v, d, e, fx, fy);
        add_x(L.kx, ph.c, ph.c2, -1.0, e, fx, fy, S0, S1, S2);
        if (DIM == 2) {
            const int64_t nx = L.nx, wrap = (int64_t)(L.ny - 1) * nx;
            nb_upd64<DIM>(ph, eta, 2, j > 0, j > 0 ? k - nx : k + wrap, k, v, d, e, fx, fy);
            add_y(L.ky, ph.c, ph.c2, +1.0, e, fx, fy, S0, S1, S2);
            nb_upd64<DIM>(ph, eta, 3, j < L.ny - 1, j < L.ny - 1 ? k + nx : k - wrap, k, v, d, e, fx, fy);
            add_y(L.ky, ph.c, ph.c2, -1.0, e, fx, fy, S0, S1, S2);
        }
        double E, Fx, Fy, T;
        upd64<DIM>(ph, eta, v, d, k, E, Fx, Fy, T);
        const double ka = L.cdt * L.sa[k], ks = L.cdt * L.ss[k];
        const double T2 = T * T;
        const double ex = ka * fma(-ph.a_r * T2, T2, E);
        const double dF = L.a + ka + ks;
        const double rE = b.E[k] - (fma(L.a, E, ex) - S0);
        const double rFx = b.Fx[k] - fma(dF, Fx, -S1);
        const double rFy = (DIM == 2) ? b.Fy[k] - fma(dF, Fy, -S2) : 0.0;
        const double rT = b.T[k] - fma(ph.c_v, T, -ex);
        vnew.E[k] = E;
        vnew.Fx[k] = Fx;
        if (DIM == 2) vnew.Fy[k] = Fy;
        vnew.T[k] = T;
        base.E[k] = (float)E;
        base.Fx[k] = (float)Fx;
        if (DIM == 2) base.Fy[k] = (float)Fy;
        base.T[k] = (float)T;
        r32.E[k] = (float)rE;
        r32.Fx[k] = (float)rFx;
        if (DIM == 2) r32.Fy[k] = (float)rFy;
        r32.T[k] = (float)rT;
        const double ic = 1.0 / ph.c;
        q = fma(rE, rE, fma(rFx * ic, rFx * ic, fma(rFy * ic, rFy * ic, rT * rT)));
    }
    if (partials) {
        for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
        __syncthreads();
        if (threadIdx.x == 0) partials[xcd_block()] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// ---------------------------------------------------------------------------
// Relaxed Jacobi sweep on the correction (any level, beta M + gamma N = rhs):
//   x: (beta M + gamma (D(w + x) - D(w))) = rhs + gamma dS(d);  out = d + omega (x - d).
// d.E == nullptr means d = 0 (first sweep of a cycle: dS = 0, no reads of d).
template <int DIM>
__global__ __launch_bounds__(kBlock32) void k_mx_sweep(Phys ph, Lvl32 L, CSoa32 w, CSoa32 d, CSoa32 rhs, float beta,
                                                       float gamma, float omega, Soa32 out,
                                                       const int* __restrict__ active)
{
    if (mx_inactive(active)) return;
    int64_t k;
    int i, j;
    if (!mx_cell(L.nx, L.ny, k, i, j)) return;
    float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f;
    if (d.E) offdiag_inc<DIM>(ph, L, w, d, i, j, k, S0, S1, S2);
    const double QE = fmaf(gamma, S0, rhs.E[k]);
    const double QFx = fmaf(gamma, S1, rhs.Fx[k]);
    const double QFy = (DIM == 2) ? fmaf(gamma, S2, rhs.Fy[k]) : 0.0;
    const double QT = rhs.T[k];
    const float dE = d.E ? d.E[k] : 0.0f, dFx = d.E ? d.Fx[k] : 0.0f;
    const float dFy = (DIM == 2 && d.E) ? d.Fy[k] : 0.0f, dT = d.E ? d.T[k] : 0.0f;
    const double ka = (double)L.cdt * L.sa[k], ks = (double)L.cdt * L.ss[k];
    float xE, xFx, xFy, xT;
    local_solve_inc(beta, gamma, L.a, ka, ks, ph.c_v, ph.a_r, QE, QFx, QFy, QT, w.T[k], dT, xE, xFx, xFy, xT);
    out.E[k] = fmaf(omega, xE - dE, dE);
    out.Fx[k] = fmaf(omega, xFx - dFx, dFx);
    if (DIM == 2) out.Fy[k] = fmaf(omega, xFy - dFy, dFy);
    out.T[k] = fmaf(omega, xT - dT, dT);
}

// Increment of A for one cell: N(d) = (D(w + d) - D(w)) - dS(d).
template <int DIM>
__device__ __forceinline__ void n_inc(const Phys& ph, const Lvl32& L, const CSoa32& w, const CSoa32& d, int64_t k,
                                      int i, int j, float& NE, float& NFx, float& NFy, float& NT)
{
    float S0, S1, S2;
    offdiag_inc<DIM>(ph, L, w, d, i, j, k, S0, S1, S2);
    const double ka = (double)L.cdt * L.sa[k], ks = (double)L.cdt * L.ss[k];
    float DE, DFx, DFy, DT;
    diag_inc(L.a, ka, ks, ph.c_v, ph.a_r, w.T[k], d.E[k], d.Fx[k], (DIM == 2) ? d.Fy[k] : 0.0f, d.T[k], DE, DFx,
             DFy, DT);
    NE = DE - S0;
    NFx = DFx - S1;
    NFy = DFy - S2;
    NT = DT;
}

// out = X + sgn N(d).
template <int DIM>
__device__ __forceinline__ void mx_apply_cell(const Phys& ph, const Lvl32& L, const CSoa32& w, const CSoa32& d,
                                              const CSoa32& X, float sgn, const Soa32& out, int64_t k, int i, int j)
{
    float NE, NFx, NFy, NT;
    n_inc<DIM>(ph, L, w, d, k, i, j, NE, NFx, NFy, NT);
    out.E[k] = fmaf(sgn, NE, X.E[k]);
    out.Fx[k] = fmaf(sgn, NFx, X.Fx[k]);
    if (DIM == 2) out.Fy[k] = fmaf(sgn, NFy, X.Fy[k]);
    out.T[k] = fmaf(sgn, NT, X.T[k]);
}

template <int DIM>
__global__ __launch_bounds__(kBlock32) void k_mx_apply(Phys ph, Lvl32 L, CSoa32 w, CSoa32 d, CSoa32 X, float sgn,
                                                       Soa32 out, const int* __restrict__ active)
{
    if (mx_inactive(active)) return;
    int64_t k;
    int i, j;
    if (!mx_cell(L.nx, L.ny, k, i, j)) return;
    mx_apply_cell<DIM>(ph, L, w, d, X, sgn, out, k, i, j);
}

// One pseudo-time step of M de/dtau + N_w(e) = g (Algorithm 3 in increment
// form).  FIRST: e_in = d_l = R(correction above) and g holds R(rho) on entry;
// g = N_w(d_l) + R(rho) is formed and stored.
template <int DIM, bool FIRST>
__device__ __forceinline__ void mx_pseudo_cell(const Phys& ph, const Lvl32& L, const CSoa32& w, const Soa32& g,
                                               const CSoa32& e, const Soa32& out, float dt, float reach, int local,
                                               int64_t k, int i, int j)
{
    const float c2 = (float)ph.c2, cv = (float)ph.c_v;
    float S0, S1, S2;
    offdiag_inc<DIM>(ph, L, w, e, i, j, k, S0, S1, S2);
    const float eE = e.E[k], eFx = e.Fx[k], eFy = (DIM == 2) ? e.Fy[k] : 0.0f, eT = e.T[k];
    const float wE = w.E[k], wFx = w.Fx[k], wFy = (DIM == 2) ? w.Fy[k] : 0.0f, wT = w.T[k];
    const double ka = (double)L.cdt * L.sa[k], ks = (double)L.cdt * L.ss[k];
    float gE = g.E[k], gFx = g.Fx[k], gFy = (DIM == 2) ? g.Fy[k] : 0.0f, gT = g.T[k];
    if (FIRST) {
        float DE, DFx, DFy, DT;
        diag_inc(L.a, ka, ks, ph.c_v, ph.a_r, wT, eE, eFx, eFy, eT, DE, DFx, DFy, DT);
        gE += DE - S0;
        gFx += DFx - S1;
        gFy += DFy - S2;
        gT += DT;
        g.E[k] = gE;
        g.Fx[k] = gFx;
        if (DIM == 2) g.Fy[k] = gFy;
        g.T[k] = gT;
    }
    const float sT = gT * rcp32(cv);
    const float ts = ray_len32(c2, wE + eE, wFx + eFx, wFy + eFy, wT + eT, gE, gFx, gFy, sT);
    const float tau = fminf(dt, ts * reach);
    const float tE = fmaf(tau, gE, eE), tFx = fmaf(tau, gFx, eFx), tFy = fmaf(tau, gFy, eFy);
    const float tT = cv * fmaf(tau, sT, eT);
    const float gm = local ? tau : dt;
    float xE, xFx, xFy, xT;
    local_solve_inc(1.0, gm, L.a, ka, ks, ph.c_v, ph.a_r, fmaf(gm, S0, tE), fmaf(gm, S1, tFx), fmaf(gm, S2, tFy), tT,
                    wT, eT, xE, xFx, xFy, xT);
    out.E[k] = xE;
    out.Fx[k] = xFx;
    if (DIM == 2) out.Fy[k] = xFy;
    out.T[k] = xT;
}

template <int DIM>
__global__ __launch_bounds__(kBlock32) void k_mx_pseudo(Phys ph, Lvl32 L, CSoa32 w, Soa32 g, CSoa32 e, Soa32 out,
                                                        double dtau, const double* __restrict__ dtau_dev,
                                                        float reach, int local, int first,
                                                        const int* __restrict__ active)
{
    if (mx_inactive(active)) return;
    int64_t k;
    int i, j;
    if (!mx_cell(L.nx, L.ny, k, i, j)) return;
    const float dt = (float)(dtau_dev ? *dtau_dev : dtau);
    if (first) mx_pseudo_cell<DIM, true>(ph, L, w, g, e, out, dt, reach, local, k, i, j);
    else mx_pseudo_cell<DIM, false>(ph, L, w, g, e, out, dt, reach, local, k, i, j);
}

// ---------------------------------------------------------------------------
// Correction from the coarse level: x = e + P(ec - dc); admissibility of the
// state base + x (FP32 on coarse levels; FP64 on the finest level, where the
// base is the FP64 state v).  out may alias e.
__device__ __forceinline__ void pw32(int i, int nc, bool periodic, int idx[2], float w[2])
{
    const int I0 = i >> 1;
    idx[0] = idx[1] = I0;
    w[0] = 1.0f;
    w[1] = 0.0f;
    if ((i & 1) == 0) return;
    int I1 = I0 + 1;
    if (I1 >= nc) {
        if (!periodic) return;
        I1 -= nc;
    }
    idx[1] = I1;
    w[0] = w[1] = 0.5f;
}

template <int DIM>
__device__ __forceinline__ void coarse_corr(int nx, int ny, int px, int py, const CSoa32& ec, const CSoa32& dc,
                                            int64_t k, float& c0, float& c1, float& c2, float& c3)
{
    const int j = (int)(k / nx), i = (int)(k - (int64_t)j * nx);
    const int nxc = nx / 2, nyc = (DIM == 2) ? ny / 2 : 1;
    int ix[2], iy[2] = {0, 0};
    float wx[2], wy[2] = {1.0f, 0.0f};
    pw32(i, nxc, px != 0, ix, wx);
    if (DIM == 2) pw32(j, nyc, py != 0, iy, wy);
    constexpr int NB = (DIM == 2) ? 2 : 1;
    c0 = c1 = c2 = c3 = 0.0f;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int64_t kc = (int64_t)iy[b] * nxc + ix[a];
            const float wgt = wx[a] * wy[b];
            c0 = fmaf(wgt, ec.E[kc] - dc.E[kc], c0);
            c1 = fmaf(wgt, ec.Fx[kc] - dc.Fx[kc], c1);
            if (DIM == 2) c2 = fmaf(wgt, ec.Fy[kc] - dc.Fy[kc], c2);
            c3 = fmaf(wgt, ec.T[kc] - dc.T[kc], c3);
        }
}

template <int DIM>
__device__ __forceinline__ void mx_prolong_cell(const Phys& ph, int nx, int ny, int px, int py, float eta,
                                                const CSoa32& w, const CSoa32& e, const CSoa32& ec, const CSoa32& dc,
                                                const Soa32& out, int64_t k)
{
    float c0, c1, c2, c3;
    coarse_corr<DIM>(nx, ny, px, py, ec, dc, k, c0, c1, c2, c3);
    const float eE = e.E[k], eFx = e.Fx[k], eFy = (DIM == 2) ? e.Fy[k] : 0.0f, eT = e.T[k];
    const float sE = w.E[k] + eE, sFx = w.Fx[k] + eFx, sFy = ((DIM == 2) ? w.Fy[k] : 0.0f) + eFy, sT = w.T[k] + eT;
    float th = 1.0f;
    const float cc2 = (float)ph.c2;
    if (!admissible32(cc2, sE + c0, sFx + c1, sFy + c2, sT + c3))
        th = eta * fminf(ray_len32(cc2, sE, sFx, sFy, sT, c0, c1, c2, c3), 1.0f);
    out.E[k] = fmaf(th, c0, eE);
    out.Fx[k] = fmaf(th, c1, eFx);
    if (DIM == 2) out.Fy[k] = fmaf(th, c2, eFy);
    out.T[k] = fmaf(th, c3, eT);
}

template <int DIM>
__global__ __launch_bounds__(kBlock32) void k_mx_prolong(Phys ph, int nx, int ny, int px, int py, float eta, CSoa32 w,
                                                         CSoa32 e, CSoa32 ec, CSoa32 dc, Soa32 out,
                                                         const int* __restrict__ active)
{
    if (mx_inactive(active)) return;
    const int64_t k = xcd_block() * kBlock32 + threadIdx.x;
    if (k >= (int64_t)nx * ny) return;
    mx_prolong_cell<DIM>(ph, nx, ny, px, py, eta, w, e, ec, dc, out, k);
}

template <int DIM>
__global__ __launch_bounds__(kBlock32) void k_mx_prolong_fine(Phys ph, int nx, int ny, int px, int py, double eta,
                                                              CSoa v, CSoa32 e, CSoa32 ec, CSoa32 dc, Soa32 out,
                                                              const int* __restrict__ active)
{
    if (mx_inactive(active)) return;
    const int64_t k = xcd_block() * kBlock32 + threadIdx.x;
    if (k >= (int64_t)nx * ny) return;
    float c0, c1, c2, c3;
    coarse_corr<DIM>(nx, ny, px, py, ec, dc, k, c0, c1, c2, c3);
    const float eE = e.E[k], eFx = e.Fx[k], eFy = (DIM == 2) ? e.Fy[k] : 0.0f, eT = e.T[k];
    const double sE = v.E[k] + (double)eE, sFx = v.Fx[k] + (double)eFx;
    const double sFy = ((DIM == 2) ? v.Fy[k] : 0.0) + (double)eFy, sT = v.T[k] + (double)eT;
    double th = 1.0;
    if (!admissible(ph.c2, sE + c0, sFx + c1, sFy + c2, sT + c3))
        th = eta * fmin(ray_len(ph.c2, sE, sFx, sFy, sT, c0, c1, c2, c3), 1.0);
    out.E[k] = (float)fma(th, (double)c0, (double)eE);
    out.Fx[k] = (float)fma(th, (double)c1, (double)eFx);
    if (DIM == 2) out.Fy[k] = (float)fma(th, (double)c2, (double)eFy);
    out.T[k] = (float)fma(th, (double)c3, (double)eT);
}

// FP32 restriction of NF fields (base, correction, residual of a level) for
// coarse cell k: full weighting, all values gathered before the sums.
template <int DIM, int NF>
__device__ __forceinline__ void mx_restrict_cell(int nxf, int nyf, int px, int py, const float* const* in,
                                                 float* const* out, int64_t k)
{
    const int nxc = nxf / 2;
    const int J = (int)(k / nxc), I = (int)(k - (int64_t)J * nxc);
    int ix[3], iy[3] = {0, 0, 0};
    float wx[3], wy[3] = {1.0f, 0.0f, 0.0f};
    auto weights = [](int c, int nf, bool per, int* idx, float* w) {
        float sum = 0.0f;
        for (int m = 0; m < 3; ++m) {
            const float base = (m == 1) ? 0.5f : 0.25f;
            int f = 2 * c - 1 + m;
            float wm = base;
            if (f < 0 || f >= nf) {
                if (per) {
                    f = f < 0 ? f + nf : f - nf;
                } else {
                    f = f < 0 ? 0 : nf - 1;
                    wm = 0.0f;
                }
            }
            idx[m] = f;
            w[m] = wm;
            sum += wm;
        }
        if (sum != 1.0f)
            for (int m = 0; m < 3; ++m) w[m] /= sum;
    };
    weights(I, nxf, px != 0, ix, wx);
    if (DIM == 2) weights(J, nyf, py != 0, iy, wy);
    constexpr int NB = (DIM == 2) ? 3 : 1;
    uint32_t off[NB * 3];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) off[b * 3 + a] = (uint32_t)iy[b] * (uint32_t)nxf + (uint32_t)ix[a];
    float val[NF][NB * 3];
#pragma unroll
    for (int q = 0; q < NF; ++q)
#pragma unroll
        for (int m = 0; m < NB * 3; ++m) val[q][m] = in[q][off[m]];
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        float s = 0.0f;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const float t = fmaf(wx[2], val[q][b * 3 + 2], fmaf(wx[1], val[q][b * 3 + 1], wx[0] * val[q][b * 3]));
            s = fmaf(wy[b], t, s);
        }
        out[q][k] = s;
    }
}

template <int DIM, int NF>
__global__ __launch_bounds__(kBlock32) void k_mx_restrict(int nxf, int nyf, int px, int py, Fields32 F,
                                                          const int* __restrict__ active)
{
    if (mx_inactive(active)) return;
    const int64_t nc = (int64_t)(nxf / 2) * ((DIM == 2) ? nyf / 2 : 1);
    const int64_t k = xcd_block() * kBlock32 + threadIdx.x;
    if (k >= nc) return;
    mx_restrict_cell<DIM, NF>(nxf, nyf, px, py, F.in, F.out, k);
}

// ---------------------------------------------------------------------------
// Bottom of the mixed cycle in one workgroup: levels lt..L-1, entered with
// w_lt, d_lt and g_lt (= R(rho)) restricted; leaves e_lt (corrected, smoothed)
// in lev[lt].e.  Same per-cell bodies and order as the grid path.
template <int DIM>
__device__ __forceinline__ Soa32 mx_tail_pseudo(const TailArgs32& A, const TailLevel32& T, float dt, Soa32 in,
                                                bool first)
{
    const int64_t n = (int64_t)T.L.nx * T.L.ny;
    for (int m = 0; m < A.pseudo_steps; ++m) {
        const Soa32 out = (in.E == T.e.E) ? T.e2 : T.e;
        for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
            const int j = (int)(k / T.L.nx), i = (int)(k - (int64_t)j * T.L.nx);
            if (first && m == 0) mx_pseudo_cell<DIM, true>(A.ph, T.L, cs(T.w), T.g, cs(in), out, dt, A.reach, A.local, k, i, j);
            else mx_pseudo_cell<DIM, false>(A.ph, T.L, cs(T.w), T.g, cs(in), out, dt, A.reach, A.local, k, i, j);
        }
        __syncthreads();
        in = out;
    }
    return in;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_mx_tail(const TailArgs32* __restrict__ Ap, double dtau,
                                                  const double* __restrict__ dtau_dev, const int* __restrict__ active)
{
    if (mx_inactive(active)) return;
    const TailArgs32& A = *Ap;
    const float dt = (float)(dtau_dev ? *dtau_dev : dtau);
    unsigned in_e2 = 0;
    auto cur = [&](int l) { return ((in_e2 >> l) & 1u) ? A.lev[l].e2 : A.lev[l].e; };
    auto set = [&](int l, const Soa32& s) {
        if (s.E == A.lev[l].e2.E) in_e2 |= 1u << l;
        else in_e2 &= ~(1u << l);
    };
    for (int l = A.lt; l < A.L; ++l) {
        const TailLevel32& T = A.lev[l];
        const int64_t n = (int64_t)T.L.nx * T.L.ny;
        if (l > A.lt) {
            const TailLevel32& F = A.lev[l - 1];
            const Soa32 ef = cur(l - 1);
            const float* in[12] = {F.w.E, F.w.Fx, F.w.Fy, F.w.T, ef.E, ef.Fx, ef.Fy, ef.T, F.rho.E, F.rho.Fx, F.rho.Fy, F.rho.T};
            float* out[12] = {T.w.E, T.w.Fx, T.w.Fy, T.w.T, T.d.E, T.d.Fx, T.d.Fy, T.d.T, T.g.E, T.g.Fx, T.g.Fy, T.g.T};
            if (DIM == 1) {  // no Fy planes
                const int keep[9] = {0, 1, 3, 4, 5, 7, 8, 9, 11};
                for (int m = 0; m < 9; ++m) {
                    in[m] = in[keep[m]];
                    out[m] = out[keep[m]];
                }
            }
            for (int64_t k = threadIdx.x; k < n; k += blockDim.x)
                mx_restrict_cell<DIM, DIM == 2 ? 12 : 9>(F.L.nx, F.L.ny, A.px, A.py, in, out, k);
            __syncthreads();
        }
        set(l, mx_tail_pseudo<DIM>(A, T, dt, T.d, true));
        if (l < A.L - 1) {
            const Soa32 e = cur(l);
            for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
                const int j = (int)(k / T.L.nx), i = (int)(k - (int64_t)j * T.L.nx);
                mx_apply_cell<DIM>(A.ph, T.L, cs(T.w), cs(e), cs(T.g), -1.0f, T.rho, k, i, j);
            }
            __syncthreads();
        }
    }
    for (int l = A.L - 2; l >= A.lt; --l) {
        const TailLevel32& T = A.lev[l];
        const TailLevel32& C = A.lev[l + 1];
        const int64_t n = (int64_t)T.L.nx * T.L.ny;
        const Soa32 e = cur(l), ec = cur(l + 1);
        for (int64_t k = threadIdx.x; k < n; k += blockDim.x)
            mx_prolong_cell<DIM>(A.ph, T.L.nx, T.L.ny, A.px, A.py, (float)A.eta, cs(T.w), cs(e), cs(ec), cs(C.d), e, k);
        __syncthreads();
        set(l, mx_tail_pseudo<DIM>(A, T, dt, e, false));
    }
    const TailLevel32& T = A.lev[A.lt];
    const Soa32 res = cur(A.lt);
    if (res.E != T.e.E) {
        const int64_t n = (int64_t)T.L.nx * T.L.ny;
        for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
            T.e.E[k] = res.E[k];
            T.e.Fx[k] = res.Fx[k];
            if (DIM == 2) T.e.Fy[k] = res.Fy[k];
            T.e.T[k] = res.T[k];
        }
    }
}

__global__ __launch_bounds__(kBlock32) void k_to_f32(int64_t n, const double* __restrict__ a, float* __restrict__ b)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock32 + threadIdx.x;
    if (k < n) b[k] = (float)a[k];
}

// ===========================================================================
#define MX_DISPATCH(DIM_, KERNEL, GRID, ...)                                                            \
    do {                                                                                                \
        if ((DIM_) == 2) hipLaunchKernelGGL(KERNEL<2>, dim3(GRID), dim3(kBlock32), 0, st, __VA_ARGS__); \
        else hipLaunchKernelGGL(KERNEL<1>, dim3(GRID), dim3(kBlock32), 0, st, __VA_ARGS__);            \
    } while (0)

void launch_mx_resid(hipStream_t st, int dim, const Phys& ph, const Lvl& L, double eta, CSoa v, CSoa32 d, CSoa b,
                     Soa vnew, Soa32 base, Soa32 r32, double* partials, const int* active)
{
    MX_DISPATCH(dim, k_mx_resid, nblk((int64_t)L.nx * L.ny), ph, L, eta, v, d, b, vnew, base, r32, partials, active);
}

void launch_mx_sweep(hipStream_t st, int dim, const Phys& ph, const Lvl32& L, CSoa32 w, CSoa32 d, CSoa32 rhs,
                     float beta, float gamma, float omega, Soa32 out, const int* active)
{
    MX_DISPATCH(dim, k_mx_sweep, nblk((int64_t)L.nx * L.ny), ph, L, w, d, rhs, beta, gamma, omega, out, active);
}

void launch_mx_apply(hipStream_t st, int dim, const Phys& ph, const Lvl32& L, CSoa32 w, CSoa32 d, CSoa32 X, float sgn,
                     Soa32 out, const int* active)
{
    MX_DISPATCH(dim, k_mx_apply, nblk((int64_t)L.nx * L.ny), ph, L, w, d, X, sgn, out, active);
}

void launch_mx_pseudo(hipStream_t st, int dim, const Phys& ph, const Lvl32& L, CSoa32 w, Soa32 g, CSoa32 e,
                      Soa32 out, double dtau, const double* dtau_dev, float reach, int local, int first,
                      const int* active)
{
    MX_DISPATCH(dim, k_mx_pseudo, nblk((int64_t)L.nx * L.ny), ph, L, w, g, e, out, dtau, dtau_dev, reach, local,
                first, active);
}

void launch_mx_prolong(hipStream_t st, int dim, const Phys& ph, int nx, int ny, int px, int py, float eta, CSoa32 w,
                       CSoa32 e, CSoa32 ec, CSoa32 dc, Soa32 out, const int* active)
{
    MX_DISPATCH(dim, k_mx_prolong, nblk((int64_t)nx * ny), ph, nx, ny, px, py, eta, w, e, ec, dc, out, active);
}

void launch_mx_prolong_fine(hipStream_t st, int dim, const Phys& ph, int nx, int ny, int px, int py, double eta,
                            CSoa v, CSoa32 e, CSoa32 ec, CSoa32 dc, Soa32 out, const int* active)
{
    MX_DISPATCH(dim, k_mx_prolong_fine, nblk((int64_t)nx * ny), ph, nx, ny, px, py, eta, v, e, ec, dc, out, active);
}

void launch_mx_restrict(hipStream_t st, int dim, int nxf, int nyf, int px, int py, const Fields32& F,
                        const int* active)
{
    const int64_t nc = (int64_t)(nxf / 2) * (dim == 2 ? nyf / 2 : 1);
    const dim3 g(nblk(nc)), b(kBlock32);
    if (dim == 2) {
        if (F.n == 12) hipLaunchKernelGGL((k_mx_restrict<2, 12>), g, b, 0, st, nxf, nyf, px, py, F, active);
        else hipLaunchKernelGGL((k_mx_restrict<2, 2>), g, b, 0, st, nxf, nyf, px, py, F, active);
    } else {
        if (F.n == 9) hipLaunchKernelGGL((k_mx_restrict<1, 9>), g, b, 0, st, nxf, nyf, px, py, F, active);
        else hipLaunchKernelGGL((k_mx_restrict<1, 2>), g, b, 0, st, nxf, nyf, px, py, F, active);
    }
}

void launch_mx_tail(hipStream_t st, int dim, const TailArgs32* args_dev, double dtau, const double* dtau_dev,
                    const int* active)
{
    if (dim == 2) hipLaunchKernelGGL(k_mx_tail<2>, dim3(1), dim3(256), 0, st, args_dev, dtau, dtau_dev, active);
    else hipLaunchKernelGGL(k_mx_tail<1>, dim3(1), dim3(256), 0, st, args_dev, dtau, dtau_dev, active);
}

void launch_to_f32(hipStream_t st, int64_t n, const double* a, float* b)
{
    hipLaunchKernelGGL(k_to_f32, dim3(nblk(n)), dim3(kBlock32), 0, st, n, a, b);
}

}  // namespace m1
