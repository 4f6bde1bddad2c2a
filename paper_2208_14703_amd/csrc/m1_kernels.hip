// m1_kernels.hip -- stencil kernels of the implicit M1 multigrid (gfx950).
//
// All kernels run one thread per cell (256-thread blocks = 4 wave64s) over a
// 1-D launch in the XCD-aware block order of m1::xcd_block(); cell (i,j) =
// (t % nx, t / nx).  Fields are SoA FP64 arrays.  The work is a memory-bound
// 5-point nonlinear stencil: no MFMA, no LDS staging in this version; the
// neighbour loads of a cell are served by L1/L2 (each cell value is fetched
// from HBM once per sweep and re-read from cache by its four neighbours).
#include "m1_internal.hpp"

namespace m1 {

constexpr int kBlock = 256;

static inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__device__ __forceinline__ bool cell_of(const Lvl& L, int64_t& k, int& i, int& j)
{
    k = xcd_block() * kBlock + threadIdx.x;
    const int64_t n = (int64_t)L.nx * L.ny;
    if (k >= n) return false;
    j = (int)(k / L.nx);
    i = (int)(k - (int64_t)j * L.nx);
    return true;
}

// ---------------------------------------------------------------------------
// Jacobi sweep of (beta M + gamma A)(u) = rhs, M = diag(1,1,1,C_v):
//   u_out = u_in + omega (local_solve(rhs + gamma S(u_in)) - u_in).
// gamma_cell (nullable) gives a per-cell gamma.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_relax(Phys ph, Lvl L, CSoa rhs, const double* __restrict__ gamma_cell,
                                                  double beta, double gamma, double omega, CSoa u, Soa out)
{
    int64_t k;
    int i, j;
    if (!cell_of(L, k, i, j)) return;
    double S0, S1, S2;
    offdiag<DIM>(ph, L, u, i, j, k, S0, S1, S2);
    const double g = gamma_cell ? gamma_cell[k] : gamma;
    const double BE = fma(g, S0, rhs.E[k]);
    const double BFx = fma(g, S1, rhs.Fx[k]);
    const double BFy = (DIM == 2) ? fma(g, S2, rhs.Fy[k]) : 0.0;
    const double ka = L.cdt * L.sa[k], ks = L.cdt * L.ss[k];
    const double Tin = u.T[k];
    double E, Fx, Fy, T;
    local_solve(beta, g, L.a, ka, ks, ph.c_v, ph.a_r, BE, BFx, BFy, rhs.T[k], Tin, E, Fx, Fy, T);
    if (omega != 1.0) {
        const double Ein = u.E[k], Fxin = u.Fx[k];
        E = fma(omega, E - Ein, Ein);
        Fx = fma(omega, Fx - Fxin, Fxin);
        if (DIM == 2) {
            const double Fyin = u.Fy[k];
            Fy = fma(omega, Fy - Fyin, Fyin);
        }
        T = fma(omega, T - Tin, Tin);
    }
    out.E[k] = E;
    out.Fx[k] = Fx;
    if (DIM == 2) out.Fy[k] = Fy;
    out.T[k] = T;
}

// ---------------------------------------------------------------------------
// One pseudo-time step (Algorithm 3) of M du/dtau + A(u) = f, fused:
//   s = M^{-1} f;  tau_i = min(dtau, tau*(u, s) (1 - (1-eta)^K))  (the pseudo
//   time reached by K explicit sub-steps, each eta of the remaining admissible
//   ray); u~ = u + tau_i s;  one Jacobi sweep of (M + g A)(u) = M u~ from u,
//   g = tau_i (local) or dtau.  With nu_l > 1 the rhs M u~ and g are stored for
//   the further sweeps (k_relax with gamma_cell).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_pseudo(Phys ph, Lvl L, CSoa f, CSoa u, Soa out, double dtau, double reach,
                                                   int local, Soa rhs_store, double* __restrict__ g_store)
{
    int64_t k;
    int i, j;
    if (!cell_of(L, k, i, j)) return;
    const double uE = u.E[k], uFx = u.Fx[k], uFy = (DIM == 2) ? u.Fy[k] : 0.0, uT = u.T[k];
    const double sE = f.E[k], sFx = f.Fx[k], sFy = (DIM == 2) ? f.Fy[k] : 0.0, sT = f.T[k] / ph.c_v;
    const double ts = ray_len(ph.c2, uE, uFx, uFy, uT, sE, sFx, sFy, sT);
    const double tau = fmin(dtau, ts * reach);
    const double tE = fma(tau, sE, uE), tFx = fma(tau, sFx, uFx), tFy = fma(tau, sFy, uFy);
    const double tT = ph.c_v * fma(tau, sT, uT);
    const double g = local ? tau : dtau;
    double S0, S1, S2;
    offdiag<DIM>(ph, L, u, i, j, k, S0, S1, S2);
    const double ka = L.cdt * L.sa[k], ks = L.cdt * L.ss[k];
    double E, Fx, Fy, T;
    local_solve(1.0, g, L.a, ka, ks, ph.c_v, ph.a_r, fma(g, S0, tE), fma(g, S1, tFx), fma(g, S2, tFy), tT, uT, E, Fx,
                Fy, T);
    out.E[k] = E;
    out.Fx[k] = Fx;
    if (DIM == 2) out.Fy[k] = Fy;
    out.T[k] = T;
    if (g_store) {
        rhs_store.E[k] = tE;
        rhs_store.Fx[k] = tFx;
        if (DIM == 2) rhs_store.Fy[k] = tFy;
        rhs_store.T[k] = tT;
        g_store[k] = g;
    }
}

// ---------------------------------------------------------------------------
// out = X + sgn A(v) (X nullable -> out = sgn A(v)); optionally stores out and
// writes per-block partial sums of r_E^2 + (r_F/c)^2 + r_T^2 for the norm.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_apply(Phys ph, Lvl L, CSoa v, CSoa X, double sgn, Soa out,
                                                  double* __restrict__ partials)
{
    __shared__ double red[kBlock / 64];
    int64_t k;
    int i, j;
    double q = 0.0;
    if (cell_of(L, k, i, j)) {
        double S0, S1, S2;
        offdiag<DIM>(ph, L, v, i, j, k, S0, S1, S2);
        const double E = v.E[k], Fx = v.Fx[k], Fy = (DIM == 2) ? v.Fy[k] : 0.0, T = v.T[k];
        const double ka = L.cdt * L.sa[k], ks = L.cdt * L.ss[k];
        const double T2 = T * T;
        const double ex = ka * fma(-ph.a_r * T2, T2, E);  // ka (E - a_r T^4)
        double aE = fma(L.a, E, ex) - S0;
        double aFx = fma(L.a + ka + ks, Fx, -S1);
        double aFy = fma(L.a + ka + ks, Fy, -S2);
        double aT = fma(ph.c_v, T, -ex);
        double rE = sgn * aE, rFx = sgn * aFx, rFy = sgn * aFy, rT = sgn * aT;
        if (X.E) {
            rE += X.E[k];
            rFx += X.Fx[k];
            if (DIM == 2) rFy += X.Fy[k];
            rT += X.T[k];
        }
        if (out.E) {
            out.E[k] = rE;
            out.Fx[k] = rFx;
            if (DIM == 2) out.Fy[k] = rFy;
            out.T[k] = rT;
        }
        const double ic = 1.0 / ph.c;
        const double fx = rFx * ic, fy = (DIM == 2) ? rFy * ic : 0.0;
        q = fma(rE, rE, fma(fx, fx, fma(fy, fy, rT * rT)));
    }
    if (partials) {
        // fixed-order block reduction: wave64 butterfly, then the 4 waves in order
        for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
        __syncthreads();
        if (threadIdx.x == 0) partials[xcd_block()] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// Sum of the partials in a fixed order by one block; writes sqrt to out[0].
__global__ __launch_bounds__(1024) void k_norm_finalize(const double* __restrict__ partials, int n,
                                                        double* __restrict__ out)
{
    __shared__ double red[16];
    double s = 0.0;
    for (int m = threadIdx.x; m < n; m += blockDim.x) s += partials[m];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        out[0] = sqrt(t);
    }
}

// ---------------------------------------------------------------------------
// Full-weighting restriction (weights 1/4, 1/2, 1/4 per axis) of up to 10
// fields from a fine level (nxf x nyf) to the coarse one.  Periodic axes wrap;
// otherwise points outside the domain are dropped and the weights renormalised.
__device__ __forceinline__ int rweights(int I, int nf, bool periodic, int idx[3], double w[3])
{
    int cnt = 0;
    double sum = 0.0;
    const double base[3] = {0.25, 0.5, 0.25};
    for (int m = 0; m < 3; ++m) {
        int f = 2 * I - 1 + m;
        if (f < 0 || f >= nf) {
            if (!periodic) continue;
            f = f < 0 ? f + nf : f - nf;
        }
        idx[cnt] = f;
        w[cnt] = base[m];
        sum += base[m];
        ++cnt;
    }
    if (sum != 1.0)
        for (int m = 0; m < cnt; ++m) w[m] /= sum;
    return cnt;
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_restrict(int nxf, int nyf, int px, int py, Fields F)
{
    const int nxc = nxf / 2, nyc = (DIM == 2) ? nyf / 2 : 1;
    const int64_t k = xcd_block() * kBlock + threadIdx.x;
    if (k >= (int64_t)nxc * nyc) return;
    const int J = (int)(k / nxc), I = (int)(k - (int64_t)J * nxc);
    int ix[3], iy[3];
    double wx[3], wy[3];
    const int cx = rweights(I, nxf, px != 0, ix, wx);
    int cy = 1;
    iy[0] = 0;
    wy[0] = 1.0;
    if (DIM == 2) cy = rweights(J, nyf, py != 0, iy, wy);
    for (int q = 0; q < F.n; ++q) {
        const double* __restrict__ src = F.in[q];
        double s = 0.0;
        for (int b = 0; b < cy; ++b) {
            double t = 0.0;
            const int64_t row = (int64_t)iy[b] * nxf;
            for (int a = 0; a < cx; ++a) t = fma(wx[a], src[row + ix[a]], t);
            s = fma(wy[b], t, s);
        }
        F.out[q][k] = s;
    }
}

// ---------------------------------------------------------------------------
// Correction from the coarse level with admissibility (eq. prolongatedSol):
//   e = P(uc - vc) (fine 2I <- coarse I, odd fine cells average two coarse
//   neighbours; periodic wrap, else the missing neighbour is dropped);
//   w = u + e; out = w if admissible, else u + eta min(tau*(u, w - u), 1) (w - u).
__device__ __forceinline__ int pweights(int i, int nc, bool periodic, int idx[2], double w[2])
{
    if ((i & 1) == 0) {
        idx[0] = i >> 1;
        w[0] = 1.0;
        return 1;
    }
    int I0 = (i - 1) >> 1, I1 = I0 + 1;
    if (I1 >= nc) {
        if (!periodic) {
            idx[0] = I0;
            w[0] = 1.0;
            return 1;
        }
        I1 -= nc;
    }
    idx[0] = I0;
    idx[1] = I1;
    w[0] = 0.5;
    w[1] = 0.5;
    return 2;
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_prolong_project(Phys ph, int nx, int ny, int px, int py, double eta, CSoa u,
                                                            CSoa uc, CSoa vc, Soa out)
{
    const int64_t k = xcd_block() * kBlock + threadIdx.x;
    if (k >= (int64_t)nx * ny) return;
    const int j = (int)(k / nx), i = (int)(k - (int64_t)j * nx);
    const int nxc = nx / 2, nyc = (DIM == 2) ? ny / 2 : 1;
    int ix[2], iy[2];
    double wx[2], wy[2];
    const int cx = pweights(i, nxc, px != 0, ix, wx);
    int cy = 1;
    iy[0] = 0;
    wy[0] = 1.0;
    if (DIM == 2) cy = pweights(j, nyc, py != 0, iy, wy);
    double e[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < cy; ++b)
        for (int a = 0; a < cx; ++a) {
            const int64_t kc = (int64_t)iy[b] * nxc + ix[a];
            const double w = wx[a] * wy[b];
            e[0] = fma(w, uc.E[kc] - vc.E[kc], e[0]);
            e[1] = fma(w, uc.Fx[kc] - vc.Fx[kc], e[1]);
            if (DIM == 2) e[2] = fma(w, uc.Fy[kc] - vc.Fy[kc], e[2]);
            e[3] = fma(w, uc.T[kc] - vc.T[kc], e[3]);
        }
    const double uE = u.E[k], uFx = u.Fx[k], uFy = (DIM == 2) ? u.Fy[k] : 0.0, uT = u.T[k];
    double wE = uE + e[0], wFx = uFx + e[1], wFy = uFy + e[2], wT = uT + e[3];
    if (!admissible(ph.c2, wE, wFx, wFy, wT)) {
        const double ts = fmin(ray_len(ph.c2, uE, uFx, uFy, uT, e[0], e[1], e[2], e[3]), 1.0);
        const double th = eta * ts;
        wE = fma(th, e[0], uE);
        wFx = fma(th, e[1], uFx);
        wFy = fma(th, e[2], uFy);
        wT = fma(th, e[3], uT);
    }
    out.E[k] = wE;
    out.Fx[k] = wFx;
    if (DIM == 2) out.Fy[k] = wFy;
    out.T[k] = wT;
}

// ---------------------------------------------------------------------------
// b = (E, Fx, Fy, C_v T) of the time step's initial state.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_make_rhs(int64_t n, double cv, CSoa v, Soa b)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    b.E[k] = v.E[k];
    b.Fx[k] = v.Fx[k];
    if (DIM == 2) b.Fy[k] = v.Fy[k];
    b.T[k] = cv * v.T[k];
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_copy(int64_t n, CSoa a, Soa b)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    b.E[k] = a.E[k];
    b.Fx[k] = a.Fx[k];
    if (DIM == 2) b.Fy[k] = a.Fy[k];
    b.T[k] = a.T[k];
}

// Index of the first cell that is not admissible (E > 0, T > 0, |F| <= cE (1 + 1e-12),
// all finite); *bad must hold INT64_MAX on entry.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_check_state(int64_t n, double c, CSoa v, unsigned long long* bad)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const double E = v.E[k], Fx = v.Fx[k], Fy = (DIM == 2) ? v.Fy[k] : 0.0, T = v.T[k];
    const bool ok = isfinite(E) && isfinite(Fx) && isfinite(Fy) && isfinite(T) && E > 0.0 && T > 0.0 &&
                    sqrt(fma(Fx, Fx, Fy * Fy)) <= c * E * (1.0 + 1e-12);
    if (!ok) atomicMin(bad, (unsigned long long)k);
}

// Index of the first opacity that is negative or not finite.
__global__ __launch_bounds__(kBlock) void k_check_sigma(int64_t n, const double* __restrict__ sa,
                                                        const double* __restrict__ ss, unsigned long long* bad)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const double a = sa[k], s = ss[k];
    if (!(isfinite(a) && isfinite(s) && a >= 0.0 && s >= 0.0)) atomicMin(bad, (unsigned long long)k);
}

// ===========================================================================
// Launchers
// ===========================================================================
#define M1_DISPATCH(DIM_, KERNEL, GRID, ...)                                                       \
    do {                                                                                           \
        if ((DIM_) == 2) hipLaunchKernelGGL(KERNEL<2>, dim3(GRID), dim3(kBlock), 0, st, __VA_ARGS__); \
        else hipLaunchKernelGGL(KERNEL<1>, dim3(GRID), dim3(kBlock), 0, st, __VA_ARGS__);         \
    } while (0)

void launch_relax(hipStream_t st, int dim, const Phys& ph, const Lvl& L, CSoa rhs, const double* gamma_cell,
                  double beta, double gamma, double omega, CSoa u, Soa out)
{
    M1_DISPATCH(dim, k_relax, nblocks((int64_t)L.nx * L.ny), ph, L, rhs, gamma_cell, beta, gamma, omega, u, out);
}

void launch_pseudo(hipStream_t st, int dim, const Phys& ph, const Lvl& L, CSoa f, CSoa u, Soa out, double dtau,
                   double reach, int local, Soa rhs_store, double* g_store)
{
    M1_DISPATCH(dim, k_pseudo, nblocks((int64_t)L.nx * L.ny), ph, L, f, u, out, dtau, reach, local, rhs_store,
                g_store);
}

unsigned apply_blocks(const Lvl& L) { return nblocks((int64_t)L.nx * L.ny); }

void launch_apply(hipStream_t st, int dim, const Phys& ph, const Lvl& L, CSoa v, CSoa X, double sgn, Soa out,
                  double* partials)
{
    M1_DISPATCH(dim, k_apply, apply_blocks(L), ph, L, v, X, sgn, out, partials);
}

void launch_norm_finalize(hipStream_t st, const double* partials, int n, double* out)
{
    hipLaunchKernelGGL(k_norm_finalize, dim3(1), dim3(1024), 0, st, partials, n, out);
}

void launch_restrict(hipStream_t st, int dim, int nxf, int nyf, int px, int py, const Fields& F)
{
    const int64_t nc = (int64_t)(nxf / 2) * (dim == 2 ? nyf / 2 : 1);
    M1_DISPATCH(dim, k_restrict, nblocks(nc), nxf, nyf, px, py, F);
}

void launch_prolong_project(hipStream_t st, int dim, const Phys& ph, int nx, int ny, int px, int py, double eta,
                            CSoa u, CSoa uc, CSoa vc, Soa out)
{
    M1_DISPATCH(dim, k_prolong_project, nblocks((int64_t)nx * ny), ph, nx, ny, px, py, eta, u, uc, vc, out);
}

void launch_make_rhs(hipStream_t st, int dim, int64_t n, double cv, CSoa v, Soa b)
{
    M1_DISPATCH(dim, k_make_rhs, nblocks(n), n, cv, v, b);
}

void launch_copy(hipStream_t st, int dim, int64_t n, CSoa a, Soa b) { M1_DISPATCH(dim, k_copy, nblocks(n), n, a, b); }

void launch_check_state(hipStream_t st, int dim, int64_t n, double c, CSoa v, unsigned long long* bad)
{
    M1_DISPATCH(dim, k_check_state, nblocks(n), n, c, v, bad);
}

void launch_check_sigma(hipStream_t st, int64_t n, const double* sa, const double* ss, unsigned long long* bad)
{
    hipLaunchKernelGGL(k_check_sigma, dim3(nblocks(n)), dim3(kBlock), 0, st, n, sa, ss, bad);
}

}  // namespace m1
