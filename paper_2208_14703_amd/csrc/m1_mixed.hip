// m1_mixed.hip -- kernels of the mixed-precision (FP32 delta-form) cycle.
//
// Per V-cycle on the finest level:
//   k_mx_resid   apply the pending FP32 correction to the FP64 state with the
//                FP64 admissibility projection, then r = b - A(v) in FP64 (the
//                stopping norm), FP32 copies of the new base state and of r,
//                and the cycle's first correction sweep (from d = 0, purely
//                local);
//   k_mx_sweep   relaxed Jacobi sweeps on the correction d: D(v+d') - D(v) =
//                r + S(v+d) - S(v) (LDS-staged form k_mx_sweep_lds; two
//                consecutive sweeps per launch: k_mx_sweep2_lds);
//   k_mx_residual_restrict  residual of the correction equation,
//                rho = r - N_v(d), restricted with v and d to level 1 as it is
//                formed (k_mx_apply + k_mx_restrict when switched off);
//   k_mx_prolong_fine  d += P(e - d_c) with the admissibility test of v + d in FP64
//                (when the sweeps are staged, fused with the first post-smoothing
//                sweep: k_mx_prolong_sweep_lds).
// Coarse levels carry a base w_l = R(w_{l-1}), a correction e_l and the
// right-hand side g_l = N_w(R d) + R(rho) of the FAS correction equation
// N_w(e) = g, smoothed by pseudo-time steps in increment form (k_mx_pseudo;
// LDS-staged on large levels: k_mx_pseudo_lds).
#include "m1_internal.hpp"
#include "m1_mixed.hpp"

namespace m1 {

constexpr int kBlock32 = 256;

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock32 - 1) / kBlock32); }

// Finest-level kernels (resid, sweep) exit at once when the stop flag is 0;
// coarse-level kernels read it with their data and gate only their stores
// (see the FP64 kernels).  `active` and `dtau_dev` are valid device pointers.
__device__ __forceinline__ uint32_t mx_lane_zero()
{
    uint32_t z = 0;
    asm("" : "+v"(z));
    return z;
}

__device__ __forceinline__ bool mx_cell(int nx, int ny, int sh, uint32_t& k, int& i, int& j)
{
    k = (uint32_t)xcd_block() * kBlock32 + threadIdx.x;
    if (k >= (uint32_t)nx * (uint32_t)ny) return false;
    ij_of(nx, sh, k, i, j);
    return true;
}

// ---------------------------------------------------------------------------
// FP64 state update with admissibility projection: w = v + d where admissible,
// else v + eta min(tau*(v, d), 1) d.
template <int DIM>
__device__ __forceinline__ void upd64(const Phys& ph, double eta, const CSoa& v, const CSoa32& d, uint32_t k,
                                      double& E, double& Fx, double& Fy, double& T)
{
    E = ld(v.E, k);
    Fx = ld(v.Fx, k);
    Fy = (DIM == 2) ? ld(v.Fy, k) : 0.0;
    T = ld(v.T, k);
    if (!d.E) return;
    const double e = ldf(d.E, k), gx = ldf(d.Fx, k), gy = (DIM == 2) ? (double)ldf(d.Fy, k) : 0.0, t = ldf(d.T, k);
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
__device__ __forceinline__ void nb_upd64(const Phys& ph, double eta, int side, bool inside, bool seg, uint32_t kn,
                                         uint32_t kc, const CSoa& v, const CSoa32& d, double& E, double& Fx, double& Fy)
{
    double lE, lFx, lFy, T;
    upd64<DIM>(ph, eta, v, d, is_ghost(ph, side, inside) ? kc : kn, lE, lFx, lFy, T);
    ghost_rule(ph, side, inside, seg, lE, lFx, lFy, E, Fx, Fy);
}

// Relaxed Jacobi update of the correction at one cell from its values: off-diagonal sums S, current
// correction d, right-hand side r, FP32 opacities and base temperature.
template <int DIM>
__device__ __forceinline__ void mx_sweep_point(const Phys& ph, const Lvl32& L, float beta, float gamma, float omega,
                                               float S0, float S1, float S2, float dE, float dFx, float dFy, float dT,
                                               float rE, float rFx, float rFy, float rT, float sa, float ss, float wT,
                                               float& oE, float& oFx, float& oFy, float& oT)
{
    const double QE = fmaf(gamma, S0, rE);
    const double QFx = fmaf(gamma, S1, rFx);
    const double QFy = (DIM == 2) ? fmaf(gamma, S2, rFy) : 0.0;
    const double QT = rT;
    const double ka = (double)L.cdt * sa, ks = (double)L.cdt * ss;
    float xE, xFx, xFy, xT;
    local_solve_inc(beta, gamma, L.a, ka, ks, ph.c_v, ph.a_r, QE, QFx, QFy, QT, wT, dT, xE, xFx, xFy, xT);
    oE = fmaf(omega, xE - dE, dE);
    oFx = fmaf(omega, xFx - dFx, dFx);
    oFy = (DIM == 2) ? fmaf(omega, xFy - dFy, dFy) : 0.0f;
    oT = fmaf(omega, xT - dT, dT);
}

// The first correction sweep of a cycle starts from d = 0: each cell needs only its own base temperature,
// residual and opacities, which mx_resid_cell has in hand (as the FP32 values it stores, those the sweep would
// read).  With z.d.E set, mx_resid_cell runs that sweep too and stores its result in z.d.
struct MxZero {
    Lvl32 L;
    float omega;
    Soa32 d;
};

// v_new = proj(v + d); r = b - A(v_new) (FP64); base32 = (float) v_new; r32 = (float) r.
// Returns the cell's share of |r|^2.  v and v_new must not alias (neighbours read v).
template <int DIM>
__device__ __forceinline__ double mx_resid_cell(const Phys& ph, const Lvl& L, double eta, const CSoa& v,
                                                const CSoa32& d, const CSoa& b, const Soa& vnew, const Soa32& base,
                                                const Soa32& r32, uint32_t k, int i, int j, const MxZero& z = {})
{
    double S0 = 0.0, S1 = 0.0, S2 = 0.0, e, fx, fy;
    const uint32_t wx = (uint32_t)(L.nx - 1);
    nb_upd64<DIM>(ph, eta, 0, i > 0, in_seg(L, 0, j), i > 0 ? k - 1 : k + wx, k, v, d, e, fx, fy);
    add_x(L.kx, ph.c, ph.c2, +1.0, e, fx, fy, S0, S1, S2);
    nb_upd64<DIM>(ph, eta, 1, i < L.nx - 1, in_seg(L, 1, j), i < L.nx - 1 ? k + 1 : k - wx, k, v, d, e, fx, fy);
    add_x(L.kx, ph.c, ph.c2, -1.0, e, fx, fy, S0, S1, S2);
    if (DIM == 2) {
        const uint32_t nx = (uint32_t)L.nx, wrap = (uint32_t)(L.ny - 1) * nx;
        nb_upd64<DIM>(ph, eta, 2, j > 0, in_seg(L, 2, i), j > 0 ? k - nx : k + wrap, k, v, d, e, fx, fy);
        add_y(L.ky, ph.c, ph.c2, +1.0, e, fx, fy, S0, S1, S2);
        nb_upd64<DIM>(ph, eta, 3, j < L.ny - 1, in_seg(L, 3, i), j < L.ny - 1 ? k + nx : k - wrap, k, v, d, e, fx, fy);
        add_y(L.ky, ph.c, ph.c2, -1.0, e, fx, fy, S0, S1, S2);
    }
    double E, Fx, Fy, T;
    upd64<DIM>(ph, eta, v, d, k, E, Fx, Fy, T);
    const double sa = ld(L.sa, k), ss = ld(L.ss, k);
    const double ka = L.cdt * sa, ks = L.cdt * ss;
    const double T2 = T * T;
    const double ex = ka * fma(-ph.a_r * T2, T2, E);
    const double dF = L.a + ka + ks;
    const double rE = ld(b.E, k) - (fma(L.a, E, ex) - S0);
    const double rFx = ld(b.Fx, k) - fma(dF, Fx, -S1);
    const double rFy = (DIM == 2) ? ld(b.Fy, k) - fma(dF, Fy, -S2) : 0.0;
    const double rT = ld(b.T, k) - fma(ph.c_v, T, -ex);
    st(vnew.E, k, E);
    st(vnew.Fx, k, Fx);
    if (DIM == 2) st(vnew.Fy, k, Fy);
    st(vnew.T, k, T);
    stf(base.E, k, (float)E);
    stf(base.Fx, k, (float)Fx);
    if (DIM == 2) stf(base.Fy, k, (float)Fy);
    stf(base.T, k, (float)T);
    stf(r32.E, k, (float)rE);
    stf(r32.Fx, k, (float)rFx);
    if (DIM == 2) stf(r32.Fy, k, (float)rFy);
    stf(r32.T, k, (float)rT);
    if (z.d.E) {
        float oE, oFx, oFy, oT;
        mx_sweep_point<DIM>(ph, z.L, 0.0f, 1.0f, z.omega, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, (float)rE,
                            (float)rFx, (DIM == 2) ? (float)rFy : 0.0f, (float)rT, (float)sa, (float)ss, (float)T, oE,
                            oFx, oFy, oT);
        stf(z.d.E, k, oE);
        stf(z.d.Fx, k, oFx);
        if (DIM == 2) stf(z.d.Fy, k, oFy);
        stf(z.d.T, k, oT);
    }
    const double ic = 1.0 / ph.c;
    return fma(rE, rE, fma(rFx * ic, rFx * ic, fma(rFy * ic, rFy * ic, rT * rT)));
}

// Fixed-order reduction of q over a 256-thread block into *dst (thread 0).
__device__ __forceinline__ void mx_block_partial(double q, double* dst)
{
    __shared__ double red[kBlock32 / 64];
    for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) *dst = (red[0] + red[1]) + (red[2] + red[3]);
}

template <int DIM>
__global__ __launch_bounds__(kBlock32) void k_mx_resid(Phys ph, Lvl L, double eta, CSoa v, CSoa32 d, CSoa b,
                                                       Soa vnew, Soa32 base, Soa32 r32, double* __restrict__ partials,
                                                       const int* __restrict__ active, MxZero z)
{
    if (*active == 0) return;
    uint32_t k;
    int i, j;
    double q = 0.0;
    if (mx_cell(L.nx, L.ny, L.sh, k, i, j)) q = mx_resid_cell<DIM>(ph, L, eta, v, d, b, vnew, base, r32, k, i, j, z);
    if (partials) mx_block_partial(q, partials + xcd_block());
}

// ---------------------------------------------------------------------------
// Relaxed Jacobi sweep on the correction (any level, beta M + gamma N = rhs):
//   x: (beta M + gamma (D(w + x) - D(w))) = rhs + gamma dS(d);  out = d + omega (x - d).
// d.E == nullptr means d = 0 (first sweep of a cycle: dS = 0, no reads of d).
// The rest of the sweep of one cell from its off-diagonal increment S and its
// correction (dE, dFx, dFy, dT).
// mx_sweep_values returns the new correction, mx_sweep_update stores it at k of out.
template <int DIM>
__device__ __forceinline__ void mx_sweep_values(const Phys& ph, const Lvl32& L, const CSoa32& w, const CSoa32& rhs,
                                                float beta, float gamma, float omega, float S0, float S1, float S2,
                                                float dE, float dFx, float dFy, float dT, uint32_t k, float& oE,
                                                float& oFx, float& oFy, float& oT)
{
    mx_sweep_point<DIM>(ph, L, beta, gamma, omega, S0, S1, S2, dE, dFx, dFy, dT, ldf(rhs.E, k), ldf(rhs.Fx, k),
                        (DIM == 2) ? ldf(rhs.Fy, k) : 0.0f, ldf(rhs.T, k), ldf(L.sa, k), ldf(L.ss, k), ldf(w.T, k),
                        oE, oFx, oFy, oT);
}
template <int DIM>
__device__ __forceinline__ void mx_sweep_update(const Phys& ph, const Lvl32& L, const CSoa32& w, const CSoa32& rhs,
                                                float beta, float gamma, float omega, float S0, float S1, float S2,
                                                float dE, float dFx, float dFy, float dT, const Soa32& out,
                                                uint32_t k)
{
    float oE, oFx, oFy, oT;
    mx_sweep_values<DIM>(ph, L, w, rhs, beta, gamma, omega, S0, S1, S2, dE, dFx, dFy, dT, k, oE, oFx, oFy, oT);
    stf(out.E, k, oE);
    stf(out.Fx, k, oFx);
    if (DIM == 2) stf(out.Fy, k, oFy);
    stf(out.T, k, oT);
}

template <int DIM>
__device__ __forceinline__ void mx_sweep_cell(const Phys& ph, const Lvl32& L, const CSoa32& w, const CSoa32& d,
                                              const CSoa32& rhs, float beta, float gamma, float omega,
                                              const Soa32& out, uint32_t k, int i, int j)
{
    float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f;
    if (d.E) offdiag_inc<DIM>(ph, L, w, d, i, j, k, S0, S1, S2);
    const float dE = d.E ? ldf(d.E, k) : 0.0f, dFx = d.E ? ldf(d.Fx, k) : 0.0f;
    const float dFy = (DIM == 2 && d.E) ? ldf(d.Fy, k) : 0.0f, dT = d.E ? ldf(d.T, k) : 0.0f;
    mx_sweep_update<DIM>(ph, L, w, rhs, beta, gamma, omega, S0, S1, S2, dE, dFx, dFy, dT, out, k);
}

// ---------------------------------------------------------------------------
// LDS-staged sweep on the correction (2-D, d given): a block owns a 64 x TY
// tile; the base and correction of the tile and its one-cell halo are loaded
// once (boundary rule or periodic image applied) and the c^2 P increment of
// each is evaluated once; cells sum their neighbours' contributions from LDS.
// The arithmetic of every cell, and its order, is that of mx_sweep_cell.
constexpr int kMxTX = 64;

template <int TY>
struct MxTile {
    static constexpr int W = kMxTX + 2, N = W * (TY + 2);
    float e[N], gx[N], gy[N], xx[N], xy[N], yy[N];
};

// Whether the 64 x TY tile at (i0, j0) and a halo of `halo` cells lie inside
// the grid (no ghost, wrap or ragged edge).
__device__ __forceinline__ bool mx_interior(const Lvl32& L, int ty, int halo, int i0, int j0)
{
    return i0 >= halo && j0 >= halo && i0 + kMxTX + halo <= L.nx && j0 + ty + halo <= L.ny;
}

// Stage the 64 x TY tile at (i0, j0): correction (after the boundary rule) and
// c^2 P increment of every tile and halo point.  d_at(k, E, Fx, Fy, T) gives
// the correction of cell k; returns the T correction of this thread's own cell
// (0 outside the grid).  INTERIOR: mx_interior with a one-cell halo, and the
// side logic drops out (same arithmetic, same result).
template <int TY, bool INTERIOR = false, class DAt>
__device__ __forceinline__ float mx_stage_tile_at(MxTile<TY>& q, const Phys& ph, const Lvl32& L, const CSoa32& w,
                                                  DAt&& d_at, int i0, int j0)
{
    static_assert(kMxTX * TY >= 2 * kMxTX + 2 * TY, "the halo needs 2 rows and 2 columns of threads");
    constexpr int W = MxTile<TY>::W;
    const float c = (float)ph.c, c2 = (float)ph.c2;
    const bool perx = ph.bc[0] == BC_PERIODIC, pery = ph.bc[2] == BC_PERIODIC;
    auto gather = [&](int li, int lj) {
        int gi = i0 + li, gj = j0 + lj, side = 0;
        const bool ox = !INTERIOR && (gi < 0 || gi >= L.nx), oy = !INTERIOR && (gj < 0 || gj >= L.ny);
        const bool need = INTERIOR || (gi <= L.nx && gj <= L.ny && !(ox && oy));
        if (ox) {
            side = gi < 0 ? 0 : 1;
            gi = perx ? (gi < 0 ? gi + L.nx : gi - L.nx) : (gi < 0 ? 0 : L.nx - 1);
        }
        if (oy) {
            side = gj < 0 ? 2 : 3;
            gj = pery ? (gj < 0 ? gj + L.ny : gj - L.ny) : (gj < 0 ? 0 : L.ny - 1);
        }
        float e = 0.0f, gx = 0.0f, gy = 0.0f, dT = 0.0f;
        DP p{0.0f, 0.0f, 0.0f};
        if (need) {
            const uint32_t k = (uint32_t)gj * (uint32_t)L.nx + (uint32_t)gi;
            float E, Fx, Fy, dE, dFx, dFy;
            d_at(k, dE, dFx, dFy, dT);
            ghost_inc(ph, side, !(ox || oy), in_seg(L, side, side < 2 ? gj : gi), ldf(w.E, k), ldf(w.Fx, k),
                      ldf(w.Fy, k), dE, dFx, dFy, E, Fx, Fy, e, gx, gy);
            p = closure_inc(c, c2, E, Fx, Fy, e, gx, gy);
        }
        const int n = (lj + 1) * W + li + 1;
        q.e[n] = e;
        q.gx[n] = gx;
        q.gy[n] = gy;
        q.xx[n] = p.xx;
        q.xy[n] = p.xy;
        q.yy[n] = p.yy;
        return dT;
    };
    const int t = threadIdx.x;
    const float own = gather(t % kMxTX, t / kMxTX);
    if (t < 2 * kMxTX) {
        gather(t % kMxTX, t < kMxTX ? -1 : TY);
    } else if (t < 2 * kMxTX + 2 * TY) {
        const int r = t - 2 * kMxTX;
        gather(r < TY ? -1 : kMxTX, r % TY);
    }
    return own;
}

template <int TY, bool INTERIOR = false>
__device__ __forceinline__ void mx_stage_tile(MxTile<TY>& q, const Phys& ph, const Lvl32& L, const CSoa32& w,
                                              const CSoa32& d, int i0, int j0)
{
    (void)mx_stage_tile_at<TY, INTERIOR>(
        q, ph, L, w,
        [&](uint32_t k, float& E, float& Fx, float& Fy, float& T) {
            E = ldf(d.E, k);
            Fx = ldf(d.Fx, k);
            Fy = ldf(d.Fy, k);
            T = 0.0f;  // the sweep reads its own cell's T correction itself
        },
        i0, j0);
}

// The sweep of this thread's cell of a staged tile (nothing outside the grid).
// OWN_T: the cell's T correction is dT_own (else it is read from d).
template <int TY, bool OWN_T = false>
__device__ __forceinline__ void mx_tile_sweep(const MxTile<TY>& q, const Phys& ph, const Lvl32& L, const CSoa32& w,
                                              const CSoa32& d, const CSoa32& rhs, float beta, float gamma,
                                              float omega, const Soa32& out, int i0, int j0, float dT_own = 0.0f)
{
    constexpr int W = MxTile<TY>::W;
    const int li = threadIdx.x % kMxTX, lj = threadIdx.x / kMxTX, i = i0 + li, j = j0 + lj;
    if (i >= L.nx || j >= L.ny) return;
    const uint32_t k = (uint32_t)j * (uint32_t)L.nx + (uint32_t)i;
    const int n = (lj + 1) * W + li + 1;
    const float c = (float)ph.c;
    float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f;  // the order of offdiag_inc: x-, x+, y-, y+
    auto nb = [&](int m, float kk, float sgn, bool xdir) {
        acc_inc(kk, sgn, xdir, c, q.e[m], q.gx[m], q.gy[m], DP{q.xx[m], q.xy[m], q.yy[m]}, S0, S1, S2);
    };
    nb(n - 1, L.kx, +1.0f, true);
    nb(n + 1, L.kx, -1.0f, true);
    nb(n - W, L.ky, +1.0f, false);
    nb(n + W, L.ky, -1.0f, false);
    mx_sweep_update<2>(ph, L, w, rhs, beta, gamma, omega, S0, S1, S2, q.e[n], q.gx[n], q.gy[n],
                       OWN_T ? dT_own : ldf(d.T, k), out, k);
}

// LDS-staged sweep on the correction (2-D, d given): a block owns a 64 x TY
// tile; see mx_stage_tile.  The arithmetic of every cell, and its order, is
// that of mx_sweep_cell.
template <int TY>
__global__ __launch_bounds__(kMxTX * TY) void k_mx_sweep_lds(Phys ph, Lvl32 L, CSoa32 w, CSoa32 d, CSoa32 rhs,
                                                            float beta, float gamma, float omega, Soa32 out,
                                                            const int* __restrict__ active)
{
    __shared__ MxTile<TY> q;
    if (*active == 0) return;
    const int ntx = (L.nx + kMxTX - 1) / kMxTX;
    const int b = (int)xcd_block();
    const int i0 = (b % ntx) * kMxTX, j0 = (b / ntx) * TY;
    if (mx_interior(L, TY, 1, i0, j0)) mx_stage_tile<TY, true>(q, ph, L, w, d, i0, j0);
    else mx_stage_tile<TY>(q, ph, L, w, d, i0, j0);
    __syncthreads();
    mx_tile_sweep<TY>(q, ph, L, w, d, rhs, beta, gamma, omega, out, i0, j0);
}

// Two correction sweeps (beta = 0, gamma = 1) in one launch, as k_relax2_lds
// does for FP64: the block stages the base and the correction of its 64 x TY
// tile and a two-cell halo (boundary rule on ghosts, the c^2 P increment of
// each point once), runs the first sweep on the tile and its one-cell ring,
// rebuilds the ring's ghosts from the cells they border (the base of such a
// cell read again from memory, as the staging of a separate sweep would), and
// runs the second sweep from LDS.  Every point's arithmetic is that of
// k_mx_sweep_lds, so the result is two such sweeps' to the bit.
template <int TY>
struct MxLds2 {
    static constexpr int W2 = kMxTX + 4, N2 = W2 * (TY + 4);  // staged: tile + 2-cell halo
    static constexpr int W1 = kMxTX + 2, N1 = W1 * (TY + 2);  // first sweep's correction: tile + ring
    float buf[9 * N2];  // e, gx, gy, xx, xy, yy and the base E, Fx, Fy; the iterate's six arrays overwrite them
};

// Off-diagonal increment of the point at index n of a W-wide LDS region with
// arrays f[0..5] = e, gx, gy, xx, xy, yy, in the order of mx_tile_sweep.
template <int W>
__device__ __forceinline__ void mx_lds_sums(const float* const* f, const Lvl32& L, float c, int n, float& S0,
                                            float& S1, float& S2)
{
    S0 = S1 = S2 = 0.0f;
    auto nb = [&](int m, float kk, float sgn, bool xdir) {
        acc_inc(kk, sgn, xdir, c, f[0][m], f[1][m], f[2][m], DP{f[3][m], f[4][m], f[5][m]}, S0, S1, S2);
    };
    nb(n - 1, L.kx, +1.0f, true);
    nb(n + 1, L.kx, -1.0f, true);
    nb(n - W, L.ky, +1.0f, false);
    nb(n + W, L.ky, -1.0f, false);
}

__device__ __forceinline__ void mx_lds_put(float* const* f, int n, float e, float gx, float gy, const DP& p)
{
    f[0][n] = e;
    f[1][n] = gx;
    f[2][n] = gy;
    f[3][n] = p.xx;
    f[4][n] = p.xy;
    f[5][n] = p.yy;
}

// The two correction sweeps of the tile at (i0, j0); every thread of the block
// calls it.  INTERIOR: mx_interior with a two-cell halo (no side logic; same
// result).
template <int TY, bool INTERIOR = false>
__device__ __forceinline__ void mx_sweep2_tile(MxLds2<TY>& q, const Phys& ph, const Lvl32& L, const CSoa32& w,
                                               const CSoa32& d, const CSoa32& rhs, float omega, const Soa32& out,
                                               int i0, int j0)
{
    using Q = MxLds2<TY>;
    constexpr int NT = kMxTX * TY, NR = 2 * kMxTX + 2 * TY;  // threads; ring points
    static_assert(NR <= NT, "one ring point per thread");
    const float c = (float)ph.c, c2 = (float)ph.c2;
    const bool perx = ph.bc[0] == BC_PERIODIC, pery = ph.bc[2] == BC_PERIODIC;
    const int xe = INTERIOR ? i0 + kMxTX - 1 : min(i0 + kMxTX, L.nx) - 1;  // the last final cell
    const int ye = INTERIOR ? j0 + TY - 1 : min(j0 + TY, L.ny) - 1;
    // the plus of half-widths (a, b) around the final cells holds (gi, gj) (as in k_relax2_lds)
    auto plus = [&](int gi, int gj, int a, int bb) {
        return (gi >= i0 && gi <= xe && gj >= j0 - a && gj <= ye + a) ||
               (gi >= i0 - a && gi <= xe + a && gj >= j0 && gj <= ye) ||
               (bb > 0 && gi >= i0 - bb && gi <= xe + bb && gj >= j0 - bb && gj <= ye + bb);
    };
    float* f2[9];
    float* f1[6];
    for (int a = 0; a < 9; ++a) f2[a] = q.buf + a * Q::N2;
    for (int a = 0; a < 6; ++a) f1[a] = q.buf + a * Q::N1;
    // 1. stage base and correction (boundary rule on ghosts) and the increments
    for (int p = threadIdx.x; p < Q::N2; p += NT) {
        const int gi = i0 + p % Q::W2 - 2, gj = j0 + p / Q::W2 - 2;
        int si = gi, sj = gj;
        bool gx_ = false, gy_ = false, nx_ = true, ny_ = true;
        if (!INTERIOR) {
            rc_axis(gi, L.nx, perx, si, gx_, nx_);
            rc_axis(gj, L.ny, pery, sj, gy_, ny_);
        }
        float e = 0.0f, gx = 0.0f, gy = 0.0f, E = 0.0f, Fx = 0.0f, Fy = 0.0f;
        DP pp{0.0f, 0.0f, 0.0f};
        if (plus(gi, gj, 2, 1) && nx_ && ny_ && !(gx_ && gy_)) {
            const uint32_t k = (uint32_t)sj * (uint32_t)L.nx + (uint32_t)si;
            const int side = gx_ ? (gi < 0 ? 0 : 1) : (gj < 0 ? 2 : 3);
            ghost_inc(ph, side, !(gx_ || gy_), in_seg(L, side, side < 2 ? sj : si), ldf(w.E, k), ldf(w.Fx, k),
                      ldf(w.Fy, k), ldf(d.E, k), ldf(d.Fx, k), ldf(d.Fy, k), E, Fx, Fy, e, gx, gy);
            pp = closure_inc(c, c2, E, Fx, Fy, e, gx, gy);
        }
        mx_lds_put(f2, p, e, gx, gy, pp);
        f2[6][p] = E;
        f2[7][p] = Fx;
        f2[8][p] = Fy;
    }
    __syncthreads();
    // 2. first sweep: item 0 is the thread's tile point, item 1 a ring point
    const int t = threadIdx.x;
    int li[2], lj[2], kind[2];  // kind: 0 unused, 1 swept, 2 ghost
    int gsx[2], gsy[2];         // swept: the cell read; ghost: the cell it borders
    float vE[2], vFx[2], vFy[2], vT[2], bE[2], bFx[2], bFy[2];
    li[0] = t % kMxTX;
    lj[0] = t / kMxTX;
    if (t < kMxTX) li[1] = t, lj[1] = -1;
    else if (t < 2 * kMxTX) li[1] = t - kMxTX, lj[1] = TY;
    else if (t < 2 * kMxTX + TY) li[1] = -1, lj[1] = t - 2 * kMxTX;
    else li[1] = kMxTX, lj[1] = t - 2 * kMxTX - TY;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        kind[m] = 0;
        gsx[m] = gsy[m] = 0;
        vE[m] = vFx[m] = vFy[m] = vT[m] = bE[m] = bFx[m] = bFy[m] = 0.0f;
        const int gi = i0 + li[m], gj = j0 + lj[m];
        if ((m == 1 && t >= NR) || !plus(gi, gj, 1, 0)) continue;
        bool gx_ = false, gy_ = false, nx_ = true, ny_ = true;
        gsx[m] = gi;
        gsy[m] = gj;
        if (!INTERIOR) {
            rc_axis(gi, L.nx, perx, gsx[m], gx_, nx_);
            rc_axis(gj, L.ny, pery, gsy[m], gy_, ny_);
        }
        kind[m] = (gx_ || gy_) ? 2 : 1;  // the plus holds no corner: at most one side is off the domain
        if (kind[m] != 1) continue;
        const uint32_t k = (uint32_t)gsy[m] * (uint32_t)L.nx + (uint32_t)gsx[m];
        const int n = (lj[m] + 2) * Q::W2 + li[m] + 2;
        float S0, S1, S2;
        mx_lds_sums<Q::W2>(f2, L, c, n, S0, S1, S2);
        mx_sweep_values<2>(ph, L, w, rhs, 0.0f, 1.0f, omega, S0, S1, S2, f2[0][n], f2[1][n], f2[2][n], ldf(d.T, k), k,
                           vE[m], vFx[m], vFy[m], vT[m]);
        bE[m] = f2[6][n];
        bFx[m] = f2[7][n];
        bFy[m] = f2[8][n];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 2; ++m)
        if (kind[m] == 1)
            mx_lds_put(f1, (lj[m] + 1) * Q::W1 + li[m] + 1, vE[m], vFx[m], vFy[m],
                       closure_inc(c, c2, bE[m], bFx[m], bFy[m], vE[m], vFx[m], vFy[m]));
    // 3. ghosts of the iterate (only tiles on a non-periodic side have any)
    const bool edge =
        !INTERIOR && ((!perx && (i0 == 0 || xe == L.nx - 1)) || (!pery && (j0 == 0 || ye == L.ny - 1)));
    if (edge) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            if (kind[m] != 2) continue;
            const int gi = i0 + li[m], gj = j0 + lj[m];
            const int side = (gi < 0 || gi >= L.nx) ? (gi < 0 ? 0 : 1) : (gj < 0 ? 2 : 3);
            const int cb = (gsy[m] - j0 + 1) * Q::W1 + gsx[m] - i0 + 1;
            const uint32_t kb = (uint32_t)gsy[m] * (uint32_t)L.nx + (uint32_t)gsx[m];
            float E, Fx, Fy, e, gx, gy;
            ghost_inc(ph, side, false, in_seg(L, side, side < 2 ? gsy[m] : gsx[m]), ldf(w.E, kb), ldf(w.Fx, kb),
                      ldf(w.Fy, kb), f1[0][cb], f1[1][cb], f1[2][cb], E, Fx, Fy, e, gx, gy);
            mx_lds_put(f1, (lj[m] + 1) * Q::W1 + li[m] + 1, e, gx, gy, closure_inc(c, c2, E, Fx, Fy, e, gx, gy));
        }
    }
    __syncthreads();
    // 4. second sweep on the final cells
    const int i = i0 + li[0], j = j0 + lj[0];
    if (INTERIOR || (i < L.nx && j < L.ny)) {
        const uint32_t k = (uint32_t)j * (uint32_t)L.nx + (uint32_t)i;
        float S0, S1, S2;
        mx_lds_sums<Q::W1>(f1, L, c, (lj[0] + 1) * Q::W1 + li[0] + 1, S0, S1, S2);
        mx_sweep_update<2>(ph, L, w, rhs, 0.0f, 1.0f, omega, S0, S1, S2, vE[0], vFx[0], vFy[0], vT[0], out, k);
    }
}

// Six waves per SIMD (three 512-thread blocks per CU at 8 rows; 80 VGPRs, three
// values spilled): without the cap two blocks fit, and the pair measured slower
// than two single sweeps.
template <int TY>
__global__ __launch_bounds__(kMxTX * TY) __attribute__((amdgpu_waves_per_eu(6))) void k_mx_sweep2_lds(
    Phys ph, Lvl32 L, CSoa32 w, CSoa32 d, CSoa32 rhs, float omega, Soa32 out, const int* __restrict__ active)
{
    __shared__ MxLds2<TY> q;
    if (*active == 0) return;
    const int ntx = (L.nx + kMxTX - 1) / kMxTX;
    const int b = (int)xcd_block();
    const int i0 = (b % ntx) * kMxTX, j0 = (b / ntx) * TY;
    if (mx_interior(L, TY, 2, i0, j0)) mx_sweep2_tile<TY, true>(q, ph, L, w, d, rhs, omega, out, i0, j0);
    else mx_sweep2_tile<TY>(q, ph, L, w, d, rhs, omega, out, i0, j0);
}

template <int DIM>
__global__ __launch_bounds__(kBlock32) void k_mx_sweep(Phys ph, Lvl32 L, CSoa32 w, CSoa32 d, CSoa32 rhs, float beta,
                                                       float gamma, float omega, Soa32 out,
                                                       const int* __restrict__ active)
{
    if (*active == 0) return;
    uint32_t k;
    int i, j;
    if (!mx_cell(L.nx, L.ny, L.sh, k, i, j)) return;
    mx_sweep_cell<DIM>(ph, L, w, d, rhs, beta, gamma, omega, out, k, i, j);
}

// N(d) of one cell from its off-diagonal increment S, base temperature and correction.
// The same from the cell's opacities (sa, ss), loaded by the caller.
__device__ __forceinline__ void n_from_sums_with(const Phys& ph, const Lvl32& L, float S0, float S1, float S2,
                                                 float wT, float dE, float dFx, float dFy, float dT, float sa,
                                                 float ss, float& NE, float& NFx, float& NFy, float& NT)
{
    const double ka = (double)L.cdt * sa, ks = (double)L.cdt * ss;
    float DE, DFx, DFy, DT;
    diag_inc(L.a, ka, ks, ph.c_v, ph.a_r, wT, dE, dFx, dFy, dT, DE, DFx, DFy, DT);
    NE = DE - S0;
    NFx = DFx - S1;
    NFy = DFy - S2;
    NT = DT;
}

__device__ __forceinline__ void n_from_sums(const Phys& ph, const Lvl32& L, float S0, float S1, float S2, float wT,
                                            float dE, float dFx, float dFy, float dT, uint32_t k, float& NE,
                                            float& NFx, float& NFy, float& NT)
{
    n_from_sums_with(ph, L, S0, S1, S2, wT, dE, dFx, dFy, dT, ldf(L.sa, k), ldf(L.ss, k), NE, NFx, NFy, NT);
}

// Increment of A for one cell: N(d) = (D(w + d) - D(w)) - dS(d).
template <int DIM>
__device__ __forceinline__ void n_inc(const Phys& ph, const Lvl32& L, const CSoa32& w, const CSoa32& d, uint32_t k,
                                      int i, int j, float& NE, float& NFx, float& NFy, float& NT)
{
    float S0, S1, S2;
    offdiag_inc<DIM>(ph, L, w, d, i, j, k, S0, S1, S2);
    n_from_sums(ph, L, S0, S1, S2, ldf(w.T, k), ldf(d.E, k), ldf(d.Fx, k), (DIM == 2) ? ldf(d.Fy, k) : 0.0f,
                ldf(d.T, k), k, NE, NFx, NFy, NT);
}

// out = X + sgn N(d).
template <int DIM>
__device__ __forceinline__ void mx_apply_cell(const Phys& ph, const Lvl32& L, const CSoa32& w, const CSoa32& d,
                                              const CSoa32& X, float sgn, const Soa32& out, uint32_t k, int i, int j,
                                              bool live = true)
{
    float NE, NFx, NFy, NT;
    n_inc<DIM>(ph, L, w, d, k, i, j, NE, NFx, NFy, NT);
    const float oE = fmaf(sgn, NE, ldf(X.E, k)), oFx = fmaf(sgn, NFx, ldf(X.Fx, k));
    const float oFy = (DIM == 2) ? fmaf(sgn, NFy, ldf(X.Fy, k)) : 0.0f, oT = fmaf(sgn, NT, ldf(X.T, k));
    if (!live) return;
    stf(out.E, k, oE);
    stf(out.Fx, k, oFx);
    if (DIM == 2) stf(out.Fy, k, oFy);
    stf(out.T, k, oT);
}

template <int DIM>
__global__ __launch_bounds__(kBlock32) void k_mx_apply(Phys ph, Lvl32 L, CSoa32 w, CSoa32 d, CSoa32 X, float sgn,
                                                       Soa32 out, const int* __restrict__ active)
{
    const bool live = active[mx_lane_zero()] != 0;
    uint32_t k;
    int i, j;
    if (!mx_cell(L.nx, L.ny, L.sh, k, i, j)) return;
    mx_apply_cell<DIM>(ph, L, w, d, X, sgn, out, k, i, j, live);
}

// The source of the explicit sub-steps of a coarse level's pseudo-time solve
// (Algorithm 3): the level's FAS right-hand side in absolute form,
// f = A(w + d) + R(rho) (d = R(correction above), g = R(rho) on entry), the
// same f as the FP64 cycle's.  Formed in FP64 from the FP32 values by the first
// pseudo-time step of a visit (its neighbour loads are those offdiag_inc has
// just made) and stored in FP32 for the later ones.
template <int DIM>
__device__ __forceinline__ void mx_ray_src(const Phys& ph, const Lvl32& L, const CSoa32& w, const CSoa32& d,
                                           const Soa32& g, uint32_t k, int i, int j, float f[4])
{
    const double c = ph.c, c2 = ph.c2;
    double S0 = 0.0, S1 = 0.0, S2 = 0.0;
    float E, Fx, Fy, e, gx, gy;
    const uint32_t wx = (uint32_t)(L.nx - 1);
    nb_inc<DIM>(ph, 0, i > 0, in_seg(L, 0, j), i > 0 ? k - 1 : k + wx, k, w, d, E, Fx, Fy, e, gx, gy);
    add_x((double)L.kx, c, c2, +1.0, (double)E + e, (double)Fx + gx, (double)Fy + gy, S0, S1, S2);
    nb_inc<DIM>(ph, 1, i < L.nx - 1, in_seg(L, 1, j), i < L.nx - 1 ? k + 1 : k - wx, k, w, d, E, Fx, Fy, e, gx, gy);
    add_x((double)L.kx, c, c2, -1.0, (double)E + e, (double)Fx + gx, (double)Fy + gy, S0, S1, S2);
    if (DIM == 2) {
        const uint32_t nx = (uint32_t)L.nx, wrap = (uint32_t)(L.ny - 1) * nx;
        nb_inc<DIM>(ph, 2, j > 0, in_seg(L, 2, i), j > 0 ? k - nx : k + wrap, k, w, d, E, Fx, Fy, e, gx, gy);
        add_y((double)L.ky, c, c2, +1.0, (double)E + e, (double)Fx + gx, (double)Fy + gy, S0, S1, S2);
        nb_inc<DIM>(ph, 3, j < L.ny - 1, in_seg(L, 3, i), j < L.ny - 1 ? k + nx : k - wrap, k, w, d, E, Fx, Fy, e,
                    gx, gy);
        add_y((double)L.ky, c, c2, -1.0, (double)E + e, (double)Fx + gx, (double)Fy + gy, S0, S1, S2);
    }
    const double uE = (double)ldf(w.E, k) + ldf(d.E, k), uFx = (double)ldf(w.Fx, k) + ldf(d.Fx, k);
    const double uFy = (DIM == 2) ? (double)ldf(w.Fy, k) + ldf(d.Fy, k) : 0.0;
    const double uT = (double)ldf(w.T, k) + ldf(d.T, k);
    const double ka = (double)L.cdt * ldf(L.sa, k), ks = (double)L.cdt * ldf(L.ss, k);
    const double T2 = uT * uT;
    const double ex = ka * fma(-ph.a_r * T2, T2, uE);  // ka (E - a_r T^4)
    const double a = L.a;
    f[0] = (float)(ldf(g.E, k) + (fma(a, uE, ex) - S0));
    f[1] = (float)(ldf(g.Fx, k) + fma(a + ka + ks, uFx, -S1));
    f[2] = (DIM == 2) ? (float)(ldf(g.Fy, k) + fma(a + ka + ks, uFy, -S2)) : 0.0f;
    f[3] = (float)(ldf(g.T, k) + fma(ph.c_v, uT, -ex));
}

// The explicit sub-steps' source of cell k: formed (FIRST; e = d then) or stored.
template <int DIM, bool FIRST>
__device__ __forceinline__ void mx_ray_src_at(const Phys& ph, const Lvl32& L, const CSoa32& w, const CSoa32& e,
                                              const Soa32& g, const Soa32& fr, uint32_t k, int i, int j, float f[4])
{
    if (FIRST) {
        mx_ray_src<DIM>(ph, L, w, e, g, k, i, j, f);
    } else {
        f[0] = ldf(fr.E, k);
        f[1] = ldf(fr.Fx, k);
        f[2] = (DIM == 2) ? ldf(fr.Fy, k) : 0.0f;
        f[3] = ldf(fr.T, k);
    }
}

// One pseudo-time step of M de/dtau + N_w(e) = g (Algorithm 3 in increment
// form).  FIRST: e_in = d_l = R(correction above) and g holds R(rho) on entry;
// g = N_w(d_l) + R(rho) is formed and stored, and so is the absolute source
// f = g + A(w) (mx_ray_src).  The explicit sub-steps move u = w + e along f
// (the FP64 cycle's ray, so that u + tau_i f, the right-hand side of the
// implicit step, is admissible); the implicit step is the FP64 one,
// u' + gamma A(u') = u + tau_i f, in increment form:
// e' + gamma N_w(e') = e + gamma g + (tau_i - gamma) f.
// The step at cell k from its off-diagonal sums S, its correction e and f.
template <int DIM, bool FIRST>
__device__ __forceinline__ void mx_pseudo_finish(const Phys& ph, const Lvl32& L, const CSoa32& w, const Soa32& g,
                                                 const Soa32& fr, const float f[4], const Soa32& out, float dt,
                                                 float reach, int local, uint32_t k, float S0, float S1, float S2,
                                                 float eE, float eFx, float eFy, float eT, bool live)
{
    const float c2 = (float)ph.c2, cv = (float)ph.c_v;
    const float wE = ldf(w.E, k), wFx = ldf(w.Fx, k), wFy = (DIM == 2) ? ldf(w.Fy, k) : 0.0f, wT = ldf(w.T, k);
    const double ka = (double)L.cdt * ldf(L.sa, k), ks = (double)L.cdt * ldf(L.ss, k);
    float gE = ldf(g.E, k), gFx = ldf(g.Fx, k), gFy = (DIM == 2) ? ldf(g.Fy, k) : 0.0f, gT = ldf(g.T, k);
    if (FIRST) {
        float DE, DFx, DFy, DT;
        diag_inc(L.a, ka, ks, ph.c_v, ph.a_r, wT, eE, eFx, eFy, eT, DE, DFx, DFy, DT);
        gE += DE - S0;
        gFx += DFx - S1;
        gFy += DFy - S2;
        gT += DT;
        if (live) {
            stf(g.E, k, gE);
            stf(g.Fx, k, gFx);
            if (DIM == 2) stf(g.Fy, k, gFy);
            stf(g.T, k, gT);
            stf(fr.E, k, f[0]);
            stf(fr.Fx, k, f[1]);
            if (DIM == 2) stf(fr.Fy, k, f[2]);
            stf(fr.T, k, f[3]);
        }
    }
    const float icv = rcp32(cv);
    const float fE = f[0], fFx = f[1], fFy = f[2];
    const float sT = gT * icv, fsT = f[3] * icv;
    const float ts = ray_len32(c2, wE + eE, wFx + eFx, wFy + eFy, wT + eT, fE, fFx, fFy, fsT);
    if (live && ts == 0.0f && ph.stalls) note_stall(ph.stalls);
    const float tau = fminf(dt, ts * reach);
    const float gm = local ? tau : dt;
    const float off = tau - gm;  // 0 in the local reading
    const float tE = fmaf(off, fE, fmaf(gm, gE, eE)), tFx = fmaf(off, fFx, fmaf(gm, gFx, eFx));
    const float tFy = fmaf(off, fFy, fmaf(gm, gFy, eFy));
    const float tT = cv * fmaf(off, fsT, fmaf(gm, sT, eT));
    float xE, xFx, xFy, xT;
    local_solve_inc(1.0, gm, L.a, ka, ks, ph.c_v, ph.a_r, fmaf(gm, S0, tE), fmaf(gm, S1, tFx), fmaf(gm, S2, tFy), tT,
                    wT, eT, xE, xFx, xFy, xT);
    if (!live) return;
    stf(out.E, k, xE);
    stf(out.Fx, k, xFx);
    if (DIM == 2) stf(out.Fy, k, xFy);
    stf(out.T, k, xT);
}

template <int DIM, bool FIRST>
__device__ __forceinline__ void mx_pseudo_cell(const Phys& ph, const Lvl32& L, const CSoa32& w, const Soa32& g,
                                               const Soa32& fr, const CSoa32& e, const Soa32& out, float dt,
                                               float reach, int local, uint32_t k, int i, int j, bool live = true)
{
    float S0, S1, S2;
    offdiag_inc<DIM>(ph, L, w, e, i, j, k, S0, S1, S2);
    float f[4];
    mx_ray_src_at<DIM, FIRST>(ph, L, w, e, g, fr, k, i, j, f);
    const float eE = ldf(e.E, k), eFx = ldf(e.Fx, k), eFy = (DIM == 2) ? ldf(e.Fy, k) : 0.0f, eT = ldf(e.T, k);
    mx_pseudo_finish<DIM, FIRST>(ph, L, w, g, fr, f, out, dt, reach, local, k, S0, S1, S2, eE, eFx, eFy, eT, live);
}

template <int DIM>
__global__ __launch_bounds__(kBlock32) void k_mx_pseudo(Phys ph, Lvl32 L, CSoa32 w, Soa32 g, Soa32 fr, CSoa32 e,
                                                        Soa32 out, double dtau, const double* __restrict__ dtau_dev,
                                                        float reach, int local, int first,
                                                        const int* __restrict__ active)
{
    const uint32_t z = mx_lane_zero();
    const float dt = (float)dtau_dev[z];
    const bool live = active[z] != 0;
    uint32_t k;
    int i, j;
    if (!mx_cell(L.nx, L.ny, L.sh, k, i, j)) return;
    if (first) mx_pseudo_cell<DIM, true>(ph, L, w, g, fr, e, out, dt, reach, local, k, i, j, live);
    else mx_pseudo_cell<DIM, false>(ph, L, w, g, fr, e, out, dt, reach, local, k, i, j, live);
}

// LDS-staged pseudo-time step (2-D, large levels): the staging of
// k_mx_sweep_lds (base and correction of a 64 x TY tile and its halo, the
// c^2 P increment of each point once); each cell sums its neighbours'
// increments from LDS in the order of offdiag_inc and finishes as
// mx_pseudo_cell, so the result is that of k_mx_pseudo to the bit.  e and out
// must not alias.  Used from 512 K cells up, as the FP64 step (measured
// slightly faster than staging the 256^2 and 512^2 levels too).
constexpr int64_t kMxPseudoLdsCells = 524288;

template <int TY, bool FIRST>
__global__ __launch_bounds__(kMxTX * TY) void k_mx_pseudo_lds(Phys ph, Lvl32 L, CSoa32 w, Soa32 g, Soa32 fr,
                                                             CSoa32 e, Soa32 out, const double* __restrict__ dtau_dev,
                                                             float reach, int local, const int* __restrict__ active)
{
    constexpr int W = MxTile<TY>::W;
    __shared__ MxTile<TY> q;
    if (*active == 0) return;
    const float dt = (float)*dtau_dev;
    const int ntx = (L.nx + kMxTX - 1) / kMxTX;
    const int b = (int)xcd_block();
    const int i0 = (b % ntx) * kMxTX, j0 = (b / ntx) * TY;
    if (mx_interior(L, TY, 1, i0, j0)) mx_stage_tile<TY, true>(q, ph, L, w, e, i0, j0);
    else mx_stage_tile<TY>(q, ph, L, w, e, i0, j0);
    __syncthreads();
    const int li = threadIdx.x % kMxTX, lj = threadIdx.x / kMxTX, i = i0 + li, j = j0 + lj;
    if (i >= L.nx || j >= L.ny) return;
    const uint32_t k = (uint32_t)j * (uint32_t)L.nx + (uint32_t)i;
    const int n = (lj + 1) * W + li + 1;
    const float c = (float)ph.c;
    float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f;  // the order of offdiag_inc: x-, x+, y-, y+
    auto nb = [&](int m, float kk, float sgn, bool xdir) {
        acc_inc(kk, sgn, xdir, c, q.e[m], q.gx[m], q.gy[m], DP{q.xx[m], q.xy[m], q.yy[m]}, S0, S1, S2);
    };
    nb(n - 1, L.kx, +1.0f, true);
    nb(n + 1, L.kx, -1.0f, true);
    nb(n - W, L.ky, +1.0f, false);
    nb(n + W, L.ky, -1.0f, false);
    float f[4];
    mx_ray_src_at<2, FIRST>(ph, L, w, e, g, fr, k, i, j, f);
    mx_pseudo_finish<2, FIRST>(ph, L, w, g, fr, f, out, dt, reach, local, k, S0, S1, S2, q.e[n], q.gx[n], q.gy[n],
                               ldf(e.T, k), true);
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
__device__ __forceinline__ void coarse_corr(int nx, int ny, int sh, int px, int py, const CSoa32& ec, const CSoa32& dc,
                                            uint32_t k, float& c0, float& c1, float& c2, float& c3)
{
    int i, j;
    ij_of(nx, sh, k, i, j);
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
            const uint32_t kc = (uint32_t)iy[b] * (uint32_t)nxc + (uint32_t)ix[a];
            const float wgt = wx[a] * wy[b];
            c0 = fmaf(wgt, ldf(ec.E, kc) - ldf(dc.E, kc), c0);
            c1 = fmaf(wgt, ldf(ec.Fx, kc) - ldf(dc.Fx, kc), c1);
            if (DIM == 2) c2 = fmaf(wgt, ldf(ec.Fy, kc) - ldf(dc.Fy, kc), c2);
            c3 = fmaf(wgt, ldf(ec.T, kc) - ldf(dc.T, kc), c3);
        }
}

template <int DIM>
__device__ __forceinline__ void mx_prolong_cell(const Phys& ph, int nx, int ny, int sh, int px, int py, float eta,
                                                const CSoa32& w, const CSoa32& e, const CSoa32& ec, const CSoa32& dc,
                                                const Soa32& out, uint32_t k, bool live = true)
{
    float c0, c1, c2, c3;
    coarse_corr<DIM>(nx, ny, sh, px, py, ec, dc, k, c0, c1, c2, c3);
    const float eE = ldf(e.E, k), eFx = ldf(e.Fx, k), eFy = (DIM == 2) ? ldf(e.Fy, k) : 0.0f, eT = ldf(e.T, k);
    const float sE = ldf(w.E, k) + eE, sFx = ldf(w.Fx, k) + eFx;
    const float sFy = ((DIM == 2) ? ldf(w.Fy, k) : 0.0f) + eFy, sT = ldf(w.T, k) + eT;
    float th = 1.0f;
    const float cc2 = (float)ph.c2;
    if (!admissible32(cc2, sE + c0, sFx + c1, sFy + c2, sT + c3))
        th = eta * fminf(ray_len32(cc2, sE, sFx, sFy, sT, c0, c1, c2, c3), 1.0f);
    if (!live) return;
    stf(out.E, k, fmaf(th, c0, eE));
    stf(out.Fx, k, fmaf(th, c1, eFx));
    if (DIM == 2) stf(out.Fy, k, fmaf(th, c2, eFy));
    stf(out.T, k, fmaf(th, c3, eT));
}

template <int DIM>
__global__ __launch_bounds__(kBlock32) void k_mx_prolong(Phys ph, int nx, int ny, int sh, int px, int py, float eta,
                                                         CSoa32 w, CSoa32 e, CSoa32 ec, CSoa32 dc, Soa32 out,
                                                         const int* __restrict__ active)
{
    const bool live = active[mx_lane_zero()] != 0;
    const uint32_t k = (uint32_t)xcd_block() * kBlock32 + threadIdx.x;
    if (k >= (uint32_t)nx * (uint32_t)ny) return;
    mx_prolong_cell<DIM>(ph, nx, ny, sh, px, py, eta, w, e, ec, dc, out, k, live);
}

// The rest of the fine correction of cell k from its coarse correction (c0..c3): the admissibility test of
// v + e + c in FP64 (eq. prolongatedSol).
template <int DIM>
__device__ __forceinline__ void mx_prolong_fine_finish(const Phys& ph, double eta, const CSoa& v, const CSoa32& e,
                                                       uint32_t k, float c0, float c1, float c2, float c3, float& oE,
                                                       float& oFx, float& oFy, float& oT)
{
    const float eE = ldf(e.E, k), eFx = ldf(e.Fx, k), eFy = (DIM == 2) ? ldf(e.Fy, k) : 0.0f, eT = ldf(e.T, k);
    const double sE = ld(v.E, k) + (double)eE, sFx = ld(v.Fx, k) + (double)eFx;
    const double sFy = ((DIM == 2) ? ld(v.Fy, k) : 0.0) + (double)eFy, sT = ld(v.T, k) + (double)eT;
    double th = 1.0;
    if (!admissible(ph.c2, sE + c0, sFx + c1, sFy + c2, sT + c3))
        th = eta * fmin(ray_len(ph.c2, sE, sFx, sFy, sT, c0, c1, c2, c3), 1.0);
    oE = (float)fma(th, (double)c0, (double)eE);
    oFx = (float)fma(th, (double)c1, (double)eFx);
    oFy = (DIM == 2) ? (float)fma(th, (double)c2, (double)eFy) : 0.0f;
    oT = (float)fma(th, (double)c3, (double)eT);
}

// The corrected correction of fine cell k: e + theta P(e_c - d_c), theta from
// the admissibility test of v + e + P(e_c - d_c) in FP64.
template <int DIM>
__device__ __forceinline__ void mx_prolong_fine_values(const Phys& ph, int nx, int ny, int sh, int px, int py,
                                                       double eta, const CSoa& v, const CSoa32& e, const CSoa32& ec,
                                                       const CSoa32& dc, uint32_t k, float& oE, float& oFx,
                                                       float& oFy, float& oT)
{
    float c0, c1, c2, c3;
    coarse_corr<DIM>(nx, ny, sh, px, py, ec, dc, k, c0, c1, c2, c3);
    mx_prolong_fine_finish<DIM>(ph, eta, v, e, k, c0, c1, c2, c3, oE, oFx, oFy, oT);
}

// The corrected correction of fine cell (i, j) of a 2-D level whose coarse
// differences ec - dc are staged: c?[(Jc - Jc0) cw + Ic - Ic0] for the coarse
// cells it reads, none across a side.  The weights, differences and order of
// coarse_corr, so the result of mx_prolong_fine_values.
__device__ __forceinline__ void mx_prolong_fine_values_staged(const Phys& ph, int nx, int ny, double eta, const CSoa& v,
                                                              const CSoa32& e, uint32_t k, int i, int j,
                                                              const float* cE, const float* cFx, const float* cFy,
                                                              const float* cT, int Ic0, int Jc0, int cw, float& oE,
                                                              float& oFx, float& oFy, float& oT)
{
    int ix[2], iy[2];
    float wx[2], wy[2];
    pw32(i, nx / 2, false, ix, wx);
    pw32(j, ny / 2, false, iy, wy);
    float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, c3 = 0.0f;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int c = (iy[b] - Jc0) * cw + ix[a] - Ic0;
            const float wgt = wx[a] * wy[b];
            c0 = fmaf(wgt, cE[c], c0);
            c1 = fmaf(wgt, cFx[c], c1);
            c2 = fmaf(wgt, cFy[c], c2);
            c3 = fmaf(wgt, cT[c], c3);
        }
    mx_prolong_fine_finish<2>(ph, eta, v, e, k, c0, c1, c2, c3, oE, oFx, oFy, oT);
}


template <int DIM>
__device__ __forceinline__ void mx_prolong_fine_cell(const Phys& ph, int nx, int ny, int sh, int px, int py,
                                                     double eta, const CSoa& v, const CSoa32& e, const CSoa32& ec,
                                                     const CSoa32& dc, const Soa32& out, uint32_t k, bool live)
{
    float E, Fx, Fy, T;
    mx_prolong_fine_values<DIM>(ph, nx, ny, sh, px, py, eta, v, e, ec, dc, k, E, Fx, Fy, T);
    if (!live) return;
    stf(out.E, k, E);
    stf(out.Fx, k, Fx);
    if (DIM == 2) stf(out.Fy, k, Fy);
    stf(out.T, k, T);
}

template <int DIM>
__global__ __launch_bounds__(kBlock32) void k_mx_prolong_fine(Phys ph, int nx, int ny, int sh, int px, int py,
                                                              double eta, CSoa v, CSoa32 e, CSoa32 ec, CSoa32 dc,
                                                              Soa32 out, const int* __restrict__ active)
{
    const bool live = active[mx_lane_zero()] != 0;
    const uint32_t k = (uint32_t)xcd_block() * kBlock32 + threadIdx.x;
    if (k >= (uint32_t)nx * (uint32_t)ny) return;
    mx_prolong_fine_cell<DIM>(ph, nx, ny, sh, px, py, eta, v, e, ec, dc, out, k, live);
}

// Coarse correction of the finest level fused with the first post-smoothing
// correction sweep (2-D; beta = 0, gamma = 1): the staging of k_mx_sweep_lds
// takes each tile and halo point's correction from mx_prolong_fine_values
// instead of memory, so the corrected correction is never stored and the
// result is k_mx_prolong_fine then k_mx_sweep_lds to the bit.
template <int TY>
__global__ __launch_bounds__(kMxTX * TY) void k_mx_prolong_sweep_lds(Phys ph, Lvl32 L, CSoa32 w, CSoa v, CSoa32 e,
                                                                    CSoa32 ec, CSoa32 dc, int sh, int px, int py,
                                                                    double eta, CSoa32 rhs, float omega, Soa32 out,
                                                                    const int* __restrict__ active)
{
    // the coarse differences ec - dc of the tile's footprint, staged once where it lies inside the coarse grid
    constexpr int CW = kMxTX / 2 + 3, CH = TY / 2 + 3, CN = CW * CH;
    __shared__ MxTile<TY> q;
    __shared__ float cE[CN], cFx[CN], cFy[CN], cT[CN];
    if (*active == 0) return;
    const int ntx = (L.nx + kMxTX - 1) / kMxTX;
    const int b = (int)xcd_block();
    const int i0 = (b % ntx) * kMxTX, j0 = (b / ntx) * TY;
    float dT;
    if (i0 >= 2 && j0 >= 2 && i0 + kMxTX + 4 <= L.nx && j0 + TY + 4 <= L.ny) {
        const int Ic0 = i0 / 2 - 1, Jc0 = j0 / 2 - 1, nxc = L.nx / 2;
        for (int c = threadIdx.x; c < CN; c += kMxTX * TY) {
            const uint32_t kc = (uint32_t)(Jc0 + c / CW) * (uint32_t)nxc + (uint32_t)(Ic0 + c % CW);
            cE[c] = ldf(ec.E, kc) - ldf(dc.E, kc);
            cFx[c] = ldf(ec.Fx, kc) - ldf(dc.Fx, kc);
            cFy[c] = ldf(ec.Fy, kc) - ldf(dc.Fy, kc);
            cT[c] = ldf(ec.T, kc) - ldf(dc.T, kc);
        }
        __syncthreads();
        dT = mx_stage_tile_at<TY, true>(
            q, ph, L, w,
            [&](uint32_t k, float& E, float& Fx, float& Fy, float& T) {
                int i, j;
                ij_of(L.nx, sh, k, i, j);
                mx_prolong_fine_values_staged(ph, L.nx, L.ny, eta, v, e, k, i, j, cE, cFx, cFy, cT, Ic0, Jc0, CW, E,
                                              Fx, Fy, T);
            },
            i0, j0);
    } else {
        auto d_at = [&](uint32_t k, float& E, float& Fx, float& Fy, float& T) {
            mx_prolong_fine_values<2>(ph, L.nx, L.ny, sh, px, py, eta, v, e, ec, dc, k, E, Fx, Fy, T);
        };
        dT = mx_interior(L, TY, 1, i0, j0) ? mx_stage_tile_at<TY, true>(q, ph, L, w, d_at, i0, j0)
                                            : mx_stage_tile_at<TY>(q, ph, L, w, d_at, i0, j0);
    }
    __syncthreads();
    mx_tile_sweep<TY, true>(q, ph, L, w, CSoa32{}, rhs, 0.0f, 1.0f, omega, out, i0, j0, dT);
}

// FP32 restriction of NF fields (base, correction, residual of a level) for
// coarse cell k: full weighting, all values gathered before the sums.
// FP32 full-weighting weights of coarse cell c (as rweights): fine 2c-1 .. 2c+1;
// off a non-periodic side the point is clamped with weight 0, the rest renormalised.
__device__ __forceinline__ void rweights32(int c, int nf, bool per, int* idx, float* w)
{
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
}

template <int DIM, int NF>
__device__ __forceinline__ void mx_restrict_cell(int nxf, int nyf, int shf, int px, int py, const float* const* in,
                                                 float* const* out, uint32_t k, bool live = true)
{
    const int nxc = nxf / 2;
    int I, J;
    ij_of(nxc, shf > 0 ? shf - 1 : -1, k, I, J);
    int ix[3], iy[3] = {0, 0, 0};
    float wx[3], wy[3] = {1.0f, 0.0f, 0.0f};
    rweights32(I, nxf, px != 0, ix, wx);
    if (DIM == 2) rweights32(J, nyf, py != 0, iy, wy);
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
        for (int m = 0; m < NB * 3; ++m) val[q][m] = ldf(in[q], off[m]);
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        float s = 0.0f;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const float t = fmaf(wx[2], val[q][b * 3 + 2], fmaf(wx[1], val[q][b * 3 + 1], wx[0] * val[q][b * 3]));
            s = fmaf(wy[b], t, s);
        }
        if (live) stf(out[q], k, s);
    }
}

template <int DIM, int NF>
__global__ __launch_bounds__(kBlock32) void k_mx_restrict(int nxf, int nyf, int shf, int px, int py, Fields32 F,
                                                          const int* __restrict__ active)
{
    const bool live = active[mx_lane_zero()] != 0;
    const uint32_t nc = (uint32_t)(nxf / 2) * (uint32_t)((DIM == 2) ? nyf / 2 : 1);
    const uint32_t k = (uint32_t)xcd_block() * kBlock32 + threadIdx.x;
    if (k >= nc) return;
    mx_restrict_cell<DIM, NF>(nxf, nyf, shf, px, py, F.in, F.out, k, live);
}

// ---------------------------------------------------------------------------
// Bottom of the mixed cycle in one workgroup: levels lt..L-1, entered with
// w_lt, d_lt and g_lt (= R(rho)) restricted; leaves e_lt (corrected, smoothed)
// in lev[lt].e.  Same per-cell bodies and order as the grid path.
template <int DIM>
__device__ __forceinline__ Soa32 mx_tail_pseudo(const TailArgs32& A, const TailLevel32& T, float dt, Soa32 in,
                                                bool first)
{
    const uint32_t n = (uint32_t)T.L.nx * (uint32_t)T.L.ny;
    for (int m = 0; m < A.pseudo_steps; ++m) {
        const Soa32 out = (in.E == T.e.E) ? T.e2 : T.e;
        for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) {
            int i, j;
            ij_of(T.L.nx, T.L.sh, k, i, j);
            if (first && m == 0)
                mx_pseudo_cell<DIM, true>(A.ph, T.L, cs(T.w), T.g, T.fr, cs(in), out, dt, A.reach, A.local, k, i, j);
            else
                mx_pseudo_cell<DIM, false>(A.ph, T.L, cs(T.w), T.g, T.fr, cs(in), out, dt, A.reach, A.local, k, i, j);
        }
        __syncthreads();
        in = out;
    }
    return in;
}

template <int DIM>
__device__ __forceinline__ void mx_tail_body(const TailArgs32& A, float dt)
{
    unsigned in_e2 = 0;
    auto cur = [&](int l) { return ((in_e2 >> l) & 1u) ? A.lev[l].e2 : A.lev[l].e; };
    auto set = [&](int l, const Soa32& s) {
        if (s.E == A.lev[l].e2.E) in_e2 |= 1u << l;
        else in_e2 &= ~(1u << l);
    };
    for (int l = A.lt; l < A.L; ++l) {
        const TailLevel32& T = A.lev[l];
        const uint32_t n = (uint32_t)T.L.nx * (uint32_t)T.L.ny;
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
            for (uint32_t k = threadIdx.x; k < n; k += blockDim.x)
                mx_restrict_cell<DIM, DIM == 2 ? 12 : 9>(F.L.nx, F.L.ny, F.L.sh, A.px, A.py, in, out, k);
            __syncthreads();
        }
        set(l, mx_tail_pseudo<DIM>(A, T, dt, T.d, true));
        if (l < A.L - 1) {
            const Soa32 e = cur(l);
            for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) {
                int i, j;
                ij_of(T.L.nx, T.L.sh, k, i, j);
                mx_apply_cell<DIM>(A.ph, T.L, cs(T.w), cs(e), cs(T.g), -1.0f, T.rho, k, i, j);
            }
            __syncthreads();
        }
    }
    for (int l = A.L - 2; l >= A.lt; --l) {
        const TailLevel32& T = A.lev[l];
        const TailLevel32& C = A.lev[l + 1];
        const uint32_t n = (uint32_t)T.L.nx * (uint32_t)T.L.ny;
        const Soa32 e = cur(l), ec = cur(l + 1);
        for (uint32_t k = threadIdx.x; k < n; k += blockDim.x)
            mx_prolong_cell<DIM>(A.ph, T.L.nx, T.L.ny, T.L.sh, A.px, A.py, (float)A.eta, cs(T.w), cs(e), cs(ec),
                                 cs(C.d), e, k);
        __syncthreads();
        set(l, mx_tail_pseudo<DIM>(A, T, dt, e, false));
    }
    const TailLevel32& T = A.lev[A.lt];
    const Soa32 res = cur(A.lt);
    if (res.E != T.e.E) {
        const uint32_t n = (uint32_t)T.L.nx * (uint32_t)T.L.ny;
        for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) {
            stf(T.e.E, k, ldf(res.E, k));
            stf(T.e.Fx, k, ldf(res.Fx, k));
            if (DIM == 2) stf(T.e.Fy, k, ldf(res.Fy, k));
            stf(T.e.T, k, ldf(res.T, k));
        }
    }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_mx_tail(const TailArgs32* __restrict__ Ap, double dtau,
                                                  const double* __restrict__ dtau_dev, const int* __restrict__ active)
{
    const float dt = (float)*dtau_dev;
    if (*active == 0) return;
    mx_tail_body<DIM>(*Ap, dt);
}

__global__ __launch_bounds__(kBlock32) void k_to_f32(int64_t n, const double* __restrict__ a, float* __restrict__ b)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock32 + threadIdx.x;
    if (k < n) b[k] = (float)a[k];
}

// ===========================================================================
// Batched mixed-precision kernels (2-D): the same per-cell bodies over work
// lists of (problem, 256-cell tile), each problem with its own control.  The
// FP64 state of a problem is in x1 when ctrl->flip is set (its residual
// kernel writes the partner buffer once per executed cycle).
__device__ __forceinline__ const Soa32& pickA(const BSlot32& s, int sel) { return sel == 0 ? s.dA : s.dB; }
__device__ __forceinline__ const Soa32& pick32(const BSlot32& s, int sel)
{
    return sel == 0 ? s.d : (sel == 1 ? s.e : s.e2);
}

// Final iterate of level l + 1 as seen by the prolongation into level l: the
// tail's result or the coarsest level's pre-smoothing (both in e) at the
// deepest level a problem smooths on the grid, else its post-smoothing (e2).
__device__ __forceinline__ const Soa32& coarse_final(const BProb& pb, const BSlot32& c, int level)
{
    const int top = pb.lt < pb.L - 1 ? pb.lt : pb.L - 1;
    return (level + 1 == top) ? c.e : c.e2;
}

// Residual with the pending correction (pend_sel; none on a step's first cycle).
__global__ __launch_bounds__(kBlock32) void kbm_resid(const BProb* __restrict__ P, const BSlot* __restrict__ S,
                                                      const BSlot32* __restrict__ S32,
                                                      const uint32_t* __restrict__ wl, int nwl, int pend_sel,
                                                      int zero)
{
    M1_BATCH_LOOP(wl, nwl)
    const BSlot& s = S[p * kMaxLevels];
    const BSlot32& s32 = S32[p * kMaxLevels];
    const bool fl = pb.ctrl->flip != 0;
    const CSoa32 d = (pb.ctrl->cycles < 0) ? CSoa32{} : cs(pickA(s32, pend_sel));
    double q = 0.0;
    if (k < (uint32_t)s.L.nx * (uint32_t)s.L.ny) {
        int i, j;
        ij_of(s.L.nx, s.L.sh, k, i, j);
        const MxZero z = zero ? MxZero{s32.L, (float)pb.omega, pickA(s32, 0)} : MxZero{};
        q = mx_resid_cell<2>(pb.ph, s.L, pb.eta, cs(fl ? s.x1 : s.x0), d, cs(s.b), fl ? s.x0 : s.x1, s32.base, s32.r32,
                             k, i, j, z);
    }
    mx_block_partial(q, pb.partials + tile);
    __syncthreads();  // the next tile of this block reuses the reduction slots
    }
}

__global__ __launch_bounds__(kBlock32) void kbm_sweep(const BProb* __restrict__ P, const BSlot32* __restrict__ S32,
                                                      const uint32_t* __restrict__ wl, int nwl, int in_sel,
                                                      int out_sel, int from_zero)
{
    M1_BATCH_LOOP(wl, nwl)
    const BSlot32& s = S32[p * kMaxLevels];
    if (k >= (uint32_t)s.L.nx * (uint32_t)s.L.ny) continue;
    int i, j;
    ij_of(s.L.nx, s.L.sh, k, i, j);
    mx_sweep_cell<2>(pb.ph, s.L, cs(s.base), from_zero ? CSoa32{} : cs(pickA(s, in_sel)), cs(s.r32), 0.0f, 1.0f,
                     (float)pb.omega, pickA(s, out_sel), k, i, j);
    }
}

// ---------------------------------------------------------------------------
// Finest-level residual of the correction equation fused with the restriction
// to level 1 (2-D): rho = X + sgn N_w(d) is formed in LDS for the fine cells
// the 3x3 stencils of a 32 x 4 coarse tile read, and w, d and rho are
// restricted into (wc, dc, gc) with the weights and order of mx_restrict_cell.
// The geometry is that of k_residual_restrict (FP64 path).
constexpr int kMrCW = 32, kMrCH = 4;
constexpr int kMrSW = 2 * kMrCW + 3, kMrSH = 2 * kMrCH + 3, kMrRW = 2 * kMrCW + 1, kMrRH = 2 * kMrCH + 1;
constexpr int kMrThreads = 512;

// LDS of one tile: the staged base states, corrections and closure increments;
// once every residual is formed, the residual of point q goes to
// (sXX, sXY, sYY, qT)[q] (the closure increments are no longer read).
struct MrLds {
    static constexpr int NS = kMrSW * kMrSH, NR = kMrRW * kMrRH;
    float sWE[NS], sWFx[NS], sWFy[NS], sWT[NS], sE[NS], sGx[NS], sGy[NS], sT[NS], sXX[NS], sXY[NS], sYY[NS];
    float qT[NR];
};
static_assert(MrLds::NR <= MrLds::NS, "residuals are kept in the closure arrays");

// The fused residual and restriction of the coarse tile at (I0, J0) (all
// threads of the block take part; no thread returns early).
// Whether every point the coarse tile at (I0, J0) stages lies inside the grid
// (as rc_interior of the FP64 kernel): no ghost, wrap or clamp, and the
// restriction weights are (1/4, 1/2, 1/4).
__device__ __forceinline__ bool mr_interior(const Lvl32& L, int I0, int J0)
{
    return I0 >= 1 && J0 >= 1 && 2 * (I0 + kMrCW) <= L.nx - 1 && 2 * (J0 + kMrCH) <= L.ny - 1;
}

template <bool INTERIOR>
__device__ __forceinline__ void mx_residual_restrict_tile(MrLds& sm, const Phys& ph, const Lvl32& L, const CSoa32& w,
                                                          const CSoa32& d, const CSoa32& X, float sgn, int px, int py,
                                                          const Soa32& wc, const Soa32& dc, const Soa32& gc, int I0,
                                                          int J0, bool live)
{
    constexpr int NS = MrLds::NS, NR = MrLds::NR;
    constexpr int RPT = (NR + kMrThreads - 1) / kMrThreads;  // residual points per thread
    const int nxc = L.nx / 2, nyc = L.ny / 2;
    const int fi0 = 2 * I0, fj0 = 2 * J0;
    const float c = (float)ph.c, c2 = (float)ph.c2;
    // each residual point's own loads (opacities, right-hand side) first, to overlap the staging
    float own[RPT][6];
    bool has[RPT];
#pragma unroll
    for (int it = 0; it < RPT; ++it) {
        const int q = threadIdx.x + it * kMrThreads;
        const int gi = fi0 + q % kMrRW - 1, gj = fj0 + q / kMrRW - 1;
        has[it] = q < NR && (INTERIOR || (gi < L.nx && gj < L.ny));
#pragma unroll
        for (int m = 0; m < 6; ++m) own[it][m] = 0.0f;
        if (has[it]) {
            const int si = (INTERIOR || gi >= 0) ? gi : (px ? gi + L.nx : 0);
            const int sj = (INTERIOR || gj >= 0) ? gj : (py ? gj + L.ny : 0);
            const uint32_t k = (uint32_t)sj * (uint32_t)L.nx + (uint32_t)si;
            own[it][0] = ldf(L.sa, k);
            own[it][1] = ldf(L.ss, k);
            own[it][2] = ldf(X.E, k);
            own[it][3] = ldf(X.Fx, k);
            own[it][4] = ldf(X.Fy, k);
            own[it][5] = ldf(X.T, k);
        }
    }
    for (int q = threadIdx.x; q < NS; q += kMrThreads) {
        const int gi = fi0 + q % kMrSW - 2, gj = fj0 + q / kMrSW - 2;
        int si = gi, sj = gj;
        bool hx = false, hy = false, nx_ = true, ny_ = true;
        if (!INTERIOR) {
            rc_axis(gi, L.nx, px != 0, si, hx, nx_);
            rc_axis(gj, L.ny, py != 0, sj, hy, ny_);
        }
        float E = 0.0f, Fx = 0.0f, Fy = 0.0f, T = 0.0f, e = 0.0f, gx = 0.0f, gy = 0.0f, t = 0.0f;
        DP p{0.0f, 0.0f, 0.0f};
        if (nx_ && ny_ && !(hx && hy)) {
            const int side = hx ? (gi < 0 ? 0 : 1) : (hy ? (gj < 0 ? 2 : 3) : 0);
            const uint32_t k = (uint32_t)sj * (uint32_t)L.nx + (uint32_t)si;
            ghost_inc(ph, side, !(hx || hy), in_seg(L, side, side < 2 ? sj : si), ldf(w.E, k), ldf(w.Fx, k),
                      ldf(w.Fy, k), ldf(d.E, k), ldf(d.Fx, k), ldf(d.Fy, k), E, Fx, Fy, e, gx, gy);
            T = ldf(w.T, k);
            t = ldf(d.T, k);
            p = closure_inc(c, c2, E, Fx, Fy, e, gx, gy);
        }
        sm.sWE[q] = E;
        sm.sWFx[q] = Fx;
        sm.sWFy[q] = Fy;
        sm.sWT[q] = T;
        sm.sE[q] = e;
        sm.sGx[q] = gx;
        sm.sGy[q] = gy;
        sm.sT[q] = t;
        sm.sXX[q] = p.xx;
        sm.sXY[q] = p.xy;
        sm.sYY[q] = p.yy;
    }
    __syncthreads();
    auto centre = [&](int ri, int rj) {
        if (!INTERIOR && fi0 + ri < 0 && !px) ri += 1;
        if (!INTERIOR && fj0 + rj < 0 && !py) rj += 1;
        return (rj + 2) * kMrSW + ri + 2;
    };
    float res[RPT][4];
#pragma unroll
    for (int it = 0; it < RPT; ++it) {
        const int q = threadIdx.x + it * kMrThreads;
        float oE = 0.0f, oFx = 0.0f, oFy = 0.0f, oT = 0.0f;
        if (has[it]) {
            const int n = centre(q % kMrRW - 1, q / kMrRW - 1);
            float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f;  // the order of offdiag_inc: x-, x+, y-, y+
            auto nb = [&](int m, float kk, float sg, bool xdir) {
                acc_inc(kk, sg, xdir, c, sm.sE[m], sm.sGx[m], sm.sGy[m], DP{sm.sXX[m], sm.sXY[m], sm.sYY[m]}, S0, S1,
                        S2);
            };
            nb(n - 1, L.kx, +1.0f, true);
            nb(n + 1, L.kx, -1.0f, true);
            nb(n - kMrSW, L.ky, +1.0f, false);
            nb(n + kMrSW, L.ky, -1.0f, false);
            float NE, NFx, NFy, NT;
            n_from_sums_with(ph, L, S0, S1, S2, sm.sWT[n], sm.sE[n], sm.sGx[n], sm.sGy[n], sm.sT[n], own[it][0],
                             own[it][1], NE, NFx, NFy, NT);
            oE = fmaf(sgn, NE, own[it][2]);
            oFx = fmaf(sgn, NFx, own[it][3]);
            oFy = fmaf(sgn, NFy, own[it][4]);
            oT = fmaf(sgn, NT, own[it][5]);
        }
        res[it][0] = oE;
        res[it][1] = oFx;
        res[it][2] = oFy;
        res[it][3] = oT;
    }
    __syncthreads();  // every closure increment has been read
#pragma unroll
    for (int it = 0; it < RPT; ++it) {
        const int q = threadIdx.x + it * kMrThreads;
        if (q < NR) {
            sm.sXX[q] = res[it][0];
            sm.sXY[q] = res[it][1];
            sm.sYY[q] = res[it][2];
            sm.qT[q] = res[it][3];
        }
    }
    __syncthreads();
    // restriction: the 12 fields of the tile's coarse cells, three per thread (a wave-uniform triple of fields)
    constexpr int NC = kMrCW * kMrCH;
    static_assert(kMrThreads == 4 * NC, "four groups of threads, three restricted fields each");
    const int cc = threadIdx.x % NC, grp = threadIdx.x / NC;
    const int ci = cc % kMrCW, cj = cc / kMrCW, I = I0 + ci, J = J0 + cj;
    if ((INTERIOR || (I < nxc && J < nyc)) && live) {
        float wx[3], wy[3];
        if (INTERIOR) {  // the weights rweights32 gives inside the grid
#pragma unroll
            for (int m = 0; m < 3; ++m) wx[m] = wy[m] = (m == 1) ? 0.5f : 0.25f;
        } else {
            int ix[3], iy[3];
            rweights32(I, L.nx, px != 0, ix, wx);
            rweights32(J, L.ny, py != 0, iy, wy);
        }
        auto restrict12 = [&](const float* src, bool staged, float* dst) {
            float s = 0.0f;
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                float v[3];
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    v[a] = staged ? src[centre(2 * ci + a - 1, 2 * cj + bb - 1)]
                                  : src[(2 * cj + bb) * kMrRW + 2 * ci + a];
                const float t = fmaf(wx[2], v[2], fmaf(wx[1], v[1], wx[0] * v[0]));
                s = fmaf(wy[bb], t, s);
            }
            stf(dst, (uint32_t)J * (uint32_t)nxc + (uint32_t)I, s);
        };
        if (grp == 0) {
            restrict12(sm.sWE, true, wc.E);
            restrict12(sm.sWFx, true, wc.Fx);
            restrict12(sm.sWFy, true, wc.Fy);
        } else if (grp == 1) {
            restrict12(sm.sWT, true, wc.T);
            restrict12(sm.sE, true, dc.E);
            restrict12(sm.sGx, true, dc.Fx);
        } else if (grp == 2) {
            restrict12(sm.sGy, true, dc.Fy);
            restrict12(sm.sT, true, dc.T);
            restrict12(sm.sXX, false, gc.E);
        } else {
            restrict12(sm.sXY, false, gc.Fx);
            restrict12(sm.sYY, false, gc.Fy);
            restrict12(sm.qT, false, gc.T);
        }
    }
}

__global__ __launch_bounds__(kMrThreads) void k_mx_residual_restrict(Phys ph, Lvl32 L, CSoa32 w, CSoa32 d, CSoa32 X,
                                                                     float sgn, int px, int py, Soa32 wc, Soa32 dc,
                                                                     Soa32 gc, const int* __restrict__ active)
{
    __shared__ MrLds sm;
    const bool live = active[mx_lane_zero()] != 0;
    const int ntx = (L.nx / 2 + kMrCW - 1) / kMrCW;
    const int b = (int)xcd_block();
    const int I0 = (b % ntx) * kMrCW, J0 = (b / ntx) * kMrCH;
    if (mr_interior(L, I0, J0))
        mx_residual_restrict_tile<true>(sm, ph, L, w, d, X, sgn, px, py, wc, dc, gc, I0, J0, live);
    else
        mx_residual_restrict_tile<false>(sm, ph, L, w, d, X, sgn, px, py, wc, dc, gc, I0, J0, live);
}

// Batched: work-list entries are the 32 x 4 coarse tiles of level `level` of
// each problem; level - 1's residual (r32 - N(d) on the finest level, else
// g - N_w(e)) is formed and restricted with w and the correction into (w, d, g).
__global__ __launch_bounds__(kMrThreads) void kbm_residual_restrict(const BProb* __restrict__ P,
                                                                    const BSlot32* __restrict__ S32,
                                                                    const uint32_t* __restrict__ wl, int nwl,
                                                                    int level, int d0_sel)
{
    __shared__ MrLds sm;
    for (int w_ = blockIdx.x; w_ < nwl; w_ += gridDim.x) {
        const uint32_t item = wl[w_];
        const int p = (int)(item >> kTileBits);
        const uint32_t tile = item & ((1u << kTileBits) - 1u);
        const BProb& pb = P[p];
        if (pb.ctrl->active == 0) continue;
        const BSlot32& c = S32[p * kMaxLevels + level];
        const BSlot32& f = S32[p * kMaxLevels + level - 1];
        const Soa32& w = (level == 1) ? f.base : f.w;
        const Soa32& d = (level == 1) ? pickA(f, d0_sel) : f.e;
        const Soa32& X = (level == 1) ? f.r32 : f.g;
        const uint32_t ntx = (uint32_t)((f.L.nx / 2 + kMrCW - 1) / kMrCW);
        // one variant only: two inlined into the work-list loop cost registers (130 against 79 VGPRs)
        mx_residual_restrict_tile<false>(sm, pb.ph, f.L, cs(w), cs(d), cs(X), -1.0f, pb.px, pb.py, c.w, c.d, c.g,
                                         (int)(tile % ntx) * kMrCW, (int)(tile / ntx) * kMrCH, true);
        __syncthreads();  // the next tile of this block reuses the LDS
    }
}

// Batched staged correction sweep (d given): work-list entries are the 64 x TY
// tiles of each problem's finest level.
template <int TY>
__global__ __launch_bounds__(kMxTX * TY) void kbm_sweep_lds(const BProb* __restrict__ P,
                                                           const BSlot32* __restrict__ S32,
                                                           const uint32_t* __restrict__ wl, int nwl, int in_sel,
                                                           int out_sel)
{
    __shared__ MxTile<TY> q;
    for (int w_ = blockIdx.x; w_ < nwl; w_ += gridDim.x) {
        const uint32_t item = wl[w_];
        const int p = (int)(item >> kTileBits);
        const uint32_t tile = item & ((1u << kTileBits) - 1u);
        const BProb& pb = P[p];
        if (pb.ctrl->active == 0) continue;
        const BSlot32& s = S32[p * kMaxLevels];
        const uint32_t ntx = (uint32_t)((s.L.nx + kMxTX - 1) / kMxTX);
        const int i0 = (int)(tile % ntx) * kMxTX, j0 = (int)(tile / ntx) * TY;
        mx_stage_tile<TY>(q, pb.ph, s.L, cs(s.base), cs(pickA(s, in_sel)), i0, j0);
        __syncthreads();
        mx_tile_sweep<TY>(q, pb.ph, s.L, cs(s.base), cs(pickA(s, in_sel)), cs(s.r32), 0.0f, 1.0f, (float)pb.omega,
                          pickA(s, out_sel), i0, j0);
        __syncthreads();  // the next tile of this block reuses the LDS
    }
}

// level 0: rho0 = r32 - N(d) (d = pickA(in_sel)); level >= 1: rho = g - N(pick32(in_sel)).
__global__ __launch_bounds__(kBlock32) void kbm_apply(const BProb* __restrict__ P, const BSlot32* __restrict__ S32,
                                                      const uint32_t* __restrict__ wl, int nwl, int level, int in_sel)
{
    M1_BATCH_LOOP(wl, nwl)
    const BSlot32& s = S32[p * kMaxLevels + level];
    if (k >= (uint32_t)s.L.nx * (uint32_t)s.L.ny) continue;
    int i, j;
    ij_of(s.L.nx, s.L.sh, k, i, j);
    if (level == 0) mx_apply_cell<2>(pb.ph, s.L, cs(s.base), cs(pickA(s, in_sel)), cs(s.r32), -1.0f, s.rho0, k, i, j);
    else mx_apply_cell<2>(pb.ph, s.L, cs(s.w), cs(pick32(s, in_sel)), cs(s.g), -1.0f, s.rho, k, i, j);
    }
}

// Into `level`: base w, correction d and R(rho) from level-1 (level 1: the
// finest base32, pickA(d0_sel), rho0; deeper: w, the pre-smoothed e, rho).
__global__ __launch_bounds__(kBlock32) void kbm_restrict(const BProb* __restrict__ P, const BSlot32* __restrict__ S32,
                                                         const uint32_t* __restrict__ wl, int nwl, int level,
                                                         int d0_sel)
{
    M1_BATCH_LOOP(wl, nwl)
    const BSlot32& c = S32[p * kMaxLevels + level];
    const BSlot32& f = S32[p * kMaxLevels + level - 1];
    if (k >= (uint32_t)c.L.nx * (uint32_t)c.L.ny) continue;
    const Soa32& w = (level == 1) ? f.base : f.w;
    const Soa32& d = (level == 1) ? pickA(f, d0_sel) : f.e;
    const Soa32& r = (level == 1) ? f.rho0 : f.rho;
    const float* in[12] = {w.E, w.Fx, w.Fy, w.T, d.E, d.Fx, d.Fy, d.T, r.E, r.Fx, r.Fy, r.T};
    float* out[12] = {c.w.E, c.w.Fx, c.w.Fy, c.w.T, c.d.E, c.d.Fx, c.d.Fy, c.d.T, c.g.E, c.g.Fx, c.g.Fy, c.g.T};
    mx_restrict_cell<2, 12>(f.L.nx, f.L.ny, f.L.sh, pb.px, pb.py, in, out, k);
    }
}

__global__ __launch_bounds__(kBlock32) void kbm_pseudo(const BProb* __restrict__ P, const BSlot32* __restrict__ S32,
                                                       const uint32_t* __restrict__ wl, int nwl, int level,
                                                       int in_sel, int out_sel, int first)
{
    M1_BATCH_LOOP(wl, nwl)
    const BSlot32& s = S32[p * kMaxLevels + level];
    if (k >= (uint32_t)s.L.nx * (uint32_t)s.L.ny) continue;
    int i, j;
    ij_of(s.L.nx, s.L.sh, k, i, j);
    const float dt = (float)pb.ctrl->dtau;
    if (first)
        mx_pseudo_cell<2, true>(pb.ph, s.L, cs(s.w), s.g, s.fr, cs(pick32(s, in_sel)), pick32(s, out_sel), dt,
                                (float)pb.reach, pb.local, k, i, j);
    else
        mx_pseudo_cell<2, false>(pb.ph, s.L, cs(s.w), s.g, s.fr, cs(pick32(s, in_sel)), pick32(s, out_sel), dt,
                                 (float)pb.reach, pb.local, k, i, j);
    }
}

// Correction of `level` >= 1 from level+1, in place on the pre-smoothed e.
__global__ __launch_bounds__(kBlock32) void kbm_prolong(const BProb* __restrict__ P, const BSlot32* __restrict__ S32,
                                                        const uint32_t* __restrict__ wl, int nwl, int level)
{
    M1_BATCH_LOOP(wl, nwl)
    const BSlot32& f = S32[p * kMaxLevels + level];
    const BSlot32& c = S32[p * kMaxLevels + level + 1];
    if (k >= (uint32_t)f.L.nx * (uint32_t)f.L.ny) continue;
    mx_prolong_cell<2>(pb.ph, f.L.nx, f.L.ny, f.L.sh, pb.px, pb.py, (float)pb.eta, cs(f.w), cs(f.e),
                       cs(coarse_final(pb, c, level)), cs(c.d), f.e, k);
    }
}

// Finest-level correction of pickA(e_sel) in place, admissibility against the FP64 state.
__global__ __launch_bounds__(kBlock32) void kbm_prolong_fine(const BProb* __restrict__ P, const BSlot* __restrict__ S,
                                                             const BSlot32* __restrict__ S32,
                                                             const uint32_t* __restrict__ wl, int nwl, int e_sel)
{
    M1_BATCH_LOOP(wl, nwl)
    const BSlot& s = S[p * kMaxLevels];
    const BSlot32& f = S32[p * kMaxLevels];
    const BSlot32& c = S32[p * kMaxLevels + 1];
    if (k >= (uint32_t)s.L.nx * (uint32_t)s.L.ny) continue;
    const Soa32& e = pickA(f, e_sel);
    mx_prolong_fine_cell<2>(pb.ph, s.L.nx, s.L.ny, s.L.sh, pb.px, pb.py, pb.eta, cs(pb.ctrl->flip ? s.x1 : s.x0),
                            cs(e), cs(coarse_final(pb, c, 0)), cs(c.d), e, k, true);
    }
}

// One block per problem with a tail: the bottom of its V-cycle.
__global__ __launch_bounds__(256) void kbm_tail(const BProb* __restrict__ P, const int* __restrict__ plist)
{
    const BProb& pb = P[plist[blockIdx.x]];
    if (pb.ctrl->active == 0) return;
    mx_tail_body<2>(*pb.tail32, (float)pb.ctrl->dtau);
}

// ===========================================================================
#define MX_DISPATCH(DIM_, KERNEL, GRID, ...)                                                            \
    do {                                                                                                \
        if ((DIM_) == 2) hipLaunchKernelGGL(KERNEL<2>, dim3(GRID), dim3(kBlock32), 0, st, __VA_ARGS__); \
        else hipLaunchKernelGGL(KERNEL<1>, dim3(GRID), dim3(kBlock32), 0, st, __VA_ARGS__);            \
    } while (0)

bool launch_mx_resid(hipStream_t st, int dim, const Phys& ph, const Lvl& L, double eta, CSoa v, CSoa32 d, CSoa b,
                     Soa vnew, Soa32 base, Soa32 r32, double* partials, const int* active, const Lvl32* zL,
                     float zomega, Soa32 zd)
{
    MxZero z{};
    if (zL && zd.E) {
        if (d.E && d.E == zd.E) return false;
        z = MxZero{*zL, zomega, zd};
    }
    MX_DISPATCH(dim, k_mx_resid, nblk((int64_t)L.nx * L.ny), ph, L, eta, v, d, b, vnew, base, r32, partials, active,
                z);
    return true;
}

void launch_mx_sweep(hipStream_t st, int dim, const Phys& ph, const Lvl32& L, CSoa32 w, CSoa32 d, CSoa32 rhs,
                     float beta, float gamma, float omega, Soa32 out, const int* active)
{
    const int rows = mx_sweep_rows();
    if (dim == 2 && d.E && rows > 0) {
        const unsigned ntx = (unsigned)((L.nx + kMxTX - 1) / kMxTX), nty = (unsigned)((L.ny + rows - 1) / rows);
        const dim3 gl(ntx * nty), bl(kMxTX * rows);
#define M1_MX_SWEEP_LDS(R)                                                                                            \
    hipLaunchKernelGGL(k_mx_sweep_lds<R>, gl, bl, 0, st, ph, L, w, d, rhs, beta, gamma, omega, out, active)
        if (rows == 4) M1_MX_SWEEP_LDS(4);
        else if (rows == 8) M1_MX_SWEEP_LDS(8);
        else M1_MX_SWEEP_LDS(16);
#undef M1_MX_SWEEP_LDS
        return;
    }
    MX_DISPATCH(dim, k_mx_sweep, nblk((int64_t)L.nx * L.ny), ph, L, w, d, rhs, beta, gamma, omega, out, active);
}

bool launch_mx_sweep2(hipStream_t st, const Phys& ph, const Lvl32& L, CSoa32 w, CSoa32 d, CSoa32 rhs, float omega,
                      Soa32 out, const int* active)
{
    const int rows = pair_rows();
    if (rows == 0 || !d.E) return false;
    const unsigned ntx = (unsigned)((L.nx + kMxTX - 1) / kMxTX), nty = (unsigned)((L.ny + rows - 1) / rows);
    const dim3 gl(ntx * nty), bl(kMxTX * rows);
    if (rows == 4) hipLaunchKernelGGL(k_mx_sweep2_lds<4>, gl, bl, 0, st, ph, L, w, d, rhs, omega, out, active);
    else if (rows == 8) hipLaunchKernelGGL(k_mx_sweep2_lds<8>, gl, bl, 0, st, ph, L, w, d, rhs, omega, out, active);
    else hipLaunchKernelGGL(k_mx_sweep2_lds<16>, gl, bl, 0, st, ph, L, w, d, rhs, omega, out, active);
    return true;
}

void launch_mx_residual_restrict(hipStream_t st, const Phys& ph, const Lvl32& L, CSoa32 w, CSoa32 d, CSoa32 X,
                                 float sgn, int px, int py, Soa32 wc, Soa32 dc, Soa32 gc, const int* active)
{
    const int nxc = L.nx / 2, nyc = L.ny / 2;
    if (nxc < 1 || nyc < 1) return;
    const unsigned nb = (unsigned)((nxc + kMrCW - 1) / kMrCW) * (unsigned)((nyc + kMrCH - 1) / kMrCH);
    hipLaunchKernelGGL(k_mx_residual_restrict, dim3(nb), dim3(kMrThreads), 0, st, ph, L, w, d, X, sgn, px, py, wc, dc,
                       gc, active);
}

void launch_mx_apply(hipStream_t st, int dim, const Phys& ph, const Lvl32& L, CSoa32 w, CSoa32 d, CSoa32 X, float sgn,
                     Soa32 out, const int* active)
{
    MX_DISPATCH(dim, k_mx_apply, nblk((int64_t)L.nx * L.ny), ph, L, w, d, X, sgn, out, active);
}

void launch_mx_pseudo(hipStream_t st, int dim, const Phys& ph, const Lvl32& L, CSoa32 w, Soa32 g, Soa32 fr,
                      CSoa32 e, Soa32 out, double dtau, const double* dtau_dev, float reach, int local, int first,
                      const int* active)
{
    const int rows = mx_sweep_rows();
    if (dim == 2 && rows > 0 && (int64_t)L.nx * L.ny >= kMxPseudoLdsCells) {
        const unsigned ntx = (unsigned)((L.nx + kMxTX - 1) / kMxTX), nty = (unsigned)((L.ny + rows - 1) / rows);
        const dim3 gl(ntx * nty), bl(kMxTX * rows);
#define M1_MX_PSEUDO_LDS(R)                                                                                           \
    do {                                                                                                              \
        if (first)                                                                                                    \
            hipLaunchKernelGGL((k_mx_pseudo_lds<R, true>), gl, bl, 0, st, ph, L, w, g, fr, e, out, dtau_dev, reach,    \
                               local, active);                                                                        \
        else                                                                                                          \
            hipLaunchKernelGGL((k_mx_pseudo_lds<R, false>), gl, bl, 0, st, ph, L, w, g, fr, e, out, dtau_dev, reach,   \
                               local, active);                                                                        \
    } while (0)
        if (rows == 4) M1_MX_PSEUDO_LDS(4);
        else if (rows == 8) M1_MX_PSEUDO_LDS(8);
        else M1_MX_PSEUDO_LDS(16);
#undef M1_MX_PSEUDO_LDS
        return;
    }
    MX_DISPATCH(dim, k_mx_pseudo, nblk((int64_t)L.nx * L.ny), ph, L, w, g, fr, e, out, dtau, dtau_dev, reach, local,
                first, active);
}

void launch_mx_prolong(hipStream_t st, int dim, const Phys& ph, int nx, int ny, int px, int py, float eta, CSoa32 w,
                       CSoa32 e, CSoa32 ec, CSoa32 dc, Soa32 out, const int* active)
{
    MX_DISPATCH(dim, k_mx_prolong, nblk((int64_t)nx * ny), ph, nx, ny, row_shift(nx), px, py, eta, w, e, ec, dc, out,
                active);
}

bool launch_mx_prolong_sweep(hipStream_t st, const Phys& ph, const Lvl32& L, CSoa32 w, CSoa v, CSoa32 e, CSoa32 ec,
                             CSoa32 dc, int px, int py, double eta, CSoa32 rhs, float omega, Soa32 out,
                             const int* active)
{
    // staged when the mixed sweeps are; 64 x 8 tiles whatever their rows (the prolongation is recomputed on the
    // halo: 8 rows measured faster than 4 or 16)
    constexpr int rows = 8;
    if (mx_sweep_rows() <= 0) return false;
    const unsigned ntx = (unsigned)((L.nx + kMxTX - 1) / kMxTX), nty = (unsigned)((L.ny + rows - 1) / rows);
    hipLaunchKernelGGL(k_mx_prolong_sweep_lds<rows>, dim3(ntx * nty), dim3(kMxTX * rows), 0, st, ph, L, w, v, e, ec,
                       dc, row_shift(L.nx), px, py, eta, rhs, omega, out, active);
    return true;
}

void launch_mx_prolong_fine(hipStream_t st, int dim, const Phys& ph, int nx, int ny, int px, int py, double eta,
                            CSoa v, CSoa32 e, CSoa32 ec, CSoa32 dc, Soa32 out, const int* active)
{
    MX_DISPATCH(dim, k_mx_prolong_fine, nblk((int64_t)nx * ny), ph, nx, ny, row_shift(nx), px, py, eta, v, e, ec, dc,
                out, active);
}

void launch_mx_restrict(hipStream_t st, int dim, int nxf, int nyf, int px, int py, const Fields32& F,
                        const int* active)
{
    const int64_t nc = (int64_t)(nxf / 2) * (dim == 2 ? nyf / 2 : 1);
    const dim3 g(nblk(nc)), b(kBlock32);
    const int shf = row_shift(nxf);
    if (dim == 2) {
        if (F.n == 12) hipLaunchKernelGGL((k_mx_restrict<2, 12>), g, b, 0, st, nxf, nyf, shf, px, py, F, active);
        else hipLaunchKernelGGL((k_mx_restrict<2, 2>), g, b, 0, st, nxf, nyf, shf, px, py, F, active);
    } else {
        if (F.n == 9) hipLaunchKernelGGL((k_mx_restrict<1, 9>), g, b, 0, st, nxf, nyf, shf, px, py, F, active);
        else hipLaunchKernelGGL((k_mx_restrict<1, 2>), g, b, 0, st, nxf, nyf, shf, px, py, F, active);
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

static unsigned bmgrid(int nwl) { return (unsigned)(nwl < 1 ? 1 : (nwl > batch_grid_cap() ? batch_grid_cap() : nwl)); }

void launch_bm_resid(hipStream_t st, const BProb* P, const BSlot* S, const BSlot32* S32, const uint32_t* wl, int nwl,
                     int pend_sel, int zero)
{
    if (nwl > 0)
        hipLaunchKernelGGL(kbm_resid, dim3(bmgrid(nwl)), dim3(kBlock32), 0, st, P, S, S32, wl, nwl, pend_sel, zero);
}
void launch_bm_residual_restrict(hipStream_t st, const BProb* P, const BSlot32* S32, const uint32_t* wl, int nwl,
                                 int level, int d0_sel)
{
    if (nwl > 0)
        hipLaunchKernelGGL(kbm_residual_restrict, dim3(bmgrid(nwl)), dim3(kMrThreads), 0, st, P, S32, wl, nwl, level,
                           d0_sel);
}

void launch_bm_sweep_lds(hipStream_t st, const BProb* P, const BSlot32* S32, const uint32_t* wl, int nwl, int in_sel,
                         int out_sel, int rows)
{
    if (nwl <= 0) return;
    const dim3 g(bmgrid(nwl)), b(kMxTX * rows);
    if (rows == 4) hipLaunchKernelGGL(kbm_sweep_lds<4>, g, b, 0, st, P, S32, wl, nwl, in_sel, out_sel);
    else if (rows == 8) hipLaunchKernelGGL(kbm_sweep_lds<8>, g, b, 0, st, P, S32, wl, nwl, in_sel, out_sel);
    else hipLaunchKernelGGL(kbm_sweep_lds<16>, g, b, 0, st, P, S32, wl, nwl, in_sel, out_sel);
}

void launch_bm_sweep(hipStream_t st, const BProb* P, const BSlot32* S32, const uint32_t* wl, int nwl, int in_sel,
                     int out_sel, int from_zero)
{
    if (nwl > 0)
        hipLaunchKernelGGL(kbm_sweep, dim3(bmgrid(nwl)), dim3(kBlock32), 0, st, P, S32, wl, nwl, in_sel, out_sel,
                           from_zero);
}
void launch_bm_apply(hipStream_t st, const BProb* P, const BSlot32* S32, const uint32_t* wl, int nwl, int level,
                     int in_sel)
{
    if (nwl > 0) hipLaunchKernelGGL(kbm_apply, dim3(bmgrid(nwl)), dim3(kBlock32), 0, st, P, S32, wl, nwl, level, in_sel);
}
void launch_bm_restrict(hipStream_t st, const BProb* P, const BSlot32* S32, const uint32_t* wl, int nwl, int level,
                        int d0_sel)
{
    if (nwl > 0)
        hipLaunchKernelGGL(kbm_restrict, dim3(bmgrid(nwl)), dim3(kBlock32), 0, st, P, S32, wl, nwl, level, d0_sel);
}
void launch_bm_pseudo(hipStream_t st, const BProb* P, const BSlot32* S32, const uint32_t* wl, int nwl, int level,
                      int in_sel, int out_sel, int first)
{
    if (nwl > 0)
        hipLaunchKernelGGL(kbm_pseudo, dim3(bmgrid(nwl)), dim3(kBlock32), 0, st, P, S32, wl, nwl, level, in_sel,
                           out_sel, first);
}
void launch_bm_prolong(hipStream_t st, const BProb* P, const BSlot32* S32, const uint32_t* wl, int nwl, int level)
{
    if (nwl > 0) hipLaunchKernelGGL(kbm_prolong, dim3(bmgrid(nwl)), dim3(kBlock32), 0, st, P, S32, wl, nwl, level);
}
void launch_bm_prolong_fine(hipStream_t st, const BProb* P, const BSlot* S, const BSlot32* S32, const uint32_t* wl,
                            int nwl, int e_sel)
{
    if (nwl > 0)
        hipLaunchKernelGGL(kbm_prolong_fine, dim3(bmgrid(nwl)), dim3(kBlock32), 0, st, P, S, S32, wl, nwl, e_sel);
}
void launch_bm_tail(hipStream_t st, const BProb* P, const int* plist, int np)
{
    if (np > 0) hipLaunchKernelGGL(kbm_tail, dim3(np), dim3(256), 0, st, P, plist);
}

}  // namespace m1
