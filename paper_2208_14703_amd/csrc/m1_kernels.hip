// m1_kernels.hip -- stencil kernels of the implicit M1 multigrid (gfx950).
//
// One-cell kernels run one thread per cell (256-thread blocks = 4 wave64s)
// over a 1-D launch in the XCD-aware block order of m1::xcd_block(); cell
// (i,j) = (t % nx, t / nx).  LDS-staged kernels (k_relax_lds, k_apply_lds,
// k_residual_restrict) own 2-D tiles and evaluate each point's closure once;
// k_relax2_lds (and its batched form) runs two consecutive finest sweeps per
// launch; k_smooth_tb runs a whole smoothing leg of a small level per launch.  Fields
// are SoA FP64 arrays.  The work is a memory-bound nonlinear 5-point stencil:
// no MFMA.  The per-cell bodies are __device__ functions shared by all these
// kernels, the batched kernels and k_tail, which runs the whole bottom of the
// V-cycle (every level small enough for one workgroup) in a single launch
// with block barriers between the phases.
//
// Cycle kernels take a device flag `active` (no effect when it is 0) and a
// device pseudo-time step `dtau_dev` (both always valid pointers), so that
// whole V-cycles can be enqueued ahead of the host's convergence check.
#include <algorithm>
#include <atomic>
#include <cfloat>

#include "m1_cells.hpp"

namespace m1 {

constexpr int kBlock = 256;
// The bottom of the cycle holds at most a few hundred cells per level: one
// thread per cell, and 256 threads leave the per-cell body its full register
// file (a 1024-thread bound caps it at 128 VGPRs and it spills).
constexpr int kTailThreads = 256;

static inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }


// Level kernels other than the finest sweep read the stop flag (and the
// pseudo-time step) together with their data and gate only their stores on
// it: on the small coarse levels a flag test ahead of the loads would add a
// memory round trip to every launch.  (Kernels of cycles enqueued past
// convergence then compute but write nothing.)  `active` and `dtau_dev` are
// always valid device pointers here.  They are read through a per-lane offset
// of 0 that the compiler cannot see as uniform, which keeps them ordinary
// vector loads: these complete in order with the data loads, so their waits
// land at the first use and not ahead of the data loads.
__device__ __forceinline__ uint32_t lane_zero()
{
    uint32_t z = 0;
    asm("" : "+v"(z));
    return z;
}

// ===========================================================================
// Grid kernels
// ===========================================================================
__device__ __forceinline__ bool cell_of(const Lvl& L, uint32_t& k, int& i, int& j)
{
    k = (uint32_t)xcd_block() * kBlock + threadIdx.x;
    if (k >= (uint32_t)L.nx * (uint32_t)L.ny) return false;
    ij_of(L.nx, L.sh, k, i, j);
    return true;
}

// Jacobi sweep; NORM (the finest level's first sweep of a cycle, beta = 0,
// gamma = 1) also writes the block partials of |b - A(u)|^2 of its input.  Two
// instantiations: the plain sweep needs fewer registers (more waves in flight).
// FINE: the finest level's sweep (beta = 0, gamma = 1, no per-cell gamma) with
// those constants folded in (exact folds, so the results are unchanged).
template <int DIM, bool NORM, bool FINE>
__global__ __launch_bounds__(kBlock) void k_relax(Phys ph, Lvl L, CSoa rhs, const double* __restrict__ gcell,
                                                  double beta, double gamma, double omega, CSoa u, Soa out,
                                                  double* __restrict__ partials, const int* __restrict__ active)
{
    if (*active == 0) return;
    if (FINE) {
        gcell = nullptr;
        beta = 0.0;
        gamma = 1.0;
    }
    uint32_t k;
    int i, j;
    const bool in = cell_of(L, k, i, j);
    if (!NORM) {
        if (in) relax_cell<DIM>(ph, L, rhs, gcell, beta, gamma, omega, u, out, k, i, j);
        return;
    }
    double q = 0.0;
    if (in) q = relax_cell<DIM, true>(ph, L, rhs, gcell, beta, gamma, omega, u, out, k, i, j);
    block_partial(q, partials + xcd_block());
}

// One colour of a red-black Gauss-Seidel sweep of the finest level: the cells
// with (i + j) % 2 == colour take the relaxed Jacobi update of u (relax_values,
// the arithmetic of every sweep), the others keep their state.  With NORM every
// cell also adds its residual of u to the block partial (the first half of a
// cycle's first sweep measures the previous result).
template <int DIM, bool NORM>
__global__ __launch_bounds__(kBlock) void k_relax_colour(Phys ph, Lvl L, CSoa rhs, double omega, int colour, CSoa u,
                                                         Soa out, double* __restrict__ partials,
                                                         const int* __restrict__ active)
{
    if (*active == 0) return;
    uint32_t k;
    int i, j;
    const bool in = cell_of(L, k, i, j);
    double q = 0.0;
    if (in) {
        const bool mine = ((i + j) & 1) == colour;
        double E = ld(u.E, k), Fx = ld(u.Fx, k), Fy = (DIM == 2) ? ld(u.Fy, k) : 0.0, T = ld(u.T, k);
        if (mine || NORM) {
            double S0, S1, S2, nE, nFx, nFy, nT;
            offdiag<DIM>(ph, L, u, i, j, k, S0, S1, S2);
            const double Ein = E, Fxin = Fx, Fyin = Fy;
            auto cen = [&](int f) { return f == 0 ? Ein : (f == 1 ? Fxin : Fyin); };
            q = relax_values<DIM, NORM>(ph, L, rhs, 1.0, 0.0, omega, S0, S1, S2, T, cen, k, nE, nFx, nFy, nT);
            if (mine) {
                E = nE;
                Fx = nFx;
                Fy = nFy;
                T = nT;
            }
        }
        st(out.E, k, E);
        st(out.Fx, k, Fx);
        if (DIM == 2) st(out.Fy, k, Fy);
        st(out.T, k, T);
    }
    if (NORM) block_partial(q, partials + xcd_block());
}

// ---------------------------------------------------------------------------
// LDS-staged 2-D stencil kernels.  A block owns a 64 x TY tile.  The states of
// the tile and of its one-cell halo (boundary rule or periodic image applied)
// are loaded once and the closure of each is evaluated once; E, F and the rows
// of c^2 P go to LDS, and each cell sums its four neighbours' fluxes from there
// instead of evaluating four closures of its own.  Every cell's arithmetic,
// and its order, is that of the one-cell-per-thread kernels (the sums of
// offdiag via acc_x/acc_y, the updates relax_update/pseudo_update), so the
// results are the same to the bit.
constexpr int kLdsTX = 64;

template <int TY>
struct LdsTile {
    static constexpr int W = kLdsTX + 2, N = W * (TY + 2);
    double E[N], Fx[N], Fy[N], XX[N], XY[N], YY[N];
};

// Whether the 64 x TY tile at (i0, j0) and its one-cell halo lie inside the
// grid (no ghost, wrap or ragged edge).
__device__ __forceinline__ bool tile_interior(const Lvl& L, int ty, int i0, int j0)
{
    return i0 >= 1 && j0 >= 1 && i0 + kLdsTX + 1 <= L.nx && j0 + ty + 1 <= L.ny;
}

// The coarse corrections uc - vc an up-leg tile reads, staged once per block
// when the tile's coarse footprint lies inside the coarse grid (no wrap or
// clamp): CW x CH coarse cells from (i0 / 2 - 1, j0 / 2 - 1).
template <int TY>
struct CoarseStage {
    static constexpr int CW = kLdsTX / 2 + 3, CH = TY / 2 + 3, N = CW * CH;
    double E[N], Fx[N], Fy[N], T[N];
};
__device__ __forceinline__ bool coarse_stage_fits(const Lvl& L, int ty, int i0, int j0)
{
    return i0 >= 2 && j0 >= 2 && i0 + kLdsTX + 4 <= L.nx && j0 + ty + 4 <= L.ny;
}
template <int TY>
__device__ __forceinline__ void stage_coarse(CoarseStage<TY>& s, const Lvl& L, const CSoa& uc, const CSoa& vc, int i0,
                                             int j0)
{
    using S = CoarseStage<TY>;
    const int Ic0 = i0 / 2 - 1, Jc0 = j0 / 2 - 1, nxc = L.nx / 2;
    for (int c = threadIdx.x; c < S::N; c += kLdsTX * TY) {
        const uint32_t kc = (uint32_t)(Jc0 + c / S::CW) * (uint32_t)nxc + (uint32_t)(Ic0 + c % S::CW);
        s.E[c] = ld(uc.E, kc) - ld(vc.E, kc);
        s.Fx[c] = ld(uc.Fx, kc) - ld(vc.Fx, kc);
        s.Fy[c] = ld(uc.Fy, kc) - ld(vc.Fy, kc);
        s.T[c] = ld(uc.T, kc) - ld(vc.T, kc);
    }
}

// Stage the tile at (i0, j0) of state u.  UP: each gathered state is first
// corrected from the coarse level (uc, vc) and projected (prolong_value, as
// k_prolong_project) and its temperature kept in qT; with cst, from the staged
// coarse corrections (prolong_value_staged).  INTERIOR: the tile is
// tile_interior, and the side logic drops out (same arithmetic, same result).
template <int TY, bool UP, bool INTERIOR = false>
__device__ __forceinline__ void stage_tile(LdsTile<TY>& q, double* qT, const Phys& ph, const Lvl& L, const CSoa& u,
                                           int i0, int j0, const CSoa& uc, const CSoa& vc, int px, int py, double eta,
                                           const CoarseStage<TY>* cst = nullptr)
{
    static_assert(kLdsTX * TY >= 2 * kLdsTX + 2 * TY, "the halo needs 2 rows and 2 columns of threads");
    constexpr int W = LdsTile<TY>::W;
    const bool perx = ph.bc[0] == BC_PERIODIC, pery = ph.bc[2] == BC_PERIODIC;
    // region point (li, lj), li in [-1, 64], lj in [-1, TY]; points outside the
    // domain take the boundary rule of their side applied to the adjacent cell
    // (or the periodic image); corners and points past a ragged edge are unused
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
        double e = 0.0, fx = 0.0, fy = 0.0, xx = 0.0, xy = 0.0, yy = 0.0, tt = 0.0;
        if (need) {
            const uint32_t k = (uint32_t)gj * (uint32_t)L.nx + (uint32_t)gi;
            double le = ld(u.E, k), lfx = ld(u.Fx, k), lfy = ld(u.Fy, k);
            if (UP && cst) {
                double wE, wFx, wFy;
                prolong_value_staged(ph, L.nx, L.ny, eta, gi, gj, le, lfx, lfy, ld(u.T, k), cst->E, cst->Fx, cst->Fy,
                                     cst->T, i0 / 2 - 1, j0 / 2 - 1, CoarseStage<TY>::CW, wE, wFx, wFy, tt);
                le = wE;
                lfx = wFx;
                lfy = wFy;
            } else if (UP) {
                double wE, wFx, wFy;
                prolong_value<2>(ph, L.nx, L.ny, px, py, eta, gi, gj, le, lfx, lfy, ld(u.T, k), uc, vc, wE, wFx, wFy,
                                 tt);
                le = wE;
                lfx = wFx;
                lfy = wFy;
            }
            ghost_rule(ph, side, !(ox || oy), in_seg(L, side, side < 2 ? gj : gi), le, lfx, lfy, e, fx, fy);
            const C2P p = closure(ph.c, ph.c2, e, fx, fy);
            xx = p_xx(p, fx);
            xy = p_xy(p, fx, fy);
            yy = p_yy(p, fy);
        }
        const int c = (lj + 1) * W + li + 1;
        q.E[c] = e;
        q.Fx[c] = fx;
        q.Fy[c] = fy;
        q.XX[c] = xx;
        q.XY[c] = xy;
        q.YY[c] = yy;
        if (UP) qT[c] = tt;
    };
    const int t = threadIdx.x;
    gather(t % kLdsTX, t / kLdsTX);  // the tile
    if (t < 2 * kLdsTX) {            // halo rows below and above
        gather(t % kLdsTX, t < kLdsTX ? -1 : TY);
    } else if (t < 2 * kLdsTX + 2 * TY) {  // halo columns left and right
        const int r = t - 2 * kLdsTX;
        gather(r < TY ? -1 : kLdsTX, r % TY);
    }
}

// Off-diagonal sum of the cell at LDS index c, in the order of offdiag: x-, x+, y-, y+.
template <int TY>
__device__ __forceinline__ void tile_sums(const LdsTile<TY>& q, const Lvl& L, double c_light, int c, double& S0,
                                          double& S1, double& S2)
{
    constexpr int W = LdsTile<TY>::W;
    S0 = S1 = S2 = 0.0;
    acc_x(L.kx, c_light, +1.0, q.E[c - 1], q.Fx[c - 1], q.Fy[c - 1], q.XX[c - 1], q.XY[c - 1], S0, S1, S2);
    acc_x(L.kx, c_light, -1.0, q.E[c + 1], q.Fx[c + 1], q.Fy[c + 1], q.XX[c + 1], q.XY[c + 1], S0, S1, S2);
    acc_y(L.ky, c_light, +1.0, q.E[c - W], q.Fx[c - W], q.Fy[c - W], q.XY[c - W], q.YY[c - W], S0, S1, S2);
    acc_y(L.ky, c_light, -1.0, q.E[c + W], q.Fx[c + W], q.Fy[c + W], q.XY[c + W], q.YY[c + W], S0, S1, S2);
}

__device__ __forceinline__ void tile_origin(const Lvl& L, int ty, int& i0, int& j0)
{
    const int ntx = (L.nx + kLdsTX - 1) / kLdsTX;
    const int b = (int)xcd_block();
    i0 = (b % ntx) * kLdsTX;
    j0 = (b / ntx) * ty;
}

// Finest-level Jacobi sweep (beta = 0, gamma = 1, no norm).  UP: the first
// sweep after the coarse-grid correction, fused with it: the corrected state
// is never stored, the sweep proceeds from it.
template <int TY, bool UP>
__global__ __launch_bounds__(kLdsTX * TY) void k_relax_lds(Phys ph, Lvl L, CSoa rhs, double omega, CSoa u, Soa out,
                                                          const int* __restrict__ active, CSoa uc, CSoa vc, int px,
                                                          int py, double eta)
{
    constexpr int W = LdsTile<TY>::W;
    __shared__ LdsTile<TY> q;
    __shared__ double qT[UP ? LdsTile<TY>::N : 1];
    __shared__ CoarseStage<UP ? TY : 2> cs_;
    if (*active == 0) return;
    int i0, j0;
    tile_origin(L, TY, i0, j0);
    if (UP && coarse_stage_fits(L, TY, i0, j0)) {  // inside the grid, coarse corrections staged
        if constexpr (UP) {
            stage_coarse<TY>(cs_, L, uc, vc, i0, j0);
            __syncthreads();
            stage_tile<TY, UP, true>(q, qT, ph, L, u, i0, j0, uc, vc, px, py, eta, &cs_);
        }
    } else if (tile_interior(L, TY, i0, j0)) {
        stage_tile<TY, UP, true>(q, qT, ph, L, u, i0, j0, uc, vc, px, py, eta);
    } else {
        stage_tile<TY, UP>(q, qT, ph, L, u, i0, j0, uc, vc, px, py, eta);
    }
    __syncthreads();
    const int li = threadIdx.x % kLdsTX, lj = threadIdx.x / kLdsTX, i = i0 + li, j = j0 + lj;
    if (i >= L.nx || j >= L.ny) return;
    const uint32_t k = (uint32_t)j * (uint32_t)L.nx + (uint32_t)i;
    const int c = (lj + 1) * W + li + 1;
    double S0, S1, S2;
    tile_sums<TY>(q, L, ph.c, c, S0, S1, S2);
    auto cen = [&](int f) { return f == 0 ? q.E[c] : (f == 1 ? q.Fx[c] : q.Fy[c]); };
    relax_update<2, false>(ph, L, rhs, 1.0, 0.0, omega, S0, S1, S2, UP ? qT[c] : ld(u.T, k), cen, out, k);
}

// out = X + sgn A(v) without norm partials (as k_apply, 2-D); stores gated on
// the stop flag, read together with the data.
template <int TY>
__global__ __launch_bounds__(kLdsTX * TY) void k_apply_lds(Phys ph, Lvl L, CSoa v, CSoa X, double sgn, Soa out,
                                                          const int* __restrict__ active)
{
    constexpr int W = LdsTile<TY>::W;
    __shared__ LdsTile<TY> q;
    const bool live = active[lane_zero()] != 0;
    int i0, j0;
    tile_origin(L, TY, i0, j0);
    stage_tile<TY, false>(q, nullptr, ph, L, v, i0, j0, CSoa{}, CSoa{}, 0, 0, 0.0);
    __syncthreads();
    const int li = threadIdx.x % kLdsTX, lj = threadIdx.x / kLdsTX, i = i0 + li, j = j0 + lj;
    if (i >= L.nx || j >= L.ny) return;
    const uint32_t k = (uint32_t)j * (uint32_t)L.nx + (uint32_t)i;
    const int c = (lj + 1) * W + li + 1;
    double S0, S1, S2;
    tile_sums<TY>(q, L, ph.c, c, S0, S1, S2);
    apply_update<2>(ph, L, q.E[c], q.Fx[c], q.Fy[c], ld(v.T, k), S0, S1, S2, X, sgn, out, k, live);
}

// ---------------------------------------------------------------------------
// Two finest-level Jacobi sweeps in one launch (temporal blocking).  A block
// owns a 64 x TY tile of final cells.  It stages the states of the tile and of
// a two-cell halo (with closures), runs the first sweep on the tile and its
// one-cell ring, puts the ring points outside the domain through the boundary
// rule of the cell they border, and runs the second sweep on the tile from
// there.  The intermediate iterate never goes to memory: against two launches
// this saves one read and one write of the state, of the right-hand side and
// of the opacities per cell, for about 14 % more closures and sweeps (the
// ring).  Every point's arithmetic is that of k_relax_lds, so the result is
// the same to the bit as two sweeps of it.
//
// Which points are needed: the second sweep needs the first sweep's iterate on
// the final cells and their four neighbours (a "plus" around the tile); the
// first sweep needs the staged state on those and on their neighbours.  Points
// off the domain on a periodic side are the periodic images (real cells, swept
// like any other); on another side only the first layer exists, as a ghost of
// the cell it borders (rc_axis).
template <int TY>
struct Lds2 {
    static constexpr int W2 = kLdsTX + 4, N2 = W2 * (TY + 4);  // staged state: tile + 2-cell halo
    static constexpr int W1 = kLdsTX + 2, N1 = W1 * (TY + 2);  // first sweep's iterate: tile + ring
    double buf[6 * N2];  // E, Fx, Fy, XX, XY, YY; the iterate's arrays overwrite the staged ones
};

// Off-diagonal sum of the point at index c of a W-wide LDS region with arrays
// f[0..5] = E, Fx, Fy, XX, XY, YY, in the order of tile_sums.
template <int W>
__device__ __forceinline__ void lds_sums(const double* const* f, const Lvl& L, double c_light, int c, double& S0,
                                         double& S1, double& S2)
{
    S0 = S1 = S2 = 0.0;
    acc_x(L.kx, c_light, +1.0, f[0][c - 1], f[1][c - 1], f[2][c - 1], f[3][c - 1], f[4][c - 1], S0, S1, S2);
    acc_x(L.kx, c_light, -1.0, f[0][c + 1], f[1][c + 1], f[2][c + 1], f[3][c + 1], f[4][c + 1], S0, S1, S2);
    acc_y(L.ky, c_light, +1.0, f[0][c - W], f[1][c - W], f[2][c - W], f[4][c - W], f[5][c - W], S0, S1, S2);
    acc_y(L.ky, c_light, -1.0, f[0][c + W], f[1][c + W], f[2][c + W], f[4][c + W], f[5][c + W], S0, S1, S2);
}

__device__ __forceinline__ void lds_put(double* const* f, const Phys& ph, int c, double e, double fx, double fy)
{
    const C2P p = closure(ph.c, ph.c2, e, fx, fy);
    f[0][c] = e;
    f[1][c] = fx;
    f[2][c] = fy;
    f[3][c] = p_xx(p, fx);
    f[4][c] = p_xy(p, fx, fy);
    f[5][c] = p_yy(p, fy);
}

// Whether the two-sweep tile at (i0, j0) and its 2-cell halo lie inside the
// grid: then no ghost, wrap or ragged edge applies.
template <int TY>
__device__ __forceinline__ bool pair_interior(const Lvl& L, int i0, int j0)
{
    return i0 >= 2 && j0 >= 2 && i0 + kLdsTX + 2 <= L.nx && j0 + TY + 2 <= L.ny;
}

// The two sweeps of the tile at (i0, j0); every thread of the block calls it.
// INTERIOR: the tile is pair_interior, and the side logic drops out (the
// arithmetic, and so the result, is the same).
template <int TY, bool INTERIOR = false>
__device__ __forceinline__ void relax2_tile(Lds2<TY>& q, const Phys& ph, const Lvl& L, const CSoa& rhs, double omega,
                                            const CSoa& u, const Soa& out, int i0, int j0)
{
    using Q = Lds2<TY>;
    constexpr int NT = kLdsTX * TY, NR = 2 * kLdsTX + 2 * TY;  // threads; ring points
    static_assert(NR <= NT, "one ring point per thread");
    const bool perx = ph.bc[0] == BC_PERIODIC, pery = ph.bc[2] == BC_PERIODIC;
    const int xe = INTERIOR ? i0 + kLdsTX - 1 : min(i0 + kLdsTX, L.nx) - 1;  // the last final cell
    const int ye = INTERIOR ? j0 + TY - 1 : min(j0 + TY, L.ny) - 1;
    // the plus of half-widths (a, b) around the final cells holds (gi, gj)
    auto plus = [&](int gi, int gj, int a, int b) {
        return (gi >= i0 && gi <= xe && gj >= j0 - a && gj <= ye + a) ||
               (gi >= i0 - a && gi <= xe + a && gj >= j0 && gj <= ye) ||
               (b > 0 && gi >= i0 - b && gi <= xe + b && gj >= j0 - b && gj <= ye + b);
    };
    double* f2[6];
    double* f1[6];
    for (int a = 0; a < 6; ++a) {
        f2[a] = q.buf + a * Q::N2;
        f1[a] = q.buf + a * Q::N1;
    }
    // 1. stage the state (boundary rule on ghosts) and its closures
    for (int p = threadIdx.x; p < Q::N2; p += NT) {
        const int gi = i0 + p % Q::W2 - 2, gj = j0 + p / Q::W2 - 2;
        int si = gi, sj = gj;
        bool gx = false, gy = false, nx_ = true, ny_ = true;
        if (!INTERIOR) {
            rc_axis(gi, L.nx, perx, si, gx, nx_);
            rc_axis(gj, L.ny, pery, sj, gy, ny_);
        }
        if (plus(gi, gj, 2, 1) && nx_ && ny_ && !(gx && gy)) {
            const uint32_t k = (uint32_t)sj * (uint32_t)L.nx + (uint32_t)si;
            const int side = gx ? (gi < 0 ? 0 : 1) : (gj < 0 ? 2 : 3);
            double e, fx, fy;
            ghost_rule(ph, side, !(gx || gy), in_seg(L, side, side < 2 ? sj : si), ld(u.E, k), ld(u.Fx, k),
                       ld(u.Fy, k), e, fx, fy);
            lds_put(f2, ph, p, e, fx, fy);
        } else {  // unused (corners, past a ragged edge)
            for (int a = 0; a < 6; ++a) f2[a][p] = 0.0;
        }
    }
    __syncthreads();
    // 2. first sweep: item 0 is the thread's tile point, item 1 a ring point
    const int t = threadIdx.x;
    int li[2], lj[2], kind[2];  // kind: 0 unused, 1 swept, 2 ghost
    int gsx[2], gsy[2];         // ghost: the cell it borders (global), and its side
    double vE[2], vFx[2], vFy[2], vT[2];
    li[0] = t % kLdsTX;
    lj[0] = t / kLdsTX;
    if (t < kLdsTX) li[1] = t, lj[1] = -1;
    else if (t < 2 * kLdsTX) li[1] = t - kLdsTX, lj[1] = TY;
    else if (t < 2 * kLdsTX + TY) li[1] = -1, lj[1] = t - 2 * kLdsTX;
    else li[1] = kLdsTX, lj[1] = t - 2 * kLdsTX - TY;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        kind[m] = 0;
        vE[m] = vFx[m] = vFy[m] = vT[m] = 0.0;
        gsx[m] = gsy[m] = 0;
        if (m == 1 && t >= NR) continue;
        const int gi = i0 + li[m], gj = j0 + lj[m];
        if (!plus(gi, gj, 1, 0)) continue;
        int si = gi, sj = gj;
        bool gx = false, gy = false, nx_ = true, ny_ = true;
        if (!INTERIOR) {
            rc_axis(gi, L.nx, perx, si, gx, nx_);
            rc_axis(gj, L.ny, pery, sj, gy, ny_);
        }
        if (gx || gy) {  // the plus holds no corner: only one side is off the domain
            kind[m] = 2;
            gsx[m] = si;
            gsy[m] = sj;
            continue;
        }
        kind[m] = 1;
        const uint32_t k = (uint32_t)sj * (uint32_t)L.nx + (uint32_t)si;
        const int c = (lj[m] + 2) * Q::W2 + li[m] + 2;
        double S0, S1, S2;
        lds_sums<Q::W2>(f2, L, ph.c, c, S0, S1, S2);
        auto cen = [&](int f) { return f2[f][c]; };
        relax_values<2, false>(ph, L, rhs, 1.0, 0.0, omega, S0, S1, S2, ld(u.T, k), cen, k, vE[m], vFx[m], vFy[m],
                               vT[m]);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 2; ++m)
        if (kind[m] == 1) lds_put(f1, ph, (lj[m] + 1) * Q::W1 + li[m] + 1, vE[m], vFx[m], vFy[m]);
    // 3. ghosts of the iterate (only tiles on a non-periodic side have any)
    const bool edge = !INTERIOR && ((!perx && (i0 == 0 || xe == L.nx - 1)) || (!pery && (j0 == 0 || ye == L.ny - 1)));
    if (edge) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            if (kind[m] != 2) continue;
            const int gi = i0 + li[m], gj = j0 + lj[m];
            const int side = (gi < 0 || gi >= L.nx) ? (gi < 0 ? 0 : 1) : (gj < 0 ? 2 : 3);
            const int cb = (gsy[m] - j0 + 1) * Q::W1 + gsx[m] - i0 + 1;
            double e, fx, fy;
            ghost_rule(ph, side, false, in_seg(L, side, side < 2 ? gsy[m] : gsx[m]), f1[0][cb], f1[1][cb], f1[2][cb],
                       e, fx, fy);
            lds_put(f1, ph, (lj[m] + 1) * Q::W1 + li[m] + 1, e, fx, fy);
        }
    }
    __syncthreads();
    // 4. second sweep on the final cells
    const int i = i0 + li[0], j = j0 + lj[0];
    if (INTERIOR || (i < L.nx && j < L.ny)) {
        const uint32_t k = (uint32_t)j * (uint32_t)L.nx + (uint32_t)i;
        const int c = (lj[0] + 1) * Q::W1 + li[0] + 1;
        double S0, S1, S2;
        lds_sums<Q::W1>(f1, L, ph.c, c, S0, S1, S2);
        auto cen = [&](int f) { return f == 0 ? vE[0] : (f == 1 ? vFx[0] : vFy[0]); };
        relax_update<2, false>(ph, L, rhs, 1.0, 0.0, omega, S0, S1, S2, vT[0], cen, out, k);
    }
}

// Six waves per SIMD (three 512-thread blocks per CU at 8 rows; 80 VGPRs, a few
// values spilled to scratch) measured faster than the four the unconstrained
// register count leaves room for: the phases are latency-bound.
template <int TY>
__global__ __launch_bounds__(kLdsTX * TY) __attribute__((amdgpu_waves_per_eu(6))) void k_relax2_lds(
    Phys ph, Lvl L, CSoa rhs, double omega, CSoa u, Soa out, const int* __restrict__ active)
{
    __shared__ Lds2<TY> q;
    if (*active == 0) return;
    int i0, j0;
    tile_origin(L, TY, i0, j0);
    if (pair_interior<TY>(L, i0, j0)) relax2_tile<TY, true>(q, ph, L, rhs, omega, u, out, i0, j0);
    else relax2_tile<TY>(q, ph, L, rhs, omega, u, out, i0, j0);
}

// ---------------------------------------------------------------------------
// Finest-level residual fused with the restriction to level 1 (2-D).  A block
// owns a 32 x 4 tile of coarse cells, i.e. the fine cells 2I-1 .. 2I+1 of each
// coarse I of the tile.  It stages the fine states of the region around them
// (per axis wrapped where periodic, else the ghost one cell beyond the side),
// evaluating each closure once; computes the residual X + sgn A(u) of the
// fine cells the restriction reads (a point dropped at a non-periodic side
// reads the clamped cell, as restrict_cell does); and restricts u and the
// residual into (vc, rc) with the weights and the order of restrict_cell.
// The fine residual is never stored and u is read once.
constexpr int kRcW = 32, kRcH = 4;                       // coarse tile
constexpr int kRsW = 2 * kRcW + 3, kRsH = 2 * kRcH + 3;  // staged fine offsets -2 .. 2 kRc
constexpr int kRrW = 2 * kRcW + 1, kRrH = 2 * kRcH + 1;  // residual offsets -1 .. 2 kRc - 1
constexpr int kRcThreads = 512;


// LDS of one fused residual-restriction tile: the staged fine states (E, F)
// and their closures; once every residual is formed, the residual of point q
// goes to (sXX, sXY, sYY, qT)[q] (the closure arrays are no longer read).
// Temperatures are not staged: each residual point loads its own with its
// right-hand side and opacities, and the restriction of T reads them from the
// cache.  That keeps a block at 40 KB.
struct RcLds {
    static constexpr int NS = kRsW * kRsH, NR = kRrW * kRrH;
    double sE[NS], sFx[NS], sFy[NS], sXX[NS], sXY[NS], sYY[NS];
    double qT[NR];
};
static_assert(RcLds::NR <= RcLds::NS, "residuals are kept in the closure arrays");

// Whether every point the tile at (I0, J0) stages lies inside the grid: then no
// ghost, wrap or clamp applies, every residual point and coarse cell of the
// tile exists and the restriction weights are (1/4, 1/2, 1/4) on both axes.
__device__ __forceinline__ bool rc_interior(const Lvl& L, int I0, int J0)
{
    return I0 >= 1 && J0 >= 1 && 2 * (I0 + kRcW) <= L.nx - 1 && 2 * (J0 + kRcH) <= L.ny - 1;
}

// The fused residual and restriction of the coarse tile at (I0, J0) (all
// threads of the block take part; no thread returns early).  INTERIOR: the
// tile is rc_interior, and the side logic drops out; the arithmetic, and so
// the result, is the same.
template <bool INTERIOR>
__device__ __forceinline__ void residual_restrict_tile(RcLds& sm, const Phys& ph, const Lvl& L, const CSoa& u,
                                                       const CSoa& X, double sgn, int px, int py, const Soa& vc,
                                                       const Soa& rc, int I0, int J0, bool live)
{
    constexpr int NS = RcLds::NS, NR = RcLds::NR;
    constexpr int RPT = (NR + kRcThreads - 1) / kRcThreads;  // residual points per thread
    const int nxc = L.nx / 2, nyc = L.ny / 2;
    const int fi0 = 2 * I0, fj0 = 2 * J0;
    // A residual point's own loads (opacities, temperature, right-hand side); false for points past the grid,
    // which belong to no coarse cell.  A point dropped at a non-periodic side reads the clamped cell.
    auto own_point = [&](int it, double o[7]) {
        const int q = threadIdx.x + it * kRcThreads;
        const int gi = fi0 + q % kRrW - 1, gj = fj0 + q / kRrW - 1;
        const bool h = q < NR && (INTERIOR || (gi < L.nx && gj < L.ny));
#pragma unroll
        for (int m = 0; m < 7; ++m) o[m] = 0.0;
        if (h) {
            const int si = (INTERIOR || gi >= 0) ? gi : (px ? gi + L.nx : 0);
            const int sj = (INTERIOR || gj >= 0) ? gj : (py ? gj + L.ny : 0);
            const uint32_t k = (uint32_t)sj * (uint32_t)L.nx + (uint32_t)si;
            o[0] = ld(L.sa, k);
            o[1] = ld(L.ss, k);
            o[2] = ld(u.T, k);
            if (X.E) {
                o[3] = ld(X.E, k);
                o[4] = ld(X.Fx, k);
                o[5] = ld(X.Fy, k);
                o[6] = ld(X.T, k);
            }
        }
        return h;
    };
    // The first point's loads are issued before the staging, so that their latency overlaps it; the few
    // threads with a second point load it when they reach it (registers held across the staging cost
    // occupancy).
    double own0[7];
    const bool has0 = own_point(0, own0);
    for (int q = threadIdx.x; q < NS; q += kRcThreads) {
        const int gi = fi0 + q % kRsW - 2, gj = fj0 + q / kRsW - 2;
        int si = gi, sj = gj;
        bool hx = false, hy = false, nx_ = true, ny_ = true;
        if (!INTERIOR) {
            rc_axis(gi, L.nx, px != 0, si, hx, nx_);
            rc_axis(gj, L.ny, py != 0, sj, hy, ny_);
        }
        double e = 0.0, fx = 0.0, fy = 0.0, xx = 0.0, xy = 0.0, yy = 0.0;
        if (nx_ && ny_ && !(hx && hy)) {
            const int side = hx ? (gi < 0 ? 0 : 1) : (hy ? (gj < 0 ? 2 : 3) : 0);
            const uint32_t k = (uint32_t)sj * (uint32_t)L.nx + (uint32_t)si;
            ghost_rule(ph, side, !(hx || hy), in_seg(L, side, side < 2 ? sj : si), ld(u.E, k), ld(u.Fx, k),
                       ld(u.Fy, k), e, fx, fy);
            const C2P p = closure(ph.c, ph.c2, e, fx, fy);
            xx = p_xx(p, fx);
            xy = p_xy(p, fx, fy);
            yy = p_yy(p, fy);
        }
        sm.sE[q] = e;
        sm.sFx[q] = fx;
        sm.sFy[q] = fy;
        sm.sXX[q] = xx;
        sm.sXY[q] = xy;
        sm.sYY[q] = yy;
    }
    __syncthreads();
    // staged index of the cell a residual point (fine offsets ri, rj) reads
    auto centre = [&](int ri, int rj) {
        if (!INTERIOR && fi0 + ri < 0 && !px) ri += 1;
        if (!INTERIOR && fj0 + rj < 0 && !py) rj += 1;
        return (rj + 2) * kRsW + ri + 2;
    };
    double res[RPT][4];
#pragma unroll
    for (int it = 0; it < RPT; ++it) {
        const int q = threadIdx.x + it * kRcThreads;
        double rE = 0.0, rFx = 0.0, rFy = 0.0, rT = 0.0;
        double o[7];
        bool h = has0;
        if (it == 0) {
#pragma unroll
            for (int m = 0; m < 7; ++m) o[m] = own0[m];
        } else {
            h = own_point(it, o);
        }
        if (h) {
            const int c = centre(q % kRrW - 1, q / kRrW - 1);
            double S0 = 0.0, S1 = 0.0, S2 = 0.0;  // the order of offdiag: x-, x+, y-, y+
            acc_x(L.kx, ph.c, +1.0, sm.sE[c - 1], sm.sFx[c - 1], sm.sFy[c - 1], sm.sXX[c - 1], sm.sXY[c - 1], S0, S1,
                  S2);
            acc_x(L.kx, ph.c, -1.0, sm.sE[c + 1], sm.sFx[c + 1], sm.sFy[c + 1], sm.sXX[c + 1], sm.sXY[c + 1], S0, S1,
                  S2);
            acc_y(L.ky, ph.c, +1.0, sm.sE[c - kRsW], sm.sFx[c - kRsW], sm.sFy[c - kRsW], sm.sXY[c - kRsW],
                  sm.sYY[c - kRsW], S0, S1, S2);
            acc_y(L.ky, ph.c, -1.0, sm.sE[c + kRsW], sm.sFx[c + kRsW], sm.sFy[c + kRsW], sm.sXY[c + kRsW],
                  sm.sYY[c + kRsW], S0, S1, S2);
            apply_values_from<2>(ph, L, sm.sE[c], sm.sFx[c], sm.sFy[c], o[2], S0, S1, S2, o[0], o[1],
                                 X.E ? &o[3] : nullptr, sgn, rE, rFx, rFy, rT);
        }
        res[it][0] = rE;
        res[it][1] = rFx;
        res[it][2] = rFy;
        res[it][3] = rT;
    }
    __syncthreads();  // every closure has been read
#pragma unroll
    for (int it = 0; it < RPT; ++it) {
        const int q = threadIdx.x + it * kRcThreads;
        if (q < NR) {
            sm.sXX[q] = res[it][0];
            sm.sXY[q] = res[it][1];
            sm.sYY[q] = res[it][2];
            sm.qT[q] = res[it][3];
        }
    }
    __syncthreads();
    // restriction: the 8 fields of the tile's coarse cells, two per thread (a wave-uniform pair of fields)
    constexpr int NC = kRcW * kRcH;
    static_assert(kRcThreads == 4 * NC, "four groups of threads, two restricted fields each");
    const int cc = threadIdx.x % NC, grp = threadIdx.x / NC;
    const int ci = cc % kRcW, cj = cc / kRcW, I = I0 + ci, J = J0 + cj;
    if ((INTERIOR || (I < nxc && J < nyc)) && live) {
        int ix[3], iy[3];
        double wx[3], wy[3];
        if (INTERIOR) {  // the weights rweights gives inside the grid
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                ix[m] = 2 * I - 1 + m;
                iy[m] = 2 * J - 1 + m;
                wx[m] = wy[m] = (m == 1) ? 0.5 : 0.25;
            }
        } else {
            rweights(I, L.nx, px != 0, ix, wx);
            rweights(J, L.ny, py != 0, iy, wy);
        }
        // fine cell 2I-1+a, 2J-1+b: residual index (2cj+b) kRrW + 2ci+a, staged cell centre(2ci+a-1, 2cj+b-1),
        // global cell (ix[a], iy[b]); all three name the cells restrict_cell reads, in its order
        auto restrict9 = [&](auto&& value, double* dst) {
            double s = 0.0;
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                double v[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) v[a] = value(a, bb);
                const double t = fma(wx[2], v[2], fma(wx[1], v[1], wx[0] * v[0]));
                s = fma(wy[bb], t, s);
            }
            st(dst, (uint32_t)J * (uint32_t)nxc + (uint32_t)I, s);
        };
        auto staged = [&](const double* src) {
            return [&, src](int a, int bb) { return src[centre(2 * ci + a - 1, 2 * cj + bb - 1)]; };
        };
        auto resid = [&](const double* src) {
            return [&, src](int a, int bb) { return src[(2 * cj + bb) * kRrW + 2 * ci + a]; };
        };
        if (grp == 0) {
            restrict9(staged(sm.sE), vc.E);
            restrict9(staged(sm.sFx), vc.Fx);
        } else if (grp == 1) {
            restrict9(staged(sm.sFy), vc.Fy);
            restrict9([&](int a, int bb) { return ld(u.T, (uint32_t)iy[bb] * (uint32_t)L.nx + (uint32_t)ix[a]); },
                      vc.T);
        } else if (grp == 2) {
            restrict9(resid(sm.sXX), rc.E);
            restrict9(resid(sm.sXY), rc.Fx);
        } else {
            restrict9(resid(sm.sYY), rc.Fy);
            restrict9(resid(sm.qT), rc.T);
        }
    }
}

__global__ __launch_bounds__(kRcThreads) void k_residual_restrict(Phys ph, Lvl L, CSoa u, CSoa X, double sgn, int px,
                                                                  int py, Soa vc, Soa rc,
                                                                  const int* __restrict__ active)
{
    __shared__ RcLds sm;
    const bool live = active[lane_zero()] != 0;
    const int ntx = (L.nx / 2 + kRcW - 1) / kRcW;
    const int b = (int)xcd_block();
    const int I0 = (b % ntx) * kRcW, J0 = (b / ntx) * kRcH;
    if (rc_interior(L, I0, J0)) residual_restrict_tile<true>(sm, ph, L, u, X, sgn, px, py, vc, rc, I0, J0, live);
    else residual_restrict_tile<false>(sm, ph, L, u, X, sgn, px, py, vc, rc, I0, J0, live);
}


// One pseudo-time step; `first`: also form the FAS right-hand side in f (u = v_l).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_pseudo(Phys ph, Lvl L, Soa f, CSoa u, Soa out, double dtau,
                                                   const double* __restrict__ dtau_dev, double reach, int local,
                                                   int first, Soa rs, double* __restrict__ gs,
                                                   const int* __restrict__ active)
{
    const uint32_t z = lane_zero();
    const double dt = dtau_dev[z];
    const bool live = active[z] != 0;
    uint32_t k;
    int i, j;
    if (!cell_of(L, k, i, j)) return;
    if (first) pseudo_cell<DIM, true>(ph, L, cs(f), f, u, out, dt, reach, local, rs, gs, k, i, j, live);
    else pseudo_cell<DIM, false>(ph, L, cs(f), f, u, out, dt, reach, local, rs, gs, k, i, j, live);
}

// LDS-staged pseudo-time step (2-D, large levels): the staging of k_relax_lds
// (state of a 64 x TY tile and its halo, closures once per point); each cell
// sums its neighbours from LDS in the order of offdiag and finishes as
// pseudo_cell, so the result is that of k_pseudo to the bit.  u and out must
// not alias.  Used from 512 K cells up: the 512^2 step is latency-bound and
// measured slightly slower staged.
constexpr int64_t kPseudoLdsCells = 524288;

template <int TY, bool FIRST>
__global__ __launch_bounds__(kLdsTX * TY) void k_pseudo_lds(Phys ph, Lvl L, Soa f, CSoa u, Soa out,
                                                           const double* __restrict__ dtau_dev, double reach,
                                                           int local, Soa rs, double* __restrict__ gs,
                                                           const int* __restrict__ active)
{
    constexpr int W = LdsTile<TY>::W;
    __shared__ LdsTile<TY> q;
    const uint32_t z = lane_zero();
    const double dt = dtau_dev[z];
    const bool live = active[z] != 0;
    int i0, j0;
    tile_origin(L, TY, i0, j0);
    if (tile_interior(L, TY, i0, j0)) stage_tile<TY, false, true>(q, nullptr, ph, L, u, i0, j0, CSoa{}, CSoa{}, 0, 0, 0.0);
    else stage_tile<TY, false>(q, nullptr, ph, L, u, i0, j0, CSoa{}, CSoa{}, 0, 0, 0.0);
    __syncthreads();
    const int li = threadIdx.x % kLdsTX, lj = threadIdx.x / kLdsTX, i = i0 + li, j = j0 + lj;
    if (i >= L.nx || j >= L.ny) return;
    const uint32_t k = (uint32_t)j * (uint32_t)L.nx + (uint32_t)i;
    const int c = (lj + 1) * W + li + 1;
    double S0, S1, S2;
    tile_sums<TY>(q, L, ph.c, c, S0, S1, S2);
    pseudo_update<2, FIRST>(ph, L, cs(f), f, q.E[c], q.Fx[c], q.Fy[c], ld(u.T, k), S0, S1, S2, out, dt, reach, local,
                            rs, gs, k, live);
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_apply(Phys ph, Lvl L, CSoa v, CSoa X, double sgn, Soa out,
                                                  double* __restrict__ partials, const int* __restrict__ active)
{
    const bool live = active[lane_zero()] != 0;
    uint32_t k;
    int i, j;
    double q = 0.0;
    if (cell_of(L, k, i, j)) q = apply_cell<DIM>(ph, L, v, X, sgn, out, k, i, j, live);
    if (partials && live) block_partial(q, partials + xcd_block());
}

__global__ __launch_bounds__(1024) void k_norm_finalize(const double* __restrict__ partials, int n,
                                                        double* __restrict__ out)
{
    const double t = block_sum(partials, n);
    if (threadIdx.x == 0) out[0] = sqrt(t);
}

// End of a V-cycle: finish the residual norm and update the cycle control
// (pseudo-time step adaptation, stopping test, cycle count).
__global__ __launch_bounds__(1024) void k_norm_control(const double* __restrict__ partials, int n, Ctrl* ctrl)
{
    if (ctrl->active == 0) return;
    const double r = sqrt(block_sum(partials, n));
    if (threadIdx.x == 0) ctrl_update(ctrl, r);
}

template <int DIM, int NF>
__global__ __launch_bounds__(kBlock) void k_restrict(int nxf, int nyf, int shf, int px, int py, Fields F,
                                                     const int* __restrict__ active)
{
    const bool live = active[lane_zero()] != 0;
    const uint32_t nc = (uint32_t)(nxf / 2) * (uint32_t)((DIM == 2) ? nyf / 2 : 1);
    const uint32_t k = (uint32_t)xcd_block() * kBlock + threadIdx.x;
    if (k >= nc) return;
    restrict_cell<DIM, NF>(nxf, nyf, shf, px, py, F.in, F.out, k, live);
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_prolong_project(Phys ph, int nx, int ny, int sh, int px, int py,
                                                            double eta, CSoa u, CSoa uc, CSoa vc, Soa out,
                                                            const int* __restrict__ active)
{
    const bool live = active[lane_zero()] != 0;
    const uint32_t k = (uint32_t)xcd_block() * kBlock + threadIdx.x;
    if (k >= (uint32_t)nx * (uint32_t)ny) return;
    prolong_cell<DIM>(ph, nx, ny, sh, px, py, eta, u, uc, vc, out, k, live);
}

template <int DIM>
__global__ __launch_bounds__(kTailThreads) void k_tail(const TailArgs* __restrict__ Ap, double dtau,
                                                       const double* __restrict__ dtau_dev,
                                                       const int* __restrict__ active)
{
    const double dt = *dtau_dev;
    if (*active == 0) return;
    tail_body<DIM>(*Ap, dt);
}

// ---------------------------------------------------------------------------
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
// all finite); *bad must hold UINT64_MAX on entry.
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

__global__ void k_ctrl_init(Ctrl* ctrl, Ctrl init) { *ctrl = init; }

// ===========================================================================
// LDS-tiled smoothing of one coarse level (2-D): all m pseudo-time steps of a
// smoothing leg in one launch.  A block owns a 16x16 tile and loads it with a
// halo of M = m cells; step s recomputes the region M - s cells around the
// tile, so no step needs another block's result (temporal blocking; the halo
// work is redundant).  LEG kLegDown: the first step forms the FAS right-hand
// side from R(rbar), read from `fr` and written to `f` (other tiles still read
// fr).  kLegUp: the load applies the prolongation and projection from level
// l + 1 (uc, vc) to the level's pre-smoothed iterate `u`.  kLegPlain: m steps
// from `u` with the right-hand side `fr` (a later visit of the level in a W- or
// F-cycle).  The per-cell arithmetic is that of the one-step kernels, so the
// results are the same to the bit.  Requires nx, ny multiples of 16, at least
// 32; u and out distinct.
constexpr int kTbTile = 16;
constexpr int kTbThreads = 512;

template <int M, int LEG>
__global__ __launch_bounds__(kTbThreads) void k_smooth_tb(Phys ph, Lvl L, CSoa fr, Soa f, CSoa u, Soa out,
                                                           const double* __restrict__ dtau_dev, double reach,
                                                           int local, CSoa uc, CSoa vc, int px, int py, double eta,
                                                           const int* __restrict__ active)
{
    constexpr bool UP = LEG == kLegUp;
    constexpr int W = kTbTile + 2 * M, NC = W * W;
    __shared__ double sE[2][NC], sFx[2][NC], sFy[2][NC], sT[2][NC];
    __shared__ double qE[NC], qFx[NC], qFy[NC], qT[NC], qa[NC], qs[NC];
    const uint32_t z = lane_zero();
    const double dt = dtau_dev[z];
    const bool live = active[z] != 0;
    const int ntx = L.nx / kTbTile;
    const int b = (int)xcd_block();
    const int bx = b % ntx, by = b / ntx;
    const int x0 = bx * kTbTile - M, y0 = by * kTbTile - M;
    // global cell of region point (li, lj), wrapped across periodic sides; false outside a non-periodic side
    auto gcell = [&](int li, int lj, int& gi, int& gj) {
        gi = x0 + li;
        gj = y0 + lj;
        if (gi < 0 || gi >= L.nx) {
            if (!px) return false;
            gi = gi < 0 ? gi + L.nx : gi - L.nx;
        }
        if (gj < 0 || gj >= L.ny) {
            if (!py) return false;
            gj = gj < 0 ? gj + L.ny : gj - L.ny;
        }
        return true;
    };
    for (int c = threadIdx.x; c < NC; c += kTbThreads) {
        int gi, gj;
        if (!gcell(c % W, c / W, gi, gj)) continue;
        const uint32_t k = (uint32_t)gj * (uint32_t)L.nx + (uint32_t)gi;
        double e = ld(u.E, k), fx = ld(u.Fx, k), fy = ld(u.Fy, k), t = ld(u.T, k);
        if (UP) {
            double we, wfx, wfy, wt;
            prolong_value<2>(ph, L.nx, L.ny, px, py, eta, gi, gj, e, fx, fy, t, uc, vc, we, wfx, wfy, wt);
            e = we;
            fx = wfx;
            fy = wfy;
            t = wt;
        }
        sE[0][c] = e;
        sFx[0][c] = fx;
        sFy[0][c] = fy;
        sT[0][c] = t;
        qE[c] = ld(fr.E, k);
        qFx[c] = ld(fr.Fx, k);
        qFy[c] = ld(fr.Fy, k);
        qT[c] = ld(fr.T, k);
        qa[c] = ld(L.sa, k);
        qs[c] = ld(L.ss, k);
    }
    __syncthreads();
    int cur = 0;
#pragma unroll 1
    for (int s = 1; s <= M; ++s) {
        const int nw = W - 2 * s, n = nw * nw;
        const bool first = LEG == kLegDown && s == 1;
        for (int q = threadIdx.x; q < n; q += kTbThreads) {
            const int li = s + q % nw, lj = s + q / nw;
            int gi, gj;
            if (!gcell(li, lj, gi, gj)) continue;
            const int c = lj * W + li;
            double S0 = 0.0, S1 = 0.0, S2 = 0.0, e, fx, fy;
            int kn = is_ghost(ph, 0, gi > 0) ? c : c - 1;
            ghost_rule(ph, 0, gi > 0, in_seg(L, 0, gj), sE[cur][kn], sFx[cur][kn], sFy[cur][kn], e, fx, fy);
            add_x(L.kx, ph.c, ph.c2, +1.0, e, fx, fy, S0, S1, S2);
            kn = is_ghost(ph, 1, gi < L.nx - 1) ? c : c + 1;
            ghost_rule(ph, 1, gi < L.nx - 1, in_seg(L, 1, gj), sE[cur][kn], sFx[cur][kn], sFy[cur][kn], e, fx, fy);
            add_x(L.kx, ph.c, ph.c2, -1.0, e, fx, fy, S0, S1, S2);
            kn = is_ghost(ph, 2, gj > 0) ? c : c - W;
            ghost_rule(ph, 2, gj > 0, in_seg(L, 2, gi), sE[cur][kn], sFx[cur][kn], sFy[cur][kn], e, fx, fy);
            add_y(L.ky, ph.c, ph.c2, +1.0, e, fx, fy, S0, S1, S2);
            kn = is_ghost(ph, 3, gj < L.ny - 1) ? c : c + W;
            ghost_rule(ph, 3, gj < L.ny - 1, in_seg(L, 3, gi), sE[cur][kn], sFx[cur][kn], sFy[cur][kn], e, fx, fy);
            add_y(L.ky, ph.c, ph.c2, -1.0, e, fx, fy, S0, S1, S2);
            const double ka = L.cdt * qa[c], ks = L.cdt * qs[c];
            double f0 = qE[c], f1 = qFx[c], f2 = qFy[c], f3 = qT[c];
            double E, Fx, Fy, T, tE, tFx, tFy, tT, g;
            bool stall;
            const bool own = li >= M && li < M + kTbTile && lj >= M && lj < M + kTbTile;  // not a halo copy
            if (first) {
                pseudo_core<2, true>(ph, L, sE[cur][c], sFx[cur][c], sFy[cur][c], sT[cur][c], S0, S1, S2, ka, ks, f0,
                                     f1, f2, f3, dt, reach, local, E, Fx, Fy, T, tE, tFx, tFy, tT, g, stall);
                qE[c] = f0;
                qFx[c] = f1;
                qFy[c] = f2;
                qT[c] = f3;
                if (live && own) {
                    const uint32_t k = (uint32_t)gj * (uint32_t)L.nx + (uint32_t)gi;
                    st(f.E, k, f0);
                    st(f.Fx, k, f1);
                    st(f.Fy, k, f2);
                    st(f.T, k, f3);
                }
            } else {
                pseudo_core<2, false>(ph, L, sE[cur][c], sFx[cur][c], sFy[cur][c], sT[cur][c], S0, S1, S2, ka, ks, f0,
                                      f1, f2, f3, dt, reach, local, E, Fx, Fy, T, tE, tFx, tFy, tT, g, stall);
            }
            if (live && own && stall && ph.stalls) note_stall(ph.stalls);
            sE[cur ^ 1][c] = E;
            sFx[cur ^ 1][c] = Fx;
            sFy[cur ^ 1][c] = Fy;
            sT[cur ^ 1][c] = T;
        }
        __syncthreads();
        cur ^= 1;
    }
    if (!live) return;
    for (int q = threadIdx.x; q < kTbTile * kTbTile; q += kTbThreads) {
        const int ti = q % kTbTile, tj = q / kTbTile;
        const int c = (M + tj) * W + M + ti;
        const uint32_t k = (uint32_t)(by * kTbTile + tj) * (uint32_t)L.nx + (uint32_t)(bx * kTbTile + ti);
        st(out.E, k, sE[cur][c]);
        st(out.Fx, k, sFx[cur][c]);
        st(out.Fy, k, sFy[cur][c]);
        st(out.T, k, sT[cur][c]);
    }
}

// ===========================================================================
// Batched kernels: persistent grid-stride loops over a work list of
// (problem, tile) entries; every problem carries its own level data, cycle
// control (dtau, stop flag) and norm partials.  Buffer selectors are the same
// for all problems (all run the same sequence of operations):
//   level 0: in_x1 picks x1 (else x0) as the current iterate;
//   level >= 1: sel 0 = v, 1 = u, 2 = u2.
__device__ __forceinline__ const Soa& pick(const BSlot& s, int sel) { return sel == 0 ? s.v : (sel == 1 ? s.u : s.u2); }

// Batched: work-list entries are the 32 x 4 coarse tiles of level `level` of
// each problem; level - 1's residual (b on the finest level, else the FAS
// right-hand side f) is formed and restricted with the state into (v, f).
__global__ __launch_bounds__(kRcThreads) void kb_residual_restrict(
    const BProb* __restrict__ P,
                                                                   const BSlot* __restrict__ S,
                                                                   const uint32_t* __restrict__ wl, int nwl,
                                                                   int level, int in_sel)
{
    __shared__ RcLds sm;
    for (int w_ = blockIdx.x; w_ < nwl; w_ += gridDim.x) {
        const uint32_t item = wl[w_];
        const int p = (int)(item >> kTileBits);
        const uint32_t tile = item & ((1u << kTileBits) - 1u);
        const BProb& pb = P[p];
        if (pb.ctrl->active == 0) continue;
        const BSlot& c = S[p * kMaxLevels + level];
        const BSlot& f = S[p * kMaxLevels + level - 1];
        const Soa& u = (level == 1) ? (in_sel ? f.x1 : f.x0) : pick(f, in_sel);
        const Soa& X = (level == 1) ? f.b : f.f;
        const uint32_t ntx = (uint32_t)((f.L.nx / 2 + kRcW - 1) / kRcW);
        // one variant only in the work-list loop: two inlined cost registers
        residual_restrict_tile<false>(sm, pb.ph, f.L, cs(u), cs(X), -1.0, pb.px, pb.py, c.v, c.f,
                                      (int)(tile % ntx) * kRcW, (int)(tile / ntx) * kRcH, true);
        __syncthreads();  // the next tile of this block reuses the LDS
    }
}


// Batched LDS-staged finest-level sweep (no norm): work-list entries are the
// 64 x TY tiles of each problem's finest level (row-major tile index); the
// staging and the arithmetic are those of k_relax_lds.  UP: the first sweep
// after the coarse-grid correction, fused with it as in k_relax_lds (the
// entries are then those of problems with a coarse level).
template <int TY, bool UP>
__global__ __launch_bounds__(kLdsTX * TY) void kb_relax_lds(const BProb* __restrict__ P, const BSlot* __restrict__ S,
                                                           const uint32_t* __restrict__ wl, int nwl, int in_x1)
{
    constexpr int W = LdsTile<TY>::W;
    __shared__ LdsTile<TY> q;
    __shared__ double qT[UP ? LdsTile<TY>::N : 1];
    for (int w_ = blockIdx.x; w_ < nwl; w_ += gridDim.x) {
        const uint32_t item = wl[w_];
        const int p = (int)(item >> kTileBits);
        const uint32_t tile = item & ((1u << kTileBits) - 1u);
        const BProb& pb = P[p];
        if (pb.ctrl->active == 0) continue;
        const BSlot& s = S[p * kMaxLevels];
        const Soa& in = in_x1 ? s.x1 : s.x0;
        const Soa& out = in_x1 ? s.x0 : s.x1;
        const uint32_t ntx = (uint32_t)((s.L.nx + kLdsTX - 1) / kLdsTX);
        const int i0 = (int)(tile % ntx) * kLdsTX, j0 = (int)(tile / ntx) * TY;
        if (UP) {
            const BSlot& cl = S[p * kMaxLevels + 1];
            stage_tile<TY, true>(q, qT, pb.ph, s.L, cs(in), i0, j0, cs(cl.u), cs(cl.v), pb.px, pb.py, pb.eta);
        } else {
            stage_tile<TY, false>(q, nullptr, pb.ph, s.L, cs(in), i0, j0, CSoa{}, CSoa{}, 0, 0, 0.0);
        }
        __syncthreads();
        const int li = threadIdx.x % kLdsTX, lj = threadIdx.x / kLdsTX, i = i0 + li, j = j0 + lj;
        if (i < s.L.nx && j < s.L.ny) {
            const uint32_t k = (uint32_t)j * (uint32_t)s.L.nx + (uint32_t)i;
            const int c = (lj + 1) * W + li + 1;
            double S0, S1, S2;
            tile_sums<TY>(q, s.L, pb.ph.c, c, S0, S1, S2);
            auto cen = [&](int f) { return f == 0 ? q.E[c] : (f == 1 ? q.Fx[c] : q.Fy[c]); };
            relax_update<2, false>(pb.ph, s.L, cs(s.b), 1.0, 0.0, pb.omega, S0, S1, S2, UP ? qT[c] : ld(in.T, k), cen,
                                   out, k);
        }
        __syncthreads();  // the next tile of this block reuses the LDS
    }
}

// Two finest-level sweeps per launch over a work list of 64 x TY tiles: the
// tile arithmetic of k_relax2_lds, per problem (x_in -> the other buffer).
// Without k_relax2_lds's six-wave cap: in the work-list loop the cap spills
// 18 values, and the batched run measured slower with it (931 vs 999 solves/s).
template <int TY>
__global__ __launch_bounds__(kLdsTX * TY) void kb_relax2_lds(
    const BProb* __restrict__ P, const BSlot* __restrict__ S, const uint32_t* __restrict__ wl, int nwl, int in_x1)
{
    __shared__ Lds2<TY> q;
    for (int w_ = blockIdx.x; w_ < nwl; w_ += gridDim.x) {
        const uint32_t item = wl[w_];
        const int p = (int)(item >> kTileBits);
        const uint32_t tile = item & ((1u << kTileBits) - 1u);
        const BProb& pb = P[p];
        if (pb.ctrl->active == 0) continue;
        const BSlot& s = S[p * kMaxLevels];
        const Soa& in = in_x1 ? s.x1 : s.x0;
        const Soa& out = in_x1 ? s.x0 : s.x1;
        const uint32_t ntx = (uint32_t)((s.L.nx + kLdsTX - 1) / kLdsTX);
        relax2_tile<TY>(q, pb.ph, s.L, cs(s.b), pb.omega, cs(in), out, (int)(tile % ntx) * kLdsTX,
                        (int)(tile / ntx) * TY);
        __syncthreads();  // the next tile of this block reuses the LDS
    }
}

template <bool NORM>
__global__ __launch_bounds__(kBlock) void kb_relax(const BProb* __restrict__ P, const BSlot* __restrict__ S,
                                                   const uint32_t* __restrict__ wl, int nwl, int in_x1)
{
    M1_BATCH_LOOP(wl, nwl)
    const BSlot& s = S[p * kMaxLevels];
    const Soa& in = in_x1 ? s.x1 : s.x0;
    const Soa& out = in_x1 ? s.x0 : s.x1;
    const bool inside = k < (uint32_t)s.L.nx * (uint32_t)s.L.ny;
    int i = 0, j = 0;
    if (inside) ij_of(s.L.nx, s.L.sh, k, i, j);
    if (!NORM) {
        if (inside) relax_cell<2>(pb.ph, s.L, cs(s.b), nullptr, 0.0, 1.0, pb.omega, cs(in), out, k, i, j);
        continue;
    }
    double q = 0.0;
    if (inside) q = relax_cell<2, true>(pb.ph, s.L, cs(s.b), nullptr, 0.0, 1.0, pb.omega, cs(in), out, k, i, j);
    block_partial(q, pb.partials + tile);
    __syncthreads();  // the next tile of this block reuses the reduction slots
    }
}

// One block per problem: finish its residual norm and update its cycle control.
// mixed: the cycle's residual kernel moved the FP64 state to the partner buffer.
__global__ __launch_bounds__(1024) void kb_norm_control(const BProb* __restrict__ P, const int* __restrict__ plist,
                                                        int mixed)
{
    const BProb& pb = P[plist[blockIdx.x]];
    if (pb.ctrl->active == 0) return;
    const double r = sqrt(block_sum(pb.partials, pb.npart));
    if (threadIdx.x == 0) {
        if (mixed) pb.ctrl->flip ^= 1;
        ctrl_update(pb.ctrl, r);
    }
}

// level 0: rf = b - A(x_cur);  level >= 1: rb = f - A(pick(in_sel)).
__global__ __launch_bounds__(kBlock) void kb_apply(const BProb* __restrict__ P, const BSlot* __restrict__ S,
                                                   const uint32_t* __restrict__ wl, int nwl, int level, int in_sel)
{
    M1_BATCH_LOOP(wl, nwl)
    const BSlot& s = S[p * kMaxLevels + level];
    if (k >= (uint32_t)s.L.nx * (uint32_t)s.L.ny) continue;
    int i, j;
    ij_of(s.L.nx, s.L.sh, k, i, j);
    if (level == 0) apply_cell<2>(pb.ph, s.L, cs(in_sel ? s.x1 : s.x0), cs(s.b), -1.0, s.rf, k, i, j);
    else apply_cell<2>(pb.ph, s.L, cs(pick(s, in_sel)), cs(s.f), -1.0, s.rb, k, i, j);
    }
}

// Restriction into `level` of the current iterate and residual of level-1.
__global__ __launch_bounds__(kBlock) void kb_restrict(const BProb* __restrict__ P, const BSlot* __restrict__ S,
                                                      const uint32_t* __restrict__ wl, int nwl, int level, int in_sel)
{
    M1_BATCH_LOOP(wl, nwl)
    const BSlot& c = S[p * kMaxLevels + level];
    const BSlot& f = S[p * kMaxLevels + level - 1];
    if (k >= (uint32_t)c.L.nx * (uint32_t)c.L.ny) continue;
    const Soa& u = (level == 1) ? (in_sel ? f.x1 : f.x0) : pick(f, in_sel);
    const Soa& r = (level == 1) ? f.rf : f.rb;
    const double* in[8] = {u.E, u.Fx, u.Fy, u.T, r.E, r.Fx, r.Fy, r.T};
    double* out[8] = {c.v.E, c.v.Fx, c.v.Fy, c.v.T, c.f.E, c.f.Fx, c.f.Fy, c.f.T};
    restrict_cell<2, 8>(f.L.nx, f.L.ny, f.L.sh, pb.px, pb.py, in, out, k);
    }
}

__global__ __launch_bounds__(kBlock) void kb_pseudo(const BProb* __restrict__ P, const BSlot* __restrict__ S,
                                                    const uint32_t* __restrict__ wl, int nwl, int level, int in_sel,
                                                    int out_sel, int first)
{
    M1_BATCH_LOOP(wl, nwl)
    const BSlot& s = S[p * kMaxLevels + level];
    if (k >= (uint32_t)s.L.nx * (uint32_t)s.L.ny) continue;
    int i, j;
    ij_of(s.L.nx, s.L.sh, k, i, j);
    const double dt = pb.ctrl->dtau;
    if (first)
        pseudo_cell<2, true>(pb.ph, s.L, cs(s.f), s.f, cs(pick(s, in_sel)), pick(s, out_sel), dt, pb.reach, pb.local,
                             Soa{}, nullptr, k, i, j);
    else
        pseudo_cell<2, false>(pb.ph, s.L, cs(s.f), s.f, cs(pick(s, in_sel)), pick(s, out_sel), dt, pb.reach,
                              pb.local, Soa{}, nullptr, k, i, j);
    }
}

// Correction of `level` from level+1.  Fine side: level 0 in place on x_cur
// (in_sel = in_x1), else pick(in_sel) -> pick(out_sel).  Coarse side: the final
// iterate of level+1, always in u (with an odd number of pseudo-time steps the
// down leg, the up leg and the tail all end there).
__global__ __launch_bounds__(kBlock) void kb_prolong(const BProb* __restrict__ P, const BSlot* __restrict__ S,
                                                     const uint32_t* __restrict__ wl, int nwl, int level, int in_sel,
                                                     int out_sel)
{
    M1_BATCH_LOOP(wl, nwl)
    const BSlot& f = S[p * kMaxLevels + level];
    const BSlot& c = S[p * kMaxLevels + level + 1];
    if (k >= (uint32_t)f.L.nx * (uint32_t)f.L.ny) continue;
    const Soa& u = (level == 0) ? (in_sel ? f.x1 : f.x0) : pick(f, in_sel);
    const Soa& o = (level == 0) ? u : pick(f, out_sel);
    prolong_cell<2>(pb.ph, f.L.nx, f.L.ny, f.L.sh, pb.px, pb.py, pb.eta, cs(u), cs(c.u), cs(c.v), o, k);
    }
}

// One workgroup per problem: the bottom of its cycle.
__global__ __launch_bounds__(kTailThreads) void kb_tail(const BProb* __restrict__ P, const int* __restrict__ plist)
{
    const BProb& pb = P[plist[blockIdx.x]];
    if (pb.ctrl->active == 0) return;
    tail_body<2>(*pb.tail, pb.ctrl->dtau);
}

// Step start, per fine tile of the starting problems (their control is not
// live): bring the state back to x0 when the previous step left it in x1
// (mixed precision), form b = (E, F, C_v T) and the tile's partial of |b|^2,
// with the same expression and reduction order as the single-problem path.
__global__ __launch_bounds__(kBlock) void kb_init_tiles(const BProb* __restrict__ P, const BSlot* __restrict__ S,
                                                        const uint32_t* __restrict__ wl, int nwl)
{
    for (int w_ = blockIdx.x; w_ < nwl; w_ += gridDim.x) {
        const uint32_t item = wl[w_];
        const int p = (int)(item >> kTileBits);
        const uint32_t tile = item & ((1u << kTileBits) - 1u);
        const BProb& pb = P[p];
        const BSlot& s = S[p * kMaxLevels];
        const uint32_t k = tile * kBlock + threadIdx.x;
        double q = 0.0;
        if (k < (uint32_t)s.L.nx * (uint32_t)s.L.ny) {
            const bool fl = pb.ctrl->flip != 0;
            const Soa& src = fl ? s.x1 : s.x0;
            const double E = ld(src.E, k), Fx = ld(src.Fx, k), Fy = ld(src.Fy, k), T = ld(src.T, k);
            if (fl) {
                st(s.x0.E, k, E);
                st(s.x0.Fx, k, Fx);
                st(s.x0.Fy, k, Fy);
                st(s.x0.T, k, T);
            }
            const double bT = pb.ph.c_v * T;
            st(s.b.E, k, E);
            st(s.b.Fx, k, Fx);
            st(s.b.Fy, k, Fy);
            st(s.b.T, k, bT);
            const double ic = 1.0 / pb.ph.c;
            const double fx = Fx * ic, fy = Fy * ic;
            q = fma(E, E, fma(fx, fx, fma(fy, fy, bT * bT)));
        }
        block_partial(q, pb.partials + tile);
        __syncthreads();  // the next tile of this block reuses the reduction slots
    }
}

// One block per starting problem: |b| for the rounding floor and a fresh
// cycle control (state in x0), its dtau carried over from the request's
// previous step when the request asks for that.
__global__ __launch_bounds__(1024) void kb_init_ctrl(const BProb* __restrict__ P, const BSlot* __restrict__ S,
                                                     const int* __restrict__ plist)
{
    const int p = plist[blockIdx.x];
    const BProb& pb = P[p];
    const double t = block_sum(pb.partials, pb.npart);
    if (threadIdx.x == 0) {
        Ctrl c = pb.proto;
        // a request's first step finds the plan's stopped control (dtau 0); later ones the last step's dtau
        if (c.carry && pb.ctrl->dtau > 0.0) c.dtau = pb.ctrl->dtau;
        c.floor_r = 16.0 * DBL_EPSILON * S[p * kMaxLevels].L.a * sqrt(t);
        c.active = 1;
        c.cycles = -1;
        c.conv = 0;
        c.flip = 0;
        *pb.ctrl = c;
    }
}

// x0 = x1 over the fine tiles of finished mixed-precision requests whose
// result is in x1 (their control is not live).
__global__ __launch_bounds__(kBlock) void kb_flip_copy(const BProb* __restrict__ P, const BSlot* __restrict__ S,
                                                       const uint32_t* __restrict__ wl, int nwl)
{
    (void)P;
    for (int w_ = blockIdx.x; w_ < nwl; w_ += gridDim.x) {
        const uint32_t item = wl[w_];
        const int p = (int)(item >> kTileBits);
        const uint32_t tile = item & ((1u << kTileBits) - 1u);
        const BSlot& s = S[p * kMaxLevels];
        const uint32_t k = tile * kBlock + threadIdx.x;
        if (k >= (uint32_t)s.L.nx * (uint32_t)s.L.ny) continue;
        st(s.x0.E, k, ld(s.x1.E, k));
        st(s.x0.Fx, k, ld(s.x1.Fx, k));
        st(s.x0.Fy, k, ld(s.x1.Fy, k));
        st(s.x0.T, k, ld(s.x1.T, k));
    }
}

__global__ void kb_gather_ctrl(const BProb* __restrict__ P, int np, Ctrl* __restrict__ out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < np) out[p] = *P[p].ctrl;
}

// ===========================================================================
// Launchers
// ===========================================================================
#define M1_DISPATCH(DIM_, KERNEL, GRID, ...)                                                          \
    do {                                                                                              \
        if ((DIM_) == 2) hipLaunchKernelGGL(KERNEL<2>, dim3(GRID), dim3(kBlock), 0, st, __VA_ARGS__); \
        else hipLaunchKernelGGL(KERNEL<1>, dim3(GRID), dim3(kBlock), 0, st, __VA_ARGS__);            \
    } while (0)

static std::atomic<int> g_sweep_rows{4};
int sweep_rows() { return g_sweep_rows.load(std::memory_order_relaxed); }
static std::atomic<int> g_mx_sweep_rows{4};
int mx_sweep_rows() { return g_mx_sweep_rows.load(std::memory_order_relaxed); }
bool set_mx_sweep_rows(int rows)
{
    if (rows != 0 && rows != 4 && rows != 8 && rows != 16) return false;
    g_mx_sweep_rows.store(rows, std::memory_order_relaxed);
    return true;
}
bool set_sweep_rows(int rows)
{
    if (rows != 0 && rows != 4 && rows != 8 && rows != 16) return false;
    g_sweep_rows.store(rows, std::memory_order_relaxed);
    return true;
}
static std::atomic<int> g_pair_rows{8};
int pair_rows() { return g_pair_rows.load(std::memory_order_relaxed); }
bool set_pair_rows(int rows)
{
    if (rows != 0 && rows != 4 && rows != 8 && rows != 16) return false;
    g_pair_rows.store(rows, std::memory_order_relaxed);
    return true;
}

bool launch_relax_lds(hipStream_t st, const Phys& ph, const Lvl& L, CSoa rhs, double omega, CSoa u, Soa out,
                      const int* active, CSoa uc, CSoa vc, int px, int py, double eta)
{
    const int rows = sweep_rows();
    if (rows == 0) return false;
    const unsigned ntx = (unsigned)((L.nx + kLdsTX - 1) / kLdsTX), nty = (unsigned)((L.ny + rows - 1) / rows);
    const dim3 gl(ntx * nty), bl(kLdsTX * rows);
    const bool up = uc.E != nullptr;
#define M1_RELAX_LDS(R, U)                                                                                            \
    hipLaunchKernelGGL((k_relax_lds<R, U>), gl, bl, 0, st, ph, L, rhs, omega, u, out, active, uc, vc, px, py, eta)
    if (rows == 4) {
        if (up) M1_RELAX_LDS(4, true);
        else M1_RELAX_LDS(4, false);
    } else if (rows == 8) {
        if (up) M1_RELAX_LDS(8, true);
        else M1_RELAX_LDS(8, false);
    } else {
        if (up) M1_RELAX_LDS(16, true);
        else M1_RELAX_LDS(16, false);
    }
#undef M1_RELAX_LDS
    return true;
}

bool launch_relax2_lds(hipStream_t st, const Phys& ph, const Lvl& L, CSoa rhs, double omega, CSoa u, Soa out,
                       const int* active)
{
    const int rows = pair_rows();
    if (rows == 0) return false;
    const unsigned ntx = (unsigned)((L.nx + kLdsTX - 1) / kLdsTX), nty = (unsigned)((L.ny + rows - 1) / rows);
    const dim3 gl(ntx * nty), bl(kLdsTX * rows);
    if (rows == 4) hipLaunchKernelGGL(k_relax2_lds<4>, gl, bl, 0, st, ph, L, rhs, omega, u, out, active);
    else if (rows == 8) hipLaunchKernelGGL(k_relax2_lds<8>, gl, bl, 0, st, ph, L, rhs, omega, u, out, active);
    else hipLaunchKernelGGL(k_relax2_lds<16>, gl, bl, 0, st, ph, L, rhs, omega, u, out, active);
    return true;
}

void launch_relax(hipStream_t st, int dim, const Phys& ph, const Lvl& L, CSoa rhs, const double* gcell, double beta,
                  double gamma, double omega, CSoa u, Soa out, double* partials, const int* active)
{
    const dim3 g(nblocks((int64_t)L.nx * L.ny)), b(kBlock);
    const bool fine = !gcell && beta == 0.0 && gamma == 1.0;
    if (dim == 2 && fine && !partials && sweep_rows() > 0) {
        launch_relax_lds(st, ph, L, rhs, omega, u, out, active, CSoa{}, CSoa{}, 0, 0, 0.0);
        return;
    }
#define M1_RELAX(D, N, F)                                                                                             \
    hipLaunchKernelGGL((k_relax<D, N, F>), g, b, 0, st, ph, L, rhs, gcell, beta, gamma, omega, u, out, partials, active)
    if (dim == 2) {
        if (partials) M1_RELAX(2, true, true);
        else if (fine) M1_RELAX(2, false, true);
        else M1_RELAX(2, false, false);
    } else {
        if (partials) M1_RELAX(1, true, true);
        else if (fine) M1_RELAX(1, false, true);
        else M1_RELAX(1, false, false);
    }
#undef M1_RELAX
}

void launch_relax_colour(hipStream_t st, int dim, const Phys& ph, const Lvl& L, CSoa rhs, double omega, int colour,
                         CSoa u, Soa out, double* partials, const int* active)
{
    const dim3 g(nblocks((int64_t)L.nx * L.ny)), b(kBlock);
#define M1_RELAX_C(D, N)                                                                                              \
    hipLaunchKernelGGL((k_relax_colour<D, N>), g, b, 0, st, ph, L, rhs, omega, colour, u, out, partials, active)
    if (dim == 2) {
        if (partials) M1_RELAX_C(2, true);
        else M1_RELAX_C(2, false);
    } else {
        if (partials) M1_RELAX_C(1, true);
        else M1_RELAX_C(1, false);
    }
#undef M1_RELAX_C
}

void launch_pseudo(hipStream_t st, int dim, const Phys& ph, const Lvl& L, Soa f, CSoa u, Soa out, double dtau,
                   const double* dtau_dev, double reach, int local, int first, Soa rs, double* gs, const int* active)
{
    const int rows = sweep_rows();
    if (dim == 2 && rows > 0 && (int64_t)L.nx * L.ny >= kPseudoLdsCells) {
        const dim3 gl((unsigned)((L.nx + kLdsTX - 1) / kLdsTX) * (unsigned)((L.ny + rows - 1) / rows)),
            bl(kLdsTX * rows);
#define M1_PSEUDO_LDS(R)                                                                                             \
    do {                                                                                                             \
        if (first)                                                                                                   \
            hipLaunchKernelGGL((k_pseudo_lds<R, true>), gl, bl, 0, st, ph, L, f, u, out, dtau_dev, reach, local, rs, \
                               gs, active);                                                                          \
        else                                                                                                         \
            hipLaunchKernelGGL((k_pseudo_lds<R, false>), gl, bl, 0, st, ph, L, f, u, out, dtau_dev, reach, local,    \
                               rs, gs, active);                                                                      \
    } while (0)
        if (rows == 4) M1_PSEUDO_LDS(4);
        else if (rows == 8) M1_PSEUDO_LDS(8);
        else M1_PSEUDO_LDS(16);
#undef M1_PSEUDO_LDS
        return;
    }
    M1_DISPATCH(dim, k_pseudo, nblocks((int64_t)L.nx * L.ny), ph, L, f, u, out, dtau, dtau_dev, reach, local, first,
                rs, gs, active);
}

unsigned apply_blocks(const Lvl& L) { return nblocks((int64_t)L.nx * L.ny); }

static std::atomic<int> g_residual_restrict{1};
int residual_restrict() { return g_residual_restrict.load(std::memory_order_relaxed); }
void set_residual_restrict(int on) { g_residual_restrict.store(on ? 1 : 0, std::memory_order_relaxed); }

void launch_residual_restrict(hipStream_t st, const Phys& ph, const Lvl& L, CSoa u, CSoa X, double sgn, int px, int py,
                              Soa vc, Soa rc, const int* active)
{
    const int nxc = L.nx / 2, nyc = L.ny / 2;
    if (nxc < 1 || nyc < 1) return;
    const unsigned nb = (unsigned)((nxc + kRcW - 1) / kRcW) * (unsigned)((nyc + kRcH - 1) / kRcH);
    hipLaunchKernelGGL(k_residual_restrict, dim3(nb), dim3(kRcThreads), 0, st, ph, L, u, X, sgn, px, py, vc, rc,
                       active);
}


void launch_apply(hipStream_t st, int dim, const Phys& ph, const Lvl& L, CSoa v, CSoa X, double sgn, Soa out,
                  double* partials, const int* active)
{
    const int rows = sweep_rows();
    if (dim == 2 && !partials && out.E && rows > 0) {
        const unsigned ntx = (unsigned)((L.nx + kLdsTX - 1) / kLdsTX), nty = (unsigned)((L.ny + rows - 1) / rows);
        const dim3 gl(ntx * nty), bl(kLdsTX * rows);
        if (rows == 4) hipLaunchKernelGGL(k_apply_lds<4>, gl, bl, 0, st, ph, L, v, X, sgn, out, active);
        else if (rows == 8) hipLaunchKernelGGL(k_apply_lds<8>, gl, bl, 0, st, ph, L, v, X, sgn, out, active);
        else hipLaunchKernelGGL(k_apply_lds<16>, gl, bl, 0, st, ph, L, v, X, sgn, out, active);
        return;
    }
    M1_DISPATCH(dim, k_apply, apply_blocks(L), ph, L, v, X, sgn, out, partials, active);
}

// Blocks of a batched launch: one per work-list entry up to a cap (tuning key
// "batch_grid"); above it each block walks several entries.
static std::atomic<int> g_batch_grid{16384};
int batch_grid_cap() { return g_batch_grid.load(std::memory_order_relaxed); }
void set_batch_grid_cap(int cap) { g_batch_grid.store(cap, std::memory_order_relaxed); }
static unsigned bgrid(int nwl) { return (unsigned)std::max(1, std::min(nwl, batch_grid_cap())); }

void launch_b_residual_restrict(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int level,
                                int in_sel)
{
    if (nwl > 0)
        hipLaunchKernelGGL(kb_residual_restrict, dim3(bgrid(nwl)), dim3(kRcThreads), 0, st, P, S, wl, nwl, level,
                           in_sel);
}

void launch_b_relax2_lds(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int in_x1,
                         int rows)
{
    if (nwl <= 0) return;
    const dim3 g(bgrid(nwl)), b(kLdsTX * rows);
    if (rows == 4) hipLaunchKernelGGL(kb_relax2_lds<4>, g, b, 0, st, P, S, wl, nwl, in_x1);
    else if (rows == 8) hipLaunchKernelGGL(kb_relax2_lds<8>, g, b, 0, st, P, S, wl, nwl, in_x1);
    else hipLaunchKernelGGL(kb_relax2_lds<16>, g, b, 0, st, P, S, wl, nwl, in_x1);
}
void launch_b_relax_lds(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int in_x1,
                        int rows, bool up)
{
    if (nwl <= 0) return;
    const dim3 g(bgrid(nwl)), b(kLdsTX * rows);
#define M1_B_RELAX_LDS(R)                                                                                             \
    if (up) hipLaunchKernelGGL((kb_relax_lds<R, true>), g, b, 0, st, P, S, wl, nwl, in_x1);                          \
    else hipLaunchKernelGGL((kb_relax_lds<R, false>), g, b, 0, st, P, S, wl, nwl, in_x1)
    if (rows == 4) {
        M1_B_RELAX_LDS(4);
    } else if (rows == 8) {
        M1_B_RELAX_LDS(8);
    } else {
        M1_B_RELAX_LDS(16);
    }
#undef M1_B_RELAX_LDS
}

void launch_b_relax(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int in_x1, int norm)
{
    if (nwl <= 0) return;
    if (norm) hipLaunchKernelGGL(kb_relax<true>, dim3(bgrid(nwl)), dim3(kBlock), 0, st, P, S, wl, nwl, in_x1);
    else hipLaunchKernelGGL(kb_relax<false>, dim3(bgrid(nwl)), dim3(kBlock), 0, st, P, S, wl, nwl, in_x1);
}
void launch_b_norm_control(hipStream_t st, const BProb* P, const int* plist, int np, int mixed)
{
    if (np > 0) hipLaunchKernelGGL(kb_norm_control, dim3(np), dim3(1024), 0, st, P, plist, mixed);
}
void launch_b_apply(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int level, int in_sel)
{
    if (nwl > 0) hipLaunchKernelGGL(kb_apply, dim3(bgrid(nwl)), dim3(kBlock), 0, st, P, S, wl, nwl, level, in_sel);
}
void launch_b_restrict(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int level,
                       int in_sel)
{
    if (nwl > 0) hipLaunchKernelGGL(kb_restrict, dim3(bgrid(nwl)), dim3(kBlock), 0, st, P, S, wl, nwl, level, in_sel);
}
void launch_b_pseudo(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int level,
                     int in_sel, int out_sel, int first)
{
    if (nwl > 0)
        hipLaunchKernelGGL(kb_pseudo, dim3(bgrid(nwl)), dim3(kBlock), 0, st, P, S, wl, nwl, level, in_sel, out_sel,
                           first);
}
void launch_b_prolong(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int level,
                      int in_sel, int out_sel)
{
    if (nwl > 0)
        hipLaunchKernelGGL(kb_prolong, dim3(bgrid(nwl)), dim3(kBlock), 0, st, P, S, wl, nwl, level, in_sel, out_sel);
}
void launch_b_tail(hipStream_t st, const BProb* P, const int* plist, int np)
{
    if (np > 0) hipLaunchKernelGGL(kb_tail, dim3(np), dim3(kTailThreads), 0, st, P, plist);
}
void launch_b_init_tiles(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl)
{
    if (nwl > 0) hipLaunchKernelGGL(kb_init_tiles, dim3(bgrid(nwl)), dim3(kBlock), 0, st, P, S, wl, nwl);
}
void launch_b_init_ctrl(hipStream_t st, const BProb* P, const BSlot* S, const int* plist, int np)
{
    if (np > 0) hipLaunchKernelGGL(kb_init_ctrl, dim3(np), dim3(1024), 0, st, P, S, plist);
}
void launch_b_flip_copy(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl)
{
    if (nwl > 0) hipLaunchKernelGGL(kb_flip_copy, dim3(bgrid(nwl)), dim3(kBlock), 0, st, P, S, wl, nwl);
}
void launch_b_gather_ctrl(hipStream_t st, const BProb* P, int np, Ctrl* out)
{
    if (np > 0) hipLaunchKernelGGL(kb_gather_ctrl, dim3((np + 255) / 256), dim3(256), 0, st, P, np, out);
}

void launch_norm_finalize(hipStream_t st, const double* partials, int n, double* out)
{
    hipLaunchKernelGGL(k_norm_finalize, dim3(1), dim3(1024), 0, st, partials, n, out);
}

void launch_norm_control(hipStream_t st, const double* partials, int n, Ctrl* ctrl)
{
    hipLaunchKernelGGL(k_norm_control, dim3(1), dim3(1024), 0, st, partials, n, ctrl);
}

void launch_ctrl_init(hipStream_t st, Ctrl* ctrl, const Ctrl& init)
{
    hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(1), 0, st, ctrl, init);
}

void launch_restrict(hipStream_t st, int dim, int nxf, int nyf, int px, int py, const Fields& F, const int* active)
{
    const int64_t nc = (int64_t)(nxf / 2) * (dim == 2 ? nyf / 2 : 1);
    const int shf = row_shift(nxf);
    const unsigned g = nblocks(nc);
    const dim3 b(kBlock);
    if (dim == 2) {
        switch (F.n) {
        case 2: hipLaunchKernelGGL((k_restrict<2, 2>), dim3(g), b, 0, st, nxf, nyf, shf, px, py, F, active); break;
        case 4: hipLaunchKernelGGL((k_restrict<2, 4>), dim3(g), b, 0, st, nxf, nyf, shf, px, py, F, active); break;
        default: hipLaunchKernelGGL((k_restrict<2, 8>), dim3(g), b, 0, st, nxf, nyf, shf, px, py, F, active); break;
        }
    } else {
        switch (F.n) {
        case 2: hipLaunchKernelGGL((k_restrict<1, 2>), dim3(g), b, 0, st, nxf, nyf, shf, px, py, F, active); break;
        case 3: hipLaunchKernelGGL((k_restrict<1, 3>), dim3(g), b, 0, st, nxf, nyf, shf, px, py, F, active); break;
        default: hipLaunchKernelGGL((k_restrict<1, 6>), dim3(g), b, 0, st, nxf, nyf, shf, px, py, F, active); break;
        }
    }
}

void launch_prolong_project(hipStream_t st, int dim, const Phys& ph, int nx, int ny, int px, int py, double eta,
                            CSoa u, CSoa uc, CSoa vc, Soa out, const int* active)
{
    M1_DISPATCH(dim, k_prolong_project, nblocks((int64_t)nx * ny), ph, nx, ny, row_shift(nx), px, py, eta, u, uc, vc,
                out, active);
}

void launch_tail(hipStream_t st, int dim, const TailArgs* args_dev, double dtau, const double* dtau_dev,
                 const int* active)
{
    if (dim == 2) hipLaunchKernelGGL(k_tail<2>, dim3(1), dim3(kTailThreads), 0, st, args_dev, dtau, dtau_dev, active);
    else hipLaunchKernelGGL(k_tail<1>, dim3(1), dim3(kTailThreads), 0, st, args_dev, dtau, dtau_dev, active);
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

bool smooth_tb_fits(int dim, const Lvl& L, int m)
{
    return dim == 2 && m >= 1 && m <= 3 && L.nx % kTbTile == 0 && L.ny % kTbTile == 0 && L.nx >= 2 * kTbTile &&
           L.ny >= 2 * kTbTile;
}

void launch_smooth_tb(hipStream_t st, const Phys& ph, const Lvl& L, int m, int leg, CSoa fr, Soa f, CSoa u, Soa out,
                      const double* dtau_dev, double reach, int local, CSoa uc, CSoa vc, int px, int py, double eta,
                      const int* active)
{
    const dim3 g((unsigned)((L.nx / kTbTile) * (L.ny / kTbTile))), b(kTbThreads);
#define M1_TB(MM)                                                                                                    \
    do {                                                                                                             \
        if (leg == kLegUp)                                                                                           \
            hipLaunchKernelGGL((k_smooth_tb<MM, kLegUp>), g, b, 0, st, ph, L, fr, f, u, out, dtau_dev, reach, local, \
                               uc, vc, px, py, eta, active);                                                         \
        else if (leg == kLegPlain)                                                                                   \
            hipLaunchKernelGGL((k_smooth_tb<MM, kLegPlain>), g, b, 0, st, ph, L, fr, f, u, out, dtau_dev, reach,     \
                               local, uc, vc, px, py, eta, active);                                                  \
        else                                                                                                         \
            hipLaunchKernelGGL((k_smooth_tb<MM, kLegDown>), g, b, 0, st, ph, L, fr, f, u, out, dtau_dev, reach,      \
                               local, uc, vc, px, py, eta, active);                                                  \
    } while (0)
    if (m == 1) M1_TB(1);
    else if (m == 2) M1_TB(2);
    else M1_TB(3);
#undef M1_TB
}

}  // namespace m1
