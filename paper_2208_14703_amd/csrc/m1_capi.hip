// m1_capi.hip -- plan (level hierarchy carved from caller workspace), the
// V-cycle / time-step drivers and the C ABI declared in include/m1.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <string>
#include <initializer_list>
#include <utility>
#include <cfloat>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/m1.h"
#include "m1_internal.hpp"
#include "m1_transfer.hpp"
#include "m1_3d.hpp"
#include "m1_trace.hpp"

namespace {

using m1::CSoa;
using m1::CSoa32;
using m1::cs;
using m1::Soa;
using m1::Soa32;

constexpr size_t kAlign = 256;
constexpr int64_t kMaxCells = int64_t(1) << 29;  // cells of a grid: byte offsets of FP64 fields fit 32 bits

struct LevelBuf {
    int nx = 0, ny = 0;
    int64_t n = 0;
    double hx = 0, hy = 0;
    m1::Lvl L{};
    Soa v{}, u{}, u2{}, f{}, rb{}, rt{};
    double* g = nullptr;
    double* sa = nullptr;
    double* ss = nullptr;
    // mixed precision (FP32): base w, restricted correction d, iterates e/e2,
    // right-hand side g, residual rho, source of the explicit sub-steps fr, opacities
    m1::Lvl32 L32{};
    Soa32 w{}, d{}, e{}, e2{}, gg{}, rho{}, fr{};
    float* sa32 = nullptr;
    float* ss32 = nullptr;
};

// Most levels of a plan: halving a side of at most 2^29 cells down to 4 gives 28.
constexpr int kMaxPlanLevels = 32;

// Side lengths of a level hierarchy (fixed capacity: plans keep no heap storage).
struct Dims {
    int n = 0;
    int nx[kMaxPlanLevels] = {}, ny[kMaxPlanLevels] = {};
    size_t size() const { return (size_t)n; }
};

// Level sizes: coarsen while every active side stays even and >= 4 after
// halving (levels == 0), or exactly `levels` levels when possible.
bool level_dims(const m1_grid& g, const m1_params& p, Dims& d)
{
    d.n = 1;
    d.nx[0] = g.nx;
    d.ny[0] = g.dim == 2 ? g.ny : 1;
    for (;;) {
        if (p.levels > 0 && d.n >= p.levels) break;
        if (d.n >= kMaxPlanLevels) break;
        const int nx = d.nx[d.n - 1], ny = d.ny[d.n - 1];
        bool ok = (nx % 2 == 0) && nx / 2 >= 4;
        if (g.dim == 2) ok = ok && (ny % 2 == 0) && ny / 2 >= 4;
        if (!ok) break;
        d.nx[d.n] = nx / 2;
        d.ny[d.n] = g.dim == 2 ? ny / 2 : 1;
        ++d.n;
    }
    return p.levels <= 0 || d.n == p.levels;
}

bool valid_bc(const m1_grid& g)
{
    for (int s = 0; s < (g.dim == 2 ? 4 : 2); ++s) {
        const m1_bc& b = g.bc[s];
        if (b.kind < M1_BC_PERIODIC || b.kind > M1_BC_INFLOW) return false;
        if (b.kind == M1_BC_DIRICHLET || b.kind == M1_BC_INFLOW) {  // an admissible wall state (|F| = cE allowed)
            if (!(std::isfinite(b.E) && std::isfinite(b.Fx) && std::isfinite(b.Fy) && b.E > 0.0)) return false;
            if (std::sqrt(b.Fx * b.Fx + (g.dim == 2 ? b.Fy * b.Fy : 0.0)) > g.c * b.E * (1.0 + 1e-12)) return false;
        }
        if (b.kind == M1_BC_INFLOW && !(b.lo >= 0.0 && b.lo <= b.hi && b.hi <= 1.0 && b.Eo > 0.0 && std::isfinite(b.Eo)))
            return false;
    }
    if ((g.bc[0].kind == M1_BC_PERIODIC) != (g.bc[1].kind == M1_BC_PERIODIC)) return false;
    if (g.dim == 2 && (g.bc[2].kind == M1_BC_PERIODIC) != (g.bc[3].kind == M1_BC_PERIODIC)) return false;
    return true;
}

bool valid_grid(const m1_grid* g)
{
    if (!g) return false;
    if (g->dim != 1 && g->dim != 2) return false;
    if (g->nx < 1 || g->ny < 1 || (g->dim == 1 && g->ny != 1)) return false;
    if ((int64_t)g->nx * g->ny > kMaxCells) return false;  // 32-bit cell byte offsets
    auto pos = [](double x) { return std::isfinite(x) && x > 0.0; };
    if (!pos(g->hx) || !pos(g->dt) || !pos(g->c) || !pos(g->c_v)) return false;
    if (g->dim == 2 && !pos(g->hy)) return false;
    if (!(std::isfinite(g->a_r) && g->a_r >= 0.0)) return false;
    return valid_bc(*g);
}

bool valid_params(const m1_params* p)
{
    if (!p) return false;
    if (p->levels < 0 || p->nu0 < 1 || p->nu_l < 1 || p->pseudo_steps < 1 || p->sub_steps < 1 || p->max_cycles < 1)
        return false;
    if (p->dtau_rule != M1_DTAU_SIGNED && p->dtau_rule != M1_DTAU_LITERAL) return false;
    if (p->precision != M1_FP64 && p->precision != M1_MIXED) return false;
    if (p->precision == M1_MIXED && p->nu_l != 1) return false;  // coarse correction steps fuse one sweep
    if (p->smoother != M1_SMOOTH_JACOBI && p->smoother != M1_SMOOTH_RBGS) return false;
    if (p->smoother == M1_SMOOTH_RBGS && p->precision != M1_FP64) return false;
    if (p->cycle != M1_CYCLE_V && p->cycle != M1_CYCLE_W && p->cycle != M1_CYCLE_F) return false;
    if (p->transfer != M1_TRANSFER_FULL && p->transfer != M1_TRANSFER_MEAN) return false;
    if (p->transfer != M1_TRANSFER_FULL && p->precision != M1_FP64) return false;
    if (!(p->eta > 0.0 && p->eta < 1.0) || !(p->omega > 0.0 && p->omega <= 1.0) || !(p->rtol > 0.0)) return false;
    if (!(p->dtau_im0 > 0.0) || !(p->dtau_min > 0.0) || !(p->dtau_max >= p->dtau_min)) return false;
    if (p->dtau_carry != 0 && p->dtau_carry != 1) return false;
    return std::isfinite(p->eps_inc) && std::isfinite(p->eps_dec);
}

// Bump allocator over the caller's workspace (or a dry run to size it).
struct Carver {
    char* base;
    size_t off = 0;
    double* take(int64_t count)
    {
        off = (off + kAlign - 1) / kAlign * kAlign;
        double* p = base ? reinterpret_cast<double*>(base + off) : nullptr;
        off += (size_t)count * sizeof(double);
        return p;
    }
    Soa soa(int64_t n, int dim)
    {
        Soa s;
        s.E = take(n);
        s.Fx = take(n);
        s.Fy = dim == 2 ? take(n) : nullptr;
        s.T = take(n);
        return s;
    }
    float* take32(int64_t count) { return reinterpret_cast<float*>(take((count + 1) / 2)); }
    Soa32 soa32(int64_t n, int dim)
    {
        Soa32 s;
        s.E = take32(n);
        s.Fx = take32(n);
        s.Fy = dim == 2 ? take32(n) : nullptr;
        s.T = take32(n);
        return s;
    }
};

}  // namespace

struct m1_plan {
    m1_grid grid{};
    m1_params params{};
    hipStream_t st = nullptr;
    int dim = 2, L = 1, px = 0, py = 0;
    double reach = 0.0;  // 1 - (1 - eta)^sub_steps
    m1::Phys ph{};
    LevelBuf lev[kMaxPlanLevels];
    Soa b{}, tmp{}, rfine{};
    double* partials = nullptr;
    int npart = 0;
    double* dscal = nullptr;
    unsigned long long* dbad = nullptr;
    unsigned long long* dstall = nullptr;  // pseudo-time stalls since the last reset
    double* hpin = nullptr;        // pinned host words: a scalar, the bad-cell index, the control copy
    bool own_hpin = true;          // false: borrowed from an engine (not freed with the plan)
    unsigned long long* hbad = nullptr;
    m1::Ctrl* dctrl = nullptr;     // device cycle control (workspace)
    m1::Ctrl* dfix = nullptr;      // always-live control for single operations (active = 1, settable dtau)
    m1::Ctrl* hctrl = nullptr;     // pinned host copy
    m1::TailArgs* dtail = nullptr; // device copy of the tail description (workspace)
    m1::TailArgs hta{};            // host source of that copy (kept: the upload may still be in flight)
    m1::TailArgs32 hta32{};
    int lt = 0;                    // first level run by the single-workgroup tail (L: none)
    bool mixed = false;
    bool tiled = true;  // LDS-tiled smoothing legs where the level shape allows (M1_TILED=0 turns them off)
    int64_t tiled_max = 0;  // ... on levels of at most this many cells
    Soa32 base32{}, r32{}, dA{}, dB{}, rho0{};  // mixed: finest-level FP32 buffers
    m1::TailArgs32* dtail32 = nullptr;           // mixed: device copy of the tail description
    // m1_step's V-cycles replayed from hipGraph recordings, keyed by the buffers a cycle starts from
    struct CycleGraph {
        const double *in_cur, *in_other;
        const float* in_pend;  // mixed, after the first cycle: the correction the cycle applies
        bool first;
        Soa cur, other;  // where the cycle leaves the state and its partner
        Soa32 pend;
        hipGraphExec_t exec;
    };
    bool graphs = false;
    hipStream_t cap = nullptr;  // private stream, only ever used for recording
    std::vector<CycleGraph> cyc;
};

namespace {

// Lay out every buffer of the plan; with c.base == nullptr only the size is computed.
void carve(m1_plan& P, Carver& c, const Dims& d)
{
    const int dim = P.grid.dim;
    P.L = d.n;
    for (auto& lv : P.lev) lv = LevelBuf{};
    const int64_t n0 = (int64_t)d.nx[0] * d.ny[0];
    P.b = c.soa(n0, dim);
    P.tmp = c.soa(n0, dim);
    P.rfine = c.soa(n0, dim);
    for (int l = 0; l < P.L; ++l) {
        LevelBuf& lv = P.lev[l];
        lv.nx = d.nx[l];
        lv.ny = d.ny[l];
        lv.n = (int64_t)lv.nx * lv.ny;
        lv.hx = P.grid.hx * std::ldexp(1.0, l);
        lv.hy = (dim == 2 ? P.grid.hy : P.grid.hx) * std::ldexp(1.0, l);
        if (l > 0) {
            lv.v = c.soa(lv.n, dim);
            lv.u = c.soa(lv.n, dim);
            lv.u2 = c.soa(lv.n, dim);
            lv.f = c.soa(lv.n, dim);
            lv.rb = c.soa(lv.n, dim);
            lv.sa = c.take(lv.n);
            lv.ss = c.take(lv.n);
            if (P.params.nu_l > 1) {
                lv.rt = c.soa(lv.n, dim);
                lv.g = c.take(lv.n);
            }
        }
    }
    if (P.params.precision == M1_MIXED) {
        P.base32 = c.soa32(n0, dim);
        P.r32 = c.soa32(n0, dim);
        P.dA = c.soa32(n0, dim);
        P.dB = c.soa32(n0, dim);
        P.rho0 = c.soa32(n0, dim);
        for (int l = 0; l < P.L; ++l) {
            LevelBuf& lv = P.lev[l];
            lv.sa32 = c.take32(lv.n);
            lv.ss32 = c.take32(lv.n);
            if (l > 0) {
                lv.w = c.soa32(lv.n, dim);
                lv.d = c.soa32(lv.n, dim);
                lv.e = c.soa32(lv.n, dim);
                lv.e2 = c.soa32(lv.n, dim);
                lv.gg = c.soa32(lv.n, dim);
                lv.rho = c.soa32(lv.n, dim);
                lv.fr = c.soa32(lv.n, dim);
            }
        }
    }
    P.npart = (int)((n0 + 255) / 256);
    P.partials = c.take(P.npart);
    P.dscal = c.take(8);
    P.dbad = reinterpret_cast<unsigned long long*>(c.take(1));
    P.dctrl = reinterpret_cast<m1::Ctrl*>(c.take((sizeof(m1::Ctrl) + 7) / 8));
    P.dfix = reinterpret_cast<m1::Ctrl*>(c.take((sizeof(m1::Ctrl) + 7) / 8));
    P.dstall = reinterpret_cast<unsigned long long*>(c.take(1));
    P.dtail = reinterpret_cast<m1::TailArgs*>(c.take((sizeof(m1::TailArgs) + 7) / 8));
    if (P.params.precision == M1_MIXED)
        P.dtail32 = reinterpret_cast<m1::TailArgs32*>(c.take((sizeof(m1::TailArgs32) + 7) / 8));
}

// Levels with at most this many cells run inside the single-workgroup tail kernel.
// Launch-shape settings (m1_tune_set): read when a plan or engine is created.
// Environment variables give the initial values.  None of them changes results.
struct Tuning {
    std::atomic<int64_t> tail_cells{256};          // levels of at most this many cells run in the one-workgroup tail
    std::atomic<int64_t> tiled_max_cells{65536};   // largest level smoothed by the LDS-tiled legs
    std::atomic<int64_t> graphs{0};                // replay V-cycles from hipGraph recordings
    Tuning()
    {
        if (const char* e = std::getenv("M1_GRAPHS")) graphs = std::atoll(e) != 0;
        if (const char* e = std::getenv("M1_SWEEP_ROWS")) (void)m1::set_sweep_rows(std::atoi(e));
        if (const char* e = std::getenv("M1_PAIR_ROWS")) (void)m1::set_pair_rows(std::atoi(e));
        if (const char* e = std::getenv("M1_MX_SWEEP_ROWS")) (void)m1::set_mx_sweep_rows(std::atoi(e));
        if (const char* e = std::getenv("M1_RESIDUAL_RESTRICT")) m1::set_residual_restrict(std::atoi(e));
        if (const char* e = std::getenv("M1_TAIL_CELLS")) tail_cells = std::atoll(e);
        if (const char* e = std::getenv("M1_TILED_MAX_CELLS")) tiled_max_cells = std::atoll(e);
        if (const char* e = std::getenv("M1_BATCH_GRID")) {
            const int v = std::atoi(e);
            if (v > 0) m1::set_batch_grid_cap(v);
        }
    }
};
Tuning& tuning()
{
    static Tuning t;
    return t;
}
int64_t tail_cells() { return tuning().tail_cells.load(); }
int64_t tiled_max_cells() { return tuning().tiled_max_cells.load(); }
bool use_graphs() { return tuning().graphs.load() != 0; }

// Boundary cells a (counted along a side of n cells) whose centres (a + 1/2)/n lie in [lo, hi]:
// a in [s0, s1).  Only inflow sides have any.
void inflow_cells(const m1_bc& b, int n, int& s0, int& s1)
{
    s0 = s1 = 0;
    if (b.kind != M1_BC_INFLOW) return;
    s0 = std::max(0, (int)std::ceil(b.lo * n - 0.5));
    s1 = std::min(n, (int)std::floor(b.hi * n - 0.5) + 1);
    if (s1 < s0) s1 = s0;
}

void fill_level_params(m1_plan& P)
{
    const m1_grid& g = P.grid;
    for (int l = 0; l < P.L; ++l) {
        LevelBuf& lv = P.lev[l];
        lv.L.nx = lv.nx;
        lv.L.ny = lv.ny;
        lv.L.sh = m1::row_shift(lv.nx);
        lv.L.kx = g.dt / (2.0 * lv.hx);
        lv.L.ky = g.dim == 2 ? g.dt / (2.0 * lv.hy) : 0.0;
        lv.L.a = 1.0 + g.c * g.dt / lv.hx;
        if (g.dim == 2) lv.L.a += g.c * g.dt / lv.hy;
        lv.L.cdt = g.c * g.dt;
        lv.L.sa = lv.sa;
        lv.L.ss = lv.ss;
        for (int sd = 0; sd < 4; ++sd) {
            const bool on = g.dim == 2 || sd < 2;
            if (on) inflow_cells(g.bc[sd], sd < 2 ? lv.ny : lv.nx, lv.L.sg0[sd], lv.L.sg1[sd]);
            else lv.L.sg0[sd] = lv.L.sg1[sd] = 0;
        }
        lv.L32 = m1::Lvl32{lv.nx, lv.ny, lv.L.sh, (float)lv.L.kx, (float)lv.L.ky, (float)lv.L.a, (float)lv.L.cdt, lv.sa32,
                           lv.ss32, {}, {}};
        for (int sd = 0; sd < 4; ++sd) {
            lv.L32.sg0[sd] = lv.L.sg0[sd];
            lv.L32.sg1[sd] = lv.L.sg1[sd];
        }
    }
}

bool same(const Soa& a, const Soa& b) { return a.E == b.E; }

m1_status hip_status(hipError_t e) { return e == hipSuccess ? M1_OK : M1_ERR_DEVICE; }

m1_status last_launch() { return hip_status(hipGetLastError()); }

// ---- building blocks of the cycle ----------------------------------------
// Per-cycle gating: the pseudo-time step and the `active` flag either come from
// the device cycle control (whole cycles enqueued ahead) or are plain values.
struct Gate {
    double dtau;
    const double* dtau_dev;
    const int* active;
};

// Gate of a single operation outside a time step: the plan's always-live
// control, with its pseudo-time step set to `dtau` (stream-ordered).
Gate fixed_gate(m1_plan& P, double dtau)
{
    m1::Ctrl fix{};
    fix.active = 1;
    fix.dtau = dtau;
    m1::launch_ctrl_init(P.st, P.dfix, fix);
    return Gate{dtau, &P.dfix->dtau, &P.dfix->active};
}

// nu finest-level sweeps.  With `control` the first sweep also reduces the
// residual norm of its input (the previous cycle's result) and the cycle
// control then updates dtau / the stop flag before the rest of the cycle runs.
// One launch of finest-level sweeps of A_0(u) = b from `in` into `out`: two
// (the fused pair) when `two` allows it and that launch shape is on, else one
// (reducing the norm of `in` into `partials` when given).  Returns the count.
int fine_launch(m1_plan& P, const CSoa& b, const CSoa& in, const Soa& out, bool two, double* partials,
                const int* active)
{
    const LevelBuf& f = P.lev[0];
    if (P.params.smoother == M1_SMOOTH_RBGS) {  // red cells into the plan's finest residual buffer, then black
        m1::launch_relax_colour(P.st, P.dim, P.ph, f.L, b, P.params.omega, 0, in, P.rfine, partials, active);
        m1::launch_relax_colour(P.st, P.dim, P.ph, f.L, b, P.params.omega, 1, cs(P.rfine), out, nullptr, active);
        return 1;
    }
    if (two && !partials && P.dim == 2 && m1::launch_relax2_lds(P.st, P.ph, f.L, b, P.params.omega, in, out, active))
        return 2;
    m1::launch_relax(P.st, P.dim, P.ph, f.L, b, nullptr, 0.0, 1.0, P.params.omega, in, out, partials, active);
    return 1;
}

void fine_sweeps(m1_plan& P, Soa& cur, Soa& other, int nu, const Gate& G, bool control = false)
{
    for (int s = 0; s < nu;) {
        const bool norm = control && s == 0;
        s += fine_launch(P, cs(P.b), cs(cur), other, nu - s >= 2, norm ? P.partials : nullptr, G.active);
        if (norm) m1::launch_norm_control(P.st, P.partials, P.npart, P.dctrl);
        std::swap(cur, other);
    }
}

// params.pseudo_steps pseudo-time steps of level l from `start`; result in u or u2.
// `first`: the smoothing starts from v_l and its first step forms f = A(v_l) + R(rbar).
Soa pseudo_smooth(m1_plan& P, int l, const Gate& G, Soa start, bool first)
{
    LevelBuf& c = P.lev[l];
    const bool store = P.params.nu_l > 1;
    Soa in = start;
    for (int m = 0; m < P.params.pseudo_steps; ++m) {
        Soa out = same(in, c.u) ? c.u2 : c.u;
        m1::launch_pseudo(P.st, P.dim, P.ph, c.L, c.f, cs(in), out, G.dtau, G.dtau_dev, P.reach,
                          P.params.pseudo_local, first && m == 0, store ? c.rt : Soa{}, store ? c.g : nullptr,
                          G.active);
        in = out;
        for (int s = 1; s < P.params.nu_l; ++s) {
            out = same(in, c.u) ? c.u2 : c.u;
            m1::launch_relax(P.st, P.dim, P.ph, c.L, cs(c.rt), c.g, 1.0, 0.0, 1.0, cs(in), out, nullptr, G.active);
            in = out;
        }
    }
    return in;
}

m1::Fields fields2(const Soa& a, const Soa& b, const Soa& ca, const Soa& cb, int dim)
{
    m1::Fields F{};
    int n = 0;
    auto add = [&](const double* i, double* o) {
        if (i) {
            F.in[n] = i;
            F.out[n] = o;
            ++n;
        }
    };
    add(a.E, ca.E);
    add(a.Fx, ca.Fx);
    if (dim == 2) add(a.Fy, ca.Fy);
    add(a.T, ca.T);
    if (b.E) {
        add(b.E, cb.E);
        add(b.Fx, cb.Fx);
        if (dim == 2) add(b.Fy, cb.Fy);
        add(b.T, cb.T);
    }
    F.n = n;
    return F;
}

// One V-cycle (Appendix A) on the finest iterate `cur` (partner buffer `other`).
// Levels below P.lt run as grid kernels; levels P.lt..L-1 run inside the
// single-workgroup tail kernel (which leaves its result in lev[lt].u).
void vcycle_impl(m1_plan& P, Soa& cur, Soa& other, const Gate& G, bool control = false)
{
    const m1_params& p = P.params;
    fine_sweeps(P, cur, other, p.nu0, G, control);
    if (P.L == 1) return;
    // residuals are restricted as they are formed (one launch per level) unless switched off
    const bool fused = P.dim == 2 && m1::residual_restrict();
    if (!fused) m1::launch_apply(P.st, P.dim, P.ph, P.lev[0].L, cs(cur), cs(P.b), -1.0, P.rfine, nullptr, G.active);
    Soa ul[kMaxPlanLevels];
    // levels smoothed by one LDS-tiled launch per leg: R(rbar) goes to rb, which the
    // down leg reads while it writes the FAS right-hand side into f
    // (only up to tiled_max_cells: larger levels stream well as one launch per step, and the halo
    // work and the large LDS blocks of the tiled form cost more than the launches it saves)
    bool tiled[kMaxPlanLevels] = {};
    for (int l = 1; l < std::min(P.lt, P.L); ++l)
        tiled[l] = P.tiled && P.lev[l].n <= P.tiled_max && m1::smooth_tb_fits(P.dim, P.lev[l].L, p.pseudo_steps);
    ul[0] = cur;
    Soa rb_prev = P.rfine;
    for (int l = 1; l < P.L; ++l) {
        LevelBuf& c = P.lev[l];
        const LevelBuf& f = P.lev[l - 1];
        if (fused)  // rbar = f - A(u) of level l - 1 (b on the finest) and both restrictions
            m1::launch_residual_restrict(P.st, P.ph, f.L, cs(ul[l - 1]), l == 1 ? cs(P.b) : cs(f.f), -1.0, P.px,
                                         P.py, c.v, tiled[l] ? c.rb : c.f, G.active);
        else
            m1::launch_restrict(P.st, P.dim, f.nx, f.ny, P.px, P.py,
                                fields2(ul[l - 1], rb_prev, c.v, tiled[l] ? c.rb : c.f, P.dim), G.active);
        if (l == P.lt) {  // the rest of the cycle below (and including) level lt
            m1::launch_tail(P.st, P.dim, P.dtail, G.dtau, G.dtau_dev, G.active);
            ul[l] = c.u;
            break;
        }
        if (tiled[l]) {
            m1::launch_smooth_tb(P.st, P.ph, c.L, p.pseudo_steps, m1::kLegDown, cs(c.rb), c.f, cs(c.v), c.u, G.dtau_dev,
                                 P.reach, p.pseudo_local, CSoa{}, CSoa{}, P.px, P.py, p.eta, G.active);
            ul[l] = c.u;
        } else {
            ul[l] = pseudo_smooth(P, l, G, c.v, true);  // also forms f = A(v) + R(rbar)
        }
        if (l < P.L - 1 && !fused) {
            m1::launch_apply(P.st, P.dim, P.ph, c.L, cs(ul[l]), cs(c.f), -1.0, c.rb, nullptr, G.active);
            rb_prev = c.rb;
        }
    }
    const int top = std::min(P.lt, P.L - 1);
    for (int l = top - 1; l >= 0; --l) {
        const LevelBuf& c = P.lev[l + 1];
        LevelBuf& f = P.lev[l];
        if (tiled[l]) {  // prolongation, projection and the post-smoothing in one launch
            const Soa out = same(ul[l], f.u) ? f.u2 : f.u;
            m1::launch_smooth_tb(P.st, P.ph, f.L, p.pseudo_steps, m1::kLegUp, cs(f.f), f.f, cs(ul[l]), out, G.dtau_dev,
                                 P.reach, p.pseudo_local, cs(ul[l + 1]), cs(c.v), P.px, P.py, p.eta, G.active);
            ul[l] = out;
            continue;
        }
        if (l == 0 && P.dim == 2 && p.nu0 > 0 && p.smoother == M1_SMOOTH_JACOBI &&
            m1::launch_relax_lds(P.st, P.ph, f.L, cs(P.b), p.omega, cs(ul[0]), other, G.active, cs(ul[1]), cs(c.v),
                                 P.px, P.py, p.eta)) {
            // correction, projection and the first post-sweep in one launch
            cur = other;
            other = ul[0];
            fine_sweeps(P, cur, other, p.nu0 - 1, G);
            continue;
        }
        m1::launch_prolong_project(P.st, P.dim, P.ph, f.nx, f.ny, P.px, P.py, p.eta, cs(ul[l]), cs(ul[l + 1]),
                                   cs(c.v), ul[l], G.active);
        if (l == 0) {
            cur = ul[0];
            fine_sweeps(P, cur, other, p.nu0, G);
        } else {
            ul[l] = pseudo_smooth(P, l, G, ul[l], false);
        }
    }
}

// ---- the plan's transfer operators ------------------------------------------
// Full weighting and linear prolongation (Sect. 4.2), or the cell-agglomeration
// pair (the 2^d-cell mean and the piecewise-constant prolongation).
bool mean_transfer(const m1_plan& P) { return P.params.transfer == M1_TRANSFER_MEAN; }

void plan_restrict(m1_plan& P, int l, const m1::Fields& F, const int* active)
{
    const LevelBuf& f = P.lev[l];
    if (mean_transfer(P)) m1::launch_restrict_mean(P.st, P.dim, f.nx, f.ny, F, active);
    else m1::launch_restrict(P.st, P.dim, f.nx, f.ny, P.px, P.py, F, active);
}

// out = u + P(uc - vc) on level l with the admissibility correction (eq. prolongatedSol)
void plan_prolong_project(m1_plan& P, int l, const CSoa& u, const CSoa& uc, const CSoa& vc, const Soa& out,
                          const int* active)
{
    const LevelBuf& f = P.lev[l];
    if (mean_transfer(P))
        m1::launch_prolong_const_project(P.st, P.dim, P.ph, f.nx, f.ny, P.params.eta, u, uc, vc, out, active);
    else
        m1::launch_prolong_project(P.st, P.dim, P.ph, f.nx, f.ny, P.px, P.py, P.params.eta, u, uc, vc, out, active);
}

// ---- W- and F-cycles (Sect. 6.3) --------------------------------------------
// The cycle written as a recursion over the coarse problems (no tail): a visit
// of level l smooths its FAS problem in pseudo time (Algorithm 3), restricts
// the iterate and its residual to level l + 1, visits that level once (V),
// twice (W) or by an F-cycle then a V-cycle (F), corrects with admissibility
// (eq. prolongatedSol) and smooths again; the coarsest level is smoothed once
// per visit.  Levels small enough for the tiled legs (as in the V-cycle) run
// each smoothing as one launch: the first of a descent forming the FAS
// right-hand side, a later visit's pre-smoothing plain, and the correction
// with the post-smoothing; the finest level's correction is fused with its
// first post-sweep.  Every launch gives the one-step kernels' bits.

// Whether level l's smoothing legs run as tiled launches.
bool rc_tiled(const m1_plan& P, int l)
{
    return l >= 1 && l < P.L && P.tiled && P.lev[l].n <= P.tiled_max &&
           m1::smooth_tb_fits(P.dim, P.lev[l].L, P.params.pseudo_steps);
}

// v_{l+1} = R(u) and R(rhs - A_l(u)) into level l + 1 (its f, or its rb when
// that level is tiled; the first pseudo-time step of the next visit turns it
// into A(v_{l+1}) + R(rbar)).
void descend(m1_plan& P, int l, const Soa& u, const Gate& G)
{
    const LevelBuf& f = P.lev[l];
    LevelBuf& c = P.lev[l + 1];
    const CSoa rhs = l == 0 ? cs(P.b) : cs(f.f);
    const Soa to = rc_tiled(P, l + 1) ? c.rb : c.f;
    if (P.dim == 2 && m1::residual_restrict() && !mean_transfer(P)) {
        m1::launch_residual_restrict(P.st, P.ph, f.L, cs(u), rhs, -1.0, P.px, P.py, c.v, to, G.active);
        return;
    }
    const Soa r = l == 0 ? P.rfine : f.rb;
    m1::launch_apply(P.st, P.dim, P.ph, f.L, cs(u), rhs, -1.0, r, nullptr, G.active);
    plan_restrict(P, l, fields2(u, r, c.v, to, P.dim), G.active);
}

Soa coarse_visit(m1_plan& P, int l, int kind, const Gate& G, Soa u, bool first);

// Visit level l + 1 as `kind` prescribes; its final iterate.
Soa visit_below(m1_plan& P, int l, int kind, const Gate& G)
{
    const LevelBuf& c = P.lev[l + 1];
    Soa uc;
    if (kind == M1_CYCLE_F) {
        uc = coarse_visit(P, l + 1, M1_CYCLE_F, G, c.v, true);
        uc = coarse_visit(P, l + 1, M1_CYCLE_V, G, uc, false);
    } else {
        uc = coarse_visit(P, l + 1, kind, G, c.v, true);
        if (kind == M1_CYCLE_W) uc = coarse_visit(P, l + 1, kind, G, uc, false);
    }
    return uc;
}

// The m pseudo-time steps of level l >= 1 from u as one tiled launch (first:
// forming f from R(rbar) in rb); the result in the level buffer u is not in.
Soa tiled_leg(m1_plan& P, int l, const Gate& G, const Soa& u, bool first)
{
    LevelBuf& c = P.lev[l];
    const Soa out = same(u, c.u) ? c.u2 : c.u;
    m1::launch_smooth_tb(P.st, P.ph, c.L, P.params.pseudo_steps, first ? m1::kLegDown : m1::kLegPlain,
                         first ? cs(c.rb) : cs(c.f), c.f, cs(u), out, G.dtau_dev, P.reach, P.params.pseudo_local,
                         CSoa{}, CSoa{}, P.px, P.py, P.params.eta, G.active);
    return out;
}

// One visit of coarse level l from the iterate u (v_l on the first visit of a
// descent, whose first pseudo-time step forms f = A(v_l) + R(rbar)).
Soa coarse_visit(m1_plan& P, int l, int kind, const Gate& G, Soa u, bool first)
{
    const bool tl = rc_tiled(P, l);
    u = tl ? tiled_leg(P, l, G, u, first) : pseudo_smooth(P, l, G, u, first);
    if (l == P.L - 1) return u;
    descend(P, l, u, G);
    const Soa uc = visit_below(P, l, kind, G);
    const LevelBuf& c = P.lev[l + 1];
    LevelBuf& f = P.lev[l];
    if (tl) {  // correction, projection and the post-smoothing in one launch
        const Soa out = same(u, f.u) ? f.u2 : f.u;
        m1::launch_smooth_tb(P.st, P.ph, f.L, P.params.pseudo_steps, m1::kLegUp, cs(f.f), f.f, cs(u), out,
                             G.dtau_dev, P.reach, P.params.pseudo_local, cs(uc), cs(c.v), P.px, P.py, P.params.eta,
                             G.active);
        return out;
    }
    plan_prolong_project(P, l, cs(u), cs(uc), cs(c.v), u, G.active);
    return pseudo_smooth(P, l, G, u, false);
}

void rcycle_impl(m1_plan& P, Soa& cur, Soa& other, const Gate& G, bool control)
{
    const m1_params& p = P.params;
    fine_sweeps(P, cur, other, p.nu0, G, control);
    if (P.L == 1) return;
    descend(P, 0, cur, G);
    const Soa uc = visit_below(P, 0, p.cycle, G);
    const LevelBuf& c = P.lev[1];
    if (P.dim == 2 && p.nu0 > 0 && p.smoother == M1_SMOOTH_JACOBI && !mean_transfer(P) &&
        m1::launch_relax_lds(P.st, P.ph, P.lev[0].L, cs(P.b), p.omega, cs(cur), other, G.active, cs(uc), cs(c.v),
                             P.px, P.py, p.eta)) {
        // correction, projection and the first post-sweep in one launch
        std::swap(cur, other);
        fine_sweeps(P, cur, other, p.nu0 - 1, G);
        return;
    }
    plan_prolong_project(P, 0, cs(cur), cs(uc), cs(c.v), cur, G.active);
    fine_sweeps(P, cur, other, p.nu0, G);
}

// One cycle of the plan's shape (the V-cycle with full weighting has its own fused form).
void cycle_impl(m1_plan& P, Soa& cur, Soa& other, const Gate& G, bool control = false)
{
    if (P.params.cycle == M1_CYCLE_V && !mean_transfer(P)) vcycle_impl(P, cur, other, G, control);
    else rcycle_impl(P, cur, other, G, control);
}

// ---- mixed precision -------------------------------------------------------
m1::Fields32 fields32(std::initializer_list<std::pair<const Soa32*, const Soa32*>> pairs, int dim)
{
    m1::Fields32 F{};
    int n = 0;
    for (auto& pr : pairs) {
        const Soa32& a = *pr.first;
        const Soa32& b = *pr.second;
        F.in[n] = a.E;
        F.out[n++] = b.E;
        F.in[n] = a.Fx;
        F.out[n++] = b.Fx;
        if (dim == 2) {
            F.in[n] = a.Fy;
            F.out[n++] = b.Fy;
        }
        F.in[n] = a.T;
        F.out[n++] = b.T;
    }
    F.n = n;
    return F;
}

bool same32(const Soa32& a, const Soa32& b) { return a.E == b.E; }

Soa32 mx_pseudo_smooth(m1_plan& P, int l, const Gate& G, Soa32 start, bool first)
{
    LevelBuf& c = P.lev[l];
    Soa32 in = start;
    for (int m = 0; m < P.params.pseudo_steps; ++m) {
        const Soa32 out = same32(in, c.e) ? c.e2 : c.e;
        m1::launch_mx_pseudo(P.st, P.dim, P.ph, c.L32, cs(c.w), c.gg, c.fr, cs(in), out, G.dtau, G.dtau_dev,
                             (float)P.reach, P.params.pseudo_local, first && m == 0, G.active);
        in = out;
    }
    return in;
}

// Mixed-precision W- and F-cycles: the recursion of the FP64 form on the FP32
// correction levels.  Level l >= 1 carries the base w, the restricted
// correction d, the iterate e/e2 and the FAS right-hand side g (and the
// explicit sub-steps' source fr); a visit smooths from d (the first of a
// descent, which forms g and fr) or from the previous visit's result.

// rho of level l (r - N(d) on the finest level, g - N_w(e) below) restricted
// with w and the correction into level l + 1 (w, d, g).
void mx_descend(m1_plan& P, int l, const Soa32& e, const Gate& G)
{
    const LevelBuf& fl = P.lev[l];
    LevelBuf& c = P.lev[l + 1];
    const Soa32& w = l == 0 ? P.base32 : fl.w;
    const Soa32& rhs = l == 0 ? P.r32 : fl.gg;
    if (P.dim == 2 && m1::residual_restrict()) {
        m1::launch_mx_residual_restrict(P.st, P.ph, fl.L32, cs(w), cs(e), cs(rhs), -1.0f, P.px, P.py, c.w, c.d, c.gg,
                                        G.active);
        return;
    }
    const Soa32& rho = l == 0 ? P.rho0 : fl.rho;
    m1::launch_mx_apply(P.st, P.dim, P.ph, fl.L32, cs(w), cs(e), cs(rhs), -1.0f, rho, G.active);
    m1::launch_mx_restrict(P.st, P.dim, fl.nx, fl.ny, P.px, P.py, fields32({{&w, &c.w}, {&e, &c.d}, {&rho, &c.gg}},
                                                                           P.dim),
                           G.active);
}

Soa32 mx_coarse_visit(m1_plan& P, int l, int kind, const Gate& G, Soa32 e, bool first);

// Visit level l + 1 as `kind` prescribes; its final iterate.
Soa32 mx_visit_below(m1_plan& P, int l, int kind, const Gate& G)
{
    const LevelBuf& c = P.lev[l + 1];
    Soa32 ec;
    if (kind == M1_CYCLE_F) {
        ec = mx_coarse_visit(P, l + 1, M1_CYCLE_F, G, c.d, true);
        ec = mx_coarse_visit(P, l + 1, M1_CYCLE_V, G, ec, false);
    } else {
        ec = mx_coarse_visit(P, l + 1, kind, G, c.d, true);
        if (kind == M1_CYCLE_W) ec = mx_coarse_visit(P, l + 1, kind, G, ec, false);
    }
    return ec;
}

Soa32 mx_coarse_visit(m1_plan& P, int l, int kind, const Gate& G, Soa32 e, bool first)
{
    e = mx_pseudo_smooth(P, l, G, e, first);
    if (l == P.L - 1) return e;
    mx_descend(P, l, e, G);
    const Soa32 ec = mx_visit_below(P, l, kind, G);
    const LevelBuf& c = P.lev[l + 1];
    const LevelBuf& fl = P.lev[l];
    m1::launch_mx_prolong(P.st, P.dim, P.ph, fl.nx, fl.ny, P.px, P.py, (float)P.params.eta, cs(fl.w), cs(e), cs(ec),
                          cs(c.d), e, G.active);
    return mx_pseudo_smooth(P, l, G, e, false);
}

// One mixed-precision cycle (V, W or F).  cur64 holds the FP64 state; the pending FP32
// correction of the previous cycle (`first`: none) is applied by the FP64
// residual kernel, which writes the updated state into the partner buffer.
// On return `pend` is this cycle's correction (applied by the next cycle or
// by the caller).  With `control` the FP64 residual norm feeds the cycle control.
// False (nothing enqueued) if the buffers would alias.
bool mx_cycle(m1_plan& P, Soa& cur64, Soa& other64, const Gate& G, bool control, bool first, Soa32& pend)
{
    const m1_params& p = P.params;
    const LevelBuf& f0 = P.lev[0];
    const float om = (float)p.omega;
    // The first pre-sweep (from a zero correction) runs inside the residual launch.  That launch reads the
    // pending correction at every cell's neighbours, so the sweep writes the correction buffer the pending
    // one is not in (where the previous cycle left it depends on nu0, the launch shapes and the level count).
    const bool zero_fused = p.nu0 >= 1;
    const Soa32 z = (!first && same32(pend, P.dA)) ? P.dB : P.dA;
    if (!m1::launch_mx_resid(P.st, P.dim, P.ph, f0.L, p.eta, cs(cur64), first ? CSoa32{} : cs(pend), cs(P.b),
                             other64, P.base32, P.r32, control ? P.partials : nullptr, G.active,
                             zero_fused ? &f0.L32 : nullptr, om, zero_fused ? z : Soa32{}))
        return false;
    std::swap(cur64, other64);
    if (control) m1::launch_norm_control(P.st, P.partials, P.npart, P.dctrl);
    auto sweeps = [&](Soa32 d, int count, bool from_zero) {
        for (int s = 0; s < count;) {
            const Soa32 out = same32(d, P.dA) ? P.dB : P.dA;
            const bool zero = from_zero && s == 0;
            if (!zero && count - s >= 2 && P.dim == 2 &&
                m1::launch_mx_sweep2(P.st, P.ph, f0.L32, cs(P.base32), cs(d), cs(P.r32), om, out, G.active)) {
                d = out;  // two sweeps, one launch
                s += 2;
                continue;
            }
            m1::launch_mx_sweep(P.st, P.dim, P.ph, f0.L32, cs(P.base32), zero ? CSoa32{} : cs(d), cs(P.r32), 0.0f,
                                1.0f, om, out, G.active);
            d = out;
            ++s;
        }
        return d;
    };
    Soa32 d = zero_fused ? sweeps(z, p.nu0 - 1, false) : sweeps(P.dB, p.nu0, true);
    if (P.L == 1) {
        pend = d;
        return true;
    }
    Soa32 el[kMaxPlanLevels];
    el[0] = d;
    if (p.cycle == M1_CYCLE_V) {
        const bool fused = P.dim == 2 && m1::residual_restrict();  // rho0 restricted as it is formed
        if (!fused)
            m1::launch_mx_apply(P.st, P.dim, P.ph, f0.L32, cs(P.base32), cs(d), cs(P.r32), -1.0f, P.rho0, G.active);
        const Soa32* wprev = &P.base32;
        const Soa32* rprev = &P.rho0;
        for (int l = 1; l < P.L; ++l) {
            LevelBuf& c = P.lev[l];
            const LevelBuf& fl = P.lev[l - 1];
            if (fused)  // rho of level l - 1 (r - N(d) on the finest, g - N_w(e) below) and the restrictions
                m1::launch_mx_residual_restrict(P.st, P.ph, fl.L32, cs(*wprev), cs(el[l - 1]),
                                                l == 1 ? cs(P.r32) : cs(fl.gg), -1.0f, P.px, P.py, c.w, c.d, c.gg,
                                                G.active);
            else
                m1::launch_mx_restrict(P.st, P.dim, fl.nx, fl.ny, P.px, P.py,
                                       fields32({{wprev, &c.w}, {&el[l - 1], &c.d}, {rprev, &c.gg}}, P.dim),
                                       G.active);
            if (l == P.lt) {  // the rest of the cycle below (and including) level lt in one workgroup
                m1::launch_mx_tail(P.st, P.dim, P.dtail32, G.dtau, G.dtau_dev, G.active);
                el[l] = c.e;
                break;
            }
            el[l] = mx_pseudo_smooth(P, l, G, c.d, true);  // forms g = N_w(d) + R(rho)
            if (l < P.L - 1 && !fused)
                m1::launch_mx_apply(P.st, P.dim, P.ph, c.L32, cs(c.w), cs(el[l]), cs(c.gg), -1.0f, c.rho, G.active);
            wprev = &c.w;
            rprev = &c.rho;
        }
        for (int l = std::min(P.lt, P.L - 1) - 1; l >= 1; --l) {
            const LevelBuf& c = P.lev[l + 1];
            const LevelBuf& fl = P.lev[l];
            m1::launch_mx_prolong(P.st, P.dim, P.ph, fl.nx, fl.ny, P.px, P.py, (float)p.eta, cs(fl.w), cs(el[l]),
                                  cs(el[l + 1]), cs(c.d), el[l], G.active);
            el[l] = mx_pseudo_smooth(P, l, G, el[l], false);
        }
    } else {  // W- or F-cycle: the coarse problems as a recursion
        mx_descend(P, 0, d, G);
        el[1] = mx_visit_below(P, 0, p.cycle, G);
    }
    const Soa32 post = same32(el[0], P.dA) ? P.dB : P.dA;
    if (P.dim == 2 && p.nu0 >= 1 &&
        m1::launch_mx_prolong_sweep(P.st, P.ph, f0.L32, cs(P.base32), cs(cur64), cs(el[0]), cs(el[1]),
                                    cs(P.lev[1].d), P.px, P.py, p.eta, cs(P.r32), om, post, G.active)) {
        pend = sweeps(post, p.nu0 - 1, false);  // the first post-sweep ran with the correction
        return true;
    }
    m1::launch_mx_prolong_fine(P.st, P.dim, P.ph, f0.nx, f0.ny, P.px, P.py, p.eta, cs(cur64), cs(el[0]), cs(el[1]),
                               cs(P.lev[1].d), el[0], G.active);
    pend = sweeps(el[0], p.nu0, false);
    return true;
}

// ---- recorded launch sequences (hipGraph) -----------------------------------
// Record what `enqueue` launches on the stream in `*slot` into an executable
// graph: during the recording the slot holds the private stream `cap` (created
// on first use), so nothing runs and the caller's stream is untouched.
template <class F>
m1_status record(hipStream_t* slot, hipStream_t& cap, F&& enqueue, hipGraphExec_t* out)
{
    *out = nullptr;
    if (!cap && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return M1_ERR_DEVICE;
    const hipStream_t saved = *slot;
    *slot = cap;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        enqueue();
        const hipError_t launch = hipGetLastError();
        e = hipStreamEndCapture(cap, &g);
        if (e == hipSuccess) e = launch;
    }
    *slot = saved;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return hip_status(e);
}

void drop_cycle_graphs(m1_plan& P)
{
    if (P.cyc.empty()) return;
    (void)hipStreamSynchronize(P.st);
    for (auto& c : P.cyc) (void)hipGraphExecDestroy(c.exec);
    P.cyc.clear();
}

// One controlled V-cycle of a time step, replayed from its recording (made on
// first use for these buffers).  Every launch of a cycle is fixed by the plan
// and the buffers it starts from: the cycle control, dtau and stop flag are
// read by the kernels from device memory.
m1_status graph_cycle(m1_plan& P, Soa& cur, Soa& other, Soa32& pend, const Gate& G, bool first)
{
    const bool f = P.mixed && first;
    const float* pk = (P.mixed && !first) ? pend.E : nullptr;
    m1_plan::CycleGraph* hit = nullptr;
    for (auto& c : P.cyc)
        if (c.in_cur == cur.E && c.in_other == other.E && c.in_pend == pk && c.first == f) hit = &c;
    if (!hit) {
        if (P.cyc.size() >= 8) drop_cycle_graphs(P);  // state buffers of earlier calls
        m1_plan::CycleGraph c{cur.E, other.E, pk, f, cur, other, pend, nullptr};
        bool ok = true;
        const m1_status s = record(&P.st, P.cap, [&] {
            if (P.mixed) ok = mx_cycle(P, c.cur, c.other, G, true, first, c.pend);
            else cycle_impl(P, c.cur, c.other, G, true);
        }, &c.exec);
        if (s == M1_OK && !ok) (void)hipGraphExecDestroy(c.exec);
        if (s != M1_OK) return s;
        if (!ok) return M1_ERR_DEVICE;
        P.cyc.push_back(c);
        hit = &P.cyc.back();
    }
    if (hipGraphLaunch(hit->exec, P.st) != hipSuccess) return M1_ERR_DEVICE;
    cur = hit->cur;
    other = hit->other;
    pend = hit->pend;
    return M1_OK;
}

// |b + sgn A_0(v)| (sgn = -1: the residual; 0: |b|) into P.dscal[0] (device)
// and, after a sync, the host.
m1_status fine_norm(m1_plan& P, const Soa& v, Soa r_out, double* out, double sgn = -1.0)
{
    m1::launch_apply(P.st, P.dim, P.ph, P.lev[0].L, cs(v), cs(P.b), sgn, r_out, P.partials, &P.dfix->active);
    m1::launch_norm_finalize(P.st, P.partials, P.npart, P.dscal);
    hipError_t e = hipMemcpyAsync(P.hpin, P.dscal, sizeof(double), hipMemcpyDeviceToHost, P.st);
    if (e != hipSuccess) return M1_ERR_DEVICE;
    e = hipStreamSynchronize(P.st);
    if (e != hipSuccess) return M1_ERR_DEVICE;
    *out = P.hpin[0];
    return last_launch();
}

double adapt_dtau(const m1_params& p, double dtau, double r0, double rprev, double r)
{
    const double d = (p.dtau_rule == M1_DTAU_LITERAL) ? std::fabs(r - rprev) / r0 : (rprev - r) / rprev;
    if (d > p.eps_inc) dtau *= 1.1;
    if (d < p.eps_dec) dtau *= 0.5;
    return std::min(std::max(dtau, p.dtau_min), p.dtau_max);
}

Soa to_soa(const m1_state* s) { return Soa{s->E, s->Fx, s->Fy, s->T}; }

bool valid_state(const m1_plan* P, const m1_state* s)
{
    if (!s || !s->E || !s->Fx || !s->T) return false;
    return (P->dim == 2) == (s->Fy != nullptr);
}

bool valid_level_state(const m1_plan* P, const m1_state* s) { return valid_state(P, s); }

}  // namespace

// ============================================================================
extern "C" {

const char* m1_strerror(m1_status s)
{
    switch (s) {
    case M1_OK: return "ok";
    case M1_ERR_ARG: return "invalid argument";
    case M1_ERR_NOT_ADMISSIBLE: return "state not admissible (E > 0, T > 0, |F| <= cE required)";
    case M1_ERR_NO_CONVERGENCE: return "no convergence within max_cycles";
    case M1_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case M1_ERR_DEVICE: return "HIP runtime error";
    case M1_ERR_BUSY: return "busy";
    case M1_ERR_BUDGET: return "request exceeds the memory budget";
    }
    return "unknown status";
}

void m1_default_params(m1_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->levels = 0;
    p->nu0 = 3;
    p->nu_l = 1;
    p->pseudo_steps = 3;
    p->sub_steps = 4;
    p->max_cycles = 10000;
    p->dtau_rule = M1_DTAU_SIGNED;
    p->pseudo_local = 1;
    p->precision = M1_FP64;
    p->dtau_carry = 1;
    p->dtau_im0 = 1e-3;
    p->eps_inc = 0.05;
    p->eps_dec = 0.0;
    p->eta = 0.9;
    p->rtol = 1e-8;
    p->dtau_min = 1e-6;
    p->dtau_max = 1e6;
    p->omega = 1.0;
}

size_t m1_workspace_bytes(const m1_grid* g, const m1_params* p)
{
    if (!valid_grid(g) || !valid_params(p)) return 0;
    Dims d;
    if (!level_dims(*g, *p, d)) return 0;
    m1_plan P;
    P.grid = *g;
    P.params = *p;
    Carver c{nullptr};
    carve(P, c, d);
    return (c.off + kAlign - 1) / kAlign * kAlign;
}

// Plan set-up.  With `wait` the opacity check and all uploads are complete on
// return; without it the plan is returned at once and the caller synchronises
// the stream and then tests *hbad (== ULLONG_MAX: opacities valid) before use.
// Pinned host words a plan needs (hpin); an engine lends each resident request one such slot.
constexpr size_t kHostSlot = (64 + sizeof(m1::Ctrl) + 63) / 64 * 64;

// Release what a plan holds besides its workspace (graph recordings, the
// recording stream, its own pinned host words); the object itself stays.
static void plan_release(m1_plan* P)
{
    drop_cycle_graphs(*P);
    if (P->cap) (void)hipStreamDestroy(P->cap);
    P->cap = nullptr;
    if (P->hpin && P->own_hpin) (void)hipHostFree(P->hpin);
    P->hpin = nullptr;
}

// Fill the plan object *P (freshly constructed) over `workspace`.  On failure
// the caller synchronises the stream and calls plan_release(P).
static m1_status plan_init(m1_plan* P, const m1_grid* g, const m1_params* p, const m1_opacity* op, void* workspace,
                           size_t workspace_bytes, void* stream, bool wait, void* host_slot)
{
    if (!valid_grid(g) || !valid_params(p) || !op || !op->sigma_a || !op->sigma_s) return M1_ERR_ARG;
    Dims dims;
    if (!level_dims(*g, *p, dims)) return M1_ERR_ARG;
    const size_t need = m1_workspace_bytes(g, p);
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0 || workspace_bytes < need)
        return M1_ERR_WORKSPACE;

    P->grid = *g;
    P->params = *p;
    P->st = static_cast<hipStream_t>(stream);
    P->dim = g->dim;
    P->px = g->bc[0].kind == M1_BC_PERIODIC;
    P->py = g->dim == 2 && g->bc[2].kind == M1_BC_PERIODIC;
    P->reach = 1.0 - std::pow(1.0 - p->eta, (double)p->sub_steps);
    P->ph.c = g->c;
    P->ph.c2 = g->c * g->c;
    P->ph.a_r = g->a_r;
    P->ph.c_v = g->c_v;
    for (int s = 0; s < 4; ++s) {
        const bool on = g->dim == 2 || s < 2;
        P->ph.bc[s] = on ? g->bc[s].kind : M1_BC_NEUMANN;
        P->ph.bcE[s] = g->bc[s].E;
        P->ph.bcFx[s] = g->bc[s].Fx;
        P->ph.bcFy[s] = g->dim == 2 ? g->bc[s].Fy : 0.0;
        P->ph.bcEo[s] = g->bc[s].kind == M1_BC_INFLOW ? g->bc[s].Eo : 0.0;
    }
    Carver c{static_cast<char*>(workspace)};
    carve(*P, c, dims);
    P->ph.stalls = P->dstall;
    P->lev[0].sa = const_cast<double*>(op->sigma_a);
    P->lev[0].ss = const_cast<double*>(op->sigma_s);
    fill_level_params(*P);

    if (host_slot) {
        P->hpin = static_cast<double*>(host_slot);
        P->own_hpin = false;
    } else if (hipHostMalloc((void**)&P->hpin, kHostSlot, hipHostMallocDefault) != hipSuccess) {
        P->hpin = nullptr;
        return M1_ERR_DEVICE;
    }
    P->hbad = reinterpret_cast<unsigned long long*>(P->hpin + 4);
    P->hctrl = reinterpret_cast<m1::Ctrl*>(P->hpin + 8);

    // levels small enough for one workgroup form the tail of the cycle
    P->lt = P->L;
    for (int l = 1; l < P->L; ++l)
        if (P->lev[l].n <= tail_cells()) {
            P->lt = l;
            break;
        }
    m1::TailArgs ta{};
    ta.ph = P->ph;
    ta.lt = P->lt;
    ta.L = P->L;
    ta.px = P->px;
    ta.py = P->py;
    ta.pseudo_steps = p->pseudo_steps;
    ta.local = p->pseudo_local;
    ta.reach = P->reach;
    ta.eta = p->eta;
    P->mixed = p->precision == M1_MIXED;
    P->tiled = p->nu_l == 1;  // the tiled legs fuse exactly one Jacobi sweep per pseudo-time step
    P->tiled_max = tiled_max_cells();
    P->graphs = use_graphs();
    // the recursion (other shapes, other transfers) runs every level by grid kernels
    const bool fused_form = p->cycle == M1_CYCLE_V && p->transfer == M1_TRANSFER_FULL;
    if (p->transfer != M1_TRANSFER_FULL) P->tiled = false;  // the up leg prolongs linearly
    const bool tail_ok = P->L <= m1::kMaxLevels && p->nu_l == 1 && fused_form;
    if (!tail_ok) P->lt = P->L;  // the tail fuses exactly one Jacobi sweep per pseudo-time step
    for (int l = 0; l < P->L && l < m1::kMaxLevels; ++l) {
        const LevelBuf& lv = P->lev[l];
        ta.lev[l] = m1::TailLevel{lv.L, lv.v, lv.u, lv.u2, lv.f, lv.rb};
    }
    m1::TailArgs32 ta32{};
    ta32.ph = P->ph;
    ta32.lt = P->lt;
    ta32.L = P->L;
    ta32.px = P->px;
    ta32.py = P->py;
    ta32.pseudo_steps = p->pseudo_steps;
    ta32.local = p->pseudo_local;
    ta32.reach = (float)P->reach;
    ta32.eta = p->eta;
    for (int l = 0; l < P->L && l < m1::kMaxLevels; ++l) {
        const LevelBuf& lv = P->lev[l];
        ta32.lev[l] = m1::TailLevel32{lv.L32, lv.w, lv.d, lv.e, lv.e2, lv.gg, lv.rho, lv.fr};
    }

    // opacity validation and the coarse opacity hierarchy
    const int64_t n0 = P->lev[0].n;
    {
        m1::Ctrl fix{};
        fix.active = 1;
        fix.dtau = P->params.dtau_im0;
        m1::launch_ctrl_init(P->st, P->dfix, fix);
        m1::launch_ctrl_init(P->st, P->dctrl, m1::Ctrl{});  // stopped, state in x0
    }
    m1_status st = hip_status(hipMemsetAsync(P->dbad, 0xff, sizeof(unsigned long long), P->st));
    if (st == M1_OK) st = hip_status(hipMemsetAsync(P->dstall, 0, sizeof(unsigned long long), P->st));
    if (st == M1_OK) {
        m1::launch_check_sigma(P->st, n0, op->sigma_a, op->sigma_s, P->dbad);
        st = hip_status(hipMemcpyAsync(P->hbad, P->dbad, sizeof(unsigned long long), hipMemcpyDeviceToHost, P->st));
    }
    if (wait) {
        if (st == M1_OK) st = hip_status(hipStreamSynchronize(P->st));
        if (st == M1_OK) st = last_launch();
        if (st == M1_OK && *P->hbad != ULLONG_MAX) st = M1_ERR_ARG;
    }
    for (int l = 1; st == M1_OK && l < P->L; ++l) {
        m1::Fields F{};
        F.in[0] = P->lev[l - 1].sa;
        F.in[1] = P->lev[l - 1].ss;
        F.out[0] = P->lev[l].sa;
        F.out[1] = P->lev[l].ss;
        F.n = 2;
        plan_restrict(*P, l - 1, F, &P->dfix->active);  // coarse opacities by the plan's restriction
        st = last_launch();
    }
    for (int l = 0; st == M1_OK && P->mixed && l < P->L; ++l) {
        m1::launch_to_f32(P->st, P->lev[l].n, P->lev[l].sa, P->lev[l].sa32);
        m1::launch_to_f32(P->st, P->lev[l].n, P->lev[l].ss, P->lev[l].ss32);
        st = last_launch();
    }
    P->hta = ta;
    P->hta32 = ta32;
    if (st == M1_OK)
        st = hip_status(hipMemcpyAsync(P->dtail, &P->hta, sizeof(ta), hipMemcpyHostToDevice, P->st));
    if (st == M1_OK && P->mixed)
        st = hip_status(hipMemcpyAsync(P->dtail32, &P->hta32, sizeof(ta32), hipMemcpyHostToDevice, P->st));
    if (st == M1_OK && wait) st = hip_status(hipStreamSynchronize(P->st));
    if (st == M1_OK) st = last_launch();
    return st;
}

static m1_status plan_setup(const m1_grid* g, const m1_params* p, const m1_opacity* op, void* workspace,
                            size_t workspace_bytes, void* stream, bool wait, m1_plan** out,
                            void* host_slot = nullptr)
{
    if (!out) return M1_ERR_ARG;
    *out = nullptr;
    m1_plan* P = new (std::nothrow) m1_plan();
    if (!P) return M1_ERR_DEVICE;
    const m1_status st = plan_init(P, g, p, op, workspace, workspace_bytes, stream, wait, host_slot);
    if (st != M1_OK) {
        if (P->hpin) (void)hipStreamSynchronize(P->st);  // set once the checks passed, before any enqueue
        plan_release(P);
        delete P;
        return st;
    }
    *out = P;
    return M1_OK;
}

m1_status m1_plan_create(const m1_grid* g, const m1_params* p, const m1_opacity* op, void* workspace,
                         size_t workspace_bytes, void* stream, m1_plan** out)
{
    return plan_setup(g, p, op, workspace, workspace_bytes, stream, true, out);
}

void m1_plan_destroy(m1_plan* P)
{
    if (!P) return;
    plan_release(P);
    delete P;
}

int32_t m1_plan_levels(const m1_plan* P) { return P ? P->L : 0; }

m1_status m1_level_dims(const m1_plan* P, int32_t level, int32_t* nx, int32_t* ny)
{
    if (!P || level < 0 || level >= P->L) return M1_ERR_ARG;
    if (nx) *nx = P->lev[level].nx;
    if (ny) *ny = P->lev[level].ny;
    return M1_OK;
}

m1_status m1_sync(m1_plan* P)
{
    if (!P) return M1_ERR_ARG;
    return hip_status(hipStreamSynchronize(P->st));
}

m1_status m1_residual(m1_plan* P, const m1_state* v, const m1_state* vn, double* norm_out, m1_state* r_out)
{
    if (!P || !valid_state(P, v) || !valid_state(P, vn) || !norm_out) return M1_ERR_ARG;
    if (r_out && !valid_state(P, r_out)) return M1_ERR_ARG;
    m1::launch_make_rhs(P->st, P->dim, P->lev[0].n, P->grid.c_v, cs(to_soa(vn)), P->b);
    return fine_norm(*P, to_soa(v), r_out ? to_soa(r_out) : Soa{}, norm_out);
}

m1_status m1_vcycle(m1_plan* P, m1_state* v, const m1_state* vn, double dtau, m1_info* info)
{
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->first_bad_cell = -1;
    }
    if (!P || !valid_state(P, v) || !valid_state(P, vn) || !(dtau > 0.0) || v->E == vn->E) return M1_ERR_ARG;
    m1::launch_make_rhs(P->st, P->dim, P->lev[0].n, P->grid.c_v, cs(to_soa(vn)), P->b);
    Soa user = to_soa(v), cur = user, other = P->tmp;
    double r0 = 0.0;
    if (info) {  // |b - A(v^n)|, the reference of the relative residual
        const m1_status e = fine_norm(*P, to_soa(vn), Soa{}, &r0);
        if (e != M1_OK) return e;
    }
    if (P->mixed) {
        Soa32 pend{};
        if (!mx_cycle(*P, cur, other, fixed_gate(*P, dtau), false, true, pend)) return M1_ERR_DEVICE;
        // apply the correction: the state is now in tmp; write the update back to v
        m1::launch_mx_resid(P->st, P->dim, P->ph, P->lev[0].L, P->params.eta, cs(cur), cs(pend), cs(P->b), user,
                            P->base32, P->r32, nullptr, &P->dfix->active);
    } else {
        cycle_impl(*P, cur, other, fixed_gate(*P, dtau));
        if (!same(cur, user)) m1::launch_copy(P->st, P->dim, P->lev[0].n, cs(cur), user);
    }
    m1_status st = last_launch();
    if (st != M1_OK || !info) return st;
    double r = 0.0;
    st = fine_norm(*P, user, Soa{}, &r);
    if (st != M1_OK) return st;
    info->cycles = 1;
    info->steps_done = 0;
    info->levels = P->L;
    info->r0 = r0;
    info->rel_residual = r0 > 0.0 ? r / r0 : 0.0;
    info->dtau = dtau;
    return M1_OK;
}

m1_status m1_step(m1_plan* P, m1_state* v, int32_t nsteps, m1_info* info)
{
    const m1::TraceRange trace("m1_step");
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->first_bad_cell = -1;
    }
    if (!P || !valid_state(P, v) || nsteps < 0) return M1_ERR_ARG;
    const m1_params& p = P->params;
    const int64_t n0 = P->lev[0].n;
    Soa user = to_soa(v);
    if (info) info->levels = P->L;

    if (hipMemsetAsync(P->dbad, 0xff, sizeof(unsigned long long), P->st) != hipSuccess ||
        hipMemsetAsync(P->dstall, 0, sizeof(unsigned long long), P->st) != hipSuccess)
        return M1_ERR_DEVICE;
    m1::launch_check_state(P->st, P->dim, n0, P->grid.c, cs(user), P->dbad);
    if (hipMemcpyAsync(P->hbad, P->dbad, sizeof(unsigned long long), hipMemcpyDeviceToHost, P->st) != hipSuccess ||
        hipStreamSynchronize(P->st) != hipSuccess)
        return M1_ERR_DEVICE;
    if (last_launch() != M1_OK) return M1_ERR_DEVICE;
    if (*P->hbad != ULLONG_MAX) {
        if (info) {
            info->first_bad_cell = (int64_t)*P->hbad;
            info->status = M1_ERR_NOT_ADMISSIBLE;
        }
        return M1_ERR_NOT_ADMISSIBLE;
    }

    m1_status status = M1_OK;
    int total = 0;
    double r0 = 0.0, rel = 0.0, dtau = p.dtau_im0;
    for (int step = 0; step < nsteps && status == M1_OK; ++step) {
        const m1::TraceRange trace_step("time step");
        m1::launch_make_rhs(P->st, P->dim, n0, P->grid.c_v, cs(user), P->b);
        double bnorm = 0.0;
        m1_status e = fine_norm(*P, user, Soa{}, &bnorm, 0.0);  // |b|
        if (e == M1_OK) e = fine_norm(*P, user, Soa{}, &r0);
        if (e != M1_OK) return e;
        // a residual at the rounding level of evaluating A counts as converged
        const double floor_r = 16.0 * DBL_EPSILON * P->lev[0].L.a * bnorm;
        rel = 0.0;
        if (!p.dtau_carry) dtau = p.dtau_im0;  // else the last step's final dtau
        if (info) info->steps_done = step + 1;
        if (r0 <= floor_r) continue;

        m1::Ctrl init{};
        init.r0 = r0;
        init.rprev = r0;
        init.dtau = dtau;
        init.rel = 1.0;
        init.floor_r = floor_r;
        init.rtol = p.rtol;
        init.eps_inc = p.eps_inc;
        init.eps_dec = p.eps_dec;
        init.dtau_min = p.dtau_min;
        init.dtau_max = p.dtau_max;
        init.active = 1;
        init.cycles = -1;  // the first control call measures r0 (no cycle done yet)
        init.max_cycles = p.max_cycles;
        init.literal = p.dtau_rule == M1_DTAU_LITERAL;
        m1::launch_ctrl_init(P->st, P->dctrl, init);
        const Gate G{dtau, &P->dctrl->dtau, &P->dctrl->active};

        // Enqueue whole cycles ahead of the host's check; kernels of cycles
        // after convergence exit at once.  Each cycle's first sweep measures the
        // residual of the previous result, so one more (partial) cycle than
        // needed is enqueued.  The chunk follows the observed rate.
        Soa cur = user, other = P->tmp;
        Soa32 pend{};
        // FP64: whether a cycle leaves the iterate in the other buffer (an odd
        // number of finest-level launches), read off the first cycle enqueued
        bool cycle_flips = false;
        int enqueued = 0, chunk = 2;
        double prev_rel = 1.0;
        int prev_cycles = 0;
        for (;;) {
            const int todo = std::min(chunk, p.max_cycles + 1 - enqueued);
            for (int c = 0; c < todo; ++c) {
                if (P->graphs) {
                    const m1_status s = graph_cycle(*P, cur, other, pend, G, enqueued + c == 0);
                    if (s != M1_OK) return s;
                } else if (P->mixed) {
                    if (!mx_cycle(*P, cur, other, G, true, enqueued + c == 0, pend)) return M1_ERR_DEVICE;
                } else {
                    cycle_impl(*P, cur, other, G, true);
                }
                if (enqueued + c == 0) cycle_flips = !same(cur, user);
            }
            enqueued += todo;
            if (hipMemcpyAsync(P->hctrl, P->dctrl, sizeof(m1::Ctrl), hipMemcpyDeviceToHost, P->st) != hipSuccess ||
                hipStreamSynchronize(P->st) != hipSuccess)
                return M1_ERR_DEVICE;
            if (last_launch() != M1_OK) return M1_ERR_DEVICE;
            const m1::Ctrl h = *P->hctrl;
            if (!h.active || enqueued >= p.max_cycles + 1) break;
            // cycles still needed at the recent convergence rate (at least 1, at most 16 per chunk)
            const int dc = h.cycles - prev_cycles;
            double need = 4.0;
            if (dc > 0 && h.rel > 0.0 && h.rel < prev_rel) {
                const double rate = std::pow(h.rel / prev_rel, 1.0 / dc);
                need = std::log(p.rtol / h.rel) / std::log(rate);
            }
            chunk = (int)std::min(16.0, std::max(1.0, std::ceil(need)));
            prev_rel = h.rel;
            prev_cycles = h.cycles;
        }
        const m1::Ctrl h = *P->hctrl;
        total += h.cycles;
        rel = h.rel;
        dtau = h.dtau;
        // FP64: the result is the iterate after h.cycles full cycles (the last cycle
        // enqueued only measured it), in `user` unless the cycles moved it an odd
        // number of times; mixed precision: every executed cycle (h.cycles + 1 of
        // them, the last one only measuring) writes the FP64 state into the other buffer
        Soa res = user;
        if (P->mixed) {
            if ((h.cycles + 1) % 2 == 1) res = P->tmp;
        } else if (cycle_flips && (h.cycles % 2 == 1)) {
            res = P->tmp;
        }
        if (!same(res, user)) m1::launch_copy(P->st, P->dim, n0, cs(res), user);
        if (!h.conv) status = M1_ERR_NO_CONVERGENCE;
    }
    auto* hstall = reinterpret_cast<unsigned long long*>(P->hpin + 2);
    if (hipMemcpyAsync(hstall, P->dstall, sizeof(unsigned long long), hipMemcpyDeviceToHost, P->st) != hipSuccess ||
        hipStreamSynchronize(P->st) != hipSuccess)
        return M1_ERR_DEVICE;
    if (info) {
        info->cycles = total;
        info->status = status;
        info->r0 = r0;
        info->rel_residual = rel;
        info->dtau = dtau;
        info->stalled_cells = (int64_t)*hstall;
    }
    return status;
}

m1_status m1_stalls(m1_plan* P, int64_t* count, int32_t reset)
{
    if (!P || !count) return M1_ERR_ARG;
    auto* hstall = reinterpret_cast<unsigned long long*>(P->hpin + 2);
    if (hipMemcpyAsync(hstall, P->dstall, sizeof(unsigned long long), hipMemcpyDeviceToHost, P->st) != hipSuccess ||
        (reset && hipMemsetAsync(P->dstall, 0, sizeof(unsigned long long), P->st) != hipSuccess) ||
        hipStreamSynchronize(P->st) != hipSuccess)
        return M1_ERR_DEVICE;
    *count = (int64_t)*hstall;
    return M1_OK;
}

}  // extern "C"

// ---- allocation-free time steps ----------------------------------------------
// The workspace of m1_step_static: one array on every device the library runs
// on, held until the process ends.  In host code its name stands for a host
// shadow, not for device memory: host code only ever uses the device address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[M1_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
// host words of the static plans (bad-cell index, control copy): pageable, one slot per device
alignas(64) double g_scratch_host[kMaxDevices][kHostSlot / sizeof(double)];

// Device address of `scratch` on device `dev` (current), looked up on the first call per device.
void* scratch_on(int dev)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_dev[dev] = ptr;
    }
    return g_scratch_dev[dev];
}

}  // namespace

extern "C" {

m1_status m1_step_static(const m1_grid* g, const m1_params* p, const m1_opacity* op, m1_state* v, int32_t nsteps,
                         void* stream, m1_info* info)
{
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->first_bad_cell = -1;
    }
    if (!g || !p || !op || !v || nsteps < 0) return M1_ERR_ARG;
    const size_t need = m1_workspace_bytes(g, p);
    if (need == 0) return M1_ERR_ARG;
    if (need > (size_t)M1_STATIC_SCRATCH_BYTES) return M1_ERR_WORKSPACE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return M1_ERR_DEVICE;
    void* ws = scratch_on(dev);
    if (!ws) return M1_ERR_DEVICE;
    m1_plan P;  // host bookkeeping on the stack; workspace: this device's scratch array
    m1_status st = plan_init(&P, g, p, op, ws, (size_t)M1_STATIC_SCRATCH_BYTES, stream, true, g_scratch_host[dev]);
    if (st == M1_OK) {
        P.graphs = false;  // a recording would create a stream and executable graphs
        st = m1_step(&P, v, nsteps, info);
    } else if (P.hpin) {
        (void)hipStreamSynchronize(P.st);
    }
    plan_release(&P);
    return st;
}

m1_status m1_apply_A(m1_plan* P, int32_t level, const m1_state* v, m1_state* out)
{
    if (!P || level < 0 || level >= P->L || !valid_level_state(P, v) || !valid_level_state(P, out)) return M1_ERR_ARG;
    m1::launch_apply(P->st, P->dim, P->ph, P->lev[level].L, cs(to_soa(v)), CSoa{}, 1.0, to_soa(out), nullptr,
                     &P->dfix->active);
    return last_launch();
}

m1_status m1_sweep(m1_plan* P, const m1_state* b, const m1_state* v_in, m1_state* v_out)
{
    if (!P || !valid_state(P, b) || !valid_state(P, v_in) || !valid_state(P, v_out) || v_in->E == v_out->E)
        return M1_ERR_ARG;
    fine_launch(*P, cs(to_soa(b)), cs(to_soa(v_in)), to_soa(v_out), false, nullptr, &P->dfix->active);
    return last_launch();
}

m1_status m1_sweeps(m1_plan* P, const m1_state* b, const m1_state* v_in, m1_state* v_out, int32_t nsweeps)
{
    if (!P || nsweeps < 1 || !valid_state(P, b) || !valid_state(P, v_in) || !valid_state(P, v_out) ||
        v_in->E == v_out->E || b->E == v_out->E)
        return M1_ERR_ARG;
    // launches alternate between v_out and the plan's spare finest-level state,
    // starting with the one that makes the last launch write v_out
    const bool pairs = P->dim == 2 && m1::pair_rows() > 0 && P->params.smoother == M1_SMOOTH_JACOBI;
    const int launches = pairs ? nsweeps / 2 + nsweeps % 2 : nsweeps;
    const Soa out = to_soa(v_out);
    Soa cur = launches % 2 ? out : P->tmp, other = launches % 2 ? P->tmp : out;
    const CSoa rhs = cs(to_soa(b));
    int s = fine_launch(*P, rhs, cs(to_soa(v_in)), cur, nsweeps >= 2, nullptr, &P->dfix->active);
    while (s < nsweeps) {
        s += fine_launch(*P, rhs, cs(cur), other, nsweeps - s >= 2, nullptr, &P->dfix->active);
        std::swap(cur, other);
    }
    if (!same(cur, out)) m1::launch_copy(P->st, P->dim, P->lev[0].n, cs(cur), out);  // the setting changed meanwhile
    return last_launch();
}

m1_status m1_pseudo_step(m1_plan* P, int32_t level, double dtau, const m1_state* f, const m1_state* u_in,
                         m1_state* u_out)
{
    if (!P || level < 0 || level >= P->L || !(dtau > 0.0) || !valid_level_state(P, f) ||
        !valid_level_state(P, u_in) || !valid_level_state(P, u_out) || u_in->E == u_out->E)
        return M1_ERR_ARG;
    if (P->params.nu_l != 1) return M1_ERR_ARG;  // the single-operation entry point fuses exactly one sweep
    const Gate G = fixed_gate(*P, dtau);
    m1::launch_pseudo(P->st, P->dim, P->ph, P->lev[level].L, to_soa(const_cast<m1_state*>(f)), cs(to_soa(u_in)),
                      to_soa(u_out), dtau, G.dtau_dev, P->reach, P->params.pseudo_local, 0, Soa{}, nullptr, G.active);
    return last_launch();
}

m1_status m1_restrict(m1_plan* P, int32_t level, const m1_state* fine, m1_state* coarse)
{
    if (!P || level < 0 || level + 1 >= P->L || !valid_level_state(P, fine) || !valid_level_state(P, coarse))
        return M1_ERR_ARG;
    plan_restrict(*P, level, fields2(to_soa(fine), Soa{}, to_soa(coarse), Soa{}, P->dim), &P->dfix->active);
    return last_launch();
}

m1_status m1_residual_restrict(m1_plan* P, int32_t level, const m1_state* u, const m1_state* rhs, m1_state* vc,
                               m1_state* rc)
{
    if (!P || level < 0 || level + 1 >= P->L || !valid_level_state(P, u) || !valid_level_state(P, rhs) ||
        !valid_level_state(P, vc) || !valid_level_state(P, rc))
        return M1_ERR_ARG;
    const LevelBuf& f = P->lev[level];
    const int* act = &P->dfix->active;
    if (P->dim == 2 && m1::residual_restrict() && !mean_transfer(*P)) {
        m1::launch_residual_restrict(P->st, P->ph, f.L, cs(to_soa(u)), cs(to_soa(rhs)), -1.0, P->px, P->py,
                                     to_soa(vc), to_soa(rc), act);
    } else {  // stored in the level's residual buffer, then restricted
        const Soa r = level == 0 ? P->rfine : P->lev[level].rb;
        m1::launch_apply(P->st, P->dim, P->ph, f.L, cs(to_soa(u)), cs(to_soa(rhs)), -1.0, r, nullptr, act);
        plan_restrict(*P, level, fields2(to_soa(u), r, to_soa(vc), to_soa(rc), P->dim), act);
    }
    return last_launch();
}

m1_status m1_prolong_project(m1_plan* P, int32_t level, const m1_state* u, const m1_state* uc, const m1_state* vc,
                             m1_state* out)
{
    if (!P || level < 0 || level + 1 >= P->L || !valid_level_state(P, u) || !valid_level_state(P, uc) ||
        !valid_level_state(P, vc) || !valid_level_state(P, out))
        return M1_ERR_ARG;
    plan_prolong_project(*P, level, cs(to_soa(u)), cs(to_soa(uc)), cs(to_soa(vc)), to_soa(out), &P->dfix->active);
    return last_launch();
}

m1_status m1_tune_set(const char* key, int64_t value)
{
    if (!key || value < 0) return M1_ERR_ARG;
    const std::string k(key);
    if (k == "tail_cells") tuning().tail_cells = value;
    else if (k == "tiled_max_cells") tuning().tiled_max_cells = value;
    else if (k == "graphs" && value <= 1) tuning().graphs = value;
    else if (k == "sweep_rows" && value <= 16 && m1::set_sweep_rows((int)value)) {}
    else if (k == "pair_rows" && value <= 16 && m1::set_pair_rows((int)value)) {}
    else if (k == "mx_sweep_rows" && value <= 16 && m1::set_mx_sweep_rows((int)value)) {}
    else if (k == "residual_restrict" && value <= 1) m1::set_residual_restrict((int)value);
    else if (k == "batch_grid" && value >= 1 && value <= (int64_t(1) << 24)) m1::set_batch_grid_cap((int)value);
    else if (k == "stage3" && value <= 2) m1::set_stage3((int)value);
    else if (k == "prolong3_lds" && value <= 1) m1::set_prolong3_lds((int)value);
    else return M1_ERR_ARG;
    return M1_OK;
}

int64_t m1_tune_get(const char* key)
{
    if (!key) return -1;
    const std::string k(key);
    if (k == "tail_cells") return tuning().tail_cells.load();
    if (k == "tiled_max_cells") return tuning().tiled_max_cells.load();
    if (k == "graphs") return tuning().graphs.load();
    if (k == "sweep_rows") return m1::sweep_rows();
    if (k == "pair_rows") return m1::pair_rows();
    if (k == "mx_sweep_rows") return m1::mx_sweep_rows();
    if (k == "residual_restrict") return m1::residual_restrict();
    if (k == "batch_grid") return m1::batch_grid_cap();
    if (k == "stage3") return m1::stage3();
    if (k == "prolong3_lds") return m1::prolong3_lds();
    return -1;
}

}  // extern "C"

// ============================================================================
// Batched / served solves: an engine over a caller-provided device arena.
// ============================================================================
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum ReqState { REQ_PENDING = 0, REQ_RUNNING = 1, REQ_DONE = 2 };

}  // namespace

struct m1_req {
    uint64_t ticket = 0;
    m1_grid grid{};
    m1_params params{};
    m1_opacity op{};
    m1_state v{};
    // state, status, progress, levels and times are read by clients (poll, wait,
    // times) from other threads: they are written under the engine's qmu
    int nsteps = 0, steps_done = 0, cycles = 0, state = REQ_PENDING, levels = 0;
    m1_status status = M1_OK;
    double rel = 0.0, r0 = 0.0, dtau = 0.0;
    size_t ws_off = 0, ws_bytes = 0;
    m1_plan* plan = nullptr;
    bool need_init = true, cancel = false;
    int slot = -1;  // the engine's pinned host slot lent to the plan
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
};

struct m1_engine {
    m1_params params{};
    hipStream_t st = nullptr;
    char* arena = nullptr;
    size_t arena_bytes = 0, pool_off = 0, pool_bytes = 0;
    int maxp = 0;
    m1::BProb* dP = nullptr;
    m1::BSlot* dS = nullptr;
    m1::BSlot32* dS32 = nullptr;  // mixed precision: FP32 buffers per (problem, level)
    uint32_t* dWL = nullptr;
    size_t wl_cap = 0;
    uint32_t* dWL2 = nullptr;     // fine tiles of step starts and of result copies
    bool mixed = false;
    int* dPL = nullptr;
    m1::Ctrl* dCtrl = nullptr;
    m1::Ctrl* hCtrl = nullptr;
    char* hslots = nullptr;           // pinned host words lent to the resident requests' plans
    std::vector<int> free_slots;
    std::map<size_t, size_t> free_;  // pool offset -> size
    std::mutex qmu;                   // pending queue and ticket table
    std::mutex rmu;                   // one round at a time
    std::deque<m1_req*> pending;
    // Requests in the device tables, in table order.  A request that leaves becomes a null
    // entry: its control stays inactive in its freed (not yet reused) workspace, so the
    // tables stay valid without a rebuild until the next admission or compaction.
    std::vector<m1_req*> running;
    // resident requests and the pool bytes they hold; atomic, so that m1_engine_memory reads them without
    // waiting for a round (a serving loop runs rounds back to back and would hold it off)
    std::atomic<int> live{0};
    std::atomic<size_t> pool_used{0};
    int64_t live_tiles = 0, dead_tiles = 0;
    std::unordered_map<uint64_t, m1_req*> reqs;
    uint64_t next = 1;
    bool dirty = true;
    struct List {
        int off = 0, n = 0;
    };
    List fine;
    List fine2;    // 64 x rows tiles of the finest levels for the staged sweep (rows == 0: none)
    List fineU, fineN;  // FP64, staged: the fine2 tiles of problems with a coarse correction, and of the others
    List fine3;    // 64 x prow tiles for two sweeps per launch (pairs only)
    int prow = 0;  // tile rows of the pair kernel
    bool pairs = false;  // FP64: consecutive finest sweeps run two per launch
    int rows = 0;
    bool fused = false;     // residuals formed and restricted in one launch per level (lists rr)
    std::vector<List> restr, pdown, up, rr;
    int n_all = 0, n_tail = 0;
    int Lmax = 1;
    std::vector<uint32_t> hwl, hwl2;
    std::vector<int> hpl;
    // one V-cycle of all running problems replayed from a hipGraph recording, made once the
    // tables have stayed the same for a round and dropped when they are rebuilt
    bool graphs = false;
    hipStream_t cap = nullptr;  // private stream, only ever used for recording
    hipGraphExec_t cyc = nullptr;
    int same_rounds = 0;
    // serving loop
    int device = 0;
    std::thread server;
    std::atomic<bool> serving{false}, stop{false};
    std::atomic<int> n_run{0};
    int serve_cycles = 4;
    m1_status serve_status = M1_OK;   // first error of the serving loop (under qmu)
    std::condition_variable work_cv;  // submit / stop -> serving loop (with qmu)
    std::condition_variable done_cv;  // request finished / loop ended -> waiters (with qmu)
};

namespace {

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool pool_alloc(m1_engine& E, size_t bytes, size_t& off)
{
    bytes = align_up(bytes);
    for (auto it = E.free_.begin(); it != E.free_.end(); ++it) {
        if (it->second >= bytes) {
            off = it->first;
            const size_t rest = it->second - bytes;
            E.free_.erase(it);
            if (rest) E.free_[off + bytes] = rest;
            E.pool_used += bytes;
            return true;
        }
    }
    return false;
}

void pool_free(m1_engine& E, size_t off, size_t bytes)
{
    bytes = align_up(bytes);
    E.pool_used -= bytes;
    auto it = E.free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != E.free_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        E.free_.erase(nx);
    }
    if (it != E.free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            E.free_.erase(it);
        }
    }
}

// Requests in a batch: 2-D, at least two levels, an odd number of pseudo-time
// steps, the engine's smoothing structure; tolerances may differ per request.
bool batch_compatible(const m1_engine& E, const m1_grid* g, const m1_params* p)
{
    if (!valid_grid(g) || !valid_params(p) || g->dim != 2) return false;
    const m1_params& e = E.params;
    if (p->nu0 != e.nu0 || p->nu_l != 1 || p->smoother != e.smoother || p->cycle != e.cycle ||
        p->transfer != e.transfer ||
        p->pseudo_steps != e.pseudo_steps ||
        p->sub_steps != e.sub_steps ||
        p->pseudo_local != e.pseudo_local || p->precision != e.precision || p->omega != e.omega || p->eta != e.eta)
        return false;
    Dims d;
    if (!level_dims(*g, *p, d) || d.n < 2 || d.n > m1::kMaxLevels) return false;
    const int* nxs = d.nx;
    const int* nys = d.ny;
    // a work-list entry holds the tile index in kTileBits bits: 256-cell tiles, and 64 x 4 tiles (the
    // staged sweep's most numerous), of the finest level must fit
    const int64_t n = (int64_t)nxs[0] * nys[0];
    const int64_t t2 = (int64_t)((nxs[0] + 63) / 64) * ((nys[0] + 3) / 4);
    if (std::max((n + 255) / 256, t2) > (int64_t(1) << m1::kTileBits)) return false;
    return true;
}

void finish(m1_engine& E, m1_req* R, m1_status st)
{
    if (R->plan) {
        m1_plan_destroy(R->plan);
        R->plan = nullptr;
    }
    if (R->slot >= 0) {
        E.free_slots.push_back(R->slot);
        R->slot = -1;
    }
    pool_free(E, R->ws_off, R->ws_bytes);
    {
        std::lock_guard<std::mutex> g(E.qmu);
        R->status = st;
        R->t_done = now_s();
        R->state = REQ_DONE;
    }
    E.done_cv.notify_all();
}

// FIFO admission: take pending requests while their workspace fits.  Their
// plans are set up without waiting; one synchronisation then checks every new
// request's opacities (a bad one leaves with M1_ERR_ARG before any cycle runs).
void admit(m1_engine& E)
{
    std::vector<m1_req*> fresh;
    for (;;) {
        m1_req* R = nullptr;
        {
            std::lock_guard<std::mutex> g(E.qmu);
            if (E.pending.empty() || E.live + (int)fresh.size() >= E.maxp) break;
            R = E.pending.front();
            if (R->cancel) {
                E.pending.pop_front();
                R->state = REQ_DONE;
                R->status = M1_ERR_BUSY;
                R->t_done = now_s();
                E.done_cv.notify_all();
                continue;
            }
            size_t off;
            if (!pool_alloc(E, R->ws_bytes, off)) break;
            R->ws_off = off;
            E.pending.pop_front();
        }
        R->slot = E.free_slots.back();  // at most maxp requests are resident: a slot is free
        E.free_slots.pop_back();
        m1_status st = plan_setup(&R->grid, &R->params, &R->op, E.arena + E.pool_off + R->ws_off, R->ws_bytes, E.st,
                                  false, &R->plan, E.hslots + (size_t)R->slot * kHostSlot);
        if (st != M1_OK) {
            finish(E, R, st);
            continue;
        }
        fresh.push_back(R);
    }
    if (fresh.empty()) return;
    const bool ok = hipStreamSynchronize(E.st) == hipSuccess && hipGetLastError() == hipSuccess;
    for (m1_req* R : fresh) {
        if (!ok || *R->plan->hbad != ULLONG_MAX) {
            finish(E, R, ok ? M1_ERR_ARG : M1_ERR_DEVICE);
            continue;
        }
        R->need_init = true;
        {
            std::lock_guard<std::mutex> g(E.qmu);
            R->t_admit = now_s();
            R->levels = R->plan->L;
            R->state = REQ_RUNNING;
        }
        E.running.push_back(R);
        ++E.live;
        E.dirty = true;
    }
}

// Device tables of the running set: per-problem data, (problem, level) slots,
// and the work lists of every level operation.
m1_status rebuild(m1_engine& E)
{
    if (E.cyc) {  // every round ends synchronised: the recording is not in flight
        (void)hipGraphExecDestroy(E.cyc);
        E.cyc = nullptr;
    }
    E.same_rounds = 0;
    E.running.erase(std::remove(E.running.begin(), E.running.end(), nullptr), E.running.end());
    E.dead_tiles = 0;
    E.live_tiles = 0;
    for (const m1_req* R : E.running) E.live_tiles += (R->plan->lev[0].n + 255) / 256;
    const int np = (int)E.running.size();
    std::vector<m1::BProb> hp(np);
    std::vector<m1::BSlot> hs((size_t)np * m1::kMaxLevels);
    std::vector<m1::BSlot32> hs32(E.mixed ? (size_t)np * m1::kMaxLevels : 0);
    E.Lmax = 1;
    for (int i = 0; i < np; ++i) {
        const m1_plan& P = *E.running[i]->plan;
        const m1_params& rp = E.running[i]->params;
        m1::BProb& b = hp[i];
        b.ph = P.ph;
        b.px = P.px;
        b.py = P.py;
        b.L = P.L;
        b.lt = P.lt;
        b.local = rp.pseudo_local;
        b.pseudo_steps = rp.pseudo_steps;
        b.npart = P.npart;
        b.eta = rp.eta;
        b.reach = P.reach;
        b.omega = rp.omega;
        b.ctrl = P.dctrl;
        b.partials = P.partials;
        b.tail = P.dtail;
        b.tail32 = P.dtail32;
        m1::Ctrl c{};
        c.dtau = rp.dtau_im0;
        c.rtol = rp.rtol;
        c.eps_inc = rp.eps_inc;
        c.eps_dec = rp.eps_dec;
        c.dtau_min = rp.dtau_min;
        c.dtau_max = rp.dtau_max;
        c.max_cycles = rp.max_cycles;
        c.literal = rp.dtau_rule == M1_DTAU_LITERAL;
        c.carry = rp.dtau_carry;
        b.proto = c;
        for (int l = 0; l < P.L; ++l) {
            m1::BSlot& s = hs[(size_t)i * m1::kMaxLevels + l];
            const LevelBuf& lv = P.lev[l];
            s.L = lv.L;
            s.v = lv.v;
            s.u = lv.u;
            s.u2 = lv.u2;
            s.f = lv.f;
            s.rb = lv.rb;
            if (l == 0) {
                s.b = P.b;
                s.x0 = to_soa(&E.running[i]->v);
                s.x1 = P.tmp;
                s.rf = P.rfine;
            }
            if (E.mixed) {
                m1::BSlot32& t = hs32[(size_t)i * m1::kMaxLevels + l];
                t.L = lv.L32;
                t.w = lv.w;
                t.d = lv.d;
                t.e = lv.e;
                t.e2 = lv.e2;
                t.g = lv.gg;
                t.rho = lv.rho;
                t.fr = lv.fr;
                if (l == 0) {
                    t.base = P.base32;
                    t.r32 = P.r32;
                    t.dA = P.dA;
                    t.dB = P.dB;
                    t.rho0 = P.rho0;
                }
            }
        }
        E.Lmax = std::max(E.Lmax, P.L);
    }
    // work lists
    E.hwl.clear();
    auto tiles = [](int64_t n) { return (uint32_t)((n + 255) / 256); };
    auto make = [&](auto pred, int level) {
        m1_engine::List L;
        L.off = (int)E.hwl.size();
        for (int i = 0; i < np; ++i) {
            const m1_plan& P = *E.running[i]->plan;
            if (level >= P.L || !pred(P)) continue;
            const uint32_t nt = tiles(P.lev[level].n);
            for (uint32_t t = 0; t < nt; ++t) E.hwl.push_back(((uint32_t)i << m1::kTileBits) | t);
        }
        L.n = (int)E.hwl.size() - L.off;
        return L;
    };
    E.fine = make([](const m1_plan&) { return true; }, 0);
    E.rows = E.mixed ? m1::mx_sweep_rows() : m1::sweep_rows();
    E.fine2 = {};
    E.fine2.off = (int)E.hwl.size();
    if (E.rows > 0) {
        for (int i = 0; i < np; ++i) {
            const LevelBuf& lv = E.running[i]->plan->lev[0];
            const uint32_t nt = (uint32_t)((lv.nx + 63) / 64) * (uint32_t)((lv.ny + E.rows - 1) / E.rows);
            for (uint32_t t = 0; t < nt; ++t) E.hwl.push_back(((uint32_t)i << m1::kTileBits) | t);
        }
    }
    E.fine2.n = (int)E.hwl.size() - E.fine2.off;
    E.fineU = E.fineN = {};
    if (!E.mixed && E.rows > 0) {
        for (int u = 1; u >= 0; --u) {
            m1_engine::List& L = u ? E.fineU : E.fineN;
            L.off = (int)E.hwl.size();
            for (int i = 0; i < np; ++i) {
                const m1_plan& P = *E.running[i]->plan;
                if ((std::min(P.lt, P.L - 1) > 0) != (u == 1)) continue;  // the predicate of up[0]
                const LevelBuf& lv = P.lev[0];
                const uint32_t nt = (uint32_t)((lv.nx + 63) / 64) * (uint32_t)((lv.ny + E.rows - 1) / E.rows);
                for (uint32_t t = 0; t < nt; ++t) E.hwl.push_back(((uint32_t)i << m1::kTileBits) | t);
            }
            L.n = (int)E.hwl.size() - L.off;
        }
    }
    // FP64, two sweeps per launch: the pre-sweeps take 1 + ceil((nu0 - 1) / 2) launches and the
    // post-sweeps ceil(nu0 / 2), an even total (2k + 2 for nu0 = 2k + 1) for odd nu0 only, which keeps
    // the cycle ending in the buffer it began from.  (The mixed engine keeps single sweeps: its pair
    // measured no faster on the batched workload.)
    E.prow = m1::pair_rows();
    E.pairs = !E.mixed && E.prow > 0 && E.params.nu0 % 2 == 1;
    E.fine3 = {};
    if (E.pairs && E.prow == E.rows) {
        E.fine3 = E.fine2;
    } else if (E.pairs) {
        E.fine3.off = (int)E.hwl.size();
        for (int i = 0; i < np; ++i) {
            const LevelBuf& lv = E.running[i]->plan->lev[0];
            const uint32_t nt = (uint32_t)((lv.nx + 63) / 64) * (uint32_t)((lv.ny + E.prow - 1) / E.prow);
            for (uint32_t t = 0; t < nt; ++t) E.hwl.push_back(((uint32_t)i << m1::kTileBits) | t);
        }
        E.fine3.n = (int)E.hwl.size() - E.fine3.off;
    }
    E.restr.assign(E.Lmax, {});
    E.pdown.assign(E.Lmax, {});
    E.up.assign(E.Lmax, {});
    E.rr.assign(E.Lmax, {});
    E.fused = m1::residual_restrict() != 0;
    for (int l = 0; l < E.Lmax; ++l) {
        auto top = [](const m1_plan& P) { return std::min(P.lt, P.L - 1); };
        if (l >= 1) {
            E.restr[l] = make([&](const m1_plan& P) { return l <= top(P); }, l);
            E.pdown[l] = make([&](const m1_plan& P) { return l < P.lt; }, l);
            if (E.fused) {  // 32 x 4 tiles of level l for the fused residual-restriction
                E.rr[l].off = (int)E.hwl.size();
                for (int i = 0; i < np; ++i) {
                    const m1_plan& P = *E.running[i]->plan;
                    if (l >= P.L || l > top(P)) continue;
                    const LevelBuf& lv = P.lev[l];
                    const uint32_t nt = (uint32_t)((lv.nx + 31) / 32) * (uint32_t)((lv.ny + 3) / 4);
                    for (uint32_t t = 0; t < nt; ++t) E.hwl.push_back(((uint32_t)i << m1::kTileBits) | t);
                }
                E.rr[l].n = (int)E.hwl.size() - E.rr[l].off;
            }
        }
        E.up[l] = make([&](const m1_plan& P) { return l < top(P); }, l);
    }
    if (E.hwl.size() > E.wl_cap) return M1_ERR_BUDGET;
    // problem lists: all, then those with a tail
    E.hpl.clear();
    for (int i = 0; i < np; ++i) E.hpl.push_back(i);
    E.n_all = np;
    for (int i = 0; i < np; ++i)
        if (E.running[i]->plan->lt < E.running[i]->plan->L) E.hpl.push_back(i);
    E.n_tail = (int)E.hpl.size() - np;
    if (np > 0) {
        if (hipMemcpyAsync(E.dP, hp.data(), sizeof(m1::BProb) * np, hipMemcpyHostToDevice, E.st) != hipSuccess ||
            hipMemcpyAsync(E.dS, hs.data(), sizeof(m1::BSlot) * hs.size(), hipMemcpyHostToDevice, E.st) !=
                hipSuccess ||
            (E.mixed && hipMemcpyAsync(E.dS32, hs32.data(), sizeof(m1::BSlot32) * hs32.size(),
                                       hipMemcpyHostToDevice, E.st) != hipSuccess) ||
            hipMemcpyAsync(E.dWL, E.hwl.data(), sizeof(uint32_t) * E.hwl.size(), hipMemcpyHostToDevice, E.st) !=
                hipSuccess ||
            hipMemcpyAsync(E.dPL, E.hpl.data(), sizeof(int) * E.hpl.size(), hipMemcpyHostToDevice, E.st) != hipSuccess)
            return M1_ERR_DEVICE;
        if (hipStreamSynchronize(E.st) != hipSuccess) return M1_ERR_DEVICE;
    }
    E.dirty = false;
    return M1_OK;
}

// Work list (uploaded to dWL2) of the finest-level tiles of the given running problems.
m1_status fine_tiles(m1_engine& E, const std::vector<int>& idx)
{
    E.hwl2.clear();
    for (int i : idx) {
        const uint32_t nt = (uint32_t)((E.running[i]->plan->lev[0].n + 255) / 256);
        for (uint32_t t = 0; t < nt; ++t) E.hwl2.push_back(((uint32_t)i << m1::kTileBits) | t);
    }
    if (E.hwl2.size() > E.wl_cap) return M1_ERR_BUDGET;
    if (!E.hwl2.empty() && hipMemcpyAsync(E.dWL2, E.hwl2.data(), sizeof(uint32_t) * E.hwl2.size(),
                                          hipMemcpyHostToDevice, E.st) != hipSuccess)
        return M1_ERR_DEVICE;
    return M1_OK;
}

// One V-cycle of every running problem: each level operation is one launch.
// Selectors: with an odd number of pseudo-time steps every level's down-leg,
// up-leg and tail results end in u; the up leg starts from u2.
void b_vcycle(m1_engine& E)
{
    const int nu0 = E.params.nu0, m = E.params.pseudo_steps;
    const uint32_t* wl = E.dWL;
    int in_x1 = 0;
    for (int s = 0; s < nu0;) {
        if (s > 0 && E.pairs && nu0 - s >= 2) {
            m1::launch_b_relax2_lds(E.st, E.dP, E.dS, wl + E.fine3.off, E.fine3.n, in_x1, E.prow);
            s += 2;
        } else {
            if (s > 0 && E.rows > 0)
                m1::launch_b_relax_lds(E.st, E.dP, E.dS, wl + E.fine2.off, E.fine2.n, in_x1, E.rows);
            else
                m1::launch_b_relax(E.st, E.dP, E.dS, wl + E.fine.off, E.fine.n, in_x1, s == 0);
            if (s == 0) m1::launch_b_norm_control(E.st, E.dP, E.dPL, E.n_all, 0);
            ++s;
        }
        in_x1 ^= 1;
    }
    if (!E.fused) m1::launch_b_apply(E.st, E.dP, E.dS, wl + E.up[0].off, E.up[0].n, 0, in_x1);
    for (int l = 1; l < E.Lmax; ++l) {
        if (E.fused)
            m1::launch_b_residual_restrict(E.st, E.dP, E.dS, wl + E.rr[l].off, E.rr[l].n, l, l == 1 ? in_x1 : 1);
        else
            m1::launch_b_restrict(E.st, E.dP, E.dS, wl + E.restr[l].off, E.restr[l].n, l, l == 1 ? in_x1 : 1);
        int in = 0;
        for (int k = 0; k < m; ++k) {
            const int out = (in == 1) ? 2 : 1;
            m1::launch_b_pseudo(E.st, E.dP, E.dS, wl + E.pdown[l].off, E.pdown[l].n, l, in, out, k == 0);
            in = out;
        }
        if (!E.fused) m1::launch_b_apply(E.st, E.dP, E.dS, wl + E.up[l].off, E.up[l].n, l, 1);
    }
    m1::launch_b_tail(E.st, E.dP, E.dPL + E.n_all, E.n_tail);
    // staged: the finest level's coarse correction runs with its first post-sweep (then pairs, which keeps
    // the launch count of the post leg, ceil(nu0 / 2) for odd nu0)
    const bool up_fused = E.rows > 0 && nu0 >= 1;
    for (int l = E.Lmax - 2; l >= 0; --l) {
        if (l == 0) {
            if (!up_fused) m1::launch_b_prolong(E.st, E.dP, E.dS, wl + E.up[0].off, E.up[0].n, 0, in_x1, 0);
        } else {
            m1::launch_b_prolong(E.st, E.dP, E.dS, wl + E.up[l].off, E.up[l].n, l, 1, 2);
            int in = 2;
            for (int k = 0; k < m; ++k) {
                const int out = (in == 1) ? 2 : 1;
                m1::launch_b_pseudo(E.st, E.dP, E.dS, wl + E.up[l].off, E.up[l].n, l, in, out, 0);
                in = out;
            }
        }
    }
    int s0 = 0;
    if (up_fused) {
        m1::launch_b_relax_lds(E.st, E.dP, E.dS, wl + E.fineU.off, E.fineU.n, in_x1, E.rows, true);
        m1::launch_b_relax_lds(E.st, E.dP, E.dS, wl + E.fineN.off, E.fineN.n, in_x1, E.rows);
        in_x1 ^= 1;
        s0 = 1;
    }
    for (int s = s0; s < nu0;) {
        if (E.pairs && nu0 - s >= 2) {
            m1::launch_b_relax2_lds(E.st, E.dP, E.dS, wl + E.fine3.off, E.fine3.n, in_x1, E.prow);
            s += 2;
        } else {
            if (E.rows > 0) m1::launch_b_relax_lds(E.st, E.dP, E.dS, wl + E.fine2.off, E.fine2.n, in_x1, E.rows);
            else m1::launch_b_relax(E.st, E.dP, E.dS, wl + E.fine.off, E.fine.n, in_x1, 0);
            ++s;
        }
        in_x1 ^= 1;
    }
}

// One mixed-precision V-cycle of every running problem (the same sequence as
// the single-problem mixed cycle).  Fine corrections alternate dA (0) / dB (1):
// the pre-sweeps start from zero writing dA; coarse levels go d -> e / e2 with
// the down leg ending in e and the up leg in e2 (odd pseudo_steps).
void bm_vcycle(m1_engine& E)
{
    const int nu0 = E.params.nu0, m = E.params.pseudo_steps;
    const uint32_t* wl = E.dWL;
    // the correction the previous cycle left: its pre-sweeps started from buffer 1
    // (the first one, from zero, writes buffer 0) and every sweep of either leg
    // moved it, 2 nu0 moves in all, so it ends in buffer 1 whatever nu0
    const int pend = 1;
    // the first pre-sweep (from a zero correction, into buffer 0) runs inside the residual launch
    const bool zero_fused = nu0 >= 1;
    m1::launch_bm_resid(E.st, E.dP, E.dS, E.dS32, wl + E.fine.off, E.fine.n, pend, zero_fused);
    m1::launch_b_norm_control(E.st, E.dP, E.dPL, E.n_all, 1);
    int d = zero_fused ? 0 : 1;
    for (int s = zero_fused ? 1 : 0; s < nu0; ++s) {
        const int out = d ^ 1;
        if (s > 0 && E.rows > 0)
            m1::launch_bm_sweep_lds(E.st, E.dP, E.dS32, wl + E.fine2.off, E.fine2.n, d, out, E.rows);
        else
            m1::launch_bm_sweep(E.st, E.dP, E.dS32, wl + E.fine.off, E.fine.n, d, out, s == 0);
        d = out;
    }
    const int d0 = d;
    if (!E.fused) m1::launch_bm_apply(E.st, E.dP, E.dS32, wl + E.up[0].off, E.up[0].n, 0, d0);
    for (int l = 1; l < E.Lmax; ++l) {
        if (E.fused) m1::launch_bm_residual_restrict(E.st, E.dP, E.dS32, wl + E.rr[l].off, E.rr[l].n, l, d0);
        else m1::launch_bm_restrict(E.st, E.dP, E.dS32, wl + E.restr[l].off, E.restr[l].n, l, d0);
        int in = 0;
        for (int k = 0; k < m; ++k) {
            const int out = (in == 1) ? 2 : 1;
            m1::launch_bm_pseudo(E.st, E.dP, E.dS32, wl + E.pdown[l].off, E.pdown[l].n, l, in, out, k == 0);
            in = out;
        }
        if (!E.fused) m1::launch_bm_apply(E.st, E.dP, E.dS32, wl + E.up[l].off, E.up[l].n, l, 1);
    }
    m1::launch_bm_tail(E.st, E.dP, E.dPL + E.n_all, E.n_tail);
    for (int l = E.Lmax - 2; l >= 1; --l) {
        m1::launch_bm_prolong(E.st, E.dP, E.dS32, wl + E.up[l].off, E.up[l].n, l);
        int in = 1;
        for (int k = 0; k < m; ++k) {
            const int out = (in == 1) ? 2 : 1;
            m1::launch_bm_pseudo(E.st, E.dP, E.dS32, wl + E.up[l].off, E.up[l].n, l, in, out, 0);
            in = out;
        }
    }
    m1::launch_bm_prolong_fine(E.st, E.dP, E.dS, E.dS32, wl + E.up[0].off, E.up[0].n, d0);
    d = d0;
    for (int s = 0; s < nu0; ++s) {
        const int out = d ^ 1;
        if (E.rows > 0) m1::launch_bm_sweep_lds(E.st, E.dP, E.dS32, wl + E.fine2.off, E.fine2.n, d, out, E.rows);
        else m1::launch_bm_sweep(E.st, E.dP, E.dS32, wl + E.fine.off, E.fine.n, d, out, 0);
        d = out;
    }
}

}  // namespace

extern "C" {

size_t m1_engine_request_bytes(const m1_grid* g, const m1_params* p) { return align_up(m1_workspace_bytes(g, p)); }

m1_status m1_engine_create(const m1_params* p, void* arena, size_t arena_bytes, int32_t max_requests, void* stream,
                           m1_engine** out)
{
    if (!out) return M1_ERR_ARG;
    *out = nullptr;
    if (!valid_params(p) || max_requests < 1 || max_requests > (1 << (32 - m1::kTileBits)) ||
        p->pseudo_steps % 2 == 0 || p->nu_l != 1 || p->smoother != M1_SMOOTH_JACOBI || p->cycle != M1_CYCLE_V ||
        p->transfer != M1_TRANSFER_FULL)
        return M1_ERR_ARG;
    if (!arena || (reinterpret_cast<uintptr_t>(arena) % kAlign) != 0) return M1_ERR_WORKSPACE;
    m1_engine* E = new (std::nothrow) m1_engine();
    if (!E) return M1_ERR_DEVICE;
    E->params = *p;
    E->mixed = p->precision == M1_MIXED;
    E->graphs = use_graphs();
    E->st = static_cast<hipStream_t>(stream);
    E->arena = static_cast<char*>(arena);
    E->arena_bytes = arena_bytes;
    E->maxp = max_requests;
    if (hipGetDevice(&E->device) != hipSuccess) {
        delete E;
        return M1_ERR_DEVICE;
    }
    // tables at the start of the arena; work lists sized for the whole pool
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return E->arena + o;
    };
    E->dP = reinterpret_cast<m1::BProb*>(take(sizeof(m1::BProb) * max_requests));
    E->dS = reinterpret_cast<m1::BSlot*>(take(sizeof(m1::BSlot) * (size_t)max_requests * m1::kMaxLevels));
    E->dPL = reinterpret_cast<int*>(take(sizeof(int) * 3 * (size_t)max_requests));
    E->dCtrl = reinterpret_cast<m1::Ctrl*>(take(sizeof(m1::Ctrl) * max_requests));
    if (E->mixed)
        E->dS32 = reinterpret_cast<m1::BSlot32*>(take(sizeof(m1::BSlot32) * (size_t)max_requests * m1::kMaxLevels));
    // a 256-cell tile of a request's finest level needs more than 30 KB of its workspace and
    // appears in at most a few work-list entries: one entry per 2 KB of arena is ample
    E->wl_cap = std::max<size_t>(arena_bytes / 2048, 1 << 16);
    E->dWL = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * E->wl_cap));
    E->dWL2 = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * E->wl_cap));
    if (off >= arena_bytes) {
        delete E;
        return M1_ERR_WORKSPACE;
    }
    E->pool_off = off;
    E->pool_bytes = arena_bytes - off;
    E->free_[0] = E->pool_bytes / kAlign * kAlign;
    if (hipHostMalloc((void**)&E->hCtrl, sizeof(m1::Ctrl) * max_requests, hipHostMallocDefault) != hipSuccess) {
        delete E;
        return M1_ERR_DEVICE;
    }
    if (hipHostMalloc((void**)&E->hslots, kHostSlot * (size_t)max_requests, hipHostMallocDefault) != hipSuccess) {
        (void)hipHostFree(E->hCtrl);
        delete E;
        return M1_ERR_DEVICE;
    }
    for (int i = max_requests - 1; i >= 0; --i) E->free_slots.push_back(i);
    *out = E;
    return M1_OK;
}

void m1_engine_destroy(m1_engine* E)
{
    if (!E) return;
    (void)m1_serve_stop(E);
    (void)hipStreamSynchronize(E->st);
    for (auto& kv : E->reqs) {
        if (kv.second->plan) m1_plan_destroy(kv.second->plan);
        delete kv.second;
    }
    if (E->hCtrl) (void)hipHostFree(E->hCtrl);
    if (E->hslots) (void)hipHostFree(E->hslots);
    if (E->cyc) (void)hipGraphExecDestroy(E->cyc);
    if (E->cap) (void)hipStreamDestroy(E->cap);
    delete E;
}

m1_status m1_batch_submit(m1_engine* E, const m1_grid* g, const m1_params* p, const m1_opacity* op, m1_state* v,
                          int32_t nsteps, uint64_t* ticket)
{
    if (!E || !ticket || !op || !op->sigma_a || !op->sigma_s || !v || !v->E || !v->Fx || !v->Fy || !v->T ||
        nsteps < 1)
        return M1_ERR_ARG;
    const m1_params& pp = p ? *p : E->params;
    if (!batch_compatible(*E, g, &pp)) return M1_ERR_ARG;
    const size_t need = m1_engine_request_bytes(g, &pp);
    if (need == 0) return M1_ERR_ARG;
    if (need > E->pool_bytes) return M1_ERR_BUDGET;
    m1_req* R = new (std::nothrow) m1_req();
    if (!R) return M1_ERR_DEVICE;
    R->grid = *g;
    R->params = pp;
    R->op = *op;
    R->v = *v;
    R->nsteps = nsteps;
    R->ws_bytes = need;
    R->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(E->qmu);
        R->ticket = E->next++;
        E->reqs[R->ticket] = R;
        E->pending.push_back(R);
        *ticket = R->ticket;
    }
    E->work_cv.notify_one();
    return M1_OK;
}

m1_status m1_batch_run(m1_engine* E, int32_t cycles, int32_t* n_running, int32_t* n_pending)
{
    if (!E || cycles < 1) return M1_ERR_ARG;
    std::lock_guard<std::mutex> lk(E->rmu);
    const m1::TraceRange trace("engine round");
    admit(*E);
    m1_status st = M1_OK;
    if (E->live > 0) {
        if (E->dirty) st = rebuild(*E);
        if (st != M1_OK) return st;
        // step starts: b, |b| and a fresh control per starting problem (state back in x0 first)
        std::vector<int> init;
        for (int i = 0; i < (int)E->running.size(); ++i)
            if (E->running[i] && E->running[i]->need_init) {
                init.push_back(i);
                E->running[i]->need_init = false;
            }
        if (!init.empty()) {
            st = fine_tiles(*E, init);
            if (st != M1_OK) return st;
            int* dinit = E->dPL + 2 * E->maxp;
            if (hipMemcpyAsync(dinit, init.data(), sizeof(int) * init.size(), hipMemcpyHostToDevice, E->st) !=
                hipSuccess)
                return M1_ERR_DEVICE;
            m1::launch_b_init_tiles(E->st, E->dP, E->dS, E->dWL2, (int)E->hwl2.size());
            m1::launch_b_init_ctrl(E->st, E->dP, E->dS, dinit, (int)init.size());
        }
        const bool replay = E->graphs && E->same_rounds > 0;
        if (replay && !E->cyc) {
            st = record(&E->st, E->cap, [&] {
                if (E->mixed) bm_vcycle(*E);
                else b_vcycle(*E);
            }, &E->cyc);
            if (st != M1_OK) return st;
        }
        for (int c = 0; c < cycles; ++c) {
            if (replay) {
                if (hipGraphLaunch(E->cyc, E->st) != hipSuccess) return M1_ERR_DEVICE;
            } else if (E->mixed) {
                bm_vcycle(*E);
            } else {
                b_vcycle(*E);
            }
        }
        ++E->same_rounds;
        const int np = (int)E->running.size();
        m1::launch_b_gather_ctrl(E->st, E->dP, np, E->dCtrl);
        if (hipMemcpyAsync(E->hCtrl, E->dCtrl, sizeof(m1::Ctrl) * np, hipMemcpyDeviceToHost, E->st) != hipSuccess ||
            hipStreamSynchronize(E->st) != hipSuccess || hipGetLastError() != hipSuccess)
            return M1_ERR_DEVICE;
        // retire: cancelled, failed and completed requests leave with their state in x0
        std::vector<std::pair<int, m1_status>> done;
        std::vector<int> back;  // table indices whose state must be copied back from x1
        for (int i = 0; i < np; ++i) {
            m1_req* R = E->running[i];
            if (!R) continue;
            const m1::Ctrl& h = E->hCtrl[i];
            m1_status out = M1_OK;
            bool leaves = false;
            {
                std::lock_guard<std::mutex> g(E->qmu);
                const bool cancel = R->cancel;
                if (!h.active || cancel) {
                    R->cycles += std::max(h.cycles, 0);
                    R->rel = h.rel;
                    R->r0 = h.r0;
                    R->dtau = h.dtau;
                }
                if (cancel) {
                    out = M1_ERR_BUSY;
                    leaves = true;
                } else if (!h.active && !h.conv) {
                    out = M1_ERR_NO_CONVERGENCE;
                    leaves = true;
                } else if (!h.active) {
                    R->steps_done += 1;
                    leaves = R->steps_done >= R->nsteps;
                    if (!leaves) R->need_init = true;
                }
            }
            if (leaves) {
                done.push_back({i, out});
                if (h.flip) back.push_back(i);
            }
        }
        if (!back.empty()) {
            st = fine_tiles(*E, back);
            if (st != M1_OK) return st;
            m1::launch_b_flip_copy(E->st, E->dP, E->dS, E->dWL2, (int)E->hwl2.size());
        }
        bool stop = false;  // a cancelled request may leave mid-step: stop its kernels before its entry goes dead
        for (auto& d : done)
            if (E->hCtrl[d.first].active) {
                m1::launch_ctrl_init(E->st, E->running[d.first]->plan->dctrl, m1::Ctrl{});
                stop = true;
            }
        if ((!back.empty() || stop) &&
            (hipStreamSynchronize(E->st) != hipSuccess || hipGetLastError() != hipSuccess))
            return M1_ERR_DEVICE;
        for (auto& d : done) {
            m1_req* R = E->running[d.first];
            const int64_t t = (R->plan->lev[0].n + 255) / 256;
            finish(*E, R, d.second);
            E->running[d.first] = nullptr;
            --E->live;
            E->live_tiles -= t;
            E->dead_tiles += t;
        }
        // compact once dead entries would cost more block iterations than live ones
        if (E->dead_tiles > E->live_tiles) E->dirty = true;
    }
    E->n_run.store(E->live);
    std::lock_guard<std::mutex> g(E->qmu);
    if (n_running) *n_running = (int32_t)E->live;
    if (n_pending) *n_pending = (int32_t)E->pending.size();
    return M1_OK;
}

m1_status m1_engine_memory(m1_engine* E, size_t* pool_in_use, size_t* pool_bytes, int32_t* resident,
                           int32_t* pending)
{
    if (!E || !pool_in_use || !pool_bytes) return M1_ERR_ARG;
    *pool_bytes = E->pool_bytes;
    *pool_in_use = E->pool_used.load();
    if (resident) *resident = E->live.load();
    if (pending) {
        std::lock_guard<std::mutex> q(E->qmu);
        *pending = (int32_t)E->pending.size();
    }
    return M1_OK;
}

m1_status m1_batch_poll(m1_engine* E, uint64_t ticket, m1_info* info)
{
    if (!E) return M1_ERR_ARG;
    std::lock_guard<std::mutex> lk(E->qmu);
    auto it = E->reqs.find(ticket);
    if (it == E->reqs.end()) return M1_ERR_ARG;
    const m1_req* R = it->second;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->cycles = R->cycles;
        info->status = R->status;
        info->levels = R->levels;
        info->steps_done = R->steps_done;
        info->r0 = R->r0;
        info->rel_residual = R->rel;
        info->dtau = R->dtau;
        info->first_bad_cell = -1;
    }
    return R->state == REQ_DONE ? M1_OK : M1_ERR_BUSY;
}

m1_status m1_batch_wait(m1_engine* E, uint64_t ticket, m1_info* info)
{
    if (!E) return M1_ERR_ARG;
    m1_info tmp;
    if (!info) info = &tmp;
    for (;;) {
        m1_status s = m1_batch_poll(E, ticket, info);
        if (s != M1_ERR_BUSY) return s == M1_OK ? (m1_status)info->status : s;
        if (E->serving.load()) {
            // the serving loop drives the rounds: sleep until a request finishes
            std::unique_lock<std::mutex> lk(E->qmu);
            auto it = E->reqs.find(ticket);
            if (it == E->reqs.end()) return M1_ERR_ARG;
            const m1_req* R = it->second;
            E->done_cv.wait(lk, [&] { return R->state == REQ_DONE || !E->serving.load(); });
            if (R->state != REQ_DONE && E->serve_status != M1_OK) return E->serve_status;
            continue;
        }
        s = m1_batch_run(E, 4, nullptr, nullptr);
        if (s != M1_OK) return s;
    }
}

m1_status m1_batch_cancel(m1_engine* E, uint64_t ticket)
{
    if (!E) return M1_ERR_ARG;
    std::lock_guard<std::mutex> lk(E->qmu);
    auto it = E->reqs.find(ticket);
    if (it == E->reqs.end()) return M1_ERR_ARG;
    it->second->cancel = true;
    return M1_OK;
}

m1_status m1_batch_times(m1_engine* E, uint64_t ticket, double* t_submit, double* t_admit, double* t_done)
{
    if (!E) return M1_ERR_ARG;
    std::lock_guard<std::mutex> lk(E->qmu);
    auto it = E->reqs.find(ticket);
    if (it == E->reqs.end()) return M1_ERR_ARG;
    if (t_submit) *t_submit = it->second->t_submit;
    if (t_admit) *t_admit = it->second->t_admit;
    if (t_done) *t_done = it->second->t_done;
    return M1_OK;
}

m1_status m1_batch_release(m1_engine* E, uint64_t ticket)
{
    if (!E) return M1_ERR_ARG;
    std::lock_guard<std::mutex> lk(E->qmu);
    auto it = E->reqs.find(ticket);
    if (it == E->reqs.end() || it->second->state != REQ_DONE) return M1_ERR_ARG;
    delete it->second;
    E->reqs.erase(it);
    return M1_OK;
}

static void serve_loop(m1_engine* E)
{
    if (hipSetDevice(E->device) != hipSuccess) {
        std::lock_guard<std::mutex> lk(E->qmu);
        E->serve_status = M1_ERR_DEVICE;
    } else {
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(E->qmu);
                E->work_cv.wait(lk, [&] { return E->stop.load() || !E->pending.empty() || E->n_run.load() > 0; });
                if (E->stop.load()) break;
            }
            const m1_status s = m1_batch_run(E, E->serve_cycles, nullptr, nullptr);
            if (s != M1_OK) {
                std::lock_guard<std::mutex> lk(E->qmu);
                E->serve_status = s;
                break;
            }
        }
    }
    {
        std::lock_guard<std::mutex> lk(E->qmu);
        E->serving.store(false);
    }
    E->done_cv.notify_all();
}

m1_status m1_serve_start(m1_engine* E, int32_t cycles)
{
    if (!E || cycles < 1) return M1_ERR_ARG;
    if (E->serving.load() || E->server.joinable()) return M1_ERR_BUSY;
    {
        std::lock_guard<std::mutex> lk(E->qmu);
        E->serve_status = M1_OK;
    }
    E->serve_cycles = cycles;
    E->stop.store(false);
    E->serving.store(true);
    try {
        E->server = std::thread(serve_loop, E);
    } catch (...) {
        E->serving.store(false);
        return M1_ERR_DEVICE;
    }
    return M1_OK;
}

m1_status m1_serve_stop(m1_engine* E)
{
    if (!E) return M1_ERR_ARG;
    if (!E->server.joinable()) return M1_OK;
    {
        std::lock_guard<std::mutex> lk(E->qmu);
        E->stop.store(true);
    }
    E->work_cv.notify_all();
    E->server.join();
    std::lock_guard<std::mutex> lk(E->qmu);
    return E->serve_status;
}

}  // extern "C"
