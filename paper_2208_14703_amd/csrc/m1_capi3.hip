// m1_capi3.hip -- plans, V-cycles and time steps of the three-dimensional
// method behind the C ABI (include/m1.h, "three dimensions").
//
// The hierarchy halves every side per level (Sect. 4.2 with d = 3: R = 2^-3 P^T,
// trilinear P), coarse opacities by full weighting, the FAS coarse problems
// smoothed by pseudo-time steps (Algorithm 3), the V-cycle (and the W and F
// shapes of Sect. 6.3 as a recursion) and the time-step driver of Appendix A
// with the cycle control on the device (the same control
// kernel as the 2-D plans).  Every level runs the grid kernels of
// m1_kernels3.hip (one cell per thread, or staged in LDS where that pays);
// FP64 only.
#include <algorithm>
#include <cfloat>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>

#include "m1.h"
#include "m1_3d.hpp"
#include "m1_trace.hpp"

namespace {

constexpr int kMaxLevels3 = 16;
constexpr size_t kAlign3 = 256;
constexpr int64_t kMaxCells3 = int64_t(1) << 29;  // 32-bit byte offsets of a field

struct Level3 {
    int nx, ny, nz;
    int64_t n;
    m1::Lvl3 L;
    m1::Soa3 v, u, u2, f, rb;
};

}  // namespace

struct m1_plan3 {
    m1_grid3 grid;
    m1_params params;
    hipStream_t st = nullptr;
    int L = 0;
    Level3 lev[kMaxLevels3];
    m1::Phys3 ph{};
    int px = 0, py = 0, pz = 0;
    double reach = 0.0;
    m1::Soa3 b{}, tmp{}, rfine{};
    double* partials = nullptr;
    int npart = 0;
    double* dscal = nullptr;
    unsigned long long* dbad = nullptr;
    unsigned long long* dstall = nullptr;  // pseudo-time stalls of the last m1_step3
    m1::Ctrl* dctrl = nullptr;
    m1::Ctrl* dfix = nullptr;
    double* hpin = nullptr;  // pinned host slot: scalars, the bad-cell index and a control copy
};

namespace {

struct Bump {
    char* base;
    size_t off = 0;
    double* take(int64_t n)
    {
        off = (off + kAlign3 - 1) / kAlign3 * kAlign3;
        double* p = base ? reinterpret_cast<double*>(base + off) : nullptr;
        off += (size_t)n * sizeof(double);
        return p;
    }
    m1::Soa3 soa(int64_t n) { return m1::Soa3{take(n), take(n), take(n), take(n), take(n)}; }
};

bool valid_grid3(const m1_grid3* g)
{
    if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1) return false;
    if ((int64_t)g->nx * g->ny * g->nz > kMaxCells3) return false;
    auto pos = [](double x) { return std::isfinite(x) && x > 0.0; };
    if (!pos(g->hx) || !pos(g->hy) || !pos(g->hz) || !pos(g->dt) || !pos(g->c) || !pos(g->c_v)) return false;
    if (!(std::isfinite(g->a_r) && g->a_r >= 0.0)) return false;
    for (int s = 0; s < 6; ++s) {
        const m1_bc3& b = g->bc[s];
        if (b.kind < M1_BC_PERIODIC || b.kind > M1_BC_DIRICHLET) return false;
        if ((b.kind == M1_BC_PERIODIC) != (g->bc[s ^ 1].kind == M1_BC_PERIODIC)) return false;
        if (b.kind == M1_BC_DIRICHLET) {
            if (!(std::isfinite(b.E) && b.E > 0.0 && std::isfinite(b.Fx) && std::isfinite(b.Fy) && std::isfinite(b.Fz)))
                return false;
            if (std::sqrt(b.Fx * b.Fx + b.Fy * b.Fy + b.Fz * b.Fz) > g->c * b.E * (1.0 + 1e-12)) return false;
        }
    }
    return true;
}

bool valid_params3(const m1_params* p)
{
    if (!p) return false;
    if (p->levels < 0 || p->nu0 < 1 || p->nu_l != 1 || p->pseudo_steps < 1 || p->sub_steps < 1 || p->max_cycles < 1)
        return false;
    if (p->dtau_rule != M1_DTAU_SIGNED && p->dtau_rule != M1_DTAU_LITERAL) return false;
    if (p->precision != M1_FP64 || p->smoother != M1_SMOOTH_JACOBI ||
        (p->cycle != M1_CYCLE_V && p->cycle != M1_CYCLE_W && p->cycle != M1_CYCLE_F) ||
        p->transfer != M1_TRANSFER_FULL)
        return false;
    if (!(p->eta > 0.0 && p->eta < 1.0) || !(p->omega > 0.0 && p->omega <= 1.0) || !(p->rtol > 0.0)) return false;
    if (!(p->dtau_im0 > 0.0) || !(p->dtau_min > 0.0) || !(p->dtau_max >= p->dtau_min)) return false;
    if (p->dtau_carry != 0 && p->dtau_carry != 1) return false;
    return std::isfinite(p->eps_inc) && std::isfinite(p->eps_dec);
}

// Level sizes: halve every side while all stay even and at least 8 (coarsest side >= 4), up to `levels`.
int level_count3(const m1_grid3& g, const m1_params& p, int nx[], int ny[], int nz[])
{
    int L = 1;
    nx[0] = g.nx;
    ny[0] = g.ny;
    nz[0] = g.nz;
    while (L < kMaxLevels3 && (p.levels == 0 || L < p.levels)) {
        const int a = nx[L - 1], b = ny[L - 1], c = nz[L - 1];
        if (a % 2 || b % 2 || c % 2 || a / 2 < 4 || b / 2 < 4 || c / 2 < 4) break;
        nx[L] = a / 2;
        ny[L] = b / 2;
        nz[L] = c / 2;
        ++L;
    }
    return L;
}

// Carve the plan's buffers from `base` (nullptr: only count the bytes).
size_t carve3(m1_plan3* P, char* base, int L, const int nx[], const int ny[], const int nz[])
{
    Bump c{base};
    const int64_t n0 = (int64_t)nx[0] * ny[0] * nz[0];
    m1::Soa3 b = c.soa(n0), tmp = c.soa(n0), rfine = c.soa(n0);
    if (P) {
        P->b = b;
        P->tmp = tmp;
        P->rfine = rfine;
    }
    for (int l = 1; l < L; ++l) {
        const int64_t n = (int64_t)nx[l] * ny[l] * nz[l];
        m1::Soa3 v = c.soa(n), u = c.soa(n), u2 = c.soa(n), f = c.soa(n), rb = c.soa(n);
        double* sa = c.take(n);
        double* ss = c.take(n);
        if (P) {
            Level3& lv = P->lev[l];
            lv.v = v;
            lv.u = u;
            lv.u2 = u2;
            lv.f = f;
            lv.rb = rb;
            lv.L.sa = sa;
            lv.L.ss = ss;
        }
    }
    // one norm partial per block of the one-cell kernels (256 cells) or of a staged sweep, whichever is more
    const int npart = (int)std::max<int64_t>((n0 + 255) / 256, m1::staged3_blocks(nx[0], ny[0], nz[0]));
    double* partials = c.take(npart);
    double* dscal = c.take(8);
    double* dbad = c.take(1);
    double* dstall = c.take(1);
    const int64_t nctrl = (int64_t)((sizeof(m1::Ctrl) + 7) / 8);
    double* dctrl = c.take(nctrl);
    double* dfix = c.take(nctrl);
    if (P) {
        P->partials = partials;
        P->npart = npart;
        P->dscal = dscal;
        P->dbad = reinterpret_cast<unsigned long long*>(dbad);
        P->dstall = reinterpret_cast<unsigned long long*>(dstall);
        P->dctrl = reinterpret_cast<m1::Ctrl*>(dctrl);
        P->dfix = reinterpret_cast<m1::Ctrl*>(dfix);
    }
    return (c.off + kAlign3 - 1) / kAlign3 * kAlign3;
}

m1_status status_of(hipError_t e) { return e == hipSuccess ? M1_OK : M1_ERR_DEVICE; }

bool valid_state3(const m1_state3* s) { return s && s->E && s->Fx && s->Fy && s->Fz && s->T; }
m1::Soa3 soa3(const m1_state3* s) { return m1::Soa3{s->E, s->Fx, s->Fy, s->Fz, s->T}; }
bool same3(const m1::Soa3& a, const m1::Soa3& b) { return a.E == b.E; }

struct Gate3 {
    double dtau;
    const double* dtau_dev;
    const int* active;
};

Gate3 fixed_gate3(m1_plan3& P, double dtau)
{
    m1::Ctrl fix{};
    fix.active = 1;
    fix.dtau = dtau;
    m1::launch_ctrl_init(P.st, P.dfix, fix);
    return Gate3{dtau, &P.dfix->dtau, &P.dfix->active};
}

// The three stencil operations, staged where the level is wide enough (bitwise the one-cell forms; by
// default the sweeps and A on the large levels, the pseudo-time steps never).  The sweep reduces its input's
// residual norm into `partials` when given and returns the number of partials.
unsigned relax3(m1_plan3& P, const m1::CSoa3& b, const m1::CSoa3& in, const m1::Soa3& out, const int* active,
                double* partials = nullptr)
{
    const m1::Lvl3& L = P.lev[0].L;
    if (m1::stage3_fits(L, true))
        return m1::launch3_relax_staged(P.st, P.ph, L, b, P.params.omega, in, out, active, partials);
    return m1::launch3_relax(P.st, P.ph, L, b, P.params.omega, in, out, active, partials);
}

void apply3(m1_plan3& P, int l, const m1::CSoa3& v, const m1::CSoa3& x, double sgn, const m1::Soa3& out,
            const int* active)
{
    const m1::Lvl3& L = P.lev[l].L;
    if (m1::stage3_fits(L, true)) m1::launch3_apply_staged(P.st, P.ph, L, v, x, sgn, out, active);
    else m1::launch3_apply(P.st, P.ph, L, v, x, sgn, out, nullptr, active);
}

void pseudo3(m1_plan3& P, int l, const m1::CSoa3& f, const m1::CSoa3& in, const m1::Soa3& out, double dtau,
             const double* dtau_dev, const int* active)
{
    const m1::Lvl3& L = P.lev[l].L;
    if (m1::stage3_fits(L, false))
        m1::launch3_pseudo_staged(P.st, P.ph, L, f, in, out, dtau, dtau_dev, P.reach, P.params.pseudo_local, active);
    else
        m1::launch3_pseudo(P.st, P.ph, L, f, in, out, dtau, dtau_dev, P.reach, P.params.pseudo_local, active);
}

// nu finest-level sweeps.  With `control` the first sweep also reduces the residual norm of its input (the
// previous cycle's result) and the cycle control updates dtau / the stop flag before the rest of the cycle.
void sweeps3(m1_plan3& P, m1::Soa3& cur, m1::Soa3& other, int nu, const Gate3& G, bool control = false)
{
    for (int s = 0; s < nu; ++s) {
        const bool norm = control && s == 0;
        const unsigned np = relax3(P, m1::cs3(P.b), m1::cs3(cur), other, G.active, norm ? P.partials : nullptr);
        if (norm) m1::launch_norm_control(P.st, P.partials, (int)np, P.dctrl);
        std::swap(cur, other);
    }
}

// m pseudo-time steps of level l from `start` (alternating between u and u2); returns where the result is.
m1::Soa3 smooth3(m1_plan3& P, int l, const Gate3& G, m1::Soa3 start)
{
    Level3& c = P.lev[l];
    m1::Soa3 in = start;
    for (int m = 0; m < P.params.pseudo_steps; ++m) {
        const m1::Soa3 out = same3(in, c.u) ? c.u2 : c.u;
        pseudo3(P, l, m1::cs3(c.f), m1::cs3(in), out, G.dtau, G.dtau_dev, G.active);
        in = out;
    }
    return in;
}

m1::Fields fields3(const m1::Soa3& a, const m1::Soa3& b, const m1::Soa3& ca, const m1::Soa3& cb)
{
    m1::Fields F{};
    const double* in[5] = {a.E, a.Fx, a.Fy, a.Fz, a.T};
    double* out[5] = {ca.E, ca.Fx, ca.Fy, ca.Fz, ca.T};
    for (int q = 0; q < 5; ++q) {
        F.in[q] = in[q];
        F.out[q] = out[q];
    }
    F.n = 5;
    if (b.E) {
        const double* in2[5] = {b.E, b.Fx, b.Fy, b.Fz, b.T};
        double* out2[5] = {cb.E, cb.Fx, cb.Fy, cb.Fz, cb.T};
        for (int q = 0; q < 5; ++q) {
            F.in[5 + q] = in2[q];
            F.out[5 + q] = out2[q];
        }
        F.n = 10;
    }
    return F;
}

// One V-cycle (Appendix A) on the finest iterate cur (partner buffer other): nu0 sweeps; per coarse level
// v_l = R(u_{l-1}), f_l = A_l(v_l) + R(rbar_{l-1}), m pseudo-time steps from v_l and rbar_l = f_l - A_l(u_l);
// upward u_l <- projected(u_l + P(u_{l+1} - v_{l+1})) and the same smoothing again.  `control`: the first
// sweep feeds the previous result's residual norm to the cycle control (sweeps3).
void vcycle3(m1_plan3& P, m1::Soa3& cur, m1::Soa3& other, const Gate3& G, bool control)
{
    const m1_params& p = P.params;
    sweeps3(P, cur, other, p.nu0, G, control);
    if (P.L == 1) return;
    m1::Soa3 ul[kMaxLevels3];
    ul[0] = cur;
    apply3(P, 0, m1::cs3(cur), m1::cs3(P.b), -1.0, P.rfine, G.active);
    m1::Soa3 rprev = P.rfine;
    for (int l = 1; l < P.L; ++l) {
        Level3& c = P.lev[l];
        const Level3& f = P.lev[l - 1];
        m1::launch3_restrict(P.st, f.nx, f.ny, f.nz, P.px, P.py, P.pz, fields3(ul[l - 1], rprev, c.v, c.rb), G.active);
        apply3(P, l, m1::cs3(c.v), m1::cs3(c.rb), 1.0, c.f, G.active);
        ul[l] = smooth3(P, l, G, c.v);
        if (l < P.L - 1) {
            apply3(P, l, m1::cs3(ul[l]), m1::cs3(c.f), -1.0, c.rb, G.active);
            rprev = c.rb;
        }
    }
    for (int l = P.L - 2; l >= 0; --l) {
        const Level3& c = P.lev[l + 1];
        const Level3& f = P.lev[l];
        m1::launch3_prolong_project(P.st, P.ph, f.nx, f.ny, f.nz, P.px, P.py, P.pz, p.eta, m1::cs3(ul[l]),
                                    m1::cs3(ul[l + 1]), m1::cs3(c.v), ul[l], G.active);
        if (l == 0) {
            cur = ul[0];
            sweeps3(P, cur, other, p.nu0, G);
        } else {
            ul[l] = smooth3(P, l, G, ul[l]);
        }
    }
}

// W- and F-cycles (Sect. 6.3) as a recursion over the coarse FAS problems.  A visit of coarse level l takes
// m pseudo-time steps from u_l; above the coarsest level it then forms rbar_l = f_l - A_l(u_l), restricts
// (u_l, rbar_l) to v_{l+1} and f_{l+1} = A(v_{l+1}) + R(rbar_l), visits level l+1 once (V), twice (W) or by an
// F-visit then a V-visit (F), corrects u_l by the projected prolongation of u_{l+1} - v_{l+1} and smooths
// again.  The finest level takes nu0 sweeps each side.  One visit per level gives vcycle3's launches.
struct Rec3 {
    m1_plan3& P;
    const Gate3& G;
    m1::Soa3 ul[kMaxLevels3];
};

void descend3(Rec3& R, int l)
{
    m1_plan3& P = R.P;
    Level3& f = P.lev[l];
    Level3& c = P.lev[l + 1];
    const m1::Soa3 rbar = l == 0 ? P.rfine : f.rb;
    if (l == 0) apply3(P, 0, m1::cs3(R.ul[0]), m1::cs3(P.b), -1.0, rbar, R.G.active);
    else apply3(P, l, m1::cs3(R.ul[l]), m1::cs3(f.f), -1.0, rbar, R.G.active);
    m1::launch3_restrict(P.st, f.nx, f.ny, f.nz, P.px, P.py, P.pz, fields3(R.ul[l], rbar, c.v, c.rb), R.G.active);
    apply3(P, l + 1, m1::cs3(c.v), m1::cs3(c.rb), 1.0, c.f, R.G.active);
    R.ul[l + 1] = c.v;  // the first pseudo-time step reads v_{l+1} and writes an iterate buffer
}

void visit3(Rec3& R, int l, int kind);

void below3(Rec3& R, int l, int kind)
{
    if (kind == M1_CYCLE_F) {
        visit3(R, l + 1, M1_CYCLE_F);
        visit3(R, l + 1, M1_CYCLE_V);
    } else {
        for (int t = 0; t < (kind == M1_CYCLE_W ? 2 : 1); ++t) visit3(R, l + 1, kind);
    }
    m1_plan3& P = R.P;
    const Level3& f = P.lev[l];
    const Level3& c = P.lev[l + 1];
    m1::launch3_prolong_project(P.st, P.ph, f.nx, f.ny, f.nz, P.px, P.py, P.pz, P.params.eta, m1::cs3(R.ul[l]),
                                m1::cs3(R.ul[l + 1]), m1::cs3(c.v), R.ul[l], R.G.active);
}

void visit3(Rec3& R, int l, int kind)
{
    R.ul[l] = smooth3(R.P, l, R.G, R.ul[l]);
    if (l == R.P.L - 1) return;
    descend3(R, l);
    below3(R, l, kind);
    R.ul[l] = smooth3(R.P, l, R.G, R.ul[l]);
}

// One cycle of the plan's shape on the finest iterate cur (partner buffer other); `control` as in sweeps3.
void cycle3(m1_plan3& P, m1::Soa3& cur, m1::Soa3& other, const Gate3& G, bool control = false)
{
    if (P.params.cycle == M1_CYCLE_V) {
        vcycle3(P, cur, other, G, control);
        return;
    }
    sweeps3(P, cur, other, P.params.nu0, G, control);
    if (P.L == 1) return;
    Rec3 R{P, G, {}};
    R.ul[0] = cur;
    descend3(R, 0);
    below3(R, 0, P.params.cycle);
    sweeps3(P, cur, other, P.params.nu0, G);
}

// |x + sgn A_0(v)| (x = b, sgn = -1: the residual; sgn = 0: |b|) to the host, r_out written when set.
m1_status fine_norm3(m1_plan3& P, const m1::Soa3& v, const m1::Soa3& r_out, double* out, double sgn = -1.0)
{
    m1::launch3_apply(P.st, P.ph, P.lev[0].L, m1::cs3(v), m1::cs3(P.b), sgn, r_out, P.partials, &P.dfix->active);
    m1::launch_norm_finalize(P.st, P.partials, P.npart, P.dscal);
    if (hipMemcpyAsync(P.hpin, P.dscal, sizeof(double), hipMemcpyDeviceToHost, P.st) != hipSuccess ||
        hipStreamSynchronize(P.st) != hipSuccess)
        return M1_ERR_DEVICE;
    *out = P.hpin[0];
    return status_of(hipGetLastError());
}

bool level_ok(const m1_plan3* P, int level) { return P && level >= 0 && level < P->L; }

}  // namespace

extern "C" {

size_t m1_workspace3_bytes(const m1_grid3* g, const m1_params* p)
{
    if (!valid_grid3(g) || !valid_params3(p)) return 0;
    int nx[kMaxLevels3], ny[kMaxLevels3], nz[kMaxLevels3];
    const int L = level_count3(*g, *p, nx, ny, nz);
    if (p->levels > L) return 0;  // more levels than the sides allow
    return carve3(nullptr, nullptr, L, nx, ny, nz);
}

m1_status m1_plan3_create(const m1_grid3* g, const m1_params* p, const m1_opacity* op, void* workspace,
                          size_t workspace_bytes, void* stream, m1_plan3** out)
{
    if (!out) return M1_ERR_ARG;
    *out = nullptr;
    if (!valid_grid3(g) || !valid_params3(p) || !op || !op->sigma_a || !op->sigma_s) return M1_ERR_ARG;
    int nx[kMaxLevels3], ny[kMaxLevels3], nz[kMaxLevels3];
    const int L = level_count3(*g, *p, nx, ny, nz);
    if (p->levels > L) return M1_ERR_ARG;
    const size_t need = carve3(nullptr, nullptr, L, nx, ny, nz);
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign3 != 0 || workspace_bytes < need)
        return M1_ERR_WORKSPACE;
    m1_plan3* P = new (std::nothrow) m1_plan3();
    if (!P) return M1_ERR_DEVICE;
    P->grid = *g;
    P->params = *p;
    P->st = static_cast<hipStream_t>(stream);
    P->L = L;
    carve3(P, static_cast<char*>(workspace), L, nx, ny, nz);
    P->ph.c = g->c;
    P->ph.c2 = g->c * g->c;
    P->ph.a_r = g->a_r;
    P->ph.c_v = g->c_v;
    for (int s = 0; s < 6; ++s) {
        P->ph.bc[s] = g->bc[s].kind;
        P->ph.bcE[s] = g->bc[s].E;
        P->ph.bcFx[s] = g->bc[s].Fx;
        P->ph.bcFy[s] = g->bc[s].Fy;
        P->ph.bcFz[s] = g->bc[s].Fz;
    }
    P->ph.stalls = P->dstall;
    P->px = g->bc[0].kind == M1_BC_PERIODIC;
    P->py = g->bc[2].kind == M1_BC_PERIODIC;
    P->pz = g->bc[4].kind == M1_BC_PERIODIC;
    P->reach = 1.0 - std::pow(1.0 - p->eta, p->sub_steps);  // the closed form of the sub-steps' pseudo time
    for (int l = 0; l < L; ++l) {
        Level3& lv = P->lev[l];
        lv.nx = nx[l];
        lv.ny = ny[l];
        lv.nz = nz[l];
        lv.n = (int64_t)nx[l] * ny[l] * nz[l];
        const double s = std::ldexp(1.0, l);
        const double hx = g->hx * s, hy = g->hy * s, hz = g->hz * s;
        lv.L.nx = nx[l];
        lv.L.ny = ny[l];
        lv.L.nz = nz[l];
        lv.L.kx = g->dt / (2.0 * hx);
        lv.L.ky = g->dt / (2.0 * hy);
        lv.L.kz = g->dt / (2.0 * hz);
        lv.L.a = 1.0 + g->c * g->dt / hx + g->c * g->dt / hy + g->c * g->dt / hz;
        lv.L.cdt = g->c * g->dt;
        if (l == 0) {
            lv.L.sa = op->sigma_a;
            lv.L.ss = op->sigma_s;
        }
    }
    m1_status st = M1_OK;
    if (hipHostMalloc((void**)&P->hpin, 256, hipHostMallocDefault) != hipSuccess) {
        P->hpin = nullptr;
        st = M1_ERR_DEVICE;
    }
    if (st == M1_OK) {  // opacities >= 0 and finite
        st = status_of(hipMemsetAsync(P->dbad, 0xff, sizeof(unsigned long long), P->st));
        if (st == M1_OK) m1::launch_check_sigma(P->st, P->lev[0].n, op->sigma_a, op->sigma_s, P->dbad);
        if (st == M1_OK)
            st = status_of(hipMemcpyAsync(P->hpin, P->dbad, sizeof(unsigned long long), hipMemcpyDeviceToHost, P->st));
        if (st == M1_OK) st = status_of(hipStreamSynchronize(P->st));
        if (st == M1_OK) st = status_of(hipGetLastError());
        if (st == M1_OK && *reinterpret_cast<unsigned long long*>(P->hpin) != ULLONG_MAX) st = M1_ERR_ARG;
    }
    if (st == M1_OK) {
        (void)fixed_gate3(*P, p->dtau_im0);
        for (int l = 1; l < L; ++l) {  // coarse opacities by full weighting
            const Level3& f = P->lev[l - 1];
            m1::Fields F{};
            F.in[0] = f.L.sa;
            F.in[1] = f.L.ss;
            F.out[0] = const_cast<double*>(P->lev[l].L.sa);
            F.out[1] = const_cast<double*>(P->lev[l].L.ss);
            F.n = 2;
            m1::launch3_restrict(P->st, f.nx, f.ny, f.nz, P->px, P->py, P->pz, F, &P->dfix->active);
        }
        st = status_of(hipStreamSynchronize(P->st));
        if (st == M1_OK) st = status_of(hipGetLastError());
    }
    if (st != M1_OK) {
        if (P->hpin) (void)hipHostFree(P->hpin);
        delete P;
        return st;
    }
    *out = P;
    return M1_OK;
}

void m1_plan3_destroy(m1_plan3* P)
{
    if (!P) return;
    (void)hipStreamSynchronize(P->st);
    if (P->hpin) (void)hipHostFree(P->hpin);
    delete P;
}

int32_t m1_plan3_levels(const m1_plan3* P) { return P ? P->L : 0; }

m1_status m1_level3_dims(const m1_plan3* P, int32_t level, int32_t* nx, int32_t* ny, int32_t* nz)
{
    if (!level_ok(P, level) || !nx || !ny || !nz) return M1_ERR_ARG;
    *nx = P->lev[level].nx;
    *ny = P->lev[level].ny;
    *nz = P->lev[level].nz;
    return M1_OK;
}

m1_status m1_apply3(m1_plan3* P, int32_t level, const m1_state3* v, m1_state3* out)
{
    if (!level_ok(P, level) || !valid_state3(v) || !valid_state3(out)) return M1_ERR_ARG;
    apply3(*P, level, m1::cs3(soa3(v)), m1::CSoa3{}, 1.0, soa3(out), &P->dfix->active);
    return status_of(hipGetLastError());
}

m1_status m1_sweep3(m1_plan3* P, const m1_state3* b, const m1_state3* v_in, m1_state3* v_out)
{
    if (!P || !valid_state3(b) || !valid_state3(v_in) || !valid_state3(v_out) || v_in->E == v_out->E) return M1_ERR_ARG;
    relax3(*P, m1::cs3(soa3(b)), m1::cs3(soa3(v_in)), soa3(v_out), &P->dfix->active);
    return status_of(hipGetLastError());
}

m1_status m1_pseudo_step3(m1_plan3* P, int32_t level, double dtau, const m1_state3* f, const m1_state3* u_in,
                          m1_state3* u_out)
{
    if (!level_ok(P, level) || !(dtau > 0.0) || !valid_state3(f) || !valid_state3(u_in) || !valid_state3(u_out) ||
        u_in->E == u_out->E)
        return M1_ERR_ARG;
    const Gate3 G = fixed_gate3(*P, dtau);
    pseudo3(*P, level, m1::cs3(soa3(f)), m1::cs3(soa3(u_in)), soa3(u_out), dtau, G.dtau_dev, G.active);
    return status_of(hipGetLastError());
}

m1_status m1_restrict3(m1_plan3* P, int32_t level, const m1_state3* fine, m1_state3* coarse)
{
    if (!P || level < 0 || level + 1 >= P->L || !valid_state3(fine) || !valid_state3(coarse)) return M1_ERR_ARG;
    const Level3& f = P->lev[level];
    m1::launch3_restrict(P->st, f.nx, f.ny, f.nz, P->px, P->py, P->pz, fields3(soa3(fine), m1::Soa3{}, soa3(coarse),
                                                                                m1::Soa3{}),
                         &P->dfix->active);
    return status_of(hipGetLastError());
}

m1_status m1_prolong_project3(m1_plan3* P, int32_t level, const m1_state3* u, const m1_state3* uc,
                              const m1_state3* vc, m1_state3* out)
{
    if (!P || level < 0 || level + 1 >= P->L || !valid_state3(u) || !valid_state3(uc) || !valid_state3(vc) ||
        !valid_state3(out))
        return M1_ERR_ARG;
    const Level3& f = P->lev[level];
    m1::launch3_prolong_project(P->st, P->ph, f.nx, f.ny, f.nz, P->px, P->py, P->pz, P->params.eta,
                                m1::cs3(soa3(u)), m1::cs3(soa3(uc)), m1::cs3(soa3(vc)), soa3(out), &P->dfix->active);
    return status_of(hipGetLastError());
}

m1_status m1_residual3(m1_plan3* P, const m1_state3* v, const m1_state3* vn, double* norm_out, m1_state3* r_out)
{
    if (!P || !valid_state3(v) || !valid_state3(vn) || !norm_out) return M1_ERR_ARG;
    if (r_out && !valid_state3(r_out)) return M1_ERR_ARG;
    m1::launch3_make_rhs(P->st, P->lev[0].n, P->grid.c_v, m1::cs3(soa3(vn)), P->b);
    (void)fixed_gate3(*P, P->params.dtau_im0);
    return fine_norm3(*P, soa3(v), r_out ? soa3(r_out) : m1::Soa3{}, norm_out);
}

m1_status m1_vcycle3(m1_plan3* P, m1_state3* v, const m1_state3* vn, double dtau)
{
    if (!P || !valid_state3(v) || !valid_state3(vn) || !(dtau > 0.0) || v->E == vn->E) return M1_ERR_ARG;
    m1::launch3_make_rhs(P->st, P->lev[0].n, P->grid.c_v, m1::cs3(soa3(vn)), P->b);
    m1::Soa3 user = soa3(v), cur = user, other = P->tmp;
    cycle3(*P, cur, other, fixed_gate3(*P, dtau));
    if (!same3(cur, user)) m1::launch3_copy(P->st, P->lev[0].n, m1::cs3(cur), user);
    return status_of(hipGetLastError());
}

m1_status m1_step3(m1_plan3* P, m1_state3* v, int32_t nsteps, m1_info* info)
{
    const m1::TraceRange trace("m1_step3");
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->first_bad_cell = -1;
    }
    if (!P || !valid_state3(v) || nsteps < 0) return M1_ERR_ARG;
    const m1_params& p = P->params;
    const int64_t n0 = P->lev[0].n;
    const m1::Soa3 user = soa3(v);
    if (info) info->levels = P->L;
    auto* hbad = reinterpret_cast<unsigned long long*>(P->hpin + 4);
    if (hipMemsetAsync(P->dbad, 0xff, sizeof(unsigned long long), P->st) != hipSuccess ||
        hipMemsetAsync(P->dstall, 0, sizeof(unsigned long long), P->st) != hipSuccess)
        return M1_ERR_DEVICE;
    m1::launch3_check_state(P->st, n0, P->grid.c, m1::cs3(user), P->dbad);
    if (hipMemcpyAsync(hbad, P->dbad, sizeof(unsigned long long), hipMemcpyDeviceToHost, P->st) != hipSuccess ||
        hipStreamSynchronize(P->st) != hipSuccess || hipGetLastError() != hipSuccess)
        return M1_ERR_DEVICE;
    if (*hbad != ULLONG_MAX) {
        if (info) {
            info->first_bad_cell = (int64_t)*hbad;
            info->status = M1_ERR_NOT_ADMISSIBLE;
        }
        return M1_ERR_NOT_ADMISSIBLE;
    }
    m1_status status = M1_OK;
    int total = 0;
    double r0 = 0.0, rel = 0.0, dtau = p.dtau_im0;
    auto* hctrl = reinterpret_cast<m1::Ctrl*>(P->hpin + 8);
    for (int step = 0; step < nsteps && status == M1_OK; ++step) {
        m1::launch3_make_rhs(P->st, n0, P->grid.c_v, m1::cs3(user), P->b);
        (void)fixed_gate3(*P, p.dtau_im0);
        double bnorm = 0.0;
        m1_status e = fine_norm3(*P, user, m1::Soa3{}, &bnorm, 0.0);
        if (e == M1_OK) e = fine_norm3(*P, user, m1::Soa3{}, &r0);
        if (e != M1_OK) return e;
        const double floor_r = 16.0 * DBL_EPSILON * P->lev[0].L.a * bnorm;  // A's rounding level
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
        const Gate3 G{dtau, &P->dctrl->dtau, &P->dctrl->active};
        // whole cycles enqueued ahead of the host's check; each cycle's first sweep measures the residual of the
        // previous result and the control updates dtau / the stop flag on the device, so one more (partial)
        // cycle than needed is enqueued; kernels of cycles after the stop store nothing
        m1::Soa3 cur = user, other = P->tmp;
        bool flips = false;
        int enqueued = 0, chunk = 2, prev_cycles = 0;
        double prev_rel = 1.0;
        for (;;) {
            const int todo = std::min(chunk, p.max_cycles + 1 - enqueued);
            for (int c = 0; c < todo; ++c) {
                cycle3(*P, cur, other, G, true);
                if (enqueued + c == 0) flips = !same3(cur, user);
            }
            enqueued += todo;
            if (hipMemcpyAsync(hctrl, P->dctrl, sizeof(m1::Ctrl), hipMemcpyDeviceToHost, P->st) != hipSuccess ||
                hipStreamSynchronize(P->st) != hipSuccess || hipGetLastError() != hipSuccess)
                return M1_ERR_DEVICE;
            if (!hctrl->active || enqueued >= p.max_cycles + 1) break;
            // cycles still needed at the recent convergence rate (at least 1, at most 16 per chunk)
            const int dc = hctrl->cycles - prev_cycles;
            double need = 4.0;
            if (dc > 0 && hctrl->rel > 0.0 && hctrl->rel < prev_rel) {
                const double rate = std::pow(hctrl->rel / prev_rel, 1.0 / dc);
                need = std::log(p.rtol / hctrl->rel) / std::log(rate);
            }
            chunk = (int)std::min(16.0, std::max(1.0, std::ceil(need)));
            prev_rel = hctrl->rel;
            prev_cycles = hctrl->cycles;
        }
        const m1::Ctrl h = *hctrl;
        total += h.cycles;
        rel = h.rel;
        dtau = h.dtau;
        // the result is the iterate after h.cycles full cycles (the last cycle enqueued only measured it), in
        // `user` unless a cycle moves it to the other buffer and h.cycles is odd
        const m1::Soa3 res = (flips && h.cycles % 2 == 1) ? P->tmp : user;
        if (!same3(res, user)) m1::launch3_copy(P->st, n0, m1::cs3(res), user);
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

}  // extern "C"
