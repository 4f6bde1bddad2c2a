// m1_internal.hpp -- kernel launchers and device-side control structures
// shared by the plan/driver code and the kernels.
#pragma once

#include "m1_device.hpp"
#include "m1_mixed.hpp"

namespace m1 {

// log2(nx) when nx is a power of two, else -1 (the row shift of Lvl::sh).
inline int row_shift(int nx)
{
    if (nx < 1 || (nx & (nx - 1)) != 0) return -1;
    int sh = 0;
    while ((1 << sh) < nx) ++sh;
    return sh;
}


constexpr int kMaxLevels = 24;

// Up to 10 fields restricted by one launch (in[q] -> out[q]).
struct Fields {
    const double* in[10];
    double* out[10];
    int n;
};

// Up to 12 FP32 fields restricted by one launch.
struct Fields32 {
    const float* in[12];
    float* out[12];
    int n;
};

// Device-side cycle control of one time step (pseudo-time step adaptation and
// the stopping test of the relative residual), updated after every V-cycle.
struct Ctrl {
    double r0, rprev, dtau, rel, floor_r, rtol, eps_inc, eps_dec, dtau_min, dtau_max;
    int active, cycles, conv, max_cycles, literal;
    int flip;  // batched mixed precision: the FP64 state of the step is in x1 (toggled by every executed cycle)
    int carry;  // batched: a step start keeps the dtau the previous step of the request ended with
};

// One level of the single-workgroup bottom of the V-cycle.
struct TailLevel {
    Lvl L;
    Soa v, u, u2, f, rb;
};

struct TailArgs {
    Phys ph;
    int lt, L, px, py, pseudo_steps, local;
    double reach, eta;
    TailLevel lev[kMaxLevels];
};

// one colour of a red-black Gauss-Seidel sweep (cells with (i + j) % 2 == colour updated, the others copied);
// with partials, the residual norm of u over all cells
void launch_relax_colour(hipStream_t st, int dim, const Phys& ph, const Lvl& L, CSoa rhs, double omega, int colour,
                         CSoa u, Soa out, double* partials, const int* active);
void launch_relax(hipStream_t st, int dim, const Phys& ph, const Lvl& L, CSoa rhs, const double* gcell, double beta,
                  double gamma, double omega, CSoa u, Soa out, double* partials, const int* active);
void launch_pseudo(hipStream_t st, int dim, const Phys& ph, const Lvl& L, Soa f, CSoa u, Soa out, double dtau,
                   const double* dtau_dev, double reach, int local, int first, Soa rs, double* gs, const int* active);
unsigned apply_blocks(const Lvl& L);
void launch_apply(hipStream_t st, int dim, const Phys& ph, const Lvl& L, CSoa v, CSoa X, double sgn, Soa out,
                  double* partials, const int* active);
void launch_norm_finalize(hipStream_t st, const double* partials, int n, double* out);
void launch_norm_control(hipStream_t st, const double* partials, int n, Ctrl* ctrl);
void launch_ctrl_init(hipStream_t st, Ctrl* ctrl, const Ctrl& init);
void launch_restrict(hipStream_t st, int dim, int nxf, int nyf, int px, int py, const Fields& F, const int* active);
void launch_prolong_project(hipStream_t st, int dim, const Phys& ph, int nx, int ny, int px, int py, double eta,
                            CSoa u, CSoa uc, CSoa vc, Soa out, const int* active);
void launch_tail(hipStream_t st, int dim, const TailArgs* args_dev, double dtau, const double* dtau_dev,
                 const int* active);
// LDS-tiled smoothing leg of one coarse level (all m pseudo-time steps in one launch).  Legs: the first
// smoothing of a descent (forms the FAS right-hand side from R(rbar)), the correction from the level below
// with the post-smoothing, and plain smoothing (a later visit in a W- or F-cycle).
constexpr int kLegDown = 0, kLegUp = 1, kLegPlain = 2;
bool smooth_tb_fits(int dim, const Lvl& L, int m);
void launch_smooth_tb(hipStream_t st, const Phys& ph, const Lvl& L, int m, int leg, CSoa fr, Soa f, CSoa u, Soa out,
                      const double* dtau_dev, double reach, int local, CSoa uc, CSoa vc, int px, int py, double eta,
                      const int* active);
void launch_make_rhs(hipStream_t st, int dim, int64_t n, double cv, CSoa v, Soa b);
void launch_copy(hipStream_t st, int dim, int64_t n, CSoa a, Soa b);
void launch_check_state(hipStream_t st, int dim, int64_t n, double c, CSoa v, unsigned long long* bad);
void launch_check_sigma(hipStream_t st, int64_t n, const double* sa, const double* ss, unsigned long long* bad);

// One level of the mixed-precision single-workgroup tail.
struct TailLevel32 {
    Lvl32 L;
    Soa32 w, d, e, e2, g, rho;
    Soa32 fr;  // source of the explicit sub-steps, A(w + d) + R(rho)
};

struct TailArgs32 {
    Phys ph;
    int lt, L, px, py, pseudo_steps, local;
    float reach;
    double eta;
    TailLevel32 lev[kMaxLevels];
};

// ---- batched execution (many independent problems, one launch per level op) ----
// Work-list entries pack (problem << kTileBits) | tile; a tile is 256 cells of
// one level of one problem.
constexpr int kTileBits = 20;

// One (problem, level) of a batch: device pointers of that level's buffers.
struct BSlot {
    Lvl L;
    Soa v, u, u2, f, rb;  // level >= 1
    Soa b, x0, x1, rf;    // level 0: rhs, the two iterate buffers (x0 = the request's state), residual
};

// One (problem, level) of a mixed-precision batch: the FP32 buffers of that level.
struct BSlot32 {
    Lvl32 L;
    Soa32 w, d, e, e2, g, rho, fr;  // level >= 1 (fr: source of the explicit sub-steps)
    Soa32 base, r32, dA, dB, rho0;  // level 0
};

// Per-problem data of a batch.
struct BProb {
    Phys ph;
    int px, py, L, lt, local, pseudo_steps, npart, pad_;
    double eta, reach, omega;
    Ctrl* ctrl;
    double* partials;
    const TailArgs* tail;
    const TailArgs32* tail32;  // mixed precision
    Ctrl proto;  // solver tolerances of this problem, copied into ctrl at every step start
};

// Batched kernels loop over a work list: block-stride over entries, skipping
// problems whose step has stopped; k is the cell of the entry's 256-cell tile.
#define M1_BATCH_LOOP(wl, nwl)                                          \
    for (int w_ = blockIdx.x; w_ < (nwl); w_ += gridDim.x) {            \
        const uint32_t item = (wl)[w_];                                 \
        const int p = (int)(item >> kTileBits);                         \
        const uint32_t tile = item & ((1u << kTileBits) - 1u);          \
        const BProb& pb = P[p];                                         \
        if (pb.ctrl->active == 0) continue;                             \
        const uint32_t k = tile * 256u + threadIdx.x;

// mixed precision (m1_mixed.hip)
int batch_grid_cap();
void set_batch_grid_cap(int cap);
// rows of the LDS-staged finest sweep's 64-wide tile (0: one-cell-per-thread sweep)
int sweep_rows();
bool set_sweep_rows(int rows);
// rows of the 64-wide tile of the fused pair of finest sweeps, FP64 and mixed
// precision (0: sweeps launched one by one)
int pair_rows();
bool set_pair_rows(int rows);
// the same for the mixed-precision correction sweeps
int mx_sweep_rows();
bool set_mx_sweep_rows(int rows);
// finest-level residual fused with the restriction to level 1 (launch shape; 0: two kernels)
int residual_restrict();
void set_residual_restrict(int on);
// 2-D: coarse (vc, rc) = R(u), R(X + sgn A(u)) of the fine level L, without storing the fine residual
void launch_residual_restrict(hipStream_t st, const Phys& ph, const Lvl& L, CSoa u, CSoa X, double sgn, int px, int py,
                              Soa vc, Soa rc, const int* active);
// LDS-staged finest-level sweep (2-D, beta = 0, gamma = 1, no norm); with uc.E
// non-null the gathered states are first corrected from level 1 (uc, vc) and
// projected, as by launch_prolong_project.  false (nothing launched) when the
// staged sweep is switched off.
bool launch_relax_lds(hipStream_t st, const Phys& ph, const Lvl& L, CSoa rhs, double omega, CSoa u, Soa out,
                      const int* active, CSoa uc, CSoa vc, int px, int py, double eta);
// two finest-level sweeps (2-D, beta = 0, gamma = 1, no norm) in one launch, u -> out
// (distinct buffers); false (nothing launched) when the fused pair is switched off
bool launch_relax2_lds(hipStream_t st, const Phys& ph, const Lvl& L, CSoa rhs, double omega, CSoa u, Soa out,
                       const int* active);
// batched FP64 kernels (m1_kernels.hip); `wl` is a work list of nwl entries,
// `plist` a list of problem indices
// fused residual of level - 1 and restriction to `level` over a work list of 32 x 4 coarse tiles
void launch_b_residual_restrict(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int level,
                                int in_sel);
void launch_b_relax(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int in_x1, int norm);
// two finest-level sweeps per launch over a work list of 64 x rows tiles (rows 4, 8 or 16)
void launch_b_relax2_lds(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int in_x1,
                         int rows);
// staged finest-level sweep over a work list of 64 x rows tiles (rows 4, 8 or 16)
void launch_b_relax_lds(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int in_x1,
                        int rows, bool up = false);
void launch_b_norm_control(hipStream_t st, const BProb* P, const int* plist, int np, int mixed);
void launch_b_apply(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int level, int in_sel);
void launch_b_restrict(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int level,
                       int in_sel);
void launch_b_pseudo(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int level,
                     int in_sel, int out_sel, int first);
void launch_b_prolong(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl, int level,
                      int in_sel, int out_sel);
void launch_b_tail(hipStream_t st, const BProb* P, const int* plist, int np);
void launch_b_init_tiles(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl);
void launch_b_init_ctrl(hipStream_t st, const BProb* P, const BSlot* S, const int* plist, int np);
void launch_b_flip_copy(hipStream_t st, const BProb* P, const BSlot* S, const uint32_t* wl, int nwl);
void launch_b_gather_ctrl(hipStream_t st, const BProb* P, int np, Ctrl* out);

// zL, zd: also the cycle's first correction sweep (from d = 0; level zL, relaxation zomega) into zd
// (false, nothing launched: zd is the buffer of d -- the launch reads d at every cell's neighbours while the
// fused sweep writes zd)
bool launch_mx_resid(hipStream_t st, int dim, const Phys& ph, const Lvl& L, double eta, CSoa v, CSoa32 d, CSoa b,
                     Soa vnew, Soa32 base, Soa32 r32, double* partials, const int* active,
                     const Lvl32* zL = nullptr, float zomega = 0.0f, Soa32 zd = {});
// two mixed-precision correction sweeps (2-D, beta = 0, gamma = 1, d given) in one launch, d -> out;
// false (nothing launched) when the pair launch shape is off
bool launch_mx_sweep2(hipStream_t st, const Phys& ph, const Lvl32& L, CSoa32 w, CSoa32 d, CSoa32 rhs, float omega,
                      Soa32 out, const int* active);
void launch_mx_sweep(hipStream_t st, int dim, const Phys& ph, const Lvl32& L, CSoa32 w, CSoa32 d, CSoa32 rhs,
                     float beta, float gamma, float omega, Soa32 out, const int* active);
// 2-D: coarse (wc, dc, gc) = R(w), R(d), R(X + sgn N_w(d)) of the fine level L, without storing rho
void launch_mx_residual_restrict(hipStream_t st, const Phys& ph, const Lvl32& L, CSoa32 w, CSoa32 d, CSoa32 X,
                                 float sgn, int px, int py, Soa32 wc, Soa32 dc, Soa32 gc, const int* active);
void launch_mx_apply(hipStream_t st, int dim, const Phys& ph, const Lvl32& L, CSoa32 w, CSoa32 d, CSoa32 X, float sgn,
                     Soa32 out, const int* active);
// fr: the source of the explicit sub-steps, A(w + d) + R(rho), formed by the first pseudo-time step of a visit
// (first != 0) and read by the others.
void launch_mx_pseudo(hipStream_t st, int dim, const Phys& ph, const Lvl32& L, CSoa32 w, Soa32 g, Soa32 fr,
                      CSoa32 e, Soa32 out, double dtau, const double* dtau_dev, float reach, int local, int first,
                      const int* active);
void launch_mx_prolong(hipStream_t st, int dim, const Phys& ph, int nx, int ny, int px, int py, float eta, CSoa32 w,
                       CSoa32 e, CSoa32 ec, CSoa32 dc, Soa32 out, const int* active);
void launch_mx_prolong_fine(hipStream_t st, int dim, const Phys& ph, int nx, int ny, int px, int py, double eta,
                            CSoa v, CSoa32 e, CSoa32 ec, CSoa32 dc, Soa32 out, const int* active);
// 2-D: the coarse correction of the finest level and the first post-smoothing
// sweep in one launch (LDS-staged; false, nothing launched, when unstaged)
bool launch_mx_prolong_sweep(hipStream_t st, const Phys& ph, const Lvl32& L, CSoa32 w, CSoa v, CSoa32 e, CSoa32 ec,
                             CSoa32 dc, int px, int py, double eta, CSoa32 rhs, float omega, Soa32 out,
                             const int* active);
void launch_mx_restrict(hipStream_t st, int dim, int nxf, int nyf, int px, int py, const Fields32& F,
                        const int* active);
void launch_mx_tail(hipStream_t st, int dim, const TailArgs32* args_dev, double dtau, const double* dtau_dev,
                    const int* active);
void launch_to_f32(hipStream_t st, int64_t n, const double* a, float* b);

// batched mixed-precision kernels (m1_mixed.hip).  Fine-level selectors: the
// FP64 state is x0 or x1 by ctrl->flip; sel 0/1 picks dA/dB.  Coarse levels:
// sel 0 = d, 1 = e, 2 = e2.
// zero: also the first pre-sweep (from a zero correction) into buffer 0
void launch_bm_resid(hipStream_t st, const BProb* P, const BSlot* S, const BSlot32* S32, const uint32_t* wl, int nwl,
                     int pend_sel, int zero);
void launch_bm_sweep(hipStream_t st, const BProb* P, const BSlot32* S32, const uint32_t* wl, int nwl, int in_sel,
                     int out_sel, int from_zero);
// fused residual of level - 1 and restriction to `level` over a work list of 32 x 4 coarse tiles
void launch_bm_residual_restrict(hipStream_t st, const BProb* P, const BSlot32* S32, const uint32_t* wl, int nwl,
                                 int level, int d0_sel);
// staged correction sweep (d given) over a work list of 64 x rows tiles of the finest levels
void launch_bm_sweep_lds(hipStream_t st, const BProb* P, const BSlot32* S32, const uint32_t* wl, int nwl, int in_sel,
                         int out_sel, int rows);
void launch_bm_apply(hipStream_t st, const BProb* P, const BSlot32* S32, const uint32_t* wl, int nwl, int level,
                     int in_sel);
void launch_bm_restrict(hipStream_t st, const BProb* P, const BSlot32* S32, const uint32_t* wl, int nwl, int level,
                        int d0_sel);
void launch_bm_pseudo(hipStream_t st, const BProb* P, const BSlot32* S32, const uint32_t* wl, int nwl, int level,
                      int in_sel, int out_sel, int first);
void launch_bm_prolong(hipStream_t st, const BProb* P, const BSlot32* S32, const uint32_t* wl, int nwl, int level);
void launch_bm_prolong_fine(hipStream_t st, const BProb* P, const BSlot* S, const BSlot32* S32, const uint32_t* wl,
                            int nwl, int e_sel);
void launch_bm_tail(hipStream_t st, const BProb* P, const int* plist, int np);

}  // namespace m1
