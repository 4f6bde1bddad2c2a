// m1_3d.hpp -- the three-dimensional form of the cycle operations (device
// structures and kernel launchers; kernels in m1_kernels3.hip).
//
// The paper writes its scheme in 1-D and says the extension to more
// dimensions is direct (Sect. 2.2); its restriction is R = 2^-d P^T for
// d = 1, 2, 3 (Sect. 4.2).  In 3-D a state has five fields (E, Fx, Fy, Fz, T),
// each nx*ny*nz doubles with x fastest; sides are x-, x+, y-, y+, z-, z+.
#pragma once

#include "m1_internal.hpp"

namespace m1 {

struct Phys3 {
    double c, c2, a_r, c_v;
    int bc[6];
    double bcE[6], bcFx[6], bcFy[6], bcFz[6];
    unsigned long long* stalls;  // pseudo-time stall counter (device; may be null)
};

// One level: cells numbered k = (z ny + y) nx + x in 32 bits.
struct Lvl3 {
    int nx, ny, nz;
    double kx, ky, kz;  // dt / (2 h) per axis
    double a;           // 1 + c dt (1/hx + 1/hy + 1/hz)
    double cdt;         // c dt
    const double* sa;
    const double* ss;
};

struct Soa3 {
    double *E, *Fx, *Fy, *Fz, *T;
};
struct CSoa3 {
    const double *E, *Fx, *Fy, *Fz, *T;
};
inline CSoa3 cs3(const Soa3& s) { return CSoa3{s.E, s.Fx, s.Fy, s.Fz, s.T}; }

// out = x + sgn A_l(v) (x.E null: sgn A_l(v)); with partials, each block's sum
// of r_E^2 + |r_F/c|^2 + r_T^2 of out goes to partials[block] (256-thread blocks).
void launch3_apply(hipStream_t st, const Phys3& ph, const Lvl3& L, CSoa3 v, CSoa3 x, double sgn, Soa3 out,
                   double* partials, const int* active);
// One relaxed Jacobi sweep of A(u) = b (Algorithm 1): out = u + omega (J(u) - u).  With partials, the
// block sums of r_E^2 + |r_F/c|^2 + r_T^2 of the input's residual b - A(u) (per cell the value k3_apply
// gives) go to partials[block]; returns the number of blocks (of partials written).
unsigned launch3_relax(hipStream_t st, const Phys3& ph, const Lvl3& L, CSoa3 b, double omega, CSoa3 in, Soa3 out,
                       const int* active, double* partials = nullptr);
// One pseudo-time step (Algorithm 3) of M du/dtau + A_l(u) = f with one Jacobi
// sweep; reach = 1 - (1 - eta)^K; dtau from dtau_dev when not null.
void launch3_pseudo(hipStream_t st, const Phys3& ph, const Lvl3& L, CSoa3 f, CSoa3 in, Soa3 out, double dtau,
                    const double* dtau_dev, double reach, int local, const int* active);
// The same three operations staged (2.5-D blocking: closures of a 64 x 4 tile and its ring once per z-plane
// in LDS), bitwise equal to the one-cell forms above; the apply form without the norm partials.  Launch
// shape "stage3": 0 one-cell kernels only; 1 (default) staged sweeps and A (stage3_fits with sweep = true) on
// levels of at least kStage3MinCells cells (on smaller ones too few blocks, each marching through 8 planes in
// sequence); 2 every staged form on every level.  Levels narrower than kStage3MinNx keep the one-cell kernels (most of a 64-wide
// tile would idle).
constexpr int kStage3MinNx = 32;
constexpr int64_t kStage3MinCells = int64_t(1) << 23;
bool stage3_fits(const Lvl3& L, bool sweep);
// Blocks of one staged launch on an nx x ny x nz level (each writes one norm partial when it reduces one): on
// thin levels more than the one-cell kernels' ceil(n / 256).
int64_t staged3_blocks(int nx, int ny, int nz);
void set_stage3(int mode);
int stage3();
void launch3_apply_staged(hipStream_t st, const Phys3& ph, const Lvl3& L, CSoa3 v, CSoa3 x, double sgn, Soa3 out,
                          const int* active);
unsigned launch3_relax_staged(hipStream_t st, const Phys3& ph, const Lvl3& L, CSoa3 b, double omega, CSoa3 in,
                              Soa3 out, const int* active, double* partials = nullptr);
void launch3_pseudo_staged(hipStream_t st, const Phys3& ph, const Lvl3& L, CSoa3 f, CSoa3 in, Soa3 out,
                           double dtau, const double* dtau_dev, double reach, int local, const int* active);
// Full weighting R = 2^-3 P^T of the fields in F from a fine nxf x nyf x nzf level.
void launch3_restrict(hipStream_t st, int nxf, int nyf, int nzf, int px, int py, int pz, const Fields& F,
                      const int* active);
// out = u + P(uc - vc) (trilinear) with the admissibility correction (eq. prolongatedSol).  Launch shape
// "prolong3_lds": 1 (default) the coarse differences of a 32 x 4 x 2 coarse tile staged in LDS once, 0 one
// fine cell per thread reading its coarse cells; the same bits either way.
void set_prolong3_lds(int on);
int prolong3_lds();
void launch3_prolong_project(hipStream_t st, const Phys3& ph, int nx, int ny, int nz, int px, int py, int pz,
                             double eta, CSoa3 u, CSoa3 uc, CSoa3 vc, Soa3 out, const int* active);
// b = (E, F, C_v T) of v.
void launch3_make_rhs(hipStream_t st, int64_t n, double cv, CSoa3 v, Soa3 b);
// Smallest index of a cell that is not admissible (E > 0, T > 0, |F| <= cE, all finite) into *bad.
void launch3_check_state(hipStream_t st, int64_t n, double c, CSoa3 v, unsigned long long* bad);
// Copy of a state.
void launch3_copy(hipStream_t st, int64_t n, CSoa3 a, Soa3 b);

}  // namespace m1
