// m1_transfer.hip -- the cell-agglomeration pair of grid-transfer operators.
//
// Sect. 6.3 leaves the transfer operators open as a choice that changes the
// speed of the method; Sect. 4.2 builds its restriction from its prolongation
// as R = 2^-d P^T.  Here coarse cell (I, J) is the union of fine cells
// 2I..2I+1 x 2J..2J+1: the prolongation gives each of them the coarse value,
// so R = 2^-d P^T is their mean.  Neither operator reads a ghost, so the side
// conditions play no part.  One thread per output cell, in the XCD-aware block
// order of the other grid kernels; the stop flag gates the stores.
#include "m1_transfer.hpp"

namespace m1 {

namespace {

constexpr int kTB = 256;

unsigned tblocks(int64_t n) { return (unsigned)((n + kTB - 1) / kTB); }

// 0 in a vector register: keeps the flag read an ordinary vector load, ordered
// with the data loads (as in the other kernel files).
__device__ __forceinline__ uint32_t vzero()
{
    uint32_t z = 0;
    asm("" : "+v"(z));
    return z;
}

}  // namespace

// Sum of the 2^d children in the order (2I, 2J), (2I+1, 2J), (2I, 2J+1),
// (2I+1, 2J+1), times 2^-d: the scaling is exact, so this rounds like the
// weighted sum of the same terms in that order.
template <int DIM, int NF>
__global__ __launch_bounds__(kTB) void k_restrict_mean(int nxf, int nyf, Fields F, const int* __restrict__ active)
{
    const bool live = active[vzero()] != 0;
    const int nxc = nxf / 2;
    const uint32_t nc = (uint32_t)nxc * (uint32_t)((DIM == 2) ? nyf / 2 : 1);
    const uint32_t k = (uint32_t)xcd_block() * kTB + threadIdx.x;
    if (k >= nc) return;
    const uint32_t I = k % (uint32_t)nxc, J = k / (uint32_t)nxc;
    const uint32_t f0 = ((DIM == 2) ? 2u * J * (uint32_t)nxf : 0u) + 2u * I;
    double v[NF][(DIM == 2) ? 4 : 2];
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        v[q][0] = ld(F.in[q], f0);
        v[q][1] = ld(F.in[q], f0 + 1);
        if (DIM == 2) {
            v[q][2] = ld(F.in[q], f0 + (uint32_t)nxf);
            v[q][3] = ld(F.in[q], f0 + (uint32_t)nxf + 1);
        }
    }
    if (!live) return;
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        const double s = (DIM == 2) ? ((v[q][0] + v[q][1]) + v[q][2]) + v[q][3] : v[q][0] + v[q][1];
        st(F.out[q], k, s * ((DIM == 2) ? 0.25 : 0.5));
    }
}

template <int DIM>
__global__ __launch_bounds__(kTB) void k_prolong_const_project(Phys ph, int nx, int ny, double eta, CSoa u, CSoa uc,
                                                               CSoa vc, Soa out, const int* __restrict__ active)
{
    const bool live = active[vzero()] != 0;
    const uint32_t k = (uint32_t)xcd_block() * kTB + threadIdx.x;
    if (k >= (uint32_t)nx * (uint32_t)ny) return;
    const uint32_t i = k % (uint32_t)nx, j = k / (uint32_t)nx;
    const uint32_t kc = (DIM == 2) ? (j >> 1) * (uint32_t)(nx / 2) + (i >> 1) : (i >> 1);
    const double uE = ld(u.E, k), uFx = ld(u.Fx, k), uFy = (DIM == 2) ? ld(u.Fy, k) : 0.0, uT = ld(u.T, k);
    const double e0 = ld(uc.E, kc) - ld(vc.E, kc);
    const double e1 = ld(uc.Fx, kc) - ld(vc.Fx, kc);
    const double e2 = (DIM == 2) ? ld(uc.Fy, kc) - ld(vc.Fy, kc) : 0.0;
    const double e3 = ld(uc.T, kc) - ld(vc.T, kc);
    double wE = uE + e0, wFx = uFx + e1, wFy = uFy + e2, wT = uT + e3;
    if (!admissible(ph.c2, wE, wFx, wFy, wT)) {  // eq. prolongatedSol: the largest admissible part of the step
        const double th = eta * fmin(ray_len(ph.c2, uE, uFx, uFy, uT, e0, e1, e2, e3), 1.0);
        wE = fma(th, e0, uE);
        wFx = fma(th, e1, uFx);
        wFy = fma(th, e2, uFy);
        wT = fma(th, e3, uT);
    }
    if (!live) return;
    st(out.E, k, wE);
    st(out.Fx, k, wFx);
    if (DIM == 2) st(out.Fy, k, wFy);
    st(out.T, k, wT);
}

void launch_restrict_mean(hipStream_t st, int dim, int nxf, int nyf, const Fields& F, const int* active)
{
    const int64_t nc = (int64_t)(nxf / 2) * (dim == 2 ? nyf / 2 : 1);
    const dim3 g(tblocks(nc)), b(kTB);
    if (dim == 2) {
        switch (F.n) {
        case 2: hipLaunchKernelGGL((k_restrict_mean<2, 2>), g, b, 0, st, nxf, nyf, F, active); break;
        case 4: hipLaunchKernelGGL((k_restrict_mean<2, 4>), g, b, 0, st, nxf, nyf, F, active); break;
        default: hipLaunchKernelGGL((k_restrict_mean<2, 8>), g, b, 0, st, nxf, nyf, F, active); break;
        }
    } else {
        switch (F.n) {
        case 2: hipLaunchKernelGGL((k_restrict_mean<1, 2>), g, b, 0, st, nxf, nyf, F, active); break;
        case 3: hipLaunchKernelGGL((k_restrict_mean<1, 3>), g, b, 0, st, nxf, nyf, F, active); break;
        default: hipLaunchKernelGGL((k_restrict_mean<1, 6>), g, b, 0, st, nxf, nyf, F, active); break;
        }
    }
}

void launch_prolong_const_project(hipStream_t st, int dim, const Phys& ph, int nx, int ny, double eta, CSoa u,
                                  CSoa uc, CSoa vc, Soa out, const int* active)
{
    const dim3 g(tblocks((int64_t)nx * ny)), b(kTB);
    if (dim == 2)
        hipLaunchKernelGGL((k_prolong_const_project<2>), g, b, 0, st, ph, nx, ny, eta, u, uc, vc, out, active);
    else
        hipLaunchKernelGGL((k_prolong_const_project<1>), g, b, 0, st, ph, nx, ny, eta, u, uc, vc, out, active);
}

}  // namespace m1
