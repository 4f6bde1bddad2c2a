// m1_internal.hpp -- kernel launchers shared by the plan/driver code.
#pragma once

#include "m1_device.hpp"

namespace m1 {

struct Fields;

void launch_relax(hipStream_t st, int dim, const Phys& ph, const Lvl& L, CSoa rhs, const double* gamma_cell,
                  double beta, double gamma, double omega, CSoa u, Soa out);
void launch_pseudo(hipStream_t st, int dim, const Phys& ph, const Lvl& L, CSoa f, CSoa u, Soa out, double dtau,
                   double reach, int local, Soa rhs_store, double* g_store);
unsigned apply_blocks(const Lvl& L);
void launch_apply(hipStream_t st, int dim, const Phys& ph, const Lvl& L, CSoa v, CSoa X, double sgn, Soa out,
                  double* partials);
void launch_norm_finalize(hipStream_t st, const double* partials, int n, double* out);
void launch_restrict(hipStream_t st, int dim, int nxf, int nyf, int px, int py, const Fields& F);
void launch_prolong_project(hipStream_t st, int dim, const Phys& ph, int nx, int ny, int px, int py, double eta,
                            CSoa u, CSoa uc, CSoa vc, Soa out);
void launch_make_rhs(hipStream_t st, int dim, int64_t n, double cv, CSoa v, Soa b);
void launch_copy(hipStream_t st, int dim, int64_t n, CSoa a, Soa b);
void launch_check_state(hipStream_t st, int dim, int64_t n, double c, CSoa v, unsigned long long* bad);
void launch_check_sigma(hipStream_t st, int64_t n, const double* sa, const double* ss, unsigned long long* bad);

struct Fields {
    const double* in[10];
    double* out[10];
    int n;
};

}  // namespace m1
