// m1_transfer.hpp -- launchers of the cell-agglomeration transfer pair, used
// in place of full weighting (Sect. 4.2) when a plan selects it.
#pragma once

#include "m1_internal.hpp"

namespace m1 {

// Coarse cell k of each field in F: the mean of its 2^d fine cells.
void launch_restrict_mean(hipStream_t st, int dim, int nxf, int nyf, const Fields& F, const int* active);

// out = u + P0(uc - vc), P0 piecewise constant, with the admissibility
// correction of eq. prolongatedSol (in place when out == u).
void launch_prolong_const_project(hipStream_t st, int dim, const Phys& ph, int nx, int ny, double eta, CSoa u,
                                  CSoa uc, CSoa vc, Soa out, const int* active);

}  // namespace m1
