// Kernels of the Gram-Schmidt step of FGMRES with the second projection delayed by one step (DCGS2:
// classical Gram-Schmidt with reorthogonalisation, the second pass of a new basis vector merged into
// the first pass of the next step).  All vectors are device arrays of n doubles; the basis V holds
// its vectors ldv apart.
#pragma once

#include <hip/hip_runtime.h>

namespace sg {

// Largest number of final basis vectors of one step (the FGMRES restart length is at most 64).
constexpr int kDcgsMaxBasis = 64;

// Pass A of step j.  With V[0..j-1] the final (orthonormal) basis vectors, u the tentative j-th one and
// w = A z_j, partial[blk][0..2j+1] = this block's share of
//     [V^T u (j values), V^T w (j values), u.u, u.w].
// nblk blocks of 256 threads; reduce with launch_reduce_partials(partial, nblk, 2j + 2, ...).
hipError_t launch_dcgs_dots(const double* V, long long ldv, int j, const double* u, const double* w, long long n,
                            double* partial, int nblk, hipStream_t s);

// Pass B of step j, from the reduced pass-A values r = [a (j), b (j), u.u, u.w]:
//     nu = sqrt(u.u - |a|^2)             (Pythagoras: V orthonormal; 0 where not positive)
//     e  = (u.w - a.b) / nu              (the projection of w onto the final j-th vector; 0 if nu = 0)
//     u     <- (u - V a) / nu            (the final j-th basis vector, written over u)
//     unext <- w - V b - e u             (the next tentative vector, orthogonal to V[0..j] once)
// and partial[blk] = this block's share of |unext|^2.  Sums over the basis run in ascending order, so a
// host recomputing nu and e from r in the same order obtains the same values.
hipError_t launch_dcgs_update(const double* V, long long ldv, int j, const double* r, double* u, const double* w,
                              double* unext, long long n, double* partial, int nblk, hipStream_t s);

}  // namespace sg
