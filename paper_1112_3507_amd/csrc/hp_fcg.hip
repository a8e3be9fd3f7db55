// hp_fcg.hip -- the scalar steps of the learned flexible CG on the device, so that an iteration
// synchronises with the host only once (for its convergence check).
//
// The learned preconditioner stage is z = g y + M (r - g A y) with y the network's estimate,
// M one V-cycle and g = <r, y> / <y, A y> the A-norm-optimal step (0 when the network points
// uphill or returns something non-finite); the FCG recurrences take alpha = <p, r> / <p, A p> and
// beta = -<z, A p_old> / <p_old, A p_old>. The dot products land in device slots (second
// reduction stage); these kernels turn them into g, alpha and beta and apply g.
#include "hp_internal.h"

#include <cmath>

namespace hp {

namespace {

// one thread: the scalar of `what` from the slots
__global__ void k_fcg_scalar(double* __restrict__ sc, int what) {
    switch (what) {
        case FCG_GAMMA: {  // g = S_T1 / S_T2 = <r, y> / <y, A y>
            const double ry = sc[S_T1], yay = sc[S_T2];
            sc[S_GAMMA] = (ry > 0.0 && yay > 0.0 && std::isfinite(ry) && std::isfinite(yay)) ? ry / yay : 0.0;
            break;
        }
        case FCG_ALPHA: {  // alpha = S_T1 / S_PQ = <p, r> / <p, A p> (0 if p^T A p is not positive)
            const double pq = sc[S_PQ];
            sc[S_ALPHA] = (pq > 0.0 && std::isfinite(pq)) ? sc[S_T1] / pq : 0.0;
            break;
        }
        default: {  // FCG_BETA: beta = -S_T1 / S_PQ = -<z, A p_old> / <p_old, A p_old>
            const double pq = sc[S_PQ];
            sc[S_BETA] = (pq > 0.0 && std::isfinite(pq)) ? -sc[S_T1] / pq : 0.0;
            break;
        }
    }
}

// SUB: y = x - g y (y = x when g = 0: a non-finite y is not carried along);
// else y = y + g x (unchanged when g = 0)
template <bool SUB>
__global__ __launch_bounds__(kBlock) void k_fcg_gamma_update(double* __restrict__ y, const double* __restrict__ x,
                                                             const double* __restrict__ sc, int64_t n) {
    const double g = sc[S_GAMMA];
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x; a < n; a += stride) {
        if (SUB)
            y[a] = (g == 0.0) ? x[a] : x[a] - g * y[a];
        else if (g != 0.0)
            y[a] += g * x[a];
    }
}

unsigned grid_for(int64_t n) {
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

void launch_fcg_scalar(double* scal, int what, hipStream_t s) {
    hipLaunchKernelGGL(k_fcg_scalar, dim3(1), dim3(1), 0, s, scal, what);
}

void launch_fcg_gamma_update(double* y, const double* x, const double* scal, int64_t n, bool sub, hipStream_t s) {
    if (sub)
        hipLaunchKernelGGL(k_fcg_gamma_update<true>, dim3(grid_for(n)), dim3(kBlock), 0, s, y, x, scal, n);
    else
        hipLaunchKernelGGL(k_fcg_gamma_update<false>, dim3(grid_for(n)), dim3(kBlock), 0, s, y, x, scal, n);
}

}  // namespace hp
