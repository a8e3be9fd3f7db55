// hp_coarse.hip -- the coarsest multigrid level: its dense operator, assembled on the device, and
// the operator's inverse by blocked Gauss-Jordan elimination.
//
// The coarsest level holds at most a few thousand cells, so the V-cycle solves it exactly with
// one dense matrix-vector product by the stored inverse. The operator is the same seven-point
// flux-form matrix as on every other level (paper, Section 2, eq. Poiss times dt^2 with the
// coefficients of eqs. cpoiss/kappapoiss and the face factor of step (viii)); it is symmetric
// positive definite when m > 0 and rho > 0, so elimination needs no pivoting and every pivot
// (a diagonal entry of a Schur complement) is positive.
#include "hp_internal.h"

#include <cmath>

namespace hp {

// ------------------------------------------------------------------------------------------
// assembly: one thread per matrix entry (row a, column b), row-major, n = nx ny nz

__global__ __launch_bounds__(kBlock) void k_coarse_assemble(const double* __restrict__ rho,
                                                            const double* __restrict__ m, int nx, int ny,
                                                            int nz, int px, int py, int pz, double cx,
                                                            double cy, double cz, int face_rule,
                                                            double* __restrict__ A) {
    const int n = nx * ny * nz;
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int a = (int)(e / n), b = (int)(e - (int64_t)a * n);
    const int c[3] = {a % nx, (a / nx) % ny, a / (nx * ny)};
    const int dims[3] = {nx, ny, nz}, per[3] = {px, py, pz};
    const int stride[3] = {1, nx, nx * ny};
    const double cd[3] = {cx, cy, cz};
    double v = 0.0;
    if (a == b) v += m[a];
    const double ra = rho[a];
    // faces in the order x-, x+, y-, y+, z-, z+ (a diagonal entry accumulates them in that order)
    for (int d = 0; d < 3; ++d)
        for (int s = -1; s <= 1; s += 2) {
            int t = c[d] + s;
            if (t < 0 || t >= dims[d]) {
                if (!per[d] || dims[d] < 2) continue;  // Neumann wall: no face
                t = (t + dims[d]) % dims[d];
            }
            const int nb = a + (t - c[d]) * stride[d];
            if (a != b && nb != b) continue;
            const double rb = rho[nb];
            const double kappa = face_rule == 1 ? 0.5 * (1.0 / ra + 1.0 / rb) : 2.0 / (ra + rb);
            const double w = cd[d] * kappa;
            v = (a == b) ? v + w : v - w;
        }
    A[e] = v;
}

void launch_coarse_assemble(const double* rho, const double* m, const int n[3], const int per[3],
                            const double cd[3], int face_rule, double* A, hipStream_t s) {
    const int64_t N = (int64_t)n[0] * n[1] * n[2];
    const unsigned blocks = (unsigned)((N * N + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_coarse_assemble, dim3(blocks), dim3(kBlock), 0, s, rho, m, n[0], n[1], n[2],
                       per[0], per[1], per[2], cd[0], cd[1], cd[2], face_rule, A);
}

// ------------------------------------------------------------------------------------------
// inverse by blocked Gauss-Jordan elimination, in place
//
// The matrix is cut into kGJ-wide block rows and columns. Step K eliminates block column K:
// with D the inverse of the diagonal block A_KK (the Schur complement block left by steps
// 0 .. K-1), the block row becomes A_Kj <- D A_Kj, every other block row loses its multiple
// A_ij <- A_ij - A_iK A_Kj (old A_iK, new A_Kj), block column K takes A_iK <- -A_iK D, and the
// diagonal block becomes D. After the last step the array holds the inverse. This is the
// unblocked Gauss-Jordan sweep grouped by kGJ pivots: the same pivots, with the products summed in
// another order (and each pivot applied through its reciprocal).
//
// Two launches per step: k_gj_panel (one workgroup per block column) inverts A_KK in LDS by the
// unblocked sweep, updates its tile of block row K and saves its rows of the old block column K
// to the workspace; k_gj_update (one workgroup per tile) applies the rank-kGJ update. Neither
// launch writes what another workgroup of it reads:
//   k_gj_panel writes block row K outside block column K; it reads block column K and its own tile.
//   k_gj_update writes tiles outside block row K (and A_KK); it reads block row K outside block
//   column K and the workspace.
// Workspace layout (doubles): old block column K, n x kGJ row-major, then D, kGJ x kGJ.

constexpr int kGJ = 32;
constexpr int kGJThreads = 256;
constexpr int kGJPer = kGJ * kGJ / kGJThreads;  // entries of a kGJ x kGJ tile per thread

int64_t spd_inverse_work(int n) { return (int64_t)n * kGJ + kGJ * kGJ; }

// 1/x from the hardware estimate and two Newton steps (within an ulp or so). A zero, infinite or
// NaN pivot gives a result that is not finite; the pivot flag is taken from the pivot itself.
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

__global__ __launch_bounds__(kGJThreads) void k_gj_panel(double* __restrict__ a, double* __restrict__ work,
                                                         int n, int k0, int* __restrict__ flag) {
    __shared__ double Db[2][kGJ][kGJ + 1];  // the diagonal block, ping-ponged between pivots
    __shared__ double T[kGJ][kGJ + 1];
    const int t = threadIdx.x;
    const int bk = min(kGJ, n - k0);
    const int j0 = blockIdx.x * kGJ;
    const int nc = min(kGJ, n - j0);  // columns of this block column, rows of this row tile
    // every global read of the kernel up front, from clamped (in-range) indices, so that they are
    // in flight together: the diagonal block, this tile of block row K, and this tile's rows of
    // block column K; the padding is selected afterwards
    double dv[kGJPer], tv[kGJPer], cv[kGJPer];
#pragma unroll
    for (int u = 0; u < kGJPer; ++u) {
        const int e = t + kGJThreads * u, r = e / kGJ, c = e % kGJ;
        const int64_t rk = (int64_t)(k0 + min(r, bk - 1)) * n;
        dv[u] = a[rk + k0 + min(c, bk - 1)];
        tv[u] = a[rk + j0 + min(c, nc - 1)];
        cv[u] = a[(int64_t)(j0 + min(r, nc - 1)) * n + k0 + min(c, bk - 1)];
    }
    // the diagonal block, padded to kGJ x kGJ with the identity (which the sweep leaves alone);
    // the row-panel tile, padded with zeros
#pragma unroll
    for (int u = 0; u < kGJPer; ++u) {
        const int e = t + kGJThreads * u, r = e / kGJ, c = e % kGJ;
        Db[0][r][c] = (r < bk && c < bk) ? dv[u] : (r == c ? 1.0 : 0.0);
        T[r][c] = (r < bk && c < nc) ? tv[u] : 0.0;
    }
    // unblocked Gauss-Jordan: pivot p scales row p by its reciprocal, the other rows lose their
    // multiple of it, column p takes the negated multipliers and 1/pivot on the diagonal. Every
    // entry of a step is read before the reciprocal is formed and the result is selected, not
    // branched to, so each step costs one LDS round trip, the reciprocal and one barrier.
    bool bad = false;
    for (int p = 0; p < kGJ; ++p) {
        __syncthreads();
        const double(*S)[kGJ + 1] = Db[p & 1];
        double(*W)[kGJ + 1] = Db[(p + 1) & 1];
        const double piv = S[p][p];
        double dpc[kGJPer], drp[kGJPer], drc[kGJPer];
#pragma unroll
        for (int u = 0; u < kGJPer; ++u) {
            const int e = t + kGJThreads * u, r = e / kGJ, c = e % kGJ;
            dpc[u] = S[p][c];
            drp[u] = S[r][p];
            drc[u] = S[r][c];
        }
        const double rp = rcp_nr(piv);
#pragma unroll
        for (int u = 0; u < kGJPer; ++u) {
            // keeps the read of drc[u] up front (otherwise it can sink under the c != p branch)
            asm volatile("" : "+v"(drc[u]));
            const int e = t + kGJThreads * u, r = e / kGJ, c = e % kGJ;
            const double f = drp[u] * rp;
            const double other = (c == p) ? -f : drc[u] - f * dpc[u];
            const double prow = (c == p) ? rp : dpc[u] * rp;
            W[r][c] = (r == p) ? prow : other;
        }
        bad = bad || (p < bk && !(piv > 0.0 && piv < INFINITY));
    }
    if (bad && blockIdx.x == 0 && t == 0) *flag = 1;
    double(*D)[kGJ + 1] = Db[kGJ & 1];
    __syncthreads();
    if (j0 == k0) {
        for (int e = t; e < kGJ * kGJ; e += kGJThreads) work[(int64_t)n * kGJ + e] = D[e / kGJ][e % kGJ];
    } else {
        // the padding of D (identity) and T (zero rows) adds exact zeros to the sums
        for (int e = t; e < kGJ * kGJ; e += kGJThreads) {
            const int r = e / kGJ, c = e % kGJ;
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < kGJ; ++q) s += D[r][q] * T[q][c];
            if (r < bk && c < nc) a[(int64_t)(k0 + r) * n + j0 + c] = s;
        }
    }
    // this tile's rows of block column K as they were before this step (the update reads them)
#pragma unroll
    for (int u = 0; u < kGJPer; ++u) {
        const int e = t + kGJThreads * u, r = e / kGJ, q = e % kGJ;
        if (r < nc && q < bk) work[(int64_t)(j0 + r) * kGJ + q] = cv[u];
    }
}

__global__ __launch_bounds__(kGJThreads) void k_gj_update(double* __restrict__ a,
                                                          const double* __restrict__ work, int n, int k0) {
    __shared__ double C[kGJ][kGJ + 1];  // old block column K, this tile's rows
    __shared__ double P[kGJ][kGJ + 1];  // new block row K, this tile's columns (D for column K)
    const int t = threadIdx.x;
    const int bk = min(kGJ, n - k0);
    const int i0 = blockIdx.y * kGJ, j0 = blockIdx.x * kGJ;
    const double* Dw = work + (int64_t)n * kGJ;
    if (i0 == k0) {
        if (j0 == k0)
            for (int e = t; e < kGJ * kGJ; e += kGJThreads) {
                const int r = e / kGJ, c = e % kGJ;
                if (r < bk && c < bk) a[(int64_t)(k0 + r) * n + k0 + c] = Dw[e];
            }
        return;
    }
    const bool colK = (j0 == k0);
    const int nr = min(kGJ, n - i0), nc = min(kGJ, n - j0);
    // block row K's tile (D for block column K), row stride ps
    const double* Ps = colK ? Dw : a + (int64_t)k0 * n + j0;
    const int64_t ps = colK ? kGJ : n;
    // thread t updates row t / 8 of the tile, columns t % 8 + 8 u
    const int r = t / 8;
    // every global read up front, from clamped indices; the zero padding is selected afterwards
    double cv[kGJPer], pv[kGJPer], old[kGJPer];
#pragma unroll
    for (int u = 0; u < kGJPer; ++u) {
        const int e = t + kGJThreads * u, er = e / kGJ, ec = e % kGJ;
        cv[u] = work[(int64_t)(i0 + min(er, nr - 1)) * kGJ + min(ec, bk - 1)];
        pv[u] = Ps[(int64_t)min(er, bk - 1) * ps + min(ec, nc - 1)];
        old[u] = a[(int64_t)(i0 + min(r, nr - 1)) * n + j0 + min(t % 8 + 8 * u, nc - 1)];
    }
#pragma unroll
    for (int u = 0; u < kGJPer; ++u) {
        const int e = t + kGJThreads * u, er = e / kGJ, ec = e % kGJ;
        C[er][ec] = (er < nr && ec < bk) ? cv[u] : 0.0;
        P[er][ec] = (er < bk && ec < nc) ? pv[u] : 0.0;
    }
    __syncthreads();
    // the zero padding of C and P adds exact zeros to the sums
    double s[kGJPer];
#pragma unroll
    for (int u = 0; u < kGJPer; ++u) s[u] = 0.0;
#pragma unroll
    for (int q = 0; q < kGJ; ++q) {
        const double cq = C[r][q];
#pragma unroll
        for (int u = 0; u < kGJPer; ++u) s[u] += cq * P[q][t % 8 + 8 * u];
    }
#pragma unroll
    for (int u = 0; u < kGJPer; ++u) {
        const int c = t % 8 + 8 * u;
        if (r < nr && c < nc) a[(int64_t)(i0 + r) * n + j0 + c] = colK ? -s[u] : old[u] - s[u];
    }
}

// x = (x + x^T) / 2 in place (one thread per pair i < j)
__global__ __launch_bounds__(kBlock) void k_symmetrize(double* __restrict__ x, int n) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
    if (i >= j) return;
    const double v = 0.5 * (x[(int64_t)i * n + j] + x[(int64_t)j * n + i]);
    x[(int64_t)i * n + j] = v;
    x[(int64_t)j * n + i] = v;
}

void launch_spd_inverse(double* a, double* work, int n, int* flag, hipStream_t s) {
    const unsigned nt = (unsigned)((n + kGJ - 1) / kGJ);
    for (int k0 = 0; k0 < n; k0 += kGJ) {
        hipLaunchKernelGGL(k_gj_panel, dim3(nt), dim3(kGJThreads), 0, s, a, work, n, k0, flag);
        hipLaunchKernelGGL(k_gj_update, dim3(nt, nt), dim3(kGJThreads), 0, s, a, (const double*)work, n, k0);
    }
    const unsigned blocks = (unsigned)(((int64_t)n * n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_symmetrize, dim3(blocks), dim3(kBlock), 0, s, a, n);
}

}  // namespace hp
