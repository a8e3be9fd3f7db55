// hp_kernels.hip -- gfx950 kernels of the pressure solve (FP64 and FP32 instantiations).
//
// Operator (paper, Section 2, eq. Poiss times dt^2, coefficients eqs. cpoiss/kappapoiss, face
// factor of step (viii)): (A p)_a = m_a p_a + sum_f w_f (p_a - p_b), w_f = c_d * 2/(rho_a+rho_b),
// c_d = dt^2 / h_d^2. Every stencil kernel evaluates faces in flux form, so A * const = m * const
// exactly and the two cells of a face see bit-identical weights (rho_a + rho_b is commutative).
//
// Reductions are deterministic: each workgroup reduces in a fixed butterfly/tree order and
// writes one partial; the last workgroup to finish (atomic ticket) sums the partials in index
// order and applies the scalar update of the CG recurrence on the device.
#include "hp_internal.h"

#include <algorithm>
#include <cmath>

namespace hp {

// ------------------------------------------------------------------------------------------
// small helpers

__device__ __forceinline__ int flat_tid() {
    return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
}
__device__ __forceinline__ int flat_bid() {
    return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}
__device__ __forceinline__ int num_blocks() { return gridDim.x * gridDim.y * gridDim.z; }

// Reciprocal: hardware estimate refined by two Newton steps (error within a couple of ulp).
__device__ __forceinline__ double fast_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename T>
__device__ __forceinline__ T face_kappa(T ra, T rb) {
    return T(2) * fast_rcp(ra + rb);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup in a fixed order; result valid in thread 0. Every thread must call.
__device__ double block_sum(double v) {
    __shared__ double ws[kBlock / 64];
    const int tid = flat_tid();
    v = wave_sum(v);
    __syncthreads();
    if ((tid & 63) == 0) ws[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0) {
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) s += ws[w];
    }
    return s;
}

// Two-stage deterministic reduction with the last-workgroup epilogue. Every thread must call.
__device__ void red_finish(double v, const RedCtl& rc) {
    __shared__ int is_last;
    const int tid = flat_tid();
    const int nb = num_blocks();
    double s = block_sum(v);
    if (tid == 0) {
        rc.partials[flat_bid()] = s;
        __threadfence();
        unsigned t = atomicAdd(rc.counter, 1u);
        is_last = (t == (unsigned)(nb - 1));
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    double acc = 0.0;
    for (int b = tid; b < nb; b += kBlock)
        acc += __hip_atomic_load(&rc.partials[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    double tot = block_sum(acc);
    if (tid == 0) {
        double* sc = rc.scal;
        switch (rc.op) {
            case OP_STORE: sc[rc.slot] = tot; break;
            case OP_ALPHA:
                sc[S_PQ] = tot;
                if (!(tot > 0.0) || !isfinite(tot)) {
                    sc[S_FLAG] = 1.0;
                    sc[S_ALPHA] = 0.0;
                } else {
                    sc[S_ALPHA] = sc[S_RZ] / tot;
                }
                break;
            case OP_BETA:
                sc[S_BETA] = tot / sc[S_RZ];
                sc[S_RZ] = tot;
                break;
            case OP_RZINIT:
                sc[S_RZ] = tot;
                sc[S_BETA] = 0.0;
                break;
            default: break;
        }
        __hip_atomic_store(rc.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Launch shape over cells: 256-thread 3D workgroups sized to the level.
static inline int pow2_at_least(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}
struct Shape3 {
    dim3 grid, block;
};
static Shape3 cells_shape(int nx, int ny, int nz) {
    int bx = std::min(64, pow2_at_least(nx));
    int by = std::min(kBlock / bx, pow2_at_least(ny));
    int bz = kBlock / (bx * by);
    Shape3 s;
    s.block = dim3(bx, by, bz);
    s.grid = dim3((nx + bx - 1) / bx, (ny + by - 1) / by, (nz + bz - 1) / bz);
    return s;
}
int64_t reduce_blocks_cells(int nx, int ny, int nz) {
    Shape3 s = cells_shape(nx, ny, nz);
    return (int64_t)s.grid.x * s.grid.y * s.grid.z;
}
static inline int vec_blocks(int64_t n) {
    int64_t b = (n + 4 * kBlock - 1) / (4 * kBlock);
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 2048));
}
int64_t reduce_blocks_vec(int64_t n) { return vec_blocks(n); }

// ------------------------------------------------------------------------------------------
// Stencil core: visits the (up to six) faces of cell (i,j,k) at flat index a.
// F(nb) is called with the neighbour's flat index once per face.

template <typename T, typename F>
__device__ __forceinline__ void for_faces(const Geo<T>& g, int i, int j, int k, int a, F&& f) {
    const int sx = 1, sy = g.nx, sz = g.nx * g.ny;
    if (i > 0) f(a - sx, g.cx); else if (g.px) f(a + (g.nx - 1) * sx, g.cx);
    if (i < g.nx - 1) f(a + sx, g.cx); else if (g.px) f(a - (g.nx - 1) * sx, g.cx);
    if (j > 0) f(a - sy, g.cy); else if (g.py) f(a + (g.ny - 1) * sy, g.cy);
    if (j < g.ny - 1) f(a + sy, g.cy); else if (g.py) f(a - (g.ny - 1) * sy, g.cy);
    if (k > 0) f(a - sz, g.cz); else if (g.pz) f(a + (g.nz - 1) * sz, g.cz);
    if (k < g.nz - 1) f(a + sz, g.cz); else if (g.pz) f(a - (g.nz - 1) * sz, g.cz);
}

// ------------------------------------------------------------------------------------------
// coefficient setup

__global__ __launch_bounds__(kBlock) void k_setup_coef(const double* __restrict__ rho,
                                                       const double* __restrict__ c2,
                                                       double* __restrict__ rho_out,
                                                       double* __restrict__ m,
                                                       float* __restrict__ rho32,
                                                       float* __restrict__ m32, int64_t n,
                                                       int* bad) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    double r = rho[a], c = c2[a];
    bool ok = (r > 0.0) && (c > 0.0) && isfinite(r) && isfinite(c);
    if (!ok) {
        atomicOr(bad, 1);
        r = 1.0;
        c = 1.0;
    }
    double mm = 1.0 / (r * c);
    rho_out[a] = r;
    m[a] = mm;
    rho32[a] = (float)r;
    m32[a] = (float)mm;
}

void launch_setup_coef(const double* rho, const double* c2, double* rho_out, double* m,
                       float* rho32, float* m32, int64_t n, int* bad, hipStream_t s) {
    int blocks = (int)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_setup_coef, dim3(blocks), dim3(kBlock), 0, s, rho, c2, rho_out, m,
                       rho32, m32, n, bad);
}

// mean over the children of each coarse cell
__global__ __launch_bounds__(kBlock) void k_coarsen_coef(Transfer t, const double* __restrict__ rf,
                                                         const double* __restrict__ mf,
                                                         double* __restrict__ rc,
                                                         double* __restrict__ mc,
                                                         float* __restrict__ rc32,
                                                         float* __restrict__ mc32) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    int J = blockIdx.y * blockDim.y + threadIdx.y;
    int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (I >= t.ncx || J >= t.ncy || K >= t.ncz) return;
    double sr = 0.0, sm = 0.0;
    int cnt = 0;
    for (int dk = 0; dk <= t.fz; ++dk)
        for (int dj = 0; dj <= t.fy; ++dj)
            for (int di = 0; di <= t.fx; ++di) {
                int i = t.fx ? 2 * I + di : I;
                int j = t.fy ? 2 * J + dj : J;
                int k = t.fz ? 2 * K + dk : K;
                int64_t a = i + (int64_t)t.nfx * (j + (int64_t)t.nfy * k);
                sr += rf[a];
                sm += mf[a];
                ++cnt;
            }
    int64_t c = I + (int64_t)t.ncx * (J + (int64_t)t.ncy * K);
    double inv = 1.0 / cnt;
    rc[c] = sr * inv;
    mc[c] = sm * inv;
    rc32[c] = (float)(sr * inv);
    mc32[c] = (float)(sm * inv);
}

void launch_coarsen_coef(const Transfer& t, const double* rho_f, const double* m_f,
                         double* rho_c, double* m_c, float* rho32_c, float* m32_c, hipStream_t s) {
    Shape3 sh = cells_shape(t.ncx, t.ncy, t.ncz);
    hipLaunchKernelGGL(k_coarsen_coef, sh.grid, sh.block, 0, s, t, rho_f, m_f, rho_c, m_c,
                       rho32_c, m32_c);
}

__global__ __launch_bounds__(kBlock) void k_jacobi_diag(Geo<double> g, const double* __restrict__ rho,
                                                        const double* __restrict__ m,
                                                        double* __restrict__ dinv) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= g.nx || j >= g.ny || k >= g.nz) return;
    int a = i + g.nx * (j + g.ny * k);
    double ra = rho[a];
    double d = m[a];
    for_faces(g, i, j, k, a, [&](int nb, double c) { d += c * face_kappa(ra, rho[nb]); });
    dinv[a] = 1.0 / d;
}

void launch_jacobi_diag(const Geo<double>& g, const double* rho, const double* m, double* dinv,
                        hipStream_t s) {
    Shape3 sh = cells_shape(g.nx, g.ny, g.nz);
    hipLaunchKernelGGL(k_jacobi_diag, sh.grid, sh.block, 0, s, g, rho, m, dinv);
}

// ------------------------------------------------------------------------------------------
// operator apply / residual

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_apply(Geo<T> g, const T* __restrict__ rho,
                                                  const T* __restrict__ m,
                                                  const T* __restrict__ x,
                                                  const T* __restrict__ b, T* __restrict__ y,
                                                  RedCtl rc) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z * blockDim.z + threadIdx.z;
    double part = 0.0;
    if (i < g.nx && j < g.ny && k < g.nz) {
        int a = i + g.nx * (j + g.ny * k);
        T ra = rho[a], xa = x[a];
        T acc = m[a] * xa;
        for_faces(g, i, j, k, a,
                  [&](int nb, T c) { acc += c * face_kappa(ra, rho[nb]) * (xa - x[nb]); });
        if (MODE >= 2) acc = b[a] - acc;
        y[a] = acc;
        if (MODE == 1) part = (double)xa * (double)acc;
        if (MODE == 3) part = (double)acc * (double)acc;
    }
    if (MODE == 1 || MODE == 3) red_finish(part, rc);
}

template <typename T>
void launch_apply(const Geo<T>& g, const T* rho, const T* m, const T* x, const T* b, T* y,
                  int mode, const RedCtl& rc, hipStream_t s) {
    Shape3 sh = cells_shape(g.nx, g.ny, g.nz);
    switch (mode) {
        case 0: hipLaunchKernelGGL((k_apply<T, 0>), sh.grid, sh.block, 0, s, g, rho, m, x, b, y, rc); break;
        case 1: hipLaunchKernelGGL((k_apply<T, 1>), sh.grid, sh.block, 0, s, g, rho, m, x, b, y, rc); break;
        case 2: hipLaunchKernelGGL((k_apply<T, 2>), sh.grid, sh.block, 0, s, g, rho, m, x, b, y, rc); break;
        default: hipLaunchKernelGGL((k_apply<T, 3>), sh.grid, sh.block, 0, s, g, rho, m, x, b, y, rc); break;
    }
}

// ------------------------------------------------------------------------------------------
// red-black Gauss-Seidel

template <typename T>
__global__ __launch_bounds__(kBlock) void k_rbgs(Geo<T> g, const T* __restrict__ rho,
                                                 const T* __restrict__ m,
                                                 const T* __restrict__ r, T* __restrict__ z,
                                                 int colour) {
    int tx = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (j >= g.ny || k >= g.nz) return;
    int i = 2 * tx + ((colour + j + k) & 1);
    if (i >= g.nx) return;
    int a = i + g.nx * (j + g.ny * k);
    T ra = rho[a];
    T sw = T(0), swz = T(0);
    for_faces(g, i, j, k, a, [&](int nb, T c) {
        T w = c * face_kappa(ra, rho[nb]);
        sw += w;
        swz += w * z[nb];
    });
    z[a] = (r[a] + swz) / (m[a] + sw);
}

// First red half sweep from z = 0: red cells r/D, black cells 0 (writes every cell).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rbgs_zero(Geo<T> g, const T* __restrict__ rho,
                                                      const T* __restrict__ m,
                                                      const T* __restrict__ r,
                                                      T* __restrict__ z) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= g.nx || j >= g.ny || k >= g.nz) return;
    int a = i + g.nx * (j + g.ny * k);
    if ((i + j + k) & 1) {
        z[a] = T(0);
        return;
    }
    T ra = rho[a];
    T sw = T(0);
    for_faces(g, i, j, k, a, [&](int nb, T c) { sw += c * face_kappa(ra, rho[nb]); });
    z[a] = r[a] / (m[a] + sw);
}

template <typename T>
void launch_rbgs(const Geo<T>& g, const T* rho, const T* m, const T* r, T* z, int colour,
                 hipStream_t s) {
    Shape3 sh = cells_shape((g.nx + 1) / 2, g.ny, g.nz);
    hipLaunchKernelGGL((k_rbgs<T>), sh.grid, sh.block, 0, s, g, rho, m, r, z, colour);
}

template <typename T>
void launch_rbgs_zero(const Geo<T>& g, const T* rho, const T* m, const T* r, T* z,
                      hipStream_t s) {
    Shape3 sh = cells_shape(g.nx, g.ny, g.nz);
    hipLaunchKernelGGL((k_rbgs_zero<T>), sh.grid, sh.block, 0, s, g, rho, m, r, z);
}

// ------------------------------------------------------------------------------------------
// transfers

// Fine taps of coarse index I along one axis for R = P^T / 2 (P: weights 3/4 parent, 1/4 the
// second-nearest coarse cell; mirrored at a Neumann end, wrapped on a periodic axis).
__device__ __forceinline__ int restrict_taps(int I, int nf, int coarsened, int periodic,
                                             int* idx, float* w) {
    if (!coarsened) {
        idx[0] = I;
        w[0] = 1.0f;
        return 1;
    }
    const int nc = nf >> 1;
    int cnt = 0;
#pragma unroll
    for (int s = -1; s <= 2; ++s) {
        int i = 2 * I + s;
        if (i < 0 || i >= nf) {
            if (!periodic) continue;
            i = (i + nf) % nf;
        }
        int parent = i >> 1;
        int other = (i & 1) ? parent + 1 : parent - 1;
        if (other < 0 || other >= nc) other = periodic ? (other + nc) % nc : parent;
        float p = (parent == I ? 0.75f : 0.0f) + (other == I ? 0.25f : 0.0f);
        idx[cnt] = i;
        w[cnt] = 0.5f * p;
        ++cnt;
    }
    return cnt;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(Transfer t, const T* __restrict__ fine,
                                                     T* __restrict__ coarse) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    int J = blockIdx.y * blockDim.y + threadIdx.y;
    int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (I >= t.ncx || J >= t.ncy || K >= t.ncz) return;
    int ix[4], iy[4], iz[4];
    float wx[4], wy[4], wz[4];
    int nxs = restrict_taps(I, t.nfx, t.fx, t.perx, ix, wx);
    int nys = restrict_taps(J, t.nfy, t.fy, t.pery, iy, wy);
    int nzs = restrict_taps(K, t.nfz, t.fz, t.perz, iz, wz);
    T acc = T(0);
    for (int c = 0; c < nzs; ++c) {
        T accy = T(0);
        for (int b = 0; b < nys; ++b) {
            const T* row = fine + (int64_t)t.nfx * (iy[b] + (int64_t)t.nfy * iz[c]);
            T accx = T(0);
            for (int q = 0; q < nxs; ++q) accx += (T)wx[q] * row[ix[q]];
            accy += (T)wy[b] * accx;
        }
        acc += (T)wz[c] * accy;
    }
    coarse[I + (int64_t)t.ncx * (J + (int64_t)t.ncy * K)] = acc;
}

template <typename T>
void launch_restrict(const Transfer& t, const T* fine, T* coarse, hipStream_t s) {
    Shape3 sh = cells_shape(t.ncx, t.ncy, t.ncz);
    hipLaunchKernelGGL((k_restrict<T>), sh.grid, sh.block, 0, s, t, fine, coarse);
}

// Coarse taps of fine index i along one axis for P.
__device__ __forceinline__ int prolong_taps(int i, int nc, int coarsened, int periodic, int* idx,
                                            float* w) {
    if (!coarsened) {
        idx[0] = i;
        w[0] = 1.0f;
        return 1;
    }
    int parent = i >> 1;
    int other = (i & 1) ? parent + 1 : parent - 1;
    if (other < 0 || other >= nc) other = periodic ? (other + nc) % nc : parent;
    idx[0] = parent;
    w[0] = 0.75f;
    idx[1] = other;
    w[1] = 0.25f;
    return 2;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_add(Transfer t, const T* __restrict__ coarse,
                                                        T* __restrict__ fine) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= t.nfx || j >= t.nfy || k >= t.nfz) return;
    int ix[2], iy[2], iz[2];
    float wx[2], wy[2], wz[2];
    int nxs = prolong_taps(i, t.ncx, t.fx, t.perx, ix, wx);
    int nys = prolong_taps(j, t.ncy, t.fy, t.pery, iy, wy);
    int nzs = prolong_taps(k, t.ncz, t.fz, t.perz, iz, wz);
    T acc = T(0);
    for (int c = 0; c < nzs; ++c) {
        T accy = T(0);
        for (int b = 0; b < nys; ++b) {
            const T* row = coarse + (int64_t)t.ncx * (iy[b] + (int64_t)t.ncy * iz[c]);
            T accx = T(0);
            for (int q = 0; q < nxs; ++q) accx += (T)wx[q] * row[ix[q]];
            accy += (T)wy[b] * accx;
        }
        acc += (T)wz[c] * accy;
    }
    fine[i + (int64_t)t.nfx * (j + (int64_t)t.nfy * k)] += acc;
}

template <typename T>
void launch_prolong_add(const Transfer& t, const T* coarse, T* fine, hipStream_t s) {
    Shape3 sh = cells_shape(t.nfx, t.nfy, t.nfz);
    hipLaunchKernelGGL((k_prolong_add<T>), sh.grid, sh.block, 0, s, t, coarse, fine);
}

// ------------------------------------------------------------------------------------------
// coarsest solve: x = Ainv b with the symmetric FP64 inverse, one wave64 per row

template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_solve(const double* __restrict__ ainv, int nc,
                                                         const T* __restrict__ b,
                                                         T* __restrict__ x) {
    int lane = threadIdx.x & 63;
    int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    double acc = 0.0;
    if (row < nc) {
        const double* arow = ainv + (int64_t)row * nc;
        for (int c = lane; c < nc; c += 64) acc += arow[c] * (double)b[c];
    }
    acc = wave_sum(acc);
    if (row < nc && lane == 0) x[row] = (T)acc;
}

template <typename T>
void launch_coarse_solve(const double* ainv, int nc, const T* b, T* x, hipStream_t s) {
    int blocks = (nc + (kBlock / 64) - 1) / (kBlock / 64);
    hipLaunchKernelGGL((k_coarse_solve<T>), dim3(blocks), dim3(kBlock), 0, s, ainv, nc, b, x);
}

// ------------------------------------------------------------------------------------------
// vector kernels (grid-stride, fixed grid per n => deterministic)

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dot(const T* __restrict__ x, const T* __restrict__ y,
                                                int64_t n, RedCtl rc) {
    double acc = 0.0;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x; a < n; a += stride)
        acc += (double)x[a] * (double)y[a];
    red_finish(acc, rc);
}

template <typename T>
void launch_dot(const T* x, const T* y, int64_t n, const RedCtl& rc, hipStream_t s) {
    hipLaunchKernelGGL((k_dot<T>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, x, y, n, rc);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpy2_norm(T* __restrict__ x, const T* __restrict__ p,
                                                       T* __restrict__ r,
                                                       const T* __restrict__ q, int64_t n,
                                                       RedCtl rc) {
    const T alpha = (T)rc.scal[S_ALPHA];
    double acc = 0.0;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x; a < n; a += stride) {
        x[a] += alpha * p[a];
        T ra = r[a] - alpha * q[a];
        r[a] = ra;
        acc += (double)ra * (double)ra;
    }
    red_finish(acc, rc);
}

template <typename T>
void launch_axpy2_norm(T* x, const T* p, T* r, const T* q, int64_t n, const RedCtl& rc,
                       hipStream_t s) {
    hipLaunchKernelGGL((k_axpy2_norm<T>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, x, p, r, q, n,
                       rc);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_xpby(const T* __restrict__ z, T* __restrict__ p,
                                                 int64_t n, const double* __restrict__ scal) {
    const T beta = (T)scal[S_BETA];
    int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (a < n) p[a] = z[a] + beta * p[a];
}

template <typename T>
void launch_xpby(const T* z, T* p, int64_t n, const double* scal, hipStream_t s) {
    hipLaunchKernelGGL((k_xpby<T>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, z, p, n, scal);
}

__global__ __launch_bounds__(kBlock) void k_jacobi_apply(const double* __restrict__ dinv,
                                                         const double* __restrict__ r,
                                                         double* __restrict__ z, int64_t n,
                                                         RedCtl rc) {
    double acc = 0.0;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x; a < n; a += stride) {
        double za = dinv[a] * r[a];
        z[a] = za;
        acc += r[a] * za;
    }
    red_finish(acc, rc);
}

void launch_jacobi_apply(const double* dinv, const double* r, double* z, int64_t n,
                         const RedCtl& rc, hipStream_t s) {
    hipLaunchKernelGGL(k_jacobi_apply, dim3(vec_blocks(n)), dim3(kBlock), 0, s, dinv, r, z, n, rc);
}

__global__ __launch_bounds__(kBlock) void k_cast_scale_f32(const double* __restrict__ src,
                                                           float* __restrict__ dst, double scale,
                                                           int64_t n) {
    int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (a < n) dst[a] = (float)(src[a] * scale);
}

void launch_cast_scale_f32(const double* src, float* dst, double scale, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_cast_scale_f32, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, src, dst, scale, n);
}

__global__ __launch_bounds__(kBlock) void k_axpy_from_f32(double* __restrict__ x,
                                                          const float* __restrict__ d,
                                                          double scale, int64_t n) {
    int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (a < n) x[a] += scale * (double)d[a];
}

void launch_axpy_from_f32(double* x, const float* d, double scale, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy_from_f32, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, x, d, scale, n);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T* __restrict__ x, T v, int64_t n) {
    int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (a < n) x[a] = v;
}

template <typename T>
void launch_fill(T* x, T v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_fill<T>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, x, v, n);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(const T* __restrict__ src, T* __restrict__ dst,
                                                 int64_t n) {
    int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (a < n) dst[a] = src[a];
}

template <typename T>
void launch_copy(const T* src, T* dst, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_copy<T>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, src, dst, n);
}

__global__ __launch_bounds__(kBlock) void k_check_finite(const double* __restrict__ x, int64_t n,
                                                         int* bad) {
    int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (a < n && !isfinite(x[a])) atomicOr(bad, 1);
}

void launch_check_finite(const double* x, int64_t n, int* bad, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, x, n, bad);
}

// ------------------------------------------------------------------------------------------
// explicit instantiations

#define HP_INST(T)                                                                              \
    template void launch_apply<T>(const Geo<T>&, const T*, const T*, const T*, const T*, T*,    \
                                  int, const RedCtl&, hipStream_t);                            \
    template void launch_rbgs<T>(const Geo<T>&, const T*, const T*, const T*, T*, int,          \
                                 hipStream_t);                                                  \
    template void launch_rbgs_zero<T>(const Geo<T>&, const T*, const T*, const T*, T*,          \
                                      hipStream_t);                                             \
    template void launch_restrict<T>(const Transfer&, const T*, T*, hipStream_t);               \
    template void launch_prolong_add<T>(const Transfer&, const T*, T*, hipStream_t);            \
    template void launch_coarse_solve<T>(const double*, int, const T*, T*, hipStream_t);        \
    template void launch_dot<T>(const T*, const T*, int64_t, const RedCtl&, hipStream_t);       \
    template void launch_axpy2_norm<T>(T*, const T*, T*, const T*, int64_t, const RedCtl&,      \
                                       hipStream_t);                                            \
    template void launch_xpby<T>(const T*, T*, int64_t, const double*, hipStream_t);            \
    template void launch_fill<T>(T*, T, int64_t, hipStream_t);                                  \
    template void launch_copy<T>(const T*, T*, int64_t, hipStream_t);

HP_INST(double)
HP_INST(float)

}  // namespace hp
