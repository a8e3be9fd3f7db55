// hp_kernels.hip -- gfx950 kernels of the pressure solve (FP64 and FP32 instantiations).
//
// Operator (paper, Section 2, eq. Poiss times dt^2, coefficients eqs. cpoiss/kappapoiss, face
// factor of step (viii)): (A p)_a = m_a p_a + sum_f w_f (p_a - p_b), w_f = c_d * 2/(rho_a+rho_b),
// c_d = dt^2 / h_d^2. Every stencil kernel evaluates faces in flux form, so A * const = m * const
// exactly and the two cells of a face see bit-identical weights (rho_a + rho_b is commutative).
//
// Reductions are deterministic: each workgroup reduces in a fixed butterfly/tree order and
// writes one partial; a one-workgroup kernel then sums the partials in index order and applies
// the scalar update of the CG recurrence on the device (no atomics, so no serialisation of
// thousands of workgroups on one address).
//
// Large levels use z-marching kernels: a workgroup owns a 64-wide (apply) or 128-wide
// (red-black, two cells per thread) by 4-row column tile and walks a chunk of z planes, keeping
// the z neighbours of the current plane in registers so every array is streamed once. Tiles are
// numbered so that each of the 8 XCDs (which receive workgroups round-robin) works on one
// contiguous range of z chunks, keeping y halos in its own L2.
#include <initializer_list>
#include <type_traits>

#include "hp_internal.h"

#include <hip/hip_ext.h>

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

// kappa = 1/rho at the face between cells of face densities ra and rb. FR = 0 (the default): the
// factor 2 / (ra + rb) of the face-velocity update (step (viii)); FR = 1: the mean of the two
// cells' kappa, (1/ra + 1/rb) / 2.
template <int FR, typename T>
__device__ __forceinline__ T face_kappa(T ra, T rb) {
    if constexpr (FR == 1) return T(0.5) * (fast_rcp(ra) + fast_rcp(rb));
    return T(2) * fast_rcp(ra + rb);
}

// the face rule of a launch as the compile-time constant FRV of the statement it runs
#define WITH_FACE_RULE(rule, ...)      \
    do {                               \
        if (rule) {                    \
            constexpr int FRV = 1;     \
            __VA_ARGS__;               \
        } else {                       \
            constexpr int FRV = 0;     \
            __VA_ARGS__;               \
        }                              \
    } while (0)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup in a fixed order; result valid in thread 0. Every thread must call.
__device__ double block_sum(double v) {
    __shared__ double ws[16];
    const int tid = flat_tid();
    const int nw = (blockDim.x * blockDim.y * blockDim.z) >> 6;
    v = wave_sum(v);
    __syncthreads();
    if ((tid & 63) == 0) ws[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0)
        for (int w = 0; w < nw; ++w) s += ws[w];
    return s;
}

// First stage of a deterministic reduction: the workgroup total goes to partials[workgroup].
// Every thread must call. The second stage is k_finalize (one workgroup, fixed order).
__device__ void block_partial(double v, double* partials) {
    double s = block_sum(v);
    if (flat_tid() == 0) partials[flat_bid()] = s;
}

// The host reads the residual-norm partials of the CG residual update and the breakdown flag as
// they stand when that kernel runs; with rc.partials and rc.flag_out in mapped pinned host memory
// the kernel delivers both itself (no copy launch behind it): workgroup 0 copies the flag.
__device__ __forceinline__ void export_flag(const RedCtl& rc) {
    if (rc.flag_out && flat_bid() == 0 && flat_tid() == 0) rc.flag_out[0] = rc.scal[S_FLAG];
}

__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict__ partials, int nb,
                                                     const double* __restrict__ partials2, int nb2,
                                                     double* __restrict__ sc, int op, int slot) {
    const int tid = threadIdx.x;
    // the scalar the op combines with, and the first kU partials of each list, are loaded before
    // anything is summed (one memory round trip instead of one per partial); the sum order is
    // that of the plain strided loop
    constexpr int kU = 4;
    const double rz = sc[S_RZ];
    // (clamped indices: the loads are unconditional; partials2 may be absent, nb is at least 1)
    const double* q2 = nb2 > 0 ? partials2 : partials;
    const int l1 = max(nb, 1) - 1, l2 = nb2 > 0 ? nb2 - 1 : l1;
    double v[2][kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int b = tid + u * kBlock;
        v[0][u] = partials[min(b, l1)];
        v[1][u] = q2[min(b, l2)];
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kU; ++u)
        if (tid + u * kBlock < nb) acc += v[0][u];
    for (int b = tid + kU * kBlock; b < nb; b += kBlock) acc += partials[b];
#pragma unroll
    for (int u = 0; u < kU; ++u)
        if (tid + u * kBlock < nb2) acc += v[1][u];
    for (int b = tid + kU * kBlock; b < nb2; b += kBlock) acc += partials2[b];
    double tot = block_sum(acc);
    if (tid != 0) return;
    switch (op) {
        case OP_STORE: sc[slot] = tot; break;
        case OP_ALPHA:
            sc[S_PQ] = tot;
            if (!(tot > 0.0) || !isfinite(tot)) {
                sc[S_FLAG] = 1.0;
                sc[S_ALPHA] = 0.0;
            } else {
                sc[S_ALPHA] = rz / tot;
            }
            break;
        case OP_BETA:
            sc[S_BETA] = tot / rz;
            sc[S_RZ] = tot;
            break;
        case OP_RZINIT:
            sc[S_RZ] = tot;
            sc[S_BETA] = 0.0;
            break;
        default: break;
    }
}

// second stage over nb partials (and, for a reduction split over two launches, nb2 more)
static void finalize(const RedCtl& rc, int nb, hipStream_t s, const double* partials2 = nullptr, int nb2 = 0) {
    if (rc.op == OP_NONE) return;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, rc.partials, nb, partials2, nb2, rc.scal,
                       rc.op, rc.slot);
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
struct ZTiles;
static int64_t zm_blocks(int nx, int ny, int nz);
int64_t reduce_blocks_cells(int nx, int ny, int nz) {
    Shape3 s = cells_shape(nx, ny, nz);
    return std::max<int64_t>((int64_t)s.grid.x * s.grid.y * s.grid.z, zm_blocks(nx, ny, nz));
}
static inline int vec_blocks(int64_t n) {
    int64_t b = (n + 4 * kBlock - 1) / (4 * kBlock);
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 2048));
}
int64_t reduce_blocks_vec(int64_t n) { return vec_blocks(n); }

// ------------------------------------------------------------------------------------------
// Stencil core: visits the six faces of cell (i,j,k) at flat index a in the order x-, x+, y-, y+,
// z-, z+. F(nb, c) is called once per face with the neighbour's flat index and the face factor; a
// face that does not exist (the end of a Neumann axis) gets factor 0 and the cell itself as a
// stand-in neighbour. No call is conditional, so every neighbour load can be in flight at once
// (with a branch per face each load waited for the one before it).

template <typename T, typename F>
__device__ __forceinline__ void for_faces(const Geo<T>& g, int i, int j, int k, int a, F&& f) {
    const int sy = g.nx, sz = g.nx * g.ny;
    const int oxm = i > 0 ? -1 : (g.px ? g.nx - 1 : 0);
    const int oxp = i < g.nx - 1 ? 1 : (g.px ? -(g.nx - 1) : 0);
    const int oym = j > 0 ? -sy : (g.py ? (g.ny - 1) * sy : 0);
    const int oyp = j < g.ny - 1 ? sy : (g.py ? -(g.ny - 1) * sy : 0);
    const int ozm = k > 0 ? -sz : (g.pz ? (g.nz - 1) * sz : 0);
    const int ozp = k < g.nz - 1 ? sz : (g.pz ? -(g.nz - 1) * sz : 0);
    f(a + oxm, (i > 0 || g.px) ? g.cx : T(0));
    f(a + oxp, (i < g.nx - 1 || g.px) ? g.cx : T(0));
    f(a + oym, (j > 0 || g.py) ? g.cy : T(0));
    f(a + oyp, (j < g.ny - 1 || g.py) ? g.cy : T(0));
    f(a + ozm, (k > 0 || g.pz) ? g.cz : T(0));
    f(a + ozp, (k < g.nz - 1 || g.pz) ? g.cz : T(0));
}

// ------------------------------------------------------------------------------------------
// coefficient setup

// position of cell (i, j, k) in the red-black split order: colour c = (i + j + k) & 1 at half
// position c nx/2 + i/2 of its row
__device__ __forceinline__ int split_index(int i, int j, int k, int nx, int ny) {
    return (j + ny * k) * nx + (((i + j + k) & 1) ? (nx >> 1) : 0) + (i >> 1);
}

// m = 1 / (rho_mass c2) (the mass term with the density of time level n) and the face density
// rho_face (time level n+1; the same array as rho_mass in the one-density form), with the
// Lax-Milgram check that all three are positive and finite. rho_out and m in natural order; with
// split32 (nx even) the FP32 copies go to split order, and so do FP64 copies into rho_split and
// m_split where those are given.
__global__ __launch_bounds__(kBlock) void k_setup_coef(const double* __restrict__ rho_mass,
                                                       const double* __restrict__ rho_face,
                                                       const double* __restrict__ c2,
                                                       double* __restrict__ rho_out,
                                                       double* __restrict__ m,
                                                       double* __restrict__ rho_split,
                                                       double* __restrict__ m_split,
                                                       float* __restrict__ rho32,
                                                       float* __restrict__ m32, int64_t n, int nx,
                                                       int ny, int split32, int* bad) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    double rm = rho_mass[a], rf = rho_face[a], c = c2[a];
    bool ok = (rm > 0.0) && (rf > 0.0) && (c > 0.0) && isfinite(rm) && isfinite(rf) && isfinite(c);
    if (!ok) {
        atomicOr(bad, 1);
        rm = 1.0;
        rf = 1.0;
        c = 1.0;
    }
    double mm = 1.0 / (rm * c);
    rho_out[a] = rf;
    m[a] = mm;
    int64_t a32 = a;
    if (split32) {
        const int64_t row = a / nx;
        a32 = split_index((int)(a - row * nx), (int)(row % ny), (int)(row / ny), nx, ny);
        if (rho_split) {
            rho_split[a32] = rf;
            m_split[a32] = mm;
        }
    }
    rho32[a32] = (float)rf;
    m32[a32] = (float)mm;
}

void launch_setup_coef(const double* rho_mass, const double* rho_face, const double* c2, double* rho_out,
                       double* m, double* rho_split, double* m_split, float* rho32, float* m32, int nx,
                       int ny, int nz, bool split32, int* bad, hipStream_t s) {
    const int64_t n = (int64_t)nx * ny * nz;
    int blocks = (int)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_setup_coef, dim3(blocks), dim3(kBlock), 0, s, rho_mass, rho_face, c2, rho_out, m,
                       rho_split, m_split, rho32, m32, n, nx, ny, split32 ? 1 : 0, bad);
}

// Inhomogeneous Neumann data on boundary `side` of axis d: b_a += coef q_f for the cell a next to
// each boundary face f, q the prescribed outward normal flux (coef = dt^2 / h_d). One thread per
// face; q is indexed over the plane of the other two axes, lower axis fastest. Natural layout.
__global__ __launch_bounds__(kBlock) void k_neumann_rhs(int nx, int ny, int nz, int d, int side, double coef,
                                                        const double* __restrict__ q,
                                                        double* __restrict__ b) {
    const int n[3] = {nx, ny, nz};
    const int e0 = d == 0 ? 1 : 0, e1 = d == 2 ? 1 : 2;
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= (int64_t)n[e0] * n[e1]) return;
    int c[3];
    c[d] = side ? n[d] - 1 : 0;
    c[e0] = (int)(f % n[e0]);
    c[e1] = (int)(f / n[e0]);
    const int64_t a = c[0] + (int64_t)nx * (c[1] + (int64_t)ny * c[2]);
    b[a] += coef * q[f];
}

void launch_neumann_rhs(int nx, int ny, int nz, int d, int side, double coef, const double* q, double* b,
                        hipStream_t s) {
    const int n[3] = {nx, ny, nz};
    const int64_t nf = (int64_t)n[d == 0 ? 1 : 0] * n[d == 2 ? 1 : 2];
    hipLaunchKernelGGL(k_neumann_rhs, dim3((unsigned)((nf + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       nx, ny, nz, d, side, coef, q, b);
}

// mean over the children of each coarse cell (natural order; the FP32 copies in split order with
// split32)
__global__ __launch_bounds__(kBlock) void k_coarsen_coef(Transfer t, const double* __restrict__ rf,
                                                         const double* __restrict__ mf,
                                                         double* __restrict__ rc,
                                                         double* __restrict__ mc,
                                                         float* __restrict__ rc32,
                                                         float* __restrict__ mc32, int split32) {
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
    const int64_t c32 = split32 ? split_index(I, J, K, t.ncx, t.ncy) : c;
    rc32[c32] = (float)(sr * inv);
    mc32[c32] = (float)(sm * inv);
}

void launch_coarsen_coef(const Transfer& t, const double* rho_f, const double* m_f,
                         double* rho_c, double* m_c, float* rho32_c, float* m32_c, bool split32,
                         hipStream_t s) {
    Shape3 sh = cells_shape(t.ncx, t.ncy, t.ncz);
    hipLaunchKernelGGL(k_coarsen_coef, sh.grid, sh.block, 0, s, t, rho_f, m_f, rho_c, m_c,
                       rho32_c, m32_c, split32 ? 1 : 0);
}

// inverse diagonal 1 / (m_a + sum_f w_f) in FP64, and its FP32 counterpart computed from the
// FP32 coefficient copies (so each precision's smoother uses its own operator's diagonal); the
// inputs are in natural order, the outputs in natural or (split) in split order
__global__ __launch_bounds__(kBlock) void k_jacobi_diag(Geo<double> g, Geo<float> g32,
                                                        const double* __restrict__ rho,
                                                        const double* __restrict__ m,
                                                        const float* __restrict__ rho32,
                                                        const float* __restrict__ m32,
                                                        double* __restrict__ dinv,
                                                        float* __restrict__ dinv32, int split) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= g.nx || j >= g.ny || k >= g.nz) return;
    int a = i + g.nx * (j + g.ny * k);
    const double ra = rho[a], ma = m[a];
    double d = ma;
    double rn[6];  // the face neighbours' rho, in the order of for_faces
    int f = 0;
    for_faces(g, i, j, k, a, [&](int nb, double c) {
        const double rb = rho[nb];
        rn[f++] = rb;
        d += c * (g.frule ? face_kappa<1>(ra, rb) : face_kappa<0>(ra, rb));
    });
    const int ao = split ? split_index(i, j, k, g.nx, g.ny) : a;
    dinv[ao] = 1.0 / d;
    if (dinv32) {
        // the FP32 copies are the FP64 values rounded to nearest, so the FP32 diagonal takes
        // them from the FP64 loads (rho32 and m32 are not read again)
        const float ra32 = (float)ra;
        float d32 = (float)ma;
        f = 0;
        for_faces(g32, i, j, k, a, [&](int nb, float c) {
            const float rb32 = (float)rn[f++];
            d32 += c * (g32.frule ? face_kappa<1>(ra32, rb32) : face_kappa<0>(ra32, rb32));
        });
        dinv32[ao] = 1.0f / d32;
    }
}

// ------------------------------------------------------------------------------------------
// operator apply / residual

template <typename T, int MODE, int FR = 0>
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
                  [&](int nb, T c) { acc += c * face_kappa<FR>(ra, rho[nb]) * (xa - x[nb]); });
        if (MODE >= 2) acc = b[a] - acc;
        y[a] = acc;
        if (MODE == 1) part = (double)xa * (double)acc;
        if (MODE == 3) part = (double)acc * (double)acc;
    }
    if (MODE == 1 || MODE == 3) block_partial(part, rc.partials);
}

// ---- z-marching operator apply (large levels) ----

struct ZTiles {
    int tx, ty, tz;  // tiles along x, y and z chunks
    int kz;          // planes per z chunk
    int rev = 0;     // tiles in reverse order
};

// Tile of this workgroup, XCD-contiguous: hardware dispatches workgroup L to XCD L % 8. In
// reverse order the workgroups dispatched first take the tiles that the forward order reaches
// last, so a pass over the finest grid that follows a forward pass over the same arrays starts
// on the data still held by the memory-side cache; consecutive finest-level passes alternate.
__device__ __forceinline__ void ztile(const ZTiles& t, int& bx, int& by, int& bz) {
    unsigned total = (unsigned)t.tx * t.ty * t.tz;
    unsigned L = blockIdx.x;
    if ((total & 7u) == 0) L = (L & 7u) * (total >> 3) + (L >> 3);
    if (t.rev) L = total - 1u - L;
    bx = (int)(L % (unsigned)t.tx);
    by = (int)((L / (unsigned)t.tx) % (unsigned)t.ty);
    bz = (int)(L / ((unsigned)t.tx * t.ty));
}

// Workgroups of `rows` waves, one x row of xw columns per wave; z chunks of at least kmin planes
// (4: chunks of 2 or 8 planes were measured slower at 256^3).
constexpr int kZMin = 4;
static ZTiles ztiles(int nx, int ny, int nz, int xw, int kmin = kZMin, int rows = 4) {
    ZTiles t;
    t.tx = (nx + xw - 1) / xw;
    t.ty = (ny + rows - 1) / rows;
    int cols = t.tx * t.ty;
    t.kz = nz;
    // aim for >= 8192 waves (32 per CU) with chunks of at least kmin planes
    const int target = 8192 / rows;
    while (t.kz > kmin && (int64_t)cols * ((nz + t.kz - 1) / t.kz) < target) t.kz = (t.kz + 1) / 2;
    t.tz = (nz + t.kz - 1) / t.kz;
    return t;
}

// In-plane neighbour offsets of column (i, j): offset and presence of the x-, x+, y-, y+ faces.
template <typename T>
struct PlaneNb {
    int oxm, oxp, oym, oyp;
    bool hxm, hxp, hym, hyp;
    __device__ __forceinline__ PlaneNb(const Geo<T>& g, int i, int j) {
        hxm = (i > 0) || g.px;
        oxm = (i > 0) ? -1 : (g.nx - 1);
        hxp = (i < g.nx - 1) || g.px;
        oxp = (i < g.nx - 1) ? 1 : -(g.nx - 1);
        hym = (j > 0) || g.py;
        oym = (j > 0) ? -g.nx : (g.ny - 1) * g.nx;
        hyp = (j < g.ny - 1) || g.py;
        oyp = (j < g.ny - 1) ? g.nx : -(g.ny - 1) * g.nx;
    }
};

// plane index of the z neighbour of plane k in direction s; -1 if there is no face
__device__ __forceinline__ int zplane(int k, int s, int nz, int pz) {
    int t = k + s;
    if (t >= 0 && t < nz) return t;
    if (!pz) return -1;
    return t < 0 ? t + nz : t - nz;
}

// Branch-free face table of one column: offsets of the four in-plane neighbours (0, i.e. the
// cell itself, where the face is absent) and their dt^2/h^2 factors (0 where absent). An absent
// face then contributes c * kappa * (x_a - x_a) = 0 exactly and nothing to the diagonal.
template <typename T>
struct FaceTab {
    int o[4];
    T c[4];
    __device__ __forceinline__ FaceTab(const Geo<T>& g, int i, int j) {
        const PlaneNb<T> nb(g, i, j);
        o[0] = nb.hxm ? nb.oxm : 0; c[0] = nb.hxm ? g.cx : T(0);
        o[1] = nb.hxp ? nb.oxp : 0; c[1] = nb.hxp ? g.cx : T(0);
        o[2] = nb.hym ? nb.oym : 0; c[2] = nb.hym ? g.cy : T(0);
        o[3] = nb.hyp ? nb.oyp : 0; c[3] = nb.hyp ? g.cy : T(0);
    }
};

// offset (in cells) from plane k to its z neighbour in direction s, and whether the face exists
__device__ __forceinline__ int zoff(int k, int s, int nz, int pz, int sz, bool& has) {
    int t = k + s;
    has = true;
    if (t >= 0 && t < nz) return s * sz;
    if (!pz) {
        has = false;
        return 0;
    }
    return (t < 0 ? t + nz : t - nz) * sz - k * sz;
}

// Software-pipelined z march: all loads of plane k+1 are issued before plane k is computed
// (unconditionally, with clamped addresses), so each wave keeps two planes of loads in flight.
template <typename T, int MODE, int FR = 0>
__global__ __launch_bounds__(kBlock) void k_apply_zm(Geo<T> g, ZTiles zt,
                                                     const T* __restrict__ rho,
                                                     const T* __restrict__ m,
                                                     const T* __restrict__ x,
                                                     const T* __restrict__ b, T* __restrict__ y,
                                                     double* __restrict__ partials) {
    int bx, by, bz;
    ztile(zt, bx, by, bz);
    const int i = bx * 64 + (threadIdx.x & 63);
    const int j = by * 4 + (threadIdx.x >> 6);
    const int k0 = bz * zt.kz;
    const int k1 = min(k0 + zt.kz, g.nz);
    const int sz = g.nx * g.ny;
    double part = 0.0;
    if (i < g.nx && j < g.ny) {
        const FaceTab<T> ft(g, i, j);
        const int col = i + g.nx * j;
        // plane k0: centre, below, above
        int a = col + k0 * sz;
        bool hm, hp;
        int om = zoff(k0, -1, g.nz, g.pz, sz, hm);
        int op = zoff(k0, 1, g.nz, g.pz, sz, hp);
        T xc = x[a], rc = rho[a];
        T xm = x[a + om];
        T wzm = hm ? g.cz * face_kappa<FR>(rc, rho[a + om]) : T(0);
        T xn = x[a + op], rn = rho[a + op];
        T czp = hp ? g.cz : T(0);
        T xv[4], rv[4], mv, bv = T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            xv[q] = x[a + ft.o[q]];
            rv[q] = rho[a + ft.o[q]];
        }
        mv = m[a];
        if (MODE >= 2) bv = b[a];
        for (int k = k0; k < k1; ++k) {
            // prefetch plane k+1 (clamped to the chunk) and the column two planes up
            const int kn = min(k + 1, k1 - 1);
            const int an = col + kn * sz;
            bool hpn;
            const int opn = zoff(kn, 1, g.nz, g.pz, sz, hpn);
            T xvn[4], rvn[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                xvn[q] = x[an + ft.o[q]];
                rvn[q] = rho[an + ft.o[q]];
            }
            const T mvn = m[an];
            const T bvn = (MODE >= 2) ? b[an] : T(0);
            const T xnn = x[an + opn], rnn = rho[an + opn];
            // plane k
            T acc = mv * xc;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc += ft.c[q] * face_kappa<FR>(rc, rv[q]) * (xc - xv[q]);
            acc += wzm * (xc - xm);
            const T wzp = czp * face_kappa<FR>(rc, rn);
            acc += wzp * (xc - xn);
            if (MODE >= 2) acc = bv - acc;
            y[a] = acc;
            if (MODE == 1) part += (double)xc * (double)acc;
            if (MODE == 3) part += (double)acc * (double)acc;
            // advance: the z+ face of plane k is the z- face of plane k+1
            wzm = wzp;
            xm = xc;
            xc = xn;
            rc = rn;
            xn = xnn;
            rn = rnn;
            czp = hpn ? g.cz : T(0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                xv[q] = xvn[q];
                rv[q] = rvn[q];
            }
            mv = mvn;
            bv = bvn;
            a = an;
        }
    }
    if (MODE == 1 || MODE == 3) block_partial(part, partials);
}

// Inverse diagonals of the large levels by a z march: the same values as k_jacobi_diag (faces
// summed in the same order from the same operands), with each rho plane of a column loaded once
// per chunk and the loads of plane k+1 in flight while plane k is computed (one thread per cell
// reads the two z-neighbour planes again, from other workgroups' tiles). Natural-order inputs;
// SPLIT writes the outputs in split order (a wave's 64 cells of a row go to two runs of 32).
template <int FR, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_jacobi_diag_zm(Geo<double> g, Geo<float> g32, ZTiles zt,
                                                           const double* __restrict__ rho,
                                                           const double* __restrict__ m,
                                                           double* __restrict__ dinv,
                                                           float* __restrict__ dinv32) {
    int bx, by, bz;
    ztile(zt, bx, by, bz);
    const int i = bx * 64 + (threadIdx.x & 63);
    const int j = by * 4 + (threadIdx.x >> 6);
    const int k0 = bz * zt.kz;
    const int k1 = min(k0 + zt.kz, g.nz);
    const int sz = g.nx * g.ny;
    if (i >= g.nx || j >= g.ny) return;
    const FaceTab<double> ft(g, i, j);
    const FaceTab<float> ft32(g32, i, j);
    const int col = i + g.nx * j;
    int a = col + k0 * sz;
    bool hm, hp;
    const int om = zoff(k0, -1, g.nz, g.pz, sz, hm);
    const int op = zoff(k0, 1, g.nz, g.pz, sz, hp);
    // rho of the cell and of its z neighbours (the cell itself where a face is absent, with
    // factor 0, as in for_faces)
    double rc = rho[a], rm = rho[a + om], rn = rho[a + op], mv = m[a];
    double czm = hm ? g.cz : 0.0, czp = hp ? g.cz : 0.0;
    float czm32 = hm ? g32.cz : 0.0f, czp32 = hp ? g32.cz : 0.0f;
    double rv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) rv[q] = rho[a + ft.o[q]];
    for (int k = k0; k < k1; ++k) {
        // plane k+1 (clamped to the chunk) and the column above it
        const int kn = min(k + 1, k1 - 1);
        const int an = col + kn * sz;
        bool hpn;
        const int opn = zoff(kn, 1, g.nz, g.pz, sz, hpn);
        double rvn[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) rvn[q] = rho[an + ft.o[q]];
        const double mvn = m[an];
        const double rnn = rho[an + opn];
        // plane k: faces x-, x+, y-, y+, z-, z+
        double d = mv;
#pragma unroll
        for (int q = 0; q < 4; ++q) d += ft.c[q] * face_kappa<FR>(rc, rv[q]);
        d += czm * face_kappa<FR>(rc, rm);
        d += czp * face_kappa<FR>(rc, rn);
        const int ao = SPLIT ? split_index(i, j, k, g.nx, g.ny) : a;
        dinv[ao] = 1.0 / d;
        if (dinv32) {
            // the FP32 copies are the FP64 values rounded to nearest
            const float rc32 = (float)rc;
            float d32 = (float)mv;
#pragma unroll
            for (int q = 0; q < 4; ++q) d32 += ft32.c[q] * face_kappa<FR>(rc32, (float)rv[q]);
            d32 += czm32 * face_kappa<FR>(rc32, (float)rm);
            d32 += czp32 * face_kappa<FR>(rc32, (float)rn);
            dinv32[ao] = 1.0f / d32;
        }
        // advance: the z+ face of plane k is the z- face of plane k+1
        rm = rc;
        rc = rn;
        rn = rnn;
        mv = mvn;
        czm = czp;
        czm32 = czp32;
        czp = hpn ? g.cz : 0.0;
        czp32 = hpn ? g32.cz : 0.0f;
#pragma unroll
        for (int q = 0; q < 4; ++q) rv[q] = rvn[q];
        a = an;
    }
}

// Cell pairs (i0, i0 + 1), i0 even, loaded and stored as one 2-vector; needs nx even and
// 2-vector-aligned arrays.
template <typename T>
struct Pair {
    T v0, v1;
};
template <typename T>
__device__ __forceinline__ Pair<T> ldp(const T* __restrict__ p) {
    using V = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
    const V v = *reinterpret_cast<const V*>(p);
    return {(T)v.x, (T)v.y};
}
template <typename T>
__device__ __forceinline__ void stp(T* __restrict__ p, T v0, T v1) {
    using V = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
    V v;
    v.x = v0;
    v.y = v1;
    *reinterpret_cast<V*>(p) = v;
}

// Operator apply over cell pairs: the same z march and face order as k_apply_zm, with half the
// memory instructions (pair loads for the cell, its y and z neighbours, m and b; two scalar
// loads for the outer x neighbours) and the pair's shared x face weighted once.
template <typename T, int MODE, int FR = 0>
__global__ __launch_bounds__(kBlock) void k_apply_zp(Geo<T> g, ZTiles zt,
                                                     const T* __restrict__ rho,
                                                     const T* __restrict__ m,
                                                     const T* __restrict__ x,
                                                     const T* __restrict__ b, T* __restrict__ y,
                                                     double* __restrict__ partials) {
    int bx, by, bz;
    ztile(zt, bx, by, bz);
    const int i0 = (bx * 64 + (threadIdx.x & 63)) * 2;
    const int j = by * 4 + (threadIdx.x >> 6);
    const int k0 = bz * zt.kz;
    const int k1 = min(k0 + zt.kz, g.nz);
    const int sz = g.nx * g.ny;
    double part = 0.0;
    if (i0 < g.nx && j < g.ny) {
        const FaceTab<T> f0(g, i0, j), f1(g, i0 + 1, j);
        const int oxl = f0.o[0], oxr = 1 + f1.o[1];   // outer x neighbours, from the pair base
        const T cxl = f0.c[0], cxr = f1.c[1];
        const int oym = f0.o[2], oyp = f0.o[3];
        const T cym = f0.c[2], cyp = f0.c[3];
        const int col = i0 + g.nx * j;
        int a = col + k0 * sz;
        bool hm, hp;
        const int om = zoff(k0, -1, g.nz, g.pz, sz, hm);
        const int op = zoff(k0, 1, g.nz, g.pz, sz, hp);
        Pair<T> xc = ldp(x + a), rc = ldp(rho + a);
        const Pair<T> xm0 = ldp(x + a + om), rm0 = ldp(rho + a + om);
        Pair<T> xm = xm0;
        T wzm0 = hm ? g.cz * face_kappa<FR>(rc.v0, rm0.v0) : T(0);
        T wzm1 = hm ? g.cz * face_kappa<FR>(rc.v1, rm0.v1) : T(0);
        Pair<T> xn = ldp(x + a + op), rn = ldp(rho + a + op);
        T czp = hp ? g.cz : T(0);
        T xl = x[a + oxl], xr = x[a + oxr], rl = rho[a + oxl], rr = rho[a + oxr];
        Pair<T> xym = ldp(x + a + oym), xyp = ldp(x + a + oyp);
        Pair<T> rym = ldp(rho + a + oym), ryp = ldp(rho + a + oyp);
        Pair<T> mv = ldp(m + a);
        Pair<T> bv = {T(0), T(0)};
        if (MODE >= 2) bv = ldp(b + a);
        for (int k = k0; k < k1; ++k) {
            // prefetch plane k+1 (clamped to the chunk) and the pair two planes up
            const int kn = min(k + 1, k1 - 1);
            const int an = col + kn * sz;
            bool hpn;
            const int opn = zoff(kn, 1, g.nz, g.pz, sz, hpn);
            const T xln = x[an + oxl], xrn = x[an + oxr], rln = rho[an + oxl], rrn = rho[an + oxr];
            const Pair<T> xymn = ldp(x + an + oym), xypn = ldp(x + an + oyp);
            const Pair<T> rymn = ldp(rho + an + oym), rypn = ldp(rho + an + oyp);
            const Pair<T> mvn = ldp(m + an);
            Pair<T> bvn = {T(0), T(0)};
            if (MODE >= 2) bvn = ldp(b + an);
            const Pair<T> xnn = ldp(x + an + opn), rnn = ldp(rho + an + opn);
            // plane k
            const T wx = g.cx * face_kappa<FR>(rc.v0, rc.v1);
            const T wzp0 = czp * face_kappa<FR>(rc.v0, rn.v0);
            const T wzp1 = czp * face_kappa<FR>(rc.v1, rn.v1);
            T acc0 = mv.v0 * xc.v0;
            acc0 += cxl * face_kappa<FR>(rc.v0, rl) * (xc.v0 - xl);
            acc0 += wx * (xc.v0 - xc.v1);
            acc0 += cym * face_kappa<FR>(rc.v0, rym.v0) * (xc.v0 - xym.v0);
            acc0 += cyp * face_kappa<FR>(rc.v0, ryp.v0) * (xc.v0 - xyp.v0);
            acc0 += wzm0 * (xc.v0 - xm.v0);
            acc0 += wzp0 * (xc.v0 - xn.v0);
            T acc1 = mv.v1 * xc.v1;
            acc1 += wx * (xc.v1 - xc.v0);
            acc1 += cxr * face_kappa<FR>(rc.v1, rr) * (xc.v1 - xr);
            acc1 += cym * face_kappa<FR>(rc.v1, rym.v1) * (xc.v1 - xym.v1);
            acc1 += cyp * face_kappa<FR>(rc.v1, ryp.v1) * (xc.v1 - xyp.v1);
            acc1 += wzm1 * (xc.v1 - xm.v1);
            acc1 += wzp1 * (xc.v1 - xn.v1);
            if (MODE >= 2) {
                acc0 = bv.v0 - acc0;
                acc1 = bv.v1 - acc1;
            }
            stp(y + a, acc0, acc1);
            if (MODE == 1) part += (double)xc.v0 * (double)acc0 + (double)xc.v1 * (double)acc1;
            if (MODE == 3) part += (double)acc0 * (double)acc0 + (double)acc1 * (double)acc1;
            // advance: the z+ faces of plane k are the z- faces of plane k+1
            wzm0 = wzp0;
            wzm1 = wzp1;
            xm = xc;
            xc = xn;
            rc = rn;
            xn = xnn;
            rn = rnn;
            czp = hpn ? g.cz : T(0);
            xl = xln; xr = xrn; rl = rln; rr = rrn;
            xym = xymn; xyp = xypn; rym = rymn; ryp = rypn;
            mv = mvn;
            bv = bvn;
            a = an;
        }
    }
    if (MODE == 1 || MODE == 3) block_partial(part, partials);
}

// ---- red-black split layout (finest level) ----
constexpr int kRowsS = 4;     // x rows per workgroup of the split-layout kernels
// Waves per row of the split kernels: a row tile spans 64 XW half positions, two waves where
// rows have more than 64 half positions (up to 256 cells: the whole row), else one.
static inline int split_xw(int hx) { return hx > 64 ? 2 : 1; }
// Thread (t, j) owns the cell pair (2t, 2t+1) of row j: half position t of the red and of the
// black half of the row. Cell 2t has the colour of the row parity p = (j + k) & 1; cell 2t-1
// (half position t-1) the other colour and cell 2t+2 (half position t+1) the same colour. The
// y and z neighbour rows have parity 1 - p, so there cell 2t has colour 1 - p.

__device__ __forceinline__ int srow(int j, int k, int nx, int ny) { return (k * ny + j) * nx; }

// values of the cells (2t, 2t+1) of the row at rb whose parity is par
template <typename T>
__device__ __forceinline__ Pair<T> lds(const T* __restrict__ a, int rb, int hx, int t, int par) {
    const T r = a[rb + t], b = a[rb + hx + t];
    return par ? Pair<T>{b, r} : Pair<T>{r, b};
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_relayout(const T* __restrict__ src, T* __restrict__ dst,
                                                     int nx, int ny, int64_t npairs, int to_split) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npairs) return;
    const int hx = nx >> 1;
    const int64_t row = q / hx;
    const int t = (int)(q - row * hx);
    const int p = (int)((row % ny + row / ny) & 1);
    const int64_t rb = row * nx;
    const int64_t ae = rb + p * hx + t, ao = rb + (1 - p) * hx + t;
    if (to_split) {
        const T v0 = src[rb + 2 * t], v1 = src[rb + 2 * t + 1];
        dst[ae] = v0;
        dst[ao] = v1;
    } else {
        const T v0 = src[ae], v1 = src[ao];
        dst[rb + 2 * t] = v0;
        dst[rb + 2 * t + 1] = v1;
    }
}

// plane below / above k (the plane itself where a Neumann end has no face)
__device__ __forceinline__ int kbelow(int k, int nz, int pz) { return k > 0 ? k - 1 : (pz ? nz - 1 : k); }
__device__ __forceinline__ int kabove(int k, int nz, int pz) { return k < nz - 1 ? k + 1 : (pz ? 0 : k); }

// Per-thread neighbour rows and face factors of column pair t, row j (absent faces: factor 0 and
// an in-bounds stand-in index).
template <typename T>
struct SplitCol {
    int tm, tp, jm, jp;
    T cxl, cxr, cym, cyp;
    __device__ __forceinline__ SplitCol(const Geo<T>& g, int t, int j) {
        const int hx = g.nx >> 1;
        tm = t > 0 ? t - 1 : hx - 1;
        tp = t < hx - 1 ? t + 1 : 0;
        cxl = (t > 0 || g.px) ? g.cx : T(0);       // x- face of cell 2t
        cxr = (t < hx - 1 || g.px) ? g.cx : T(0);  // x+ face of cell 2t+1
        jm = j > 0 ? j - 1 : (g.py ? g.ny - 1 : j);
        jp = j < g.ny - 1 ? j + 1 : (g.py ? 0 : j);
        cym = (j > 0 || g.py) ? g.cy : T(0);
        cyp = (j < g.ny - 1 || g.py) ? g.cy : T(0);
    }
};

// Neighbour exchange of the split kernels: a workgroup covers kRowsS rows of one row tile (kTW
// half positions, kXW waves per row), and per plane every thread stores the values of its cells
// that neighbours need into LDS, together with the rows just below and above the workgroup
// (loaded by all threads of the workgroup, a few entries each). After one barrier the y
// neighbours are read from the rows beside a thread's own and the outer x neighbour from the
// adjacent position. Where a row tile covers the whole row (FULL: nx/2 <= kTW) the periodic x
// wrap is in LDS too; otherwise the thread at the edge of a tile reads that neighbour from
// memory. Two plane slots make one barrier per plane enough: a slot is rewritten two planes
// later, after every wave has passed the barrier of the plane in between. The grid covers whole
// rows (ny a multiple of kRowsS); positions beyond the row (t >= nx/2) work on a clamped copy of
// the last one and store nothing.
//
// The z march keeps the column of the cell (planes k-1 .. k+2) in a ring of registers and the
// values of the next plane in the second of two records, and is unrolled by four so that both
// rotate by renaming: a register move at the loop end would wait for loads still in flight.
static_assert(kRowsS >= 2, "the split kernels need separate first and last rows");

// Workgroups the split kernels aim for with two-wave rows (one-wave rows aim for a wave count).
constexpr int kSplitWG2 = 768;
// Tiles of the split kernels over hx = nx/2 half positions: 64 XW per tile, kRowsS rows, z chunks
// of at least kZMin planes.  Two-wave rows (the finest level of 256^3 and up) take about
// kSplitWG2 workgroups, three per CU: at 256^3 the operator apply and the half sweeps ran
// 2-4% faster with 768 than with 1024, and 10-20% slower with counts that do not split evenly
// over the 32 CUs of an XCD (640, 704, 832, 896, 1152).  One-wave rows aim for about 8192 waves.
static ZTiles split_tiles(int hx, int ny, int nz) {
    const int xw = split_xw(hx), tw = 64 * xw;
    ZTiles t;
    t.tx = (hx + tw - 1) / tw;
    t.ty = (ny + kRowsS - 1) / kRowsS;
    const int cols = t.tx * t.ty;
    const int wg = xw == 2 ? kSplitWG2 : 0;
    t.kz = nz;
    if (wg > 0) {
        const int want = std::max(1, std::min(nz, (wg + cols / 2) / cols));
        t.kz = std::max((nz + want - 1) / want, std::min(kZMin, nz));
    } else {
        const int target = 8192 / (xw * kRowsS);
        while (t.kz > kZMin && (int64_t)cols * ((nz + t.kz - 1) / t.kz) < target) t.kz = (t.kz + 1) / 2;
    }
    t.tz = (nz + t.kz - 1) / t.kz;
    return t;
}

template <bool FULL, int XW>
struct SplitLane {
    static constexpr int kTW = 64 * XW;
    int lane;    // position in the row tile, 0 .. kTW-1 (the LDS column)
    int w;       // row of the workgroup
    int tl, t, j, j0;
    int lm, lp;  // LDS columns of the half positions t-1 and t+1 (own column where memory supplies)
    bool act, gl, gr;
    __device__ __forceinline__ SplitLane(int bx, int by, int hx) {
        lane = threadIdx.x % kTW;
        // a row is a whole number of waves, so the row index is uniform across the wave: kept in a
        // scalar register, and with it every row base address
        w = __builtin_amdgcn_readfirstlane(threadIdx.x / kTW);
        tl = bx * kTW + lane;
        act = tl < hx;
        t = act ? tl : hx - 1;
        j0 = by * kRowsS;
        j = j0 + w;
        if (FULL) {  // the tile is the whole row: wrap in LDS
            gl = gr = false;
            lm = t > 0 ? t - 1 : hx - 1;
            lp = t < hx - 1 ? t + 1 : 0;
        } else {
            gl = lane == 0;
            gr = !(lane < kTW - 1 && tl + 1 < hx);
            lm = gl ? lane : lane - 1;
            lp = gr ? lane : lane + 1;
        }
    }
};

// Rows just below (side 0) and above (side 1) the workgroup's rows j0 .. j0+kRowsS-1; the edge
// row itself where a Neumann end has no such row.
__device__ __forceinline__ int halo_row(int side, int j0, int ny, int py) {
    if (side == 0) return j0 > 0 ? j0 - 1 : (py ? ny - 1 : j0);
    return j0 + kRowsS < ny ? j0 + kRowsS : (py ? 0 : j0 + kRowsS - 1);
}

// Entries at half position t of the red and of the black half of a row, as loaded; the cells
// (2t, 2t+1) of a row of parity par are pos(h, par). Loaded values stay in this form and cells
// are selected only where they are used, so that no select waits for a load still in flight.
template <typename T>
struct HalfPair {
    T r, b;
};
template <typename T>
__device__ __forceinline__ HalfPair<T> ldh(const T* __restrict__ a, int rb, int hx, int t) {
    return {a[rb + t], a[rb + hx + t]};
}
// Streaming loads of values that the next passes over the finest level do not read: they leave the
// 256 MB memory-side cache to the arrays those passes do read (see k_xpby_x)
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
    return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ HalfPair<T> ldh_stream(const T* __restrict__ a, int rb, int hx, int t) {
    return {ld_stream(&a[rb + t]), ld_stream(&a[rb + hx + t])};
}
template <typename T>
__device__ __forceinline__ Pair<T> pos(const HalfPair<T>& h, int par) {
    return par ? Pair<T>{h.b, h.r} : Pair<T>{h.r, h.b};
}

// Operator apply in the split layout: the pair march of k_apply_zp with each pair read from the
// two halves of its row; pairs of x and rho of the current plane are exchanged through LDS. The
// column pairs of x (planes k-1 .. k+2) and rho (k .. k+2) form the register rings.
template <typename T, int MODE, bool FULL, int XW, int FR = 0>
__global__ __launch_bounds__(64 * XW * kRowsS) void k_apply_zs(Geo<T> g, ZTiles zt,
                                                     const T* __restrict__ rho,
                                                     const T* __restrict__ m,
                                                     const T* __restrict__ x,
                                                     const T* __restrict__ b, T* __restrict__ y,
                                                     double* __restrict__ partials) {
    constexpr int kTW = 64 * XW, kBlockS = kTW * kRowsS;
    __shared__ T sx[2][2][kRowsS + 2][2][kTW];  // [plane slot][x, rho][row][cell of the pair][column]
    int bx, by, bz;
    ztile(zt, bx, by, bz);
    const int nx = g.nx, ny = g.ny, hx = nx >> 1;
    const SplitLane<FULL, XW> L(bx, by, hx);
    const int t = L.t, j = L.j, lane = L.lane, w = L.w;
    const SplitCol<T> sc(g, t, j);
    const int lm = L.lm, lp = L.lp;
    const int k0 = bz * zt.kz;
    const int k1 = min(k0 + zt.kz, g.nz);
    double part = 0.0;
    // halo items: 2 rows x (x, rho) x (red, black half) x kTW columns, a few per thread
    constexpr int HI = 8 * kTW, NH = (HI + kBlockS - 1) / kBlockS;
    // what a plane contributes besides the column: m and b, the outer x neighbours where memory
    // supplies them, this thread's halo entries
    struct Own {
        HalfPair<T> mh, bh;
        T xl, xr, rl, rr;
        T h[NH];
    };
    auto load_own = [&](int kp, Own& o) {
        const int pp = (j + kp) & 1;
        const int rbp = srow(j, kp, nx, ny);
        o.mh = ldh_stream(m, rbp, hx, t);   // m is next read by the post-smoothing
        o.bh = MODE >= 2 ? ldh(b, rbp, hx, t) : HalfPair<T>{T(0), T(0)};
        if (!FULL) {
            o.xl = L.gl ? x[rbp + (1 - pp) * hx + sc.tm] : T(0);
            o.rl = L.gl ? rho[rbp + (1 - pp) * hx + sc.tm] : T(0);
            o.xr = L.gr ? x[rbp + pp * hx + sc.tp] : T(0);
            o.rr = L.gr ? rho[rbp + pp * hx + sc.tp] : T(0);
        }
#pragma unroll
        for (int n = 0; n < NH; ++n) {
            const int i = threadIdx.x + n * kBlockS;
            T v = T(0);
            if (i < HI) {
                const int col = i % kTW, rest = i / kTW;
                const int half = rest & 1, arr = (rest >> 1) & 1, side = rest >> 2;
                const int tp = min(bx * kTW + col, hx - 1);
                const int jr = halo_row(side, L.j0, ny, g.py);
                v = (arr ? rho : x)[srow(jr, kp, nx, ny) + half * hx + tp];
            }
            o.h[n] = v;
        }
    };
    auto store_halo = [&](int k, int sl, const Own& o) {
#pragma unroll
        for (int n = 0; n < NH; ++n) {
            const int i = threadIdx.x + n * kBlockS;
            if (i < HI) {
                const int col = i % kTW, rest = i / kTW;
                const int half = rest & 1, arr = (rest >> 1) & 1, side = rest >> 2;
                const int jr = halo_row(side, L.j0, ny, g.py);
                sx[sl][arr][side ? kRowsS + 1 : 0][half ^ ((jr + k) & 1)][col] = o.h[n];
            }
        }
    };
    auto step = [&](int k, const HalfPair<T>& Xm, const HalfPair<T>& Xc, const HalfPair<T>& Xn,
                    HalfPair<T>& Xnn, const HalfPair<T>& Rc, const HalfPair<T>& Rn, HalfPair<T>& Rnn,
                    T& wzm0, T& wzm1, const Own& c, Own& nxt) {
        // prefetch plane k+1 (clamped to the chunk) and the column two planes up
        const int kn = min(k + 1, k1 - 1);
        load_own(kn, nxt);
        const int rbnn = srow(j, kabove(kn, g.nz, g.pz), nx, ny);
        Xnn = ldh(x, rbnn, hx, t);
        Rnn = ldh(rho, rbnn, hx, t);
        const int p = (j + k) & 1;
        const int rb = srow(j, k, nx, ny);
        const Pair<T> xc = pos(Xc, p), rc = pos(Rc, p);
        // exchange plane k
        const int sl = k & 1;
        sx[sl][0][w + 1][0][lane] = xc.v0;
        sx[sl][0][w + 1][1][lane] = xc.v1;
        sx[sl][1][w + 1][0][lane] = rc.v0;
        sx[sl][1][w + 1][1][lane] = rc.v1;
        store_halo(k, sl, c);
        __syncthreads();
        T xl = sx[sl][0][w + 1][1][lm], rl = sx[sl][1][w + 1][1][lm];
        T xr = sx[sl][0][w + 1][0][lp], rr = sx[sl][1][w + 1][0][lp];
        if (!FULL) {
            if (L.gl) {
                xl = c.xl;
                rl = c.rl;
            }
            if (L.gr) {
                xr = c.xr;
                rr = c.rr;
            }
        }
        const Pair<T> xym = {sx[sl][0][w][0][lane], sx[sl][0][w][1][lane]};
        const Pair<T> xyp = {sx[sl][0][w + 2][0][lane], sx[sl][0][w + 2][1][lane]};
        const Pair<T> rym = {sx[sl][1][w][0][lane], sx[sl][1][w][1][lane]};
        const Pair<T> ryp = {sx[sl][1][w + 2][0][lane], sx[sl][1][w + 2][1][lane]};
        const Pair<T> xm = pos(Xm, p ^ 1), xn = pos(Xn, p ^ 1), rn = pos(Rn, p ^ 1);
        const Pair<T> mv = pos(c.mh, p);
        // plane k
        const T czp = (k < g.nz - 1 || g.pz) ? g.cz : T(0);
        const T wx = g.cx * face_kappa<FR>(rc.v0, rc.v1);
        const T wzp0 = czp * face_kappa<FR>(rc.v0, rn.v0);
        const T wzp1 = czp * face_kappa<FR>(rc.v1, rn.v1);
        T acc0 = mv.v0 * xc.v0;
        acc0 += ((t > 0 || g.px) ? g.cx : T(0)) * face_kappa<FR>(rc.v0, rl) * (xc.v0 - xl);
        acc0 += wx * (xc.v0 - xc.v1);
        acc0 += sc.cym * face_kappa<FR>(rc.v0, rym.v0) * (xc.v0 - xym.v0);
        acc0 += sc.cyp * face_kappa<FR>(rc.v0, ryp.v0) * (xc.v0 - xyp.v0);
        acc0 += wzm0 * (xc.v0 - xm.v0);
        acc0 += wzp0 * (xc.v0 - xn.v0);
        T acc1 = mv.v1 * xc.v1;
        acc1 += wx * (xc.v1 - xc.v0);
        acc1 += ((t < hx - 1 || g.px) ? g.cx : T(0)) * face_kappa<FR>(rc.v1, rr) * (xc.v1 - xr);
        acc1 += sc.cym * face_kappa<FR>(rc.v1, rym.v1) * (xc.v1 - xym.v1);
        acc1 += sc.cyp * face_kappa<FR>(rc.v1, ryp.v1) * (xc.v1 - xyp.v1);
        acc1 += wzm1 * (xc.v1 - xm.v1);
        acc1 += wzp1 * (xc.v1 - xn.v1);
        if (MODE >= 2) {
            const Pair<T> bv = pos(c.bh, p);
            acc0 = bv.v0 - acc0;
            acc1 = bv.v1 - acc1;
        }
        if (L.act) {
            y[rb + p * hx + t] = acc0;
            y[rb + (1 - p) * hx + t] = acc1;
            if (MODE == 1) part += (double)xc.v0 * (double)acc0 + (double)xc.v1 * (double)acc1;
            if (MODE == 3) part += (double)acc0 * (double)acc0 + (double)acc1 * (double)acc1;
        }
        // the z+ faces of plane k are the z- faces of plane k+1
        wzm0 = wzp0;
        wzm1 = wzp1;
    };
    HalfPair<T> X0, X1, X2, X3 = {T(0), T(0)}, R0, R1, R2, R3 = {T(0), T(0)};
    T wzm0, wzm1;
    {
        const int p0 = (j + k0) & 1;
        const int rbm = srow(j, kbelow(k0, g.nz, g.pz), nx, ny), rb = srow(j, k0, nx, ny);
        const int rbp = srow(j, kabove(k0, g.nz, g.pz), nx, ny);
        X0 = ldh(x, rbm, hx, t);
        X1 = ldh(x, rb, hx, t);
        X2 = ldh(x, rbp, hx, t);
        R0 = ldh(rho, rbm, hx, t);
        R1 = ldh(rho, rb, hx, t);
        R2 = ldh(rho, rbp, hx, t);
        const Pair<T> rc = pos(R1, p0), rm = pos(R0, p0 ^ 1);
        const T czm0 = (k0 > 0 || g.pz) ? g.cz : T(0);
        wzm0 = czm0 * face_kappa<FR>(rc.v0, rm.v0);
        wzm1 = czm0 * face_kappa<FR>(rc.v1, rm.v1);
    }
    Own A, B;
    load_own(k0, A);
    int k = k0;
    for (; k + 4 <= k1; k += 4) {
        step(k, X0, X1, X2, X3, R1, R2, R3, wzm0, wzm1, A, B);
        step(k + 1, X1, X2, X3, X0, R2, R3, R0, wzm0, wzm1, B, A);
        step(k + 2, X2, X3, X0, X1, R3, R0, R1, wzm0, wzm1, A, B);
        step(k + 3, X3, X0, X1, X2, R0, R1, R2, wzm0, wzm1, B, A);
    }
    if (k < k1) step(k, X0, X1, X2, X3, R1, R2, R3, wzm0, wzm1, A, B);
    if (k + 1 < k1) step(k + 1, X1, X2, X3, X0, R2, R3, R0, wzm0, wzm1, B, A);
    if (k + 2 < k1) step(k + 2, X2, X3, X0, X1, R3, R0, R1, wzm0, wzm1, A, B);
    if (MODE == 1 || MODE == 3) block_partial(part, partials);
}

// Half sweep of colour c in the split layout: one thread per cell of colour c (half position t
// of row j), marching in z. Every neighbour has the other colour: x neighbours at half positions
// t (the pair partner) and t-1 or t+1, y neighbours at t in rows j-1 and j+1, z neighbours at t
// in the planes below and above; the other colour's z and rho at t of planes k-1 .. k+2 form the
// register ring, and those of the current plane are exchanged through LDS for the x and y
// neighbours. DOT also reduces <r, z> over the cells of colour c (the black and the red sweep of a
// post-smoothing reduce half each); RESID instead writes t = r - A z on the
// cells of colour c only. ZG (with RESID, colour red): z holds the zero-guess pre-smoothing,
// whose red values are r dinv, so r - (m + sum w) z vanishes on red cells and t = sum_f w_f z_nb
// (r and m are not read).
template <typename T, bool DOT, bool RESID, bool ZG, bool FULL, int XW, int FR = 0>
__global__ __launch_bounds__(64 * XW * kRowsS) void k_rbgs_zs(Geo<T> g, ZTiles zt,
                                                    const T* __restrict__ rho,
                                                    const T* __restrict__ m,
                                                    const T* __restrict__ r, T* __restrict__ z,
                                                    int colour, double* __restrict__ partials,
                                                    T* __restrict__ tout) {
    constexpr int kTW = 64 * XW, kBlockS = kTW * kRowsS;
    __shared__ T sx[2][2][kRowsS + 2][kTW];  // [plane slot][z, rho of the other colour][row][column]
    int bx, by, bz;
    ztile(zt, bx, by, bz);
    const int nx = g.nx, ny = g.ny, hx = nx >> 1;
    const SplitLane<FULL, XW> L(bx, by, hx);
    const int t = L.t, j = L.j, lane = L.lane, w = L.w;
    const int ch = colour * hx, oh = (colour ^ 1) * hx;
    const SplitCol<T> sc(g, t, j);
    const int lm = L.lm, lp = L.lp;
    const int k0 = bz * zt.kz;
    const int k1 = min(k0 + zt.kz, g.nz);
    constexpr bool RM = !(RESID && ZG);  // r and m are read
    double dsum = 0.0;
    // halo items: 2 rows x (z, rho) x kTW columns of the other colour
    constexpr int HI = 4 * kTW, NH = (HI + kBlockS - 1) / kBlockS;
    // what a plane contributes besides the other colour's column: this colour's rho, r and m,
    // the outer x neighbour where memory supplies it, halo entries
    struct Own {
        T ra, rr, mm, zx, rx;
        T h[NH];
    };
    auto load_own = [&](int kp, Own& o) {
        const int rbp = srow(j, kp, nx, ny);
        o.ra = rho[rbp + ch + t];
        o.rr = RM ? ld_stream(&r[rbp + ch + t]) : T(0);   // next read a pass later at the earliest
        o.mm = RM ? ld_stream(&m[rbp + ch + t]) : T(0);
        if (!FULL) {
            const int ep = ((j + kp) & 1) ^ colour;
            const bool gxp = ep ? L.gr : L.gl;
            const int txp = ep ? sc.tp : sc.tm;
            o.zx = gxp ? z[rbp + oh + txp] : T(0);
            o.rx = gxp ? rho[rbp + oh + txp] : T(0);
        }
#pragma unroll
        for (int n = 0; n < NH; ++n) {
            const int i = threadIdx.x + n * kBlockS;
            T v = T(0);
            if (i < HI) {
                const int col = i % kTW, rest = i / kTW;
                const int arr = rest & 1, side = rest >> 1;
                const int tp = min(bx * kTW + col, hx - 1);
                v = (arr ? rho : z)[srow(halo_row(side, L.j0, ny, g.py), kp, nx, ny) + oh + tp];
            }
            o.h[n] = v;
        }
    };
    auto step = [&](int k, const T& zom, const T& zoc, const T& zon, T& zonn, const T& rom, const T& roc,
                    const T& ron, T& ronn, const Own& c, Own& nxt) {
        const int kn = min(k + 1, k1 - 1);
        load_own(kn, nxt);
        const int rbnn = srow(j, kabove(kn, g.nz, g.pz), nx, ny);
        zonn = z[rbnn + oh + t];
        ronn = rho[rbnn + oh + t];
        const int rb = srow(j, k, nx, ny);
        const int e = ((j + k) & 1) ^ colour;  // 0: the cell is 2t (extra x neighbour at t-1), 1: 2t+1
        // exchange the other colour of plane k
        const int sl = k & 1;
        sx[sl][0][w + 1][lane] = zoc;
        sx[sl][1][w + 1][lane] = roc;
#pragma unroll
        for (int n = 0; n < NH; ++n) {
            const int i = threadIdx.x + n * kBlockS;
            if (i < HI) {
                const int col = i % kTW, rest = i / kTW;
                sx[sl][rest & 1][(rest >> 1) ? kRowsS + 1 : 0][col] = c.h[n];
            }
        }
        __syncthreads();
        const int ln = e ? lp : lm;
        T zx = sx[sl][0][w + 1][ln], rx = sx[sl][1][w + 1][ln];
        if (!FULL && (e ? L.gr : L.gl)) {
            zx = c.zx;
            rx = c.rx;
        }
        const T zy0 = sx[sl][0][w][lane], ry0 = sx[sl][1][w][lane];
        const T zy1 = sx[sl][0][w + 2][lane], ry1 = sx[sl][1][w + 2][lane];
        // faces in the order x-, x+, y-, y+, z-, z+
        const T ra = c.ra;
        const T czm = (k > 0 || g.pz) ? g.cz : T(0);
        const T czp = (k < g.nz - 1 || g.pz) ? g.cz : T(0);
        const T wp = g.cx * face_kappa<FR>(ra, roc);                    // pair partner
        const T cxo = ((e ? t < hx - 1 : t > 0) || g.px) ? g.cx : T(0);  // outer x face factor
        const T we = cxo * face_kappa<FR>(ra, rx);                      // outer x neighbour
        const T w0 = e ? wp : we, v0 = e ? zoc : zx;
        const T w1 = e ? we : wp, v1 = e ? zx : zoc;
        T sw = w0, swz = w0 * v0;
        sw += w1;
        swz += w1 * v1;
        const T wy0 = sc.cym * face_kappa<FR>(ra, ry0), wy1 = sc.cyp * face_kappa<FR>(ra, ry1);
        sw += wy0;
        swz += wy0 * zy0;
        sw += wy1;
        swz += wy1 * zy1;
        const T wzm = czm * face_kappa<FR>(ra, rom), wzp = czp * face_kappa<FR>(ra, ron);
        sw += wzm + wzp;
        swz += wzm * zom + wzp * zon;
        if (L.act) {
            if (RESID && ZG) {
                tout[rb + ch + t] = swz;
            } else if (RESID) {
                const T zs = z[rb + ch + t];
                tout[rb + ch + t] = c.rr + swz - (c.mm + sw) * zs;
            } else {
                const T znew = (c.rr + swz) / (c.mm + sw);
                z[rb + ch + t] = znew;
                if (DOT) dsum += (double)c.rr * (double)znew;
            }
        }
    };
    // other colour at t: planes k0-1, k0, k0+1
    T z0, z1, z2, z3 = T(0), q0, q1, q2, q3 = T(0);
    {
        const int rbm = srow(j, kbelow(k0, g.nz, g.pz), nx, ny), rb = srow(j, k0, nx, ny);
        const int rbp = srow(j, kabove(k0, g.nz, g.pz), nx, ny);
        z0 = z[rbm + oh + t]; z1 = z[rb + oh + t]; z2 = z[rbp + oh + t];
        q0 = rho[rbm + oh + t]; q1 = rho[rb + oh + t]; q2 = rho[rbp + oh + t];
    }
    Own A, B;
    load_own(k0, A);
    int k = k0;
    for (; k + 4 <= k1; k += 4) {
        step(k, z0, z1, z2, z3, q0, q1, q2, q3, A, B);
        step(k + 1, z1, z2, z3, z0, q1, q2, q3, q0, B, A);
        step(k + 2, z2, z3, z0, z1, q2, q3, q0, q1, A, B);
        step(k + 3, z3, z0, z1, z2, q3, q0, q1, q2, B, A);
    }
    if (k < k1) step(k, z0, z1, z2, z3, q0, q1, q2, q3, A, B);
    if (k + 1 < k1) step(k + 1, z1, z2, z3, z0, q1, q2, q3, q0, B, A);
    if (k + 2 < k1) step(k + 2, z2, z3, z0, z1, q2, q3, q0, q1, A, B);
    if (DOT) block_partial(dsum, partials);
}

// Zero-guess pre-smoothing in the split layout, one pass: z_red = r dinv on red cells and
// z_black = dinv_b (r_b + sum_f w_f (r dinv)_nb) on black cells, whose neighbours are all red.
// The red q = r dinv and rho of the current plane are exchanged through LDS; the red column
// (r, dinv and rho at t, planes k-1 .. k+2) forms the register ring.
// UPD: the CG residual update of the iteration is folded in: the pass reads r and q, smooths
// r' = r - alpha q (alpha = scal[S_ALPHA]), writes r' to rn (a second array: other workgroups
// read r around their tiles meanwhile) and reduces ||r'||^2 over its cells into partials, with
// the breakdown flag copied by workgroup 0 (as r -= alpha q does).
template <typename T, bool FULL, int XW, bool UPD, int FR = 0>
__global__ __launch_bounds__(64 * XW * kRowsS) void k_presmooth_zs(Geo<T> g, ZTiles zt,
                                                         const T* __restrict__ rho,
                                                         const T* __restrict__ dinv,
                                                         const T* __restrict__ r,
                                                         T* __restrict__ z, const T* __restrict__ qv,
                                                         T* __restrict__ rn, RedCtl rc) {
    constexpr int kTW = 64 * XW, kBlockS = kTW * kRowsS;
    __shared__ T sx[2][2][kRowsS + 2][kTW];  // [plane slot][red q, red rho][row][column]
    int bx, by, bz;
    ztile(zt, bx, by, bz);
    const int nx = g.nx, ny = g.ny, hx = nx >> 1;
    const SplitLane<FULL, XW> L(bx, by, hx);
    const int t = L.t, j = L.j, lane = L.lane, w = L.w;
    const SplitCol<T> sc(g, t, j);
    const int lm = L.lm, lp = L.lp;
    const int k0 = bz * zt.kz;
    const int k1 = min(k0 + zt.kz, g.nz);
    const T alpha = UPD ? (T)rc.scal[S_ALPHA] : T(0);
    double nacc = 0.0;
    // red entries at t of one plane: r (and q), dinv and rho; r' = r - alpha q is formed at use
    struct Red {
        T r, q, d, rho;
    };
    auto ldred = [&](int rbp, Red& o) {
        o.r = r[rbp + t];
        o.q = UPD ? ld_stream(&qv[rbp + t]) : T(0);
        o.d = dinv[rbp + t];
        o.rho = rho[rbp + t];
    };
    // halo items: 2 rows x (q from r and dinv, rho) x kTW columns of the red half
    constexpr int HI = 4 * kTW, NH = (HI + kBlockS - 1) / kBlockS;
    // the black cell of a plane, its outer x neighbour where memory supplies it, halo entries
    struct Own {
        T rho, r, q, d, xr, xq, xd, xrho;
        T h0[NH], h1[NH], h2[NH];
    };
    auto load_own = [&](int kp, Own& o) {
        const int rbp = srow(j, kp, nx, ny);
        o.rho = rho[rbp + hx + t];
        o.r = r[rbp + hx + t];
        o.q = UPD ? ld_stream(&qv[rbp + hx + t]) : T(0);
        o.d = dinv[rbp + hx + t];
        if (!FULL) {
            const int ep = ((j + kp) & 1) ^ 1;
            const bool gxp = ep ? L.gr : L.gl;
            const int txp = ep ? sc.tp : sc.tm;
            o.xr = gxp ? r[rbp + txp] : T(0);
            o.xq = (UPD && gxp) ? qv[rbp + txp] : T(0);
            o.xd = gxp ? dinv[rbp + txp] : T(0);
            o.xrho = gxp ? rho[rbp + txp] : T(0);
        }
#pragma unroll
        for (int n = 0; n < NH; ++n) {
            const int i = threadIdx.x + n * kBlockS;
            T v0 = T(0), v1 = T(1), v2 = T(0);
            if (i < HI) {
                const int col = i % kTW, rest = i / kTW;
                const int arr = rest & 1, side = rest >> 1;
                const int tp = min(bx * kTW + col, hx - 1);
                const int a = srow(halo_row(side, L.j0, ny, g.py), kp, nx, ny) + tp;
                if (arr) {
                    v0 = rho[a];
                } else {
                    v0 = r[a];
                    v1 = dinv[a];
                    if (UPD) v2 = qv[a];
                }
            }
            o.h0[n] = v0;
            o.h1[n] = v1;
            o.h2[n] = v2;
        }
    };
    // r' of a loaded (r, q) pair (r itself without UPD)
    auto rup = [&](T rv, T q) { return UPD ? rv - alpha * q : rv; };
    auto step = [&](int k, const Red& cm, const Red& cc, const Red& cn, Red& cnn, const Own& c, Own& nxt) {
        const int kn = min(k + 1, k1 - 1);
        load_own(kn, nxt);
        ldred(srow(j, kabove(kn, g.nz, g.pz), nx, ny), cnn);
        const int rb = srow(j, k, nx, ny);
        const int e = ((j + k) & 1) ^ 1;
        const T rcr = rup(cc.r, cc.q), rcb = rup(c.r, c.q);   // r' of this plane's red and black cell
        const T qm = rup(cm.r, cm.q) * cm.d, qc = rcr * cc.d, qn = rup(cn.r, cn.q) * cn.d;
        // exchange the red cells of plane k
        const int sl = k & 1;
        sx[sl][0][w + 1][lane] = qc;
        sx[sl][1][w + 1][lane] = cc.rho;
#pragma unroll
        for (int n = 0; n < NH; ++n) {
            const int i = threadIdx.x + n * kBlockS;
            if (i < HI) {
                const int col = i % kTW, rest = i / kTW;
                // rho entries carry v2 = 0: rup leaves them as loaded
                sx[sl][rest & 1][(rest >> 1) ? kRowsS + 1 : 0][col] = rup(c.h0[n], c.h2[n]) * c.h1[n];
            }
        }
        __syncthreads();
        const int ln = e ? lp : lm;
        T qx = sx[sl][0][w + 1][ln], rx = sx[sl][1][w + 1][ln];
        if (!FULL && (e ? L.gr : L.gl)) {
            qx = rup(c.xr, c.xq) * c.xd;
            rx = c.xrho;
        }
        const T qy0 = sx[sl][0][w][lane], ry0 = sx[sl][1][w][lane];
        const T qy1 = sx[sl][0][w + 2][lane], ry1 = sx[sl][1][w + 2][lane];
        // faces of the black cell in the order x-, x+, y-, y+, z-, z+
        const T rbr = c.rho;
        const T czm = (k > 0 || g.pz) ? g.cz : T(0);
        const T czp = (k < g.nz - 1 || g.pz) ? g.cz : T(0);
        const T wp = g.cx * face_kappa<FR>(rbr, cc.rho);
        const T cxo = ((e ? t < hx - 1 : t > 0) || g.px) ? g.cx : T(0);
        const T we = cxo * face_kappa<FR>(rbr, rx);
        T swq = (e ? wp : we) * (e ? qc : qx);
        swq += (e ? we : wp) * (e ? qx : qc);
        swq += sc.cym * face_kappa<FR>(rbr, ry0) * qy0;
        swq += sc.cyp * face_kappa<FR>(rbr, ry1) * qy1;
        const T wzm = czm * face_kappa<FR>(rbr, cm.rho), wzp = czp * face_kappa<FR>(rbr, cn.rho);
        swq += wzm * qm + wzp * qn;
        if (L.act) {
            // the red values are next read by the prolongation after the coarse levels; the
            // black ones by the residual right after this pass
            __builtin_nontemporal_store(qc, &z[rb + t]);
            z[rb + hx + t] = (rcb + swq) * c.d;
            if (UPD) {
                rn[rb + t] = rcr;
                rn[rb + hx + t] = rcb;
                nacc += (double)rcr * (double)rcr + (double)rcb * (double)rcb;
            }
        }
    };
    Red C0, C1, C2, C3 = {T(0), T(0), T(0), T(0)};
    ldred(srow(j, kbelow(k0, g.nz, g.pz), nx, ny), C0);
    ldred(srow(j, k0, nx, ny), C1);
    ldred(srow(j, kabove(k0, g.nz, g.pz), nx, ny), C2);
    Own A, B;
    load_own(k0, A);
    int k = k0;
    for (; k + 4 <= k1; k += 4) {
        step(k, C0, C1, C2, C3, A, B);
        step(k + 1, C1, C2, C3, C0, B, A);
        step(k + 2, C2, C3, C0, C1, A, B);
        step(k + 3, C3, C0, C1, C2, B, A);
    }
    if (k < k1) step(k, C0, C1, C2, C3, A, B);
    if (k + 1 < k1) step(k + 1, C1, C2, C3, C0, B, A);
    if (k + 2 < k1) step(k + 2, C2, C3, C0, C1, A, B);
    if (UPD) {
        block_partial(nacc, rc.partials);
        export_flag(rc);
    }
}

// Launch one split kernel over its tiles: one wave per row for rows of up to 64 half positions,
// else two; FULL where the row tile spans the whole row. F(full, xw) names the instance.
enum SplitShape { SPLIT_FULL1, SPLIT_FULL2, SPLIT_TILED2 };
static inline SplitShape split_shape(int hx) {
    return hx <= 64 ? SPLIT_FULL1 : (hx <= 128 ? SPLIT_FULL2 : SPLIT_TILED2);
}
static inline dim3 split_block(int hx) { return dim3(64 * split_xw(hx) * kRowsS); }

// Kernel timing: the events handed over by set_launch_events are attached to the next split-layout
// stencil launch of this thread, which records its own start and end into them (the dispatch's
// time stamps, without marker packets around it).
namespace {
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;
}
void set_launch_events(hipEvent_t start, hipEvent_t stop) {
    t_ev_start = start;
    t_ev_stop = stop;
}
bool launch_events_pending() { return t_ev_start != nullptr; }

template <typename K, typename... Args>
static void launch_split(K kernel, dim3 grid, dim3 block, hipStream_t s, Args... args) {
    if (t_ev_start) {
        hipEvent_t a = t_ev_start, b = t_ev_stop;
        t_ev_start = t_ev_stop = nullptr;
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, a, b, 0, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    }
}

template <typename T, int MODE>
static void launch_apply_zs(const Geo<T>& g, const ZTiles& zt, const T* rho, const T* m, const T* x,
                            const T* b, T* y, double* partials, hipStream_t s) {
    const int hx = g.nx >> 1;
    const dim3 grid(zt.tx * zt.ty * zt.tz), block = split_block(hx);
    switch (split_shape(hx)) {
        case SPLIT_FULL1:
            WITH_FACE_RULE(g.frule,
                launch_split(k_apply_zs<T, MODE, true, 1, FRV>, grid, block, s, g, zt, rho, m, x, b, y, partials));
            break;
        case SPLIT_FULL2:
            WITH_FACE_RULE(g.frule,
                launch_split(k_apply_zs<T, MODE, true, 2, FRV>, grid, block, s, g, zt, rho, m, x, b, y, partials));
            break;
        default:
            WITH_FACE_RULE(g.frule,
                launch_split(k_apply_zs<T, MODE, false, 2, FRV>, grid, block, s, g, zt, rho, m, x, b, y, partials));
            break;
    }
}
template <typename T, bool DOT, bool RESID, bool ZG>
static void launch_rbgs_zs(const Geo<T>& g, const ZTiles& zt, const T* rho, const T* m, const T* r, T* z,
                           int colour, double* partials, T* tout, hipStream_t s) {
    const int hx = g.nx >> 1;
    const dim3 grid(zt.tx * zt.ty * zt.tz), block = split_block(hx);
    switch (split_shape(hx)) {
        case SPLIT_FULL1:
            WITH_FACE_RULE(g.frule,
                launch_split(k_rbgs_zs<T, DOT, RESID, ZG, true, 1, FRV>, grid, block, s, g, zt, rho, m, r, z, colour,
                         partials, tout));
            break;
        case SPLIT_FULL2:
            WITH_FACE_RULE(g.frule,
                launch_split(k_rbgs_zs<T, DOT, RESID, ZG, true, 2, FRV>, grid, block, s, g, zt, rho, m, r, z, colour,
                         partials, tout));
            break;
        default:
            WITH_FACE_RULE(g.frule,
                launch_split(k_rbgs_zs<T, DOT, RESID, ZG, false, 2, FRV>, grid, block, s, g, zt, rho, m, r, z, colour,
                         partials, tout));
            break;
    }
}
template <typename T, bool UPD = false>
static void launch_presmooth_zs(const Geo<T>& g, const ZTiles& zt, const T* rho, const T* dinv, const T* r,
                                T* z, hipStream_t s, const T* q = nullptr, T* rn = nullptr,
                                const RedCtl& rc = RedCtl{}) {
    const int hx = g.nx >> 1;
    const dim3 grid(zt.tx * zt.ty * zt.tz), block = split_block(hx);
    switch (split_shape(hx)) {
        case SPLIT_FULL1:
            WITH_FACE_RULE(g.frule,
                hipLaunchKernelGGL((k_presmooth_zs<T, true, 1, UPD, FRV>), grid, block, 0, s, g, zt, rho, dinv, r, z, q,
                               rn, rc));
            break;
        case SPLIT_FULL2:
            WITH_FACE_RULE(g.frule,
                hipLaunchKernelGGL((k_presmooth_zs<T, true, 2, UPD, FRV>), grid, block, 0, s, g, zt, rho, dinv, r, z, q,
                               rn, rc));
            break;
        default:
            WITH_FACE_RULE(g.frule,
                hipLaunchKernelGGL((k_presmooth_zs<T, false, 2, UPD, FRV>), grid, block, 0, s, g, zt, rho, dinv, r, z, q,
                               rn, rc));
            break;
    }
}

// The residual update r' = r - alpha q of a CG iteration with ||r'||^2 (under rc), folded into
// the zero-guess pre-smoothing z of the next V-cycle on a split level; returns the number of
// partials
template <typename T>
int launch_presmooth_update(const Geo<T>& g, const T* rho, const T* dinv, const T* r, const T* q, T* rn, T* z,
                            const RedCtl& rc, hipStream_t s) {
    ZTiles zt = split_tiles(g.nx >> 1, g.ny, g.nz);
    zt.rev = g.rev;
    launch_presmooth_zs<T, true>(g, zt, rho, dinv, r, z, s, q, rn, rc);
    return zt.tx * zt.ty * zt.tz;
}

static bool use_zm(int nx, int ny, int nz) { return nx >= 64 && ny >= 4 && nz >= 8; }

void launch_jacobi_diag(const Geo<double>& g, const Geo<float>& g32, const double* rho,
                        const double* m, const float* rho32, const float* m32, double* dinv,
                        float* dinv32, bool split_out, hipStream_t s) {
    if (use_zm(g.nx, g.ny, g.nz)) {
        const ZTiles zt = ztiles(g.nx, g.ny, g.nz, 64);
        const dim3 grid(zt.tx * zt.ty * zt.tz), block(kBlock);
        if (split_out)
            WITH_FACE_RULE(g.frule, hipLaunchKernelGGL((k_jacobi_diag_zm<FRV, true>), grid, block, 0, s, g,
                                                       g32, zt, rho, m, dinv, dinv32));
        else
            WITH_FACE_RULE(g.frule, hipLaunchKernelGGL((k_jacobi_diag_zm<FRV, false>), grid, block, 0, s, g,
                                                       g32, zt, rho, m, dinv, dinv32));
        return;
    }
    Shape3 sh = cells_shape(g.nx, g.ny, g.nz);
    hipLaunchKernelGGL(k_jacobi_diag, sh.grid, sh.block, 0, s, g, g32, rho, m, rho32, m32, dinv, dinv32,
                       split_out ? 1 : 0);
}
// largest workgroup count of the reducing z-march launches of a level (one partial per group):
// cells (x width 64), cell pairs (width 128) and the split layout (64 half positions)
static int64_t zm_blocks(int nx, int ny, int nz) {
    int64_t nb = 0;
    for (int v = 0; v < 3; ++v) {
        ZTiles t = v == 0 ? ztiles(nx, ny, nz, 64) : v == 1 ? ztiles(nx, ny, nz, 128)
                                                             : split_tiles(std::max(nx >> 1, 1), ny, nz);
        nb = std::max<int64_t>(nb, (int64_t)t.tx * t.ty * t.tz);
    }
    return nb;
}

// pair kernels: z-march shape, nx even and every array aligned for 2-vector access
template <typename T>
static bool use_zp(const Geo<T>& g, std::initializer_list<const T*> arrays) {
    if (sizeof(T) != 8 || !use_zm(g.nx, g.ny, g.nz) || (g.nx & 1)) return false;
    for (const T* p : arrays)
        if (p && (reinterpret_cast<uintptr_t>(p) % (2 * sizeof(T))) != 0) return false;
    return true;
}

template <typename T>
void launch_apply(const Geo<T>& g, const T* rho, const T* m, const T* x, const T* b, T* y,
                  int mode, const RedCtl& rc, hipStream_t s) {
    int nb;
    if (g.split) {
        ZTiles zt = split_tiles(g.nx >> 1, g.ny, g.nz);
        zt.rev = g.rev;
        nb = zt.tx * zt.ty * zt.tz;
        switch (mode) {
            case 0: launch_apply_zs<T, 0>(g, zt, rho, m, x, b, y, rc.partials, s); break;
            case 1: launch_apply_zs<T, 1>(g, zt, rho, m, x, b, y, rc.partials, s); break;
            case 2: launch_apply_zs<T, 2>(g, zt, rho, m, x, b, y, rc.partials, s); break;
            default: launch_apply_zs<T, 3>(g, zt, rho, m, x, b, y, rc.partials, s); break;
        }
    } else if (use_zp(g, {rho, m, x, b, y})) {
        ZTiles zt = ztiles(g.nx, g.ny, g.nz, 128);
        zt.rev = g.rev;
        nb = zt.tx * zt.ty * zt.tz;
        dim3 grid(nb), block(kBlock);
        WITH_FACE_RULE(g.frule, switch (mode) {
            case 0: hipLaunchKernelGGL((k_apply_zp<T, 0, FRV>), grid, block, 0, s, g, zt, rho, m, x, b, y, rc.partials); break;
            case 1: hipLaunchKernelGGL((k_apply_zp<T, 1, FRV>), grid, block, 0, s, g, zt, rho, m, x, b, y, rc.partials); break;
            case 2: hipLaunchKernelGGL((k_apply_zp<T, 2, FRV>), grid, block, 0, s, g, zt, rho, m, x, b, y, rc.partials); break;
            default: hipLaunchKernelGGL((k_apply_zp<T, 3, FRV>), grid, block, 0, s, g, zt, rho, m, x, b, y, rc.partials); break;
        });
    } else if (use_zm(g.nx, g.ny, g.nz)) {
        ZTiles zt = ztiles(g.nx, g.ny, g.nz, 64);
        zt.rev = g.rev;
        nb = zt.tx * zt.ty * zt.tz;
        dim3 grid(nb), block(kBlock);
        WITH_FACE_RULE(g.frule, switch (mode) {
            case 0: hipLaunchKernelGGL((k_apply_zm<T, 0, FRV>), grid, block, 0, s, g, zt, rho, m, x, b, y, rc.partials); break;
            case 1: hipLaunchKernelGGL((k_apply_zm<T, 1, FRV>), grid, block, 0, s, g, zt, rho, m, x, b, y, rc.partials); break;
            case 2: hipLaunchKernelGGL((k_apply_zm<T, 2, FRV>), grid, block, 0, s, g, zt, rho, m, x, b, y, rc.partials); break;
            default: hipLaunchKernelGGL((k_apply_zm<T, 3, FRV>), grid, block, 0, s, g, zt, rho, m, x, b, y, rc.partials); break;
        });
    } else {
        Shape3 sh = cells_shape(g.nx, g.ny, g.nz);
        nb = sh.grid.x * sh.grid.y * sh.grid.z;
        WITH_FACE_RULE(g.frule, switch (mode) {
            case 0: hipLaunchKernelGGL((k_apply<T, 0, FRV>), sh.grid, sh.block, 0, s, g, rho, m, x, b, y, rc); break;
            case 1: hipLaunchKernelGGL((k_apply<T, 1, FRV>), sh.grid, sh.block, 0, s, g, rho, m, x, b, y, rc); break;
            case 2: hipLaunchKernelGGL((k_apply<T, 2, FRV>), sh.grid, sh.block, 0, s, g, rho, m, x, b, y, rc); break;
            default: hipLaunchKernelGGL((k_apply<T, 3, FRV>), sh.grid, sh.block, 0, s, g, rho, m, x, b, y, rc); break;
        });
    }
    if (mode == 1 || mode == 3) finalize(rc, nb, s);
}

// ------------------------------------------------------------------------------------------
// red-black Gauss-Seidel

template <typename T, int FR = 0>
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
        const T zn = z[nb];  // at a missing face the cell's own old value, which must not count
        T w = c * face_kappa<FR>(ra, rho[nb]);
        sw += w;
        swz += w * (c != T(0) ? zn : T(0));
    });
    z[a] = (r[a] + swz) / (m[a] + sw);
}

// First red half sweep from z = 0: red cells r/D, black cells 0 (writes every cell).
template <typename T, int FR = 0>
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
    for_faces(g, i, j, k, a, [&](int nb, T c) { sw += c * face_kappa<FR>(ra, rho[nb]); });
    z[a] = r[a] / (m[a] + sw);
}

// Z-marching red-black half sweep: each thread owns the cell pair (i0, i0+1) of one row and
// updates, plane by plane, the member of colour `colour` (the colour alternates with k). The
// z neighbours of the updated cell are the other-colour cells of the pairs one plane up and
// down, which this sweep never writes, so they are kept in registers. The loads of plane k+1
// (the in-plane neighbours of its active member, its r and m, the pair two planes up) are
// issued before plane k is computed. ZERO: first red sweep from z = 0 (red cells r / D, black
// cells 0; no z loads).
// DOT: also reduce <r, z> over every cell with the final values (the other member's z is
// unchanged by the sweep), one partial per workgroup.
// RESID: instead of updating z, write the residual t = r - A z of the cells of `colour` to `t`
// and 0 for the other colour (exact right after a Gauss-Seidel half sweep of the other colour).
template <typename T, bool ZERO, bool DOT, bool RESID, int FR = 0>
__global__ __launch_bounds__(kBlock) void k_rbgs_zm(Geo<T> g, ZTiles zt,
                                                    const T* __restrict__ rho,
                                                    const T* __restrict__ m,
                                                    const T* __restrict__ r, T* __restrict__ z,
                                                    int colour, double* __restrict__ partials,
                                                    T* __restrict__ t = nullptr) {
    int bx, by, bz;
    ztile(zt, bx, by, bz);
    const int i0 = (bx * 64 + (threadIdx.x & 63)) * 2;
    const int j = by * 4 + (threadIdx.x >> 6);
    double dsum = 0.0;
    if (i0 < g.nx && j < g.ny) {
    const int k0 = bz * zt.kz;
    const int k1 = min(k0 + zt.kz, g.nz);
    const int sz = g.nx * g.ny;
    const int d1 = (i0 + 1 < g.nx) ? 1 : 0;  // 0: the pair has one cell only
    const FaceTab<T> f0(g, i0, j), f1(g, i0 + d1, j);
    const int col = i0 + g.nx * j;
    int a = col + k0 * sz;
    bool hm, hp;
    const int om = zoff(k0, -1, g.nz, g.pz, sz, hm);
    const int op = zoff(k0, 1, g.nz, g.pz, sz, hp);
    T czm = hm ? g.cz : T(0), czp = hp ? g.cz : T(0);
    // the pair at planes k-1 (m), k (c), k+1 (n)
    T rc0 = rho[a], rc1 = rho[a + d1];
    T rm0 = rho[a + om], rm1 = rho[a + om + d1];
    T rn0 = rho[a + op], rn1 = rho[a + op + d1];
    T zc0 = T(0), zc1 = T(0), zm0 = T(0), zm1 = T(0), zn0 = T(0), zn1 = T(0);
    if (!ZERO) {
        zc0 = z[a]; zc1 = z[a + d1];
        zm0 = z[a + om]; zm1 = z[a + om + d1];
        zn0 = z[a + op]; zn1 = z[a + op + d1];
    }
    int sel = (colour + j + k0) & 1;  // i0 is even: the active member of plane k0
    int o[4];
    T cf[4], rv[4], zv[4], rr, mm;
    {
        const int act = a + (sel & d1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            o[q] = sel ? f1.o[q] : f0.o[q];
            cf[q] = sel ? f1.c[q] : f0.c[q];
            rv[q] = rho[act + o[q]];
            zv[q] = ZERO ? T(0) : z[act + o[q]];
        }
        rr = r[act];
        mm = m[act];
    }
    for (int k = k0; k < k1; ++k) {
        const int seln = sel ^ 1;
        const int kn = min(k + 1, k1 - 1);
        const int an = col + kn * sz;
        bool hpn;
        const int opn = zoff(kn, 1, g.nz, g.pz, sz, hpn);
        // prefetch plane k+1 (its active member) and the pair two planes up
        int on[4];
        T cfn[4], rvn[4], zvn[4];
        const int actn = an + (seln & d1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            on[q] = seln ? f1.o[q] : f0.o[q];
            cfn[q] = seln ? f1.c[q] : f0.c[q];
            rvn[q] = rho[actn + on[q]];
            zvn[q] = ZERO ? T(0) : z[actn + on[q]];
        }
        const T rrn = r[actn], mmn = m[actn];
        const T rnn0 = rho[an + opn], rnn1 = rho[an + opn + d1];
        T znn0 = T(0), znn1 = T(0);
        if (!ZERO) {
            znn0 = z[an + opn];
            znn1 = z[an + opn + d1];
        }
        // plane k: update the active member
        const T ra = sel ? rc1 : rc0;
        T sw = T(0), swz = T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T w = cf[q] * face_kappa<FR>(ra, rv[q]);
            sw += w;
            swz += w * zv[q];
        }
        const T wzm = czm * face_kappa<FR>(ra, sel ? rm1 : rm0);
        const T wzp = czp * face_kappa<FR>(ra, sel ? rn1 : rn0);
        sw += wzm + wzp;
        swz += wzm * (sel ? zm1 : zm0) + wzp * (sel ? zn1 : zn0);
        if (RESID) {
            const T zs = sel ? zc1 : zc0;
            if (sel == 0 || d1) t[a + sel] = rr + swz - (mm + sw) * zs;
            if (seln == 0 || d1) t[a + seln] = T(0);
        }
        const T znew = RESID ? T(0) : (rr + swz) / (mm + sw);
        if (!RESID && (sel == 0 || d1)) z[a + sel] = znew;
        if (ZERO && (seln == 0 || d1)) z[a + seln] = T(0);
        if (DOT) {
            if (sel == 0 || d1) dsum += (double)rr * (double)znew;
            if (seln == 0 || d1) dsum += (double)r[a + seln] * (double)(seln ? zc1 : zc0);
        }
        // advance one plane. At plane k+1 the other pair member is updated; its z neighbours
        // are the members of planes k and k+2 that this sweep does not write, so the register
        // copies stay valid (the updated member's stale copy is never read again).
        czm = czp;
        czp = hpn ? g.cz : T(0);
        rm0 = rc0; rm1 = rc1;
        rc0 = rn0; rc1 = rn1;
        rn0 = rnn0; rn1 = rnn1;
        zm0 = zc0; zm1 = zc1;
        zc0 = zn0; zc1 = zn1;
        zn0 = znn0; zn1 = znn1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            o[q] = on[q];
            cf[q] = cfn[q];
            rv[q] = rvn[q];
            zv[q] = zvn[q];
        }
        rr = rrn;
        mm = mmn;
        sel = seln;
        a = an;
    }
    }
    if (DOT) block_partial(dsum, partials);
}

// Pre-smoothing from z = 0 in one pass: a red half sweep from zero gives z_red = r dinv (a
// pointwise value), so the following black half sweep can use r dinv of its red neighbours
// directly: z_black = dinv_b (r_b + sum_f w_f r_nb dinv_nb). Each thread owns a cell pair; the
// red-neighbour values q = r dinv of the pairs one plane up and down are kept in registers.
// Same result as the zero-guess red sweep followed by a black sweep.
template <typename T, int FR = 0>
__global__ __launch_bounds__(kBlock) void k_presmooth_zm(Geo<T> g, ZTiles zt,
                                                         const T* __restrict__ rho,
                                                         const T* __restrict__ dinv,
                                                         const T* __restrict__ r,
                                                         T* __restrict__ z) {
    int bx, by, bz;
    ztile(zt, bx, by, bz);
    const int i0 = (bx * 64 + (threadIdx.x & 63)) * 2;
    const int j = by * 4 + (threadIdx.x >> 6);
    if (i0 >= g.nx || j >= g.ny) return;
    const int k0 = bz * zt.kz;
    const int k1 = min(k0 + zt.kz, g.nz);
    const int sz = g.nx * g.ny;
    const int d1 = (i0 + 1 < g.nx) ? 1 : 0;
    const FaceTab<T> f0(g, i0, j), f1(g, i0 + d1, j);
    const int col = i0 + g.nx * j;
    int a = col + k0 * sz;
    bool hm, hp;
    const int om = zoff(k0, -1, g.nz, g.pz, sz, hm);
    const int op = zoff(k0, 1, g.nz, g.pz, sz, hp);
    T czm = hm ? g.cz : T(0), czp = hp ? g.cz : T(0);
    // pair values at planes k-1 (m), k (c), k+1 (n): rho and q = r * dinv
    T rc0 = rho[a], rc1 = rho[a + d1];
    T rm0 = rho[a + om], rm1 = rho[a + om + d1];
    T rn0 = rho[a + op], rn1 = rho[a + op + d1];
    T qc0 = r[a] * dinv[a], qc1 = r[a + d1] * dinv[a + d1];
    T qm0 = r[a + om] * dinv[a + om], qm1 = r[a + om + d1] * dinv[a + om + d1];
    T qn0 = r[a + op] * dinv[a + op], qn1 = r[a + op + d1] * dinv[a + op + d1];
    for (int k = k0; k < k1; ++k) {
        const int red = (j + k) & 1;   // pair member of colour red (i0 is even)
        const int blk = red ^ 1;
        const int kn = min(k + 1, k1 - 1);
        const int an = col + kn * sz;
        bool hpn;
        const int opn = zoff(kn, 1, g.nz, g.pz, sz, hpn);
        // prefetch the pair two planes up
        const T rnn0 = rho[an + opn], rnn1 = rho[an + opn + d1];
        const T qnn0 = r[an + opn] * dinv[an + opn];
        const T qnn1 = r[an + opn + d1] * dinv[an + opn + d1];
        // black member: in-plane neighbours are red, z neighbours are the red members up/down
        const int ab = a + blk;
        int o[4];
        T cf[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            o[q] = blk ? f1.o[q] : f0.o[q];
            cf[q] = blk ? f1.c[q] : f0.c[q];
        }
        const T rb = blk ? rc1 : rc0;
        T sw = T(0), swq = T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T w = cf[q] * face_kappa<FR>(rb, rho[ab + o[q]]);
            sw += w;
            swq += w * (r[ab + o[q]] * dinv[ab + o[q]]);
        }
        const T wzm = czm * face_kappa<FR>(rb, blk ? rm1 : rm0);
        const T wzp = czp * face_kappa<FR>(rb, blk ? rn1 : rn0);
        swq += wzm * (blk ? qm1 : qm0) + wzp * (blk ? qn1 : qn0);
        const T zb = (r[ab] + swq) * dinv[ab];
        if (red == 0 || d1) z[a + red] = red ? qc1 : qc0;
        if (blk == 0 || d1) z[ab] = zb;
        (void)sw;
        // advance one plane
        czm = czp;
        czp = hpn ? g.cz : T(0);
        rm0 = rc0; rm1 = rc1;
        rc0 = rn0; rc1 = rn1;
        rn0 = rnn0; rn1 = rnn1;
        qm0 = qc0; qm1 = qc1;
        qc0 = qn0; qc1 = qn1;
        qn0 = qnn0; qn1 = qnn1;
        a = an;
    }
}

// residual after a black half sweep: t = r - A z on red cells, 0 on black cells
template <typename T>
bool launch_resid_red(const Geo<T>& g, const T* rho, const T* m, const T* r, const T* z, T* t,
                      hipStream_t s, bool zero_guess) {
    if (g.split) {
        ZTiles zt = split_tiles(g.nx >> 1, g.ny, g.nz);
        zt.rev = g.rev;
        if (zero_guess)
            launch_rbgs_zs<T, false, true, true>(g, zt, rho, m, r, const_cast<T*>(z), 0, nullptr, t, s);
        else
            launch_rbgs_zs<T, false, true, false>(g, zt, rho, m, r, const_cast<T*>(z), 0, nullptr, t, s);
        return true;
    }
    if (!use_zm(g.nx, g.ny, g.nz)) return false;
    ZTiles zt = ztiles(g.nx, g.ny, g.nz, 128);
    zt.rev = g.rev;
    WITH_FACE_RULE(g.frule,
        hipLaunchKernelGGL((k_rbgs_zm<T, false, false, true, FRV>), dim3(zt.tx * zt.ty * zt.tz), dim3(kBlock), 0,
                       s, g, zt, rho, m, r, const_cast<T*>(z), 0, nullptr, t));
    return true;
}

// Zero-guess pre-smoothing in one pass over the cells of a level too small for the z march:
// red cells z = r dinv, black cells dinv (r + sum_f w_f (r dinv)_nb) (their neighbours are red).
template <typename T, int FR = 0>
__global__ __launch_bounds__(kBlock) void k_presmooth(Geo<T> g, const T* __restrict__ rho,
                                                      const T* __restrict__ dinv, const T* __restrict__ r,
                                                      T* __restrict__ z) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= g.nx || j >= g.ny || k >= g.nz) return;
    const int a = i + g.nx * (j + g.ny * k);
    if (!((i + j + k) & 1)) {
        z[a] = r[a] * dinv[a];
        return;
    }
    const T ra = rho[a];
    T swq = T(0);
    for_faces(g, i, j, k, a, [&](int nb, T c) { swq += c * face_kappa<FR>(ra, rho[nb]) * (r[nb] * dinv[nb]); });
    z[a] = (r[a] + swq) * dinv[a];
}

template <typename T>
bool launch_presmooth(const Geo<T>& g, const T* rho, const T* dinv, const T* r, T* z, hipStream_t s) {
    if (g.split) {
        ZTiles zt = split_tiles(g.nx >> 1, g.ny, g.nz);
        zt.rev = g.rev;
        launch_presmooth_zs<T>(g, zt, rho, dinv, r, z, s);
        return true;
    }
    if (!use_zm(g.nx, g.ny, g.nz)) {
        const Shape3 sh = cells_shape(g.nx, g.ny, g.nz);
        WITH_FACE_RULE(g.frule,
            hipLaunchKernelGGL((k_presmooth<T, FRV>), sh.grid, sh.block, 0, s, g, rho, dinv, r, z));
        return true;
    }
    ZTiles zt = ztiles(g.nx, g.ny, g.nz, 128);
    zt.rev = g.rev;
    WITH_FACE_RULE(g.frule,
        hipLaunchKernelGGL((k_presmooth_zm<T, FRV>), dim3(zt.tx * zt.ty * zt.tz), dim3(kBlock), 0, s, g, zt, rho,
                       dinv, r, z));
    return true;
}

template <typename T>
void launch_rbgs(const Geo<T>& g, const T* rho, const T* m, const T* r, T* z, int colour,
                 hipStream_t s) {
    if (g.split) {
        ZTiles zt = split_tiles(g.nx >> 1, g.ny, g.nz);
        zt.rev = g.rev;
        launch_rbgs_zs<T, false, false, false>(g, zt, rho, m, r, z, colour, nullptr, nullptr, s);
        return;
    }
    if (use_zm(g.nx, g.ny, g.nz)) {
        ZTiles zt = ztiles(g.nx, g.ny, g.nz, 128);
        zt.rev = g.rev;
        WITH_FACE_RULE(g.frule,
            hipLaunchKernelGGL((k_rbgs_zm<T, false, false, false, FRV>), dim3(zt.tx * zt.ty * zt.tz), dim3(kBlock), 0,
                           s, g, zt, rho, m, r, z, colour, nullptr));
        return;
    }
    Shape3 sh = cells_shape((g.nx + 1) / 2, g.ny, g.nz);
    WITH_FACE_RULE(g.frule,
        hipLaunchKernelGGL((k_rbgs<T, FRV>), sh.grid, sh.block, 0, s, g, rho, m, r, z, colour));
}

// Split layout: the half sweep of `colour` reducing <r, z> over its own cells into partials
// (no second stage); returns the number of partials.
template <typename T>
int launch_rbgs_own_dot(const Geo<T>& g, const T* rho, const T* m, const T* r, T* z, int colour,
                        double* partials, hipStream_t s) {
    ZTiles zt = split_tiles(g.nx >> 1, g.ny, g.nz);
    zt.rev = g.rev;
    launch_rbgs_zs<T, true, false, false>(g, zt, rho, m, r, z, colour, partials, nullptr, s);
    return zt.tx * zt.ty * zt.tz;
}

// The last half sweep of a post-smoothing with <r, z> over every cell: in the split layout the
// earlier (other-colour) sweep left nb2 partials of its own cells in partials2; otherwise the
// z-march sweep reduces both colours itself.
template <typename T>
bool launch_rbgs_dot(const Geo<T>& g, const T* rho, const T* m, const T* r, T* z, int colour,
                     const RedCtl& rc, hipStream_t s, const double* partials2, int nb2) {
    if (g.split) {
        const int nb = launch_rbgs_own_dot<T>(g, rho, m, r, z, colour, rc.partials, s);
        finalize(rc, nb, s, partials2, nb2);
        return true;
    }
    if (!use_zm(g.nx, g.ny, g.nz)) return false;
    ZTiles zt = ztiles(g.nx, g.ny, g.nz, 128);
    zt.rev = g.rev;
    const int nb = zt.tx * zt.ty * zt.tz;
    WITH_FACE_RULE(g.frule,
        hipLaunchKernelGGL((k_rbgs_zm<T, false, true, false, FRV>), dim3(nb), dim3(kBlock), 0, s, g, zt, rho, m, r, z,
                       colour, rc.partials));
    finalize(rc, nb, s);
    return true;
}

template <typename T>
void launch_rbgs_zero(const Geo<T>& g, const T* rho, const T* m, const T* r, T* z,
                      hipStream_t s) {
    if (g.split) {
        launch_fill<T>(z, T(0), (int64_t)g.nx * g.ny * g.nz, s);
        launch_rbgs<T>(g, rho, m, r, z, 0, s);
        return;
    }
    if (use_zm(g.nx, g.ny, g.nz)) {
        ZTiles zt = ztiles(g.nx, g.ny, g.nz, 128);
        zt.rev = g.rev;
        WITH_FACE_RULE(g.frule,
            hipLaunchKernelGGL((k_rbgs_zm<T, true, false, false, FRV>), dim3(zt.tx * zt.ty * zt.tz), dim3(kBlock), 0,
                           s, g, zt, rho, m, r, z, 0, nullptr));
        return;
    }
    Shape3 sh = cells_shape(g.nx, g.ny, g.nz);
    WITH_FACE_RULE(g.frule,
        hipLaunchKernelGGL((k_rbgs_zero<T, FRV>), sh.grid, sh.block, 0, s, g, rho, m, r, z));
}

// ------------------------------------------------------------------------------------------
// transfers

// Fine taps of coarse index I along one axis for R = P^T / 2 (P: weights 3/4 parent, 1/4 the
// second-nearest coarse cell; mirrored at a Neumann end, wrapped on a periodic axis).
// Fine taps of coarse index I along one axis for R = P^T / 2: always four (index, weight)
// pairs; missing taps (Neumann ends, an uncoarsened axis) get weight 0 and an in-range index, so
// the restriction is straight-line code with all its loads independent.
__device__ __forceinline__ void restrict_taps(int I, int nf, int coarsened, int periodic, int* idx,
                                              float* w) {
    if (!coarsened) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            idx[s] = I;
            w[s] = s == 0 ? 1.0f : 0.0f;
        }
        return;
    }
    const int nc = nf >> 1;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        int i = 2 * I - 1 + s;
        if (i < 0 || i >= nf) {
            if (!periodic) {
                idx[s] = 2 * I;
                w[s] = 0.0f;
                continue;
            }
            i = (i + nf) % nf;
        }
        int parent = i >> 1;
        int other = (i & 1) ? parent + 1 : parent - 1;
        if (other < 0 || other >= nc) other = periodic ? (other + nc) % nc : parent;
        float p = (parent == I ? 0.75f : 0.0f) + (other == I ? 0.25f : 0.0f);
        idx[s] = i;
        w[s] = 0.5f * p;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_restrict(Transfer t, const T* __restrict__ fine,
                                                     T* __restrict__ coarse) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    int J = blockIdx.y * blockDim.y + threadIdx.y;
    int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (I >= t.ncx || J >= t.ncy || K >= t.ncz) return;
    int ix[4], iy[4], iz[4];
    float wx[4], wy[4], wz[4];
    restrict_taps(I, t.nfx, t.fx, t.perx, ix, wx);
    restrict_taps(J, t.nfy, t.fy, t.pery, iy, wy);
    restrict_taps(K, t.nfz, t.fz, t.perz, iz, wz);
    // all 64 loads first (these levels are small: what counts is that they are in flight together)
    T v[4][4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const T* row = fine + (int64_t)t.nfx * (iy[b] + (int64_t)t.nfy * iz[c]);
#pragma unroll
            for (int q = 0; q < 4; ++q) v[c][b][q] = row[ix[q]];
        }
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        T accy = T(0);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            T accx = T(0);
#pragma unroll
            for (int q = 0; q < 4; ++q) accx += (T)wx[q] * v[c][b][q];
            accy += (T)wy[b] * accx;
        }
        acc += (T)wz[c] * accy;
    }
    coarse[I + (int64_t)t.ncx * (J + (int64_t)t.ncy * K)] = acc;
}

// ---- z-marching transfers for levels coarsened on all three axes ----
// Weights of the four fine positions 2I-1, 2I, 2I+1, 2I+2 of coarse index I along one axis for
// R = P^T / 2 (same rule as restrict_taps: Neumann ends folded onto the parent, periodic wrap).
__device__ __forceinline__ void rweights4(int I, int nf, int periodic, float* w) {
    const int nc = nf >> 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int i = 2 * I - 1 + q;
        if (i < 0 || i >= nf) {
            if (!periodic) { w[q] = 0.0f; continue; }
            i = (i + nf) % nf;
        }
        int parent = i >> 1;
        int other = (i & 1) ? parent + 1 : parent - 1;
        if (other < 0 || other >= nc) other = periodic ? (other + nc) % nc : parent;
        w[q] = 0.5f * ((parent == I ? 0.75f : 0.0f) + (other == I ? 0.25f : 0.0f));
    }
}

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// One thread per coarse column (I, J), 64 consecutive I per wave, one coarse row per wave, a
// chunk of coarse planes per workgroup. The thread loads the fine pair (2I, 2I+1) of each of the
// four fine rows as one 16-byte vector and takes 2I-1 / 2I+2 from its neighbour lanes; the
// x-y weighted sum u(k) of each fine plane is reused by the two coarse planes it feeds.
// SPLIT: the fine level uses the red-black split layout (the pair (2I, 2I+1) of a fine row sits
// at half position I of its two halves); RED_ONLY: its black cells are zero and not read.
// Index of coarse cell (I, J, K) in natural order or, CSPLIT, in the red-black split layout.
template <bool CSPLIT>
__device__ __forceinline__ int64_t coarse_idx(const Transfer& t, int I, int J, int K) {
    const int64_t rb = ((int64_t)K * t.ncy + J) * t.ncx;
    if (!CSPLIT) return rb + I;
    return rb + ((I + J + K) & 1) * (t.ncx >> 1) + (I >> 1);
}

template <typename T, bool SPLIT, bool RED_ONLY, bool CSPLIT = false>
__global__ __launch_bounds__(kBlock) void k_restrict_zm(Transfer t, ZTiles zt,
                                                        const T* __restrict__ fine,
                                                        T* __restrict__ coarse) {
    int bx, by, bz;
    ztile(zt, bx, by, bz);
    const int lane = threadIdx.x & 63;
    const int I = bx * 64 + lane;
    const int J = by * 4 + (threadIdx.x >> 6);
    const bool valid = I < t.ncx && J < t.ncy;
    const int Ic = valid ? I : t.ncx - 1, Jc = J < t.ncy ? J : t.ncy - 1;
    const int K0 = bz * zt.kz, K1 = min(K0 + zt.kz, t.ncz);
    const int nfx = t.nfx, nfy = t.nfy, nfz = t.nfz;
    const int sf = nfx * nfy;
    float wx[4], wy[4];
    rweights4(Ic, nfx, t.perx, wx);
    rweights4(Jc, nfy, t.pery, wy);
    int row[4], jr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        jr[q] = wrapi(2 * Jc - 1 + q, nfy);  // rows with w 0 are harmless
        row[q] = jr[q] * nfx;
    }
    const int xl = wrapi(2 * Ic - 1, nfx), xr = wrapi(2 * Ic + 2, nfx);
    const bool edge_l = (lane == 0) || (Ic == 0), edge_r = (lane == 63) || (Ic == t.ncx - 1);
    const int hf = nfx >> 1;
    auto plane_sum = [&](int k) -> T {
        // weighted x-y sum of fine plane k (k already wrapped / valid)
        const T* base = fine + (int64_t)k * sf;
        T u = T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T* rp = base + row[q];
            T f0, f1, left, right;
            if (SPLIT) {
                // cell 2I has the row's parity as colour; 2I-1 the other one, 2I+2 the same
                const int pf = (jr[q] + k) & 1;
                if (RED_ONLY) {
                    const T v = rp[Ic];
                    f0 = pf ? T(0) : v;
                    f1 = pf ? v : T(0);
                } else {
                    f0 = rp[pf * hf + Ic];
                    f1 = rp[(1 - pf) * hf + Ic];
                }
                left = __shfl_up(f1, 1, 64);
                right = __shfl_down(f0, 1, 64);
                if (edge_l) left = (RED_ONLY && !pf) ? T(0) : rp[(1 - pf) * hf + (xl >> 1)];
                if (edge_r) right = (RED_ONLY && pf) ? T(0) : rp[pf * hf + (xr >> 1)];
            } else {
                f0 = rp[2 * Ic];
                f1 = rp[2 * Ic + 1];
                left = __shfl_up(f1, 1, 64);
                right = __shfl_down(f0, 1, 64);
                if (edge_l) left = rp[xl];
                if (edge_r) right = rp[xr];
            }
            u += (T)wy[q] * ((T)wx[0] * left + (T)wx[1] * f0 + (T)wx[2] * f1 + (T)wx[3] * right);
        }
        return u;
    };
    // u of fine planes 2K0-1 and 2K0; plane indices wrap, so a missing Neumann plane reads a
    // valid plane that then gets weight 0
    T u0 = plane_sum(wrapi(2 * K0 - 1, nfz));
    T u1 = plane_sum(wrapi(2 * K0, nfz));
    for (int K = K0; K < K1; ++K) {
        float w[4];
        rweights4(K, nfz, t.perz, w);
        const T u2 = plane_sum(wrapi(2 * K + 1, nfz));
        const T u3 = plane_sum(wrapi(2 * K + 2, nfz));
        if (valid)
            coarse[coarse_idx<CSPLIT>(t, I, J, K)] = (T)w[0] * u0 + (T)w[1] * u1 + (T)w[2] * u2 + (T)w[3] * u3;
        // the next coarse plane starts at fine plane 2K+1
        u0 = u2;
        u1 = u3;
    }
}

static bool transfer_zm(const Transfer& t) {
    return t.fx && t.fy && t.fz && t.ncx >= 32 && t.ncy >= 4 && t.ncz >= 4;
}

// Red-only restriction from a split fine level (the residual after a zero-guess pre-smoothing
// vanishes on black cells): one thread per coarse column (I, J), 64 consecutive I per wave, one
// coarse row per wave, a chunk of coarse planes per workgroup. Each fine plane's ten fine rows
// under the workgroup's four coarse rows are loaded once (a few rows per wave), weighted in x
// (neighbour cells from the adjacent lanes) and put in LDS, where each coarse row sums its four
// rows with the y weights; the x-y sums u(k) of the fine planes then combine in z, each reused
// by the two coarse planes it feeds. The next fine plane's red entries are loaded while the
// current one is summed. The weights and their order are those of k_restrict_zm.
template <typename T, bool CSPLIT>
__global__ __launch_bounds__(kBlock) void k_restrict_red(Transfer t, ZTiles zt, const T* __restrict__ fine,
                                                         T* __restrict__ coarse) {
    constexpr int NR = 10;            // fine rows under four coarse rows
    __shared__ T sx[2][NR][64];       // [slot][fine row 2 J0 - 1 + r][lane]: x-weighted sums
    int bx, by, bz;
    ztile(zt, bx, by, bz);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int I = bx * 64 + lane;
    const int J0 = by * 4, J = J0 + w;
    const bool valid = I < t.ncx && J < t.ncy;
    const int Ic = I < t.ncx ? I : t.ncx - 1, Jc = J < t.ncy ? J : t.ncy - 1;
    const int K0 = bz * zt.kz, K1 = min(K0 + zt.kz, t.ncz);
    const int nfx = t.nfx, nfy = t.nfy, nfz = t.nfz;
    const int64_t sf = (int64_t)nfx * nfy;
    float wx[4], wy[4];
    rweights4(Ic, nfx, t.perx, wx);
    rweights4(Jc, nfy, t.pery, wy);
    // fine rows this wave loads: 2 J0 - 1 + w + 4 i (rows with w 0 are harmless)
    int jr[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) jr[i] = wrapi(min(2 * J0 - 1 + w + 4 * i, 2 * J0 - 1 + NR - 1), nfy);
    const int nri = w + 8 < NR ? 3 : 2;
    const int hl = wrapi(2 * Ic - 1, nfx) >> 1, hr = wrapi(2 * Ic + 2, nfx) >> 1;
    const bool edge_l = (lane == 0) || (Ic == 0), edge_r = (lane == 63) || (Ic == t.ncx - 1);
    // red entries at half position Ic of this wave's rows of one fine plane and the red outer
    // neighbour that a wave edge needs (cell 2I-1 is red where the row parity is 1, cell 2I+2
    // where it is 0). Every lane issues every load (valid rows and columns; what a lane does not
    // need it ignores): with loads under a branch the compiler cannot count what is in flight, and
    // waited for the next plane's loads before using the current ones.
    struct Raw {
        T c[3], e[3];
    };
    auto load_rows = [&](int k, Raw& o) {
        const T* base = fine + (int64_t)k * sf;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const T* rp = base + (int64_t)jr[i] * nfx;
            const int pf = (jr[i] + k) & 1;
            o.c[i] = rp[Ic];
            o.e[i] = rp[pf ? hl : hr];
        }
    };
    // x-y weighted sum of fine plane k from the entries in cur; loads plane kn into nxt
    auto fstep = [&](int k, int kn, int sl, const Raw& cur, Raw& nxt) -> T {
        load_rows(kn, nxt);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (i < nri) {
                const int pf = (jr[i] + k) & 1;
                const T v = cur.c[i];
                const T f0 = pf ? T(0) : v, f1 = pf ? v : T(0);
                T left = __shfl_up(f1, 1, 64), right = __shfl_down(f0, 1, 64);
                if (edge_l) left = pf ? cur.e[i] : T(0);
                if (edge_r) right = pf ? T(0) : cur.e[i];
                sx[sl][w + 4 * i][lane] = (T)wx[0] * left + (T)wx[1] * f0 + (T)wx[2] * f1 + (T)wx[3] * right;
            }
        }
        __syncthreads();
        T u = T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) u += (T)wy[q] * sx[sl][min(2 * w + q, NR - 1)][lane];
        return u;
    };
    // fine planes 2 K0 - 1, 2 K0, 2 K0 + 1, ... (indices wrap, so a missing Neumann plane reads a
    // valid plane that then gets weight 0)
    Raw A, B;
    load_rows(wrapi(2 * K0 - 1, nfz), A);
    T u0 = fstep(wrapi(2 * K0 - 1, nfz), wrapi(2 * K0, nfz), 0, A, B);
    T u1 = fstep(wrapi(2 * K0, nfz), wrapi(2 * K0 + 1, nfz), 1, B, A);
    for (int K = K0; K < K1; ++K) {
        const T u2 = fstep(wrapi(2 * K + 1, nfz), wrapi(2 * K + 2, nfz), 0, A, B);
        const T u3 = fstep(wrapi(2 * K + 2, nfz), wrapi(min(2 * K + 3, 2 * nfz - 1), nfz), 1, B, A);
        float wz[4];
        rweights4(K, nfz, t.perz, wz);
        if (valid)
            coarse[coarse_idx<CSPLIT>(t, I, J, K)] = (T)wz[0] * u0 + (T)wz[1] * u1 + (T)wz[2] * u2 + (T)wz[3] * u3;
        // the next coarse plane starts at fine plane 2K+1
        u0 = u2;
        u1 = u3;
    }
}

template <typename T>
void launch_restrict(const Transfer& t, const T* fine, T* coarse, hipStream_t s, bool red_only) {
    if (transfer_zm(t)) {
        // the red-only restriction from 256^3 and up marches chunks of eight coarse planes (1024
        // workgroups at 256^3, resident at once; four-plane chunks take two rounds of workgroups)
        ZTiles zt = ztiles(t.ncx, t.ncy, t.ncz, 64, (red_only && t.ncz >= 128) ? 8 : 2);
        zt.rev = t.rev;
        const dim3 grid(zt.tx * zt.ty * zt.tz), block(kBlock);
        // a split coarse level always has a split fine level above it
        if (!t.fsplit)
            hipLaunchKernelGGL((k_restrict_zm<T, false, false>), grid, block, 0, s, t, zt, fine, coarse);
        else if (red_only && t.csplit)
            hipLaunchKernelGGL((k_restrict_red<T, true>), grid, block, 0, s, t, zt, fine, coarse);
        else if (red_only)
            hipLaunchKernelGGL((k_restrict_red<T, false>), grid, block, 0, s, t, zt, fine, coarse);
        else if (t.csplit)
            hipLaunchKernelGGL((k_restrict_zm<T, true, false, true>), grid, block, 0, s, t, zt, fine, coarse);
        else
            hipLaunchKernelGGL((k_restrict_zm<T, true, false>), grid, block, 0, s, t, zt, fine, coarse);
        return;
    }
    Shape3 sh = cells_shape(t.ncx, t.ncy, t.ncz);
    hipLaunchKernelGGL((k_restrict<T>), sh.grid, sh.block, 0, s, t, fine, coarse);
}

// Coarse taps of fine index i along one axis for P.
// Always two (index, weight) pairs: on an axis that is not coarsened the second has weight 0 and
// the first index again, so the prolongation is straight-line code with independent loads.
__device__ __forceinline__ void prolong_taps(int i, int nc, int coarsened, int periodic, int* idx,
                                             float* w) {
    if (!coarsened) {
        idx[0] = idx[1] = i;
        w[0] = 1.0f;
        w[1] = 0.0f;
        return;
    }
    int parent = i >> 1;
    int other = (i & 1) ? parent + 1 : parent - 1;
    if (other < 0 || other >= nc) other = periodic ? (other + nc) % nc : parent;
    idx[0] = parent;
    w[0] = 0.75f;
    idx[1] = other;
    w[1] = 0.25f;
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
    prolong_taps(i, t.ncx, t.fx, t.perx, ix, wx);
    prolong_taps(j, t.ncy, t.fy, t.pery, iy, wy);
    prolong_taps(k, t.ncz, t.fz, t.perz, iz, wz);
    T* out = fine + i + (int64_t)t.nfx * (j + (int64_t)t.nfy * k);
    const T f0 = *out;
    T v[2][2][2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const T* row = coarse + (int64_t)t.ncx * (iy[b] + (int64_t)t.ncy * iz[c]);
#pragma unroll
            for (int q = 0; q < 2; ++q) v[c][b][q] = row[ix[q]];
        }
    // a weight-0 tap adds an exact zero: the sums are those over the real taps alone
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        T accy = T(0);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            T accx = T(0);
#pragma unroll
            for (int q = 0; q < 2; ++q) accx += (T)wx[q] * v[c][b][q];
            accy += (T)wy[b] * accx;
        }
        acc += (T)wz[c] * accy;
    }
    *out = f0 + acc;
}

// One thread per fine cell pair (2I, 2I+1) of one fine row j, 64 pairs per wave, one fine row
// per wave, a chunk of fine planes (even start) per workgroup. Both cells have parent column I;
// the second-nearest column is I-1 for 2I and I+1 for 2I+1 (taken from the neighbour lanes).
// The x-y interpolation v(K) of coarse planes K-1, K, K+1 is kept in registers while marching.
// RED_ONLY (split layout): only the red cells are corrected, for a black half sweep that follows
// and overwrites every black cell without reading it.
template <typename T, bool SPLIT, bool RED_ONLY = false, bool CSPLIT = false>
__global__ __launch_bounds__(kBlock) void k_prolong_zm(Transfer t, ZTiles zt,
                                                       const T* __restrict__ coarse,
                                                       T* __restrict__ fine) {
    int bx, by, bz;
    ztile(zt, bx, by, bz);
    const int lane = threadIdx.x & 63;
    const int I = bx * 64 + lane;
    const int j = by * 4 + (threadIdx.x >> 6);
    const bool valid = I < t.ncx && j < t.nfy;
    const int Ic = I < t.ncx ? I : t.ncx - 1, jc = j < t.nfy ? j : t.nfy - 1;
    const int k0 = bz * zt.kz, k1 = min(k0 + zt.kz, t.nfz);
    const int ncx = t.ncx, ncy = t.ncy, ncz = t.ncz;
    const int sc = ncx * ncy;
    // x neighbours of the parent column (mirror onto the parent at a Neumann end)
    const int xm = Ic > 0 ? Ic - 1 : (t.perx ? ncx - 1 : Ic);
    const int xp = Ic < ncx - 1 ? Ic + 1 : (t.perx ? 0 : Ic);
    // y: parent row and second row
    const int J = jc >> 1;
    int J2 = (jc & 1) ? J + 1 : J - 1;
    if (J2 < 0 || J2 >= ncy) J2 = t.pery ? (J2 + ncy) % ncy : J;
    const int rowJ = J * ncx, rowJ2 = J2 * ncx;
    const bool edge_l = (lane == 0) || (Ic == 0), edge_r = (lane == 63) || (Ic == ncx - 1);
    // v(K) for the two fine columns
    auto cv = [&](int Ix, int Jy, int K) { return coarse[coarse_idx<CSPLIT>(t, Ix, Jy, K)]; };
    auto vplane = [&](int K, T& vlo, T& vhi) {
        const T cy = T(0.75) * cv(Ic, J, K) + T(0.25) * cv(Ic, J2, K);
        T cl = __shfl_up(cy, 1, 64), cr = __shfl_down(cy, 1, 64);
        if (edge_l) cl = T(0.75) * cv(xm, J, K) + T(0.25) * cv(xm, J2, K);
        if (edge_r) cr = T(0.75) * cv(xp, J, K) + T(0.25) * cv(xp, J2, K);
        vlo = T(0.75) * cy + T(0.25) * cl;
        vhi = T(0.75) * cy + T(0.25) * cr;
    };
    auto zm = [&](int K) { return K > 0 ? K - 1 : (t.perz ? ncz - 1 : K); };
    auto zp = [&](int K) { return K < ncz - 1 ? K + 1 : (t.perz ? 0 : K); };
    int K = k0 >> 1;
    T mlo, mhi, clo, chi, nlo, nhi;
    vplane(zm(K), mlo, mhi);
    vplane(K, clo, chi);
    vplane(zp(K), nlo, nhi);
    T* fp = fine + (int64_t)jc * t.nfx + 2 * Ic;
    const int64_t sf = (int64_t)t.nfx * t.nfy;
    for (int k = k0; k < k1; ++k) {
        if ((k >> 1) != K) {  // next coarse plane
            K = k >> 1;
            mlo = clo; mhi = chi;
            clo = nlo; chi = nhi;
            vplane(zp(K), nlo, nhi);
        }
        const bool up = k & 1;
        const T dlo = T(0.75) * clo + T(0.25) * (up ? nlo : mlo);
        const T dhi = T(0.75) * chi + T(0.25) * (up ? nhi : mhi);
        if (valid) {
            if (SPLIT) {
                // cell 2I has the colour of the row's parity
                const int p = (jc + k) & 1, hf = t.nfx >> 1;
                T* q = fine + ((int64_t)k * t.nfy + jc) * t.nfx + Ic;
                if (RED_ONLY) {
                    q[0] += p ? dhi : dlo;
                } else {
                    q[p * hf] += dlo;
                    q[(1 - p) * hf] += dhi;
                }
            } else {
                T* q = fp + k * sf;
                q[0] += dlo;
                q[1] += dhi;
            }
        }
    }
}

// Red-only prolongation onto a split fine level (the following black half sweep overwrites the
// black cells): the thread and plane structure of k_prolong_zm<T, true, true>, over fine planes in
// pairs (one coarse plane each). The four coarse rows a workgroup's fine rows interpolate from
// (with one column on either side of its 64) go through LDS, one entry per thread per coarse
// plane, loaded a pair of fine planes ahead like the fine red entries; the pair loop is unrolled
// by two so that the loaded records alternate by renaming.
template <typename T, bool CSPLIT>
__global__ __launch_bounds__(kBlock) void k_prolong_red(Transfer t, ZTiles zt, const T* __restrict__ coarse,
                                                        T* __restrict__ fine) {
    __shared__ T ce[2][4][66];  // [slot][coarse row 2 by - 1 + r][column I0 - 1 + l]
    int bx, by, bz;
    ztile(zt, bx, by, bz);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int I0 = bx * 64;
    const int I = I0 + lane;
    const int j = by * 4 + w;
    const bool valid = I < t.ncx && j < t.nfy;
    const int Ic = I < t.ncx ? I : t.ncx - 1, jc = j < t.nfy ? j : t.nfy - 1;
    const int k0 = bz * zt.kz, k1 = min(k0 + zt.kz, t.nfz);  // k0 even
    const int ncx = t.ncx, ncy = t.ncy, ncz = t.ncz;
    // x neighbours of the parent column (mirror onto the parent at a Neumann end)
    auto xmo = [&](int c) { return c > 0 ? c - 1 : (t.perx ? ncx - 1 : c); };
    auto xpo = [&](int c) { return c < ncx - 1 ? c + 1 : (t.perx ? 0 : c); };
    const int xm = xmo(Ic), xp = xpo(Ic);
    // y: parent row and second row, as rows 0 .. 3 of the workgroup's coarse rows 2 by - 1 + r
    const int J = jc >> 1;
    const int dj = (jc & 1) ? 1 : -1;
    const bool has2 = (J + dj >= 0 && J + dj < ncy) || t.pery;
    const int J2 = has2 ? (J + dj + ncy) % ncy : J;
    const int rJ = min(max(J - (2 * by - 1), 0), 3), rJ2 = min(max(has2 ? rJ + dj : rJ, 0), 3);
    // coarse row of LDS row w (the rows that no fine row of the workgroup uses get any valid row)
    int Jw = 2 * by - 1 + w;
    Jw = Jw < 0 ? (t.pery ? Jw + ncy : 0) : (Jw >= ncy ? (t.pery ? Jw - ncy : ncy - 1) : Jw);
    // LDS columns of the parent column and of its neighbours; edge columns 0 and 65 hold xm(I0)
    // and xp of the last column of the tile
    const int Ilast = min(I0 + 63, ncx - 1);
    const int lc = Ic - I0 + 1;
    const int ll = Ic > I0 ? Ic - I0 : 0;
    const int lr = Ic < Ilast ? Ic - I0 + 2 : 65;
    const int edge = lane == 0 ? xmo(I0) : (lane == 1 ? xpo(Ilast) : -1);  // edge column this lane loads
    auto cv = [&](int Ix, int Jy, int K) { return coarse[coarse_idx<CSPLIT>(t, Ix, Jy, K)]; };
    auto zm = [&](int K) { return K > 0 ? K - 1 : (t.perz ? ncz - 1 : K); };
    auto zp = [&](int K) { return K < ncz - 1 ? K + 1 : (t.perz ? 0 : K); };
    // the red entry of fine plane k at half position Ic
    auto zat = [&](int k) -> T* { return fine + ((int64_t)k * t.nfy + jc) * t.nfx + Ic; };
    // v(K) for the two fine columns straight from memory (start of the march)
    auto vmem = [&](int K, T& vlo, T& vhi) {
        const T cy = T(0.75) * cv(Ic, J, K) + T(0.25) * cv(Ic, J2, K);
        const T cl = T(0.75) * cv(xm, J, K) + T(0.25) * cv(xm, J2, K);
        const T cr = T(0.75) * cv(xp, J, K) + T(0.25) * cv(xp, J2, K);
        vlo = T(0.75) * cy + T(0.25) * cl;
        vhi = T(0.75) * cy + T(0.25) * cr;
    };
    // one coarse plane's entries of this thread: its LDS entry and, for lanes 0 and 1, an edge
    struct Raw {
        T c, e;
    };
    // (unconditional loads, as in k_restrict_red: lanes without an edge column load their own
    // entry again and ignore it)
    auto load_raw = [&](int K, Raw& o) {
        o.c = cv(min(I, ncx - 1), Jw, K);
        o.e = cv(edge >= 0 ? edge : min(I, ncx - 1), Jw, K);
    };
    T mlo, mhi, clo, chi;
    vmem(zm(k0 >> 1), mlo, mhi);
    vmem(k0 >> 1, clo, chi);
    // fine planes k, k+1 of coarse plane K = k/2: the lower one takes the plane below (m), the
    // upper one the plane above (n, from the entries loaded two pairs earlier: each pair issues
    // the loads of the pair after next before it computes)
    auto pstep = [&](int k, const Raw& rn, Raw& rn2, const T& z0, const T& z1, T& z0n2, T& z1n2) {
        const int K = k >> 1;
        const int sl = K & 1;
        ce[sl][w][lane + 1] = rn.c;
        if (edge >= 0) ce[sl][w][lane == 0 ? 0 : 65] = rn.e;
        __syncthreads();
        load_raw(zp(min(K + 2, ncz - 1)), rn2);
        z0n2 = *zat(min(k + 4, k1 - 1));
        z1n2 = *zat(min(k + 5, k1 - 1));
        const T cy = T(0.75) * ce[sl][rJ][lc] + T(0.25) * ce[sl][rJ2][lc];
        const T cl = T(0.75) * ce[sl][rJ][ll] + T(0.25) * ce[sl][rJ2][ll];
        const T cr = T(0.75) * ce[sl][rJ][lr] + T(0.25) * ce[sl][rJ2][lr];
        const T nlo = T(0.75) * cy + T(0.25) * cl, nhi = T(0.75) * cy + T(0.25) * cr;
        if (valid) {
            const int p = (jc + k) & 1;  // cell 2I of plane k has colour p; plane k+1 the other
            const T dlo0 = T(0.75) * clo + T(0.25) * mlo, dhi0 = T(0.75) * chi + T(0.25) * mhi;
            *zat(k) = z0 + (p ? dhi0 : dlo0);
            if (k + 1 < k1) {
                const T dlo1 = T(0.75) * clo + T(0.25) * nlo, dhi1 = T(0.75) * chi + T(0.25) * nhi;
                *zat(k + 1) = z1 + (p ? dlo1 : dhi1);
            }
        }
        mlo = clo;
        mhi = chi;
        clo = nlo;
        chi = nhi;
    };
    // a ring of four pairs; the main loop takes four pairs with no condition between them (a pair
    // under a branch leaves the compiler unsure which loads are in flight, and it then waits for
    // the prefetched ones too), the tail the last fewer than four
    Raw R0, R1, R2, R3;
    T a0, a1, b0, b1, c0, c1, d0, d1;
    load_raw(zp(k0 >> 1), R0);
    load_raw(zp(min((k0 >> 1) + 1, ncz - 1)), R1);
    a0 = *zat(k0);
    a1 = *zat(min(k0 + 1, k1 - 1));
    b0 = *zat(min(k0 + 2, k1 - 1));
    b1 = *zat(min(k0 + 3, k1 - 1));
    int k = k0;
    for (; k + 8 <= k1; k += 8) {
        pstep(k, R0, R2, a0, a1, c0, c1);
        pstep(k + 2, R1, R3, b0, b1, d0, d1);
        pstep(k + 4, R2, R0, c0, c1, a0, a1);
        pstep(k + 6, R3, R1, d0, d1, b0, b1);
    }
    if (k < k1) pstep(k, R0, R2, a0, a1, c0, c1);
    if (k + 2 < k1) pstep(k + 2, R1, R3, b0, b1, d0, d1);
    if (k + 4 < k1) pstep(k + 4, R2, R0, c0, c1, a0, a1);
}

template <typename T>
void launch_prolong_add(const Transfer& t, const T* coarse, T* fine, hipStream_t s, bool red_only) {
    if (transfer_zm(t)) {
        // the red-only prolongation holds four plane pairs in flight (86 VGPRs, five waves per
        // SIMD): chunks of 32 fine planes at 256^3 and of 4 at 128^3 keep its workgroups (1024)
        // resident at once
        const int kmin = !red_only ? 2 : (t.nfz >= 256 ? 32 : (t.nfz >= 128 ? 4 : 2));
        ZTiles zt = ztiles(t.ncx, t.nfy, t.nfz, 64, kmin);
        zt.rev = t.rev;
        zt.kz += zt.kz & 1;  // chunks start on even fine planes
        zt.tz = (t.nfz + zt.kz - 1) / zt.kz;
        const dim3 grid(zt.tx * zt.ty * zt.tz), block(kBlock);
        if (t.fsplit && red_only && t.csplit)
            hipLaunchKernelGGL((k_prolong_red<T, true>), grid, block, 0, s, t, zt, coarse, fine);
        else if (t.fsplit && red_only)
            hipLaunchKernelGGL((k_prolong_red<T, false>), grid, block, 0, s, t, zt, coarse, fine);
        else if (t.fsplit && t.csplit)
            hipLaunchKernelGGL((k_prolong_zm<T, true, false, true>), grid, block, 0, s, t, zt, coarse, fine);
        else if (t.fsplit)
            hipLaunchKernelGGL((k_prolong_zm<T, true>), grid, block, 0, s, t, zt, coarse, fine);
        else
            hipLaunchKernelGGL((k_prolong_zm<T, false>), dim3(zt.tx * zt.ty * zt.tz), dim3(kBlock), 0, s, t,
                               zt, coarse, fine);
        return;
    }
    Shape3 sh = cells_shape(t.nfx, t.nfy, t.nfz);
    hipLaunchKernelGGL((k_prolong_add<T>), sh.grid, sh.block, 0, s, t, coarse, fine);
}

template <typename T>
void launch_relayout(const T* src, T* dst, int nx, int ny, int nz, int to_split, hipStream_t s) {
    const int64_t npairs = (int64_t)(nx >> 1) * ny * nz;
    const int64_t blocks = (npairs + kBlock - 1) / kBlock;
    hipLaunchKernelGGL((k_relayout<T>), dim3((unsigned)blocks), dim3(kBlock), 0, s, src, dst, nx, ny, npairs,
                       to_split);
}

// Natural to split order for a caller's FP64 vector entering a solve, with the checks that go
// with it in the same pass: any non-finite entry sets bit 0 of *flags, any nonzero entry the bits
// nzbit, and with rc.op != OP_NONE the squared norm is reduced under rc. Grid-stride over cell
// pairs with a bounded grid (one partial each).
__global__ __launch_bounds__(kBlock) void k_relayout_in(const double* __restrict__ src, double* __restrict__ dst,
                                                        double* __restrict__ dst2, int nx, int ny, int64_t npairs,
                                                        int* flags, int nzbit, double* __restrict__ partials,
                                                        int norm) {
    const int hx = nx >> 1;
    double acc = 0.0;
    bool finite = true, nonzero = false;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < npairs; q += (int64_t)gridDim.x * kBlock) {
        const int64_t row = q / hx;
        const int t = (int)(q - row * hx);
        const int p = (int)((row % ny + row / ny) & 1);
        const int64_t rb = row * nx;
        const double v0 = src[rb + 2 * t], v1 = src[rb + 2 * t + 1];
        if (dst) {
            dst[rb + p * hx + t] = v0;
            dst[rb + (1 - p) * hx + t] = v1;
        }
        if (dst2) {
            dst2[rb + p * hx + t] = v0;
            dst2[rb + (1 - p) * hx + t] = v1;
        }
        finite = finite && isfinite(v0) && isfinite(v1);
        nonzero = nonzero || v0 != 0.0 || v1 != 0.0;
        acc += v0 * v0 + v1 * v1;
    }
    if (!finite) atomicOr(flags, 1);
    if (nonzero && nzbit) atomicOr(flags, nzbit);
    if (norm) block_partial(acc, partials);
}

void launch_relayout_in(const double* src, double* dst, int nx, int ny, int nz, int* flags, int nzbit,
                        const RedCtl& rc, hipStream_t s, double* dst2) {
    const int64_t npairs = (int64_t)(nx >> 1) * ny * nz;
    const int nb = vec_blocks(2 * npairs);
    hipLaunchKernelGGL(k_relayout_in, dim3(nb), dim3(kBlock), 0, s, src, dst, dst2, nx, ny, npairs, flags,
                       nzbit, rc.partials, rc.op != OP_NONE ? 1 : 0);
    finalize(rc, nb, s);
}

bool split_layout_ok(int nx, int ny, int nz, const Transfer* t) {
    return use_zm(nx, ny, nz) && (nx % 2 == 0) && (ny % kRowsS == 0) && t && transfer_zm(*t);
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
        // the first kU columns of the lane are loaded together (clamped indices, products of
        // columns past nc dropped): nc <= 64 kU needs one memory round trip, not nc / 64
        constexpr int kU = 8;
        double av[kU], bv[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int c = min(lane + 64 * u, nc - 1);
            av[u] = arow[c];
            bv[u] = (double)b[c];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (lane + 64 * u < nc) acc += av[u] * bv[u];
        for (int c = lane + 64 * kU; c < nc; c += 64) acc += arow[c] * (double)b[c];
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
    block_partial(acc, rc.partials);
}

template <typename T>
void launch_dot(const T* x, const T* y, int64_t n, const RedCtl& rc, hipStream_t s) {
    hipLaunchKernelGGL((k_dot<T>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, x, y, n, rc);
    finalize(rc, vec_blocks(n), s);
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
    block_partial(acc, rc.partials);
}

template <typename T>
void launch_axpy2_norm(T* x, const T* p, T* r, const T* q, int64_t n, const RedCtl& rc,
                       hipStream_t s) {
    hipLaunchKernelGGL((k_axpy2_norm<T>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, x, p, r, q, n,
                       rc);
    finalize(rc, vec_blocks(n), s);
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

// The CG iterate update deferred by one iteration: r -= alpha q with ||r||^2 first, then
// x += alpha p together with the next direction p = z + beta p (p is read once for both).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpy_norm(T* __restrict__ r, const T* __restrict__ q,
                                                      int64_t n, RedCtl rc) {
    const T alpha = (T)rc.scal[S_ALPHA];
    double acc = 0.0;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x; a < n; a += stride) {
        T ra = r[a] - alpha * __builtin_nontemporal_load(&q[a]);
        r[a] = ra;
        acc += (double)ra * (double)ra;
    }
    block_partial(acc, rc.partials);
    export_flag(rc);
}

// The same two updates over a split finest level in the tile order of the split kernels (and in
// their direction), so that they start on what the previous pass left in the memory-side cache.
// Four planes of loads are in flight per thread.
template <typename T, int XW>
__global__ __launch_bounds__(64 * XW * kRowsS) void k_axpy_norm_zs(ZTiles zt, int nx, int ny, int nz,
                                                          T* __restrict__ r, const T* __restrict__ q,
                                                          RedCtl rc) {
    constexpr int kTW = 64 * XW;
    int bx, by, bz;
    ztile(zt, bx, by, bz);
    const int hx = nx >> 1;
    const int t = bx * kTW + (int)(threadIdx.x % kTW), j = by * kRowsS + (int)(threadIdx.x / kTW);
    const int k0 = bz * zt.kz, k1 = min(k0 + zt.kz, nz);
    const T alpha = (T)rc.scal[S_ALPHA];
    double acc = 0.0;
    if (t < hx) {
        for (int k = k0; k < k1; k += 4) {
            T rv[8], qv[8];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int a = srow(j, min(k + u, k1 - 1), nx, ny) + t;
                rv[2 * u] = r[a];
                rv[2 * u + 1] = r[a + hx];
                qv[2 * u] = ld_stream(&q[a]);   // q is not read again
                qv[2 * u + 1] = ld_stream(&q[a + hx]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (k + u < k1) {
                    const int a = srow(j, k + u, nx, ny) + t;
                    const T r0 = rv[2 * u] - alpha * qv[2 * u], r1 = rv[2 * u + 1] - alpha * qv[2 * u + 1];
                    r[a] = r0;
                    r[a + hx] = r1;
                    acc += (double)r0 * (double)r0 + (double)r1 * (double)r1;
                }
            }
        }
    }
    block_partial(acc, rc.partials);
    export_flag(rc);
}

template <typename T>
int launch_axpy_norm(T* r, const T* q, int64_t n, const RedCtl& rc, hipStream_t s, const Geo<T>* g) {
    if (g && g->split) {
        ZTiles zt = split_tiles(g->nx >> 1, g->ny, g->nz);
        zt.rev = g->rev;
        const int nb = zt.tx * zt.ty * zt.tz;
        if (split_xw(g->nx >> 1) == 1)
            hipLaunchKernelGGL((k_axpy_norm_zs<T, 1>), dim3(nb), split_block(g->nx >> 1), 0, s, zt, g->nx, g->ny,
                               g->nz, r, q, rc);
        else
            hipLaunchKernelGGL((k_axpy_norm_zs<T, 2>), dim3(nb), split_block(g->nx >> 1), 0, s, zt, g->nx, g->ny,
                               g->nz, r, q, rc);
        finalize(rc, nb, s);
        return nb;
    }
    hipLaunchKernelGGL((k_axpy_norm<T>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, r, q, n, rc);
    finalize(rc, vec_blocks(n), s);
    return vec_blocks(n);
}

template <typename T, bool XZ>
__global__ __launch_bounds__(kBlock) void k_xpby_x(const T* __restrict__ z, T* __restrict__ p,
                                                   T* __restrict__ x, int64_t n,
                                                   const double* __restrict__ scal) {
    const T alpha = (T)scal[S_ALPHA], beta = (T)scal[S_BETA];
    int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (a < n) {
        // x and z are streamed (x is next touched by this kernel's next launch, z is rewritten by
        // the next preconditioner), so that the memory-side cache keeps p for the operator apply
        // that follows (at 256^3 that apply went from 114 to 99 µs)
        const T pa = p[a];
        const T xa = XZ ? T(0) : __builtin_nontemporal_load(&x[a]);   // XZ: x is known to be zero
        __builtin_nontemporal_store(xa + alpha * pa, &x[a]);
        p[a] = __builtin_nontemporal_load(&z[a]) + beta * pa;
    }
}

template <typename T>
void launch_xpby_x(const T* z, T* p, T* x, int64_t n, const double* scal, hipStream_t s, bool xzero) {
    if (xzero)
        hipLaunchKernelGGL((k_xpby_x<T, true>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, z, p, x, n, scal);
    else
        hipLaunchKernelGGL((k_xpby_x<T, false>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, z, p, x, n, scal);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpy_alpha(T* __restrict__ x, const T* __restrict__ p,
                                                       int64_t n, const double* __restrict__ scal, int xzero) {
    const T alpha = (T)scal[S_ALPHA];
    int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (a < n) x[a] = (xzero ? T(0) : x[a]) + alpha * p[a];
}

template <typename T>
void launch_axpy_alpha(T* x, const T* p, int64_t n, const double* scal, hipStream_t s, bool xzero) {
    hipLaunchKernelGGL((k_axpy_alpha<T>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, x, p, n, scal, xzero ? 1 : 0);
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
    block_partial(acc, rc.partials);
}

void launch_jacobi_apply(const double* dinv, const double* r, double* z, int64_t n,
                         const RedCtl& rc, hipStream_t s) {
    hipLaunchKernelGGL(k_jacobi_apply, dim3(vec_blocks(n)), dim3(kBlock), 0, s, dinv, r, z, n, rc);
    finalize(rc, vec_blocks(n), s);
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

// The refinement step of mixed precision in one pass: x += scale d, where d is the FP32 solution of
// the inner solve with its last update d += alpha p (alpha = scal[S_ALPHA]) applied here in FP32
// when it is still due (PEND), exactly as the inner solve would have applied it; XZ / DZ: x / d
// have not been written yet and are zero.
template <bool XZ, bool DZ, bool PEND>
__global__ __launch_bounds__(kBlock) void k_refine_update(double* __restrict__ x, const float* __restrict__ d,
                                                          const float* __restrict__ p,
                                                          const double* __restrict__ scal, double scale,
                                                          int64_t n) {
    const float alpha = (float)scal[S_ALPHA];
    const int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (a < n) {
        float v = DZ ? 0.0f : d[a];
        if (PEND) v = v + alpha * p[a];
        x[a] = (XZ ? 0.0 : x[a]) + scale * (double)v;
    }
}

void launch_refine_update(double* x, bool xzero, const float* d, bool dzero, const float* p, bool pending,
                          const double* scal, double scale, int64_t n, hipStream_t s) {
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
#define REFINE_CASE(XZ, DZ, PEND)                                                                       \
    if (xzero == XZ && dzero == DZ && pending == PEND) {                                                \
        hipLaunchKernelGGL((k_refine_update<XZ, DZ, PEND>), grid, block, 0, s, x, d, p, scal, scale, n); \
        return;                                                                                         \
    }
    REFINE_CASE(false, false, false)
    REFINE_CASE(false, false, true)
    REFINE_CASE(false, true, false)
    REFINE_CASE(false, true, true)
    REFINE_CASE(true, false, false)
    REFINE_CASE(true, false, true)
    REFINE_CASE(true, true, false)
    REFINE_CASE(true, true, true)
#undef REFINE_CASE
}

// Streaming copy (the measured bandwidth reference of the roofline figures): each thread moves
// four 16-byte vectors, loads and stores non-temporal (nothing is reused), consecutive threads
// on consecutive vectors; an odd last double is copied by thread 0 of workgroup 0.
typedef double dbl2 __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(kBlock) void k_stream_copy(const dbl2* __restrict__ src, dbl2* __restrict__ dst,
                                                        int64_t nv, const double* __restrict__ tail_src,
                                                        double* __restrict__ tail_dst) {
    const int64_t base = (int64_t)blockIdx.x * (4 * kBlock) + threadIdx.x;
    dbl2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = base + (int64_t)u * kBlock;
        if (i < nv) v[u] = __builtin_nontemporal_load(&src[i]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = base + (int64_t)u * kBlock;
        if (i < nv) __builtin_nontemporal_store(v[u], &dst[i]);
    }
    if (tail_src && blockIdx.x == 0 && threadIdx.x == 0) *tail_dst = *tail_src;
}

void launch_stream_copy(const double* src, double* dst, int64_t n, hipStream_t s) {
    const int64_t nv = n / 2;
    const int64_t blocks = std::max<int64_t>(1, (nv + 4 * kBlock - 1) / (4 * kBlock));
    const bool odd = n & 1;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(kBlock), 0, s, (const dbl2*)src, (dbl2*)dst,
                       nv, odd ? src + n - 1 : nullptr, odd ? dst + n - 1 : nullptr);
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

__global__ __launch_bounds__(kBlock) void k_axpby(double a, const double* __restrict__ x, double b,
                                                  double* __restrict__ y, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = a * x[i] + b * y[i];
}

void launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a, x,
                       b, y, n);
}

__global__ void k_set_scalar(double* scal, int slot, double v) { scal[slot] = v; }

void launch_set_scalar(double* scal, int slot, double value, hipStream_t s) {
    hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, scal, slot, value);
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
    template int launch_rbgs_own_dot<T>(const Geo<T>&, const T*, const T*, const T*, T*, int,      \
                                        double*, hipStream_t);                                     \
    template bool launch_rbgs_dot<T>(const Geo<T>&, const T*, const T*, const T*, T*, int,      \
                                     const RedCtl&, hipStream_t, const double*, int);           \
    template bool launch_presmooth<T>(const Geo<T>&, const T*, const T*, const T*, T*,          \
                                      hipStream_t);                                             \
    template bool launch_resid_red<T>(const Geo<T>&, const T*, const T*, const T*, const T*, T*, \
                                      hipStream_t, bool);                                       \
    template void launch_restrict<T>(const Transfer&, const T*, T*, hipStream_t, bool);         \
    template void launch_relayout<T>(const T*, T*, int, int, int, int, hipStream_t);            \
    template void launch_prolong_add<T>(const Transfer&, const T*, T*, hipStream_t, bool);      \
    template void launch_coarse_solve<T>(const double*, int, const T*, T*, hipStream_t);        \
    template void launch_dot<T>(const T*, const T*, int64_t, const RedCtl&, hipStream_t);       \
    template void launch_axpy2_norm<T>(T*, const T*, T*, const T*, int64_t, const RedCtl&,      \
                                       hipStream_t);                                            \
    template int launch_axpy_norm<T>(T*, const T*, int64_t, const RedCtl&, hipStream_t,         \
                                      const Geo<T>*);                                             \
    template void launch_xpby_x<T>(const T*, T*, T*, int64_t, const double*, hipStream_t, bool); \
    template void launch_axpy_alpha<T>(T*, const T*, int64_t, const double*, hipStream_t, bool);\
    template void launch_xpby<T>(const T*, T*, int64_t, const double*, hipStream_t);            \
    template void launch_fill<T>(T*, T, int64_t, hipStream_t);                                  \
    template void launch_copy<T>(const T*, T*, int64_t, hipStream_t);                           \
    template int launch_presmooth_update<T>(const Geo<T>&, const T*, const T*, const T*, const T*, T*,  \
                                            T*, const RedCtl&, hipStream_t);

HP_INST(double)
HP_INST(float)

}  // namespace hp
