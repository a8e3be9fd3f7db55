// hp_hydro.hip -- the steps of the fractional-step algorithm either side of the pressure solve.
//
// Section 2, "The Algorithm": before the solve, steps (iv)-(v) form the right-hand side f of
// eq. fpoiss (one component) or eq. fpoiss2 (two components), here multiplied by dt^2 like the
// operator (b = dt^2 f):
//
//     b = m (P^n - dt u^n . grad P^n) - dt div u* - (2 dt / 3)(m / rho^n) G
//         - (3 dt / 4) m R_gas T^n div(rho^n kappa_c grad c^n),      m = 1 / (rho^n c2^n),
//
// with grad P^n from the density-weighted interface pressure of eq. pbnd and the central
// difference of eq. nablaP, and div u* from the interface velocity of eq. step1 applied to
// u* = (rho u)* / rho^{n+1}. After the solve, steps (vii)-(ix) update the momentum
// (eq. momupdate, grad P by eqs. pbnd and nablaP with rho^{n+1}), the interface velocities
// (step (viii): u*_{i+1/2} - dt (P_{i+1} - P_i) / h * 2 / (rho_{i+1} + rho_i)) and the total energy
// (eq. enupdate: e* - dt (P div u^{n+1} + u^{n+1} . grad P), div from the new interface
// velocities, u^{n+1} = (rho u)^{n+1} / rho^{n+1} at the cell).
//
// Boundaries as in the solve: periodic axes wrap; at a closed (Neumann) boundary the interface
// velocity is zero and the interface pressure is the cell's own; an axis of one cell has no
// gradient or divergence. The interface value of rho kappa_c is the mean of its two cells.
//
// Both passes are one thread per cell over natural-order FP64 arrays, bound by HBM bandwidth
// (about 1 flop per byte): workgroups of 64 x 4 cells in x and y so that x neighbours come from
// the same cache lines and y neighbours from rows the workgroup itself loads; z neighbours are
// re-read from the caches.
#include "hp.h"
#include "hp_internal.h"

namespace {

struct HGeo {
    int n[3];
    int per[3];   // 1: periodic with n >= 2 (wrap faces)
    double h[3];
    double dt;
};

// Neighbour of cell c along axis d in direction s (+1 / -1): its coordinate in *t, false when
// there is no face (closed boundary).
__device__ __forceinline__ bool neighbour(const HGeo& g, int d, int c, int s, int* t) {
    int q = c + s;
    const int n = g.n[d];
    if (q < 0 || q >= n) {
        if (!g.per[d]) return false;
        q = q < 0 ? n - 1 : 0;
    }
    *t = q;
    return true;
}

__device__ __forceinline__ int64_t cell(const HGeo& g, int i, int j, int k) {
    return i + (int64_t)g.n[0] * (j + (int64_t)g.n[1] * k);
}

// flat index of the neighbour of (i, j, k) along d at coordinate t
__device__ __forceinline__ int64_t along(const HGeo& g, int i, int j, int k, int d, int t) {
    return d == 0 ? cell(g, t, j, k) : d == 1 ? cell(g, i, t, k) : cell(g, i, j, t);
}

// eq. pbnd: the pressure at the interface between cells a and b
__device__ __forceinline__ double pbnd(double pa, double ra, double pb, double rb) {
    return (pb * ra + pa * rb) / (ra + rb);
}

struct RhsArgs {
    const double *rho_n, *c2_n, *p_n, *mom_n, *rho_np1, *mom_star, *visc, *temp_n, *conc_n, *rkc_n;
    double r_gas;
    int64_t N;
    double* b;
};

__global__ __launch_bounds__(256) void k_pressure_rhs(HGeo g, RhsArgs A) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const int c[3] = {i, j, k};
    const int64_t a = cell(g, i, j, k);
    const double rn = A.rho_n[a], r1 = A.rho_np1[a], pa = A.p_n[a];
    const double m = 1.0 / (rn * A.c2_n[a]);
    double adv = 0.0, divu = 0.0, dc = 0.0;
    for (int d = 0; d < 3; ++d) {
        if (g.n[d] == 1) continue;
        int th, tl;
        const bool hi = neighbour(g, d, c[d], 1, &th), lo = neighbour(g, d, c[d], -1, &tl);
        const int64_t bh = hi ? along(g, i, j, k, d, th) : a, bl = lo ? along(g, i, j, k, d, tl) : a;
        const double* ms = A.mom_star + (int64_t)d * A.N;
        // grad P^n (eqs. pbnd, nablaP with rho^n)
        const double phi = hi ? pbnd(pa, rn, A.p_n[bh], A.rho_n[bh]) : pa;
        const double plo = lo ? pbnd(A.p_n[bl], A.rho_n[bl], pa, rn) : pa;
        adv += (A.mom_n[(int64_t)d * A.N + a] / rn) * ((phi - plo) / g.h[d]);
        // div u*: interface velocities of eq. step1 with (rho u)* and rho^{n+1}
        const double uhi = hi ? (ms[a] + ms[bh]) / (r1 + A.rho_np1[bh]) : 0.0;
        const double ulo = lo ? (ms[bl] + ms[a]) / (A.rho_np1[bl] + r1) : 0.0;
        divu += (uhi - ulo) / g.h[d];
        if (A.temp_n) {  // div(rho kappa_c grad c), mean interface coefficient, no wall flux
            const double ca = A.conc_n[a], ka = A.rkc_n[a];
            const double fhi = hi ? 0.5 * (ka + A.rkc_n[bh]) * (A.conc_n[bh] - ca) / g.h[d] : 0.0;
            const double flo = lo ? 0.5 * (A.rkc_n[bl] + ka) * (ca - A.conc_n[bl]) / g.h[d] : 0.0;
            dc += (fhi - flo) / g.h[d];
        }
    }
    double b = m * (pa - g.dt * adv) - g.dt * divu;
    if (A.visc) b -= (2.0 * g.dt / 3.0) * (m / rn) * A.visc[a];
    if (A.temp_n) b -= (3.0 * g.dt / 4.0) * m * A.r_gas * A.temp_n[a] * dc;
    A.b[a] = b;
}

struct UpdArgs {
    const double *p, *rho_np1, *mom_star, *e_star;
    double *mom_out, *uface_out, *e_out;
    int64_t N;
};

__global__ __launch_bounds__(256) void k_pressure_update(HGeo g, UpdArgs A) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const int c[3] = {i, j, k};
    const int64_t a = cell(g, i, j, k);
    const double pa = A.p[a], r1 = A.rho_np1[a];
    double gp[3] = {0.0, 0.0, 0.0}, mom[3], divn = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double* ms = A.mom_star + (int64_t)d * A.N;
        double uf = 0.0;
        if (g.n[d] > 1) {
            int th, tl;
            const bool hi = neighbour(g, d, c[d], 1, &th), lo = neighbour(g, d, c[d], -1, &tl);
            const int64_t bh = hi ? along(g, i, j, k, d, th) : a, bl = lo ? along(g, i, j, k, d, tl) : a;
            const double ph = A.p[bh], pl = A.p[bl], rh = A.rho_np1[bh], rl = A.rho_np1[bl];
            // step (vii): grad P with rho^{n+1}
            const double phi = hi ? pbnd(pa, r1, ph, rh) : pa;
            const double plo = lo ? pbnd(pl, rl, pa, r1) : pa;
            gp[d] = (phi - plo) / g.h[d];
            // step (viii): the interface velocity on the high side, and the one on the low side
            // (the low neighbour's high interface) for the divergence
            if (hi) uf = (ms[a] + ms[bh]) / (r1 + rh) - g.dt * (ph - pa) / g.h[d] * 2.0 / (rh + r1);
            const double ul =
                lo ? (ms[bl] + ms[a]) / (rl + r1) - g.dt * (pa - pl) / g.h[d] * 2.0 / (r1 + rl) : 0.0;
            divn += (uf - ul) / g.h[d];
        }
        mom[d] = ms[a] - g.dt * gp[d];
        A.mom_out[(int64_t)d * A.N + a] = mom[d];
        A.uface_out[(int64_t)d * A.N + a] = uf;
    }
    // step (ix): e^{n+1} = e* - dt (P div u^{n+1} + u^{n+1} . grad P)
    double ug = 0.0;
    for (int d = 0; d < 3; ++d) ug += (mom[d] / r1) * gp[d];
    A.e_out[a] = A.e_star[a] - g.dt * (pa * divn + ug);
}

// ---- the explicit advective part (steps (i)-(iii)) and the equation of state ----

// q at distance s (+-1, +-2) along axis d from coordinate c: wrapped on a periodic axis, the edge
// cell repeated beyond a closed boundary (a zero-gradient mirror for the reconstruction)
__device__ __forceinline__ int reach(const HGeo& g, int d, int c, int s) {
    int q = c + s;
    const int n = g.n[d];
    if (g.per[d]) return ((q % n) + n) % n;
    return q < 0 ? 0 : (q >= n ? n - 1 : q);
}

// second-order ENO: the smaller in magnitude of the two one-sided differences (ties: the second)
__device__ __forceinline__ double eno_slope(double dm, double dp) { return fabs(dm) < fabs(dp) ? dm : dp; }

// the value at the interface between cells q1 (low) and q2 (high), reconstructed on the upwind
// side of the interface velocity u from the cells q0 .. q3 around it
__device__ __forceinline__ double eno_face(double u, double q0, double q1, double q2, double q3) {
    return u >= 0.0 ? q1 + 0.5 * eno_slope(q1 - q0, q2 - q1) : q2 - 0.5 * eno_slope(q2 - q1, q3 - q2);
}

struct AdvArgs {
    const double *rho, *mom, *e;
    double *rho_out, *mom_out, *e_out;
    int64_t N;
};

// One thread per cell: for every axis the fluxes through the cell's low and high interfaces of the
// five conserved fields (rho, three momenta, e), each interface velocity from eq. step1 and each
// field value reconstructed on its upwind side; q* = q - dt div(flux).
__global__ __launch_bounds__(256) void k_advect(HGeo g, AdvArgs A) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const int c[3] = {i, j, k};
    const int64_t a = cell(g, i, j, k);
    const double* q[5] = {A.rho, A.mom, A.mom + A.N, A.mom + 2 * A.N, A.e};
    double div[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int d = 0; d < 3; ++d) {
        if (g.n[d] == 1) continue;
        int64_t b[5];  // cells at -2 .. +2 along d
        for (int s = -2; s <= 2; ++s) b[s + 2] = along(g, i, j, k, d, reach(g, d, c[d], s));
        const double* md = A.mom + (int64_t)d * A.N;
        // interface velocities of eq. step1; zero at a closed boundary
        const bool hi = g.per[d] || c[d] < g.n[d] - 1, lo = g.per[d] || c[d] > 0;
        const double uh = hi ? (md[a] + md[b[3]]) / (A.rho[a] + A.rho[b[3]]) : 0.0;
        const double ul = lo ? (md[b[1]] + md[a]) / (A.rho[b[1]] + A.rho[a]) : 0.0;
        for (int f = 0; f < 5; ++f) {
            const double* qf = q[f];
            const double v0 = qf[b[0]], v1 = qf[b[1]], v2 = qf[a], v3 = qf[b[3]], v4 = qf[b[4]];
            const double fh = uh * eno_face(uh, v1, v2, v3, v4);
            const double fl = ul * eno_face(ul, v0, v1, v2, v3);
            div[f] += (fh - fl) / g.h[d];
        }
    }
    A.rho_out[a] = A.rho[a] - g.dt * div[0];
    for (int d = 0; d < 3; ++d) A.mom_out[(int64_t)d * A.N + a] = q[1 + d][a] - g.dt * div[1 + d];
    A.e_out[a] = A.e[a] - g.dt * div[4];
}

// ideal gas: P = (gamma - 1)(e - |rho u|^2 / (2 rho)), c_s^2 = gamma P / rho
__global__ __launch_bounds__(256) void k_eos(const double* __restrict__ rho, const double* __restrict__ mom,
                                             const double* __restrict__ e, double gamma, double* __restrict__ p,
                                             double* __restrict__ c2, int64_t N) {
    const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (a >= N) return;
    const double r = rho[a], mx = mom[a], my = mom[N + a], mz = mom[2 * N + a];
    const double pa = (gamma - 1.0) * (e[a] - 0.5 * (mx * mx + my * my + mz * mz) / r);
    p[a] = pa;
    if (c2) c2[a] = gamma * pa / r;
}

}  // namespace

namespace hp {

int hydro_launch_advect(const int n[3], const int bc[3], const double h[3], double dt, const double* rho,
                        const double* mom, const double* e, double* rho_out, double* mom_out, double* e_out,
                        hipStream_t s) {
    HGeo g;
    for (int d = 0; d < 3; ++d) {
        g.n[d] = n[d];
        g.per[d] = (bc[d] == HP_BC_PERIODIC && n[d] >= 2);
        g.h[d] = h[d];
    }
    g.dt = dt;
    AdvArgs A{rho, mom, e, rho_out, mom_out, e_out, (int64_t)n[0] * n[1] * n[2]};
    dim3 grid((unsigned)((n[0] + 63) / 64), (unsigned)((n[1] + 3) / 4), (unsigned)n[2]);
    hipLaunchKernelGGL(k_advect, grid, dim3(256), 0, s, g, A);
    return hipGetLastError() == hipSuccess ? HP_OK : HP_EHIP;
}

int hydro_launch_eos(int64_t N, const double* rho, const double* mom, const double* e, double gamma, double* p,
                     double* c2, hipStream_t s) {
    hipLaunchKernelGGL(k_eos, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, rho, mom, e, gamma, p, c2, N);
    return hipGetLastError() == hipSuccess ? HP_OK : HP_EHIP;
}

int hydro_launch_rhs(const int n[3], const int bc[3], const double h[3], double dt, const hp_rhs_fields* f,
                     double* rhs, hipStream_t s) {
    HGeo g;
    for (int d = 0; d < 3; ++d) {
        g.n[d] = n[d];
        g.per[d] = (bc[d] == HP_BC_PERIODIC && n[d] >= 2);
        g.h[d] = h[d];
    }
    g.dt = dt;
    RhsArgs A{f->rho_n, f->c2_n, f->p_n, f->mom_n, f->rho_np1, f->mom_star, f->visc, f->temp_n, f->conc_n,
              f->rkc_n, f->r_gas, (int64_t)n[0] * n[1] * n[2], rhs};
    dim3 grid((unsigned)((n[0] + 63) / 64), (unsigned)((n[1] + 3) / 4), (unsigned)n[2]);
    hipLaunchKernelGGL(k_pressure_rhs, grid, dim3(256), 0, s, g, A);
    return hipGetLastError() == hipSuccess ? HP_OK : HP_EHIP;
}

int hydro_launch_update(const int n[3], const int bc[3], const double h[3], double dt,
                        const hp_update_fields* f, hipStream_t s) {
    HGeo g;
    for (int d = 0; d < 3; ++d) {
        g.n[d] = n[d];
        g.per[d] = (bc[d] == HP_BC_PERIODIC && n[d] >= 2);
        g.h[d] = h[d];
    }
    g.dt = dt;
    UpdArgs A{f->p, f->rho_np1, f->mom_star, f->e_star, f->mom_out, f->uface_out, f->e_out,
              (int64_t)n[0] * n[1] * n[2]};
    dim3 grid((unsigned)((n[0] + 63) / 64), (unsigned)((n[1] + 3) / 4), (unsigned)n[2]);
    hipLaunchKernelGGL(k_pressure_update, grid, dim3(256), 0, s, g, A);
    return hipGetLastError() == hipSuccess ? HP_OK : HP_EHIP;
}

}  // namespace hp
