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
// Both passes walk z columns over natural-order FP64 arrays (HBM-bound, about 1 flop per byte):
// workgroups of 64 x 4 columns in x and y so that x neighbours come from the same cache lines and
// y neighbours from rows the workgroup itself loads; the z neighbours stay in registers.
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

// z planes per thread column in the two passes around the solve
constexpr int kHZ = 16;

// Column tile (64 x 4 columns, one chunk of kHZ planes) of this workgroup of a 1-D grid. The
// hardware hands workgroup L to XCD L % 8; numbering the tiles so that each XCD takes one
// contiguous range of them (whole x-y planes of chunks) keeps the y neighbour rows of a tile in
// the L2 of the XCD that reads them.
struct HTiles {
    int tx, ty, tz;
};

__device__ __forceinline__ void htile(const HTiles& t, int& i, int& j, int& k0) {
    const unsigned total = (unsigned)t.tx * t.ty * t.tz;
    unsigned L = blockIdx.x;
    if ((total & 7u) == 0) L = (L & 7u) * (total >> 3) + (L >> 3);
    i = (int)(L % (unsigned)t.tx) * 64 + (threadIdx.x & 63);
    j = (int)((L / (unsigned)t.tx) % (unsigned)t.ty) * 4 + (threadIdx.x >> 6);
    k0 = (int)(L / ((unsigned)t.tx * t.ty)) * kHZ;
}

static HTiles htiles(const int n[3]) {
    return HTiles{(n[0] + 63) / 64, (n[1] + 3) / 4, (n[2] + kHZ - 1) / kHZ};
}

// Neighbours of the cells of one axis, as the three values (low neighbour, cell, high neighbour)
// of each array, and whether the two faces exist.
struct Line {
    bool lo, hi;
    double p[3], rn[3], r1[3], ms[3], c[3], k[3];
};

// The contributions of one axis to the rhs (steps (iv)-(v)): u_d (grad P^n)_d, (div u*)_d and the
// d-part of div(rho kappa_c grad c); ih = 1/h_d.
__device__ __forceinline__ void rhs_axis(const Line& L, double ud, double ih, bool tc, double& adv, double& divu,
                                         double& dc) {
    const double phi = L.hi ? pbnd(L.p[1], L.rn[1], L.p[2], L.rn[2]) : L.p[1];
    const double plo = L.lo ? pbnd(L.p[0], L.rn[0], L.p[1], L.rn[1]) : L.p[1];
    adv += ud * ((phi - plo) * ih);
    const double uhi = L.hi ? (L.ms[1] + L.ms[2]) / (L.r1[1] + L.r1[2]) : 0.0;
    const double ulo = L.lo ? (L.ms[0] + L.ms[1]) / (L.r1[0] + L.r1[1]) : 0.0;
    divu += (uhi - ulo) * ih;
    if (tc) {
        const double fhi = L.hi ? 0.5 * (L.k[1] + L.k[2]) * (L.c[2] - L.c[1]) * ih : 0.0;
        const double flo = L.lo ? 0.5 * (L.k[0] + L.k[1]) * (L.c[1] - L.c[0]) * ih : 0.0;
        dc += (fhi - flo) * ih;
    }
}

// x or y neighbour line of cell a (coordinate c along axis d, stride st): the neighbours from
// memory, the cell itself from the z ring Z; ms is the momentum component of axis d
__device__ __forceinline__ void load_line(const HGeo& g, const RhsArgs& A, const double* ms, int d, int c, int64_t a,
                                          int64_t st, bool tc, const Line& Z, Line& L) {
    int tl, th;
    L.lo = neighbour(g, d, c, -1, &tl);
    L.hi = neighbour(g, d, c, 1, &th);
    const int64_t bl = L.lo ? a + (int64_t)(tl - c) * st : a, bh = L.hi ? a + (int64_t)(th - c) * st : a;
    L.p[1] = Z.p[1];
    L.rn[1] = Z.rn[1];
    L.r1[1] = Z.r1[1];
    L.ms[1] = ms[a];
    L.c[1] = Z.c[1];
    L.k[1] = Z.k[1];
    const int64_t idx[2] = {bl, bh};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int q = 2 * e;
        L.p[q] = A.p_n[idx[e]];
        L.rn[q] = A.rho_n[idx[e]];
        L.r1[q] = A.rho_np1[idx[e]];
        L.ms[q] = ms[idx[e]];
        L.c[q] = tc ? A.conc_n[idx[e]] : 0.0;
        L.k[q] = tc ? A.rkc_n[idx[e]] : 0.0;
    }
}

// One thread per (x, y) column walking kHZ planes: the x and y neighbours come from memory (the
// x ones from the same cache lines), the z neighbours of the six stencil arrays from a ring of
// registers (each plane is loaded once per column). Every load of a plane is issued whatever the
// geometry (a missing neighbour, or an axis of one cell, reads the cell itself and contributes
// nothing): with loads under branches the compiler cannot count what is in flight and waited
// for the next plane's z loads before using this plane's values.
// TC: the two-component terms (temp_n, conc_n, rkc_n given); VISC: the viscous term (visc given).
template <bool TC, bool VISC>
__global__ __launch_bounds__(256) void k_pressure_rhs(HGeo g, HTiles t, RhsArgs A) {
    int i, j, k0;
    htile(t, i, j, k0);
    if (i >= g.n[0] || j >= g.n[1]) return;
    const int nz = g.n[2];
    const int k1 = min(k0 + kHZ, nz);
    const int64_t sxy = (int64_t)g.n[0] * g.n[1];
    constexpr bool tc = TC;
    const double ih[3] = {1.0 / g.h[0], 1.0 / g.h[1], 1.0 / g.h[2]};
    const double* msz = A.mom_star + 2 * A.N;
    const int64_t col = cell(g, i, j, 0);
    // ring: z line values of planes k-1, k, k+1 (position 0, 1, 2)
    Line Z;
    auto load_plane = [&](int kp, int q) {
        const int64_t a = col + (int64_t)kp * sxy;
        Z.p[q] = A.p_n[a];
        Z.rn[q] = A.rho_n[a];
        Z.r1[q] = A.rho_np1[a];
        Z.ms[q] = msz[a];
        Z.c[q] = tc ? A.conc_n[a] : 0.0;
        Z.k[q] = tc ? A.rkc_n[a] : 0.0;
    };
    int tz = k0;
    load_plane(neighbour(g, 2, k0, -1, &tz) ? tz : k0, 0);
    load_plane(k0, 1);
    for (int k = k0; k < k1; ++k) {
        Z.lo = nz > 1 && neighbour(g, 2, k, -1, &tz);
        tz = k;
        Z.hi = nz > 1 && neighbour(g, 2, k, 1, &tz);
        load_plane(tz, 2);
        const int64_t a = col + (int64_t)k * sxy;
        const double irn = 1.0 / Z.rn[1];
        const double m = irn / A.c2_n[a];
        double adv = 0.0, divu = 0.0, dc = 0.0;
        // (an axis of one cell has no faces: its lines contribute exact zeros)
        Line L;
        load_line(g, A, A.mom_star, 0, i, a, 1, tc, Z, L);
        rhs_axis(L, A.mom_n[a] * irn, ih[0], tc, adv, divu, dc);
        load_line(g, A, A.mom_star + A.N, 1, j, a, g.n[0], tc, Z, L);
        rhs_axis(L, A.mom_n[A.N + a] * irn, ih[1], tc, adv, divu, dc);
        rhs_axis(Z, A.mom_n[2 * A.N + a] * irn, ih[2], tc, adv, divu, dc);
        double b = m * (Z.p[1] - g.dt * adv) - g.dt * divu;
        if constexpr (VISC) b -= (2.0 * g.dt / 3.0) * (m * irn) * A.visc[a];
        if (tc) b -= (3.0 * g.dt / 4.0) * m * A.r_gas * A.temp_n[a] * dc;
        A.b[a] = b;
        // the ring moves up one plane
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            Z.p[q] = Z.p[q + 1];
            Z.rn[q] = Z.rn[q + 1];
            Z.r1[q] = Z.r1[q + 1];
            Z.ms[q] = Z.ms[q + 1];
            Z.c[q] = Z.c[q + 1];
            Z.k[q] = Z.k[q + 1];
        }
    }
}

struct UpdArgs {
    const double *p, *rho_np1, *mom_star, *e_star;
    double *mom_out, *uface_out, *e_out;
    int64_t N;
};

// The updates of one axis (steps (vii)-(viii)): grad P with rho^{n+1}, the high interface
// velocity u^{n+1} (returned through uf) and the axis' part of its divergence
__device__ __forceinline__ double upd_axis(bool lo, bool hi, const double* p, const double* r, const double* ms,
                                           double dt, double ih, double& uf, double& divn) {
    const double phi = hi ? pbnd(p[1], r[1], p[2], r[2]) : p[1];
    const double plo = lo ? pbnd(p[0], r[0], p[1], r[1]) : p[1];
    uf = hi ? (ms[1] + ms[2]) / (r[1] + r[2]) - dt * (p[2] - p[1]) * ih * 2.0 / (r[2] + r[1]) : 0.0;
    const double ul = lo ? (ms[0] + ms[1]) / (r[0] + r[1]) - dt * (p[1] - p[0]) * ih * 2.0 / (r[1] + r[0]) : 0.0;
    divn += (uf - ul) * ih;
    return (phi - plo) * ih;
}

__global__ __launch_bounds__(256) void k_pressure_update(HGeo g, HTiles t, UpdArgs A) {
    int i, j, k0;
    htile(t, i, j, k0);
    if (i >= g.n[0] || j >= g.n[1]) return;
    const int nz = g.n[2];
    const int k1 = min(k0 + kHZ, nz);
    const int64_t sxy = (int64_t)g.n[0] * g.n[1];
    const double ih[3] = {1.0 / g.h[0], 1.0 / g.h[1], 1.0 / g.h[2]};
    const double* msz = A.mom_star + 2 * A.N;
    const int64_t col = cell(g, i, j, 0);
    double zp[3] = {0.0, 0.0, 0.0}, zr[3] = {1.0, 1.0, 1.0}, zm[3] = {0.0, 0.0, 0.0};
    auto load_plane = [&](int kp, int q) {
        const int64_t a = col + (int64_t)kp * sxy;
        zp[q] = A.p[a];
        zr[q] = A.rho_np1[a];
        zm[q] = msz[a];
    };
    // (unconditional loads, as in k_pressure_rhs: an axis of one cell has no faces and its
    // terms are exact zeros)
    int tz = k0;
    load_plane(neighbour(g, 2, k0, -1, &tz) ? tz : k0, 0);
    load_plane(k0, 1);
    for (int k = k0; k < k1; ++k) {
        const bool zlo = nz > 1 && neighbour(g, 2, k, -1, &tz);
        tz = k;
        const bool zhi = nz > 1 && neighbour(g, 2, k, 1, &tz);
        load_plane(tz, 2);
        const int64_t a = col + (int64_t)k * sxy;
        const int c[2] = {i, j};
        const int64_t st[2] = {1, g.n[0]};
        double gp[3] = {0.0, 0.0, 0.0}, uf[3] = {0.0, 0.0, 0.0}, divn = 0.0;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            int tl, th;
            const bool lo = neighbour(g, d, c[d], -1, &tl), hi = neighbour(g, d, c[d], 1, &th);
            const int64_t bl = lo ? a + (int64_t)(tl - c[d]) * st[d] : a;
            const int64_t bh = hi ? a + (int64_t)(th - c[d]) * st[d] : a;
            const double* ms = A.mom_star + (int64_t)d * A.N;
            const double pv[3] = {A.p[bl], zp[1], A.p[bh]};
            const double rv[3] = {A.rho_np1[bl], zr[1], A.rho_np1[bh]};
            const double mv[3] = {ms[bl], ms[a], ms[bh]};
            gp[d] = upd_axis(lo, hi, pv, rv, mv, g.dt, ih[d], uf[d], divn);
        }
        gp[2] = upd_axis(zlo, zhi, zp, zr, zm, g.dt, ih[2], uf[2], divn);
        // step (vii): momentum; step (ix): e^{n+1} = e* - dt (P div u^{n+1} + u^{n+1} . grad P)
        const double ir = 1.0 / zr[1];
        double ug = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double md = A.mom_star[(int64_t)d * A.N + a] - g.dt * gp[d];
            A.mom_out[(int64_t)d * A.N + a] = md;
            A.uface_out[(int64_t)d * A.N + a] = uf[d];
            ug += (md * ir) * gp[d];
        }
        A.e_out[a] = A.e_star[a] - g.dt * (zp[1] * divn + ug);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            zp[q] = zp[q + 1];
            zr[q] = zr[q + 1];
            zm[q] = zm[q + 1];
        }
    }
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
    const HTiles t = htiles(n);
    const dim3 grid((unsigned)t.tx * t.ty * t.tz);
    if (f->temp_n && f->visc)
        hipLaunchKernelGGL((k_pressure_rhs<true, true>), grid, dim3(256), 0, s, g, t, A);
    else if (f->temp_n)
        hipLaunchKernelGGL((k_pressure_rhs<true, false>), grid, dim3(256), 0, s, g, t, A);
    else if (f->visc)
        hipLaunchKernelGGL((k_pressure_rhs<false, true>), grid, dim3(256), 0, s, g, t, A);
    else
        hipLaunchKernelGGL((k_pressure_rhs<false, false>), grid, dim3(256), 0, s, g, t, A);
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
    const HTiles t = htiles(n);
    hipLaunchKernelGGL(k_pressure_update, dim3((unsigned)t.tx * t.ty * t.tz), dim3(256), 0, s, g, t, A);
    return hipGetLastError() == hipSuccess ? HP_OK : HP_EHIP;
}

}  // namespace hp
