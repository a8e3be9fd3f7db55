// hp_internal.h -- private declarations shared by the kernels and the solver driver of libhp.so.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "hp.h"

namespace hp {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64s)

// Device scalar slots (FP64) used by the CG drivers; kernels read alpha/beta from here so the
// host never has to round-trip them.
enum Slot {
    S_RZ = 0,      // <r, z>
    S_PQ = 1,      // <p, A p>
    S_ALPHA = 2,
    S_BETA = 3,
    S_RR = 4,      // ||r||^2
    S_BB = 5,      // ||b||^2
    S_FLAG = 6,    // breakdown flag (1.0 when p^T A p <= 0 or not finite)
    S_TMP = 7,     // scratch result of a plain dot
    S_RZ_NEW = 8,
    S_GAMMA = 9,   // learned FCG: step of the network's estimate in the preconditioner
    S_T1 = 10,     // learned FCG: dot products the scalar steps combine
    S_T2 = 11,
    S_COUNT = 16
};

// scalar steps of the learned FCG (hp_fcg.hip)
enum FcgScalar { FCG_GAMMA = 0, FCG_ALPHA = 1, FCG_BETA = 2 };

// What the second reduction stage (one workgroup) does with the total.
enum RedOp {
    OP_NONE = 0,     // no reduction at all
    OP_STORE = 1,    // scal[slot] = total
    OP_ALPHA = 2,    // scal[S_PQ] = total; scal[S_ALPHA] = scal[S_RZ] / total (flag if <= 0)
    OP_BETA = 3,     // scal[S_BETA] = total / scal[S_RZ]; scal[S_RZ] = total
    OP_RZINIT = 4    // scal[S_RZ] = total; scal[S_BETA] = 0
};

struct RedCtl {
    double* partials;        // one entry per workgroup (first stage)
    double* scal;            // device scalar slots
    int op;
    int slot;
    double* flag_out = nullptr;  // r -= alpha q only: where workgroup 0 copies the breakdown flag
};

// Geometry of one level as seen by a kernel. wx/wy/wz = dt^2 / h^2 per axis.
template <typename T>
struct Geo {
    int nx, ny, nz;
    int px, py, pz;        // 1 if the axis has a periodic wrap face (periodic and n >= 2)
    T cx, cy, cz;          // dt^2 / h_d^2
    int split;             // 1: arrays of this level use the red-black split layout
    int rev = 0;           // 1: z-march tiles in reverse order (see ztile)
    int frule = 0;         // face rule (HP_OPT_FACE_RULE): 0 kappa_f = 2/(rho_a + rho_b),
                           // 1 kappa_f = (1/rho_a + 1/rho_b)/2
};

// Red-black split layout (finest level, nx even): each x row of nx cells holds its nx/2 red
// cells and then its nx/2 black cells, both in x order, so cell (i, j, k) of colour
// c = (i + j + k) & 1 sits at (j + ny k) nx + c nx/2 + i/2.

// Coarsening relation between level l (fine) and l+1 (coarse).
struct Transfer {
    int nfx, nfy, nfz;     // fine sizes
    int ncx, ncy, ncz;     // coarse sizes
    int fx, fy, fz;        // 1 if the axis is coarsened
    int perx, pery, perz;  // 1 if the axis is periodic
    int fsplit;            // 1 if the fine level uses the red-black split layout
    int csplit = 0;        // 1 if the coarse level does
    int rev = 0;           // 1: z-march tiles in reverse order
};

// ---- launchers (hp_kernels.hip); all asynchronous on `s` ----
// Kernel timing: the next split-layout apply or half sweep launched by this thread records its
// start and end into these events (hipExtLaunchKernel); launch_events_pending tells whether that
// launch has happened yet.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
bool launch_events_pending();
// m = 1 / (rho_mass c2), face density rho_face (flag bad if any input is <= 0 or not finite), on
// an nx x ny x nz grid, into rho_out and m in natural order; with split32 the FP32 copies go to
// the red-black split order, and FP64 copies in that order into rho_split and m_split if given
void launch_setup_coef(const double* rho_mass, const double* rho_face, const double* c2, double* rho_out,
                       double* m, double* rho_split, double* m_split, float* rho32, float* m32, int nx,
                       int ny, int nz, bool split32, int* bad, hipStream_t s);
// b += dt^2 q / h_d on the cells next to boundary `side` of axis d, q the prescribed outward normal
// flux per face (natural layout; coef = dt^2 / h_d)
void launch_neumann_rhs(int nx, int ny, int nz, int d, int side, double coef, const double* q, double* b,
                        hipStream_t s);
// coarse rho and m as the means over each coarse cell's children (natural order; the FP32 copies
// in the red-black split order with split32)
void launch_coarsen_coef(const Transfer& t, const double* rho_f, const double* m_f,
                         double* rho_c, double* m_c, float* rho32_c, float* m32_c, bool split32,
                         hipStream_t s);
// dinv = 1 / (m + sum of face weights) in FP64 and (if dinv32) FP32, from natural-order rho and m;
// written in natural order, or in the red-black split order with split_out
void launch_jacobi_diag(const Geo<double>& g, const Geo<float>& g32, const double* rho,
                        const double* m, const float* rho32, const float* m32, double* dinv,
                        float* dinv32, bool split_out, hipStream_t s);

// y = A x (mode 0), y = A x with <x, y> reduced (mode 1), y = b - A x (mode 2),
// y = b - A x with <y, y> reduced (mode 3).
template <typename T>
void launch_apply(const Geo<T>& g, const T* rho, const T* m, const T* x, const T* b, T* y,
                  int mode, const RedCtl& rc, hipStream_t s);
template <typename T>
void launch_rbgs(const Geo<T>& g, const T* rho, const T* m, const T* r, T* z, int colour,
                 hipStream_t s);
// red-black half sweep that also reduces <r, z> (all cells, final values) under rc; in the split
// layout the preceding sweep of the other colour (launch_rbgs_own_dot) reduced its own cells into
// the nb2 entries of partials2, which the second stage adds; returns false (and does nothing) when
// the level uses the small-grid kernels
template <typename T>
bool launch_rbgs_dot(const Geo<T>& g, const T* rho, const T* m, const T* r, T* z, int colour,
                     const RedCtl& rc, hipStream_t s, const double* partials2 = nullptr, int nb2 = 0);
// split layout: half sweep of `colour` reducing <r, z> over its own cells into partials (no
// second stage); returns the number of partials
template <typename T>
int launch_rbgs_own_dot(const Geo<T>& g, const T* rho, const T* m, const T* r, T* z, int colour,
                        double* partials, hipStream_t s);
// t = r - A z on red cells (valid right after a black half sweep, when the residual vanishes on
// black cells); black cells of t are set to 0 in the natural layout and left unwritten in the
// split layout. zero_guess: z is the one-pass zero-guess pre-smoothing (red values r dinv), so
// the split kernel forms t = sum_f w_f z_black without reading r and m. False (nothing done)
// when the level uses the small-grid kernels.
template <typename T>
bool launch_resid_red(const Geo<T>& g, const T* rho, const T* m, const T* r, const T* z, T* t,
                      hipStream_t s, bool zero_guess = false);
// zero-guess red half sweep followed by a black half sweep, in one pass (needs dinv);
// false (nothing done) when the level uses the small-grid kernels
template <typename T>
bool launch_presmooth(const Geo<T>& g, const T* rho, const T* dinv, const T* r, T* z, hipStream_t s);
template <typename T>
void launch_rbgs_zero(const Geo<T>& g, const T* rho, const T* m, const T* r, T* z,
                      hipStream_t s);
// coarse = R fine. red_only: the fine black cells are zero (a residual from launch_resid_red)
// and are not read in the split layout.
template <typename T>
void launch_restrict(const Transfer& t, const T* fine, T* coarse, hipStream_t s,
                     bool red_only = false);
// fine += P coarse. red_only: in the split layout only red cells are corrected (valid when a
// black half sweep follows, which overwrites every black cell without reading it)
template <typename T>
void launch_prolong_add(const Transfer& t, const T* coarse, T* fine, hipStream_t s,
                        bool red_only = false);
// natural <-> red-black split layout of one finest-level vector (src and dst differ)
template <typename T>
void launch_relayout(const T* src, T* dst, int nx, int ny, int nz, int to_split, hipStream_t s);
// whether the finest level can use the split layout (t: transfer to level 1, or null)
bool split_layout_ok(int nx, int ny, int nz, const Transfer* t);
template <typename T>
void launch_coarse_solve(const double* ainv, int nc, const T* b, T* x, hipStream_t s);
// Dense coarsest operator (N x N row-major, N = n[0] n[1] n[2]) from the level's rho and m: the
// seven-point flux-form matrix with face weights cd[d] * kappa (per[d]: axis d periodic).
void launch_coarse_assemble(const double* rho, const double* m, const int n[3], const int per[3],
                            const double cd[3], int face_rule, double* A, hipStream_t s);
// In-place inverse of the dense SPD n x n matrix a (row-major) by blocked Gauss-Jordan steps;
// work holds spd_inverse_work(n) doubles; *flag is set on a pivot that is not positive and finite.
int64_t spd_inverse_work(int n);
void launch_spd_inverse(double* a, double* work, int n, int* flag, hipStream_t s);

// Deterministic dot <x, y> accumulated in FP64.
template <typename T>
void launch_dot(const T* x, const T* y, int64_t n, const RedCtl& rc, hipStream_t s);
// x += alpha p; r -= alpha q; ||r||^2 -> scal[S_RR]  (alpha = scal[S_ALPHA])
template <typename T>
void launch_axpy2_norm(T* x, const T* p, T* r, const T* q, int64_t n, const RedCtl& rc,
                       hipStream_t s);
// p = z + beta p (beta = scal[S_BETA])
template <typename T>
void launch_xpby(const T* z, T* p, int64_t n, const double* scal, hipStream_t s);
// deferred iterate update: r -= alpha q with ||r||^2 under rc (with g of a split finest level: in
// the tile order and direction of the split kernels; returns the number of per-workgroup partials
// of ||r||^2 it wrote); then x += alpha p and p = z + beta p in one flat pass over any layout;
// x += alpha p alone where the iteration ends (alpha = scal[S_ALPHA])
template <typename T>
int launch_axpy_norm(T* r, const T* q, int64_t n, const RedCtl& rc, hipStream_t s,
                     const Geo<T>* g = nullptr);
// (xzero: x is known to be zero and is written, not read, by the update)
template <typename T>
void launch_xpby_x(const T* z, T* p, T* x, int64_t n, const double* scal, hipStream_t s,
                   bool xzero = false);
template <typename T>
void launch_axpy_alpha(T* x, const T* p, int64_t n, const double* scal, hipStream_t s, bool xzero = false);
// z = dinv * r with <r, z> reduced
void launch_jacobi_apply(const double* dinv, const double* r, double* z, int64_t n,
                         const RedCtl& rc, hipStream_t s);
// dst = (float)(src * scale)
void launch_cast_scale_f32(const double* src, float* dst, double scale, int64_t n, hipStream_t s);
// x += scale * (double)d
// x += scale (d + alpha p) with d + alpha p in FP32 (alpha = scal[S_ALPHA]; the alpha p term only
// when pending); xzero / dzero: x / d have not been written and are taken as zero
void launch_refine_update(double* x, bool xzero, const float* d, bool dzero, const float* p, bool pending,
                          const double* scal, double scale, int64_t n, hipStream_t s);
template <typename T>
void launch_fill(T* x, T v, int64_t n, hipStream_t s);
// dst = src with 16-byte non-temporal loads and stores (16-byte aligned pointers)
void launch_stream_copy(const double* src, double* dst, int64_t n, hipStream_t s);
template <typename T>
void launch_copy(const T* src, T* dst, int64_t n, hipStream_t s);
// flag nonzero if any entry is not finite
void launch_check_finite(const double* x, int64_t n, int* bad, hipStream_t s);
// r' = r - alpha q with ||r'||^2 under rc (partials; flag exported as by launch_axpy_norm), folded
// into the zero-guess pre-smoothing z of the next V-cycle on the split level g; r' goes to rn
// (distinct from r). Returns the number of partials.
template <typename T>
int launch_presmooth_update(const Geo<T>& g, const T* rho, const T* dinv, const T* r, const T* q, T* rn, T* z,
                            const RedCtl& rc, hipStream_t s);

// natural -> split relayout of a solve's input with the finiteness check (bit 0 of *flags), the
// nonzero check (bits nzbit) and, under rc, its norm; where dst2 is given, a second split copy;
// with dst null only the checks (and the norm) are made
void launch_relayout_in(const double* src, double* dst, int nx, int ny, int nz, int* flags, int nzbit,
                        const RedCtl& rc, hipStream_t s, double* dst2 = nullptr);

// y = a x + b y
void launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s);
// scal[slot] = value (stream-ordered, graph-safe)
void launch_set_scalar(double* scal, int slot, double value, hipStream_t s);
// learned FCG (hp_fcg.hip): scal[S_GAMMA | S_ALPHA | S_BETA] from the slots; y = x - g y (sub)
// or y += g x with g = scal[S_GAMMA] (both skip the g term when g = 0)
void launch_fcg_scalar(double* scal, int what, hipStream_t s);
void launch_fcg_gamma_update(double* y, const double* x, const double* scal, int64_t n, bool sub, hipStream_t s);

// ---- steps either side of the solve (hp_hydro.hip); natural-layout FP64 cell arrays ----
int hydro_launch_rhs(const int n[3], const int bc[3], const double h[3], double dt, const hp_rhs_fields* f,
                     double* rhs, hipStream_t s);
int hydro_launch_update(const int n[3], const int bc[3], const double h[3], double dt,
                        const hp_update_fields* f, hipStream_t s);
int hydro_launch_advect(const int n[3], const int bc[3], const double h[3], double dt, const double* rho,
                        const double* mom, const double* e, double* rho_out, double* mom_out, double* e_out,
                        hipStream_t s);
int hydro_launch_eos(int64_t N, const double* rho, const double* mom, const double* e, double gamma, double* p,
                     double* c2, hipStream_t s);

// ---- learned stage (hp_nn.hip) ----
int nn_grid(const hp_net* net, int* nx, int* ny, int* nz);
// z = s * out_scale * net(r / s, log rho, -log(rho m), p_prev / s), s = RMS(r); p_prev may be null.
// rho and m in natural order; r, p_prev and z in natural order, or with split != 0 in the red-black
// split storage of the finest level (nx even)
int nn_apply(hp_net* net, hipStream_t stream, const double* r, const double* rho, const double* m,
             const double* pprev, double* z, int split = 0);
const char* nn_error();
// training with a loss computed by the solver: forward pass, d = estimate - x, backward + Adam
// from the physical-units output gradient coef * q
int nn_train_forward(hp_net* net, hipStream_t stream, const double* b, const double* rho,
                     const double* m, const double* pprev);
int nn_output_minus(hp_net* net, const double* x, double* d);
int nn_train_backward(hp_net* net, const double* q, double coef, float lr);

// Number of workgroups the reducing kernels use for these sizes (partials capacity).
int64_t reduce_blocks_cells(int nx, int ny, int nz);
int64_t reduce_blocks_vec(int64_t n);

}  // namespace hp
