// hp_solver.hip -- handle, multigrid hierarchy and CG drivers behind the C ABI of include/hp.h.
//
// The solve is the preconditioned conjugate gradient method the paper uses for its generalized
// Poisson equation (Section 2), with the paper's incomplete-Cholesky preconditioner (a sequential
// triangular solve) replaced by one geometric-multigrid V-cycle that runs as data-parallel
// stencil kernels. Every scalar of the CG recurrence lives on the device; the host reads one
// squared residual norm per iteration to decide convergence.
#include "hp.h"
#include "hp_internal.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

using namespace hp;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(x)                                                                         \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess)                                                             \
            return fail(HP_EHIP, "%s failed: %s", #x, hipGetErrorString(e_));              \
    } while (0)

#define CHK(x)                         \
    do {                               \
        int rc_ = (x);                 \
        if (rc_ != HP_OK) return rc_;  \
    } while (0)

struct LevelData {
    int n[3];
    double h[3];
    int coarsened[3];  // relative to the finer level
    int64_t N;
    double *rho = nullptr, *m = nullptr, *dinv = nullptr;
    float *rho32 = nullptr, *m32 = nullptr, *dinv32 = nullptr;
    double *r = nullptr, *z = nullptr, *t = nullptr;
    float *r32 = nullptr, *z32 = nullptr, *t32 = nullptr;
    int split = 0;  // arrays of this level are in the red-black split layout
};

bool can_coarsen(int n, int bc) {
    if (n % 2 != 0 || n / 2 < 2) return false;
    if (bc == HP_BC_PERIODIC && (n / 2) % 2 != 0) return false;
    return true;
}

}  // namespace

struct hp_handle {
    int device = 0;
    hipStream_t stream = nullptr;
    hp_grid grid{};
    hp_bc bc{};
    double dt = 0.0;
    std::vector<LevelData> lv;
    int nc = 0;
    double* ainv = nullptr;       // inverse of the coarsest operator (nc x nc)
    double* ainv_work = nullptr;  // workspace of the blocked Gauss-Jordan inverse
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
    double* r2 = nullptr;  // second residual array: the fused residual update writes r' there
    // the split iterate of the running solve is zero and has not been written yet (a zero initial
    // guess): its first update writes x = alpha p without reading it
    bool x_unset = false;
    // likewise for the inner FP32 solution of mixed precision within one inner solve
    bool x32_unset = false;
    float *x32 = nullptr, *r32 = nullptr, *z32 = nullptr, *p32 = nullptr, *q32 = nullptr;
    float* r32b = nullptr;  // second FP32 residual array (fused residual update)
    // split layout of the finest level: whether it is wanted, split copies of the caller's rhs and
    // iterate, natural copies of rho and m for the network
    int want_split = 0;
    double *bs = nullptr, *xs = nullptr, *rho_nat = nullptr, *m_nat = nullptr;
    double* scal = nullptr;
    double* partials = nullptr;
    double* partials2 = nullptr;  // the first half of a reduction split over two launches
    int* flag = nullptr;
    int64_t partial_cap = 0;
    double* host_scal = nullptr;  // pinned mirror of scal
    // partials of the CG residual norm and, after the last possible one (partial_cap), the
    // breakdown flag, written by the r -= alpha q kernel itself into mapped pinned host memory
    double* host_part = nullptr;
    double* dev_part = nullptr;   // the device's address of host_part
    int host_nparts = 0;          // how many partials the last r -= alpha q wrote
    int* host_flag = nullptr;     // pinned; [0] input checks, [1] coarsest pivots
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t ev_scal = nullptr;  // marks the copy of scal into host_scal
    // the coarsest inverse runs on a stream of its own, beside the finest level's relayout
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    unsigned dir = 0;              // traversal direction of the last finest-level pass
    std::vector<void*> allocs;
    // options
    int mode = HP_MODE_FP64_MGPCG;
    int max_iter = 1000;
    int nu_pre = 1, nu_post = 1;
    double inner_tol = 1e-5;
    int max_outer = 20;
    int coarsest_max = 512;
    int face_rule = 0;  // HP_OPT_FACE_RULE
    hp_stats stats{};
    // kernel timing inside solves: event pool and the (class, first event) of each timed launch
    int timing = 0;
    std::vector<hipEvent_t> tev;
    std::vector<std::pair<int, int>> spans;
    size_t tev_used = 0;
    // learned stage
    hp_net* net = nullptr;
    double *w1 = nullptr, *w2 = nullptr, *w3 = nullptr;
};

namespace {

template <typename T>
int dalloc(hp_handle* H, T** p, int64_t n) {
    void* q = nullptr;
    size_t bytes = (size_t)std::max<int64_t>(n, 1) * sizeof(T);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return fail(HP_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    H->allocs.push_back(q);
    *p = (T*)q;
    return HP_OK;
}

template <typename T>
Geo<T> geo(const hp_handle* H, const LevelData& L) {
    Geo<T> g;
    g.nx = L.n[0];
    g.ny = L.n[1];
    g.nz = L.n[2];
    g.px = (H->bc.x == HP_BC_PERIODIC && L.n[0] >= 2);
    g.py = (H->bc.y == HP_BC_PERIODIC && L.n[1] >= 2);
    g.pz = (H->bc.z == HP_BC_PERIODIC && L.n[2] >= 2);
    double dt2 = H->dt * H->dt;
    g.cx = (T)(dt2 / (L.h[0] * L.h[0]));
    g.cy = (T)(dt2 / (L.h[1] * L.h[1]));
    g.cz = (T)(dt2 / (L.h[2] * L.h[2]));
    g.split = L.split;
    g.frule = H->face_rule;
    return g;
}

// Direction of the next z-march pass over level l: passes over the finest level alternate (the
// memory-side cache keeps what the previous pass touched last), coarser levels stay forward.
int flip(hp_handle* H, int l) { return l == 0 ? (int)(H->dir ^= 1u) : 0; }

template <typename T>
Geo<T> geo_pass(hp_handle* H, const Geo<T>& g, int l) {
    Geo<T> c = g;
    c.rev = flip(H, l);
    return c;
}

Transfer transfer(const hp_handle* H, int l) {
    const LevelData& F = H->lv[l];
    const LevelData& C = H->lv[l + 1];
    Transfer t;
    t.nfx = F.n[0]; t.nfy = F.n[1]; t.nfz = F.n[2];
    t.ncx = C.n[0]; t.ncy = C.n[1]; t.ncz = C.n[2];
    t.fx = C.coarsened[0]; t.fy = C.coarsened[1]; t.fz = C.coarsened[2];
    t.perx = H->bc.x == HP_BC_PERIODIC;
    t.pery = H->bc.y == HP_BC_PERIODIC;
    t.perz = H->bc.z == HP_BC_PERIODIC;
    t.fsplit = F.split;
    t.csplit = C.split;
    return t;
}

RedCtl red(const hp_handle* H, int op, int slot = 0) {
    RedCtl rc;
    rc.partials = H->partials;
    rc.scal = H->scal;
    rc.op = op;
    rc.slot = slot;
    return rc;
}

int check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(HP_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return HP_OK;
}

// ---- kernel timing (HP_OPT_KERNEL_TIMING) ----
enum { TIME_SWEEP = 0, TIME_APPLY = 1 };

// Timing events only take time stamps (the host reads no memory behind them), so they are
// created without the system-scope release and acquire that a default event carries: that
// fence's write-back is no part of the launch they bracket.
hipEvent_t timing_event(hp_handle* H) {
    if (H->tev_used == H->tev.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
        H->tev.push_back(e);
    }
    return H->tev[H->tev_used++];
}

// times one launch: time_begin before it hands a pair of events to the launcher, which attaches
// them to the dispatch (split-layout stencils only); time_end right after it keeps the span if the
// launch took them, else drops it
void time_begin(hp_handle* H, int cls) {
    if (!H->timing) return;
    const size_t first = H->tev_used;
    hipEvent_t a = timing_event(H), b = timing_event(H);
    if (!a || !b) return;
    set_launch_events(a, b);
    H->spans.push_back({cls, (int)first});
}
void time_end(hp_handle* H) {
    if (!H->timing || H->spans.empty()) return;
    if (launch_events_pending()) {
        set_launch_events(nullptr, nullptr);
        H->spans.pop_back();
    }
}

// ---- coarsest level: dense FP64 operator and its inverse, both built on the device ----

// Enqueue the coarsest operator's assembly and inverse on the side stream, behind the work
// enqueued so far on the handle's stream (which wrote the coarsest rho and m). A pivot that is
// not positive (the operator is not positive definite) sets host_flag[1] once the handle's stream
// has waited for the side stream (join_coarse_inverse) and been synchronised.
int start_coarse_inverse(hp_handle* H) {
    LevelData& C = H->lv.back();
    const int n = (int)C.N;
    const int per[3] = {H->bc.x == HP_BC_PERIODIC, H->bc.y == HP_BC_PERIODIC,
                        H->bc.z == HP_BC_PERIODIC};
    const double dt2 = H->dt * H->dt;
    double cd[3];
    for (int d = 0; d < 3; ++d) cd[d] = dt2 / (C.h[d] * C.h[d]);
    H->host_flag[1] = 0;
    HIPCHK(hipEventRecord(H->ev_fork, H->stream));
    HIPCHK(hipStreamWaitEvent(H->side, H->ev_fork, 0));
    HIPCHK(hipMemsetAsync(H->flag + 1, 0, sizeof(int), H->side));
    launch_coarse_assemble(C.rho, C.m, C.n, per, cd, H->face_rule, H->ainv, H->side);
    launch_spd_inverse(H->ainv, H->ainv_work, n, H->flag + 1, H->side);
    CHK(check_launch());
    HIPCHK(hipMemcpyAsync(H->host_flag + 1, H->flag + 1, sizeof(int), hipMemcpyDeviceToHost, H->side));
    HIPCHK(hipEventRecord(H->ev_join, H->side));
    return HP_OK;
}

// Work enqueued on the handle's stream after this call sees the coarsest inverse.
int join_coarse_inverse(hp_handle* H) {
    HIPCHK(hipStreamWaitEvent(H->stream, H->ev_join, 0));
    return HP_OK;
}

// The coarsest inverse on its own (the caller waits for it).
int build_coarse_inverse(hp_handle* H) {
    CHK(start_coarse_inverse(H));
    CHK(join_coarse_inverse(H));
    HIPCHK(hipStreamSynchronize(H->stream));
    if (H->host_flag[1]) return fail(HP_EDOMAIN, "coarsest operator is not positive definite");
    return HP_OK;
}

// ---- finest-level storage order ----

bool split_allowed(const hp_handle* H) {
    if (H->lv.size() < 2) return false;
    const LevelData& F = H->lv[0];
    Transfer t = transfer(H, 0);
    return split_layout_ok(F.n[0], F.n[1], F.n[2], &t);
}

// Whether level l can follow a split level l-1 in the split layout: the same conditions as the
// finest level, and rows of at least 32 half positions (one wave per row, at least half of it
// busy; measured faster than the natural-order kernels down to that width).
bool split_allowed_below(const hp_handle* H, size_t l) {
    if (l + 1 >= H->lv.size()) return false;
    const LevelData& L = H->lv[l];
    Transfer t = transfer(H, (int)l);
    return L.n[0] / 2 >= 32 && split_layout_ok(L.n[0], L.n[1], L.n[2], &t);
}

// Whether level l is in split order under the split layout: the finest level where the grid
// allows it, and below it each level that allows it while the level above is split.
bool split_target(const hp_handle* H, size_t l) {
    if (!split_allowed(H)) return false;
    for (size_t q = 1; q <= l; ++q)
        if (!split_allowed_below(H, q)) return false;
    return true;
}

template <typename T>
void relayout_l(hp_handle* H, int l, const T* src, T* dst, int to_split) {
    const LevelData& L = H->lv[l];
    launch_relayout<T>(src, dst, L.n[0], L.n[1], L.n[2], to_split, H->stream);
}

// The finest level's buffers of the split layout (rhs and iterate in split order, the natural rho
// and m), allocated the first time that layout is wanted.
int alloc_split_buffers(hp_handle* H) {
    const int64_t N = H->lv[0].N;
    int rc;
    for (double** a : {&H->bs, &H->xs, &H->rho_nat, &H->m_nat})
        if (!*a && (rc = dalloc(H, a, N))) return rc;
    return HP_OK;
}

// Bring the coefficient arrays to the natural (0) or split (1) layout: the finest level and,
// below it, every level that allows it as long as the level above is split. The relayout goes
// through a scratch array of the level's size (the CG vectors p and p32 on the finest level, the
// level's residual scratch t and t32 below it); the relaid copy then takes the array's place and
// the old array becomes the scratch (on the finest level the natural rho and m, kept for the
// network's features, keep their old arrays): no copy back. fresh: the state the coefficient
// setup leaves, in which the levels that become split hold dinv and the FP32 copies in split order
// already, and rho and m in natural order below the finest level; the finest level's rho and m are
// in split order with their natural copies in rho_nat / m_nat, so it is left as it is.
int set_layout(hp_handle* H, int split, bool fresh = false) {
    LevelData& F = H->lv[0];
    if (F.split == split) return HP_OK;
    if (split && !split_allowed(H)) return fail(HP_EINVAL, "the grid does not allow the split layout");
    if (split) CHK(alloc_split_buffers(H));
    for (size_t l = 0; l < H->lv.size(); ++l) {
        LevelData& L = H->lv[l];
        const int want = split && split_target(H, l);
        if (L.split == want) {
            if (!want) break;
            continue;
        }
        if (l == 0 && fresh) {
            // the coefficient setup wrote everything in its final place
        } else if (l == 0) {
            // rho and m: to split, the natural array becomes rho_nat / m_nat and the old copy
            // there the scratch vector; back to natural, the arrays trade places with the scratch
            double** keep[2] = {&H->rho_nat, &H->m_nat};
            double** arr[2] = {&L.rho, &L.m};
            for (int q = 0; q < 2; ++q) {
                relayout_l<double>(H, 0, *arr[q], H->p, want);
                double* relaid = H->p;
                if (want) {
                    H->p = *keep[q];
                    *keep[q] = *arr[q];
                } else {
                    H->p = *arr[q];
                }
                *arr[q] = relaid;
            }
            relayout_l<double>(H, 0, L.dinv, H->p, want);
            std::swap(L.dinv, H->p);
            for (float** a : {&L.rho32, &L.m32, &L.dinv32}) {
                relayout_l<float>(H, 0, *a, H->p32, want);
                std::swap(*a, H->p32);
            }
        } else {
            // through the level's residual scratch t / t32 (its size, contents never kept between
            // V-cycles): the relaid copy takes the array's place, the old array becomes t
            for (double** a : {&L.rho, &L.m, &L.dinv}) {
                if (fresh && a == &L.dinv) continue;
                relayout_l<double>(H, (int)l, *a, L.t, want);
                std::swap(*a, L.t);
            }
            if (!fresh)
                for (float** a : {&L.rho32, &L.m32, &L.dinv32}) {
                    relayout_l<float>(H, (int)l, *a, L.t32, want);
                    std::swap(*a, L.t32);
                }
        }
        L.split = want;
    }
    CHK(check_launch());
    return HP_OK;
}

// rho and m of the finest level in natural order (for the network's features)
const double* rho_natural(const hp_handle* H) { return H->lv[0].split ? H->rho_nat : H->lv[0].rho; }
const double* m_natural(const hp_handle* H) { return H->lv[0].split ? H->m_nat : H->lv[0].m; }

template <typename T>
void relayout0(hp_handle* H, const T* src, T* dst, int to_split) {
    const LevelData& F = H->lv[0];
    launch_relayout<T>(src, dst, F.n[0], F.n[1], F.n[2], to_split, H->stream);
}

// ---- coefficients of every level ----

// rho_mass: the density of the mass term m = 1/(rho c2) (time level n); rho_face: the density of
// the face coefficients (time level n+1); the one-density form passes the same array for both
int load_coefficients(hp_handle* H, const double* rho_mass, const double* rho_face, const double* c2,
                      double dt) {
    if (!rho_mass || !rho_face || !c2) return fail(HP_EINVAL, "rho and c2 must be non-null device pointers");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(HP_EINVAL, "dt must be positive and finite");
    H->dt = dt;
    LevelData& F = H->lv[0];
    for (auto& L : H->lv) L.split = 0;  // every array below is recomputed in natural order
    H->host_flag[0] = 0;
    HIPCHK(hipMemsetAsync(H->flag, 0, sizeof(int), H->stream));
    // The FP32 copies and the Jacobi diagonals of the levels that the split layout will reach are
    // written in split order directly (set_layout then leaves them alone); on a split finest level
    // rho and m go to its arrays in split order as well and to rho_nat / m_nat in natural order
    // (whose old contents are stale), which the coarsening and the diagonals below read.
    const bool split0 = H->want_split && split_target(H, 0);
    if (split0) CHK(alloc_split_buffers(H));
    double* rho0 = split0 ? H->rho_nat : F.rho;
    double* m0 = split0 ? H->m_nat : F.m;
    launch_setup_coef(rho_mass, rho_face, c2, rho0, m0, split0 ? F.rho : nullptr, split0 ? F.m : nullptr,
                      F.rho32, F.m32, F.n[0], F.n[1], F.n[2], split0, H->flag, H->stream);
    CHK(check_launch());
    HIPCHK(hipMemcpyAsync(H->host_flag, H->flag, sizeof(int), hipMemcpyDeviceToHost, H->stream));
    // The input check is read once everything below has run: with an invalid cell the steps
    // below compute non-finite values (no index or trip count depends on a value) and the call
    // fails at the end, leaving the coefficients undefined as before.
    for (size_t l = 0; l + 1 < H->lv.size(); ++l) {
        LevelData& C = H->lv[l + 1];
        launch_coarsen_coef(transfer(H, (int)l), l == 0 ? rho0 : H->lv[l].rho, l == 0 ? m0 : H->lv[l].m,
                            C.rho, C.m, C.rho32, C.m32, H->want_split && split_target(H, l + 1), H->stream);
        CHK(check_launch());
    }
    // the coarsest inverse (it needs only the coarsest rho and m) overlaps the Jacobi diagonals
    // and the relayout to the split storage order
    CHK(start_coarse_inverse(H));
    for (size_t l = 0; l < H->lv.size(); ++l) {
        LevelData& L = H->lv[l];
        launch_jacobi_diag(geo<double>(H, L), geo<float>(H, L), l == 0 ? rho0 : L.rho, l == 0 ? m0 : L.m,
                           L.rho32, L.m32, L.dinv, L.dinv32, H->want_split && split_target(H, l), H->stream);
    }
    CHK(check_launch());
    const int rc = H->want_split ? set_layout(H, 1, true) : HP_OK;
    CHK(join_coarse_inverse(H));
    HIPCHK(hipStreamSynchronize(H->stream));
    if (H->host_flag[0]) return fail(HP_EDOMAIN, "rho and c2 must be positive and finite in every cell");
    if (H->host_flag[1]) return fail(HP_EDOMAIN, "coarsest operator is not positive definite");
    return rc;
}

// ---- V-cycle ----

template <typename T> T* lvl_r(LevelData& L);
template <typename T> T* lvl_z(LevelData& L);
template <typename T> T* lvl_t(LevelData& L);
template <typename T> const T* lvl_rho(const LevelData& L);
template <typename T> const T* lvl_m(const LevelData& L);
template <> double* lvl_r<double>(LevelData& L) { return L.r; }
template <> double* lvl_z<double>(LevelData& L) { return L.z; }
template <> double* lvl_t<double>(LevelData& L) { return L.t; }
template <> float* lvl_r<float>(LevelData& L) { return L.r32; }
template <> float* lvl_z<float>(LevelData& L) { return L.z32; }
template <> float* lvl_t<float>(LevelData& L) { return L.t32; }
template <> const double* lvl_rho<double>(const LevelData& L) { return L.rho; }
template <> const double* lvl_m<double>(const LevelData& L) { return L.m; }
template <> const float* lvl_rho<float>(const LevelData& L) { return L.rho32; }
template <> const float* lvl_m<float>(const LevelData& L) { return L.m32; }
template <typename T> const T* lvl_dinv(const LevelData& L);
template <> const double* lvl_dinv<double>(const LevelData& L) { return L.dinv; }
template <> const float* lvl_dinv<float>(const LevelData& L) { return L.dinv32; }

// V-cycle z = M r on level l. With dot != nullptr (level 0 only) the final red half sweep also
// reduces <r, z> under *dot; returns true if it did (else the caller reduces separately).
template <typename T>
// pre_done: the zero-guess pre-smoothing of the finest level has already been launched (fused
// with the CG residual update, see pcg64)
bool vcycle(hp_handle* H, int l, const T* r, T* z, const RedCtl* dot = nullptr, bool pre_done = false) {
    LevelData& L = H->lv[l];
    hipStream_t s = H->stream;
    if (l == (int)H->lv.size() - 1) {
        launch_coarse_solve<T>(H->ainv, H->nc, r, z, s);
        return false;
    }
    Geo<T> g = geo<T>(H, L);
    const T* rho = lvl_rho<T>(L);
    const T* m = lvl_m<T>(L);
    const bool fused_pre =
        (l == 0 && pre_done) || launch_presmooth<T>(geo_pass(H, g, l), rho, lvl_dinv<T>(L), r, z, s);
    if (!fused_pre) {
        launch_rbgs_zero<T>(geo_pass(H, g, l), rho, m, r, z, s);
        launch_rbgs<T>(geo_pass(H, g, l), rho, m, r, z, 1, s);
    }
    for (int it = 1; it < H->nu_pre; ++it) {
        launch_rbgs<T>(geo_pass(H, g, l), rho, m, r, z, 0, s);
        launch_rbgs<T>(geo_pass(H, g, l), rho, m, r, z, 1, s);
    }
    T* t = lvl_t<T>(L);
    // after the black half sweep the residual vanishes on black cells
    const bool red_res = launch_resid_red<T>(geo_pass(H, g, l), rho, m, r, z, t, s,
                                             fused_pre && H->nu_pre == 1);
    if (!red_res) launch_apply<T>(geo_pass(H, g, l), rho, m, z, r, t, 2, red(H, OP_NONE), s);
    LevelData& C = H->lv[l + 1];
    Transfer tr = transfer(H, l);
    tr.rev = flip(H, l);
    launch_restrict<T>(tr, t, lvl_r<T>(C), s, red_res);
    vcycle<T>(H, l + 1, lvl_r<T>(C), lvl_z<T>(C));
    // the post-smoothing starts with a black half sweep, which overwrites the black cells
    tr.rev = flip(H, l);
    launch_prolong_add<T>(tr, lvl_z<T>(C), z, s, true);
    for (int it = 0; it < H->nu_post; ++it) {
        const bool timed = (l == 0 && sizeof(T) == 8);
        const bool last_dot = dot && it == H->nu_post - 1;
        // with <r, z> wanted in the split layout the black sweep reduces its own cells, the red
        // sweep the rest
        int nb2 = 0;
        if (timed) time_begin(H, TIME_SWEEP);
        if (last_dot && g.split)
            nb2 = launch_rbgs_own_dot<T>(geo_pass(H, g, l), rho, m, r, z, 1, H->partials2, s);
        else
            launch_rbgs<T>(geo_pass(H, g, l), rho, m, r, z, 1, s);
        if (timed) time_end(H);
        if (last_dot) {
            const Geo<T> gd = geo_pass(H, g, l);
            if (timed) time_begin(H, TIME_SWEEP);
            const bool done = launch_rbgs_dot<T>(gd, rho, m, r, z, 0, *dot, s, H->partials2, nb2);
            if (!done) launch_rbgs<T>(gd, rho, m, r, z, 0, s);
            if (timed) time_end(H);
            return done;
        }
        if (timed) time_begin(H, TIME_SWEEP);
        launch_rbgs<T>(geo_pass(H, g, l), rho, m, r, z, 0, s);
        if (timed) time_end(H);
    }
    return false;
}

int read_scalars(hp_handle* H) {
    HIPCHK(hipMemcpyAsync(H->host_scal, H->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost,
                          H->stream));
    HIPCHK(hipStreamSynchronize(H->stream));
    return HP_OK;
}

// What a CG loop hands to r -= alpha q: its workgroup partials of ||r||^2 (summed on the host: no
// second reduction stage on the GPU) and the breakdown flag both go straight to host memory.
RedCtl norm_export(const hp_handle* H) {
    RedCtl rc = red(H, OP_NONE);
    rc.partials = H->dev_part;
    rc.flag_out = H->dev_part + H->partial_cap;
    return rc;
}

// Split form of read_scalars for the CG loops: post_scalars marks the point of the stream up to
// which the host wants the exported partials and flag (nparts of them, see norm_export), later
// work may be enqueued behind it, and wait_scalars blocks only until that point is reached.
int post_scalars(hp_handle* H, int nparts) {
    H->host_nparts = nparts;
    HIPCHK(hipEventRecord(H->ev_scal, H->stream));
    return HP_OK;
}

bool host_breakdown(const hp_handle* H) { return H->host_part[H->partial_cap] != 0.0; }

// ||r||^2 from the partials of the last r -= alpha q, in workgroup order
double host_rr(const hp_handle* H) {
    double s = 0.0;
    for (int i = 0; i < H->host_nparts; ++i) s += H->host_part[i];
    return s;
}

int wait_scalars(hp_handle* H) {
    HIPCHK(hipEventSynchronize(H->ev_scal));
    return HP_OK;
}

// Whether a CG loop should enqueue the next direction before it has seen the residual norm of
// the current iteration.  Doing so keeps the GPU busy across the host's convergence check; the
// price is one unused preconditioner application when the iteration turns out to be the last,
// so the look-ahead stops once the norm predicted from the last observed contraction lies within
// a factor of ten of the target.
bool look_ahead(double rr_prev, double ratio, double target) {
    return !(std::sqrt(rr_prev * ratio) <= 10.0 * target);
}

// Preconditioner z = M r with <r, z> reduced under `op` (OP_RZINIT or OP_BETA).
void precond64(hp_handle* H, const double* r, double* z, int op, bool pre_done = false) {
    int64_t N = H->lv[0].N;
    if (H->mode == HP_MODE_JACOBI_PCG) {
        launch_jacobi_apply(H->lv[0].dinv, r, z, N, red(H, op), H->stream);
    } else {
        RedCtl rc = red(H, op);
        if (!vcycle<double>(H, 0, r, z, &rc, pre_done)) launch_dot<double>(r, z, N, rc, H->stream);
    }
}

// True relative residual of x into H->z (scratch); returns HP_OK and sets *rel.
int true_residual(hp_handle* H, const double* b, const double* x, double* out, double bnorm,
                  double* rel) {
    LevelData& F = H->lv[0];
    launch_apply<double>(geo<double>(H, F), F.rho, F.m, x, b, out, 3, red(H, OP_STORE, S_TMP),
                         H->stream);
    CHK(check_launch());
    CHK(read_scalars(H));
    *rel = std::sqrt(H->host_scal[S_TMP]) / bnorm;
    return HP_OK;
}

// Next direction of the FP64 PCG: z = M r (beta from <r, z>), x += alpha p (the deferred update
// of the previous step), p = z + beta p, q = A p (alpha from <p, q>).
void next_direction64(hp_handle* H, double* x, bool pre_done = false) {
    LevelData& F = H->lv[0];
    hipStream_t s = H->stream;
    precond64(H, H->r, H->z, OP_BETA, pre_done);
    launch_xpby_x<double>(H->z, H->p, x, F.N, H->scal, s, H->x_unset);
    H->x_unset = false;
    time_begin(H, TIME_APPLY);
    launch_apply<double>(geo_pass(H, geo<double>(H, F), 0), F.rho, F.m, H->p, nullptr, H->q, 1,
                         red(H, OP_ALPHA), s);
    time_end(H);
}

// FP64 PCG (Jacobi or MG preconditioner) from the current x; r holds b - A x and
// host_scal[S_RR] its squared norm on entry.
int pcg64(hp_handle* H, const double* b, double* x, double tol, double bnorm) {
    LevelData& F = H->lv[0];
    const int64_t N = F.N;
    Geo<double> g = geo<double>(H, F);
    hipStream_t s = H->stream;
    hp_stats& st = H->stats;
    const double target = tol * bnorm;
    double rr_prev = H->host_scal[S_RR], ratio = 1.0;
    bool restart = true;
    while (true) {
        if (restart) {
            precond64(H, H->r, H->z, OP_RZINIT);
            std::swap(H->z, H->p);   // p = z (z is rewritten before it is read again)
            launch_apply<double>(geo_pass(H, g, 0), F.rho, F.m, H->p, nullptr, H->q, 1, red(H, OP_ALPHA), s);
            restart = false;
        }
        // r -= alpha q now; x += alpha p is deferred to the next direction update (or the exit).
        // The next direction only reads r and the scalars, so it may run ahead of the check; it
        // then starts with the V-cycle's zero-guess pre-smoothing, which on a split finest level
        // takes the residual update along (r' into the second residual array)
        const Geo<double> gn = geo_pass(H, g, 0);
        const bool ahead = st.iterations + 1 < H->max_iter && look_ahead(rr_prev, ratio, target);
        const bool fuse = ahead && H->mode == HP_MODE_FP64_MGPCG && F.split;
        int np;
        if (fuse) {
            np = launch_presmooth_update<double>(gn, F.rho, F.dinv, H->r, H->q, H->r2, H->z, norm_export(H), s);
            std::swap(H->r, H->r2);
        } else {
            np = launch_axpy_norm<double>(H->r, H->q, N, norm_export(H), s, &gn);
        }
        CHK(check_launch());
        CHK(post_scalars(H, np));
        if (ahead) next_direction64(H, x, fuse);
        CHK(check_launch());
        CHK(wait_scalars(H));
        st.iterations++;
        if (host_breakdown(H)) return fail(HP_EBREAKDOWN, "CG breakdown: p^T A p <= 0");
        double rr = host_rr(H);
        if (!std::isfinite(rr)) return fail(HP_ENAN, "non-finite residual in iteration %d", st.iterations);
        ratio = rr_prev > 0.0 ? rr / rr_prev : 1.0;
        rr_prev = rr;
        const bool conv = std::sqrt(rr) <= target;
        // with the look-ahead the deferred x update has already been applied
        if ((conv || st.iterations >= H->max_iter) && !ahead) {
            launch_axpy_alpha<double>(x, H->p, N, H->scal, s, H->x_unset);
            H->x_unset = false;
        }
        if (conv) {
            double rel;
            CHK(true_residual(H, b, x, H->z, bnorm, &rel));
            st.rel_residual = rel;
            if (rel <= tol) {
                st.converged = 1;
                return HP_OK;
            }
            launch_copy<double>(H->z, H->r, N, s);   // continue from the true residual
            st.restarts++;
            restart = true;
            rr_prev = rel * bnorm * rel * bnorm;
            ratio = 1.0;
            if (st.iterations >= H->max_iter) break;
            continue;
        }
        if (st.iterations >= H->max_iter) break;
        if (!ahead) next_direction64(H, x);
    }
    double rel;
    CHK(true_residual(H, b, x, H->z, bnorm, &rel));
    st.rel_residual = rel;
    return fail(HP_ENOCONV, "no convergence in %d iterations (relative residual %.3e)",
                st.iterations, rel);
}

// Next direction of the inner FP32 PCG (the same steps as next_direction64 on the FP32 vectors).
void next_direction32(hp_handle* H, bool pre_done = false) {
    LevelData& F = H->lv[0];
    hipStream_t s = H->stream;
    RedCtl rc = red(H, OP_BETA);
    if (!vcycle<float>(H, 0, H->r32, H->z32, &rc, pre_done)) launch_dot<float>(H->r32, H->z32, F.N, rc, s);
    launch_xpby_x<float>(H->z32, H->p32, H->x32, F.N, H->scal, s, H->x32_unset);
    H->x32_unset = false;
    launch_apply<float>(geo_pass(H, geo<float>(H, F), 0), F.rho32, F.m32, H->p32, nullptr, H->q32, 1,
                        red(H, OP_ALPHA), s);
}

// FP32 MG-PCG on A32 d = r32 (unit-norm r32), d = x32 starts at 0 (unset: its first update writes
// it); returns inner iterations. The last update d += alpha p is left to the caller where it is
// still due (*pending): the refinement step applies it in the same pass as x += scale d.
int inner_pcg32(hp_handle* H, double eta, int budget, int* its, bool* pending) {
    LevelData& F = H->lv[0];
    const int64_t N = F.N;
    Geo<float> g = geo<float>(H, F);
    hipStream_t s = H->stream;
    H->x32_unset = true;
    *pending = false;
    {
        RedCtl rc = red(H, OP_RZINIT);
        if (!vcycle<float>(H, 0, H->r32, H->z32, &rc)) launch_dot<float>(H->r32, H->z32, N, rc, s);
    }
    std::swap(H->z32, H->p32);   // p = z (z is rewritten before it is read again)
    launch_apply<float>(geo_pass(H, g, 0), F.rho32, F.m32, H->p32, nullptr, H->q32, 1, red(H, OP_ALPHA), s);
    *its = 0;
    double rr_prev = 1.0, ratio = 1.0;
    bool ahead = false;
    // squared residual norms of the last iterations: the inner solve stops when the residual has
    // fallen by less than 2 over four iterations (FP32 cannot resolve the operator any further,
    // e.g. when its condition number approaches 1/u_32); the outer refinement then sees whether
    // the correction helped and falls back to FP64 MG-PCG if not
    double hist[4] = {0.0, 0.0, 0.0, 0.0};
    while (*its < budget) {
        // r -= alpha q; x += alpha p is deferred to the next direction update (or the end); as in
        // pcg64 the update rides on the next pre-smoothing when the next direction runs ahead
        const Geo<float> gn = geo_pass(H, g, 0);
        ahead = *its + 1 < budget && look_ahead(rr_prev, ratio, eta);
        const bool fuse = ahead && F.split;
        int np;
        if (fuse) {
            np = launch_presmooth_update<float>(gn, F.rho32, F.dinv32, H->r32, H->q32, H->r32b, H->z32,
                                                norm_export(H), s);
            std::swap(H->r32, H->r32b);
        } else {
            np = launch_axpy_norm<float>(H->r32, H->q32, N, norm_export(H), s, &gn);
        }
        CHK(check_launch());
        CHK(post_scalars(H, np));
        if (ahead) next_direction32(H, fuse);
        CHK(check_launch());
        CHK(wait_scalars(H));
        (*its)++;
        if (host_breakdown(H)) return fail(HP_EBREAKDOWN, "inner CG breakdown");
        double rr = host_rr(H);
        if (!std::isfinite(rr)) return fail(HP_ENAN, "non-finite inner residual");
        ratio = rr_prev > 0.0 ? rr / rr_prev : 1.0;
        rr_prev = rr;
        const bool stalled = *its > 4 && rr > 0.25 * hist[*its % 4];
        hist[*its % 4] = rr;
        if (std::sqrt(rr) <= eta || *its >= budget || stalled) break;
        if (!ahead) next_direction32(H);
    }
    *pending = *its > 0 && !ahead;
    return HP_OK;
}

// Mixed precision: FP64 residual and update, FP32 MG-PCG correction.
int mixed_ir(hp_handle* H, const double* b, double* x, double tol, double bnorm) {
    LevelData& F = H->lv[0];
    const int64_t N = F.N;
    hp_stats& st = H->stats;
    double rnorm = std::sqrt(H->host_scal[S_RR]);
    while (true) {
        if (rnorm <= tol * bnorm) {
            st.converged = 1;
            st.rel_residual = rnorm / bnorm;
            return HP_OK;
        }
        if (st.outer_iterations >= H->max_outer || st.iterations >= H->max_iter) break;
        launch_cast_scale_f32(H->r, H->r32, 1.0 / rnorm, N, H->stream);
        // the inner solve need not go below what the outer tolerance still requires
        double eta = std::max(H->inner_tol, 0.5 * tol * bnorm / rnorm);
        int its = 0;
        bool pending = false;
        CHK(inner_pcg32(H, eta, H->max_iter - st.iterations, &its, &pending));
        st.iterations += its;
        // x += rnorm d (x unset on the first refinement from a zero initial guess)
        launch_refine_update(x, H->x_unset, H->x32, H->x32_unset, H->p32, pending, H->scal, rnorm, N,
                             H->stream);
        H->x_unset = false;
        launch_apply<double>(geo<double>(H, F), F.rho, F.m, x, b, H->r, 3, red(H, OP_STORE, S_RR),
                             H->stream);
        CHK(check_launch());
        CHK(read_scalars(H));
        st.outer_iterations++;
        double rn = std::sqrt(H->host_scal[S_RR]);
        if (!std::isfinite(rn)) return fail(HP_ENAN, "non-finite residual in refinement");
        if (rn > 0.5 * rnorm) {
            // refinement stagnates (FP32 inner solve cannot reduce the FP64 residual): finish
            // with FP64 MG-PCG from the current iterate
            st.fallback = 1;
            int saved = H->mode;
            H->mode = HP_MODE_FP64_MGPCG;
            int rc = pcg64(H, b, x, tol, bnorm);
            H->mode = saved;
            return rc;
        }
        rnorm = rn;
    }
    st.rel_residual = rnorm / bnorm;
    return fail(HP_ENOCONV, "mixed refinement did not converge (relative residual %.3e)",
                st.rel_residual);
}

// The three fine-grid work vectors of the learned stage (warm start, FCG preconditioner, A-norm
// training step), allocated together on first use by whichever of those calls comes first.
int ensure_net_work(hp_handle* H) {
    const int64_t N = H->lv[0].N;
    int rc;
    if (!H->w1 && (rc = dalloc(H, &H->w1, N))) return rc;
    if (!H->w2 && (rc = dalloc(H, &H->w2, N))) return rc;
    if (!H->w3 && (rc = dalloc(H, &H->w3, N))) return rc;
    return HP_OK;
}

bool net_work_ready(const hp_handle* H) { return H->w1 && H->w2 && H->w3; }

// Flexible CG (Notay's FCG with one stored direction) with the preconditioner
// B(r) = g z1 + M (r - g A z1), z1 = network estimate of A^-1 r, M = one V-cycle, and
// g = <r, z1> / <z1, A z1> the step that minimises the A-norm error of g z1 (0 if the network
// points uphill or returns non-finite values), so the network stage never makes the
// correction worse than the V-cycle alone. The network makes B nonlinear, so
// beta = -<z, q_prev> / <p_prev, q_prev> keeps the new direction A-orthogonal to the previous
// one. If the residual stops falling (less than 10x over 10 iterations) the solve finishes with
// plain FP64 MG-PCG from the current iterate. Stops on the same FP64 true residual as the other
// modes.
int fcg_learned(hp_handle* H, const double* b, double* x, double tol, double bnorm) {
    if (!H->net) return fail(HP_EINVAL, "HP_MODE_LEARNED needs a network (hp_attach_net)");
    if (!net_work_ready(H)) return fail(HP_EINVAL, "learned-stage work vectors are missing");
    LevelData& F = H->lv[0];
    const int64_t N = F.N;
    Geo<double> g = geo<double>(H, F);
    hipStream_t s = H->stream;
    hp_stats& st = H->stats;
    // Every scalar stays on the device (dot products into slots, hp_fcg.hip for g, alpha, beta);
    // the host waits once per iteration, for ||r||^2 and p^T A p.
    auto dot = [&](const double* u, const double* v, int slot) {
        launch_dot<double>(u, v, N, red(H, OP_STORE, slot), s);
    };
    // z = g y + M (r - g A y), y = net(r), g = <r, y> / <y, A y> (0 if not both positive)
    auto precond = [&](const double* r, double* z) -> int {
        // the network reads r and writes y in the finest level's storage order (its coefficient
        // inputs in natural order)
        const int rc = F.split ? nn_apply(H->net, s, r, H->rho_nat, H->m_nat, nullptr, H->w1, 1)
                               : nn_apply(H->net, s, r, F.rho, F.m, nullptr, H->w1);
        if (rc) return fail(rc, "network: %s", nn_error());
        launch_apply<double>(g, F.rho, F.m, H->w1, nullptr, H->w2, 0, red(H, OP_NONE), s);
        dot(r, H->w1, S_T1);
        dot(H->w1, H->w2, S_T2);
        launch_fcg_scalar(H->scal, FCG_GAMMA, s);
        launch_fcg_gamma_update(H->w2, r, H->scal, N, true, s);    // w2 = r - g A y
        vcycle<double>(H, 0, H->w2, z);
        launch_fcg_gamma_update(z, H->w1, H->scal, N, false, s);  // z += g y
        return check_launch();
    };
    // q = A p with p^T A p into S_PQ
    auto apply_pq = [&]() {
        launch_apply<double>(g, F.rho, F.m, H->p, nullptr, H->q, 1, red(H, OP_STORE, S_PQ), s);
    };
    std::vector<double> hist;
    bool restart = true;
    while (true) {
        if (restart) {
            CHK(precond(H->r, H->z));
            launch_copy<double>(H->z, H->p, N, s);
            apply_pq();
            restart = false;
        }
        dot(H->p, H->r, S_T1);
        launch_fcg_scalar(H->scal, FCG_ALPHA, s);          // alpha = <p, r> / p^T A p
        launch_axpy2_norm<double>(x, H->p, H->r, H->q, N, red(H, OP_STORE, S_RR), s);
        CHK(check_launch());
        CHK(read_scalars(H));
        st.iterations++;
        const double pq = H->host_scal[S_PQ];
        if (!(pq > 0.0) || !std::isfinite(pq)) return fail(HP_EBREAKDOWN, "FCG breakdown: p^T A p <= 0");
        double rr = H->host_scal[S_RR];
        if (!std::isfinite(rr)) return fail(HP_ENAN, "non-finite residual in iteration %d", st.iterations);
        if (std::sqrt(rr) <= tol * bnorm) {
            double rel;
            CHK(true_residual(H, b, x, H->z, bnorm, &rel));
            st.rel_residual = rel;
            if (rel <= tol) {
                st.converged = 1;
                return HP_OK;
            }
            launch_copy<double>(H->z, H->r, N, s);
            st.restarts++;
            restart = true;
            if (st.iterations >= H->max_iter) break;
            continue;
        }
        if (st.iterations >= H->max_iter) break;
        hist.push_back(std::sqrt(rr));
        if (hist.size() > 10 && hist.back() > 0.1 * hist[hist.size() - 11]) {
            // the learned stage is not helping: finish with plain FP64 MG-PCG (r is current)
            st.fallback = 1;
            int saved = H->mode;
            H->mode = HP_MODE_FP64_MGPCG;
            int rc = pcg64(H, b, x, tol, bnorm);
            H->mode = saved;
            return rc;
        }
        CHK(precond(H->r, H->z));
        dot(H->z, H->q, S_T1);
        launch_fcg_scalar(H->scal, FCG_BETA, s);           // beta = -<z, A p_old> / p_old^T A p_old
        launch_xpby<double>(H->z, H->p, N, H->scal, s);
        apply_pq();
        CHK(check_launch());
    }
    double rel;
    CHK(true_residual(H, b, x, H->z, bnorm, &rel));
    st.rel_residual = rel;
    return fail(HP_ENOCONV, "no convergence in %d iterations (relative residual %.3e)",
                st.iterations, rel);
}

int level_ok(const hp_handle* H, int level) {
    if (!H) return fail(HP_EINVAL, "null handle");
    if (level < 0 || level >= (int)H->lv.size()) return fail(HP_EINVAL, "level %d out of range", level);
    return HP_OK;
}

// Scratch vectors of the finest level for the building blocks, which take and return natural
// order: a split finest level is relaid through the CG work vectors p and q (FP64) or p32 and
// q32 (FP32), which hold nothing between solves.
template <typename T> T* tmp_a(hp_handle* H);
template <typename T> T* tmp_b(hp_handle* H);
template <> double* tmp_a<double>(hp_handle* H) { return H->p; }
template <> double* tmp_b<double>(hp_handle* H) { return H->q; }
template <> float* tmp_a<float>(hp_handle* H) { return H->p32; }
template <> float* tmp_b<float>(hp_handle* H) { return H->q32; }

template <typename T>
int apply_t(hp_handle* H, int level, const T* x, T* y) {
    CHK(level_ok(H, level));
    if (!x || !y) return fail(HP_EINVAL, "null vector");
    LevelData& L = H->lv[level];
    if (L.split) {
        T *a = tmp_a<T>(H), *c = tmp_b<T>(H);
        relayout_l<T>(H, level, x, a, 1);
        launch_apply<T>(geo<T>(H, L), lvl_rho<T>(L), lvl_m<T>(L), a, nullptr, c, 0, red(H, OP_NONE),
                        H->stream);
        relayout_l<T>(H, level, c, y, 0);
        return check_launch();
    }
    launch_apply<T>(geo<T>(H, L), lvl_rho<T>(L), lvl_m<T>(L), x, nullptr, y, 0, red(H, OP_NONE),
                    H->stream);
    return check_launch();
}

template <typename T>
int smooth_t(hp_handle* H, int level, const T* r, T* z, int colour) {
    CHK(level_ok(H, level));
    if (!r || !z) return fail(HP_EINVAL, "null vector");
    if (colour != 0 && colour != 1) return fail(HP_EINVAL, "colour must be 0 or 1");
    LevelData& L = H->lv[level];
    if (L.split) {
        T *a = tmp_a<T>(H), *c = tmp_b<T>(H);
        relayout_l<T>(H, level, r, a, 1);
        relayout_l<T>(H, level, z, c, 1);
        launch_rbgs<T>(geo<T>(H, L), lvl_rho<T>(L), lvl_m<T>(L), a, c, colour, H->stream);
        relayout_l<T>(H, level, c, z, 0);
        return check_launch();
    }
    launch_rbgs<T>(geo<T>(H, L), lvl_rho<T>(L), lvl_m<T>(L), r, z, colour, H->stream);
    return check_launch();
}

template <typename T>
int restrict_t(hp_handle* H, int level, const T* r, const T* z, T* rc) {
    CHK(level_ok(H, level));
    if (level + 1 >= (int)H->lv.size()) return fail(HP_EINVAL, "no coarser level below %d", level);
    if (!r || !z || !rc) return fail(HP_EINVAL, "null vector");
    LevelData& L = H->lv[level];
    LevelData& C = H->lv[level + 1];
    if (L.split) {
        T *a = tmp_a<T>(H), *c = tmp_b<T>(H);
        relayout_l<T>(H, level, r, a, 1);
        relayout_l<T>(H, level, z, c, 1);
        r = a;
        z = c;
    }
    launch_apply<T>(geo<T>(H, L), lvl_rho<T>(L), lvl_m<T>(L), z, r, lvl_t<T>(L), 2, red(H, OP_NONE),
                    H->stream);
    // a split coarse level: restrict into its scratch vector t, then back to natural order
    launch_restrict<T>(transfer(H, level), lvl_t<T>(L), C.split ? lvl_t<T>(C) : rc, H->stream);
    if (C.split) relayout_l<T>(H, level + 1, lvl_t<T>(C), rc, 0);
    return check_launch();
}

template <typename T>
int prolong_t(hp_handle* H, int level, const T* ec, T* z) {
    CHK(level_ok(H, level));
    if (level + 1 >= (int)H->lv.size()) return fail(HP_EINVAL, "no coarser level below %d", level);
    if (!ec || !z) return fail(HP_EINVAL, "null vector");
    LevelData& C = H->lv[level + 1];
    if (C.split) {  // the coarse correction in split order, in the coarse level's scratch vector t
        relayout_l<T>(H, level + 1, ec, lvl_t<T>(C), 1);
        ec = lvl_t<T>(C);
    }
    if (H->lv[level].split) {
        T* a = tmp_a<T>(H);
        relayout_l<T>(H, level, z, a, 1);
        launch_prolong_add<T>(transfer(H, level), ec, a, H->stream);
        relayout_l<T>(H, level, a, z, 0);
        return check_launch();
    }
    launch_prolong_add<T>(transfer(H, level), ec, z, H->stream);
    return check_launch();
}

template <typename T>
int coarse_t(hp_handle* H, const T* b, T* x) {
    if (!H) return fail(HP_EINVAL, "null handle");
    if (!b || !x) return fail(HP_EINVAL, "null vector");
    launch_coarse_solve<T>(H->ainv, H->nc, b, x, H->stream);
    return check_launch();
}

template <typename T>
int precond_t(hp_handle* H, const T* r, T* z) {
    if (!H) return fail(HP_EINVAL, "null handle");
    if (!r || !z) return fail(HP_EINVAL, "null vector");
    if (H->lv[0].split) {
        T *a = tmp_a<T>(H), *c = tmp_b<T>(H);
        relayout0<T>(H, r, a, 1);
        vcycle<T>(H, 0, a, c);
        relayout0<T>(H, c, z, 0);
        return check_launch();
    }
    vcycle<T>(H, 0, r, z);
    return check_launch();
}

}  // namespace

// =============================================================================================
// C ABI

extern "C" {

const char* hp_last_error(void) { return g_err.c_str(); }

int hp_setup(const hp_grid* grid, const double* rho, const double* c2, double dt, const hp_bc* bc,
             hp_handle** out) {
    return hp_setup_two_density(grid, rho, rho, c2, dt, bc, out);
}

int hp_setup_two_density(const hp_grid* grid, const double* rho_n, const double* rho_np1, const double* c2,
                         double dt, const hp_bc* bc, hp_handle** out) {
    g_err.clear();
    if (!grid || !bc || !out) return fail(HP_EINVAL, "grid, bc and out must be non-null");
    *out = nullptr;
    const int n[3] = {grid->nx, grid->ny, grid->nz};
    const double hs[3] = {grid->hx, grid->hy, grid->hz};
    const int bcs[3] = {bc->x, bc->y, bc->z};
    int64_t N = 1;
    for (int d = 0; d < 3; ++d) {
        if (n[d] < 1) return fail(HP_EINVAL, "grid size must be >= 1 on every axis");
        if (!(hs[d] > 0.0) || !std::isfinite(hs[d])) return fail(HP_EINVAL, "spacings must be positive");
        if (bcs[d] != HP_BC_PERIODIC && bcs[d] != HP_BC_NEUMANN) return fail(HP_EINVAL, "unknown boundary kind");
        if (bcs[d] == HP_BC_PERIODIC && n[d] > 1 && n[d] % 2 != 0)
            return fail(HP_EINVAL, "periodic axes need an even number of cells (red-black colouring)");
        N *= n[d];
    }
    if (N >= (int64_t)1 << 31) return fail(HP_EINVAL, "grid has too many cells (limit 2^31 - 1)");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(HP_EINVAL, "dt must be positive and finite");
    if (!rho_n || !rho_np1 || !c2) return fail(HP_EINVAL, "rho and c2 must be non-null");

    hp_handle* H = new hp_handle();
    H->grid = *grid;
    H->bc = *bc;
    H->dt = dt;
    int rc = HP_OK;
    auto bail = [&](int code) {
        hp_free(H);
        return code;
    };
    if (hipGetDevice(&H->device) != hipSuccess) return bail(fail(HP_EHIP, "no HIP device"));

    // hierarchy dimensions
    LevelData L0;
    for (int d = 0; d < 3; ++d) {
        L0.n[d] = n[d];
        L0.h[d] = hs[d];
        L0.coarsened[d] = 0;
    }
    L0.N = N;
    H->lv.push_back(L0);
    while (true) {
        const LevelData& L = H->lv.back();
        int fl[3];
        bool any = false;
        for (int d = 0; d < 3; ++d) {
            fl[d] = can_coarsen(L.n[d], bcs[d]);
            any = any || fl[d];
        }
        if (L.N <= H->coarsest_max || !any) break;
        LevelData C;
        C.N = 1;
        for (int d = 0; d < 3; ++d) {
            C.n[d] = fl[d] ? L.n[d] / 2 : L.n[d];
            C.h[d] = fl[d] ? 2.0 * L.h[d] : L.h[d];
            C.coarsened[d] = fl[d];
            C.N *= C.n[d];
        }
        H->lv.push_back(C);
    }
    H->nc = (int)H->lv.back().N;
    if (H->nc > 4096)
        return bail(fail(HP_EINVAL, "grid cannot be coarsened below 4096 cells (coarsest %d); use sizes with more factors of 2", H->nc));

    // allocations
    for (size_t l = 0; l < H->lv.size(); ++l) {
        LevelData& L = H->lv[l];
        if ((rc = dalloc(H, &L.rho, L.N)) || (rc = dalloc(H, &L.m, L.N)) ||
            (rc = dalloc(H, &L.rho32, L.N)) || (rc = dalloc(H, &L.m32, L.N)) ||
            (rc = dalloc(H, &L.dinv, L.N)) || (rc = dalloc(H, &L.dinv32, L.N)))
            return bail(rc);
        if (l > 0) {
            if ((rc = dalloc(H, &L.r, L.N)) || (rc = dalloc(H, &L.z, L.N)) ||
                (rc = dalloc(H, &L.r32, L.N)) || (rc = dalloc(H, &L.z32, L.N)))
                return bail(rc);
        }
        if (l + 1 < H->lv.size()) {
            if ((rc = dalloc(H, &L.t, L.N)) || (rc = dalloc(H, &L.t32, L.N))) return bail(rc);
        }
    }
    if ((rc = dalloc(H, &H->ainv, (int64_t)H->nc * H->nc)) ||
        (rc = dalloc(H, &H->ainv_work, spd_inverse_work(H->nc))))
        return bail(rc);
    if ((rc = dalloc(H, &H->r, N)) || (rc = dalloc(H, &H->z, N)) || (rc = dalloc(H, &H->p, N)) ||
        (rc = dalloc(H, &H->q, N)) || (rc = dalloc(H, &H->r2, N)))
        return bail(rc);
    if ((rc = dalloc(H, &H->x32, N)) || (rc = dalloc(H, &H->r32, N)) ||
        (rc = dalloc(H, &H->z32, N)) || (rc = dalloc(H, &H->p32, N)) || (rc = dalloc(H, &H->q32, N)) ||
        (rc = dalloc(H, &H->r32b, N)))
        return bail(rc);
    int64_t cap = std::max<int64_t>(reduce_blocks_vec(N), 1);
    for (auto& L : H->lv)
        cap = std::max(cap, reduce_blocks_cells(L.n[0], L.n[1], L.n[2]));
    H->partial_cap = cap;
    if ((rc = dalloc(H, &H->partials, cap)) || (rc = dalloc(H, &H->partials2, cap)) ||
        (rc = dalloc(H, &H->scal, S_COUNT)) ||
        (rc = dalloc(H, &H->flag, 2)))
        return bail(rc);
    if (hipHostMalloc((void**)&H->host_scal, S_COUNT * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&H->host_part, (cap + 1) * sizeof(double),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc((void**)&H->host_flag, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess)
        return bail(fail(HP_ENOMEM, "pinned host allocation failed"));
    if (hipHostGetDevicePointer((void**)&H->dev_part, H->host_part, 0) != hipSuccess)
        return bail(fail(HP_EHIP, "hipHostGetDevicePointer failed"));
    if (hipEventCreate(&H->ev0) != hipSuccess || hipEventCreate(&H->ev1) != hipSuccess ||
        hipEventCreateWithFlags(&H->ev_scal, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&H->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&H->ev_join, hipEventDisableTiming) != hipSuccess)
        return bail(fail(HP_EHIP, "hipEventCreate failed"));
    if (hipStreamCreateWithFlags(&H->side, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(HP_EHIP, "hipStreamCreateWithFlags failed"));
    if (hipMemsetAsync(H->scal, 0, S_COUNT * sizeof(double), H->stream) != hipSuccess)
        return bail(fail(HP_EHIP, "hipMemsetAsync failed"));
    H->want_split = split_allowed(H) ? 1 : 0;
    if ((rc = load_coefficients(H, rho_n, rho_np1, c2, dt))) return bail(rc);
    H->stats.levels = (int)H->lv.size();
    *out = H;
    return HP_OK;
}

void hp_free(hp_handle* H) {
    if (!H) return;
    if (H->stream) (void)hipStreamSynchronize(H->stream);
    else (void)hipDeviceSynchronize();
    for (void* p : H->allocs) (void)hipFree(p);
    if (H->host_scal) (void)hipHostFree(H->host_scal);
    if (H->host_part) (void)hipHostFree(H->host_part);
    if (H->host_flag) (void)hipHostFree(H->host_flag);
    if (H->ev0) (void)hipEventDestroy(H->ev0);
    if (H->ev1) (void)hipEventDestroy(H->ev1);
    if (H->ev_scal) (void)hipEventDestroy(H->ev_scal);
    if (H->ev_fork) (void)hipEventDestroy(H->ev_fork);
    if (H->ev_join) (void)hipEventDestroy(H->ev_join);
    if (H->side) {
        (void)hipStreamSynchronize(H->side);
        (void)hipStreamDestroy(H->side);
    }
    for (hipEvent_t e : H->tev) (void)hipEventDestroy(e);
    delete H;
}

int hp_set_stream(hp_handle* H, void* stream) {
    if (!H) return fail(HP_EINVAL, "null handle");
    H->stream = (hipStream_t)stream;
    return HP_OK;
}

int hp_set_option(hp_handle* H, int key, double v) {
    if (!H) return fail(HP_EINVAL, "null handle");
    switch (key) {
        case HP_OPT_MODE:
            if (v != HP_MODE_JACOBI_PCG && v != HP_MODE_FP64_MGPCG && v != HP_MODE_MIXED_IR &&
                v != HP_MODE_LEARNED)
                return fail(HP_EINVAL, "unknown mode");
            H->mode = (int)v;
            return HP_OK;
        case HP_OPT_MAX_ITER:
            if (!(v >= 1)) return fail(HP_EINVAL, "max_iter must be >= 1");
            H->max_iter = (int)v;
            return HP_OK;
        case HP_OPT_NU_PRE:
        case HP_OPT_NU_POST:
            if (!(v >= 1 && v <= 8)) return fail(HP_EINVAL, "smoothing sweeps must be in 1..8");
            (key == HP_OPT_NU_PRE ? H->nu_pre : H->nu_post) = (int)v;
            return HP_OK;
        case HP_OPT_INNER_TOL:
            if (!(v > 0.0 && v < 1.0)) return fail(HP_EINVAL, "inner tolerance must be in (0, 1)");
            H->inner_tol = v;
            return HP_OK;
        case HP_OPT_MAX_OUTER:
            if (!(v >= 1)) return fail(HP_EINVAL, "max_outer must be >= 1");
            H->max_outer = (int)v;
            return HP_OK;
        case HP_OPT_KERNEL_TIMING:
            if (v != 0.0 && v != 1.0) return fail(HP_EINVAL, "kernel timing must be 0 or 1");
            H->timing = (int)v;
            return HP_OK;
        case HP_OPT_FACE_RULE: {
            if (v != 0.0 && v != 1.0) return fail(HP_EINVAL, "face rule must be 0 or 1");
            if ((int)v == H->face_rule) return HP_OK;
            H->face_rule = (int)v;
            // the rule enters the Jacobi diagonals of every level and the coarsest inverse:
            // recomputed in natural order, then the layout is restored
            const int was_split = H->lv[0].split;
            int rc = set_layout(H, 0);
            if (rc) return rc;
            for (auto& L : H->lv)
                launch_jacobi_diag(geo<double>(H, L), geo<float>(H, L), L.rho, L.m, L.rho32, L.m32, L.dinv,
                                   L.dinv32, false, H->stream);
            CHK(check_launch());
            CHK(build_coarse_inverse(H));
            return was_split ? set_layout(H, 1) : HP_OK;
        }
        case HP_OPT_LAYOUT: {
            if (v != 0.0 && v != 1.0) return fail(HP_EINVAL, "layout must be 0 (natural) or 1 (split)");
            if (v == 1.0 && !split_allowed(H)) return fail(HP_EINVAL, "the grid does not allow the split layout");
            int rc = set_layout(H, (int)v);
            if (rc == HP_OK) H->want_split = (int)v;
            return rc;
        }
        default:
            return fail(HP_EINVAL, "unknown or read-only option %d", key);
    }
}

int hp_get_option(const hp_handle* H, int key, double* v) {
    if (!H || !v) return fail(HP_EINVAL, "null argument");
    switch (key) {
        case HP_OPT_MODE: *v = H->mode; return HP_OK;
        case HP_OPT_MAX_ITER: *v = H->max_iter; return HP_OK;
        case HP_OPT_NU_PRE: *v = H->nu_pre; return HP_OK;
        case HP_OPT_NU_POST: *v = H->nu_post; return HP_OK;
        case HP_OPT_INNER_TOL: *v = H->inner_tol; return HP_OK;
        case HP_OPT_MAX_OUTER: *v = H->max_outer; return HP_OK;
        case HP_OPT_COARSEST_MAX: *v = H->coarsest_max; return HP_OK;
        case HP_OPT_LAYOUT: *v = H->lv[0].split; return HP_OK;
        case HP_OPT_KERNEL_TIMING: *v = H->timing; return HP_OK;
        case HP_OPT_FACE_RULE: *v = H->face_rule; return HP_OK;
        default: return fail(HP_EINVAL, "unknown option %d", key);
    }
}

int hp_update_coefficients(hp_handle* H, const double* rho, const double* c2, double dt) {
    return hp_update_coefficients_two_density(H, rho, rho, c2, dt);
}

int hp_update_coefficients_two_density(hp_handle* H, const double* rho_n, const double* rho_np1,
                                       const double* c2, double dt) {
    if (!H) return fail(HP_EINVAL, "null handle");
    g_err.clear();
    return load_coefficients(H, rho_n, rho_np1, c2, dt);
}

int hp_neumann_rhs(hp_handle* H, int axis, int side, const double* q, double* rhs) {
    if (!H) return fail(HP_EINVAL, "null handle");
    g_err.clear();
    if (!q || !rhs) return fail(HP_EINVAL, "null vector");
    if (axis < 0 || axis > 2 || (side != 0 && side != 1)) return fail(HP_EINVAL, "axis must be 0..2, side 0 or 1");
    const int bcs[3] = {H->bc.x, H->bc.y, H->bc.z};
    if (bcs[axis] != HP_BC_NEUMANN) return fail(HP_EINVAL, "Neumann data needs a Neumann axis");
    const LevelData& F = H->lv[0];
    launch_neumann_rhs(F.n[0], F.n[1], F.n[2], axis, side, H->dt * H->dt / F.h[axis], q, rhs, H->stream);
    return check_launch();
}

int hp_get_stats(const hp_handle* H, hp_stats* out) {
    if (!H || !out) return fail(HP_EINVAL, "null argument");
    *out = H->stats;
    return HP_OK;
}

int hp_solve(hp_handle* H, const double* b, double* x, double tol) {
    if (!H) return fail(HP_EINVAL, "null handle");
    g_err.clear();
    if (!b || !x) return fail(HP_EINVAL, "rhs and p must be non-null");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(HP_EINVAL, "tol must be positive");
    hp_stats& st = H->stats;
    int levels = st.levels;
    st = hp_stats{};
    st.levels = levels;
    H->dir = 0;  // the same sequence of pass directions (and so of reduction orders) every solve
    LevelData& F = H->lv[0];
    const int64_t N = F.N;
    hipStream_t s = H->stream;
    H->spans.clear();
    H->tev_used = 0;
    HIPCHK(hipEventRecord(H->ev0, s));
    HIPCHK(hipMemsetAsync(H->flag, 0, sizeof(int), s));
    HIPCHK(hipMemsetAsync(H->scal, 0, S_COUNT * sizeof(double), s));
    // in the split layout the solve runs on split copies of b and x (made in the pass that checks
    // them, takes ||b|| and notes whether x is zero; the pass over b also leaves b in r, the initial
    // residual when x is zero); x is copied back at the end
    double* xu = x;
    int rc;
    if (F.split) {
        launch_relayout_in(b, H->bs, F.n[0], F.n[1], F.n[2], H->flag, 0, red(H, OP_STORE, S_BB), s, H->r);
        // x is only checked here; it is relaid only where it is not zero
        launch_relayout_in(x, nullptr, F.n[0], F.n[1], F.n[2], H->flag, 2, red(H, OP_NONE), s);
        b = H->bs;
        x = H->xs;
        if ((rc = check_launch())) return rc;
        HIPCHK(hipMemcpyAsync(H->host_flag, H->flag, sizeof(int), hipMemcpyDeviceToHost, s));
        if ((rc = read_scalars(H))) return rc;
        if (*H->host_flag & 1) {
            st.status = HP_ENAN;
            return fail(HP_ENAN, "rhs or initial guess contains non-finite values");
        }
        if (*H->host_flag & 2) {
            launch_relayout_in(xu, H->xs, F.n[0], F.n[1], F.n[2], H->flag, 0, red(H, OP_NONE), s);
            launch_apply<double>(geo<double>(H, F), F.rho, F.m, x, b, H->r, 3, red(H, OP_STORE, S_RR), s);
            if ((rc = check_launch()) || (rc = read_scalars(H))) return rc;
        } else {  // x = 0: the initial residual is b itself, already in r; the split x stays unset
            H->host_scal[S_RR] = H->host_scal[S_BB];
            H->x_unset = true;
        }
    } else {
        launch_check_finite(b, N, H->flag, s);
        launch_check_finite(x, N, H->flag, s);
        launch_dot<double>(b, b, N, red(H, OP_STORE, S_BB), s);
        launch_apply<double>(geo<double>(H, F), F.rho, F.m, x, b, H->r, 3, red(H, OP_STORE, S_RR), s);
        if ((rc = check_launch())) return rc;
        HIPCHK(hipMemcpyAsync(H->host_flag, H->flag, sizeof(int), hipMemcpyDeviceToHost, s));
        if ((rc = read_scalars(H))) return rc;
        if (*H->host_flag) {
            st.status = HP_ENAN;
            return fail(HP_ENAN, "rhs or initial guess contains non-finite values");
        }
    }
    double bnorm = std::sqrt(H->host_scal[S_BB]);
    if (bnorm == 0.0) {
        launch_fill<double>(xu, 0.0, N, s);
        st.converged = 1;
        st.rel_residual = 0.0;
        rc = HP_OK;
    } else if (std::sqrt(H->host_scal[S_RR]) <= tol * bnorm) {
        st.converged = 1;
        st.rel_residual = std::sqrt(H->host_scal[S_RR]) / bnorm;
        rc = HP_OK;
    } else {
        // FP64 MG-PCG, Jacobi-PCG and mixed precision take an unset (zero) split iterate; the
        // learned form gets zeros
        if (H->x_unset && H->mode == HP_MODE_LEARNED) {
            launch_fill<double>(x, 0.0, N, s);
            H->x_unset = false;
        }
        if (H->mode == HP_MODE_MIXED_IR)
            rc = mixed_ir(H, b, x, tol, bnorm);
        else if (H->mode == HP_MODE_LEARNED)
            rc = fcg_learned(H, b, x, tol, bnorm);
        else
            rc = pcg64(H, b, x, tol, bnorm);
    }
    // an iterate that was never written is the caller's zero initial guess, already in place
    if (F.split && bnorm != 0.0 && !H->x_unset) relayout0<double>(H, x, xu, 0);
    H->x_unset = false;
    HIPCHK(hipEventRecord(H->ev1, s));
    HIPCHK(hipEventSynchronize(H->ev1));
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, H->ev0, H->ev1);
    st.time_ms = ms;
    for (const auto& sp : H->spans) {
        float d = 0.0f;
        if (hipEventElapsedTime(&d, H->tev[sp.second], H->tev[sp.second + 1]) != hipSuccess) continue;
        if (sp.first == TIME_SWEEP) {
            st.timed_sweeps++;
            st.sweep_ms += d;
        } else {
            st.timed_applies++;
            st.apply_ms += d;
        }
    }
    if (st.timed_sweeps) st.sweep_ms /= st.timed_sweeps;
    if (st.timed_applies) st.apply_ms /= st.timed_applies;
    st.status = rc;
    return rc;
}

// ---- building blocks ----

int hp_num_levels(const hp_handle* H) { return H ? (int)H->lv.size() : 0; }

int hp_level_info(const hp_handle* H, int level, int* n, double* hs) {
    CHK(level_ok(H, level));
    const LevelData& L = H->lv[level];
    for (int d = 0; d < 3; ++d) {
        if (n) n[d] = L.n[d];
        if (hs) hs[d] = L.h[d];
    }
    return HP_OK;
}

int hp_apply(hp_handle* H, int level, const double* x, double* y) { return apply_t(H, level, x, y); }
int hp_apply_f32(hp_handle* H, int level, const float* x, float* y) { return apply_t(H, level, x, y); }

int hp_smooth(hp_handle* H, int level, const double* r, double* z, int colour) { return smooth_t(H, level, r, z, colour); }
int hp_smooth_f32(hp_handle* H, int level, const float* r, float* z, int colour) { return smooth_t(H, level, r, z, colour); }

int hp_restrict_residual(hp_handle* H, int level, const double* r, const double* z, double* rc) { return restrict_t(H, level, r, z, rc); }
int hp_restrict_residual_f32(hp_handle* H, int level, const float* r, const float* z, float* rc) { return restrict_t(H, level, r, z, rc); }

int hp_prolong_add(hp_handle* H, int level, const double* ec, double* z) { return prolong_t(H, level, ec, z); }
int hp_prolong_add_f32(hp_handle* H, int level, const float* ec, float* z) { return prolong_t(H, level, ec, z); }

int hp_coarse_solve(hp_handle* H, const double* b, double* x) { return coarse_t(H, b, x); }
int hp_coarse_solve_f32(hp_handle* H, const float* b, float* x) { return coarse_t(H, b, x); }

int hp_precond(hp_handle* H, const double* r, double* z) { return precond_t(H, r, z); }
int hp_precond_f32(hp_handle* H, const float* r, float* z) { return precond_t(H, r, z); }

int hp_residual(hp_handle* H, const double* b, const double* x, double* r, double* rel) {
    if (!H) return fail(HP_EINVAL, "null handle");
    if (!b || !x || !r) return fail(HP_EINVAL, "null vector");
    LevelData& F = H->lv[0];
    if (F.split) {
        relayout0<double>(H, b, H->p, 1);
        relayout0<double>(H, x, H->q, 1);
        launch_apply<double>(geo<double>(H, F), F.rho, F.m, H->q, H->p, H->z, 3, red(H, OP_STORE, S_RR),
                             H->stream);
        relayout0<double>(H, H->z, r, 0);
    } else {
        launch_apply<double>(geo<double>(H, F), F.rho, F.m, x, b, r, 3, red(H, OP_STORE, S_RR), H->stream);
    }
    launch_dot<double>(b, b, F.N, red(H, OP_STORE, S_BB), H->stream);
    CHK(check_launch());
    if (rel) {
        CHK(read_scalars(H));
        double bb = H->host_scal[S_BB];
        *rel = bb > 0.0 ? std::sqrt(H->host_scal[S_RR] / bb) : std::sqrt(H->host_scal[S_RR]);
    }
    return HP_OK;
}

int hp_attach_net(hp_handle* H, hp_net* net) {
    if (!H) return fail(HP_EINVAL, "null handle");
    if (net) {
        int nx, ny, nz;
        nn_grid(net, &nx, &ny, &nz);
        const LevelData& F = H->lv[0];
        if (nx != F.n[0] || ny != F.n[1] || nz != F.n[2])
            return fail(HP_EINVAL, "network grid %dx%dx%d differs from the solver grid %dx%dx%d", nx, ny,
                        nz, F.n[0], F.n[1], F.n[2]);
        CHK(ensure_net_work(H));
    }
    H->net = net;
    return HP_OK;
}

int hp_warm_start(hp_handle* H, const double* b, const double* p_prev, double* x) {
    if (!H) return fail(HP_EINVAL, "null handle");
    g_err.clear();
    if (!H->net) return fail(HP_EINVAL, "hp_warm_start needs a network (hp_attach_net)");
    if (!b || !x) return fail(HP_EINVAL, "null vector");
    if (!net_work_ready(H)) return fail(HP_EINVAL, "learned-stage work vectors are missing");
    LevelData& F = H->lv[0];
    const int64_t N = F.N;
    hipStream_t s = H->stream;
    int rc = nn_apply(H->net, s, b, rho_natural(H), m_natural(H), p_prev, x);
    if (rc) return fail(rc, "network: %s", nn_error());
    const double* xa = x;  // x in the finest level's layout
    if (F.split) {
        relayout0<double>(H, x, H->p, 1);
        xa = H->p;
    }
    launch_apply<double>(geo<double>(H, F), F.rho, F.m, xa, nullptr, H->w2, 0, red(H, OP_NONE), s);
    launch_dot<double>(b, x, N, red(H, OP_STORE, S_TMP), s);
    CHK(check_launch());
    CHK(read_scalars(H));
    const double bx = H->host_scal[S_TMP];
    launch_dot<double>(xa, H->w2, N, red(H, OP_STORE, S_TMP), s);
    CHK(check_launch());
    CHK(read_scalars(H));
    const double xax = H->host_scal[S_TMP];
    const double gam = (bx > 0.0 && xax > 0.0 && std::isfinite(bx) && std::isfinite(xax)) ? bx / xax : 0.0;
    launch_axpby(0.0, x, gam, x, N, s);
    if (gam == 0.0) launch_fill<double>(x, 0.0, N, s);
    return check_launch();
}

int hp_nn_train_step_anorm(hp_handle* H, hp_net* net, const double* b, const double* p_prev,
                           const double* x, float lr, double* loss) {
    if (!H || !net) return fail(HP_EINVAL, "null handle or network");
    g_err.clear();
    if (!b || !x) return fail(HP_EINVAL, "null vector");
    if (!(lr > 0.f)) return fail(HP_EINVAL, "learning rate must be positive");
    int nx, ny, nz;
    nn_grid(net, &nx, &ny, &nz);
    LevelData& F = H->lv[0];
    if (nx != F.n[0] || ny != F.n[1] || nz != F.n[2]) return fail(HP_EINVAL, "network grid differs from the solver grid");
    CHK(ensure_net_work(H));
    const int64_t N = F.N;
    hipStream_t s = H->stream;
    Geo<double> g = geo<double>(H, F);
    int rc = nn_train_forward(net, s, b, rho_natural(H), m_natural(H), p_prev);
    if (rc) return fail(rc, "network: %s", nn_error());
    // <x, A x> (A in the finest level's layout)
    const double* xa = x;
    if (F.split) {
        relayout0<double>(H, x, H->p, 1);
        xa = H->p;
    }
    launch_apply<double>(g, F.rho, F.m, xa, nullptr, H->w2, 0, red(H, OP_NONE), s);
    launch_dot<double>(xa, H->w2, N, red(H, OP_STORE, S_TMP), s);
    CHK(check_launch());
    CHK(read_scalars(H));
    const double xax = H->host_scal[S_TMP];
    if (!(xax > 0.0)) return fail(HP_EINVAL, "target must be nonzero");
    // d = estimate - x, q = A d, loss = <d, q> / <x, A x>
    if ((rc = nn_output_minus(net, x, H->w1))) return fail(rc, "network: %s", nn_error());
    const double* da = H->w1;
    if (F.split) {
        relayout0<double>(H, H->w1, H->p, 1);
        da = H->p;
    }
    launch_apply<double>(g, F.rho, F.m, da, nullptr, H->w2, 0, red(H, OP_NONE), s);
    launch_dot<double>(da, H->w2, N, red(H, OP_STORE, S_TMP), s);
    CHK(check_launch());
    CHK(read_scalars(H));
    if (loss) *loss = H->host_scal[S_TMP] / xax;
    // dL/d(estimate) = 2 A d / <x, A x>, handed to the network in natural order
    const double* gd = H->w2;
    if (F.split) {
        relayout0<double>(H, H->w2, H->q, 0);
        gd = H->q;
    }
    if ((rc = nn_train_backward(net, gd, 2.0 / xax, lr))) return fail(rc, "network: %s", nn_error());
    return check_launch();
}

int hp_pressure_rhs(hp_handle* H, const hp_rhs_fields* f, double* rhs) {
    if (!H) return fail(HP_EINVAL, "null handle");
    g_err.clear();
    if (!f || !rhs || !f->rho_n || !f->c2_n || !f->p_n || !f->mom_n || !f->rho_np1 || !f->mom_star)
        return fail(HP_EINVAL, "null field");
    if (f->temp_n && (!f->conc_n || !f->rkc_n)) return fail(HP_EINVAL, "two components need conc_n and rkc_n");
    const LevelData& F = H->lv[0];
    // rhs may not overlap any input (the momenta span three cell arrays)
    const double* ins[] = {f->rho_n, f->c2_n, f->p_n, f->mom_n, f->rho_np1, f->mom_star, f->visc, f->temp_n,
                           f->conc_n, f->rkc_n};
    const int spans[] = {1, 1, 1, 3, 1, 3, 1, 1, 1, 1};
    for (int q = 0; q < 10; ++q)
        if (ins[q] && rhs < ins[q] + spans[q] * F.N && ins[q] < rhs + F.N)
            return fail(HP_EINVAL, "rhs must not overlap an input");
    const int bcs[3] = {H->bc.x, H->bc.y, H->bc.z};
    if (hydro_launch_rhs(F.n, bcs, F.h, H->dt, f, rhs, H->stream) != HP_OK) return check_launch();
    return check_launch();
}

int hp_pressure_update(hp_handle* H, const hp_update_fields* f) {
    if (!H) return fail(HP_EINVAL, "null handle");
    g_err.clear();
    if (!f || !f->p || !f->rho_np1 || !f->mom_star || !f->e_star || !f->mom_out || !f->uface_out || !f->e_out)
        return fail(HP_EINVAL, "null field");
    const LevelData& F = H->lv[0];
    const int64_t N = F.N;
    // inputs and outputs as byte ranges (momenta span three cell arrays): no output may overlap
    // any other array of the call
    struct R { const char* lo; const char* hi; };
    auto rng = [&](const double* q, int arrays) { return R{(const char*)q, (const char*)(q + arrays * N)}; };
    const R arr[] = {rng(f->p, 1), rng(f->rho_np1, 1), rng(f->mom_star, 3), rng(f->e_star, 1),
                     rng(f->mom_out, 3), rng(f->uface_out, 3), rng(f->e_out, 1)};
    for (int o = 4; o < 7; ++o)
        for (int q = 0; q < 7; ++q)
            if (q != o && arr[o].lo < arr[q].hi && arr[q].lo < arr[o].hi)
                return fail(HP_EINVAL, "outputs must not alias inputs or each other");
    const int bcs[3] = {H->bc.x, H->bc.y, H->bc.z};
    if (hydro_launch_update(F.n, bcs, F.h, H->dt, f, H->stream) != HP_OK) return check_launch();
    return check_launch();
}

int hp_advect(hp_handle* H, const double* rho, const double* mom, const double* e, double* rho_out,
              double* mom_out, double* e_out) {
    if (!H) return fail(HP_EINVAL, "null handle");
    g_err.clear();
    if (!rho || !mom || !e || !rho_out || !mom_out || !e_out) return fail(HP_EINVAL, "null field");
    const LevelData& F = H->lv[0];
    const int64_t N = F.N;
    struct R { const char* lo; const char* hi; };
    auto rng = [&](const double* q, int arrays) { return R{(const char*)q, (const char*)(q + arrays * N)}; };
    const R arr[] = {rng(rho, 1), rng(mom, 3), rng(e, 1), rng(rho_out, 1), rng(mom_out, 3), rng(e_out, 1)};
    for (int o = 3; o < 6; ++o)
        for (int q = 0; q < 6; ++q)
            if (q != o && arr[o].lo < arr[q].hi && arr[q].lo < arr[o].hi)
                return fail(HP_EINVAL, "outputs must not alias inputs or each other");
    const int bcs[3] = {H->bc.x, H->bc.y, H->bc.z};
    if (hydro_launch_advect(F.n, bcs, F.h, H->dt, rho, mom, e, rho_out, mom_out, e_out, H->stream) != HP_OK)
        return check_launch();
    return check_launch();
}

int hp_eos_ideal(hp_handle* H, const double* rho, const double* mom, const double* e, double gamma, double* p,
                 double* c2) {
    if (!H) return fail(HP_EINVAL, "null handle");
    g_err.clear();
    if (!rho || !mom || !e || !p) return fail(HP_EINVAL, "null field");
    if (!(gamma > 1.0) || !std::isfinite(gamma)) return fail(HP_EINVAL, "gamma must be > 1");
    if (hydro_launch_eos(H->lv[0].N, rho, mom, e, gamma, p, c2, H->stream) != HP_OK) return check_launch();
    return check_launch();
}

int hp_axpby(hp_handle* H, double a, const double* x, double b, double* y, long long n) {
    if (!H) return fail(HP_EINVAL, "null handle");
    g_err.clear();
    if (n < 0 || (n > 0 && (!x || !y))) return fail(HP_EINVAL, "null vector or negative length");
    if (n > 0) launch_axpby(a, x, b, y, (int64_t)n, H->stream);
    return check_launch();
}

int hp_stream_copy(const double* src, double* dst, long long n, void* stream) {
    g_err.clear();
    if (n < 0 || (n > 0 && (!src || !dst))) return fail(HP_EINVAL, "null pointer or negative length");
    if (((uintptr_t)src | (uintptr_t)dst) & 15) return fail(HP_EINVAL, "pointers must be 16-byte aligned");
    if (n > 0 && src < dst + n && dst < src + n) return fail(HP_EINVAL, "source and destination overlap");
    launch_stream_copy(src, dst, (int64_t)n, (hipStream_t)stream);
    return check_launch();
}

int hp_dot(hp_handle* H, const double* x, const double* y, long long n, double* out) {
    if (!H || !out || (n > 0 && (!x || !y))) return fail(HP_EINVAL, "null argument");
    if (n < 0 || reduce_blocks_vec(n) > H->partial_cap) return fail(HP_EINVAL, "bad length");
    launch_dot<double>(x, y, n, red(H, OP_STORE, S_TMP), H->stream);
    CHK(check_launch());
    CHK(read_scalars(H));
    *out = H->host_scal[S_TMP];
    return HP_OK;
}

}  // extern "C"
