/*
 * hp_oracle.c -- FP64 CPU oracle for the generalized Poisson (Helmholtz) pressure solve.
 *
 * TEST INFRASTRUCTURE ONLY. Only tests, the smoke check and the benchmark's CPU-baseline leg
 * may load this library. The GPU library never links, calls or includes anything from here,
 * and this file includes nothing from the GPU library.
 *
 * What it computes (paper, Section 2 "A Solver for the Generalized Poisson Equation" and
 * eqs. Poiss, cpoiss, kappapoiss, vonNeumannBC):
 *
 *     c~ P - div(kappa grad P) = f,   c~ = 1/(dt^2 rho c_s^2),   kappa = 1/rho,
 *
 * multiplied through by dt^2, so that the mass term is m = 1/(rho c^2) and the right-hand side
 * is b = dt^2 f (the relative residual is unchanged by this positive scaling).
 *
 * Two densities (eqs. cpoiss and kappapoiss): the mass term takes the density of time level n,
 * m = 1/(rho^n c^2), and the face coefficient that of time level n+1, kappa = 1/rho^{n+1}. The
 * "2" entry points take both (rho_mass = rho^n, rho_face = rho^{n+1}); the one-density entry
 * points pass the same array for both.
 *
 * Discretization (cell-centred finite volumes on an equidistant rectangular grid; the paper's
 * Section 5 grid description): cell a = (i, j, k), centre ((i+1/2) hx, (j+1/2) hy, (k+1/2) hz).
 * For every pair of cells (a, b) adjacent along axis d there is a face f with
 *
 *     kappa_f = 2 / (rho_a + rho_b)        (face rule 0, the default: the face factor of the
 *                                           face-velocity update, step (viii) of the
 *                                           fractional-step algorithm)
 *     kappa_f = (1/rho_a + 1/rho_b) / 2    (face rule 1: the mean of kappa = 1/rho of the two
 *                                           cells, the other reading of eq. kappapoiss; the "3"
 *                                           entry points take the rule)
 *     w_f     = dt^2 kappa_f / h_d^2
 *
 * Interior faces join cells whose index along d differs by one. On a periodic axis with n >= 2
 * a wrap face joins cells 0 and n-1 (for n = 2 this is a second face between the same pair and
 * both count). An axis with n = 1 has no faces. A homogeneous Neumann boundary face carries zero
 * flux (eq. vonNeumannBC) and is omitted. Then
 *
 *     (A p)_a = m_a p_a + sum_{f at a} w_f (p_a - p_other(f)),
 *
 * i.e. A = diag(m) + sum_f w_f (e_a - e_b)(e_a - e_b)^T, symmetric positive definite
 * (the discrete counterpart of the Lax-Milgram conditions kappa, c~ > 0 in Section 2).
 *
 * The solve is the paper's preconditioned conjugate gradient (Section 2) with a diagonal
 * (Jacobi) preconditioner, in FP64 throughout. Dot products are deterministic: fixed chunks of
 * OR_CHUNK elements summed sequentially, chunk sums added in index order, so the result does
 * not depend on the OpenMP thread count.
 *
 * Build: gcc -O2 -fopenmp -fPIC -shared -ffp-contract=off -std=c11 -o libhporacle.so hp_oracle.c
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define OR_CHUNK 4096

typedef struct {
    int n[3];     /* cells along x, y, z */
    double h[3];  /* spacings */
    int bc[3];    /* 0 = periodic, 1 = homogeneous Neumann */
} or_grid;

typedef struct {
    int iterations;       /* CG iterations performed */
    int restarts;         /* true-residual restarts */
    int converged;        /* 1 if the true relative residual met tol */
    int stagnated;        /* 1 if stopped because the true residual no longer decreased */
    double rel_residual;  /* final true ||b - A x|| / ||b|| */
    int n_coef;           /* number of (alpha, beta) pairs written */
} or_stats;

static inline int64_t or_cell(const or_grid* g, int i, int j, int k) {
    return (int64_t)i + (int64_t)g->n[0] * ((int64_t)j + (int64_t)g->n[1] * (int64_t)k);
}

/* Neighbour index of cell (i,j,k) along axis d in direction s (+1/-1); -1 when there is no face. */
static int64_t or_neighbor(const or_grid* g, int i, int j, int k, int d, int s) {
    int c[3] = {i, j, k};
    int n = g->n[d];
    int t = c[d] + s;
    if (t < 0 || t >= n) {
        if (g->bc[d] != 0 || n < 2) return -1; /* Neumann boundary or single-cell axis */
        t = (t + n) % n;                        /* periodic wrap face */
    }
    c[d] = t;
    return or_cell(g, c[0], c[1], c[2]);
}

int or_version(void) { return 1; }

/* kappa at the face between cells of (face) densities ra and rb under face rule `rule` */
static double or_face_kappa(double ra, double rb, int rule) {
    return rule == 1 ? 0.5 * (1.0 / ra + 1.0 / rb) : 2.0 / (ra + rb);
}

/* Number of rows = cells. */
int64_t or_ncells(const or_grid* g) { return (int64_t)g->n[0] * g->n[1] * g->n[2]; }

/*
 * Assemble A in CSR form (rows sorted by column, duplicate faces summed).
 * rowptr has ncells+1 entries; colind/val must hold 7*ncells entries.
 * Returns the number of nonzeros.
 */
int64_t or_assemble3(const or_grid* g, const double* rho_mass, const double* rho_face,
                     const double* c2, double dt, int rule, int64_t* rowptr, int64_t* colind,
                     double* val) {
    int64_t N = or_ncells(g);
    /* first pass: count distinct columns per row */
    int64_t* cnt = (int64_t*)calloc((size_t)N, sizeof(int64_t));
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < N; ++a) {
        int i = (int)(a % g->n[0]);
        int j = (int)((a / g->n[0]) % g->n[1]);
        int k = (int)(a / ((int64_t)g->n[0] * g->n[1]));
        int64_t cols[7];
        int nc = 0;
        cols[nc++] = a;
        for (int d = 0; d < 3; ++d)
            for (int s = -1; s <= 1; s += 2) {
                int64_t b = or_neighbor(g, i, j, k, d, s);
                if (b < 0) continue;
                int dup = 0;
                for (int q = 0; q < nc; ++q)
                    if (cols[q] == b) dup = 1;
                if (!dup) cols[nc++] = b;
            }
        cnt[a] = nc;
    }
    rowptr[0] = 0;
    for (int64_t a = 0; a < N; ++a) rowptr[a + 1] = rowptr[a] + cnt[a];
    free(cnt);
    double dt2 = dt * dt;
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < N; ++a) {
        int i = (int)(a % g->n[0]);
        int j = (int)((a / g->n[0]) % g->n[1]);
        int k = (int)(a / ((int64_t)g->n[0] * g->n[1]));
        int64_t cols[7];
        double vals[7];
        int nc = 0;
        double m = 1.0 / (rho_mass[a] * c2[a]);
        cols[nc] = a;
        vals[nc] = m;
        nc++;
        for (int d = 0; d < 3; ++d)
            for (int s = -1; s <= 1; s += 2) {
                int64_t b = or_neighbor(g, i, j, k, d, s);
                if (b < 0) continue;
                double kappa = or_face_kappa(rho_face[a], rho_face[b], rule);
                double w = dt2 * kappa / (g->h[d] * g->h[d]);
                vals[0] += w; /* diagonal */
                int q;
                for (q = 1; q < nc; ++q)
                    if (cols[q] == b) break;
                if (q == nc) {
                    cols[nc] = b;
                    vals[nc] = 0.0;
                    nc++;
                }
                vals[q] -= w;
            }
        /* insertion sort by column */
        for (int p = 1; p < nc; ++p) {
            int64_t cc = cols[p];
            double vv = vals[p];
            int q = p - 1;
            while (q >= 0 && cols[q] > cc) {
                cols[q + 1] = cols[q];
                vals[q + 1] = vals[q];
                --q;
            }
            cols[q + 1] = cc;
            vals[q + 1] = vv;
        }
        int64_t base = rowptr[a];
        for (int p = 0; p < nc; ++p) {
            colind[base + p] = cols[p];
            val[base + p] = vals[p];
        }
    }
    return rowptr[N];
}

int64_t or_assemble2(const or_grid* g, const double* rho_mass, const double* rho_face,
                     const double* c2, double dt, int64_t* rowptr, int64_t* colind, double* val) {
    return or_assemble3(g, rho_mass, rho_face, c2, dt, 0, rowptr, colind, val);
}

int64_t or_assemble(const or_grid* g, const double* rho, const double* c2, double dt,
                    int64_t* rowptr, int64_t* colind, double* val) {
    return or_assemble3(g, rho, rho, c2, dt, 0, rowptr, colind, val);
}

/* y = A x (CSR) */
void or_spmv(int64_t N, const int64_t* rowptr, const int64_t* colind, const double* val,
             const double* x, double* y) {
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < N; ++a) {
        double s = 0.0;
        for (int64_t p = rowptr[a]; p < rowptr[a + 1]; ++p) s += val[p] * x[colind[p]];
        y[a] = s;
    }
}

/* Deterministic dot product: chunk partial sums in parallel, then summed in chunk order. */
double or_dot(int64_t N, const double* x, const double* y) {
    int64_t nch = (N + OR_CHUNK - 1) / OR_CHUNK;
    double* part = (double*)malloc((size_t)(nch > 0 ? nch : 1) * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nch; ++c) {
        int64_t lo = c * OR_CHUNK, hi = lo + OR_CHUNK < N ? lo + OR_CHUNK : N;
        double s = 0.0;
        for (int64_t a = lo; a < hi; ++a) s += x[a] * y[a];
        part[c] = s;
    }
    double s = 0.0;
    for (int64_t c = 0; c < nch; ++c) s += part[c];
    free(part);
    return s;
}

/*
 * Matrix-free residual r = b - A x straight from the face definition (no CSR), for sizes where
 * the CSR matrix does not fit. Used to certify a solution returned by another solver.
 */
void or_residual_mf3(const or_grid* g, const double* rho_mass, const double* rho_face,
                     const double* c2, double dt, int rule, const double* x, const double* b,
                     double* r) {
    int64_t N = or_ncells(g);
    double dt2 = dt * dt;
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < N; ++a) {
        int i = (int)(a % g->n[0]);
        int j = (int)((a / g->n[0]) % g->n[1]);
        int k = (int)(a / ((int64_t)g->n[0] * g->n[1]));
        double ax = x[a] / (rho_mass[a] * c2[a]);
        for (int d = 0; d < 3; ++d)
            for (int s = -1; s <= 1; s += 2) {
                int64_t nb = or_neighbor(g, i, j, k, d, s);
                if (nb < 0) continue;
                double w = dt2 * or_face_kappa(rho_face[a], rho_face[nb], rule) / (g->h[d] * g->h[d]);
                ax += w * (x[a] - x[nb]);
            }
        r[a] = b[a] - ax;
    }
}

void or_residual_mf2(const or_grid* g, const double* rho_mass, const double* rho_face,
                     const double* c2, double dt, const double* x, const double* b, double* r) {
    or_residual_mf3(g, rho_mass, rho_face, c2, dt, 0, x, b, r);
}

void or_residual_mf(const or_grid* g, const double* rho, const double* c2, double dt,
                    const double* x, const double* b, double* r) {
    or_residual_mf3(g, rho, rho, c2, dt, 0, x, b, r);
}

/*
 * Inhomogeneous Neumann data on one boundary (the stability problem of Section 2 prescribes the
 * outward normal derivative of the solution on the x boundaries). The datum is the outward normal
 * flux q = kappa dphi/dn through each boundary face (for the stability problem kappa = 1, so
 * q = dphi/dn; a perturbation of kappa leaves the prescribed flux unchanged). The operator keeps
 * no flux there, so in the dt^2-scaled equation the known flux moves to the right-hand side:
 *
 *     b_a += dt^2 q / h_d
 *
 * for every cell a next to boundary `side` (0: low, 1: high) of axis d, which must be a Neumann
 * axis. q holds one value per boundary face, indexed over the plane of the two other axes with
 * the lower-numbered axis fastest (x: j + ny k; y: i + nx k; z: i + nx j).
 */
void or_neumann_rhs(const or_grid* g, double dt, int d, int side, const double* q, double* b) {
    int e0 = d == 0 ? 1 : 0, e1 = d == 2 ? 1 : 2;  /* the two other axes, lower first */
    int n0 = g->n[e0], n1 = g->n[e1];
    double f = dt * dt / g->h[d];
    for (int v = 0; v < n1; ++v)
        for (int u = 0; u < n0; ++u) {
            int c[3];
            c[d] = side ? g->n[d] - 1 : 0;
            c[e0] = u;
            c[e1] = v;
            b[or_cell(g, c[0], c[1], c[2])] += f * q[u + (int64_t)n0 * v];
        }
}

/*
 * Jacobi-preconditioned conjugate gradient on a CSR matrix (paper, Section 2: PCG).
 *   x        in: initial guess, out: solution
 *   tol      stop when the true ||b - A x||_2 <= tol ||b||_2
 *   maxiter  iteration cap
 *   stag_window  if > 0: every stag_window iterations the true residual is recomputed; the solve
 *            stops (stagnated = 1) once the recursive residual has drifted 100x below it, or after
 *            5 restarts, i.e. when the true residual has reached the accuracy FP64 attains for
 *            this system. This lets tol be set below that level (reference solutions).
 *   alpha_out/beta_out  optional (may be NULL), capacity coef_cap: CG coefficients for a Lanczos
 *            estimate of the spectrum of D^-1 A.
 * Returns 0 on convergence or stagnation, 1 when maxiter was reached, -1 on breakdown
 * (p^T A p <= 0 or non-finite), -2 on allocation failure.
 */
int or_pcg(int64_t N, const int64_t* rowptr, const int64_t* colind, const double* val,
           const double* b, double* x, double tol, int maxiter, int stag_window,
           double* alpha_out, double* beta_out, int coef_cap, or_stats* st) {
    memset(st, 0, sizeof(*st));
    double* r = (double*)malloc((size_t)N * sizeof(double));
    double* z = (double*)malloc((size_t)N * sizeof(double));
    double* p = (double*)malloc((size_t)N * sizeof(double));
    double* q = (double*)malloc((size_t)N * sizeof(double));
    double* dinv = (double*)malloc((size_t)N * sizeof(double));
    if (!r || !z || !p || !q || !dinv) {
        free(r); free(z); free(p); free(q); free(dinv);
        return -2;
    }
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < N; ++a) {
        double d = 0.0;
        for (int64_t t = rowptr[a]; t < rowptr[a + 1]; ++t)
            if (colind[t] == a) d = val[t];
        dinv[a] = 1.0 / d;
    }
    double bnorm = sqrt(or_dot(N, b, b));
    int status = 1;
    int it = 0; /* before the first jump to done, which reads it */
    if (bnorm == 0.0) {
        memset(x, 0, (size_t)N * sizeof(double));
        st->converged = 1;
        st->rel_residual = 0.0;
        status = 0;
        goto done;
    }
    /* r = b - A x */
    or_spmv(N, rowptr, colind, val, x, q);
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < N; ++a) r[a] = b[a] - q[a];
    double rtrue = sqrt(or_dot(N, r, r)) / bnorm;
    if (rtrue <= tol) {
        st->converged = 1;
        st->rel_residual = rtrue;
        status = 0;
        goto done;
    }
    int restart = 1;
    double rz = 0.0;
    while (it < maxiter) {
        if (restart) {
#pragma omp parallel for schedule(static)
            for (int64_t a = 0; a < N; ++a) {
                z[a] = dinv[a] * r[a];
                p[a] = z[a];
            }
            rz = or_dot(N, r, z);
            restart = 0;
        }
        or_spmv(N, rowptr, colind, val, p, q);
        double pq = or_dot(N, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) {
            status = -1;
            break;
        }
        double alpha = rz / pq;
#pragma omp parallel for schedule(static)
        for (int64_t a = 0; a < N; ++a) {
            x[a] += alpha * p[a];
            r[a] -= alpha * q[a];
        }
        ++it;
        double rrec = sqrt(or_dot(N, r, r)) / bnorm;
        int check = rrec <= tol || (stag_window > 0 && it % stag_window == 0);
        if (check) {
            or_spmv(N, rowptr, colind, val, x, q);
#pragma omp parallel for schedule(static)
            for (int64_t a = 0; a < N; ++a) q[a] = b[a] - q[a];
            rtrue = sqrt(or_dot(N, q, q)) / bnorm;
            if (rtrue <= tol) {
                st->converged = 1;
                status = 0;
                break;
            }
            if (stag_window > 0 && rrec < 1e-2 * rtrue) {
                /* the recurrence has drifted far below the true residual: the true residual is
                   at the accuracy FP64 can attain for this system */
                st->stagnated = 1;
                status = 0;
                break;
            }
            if (rrec <= tol) {
                /* recursive residual drifted from the true one: restart from the true residual */
                if (stag_window > 0 && st->restarts >= 5) {
                    st->stagnated = 1;
                    status = 0;
                    break;
                }
                memcpy(r, q, (size_t)N * sizeof(double));
                restart = 1;
                st->restarts++;
                continue;
            }
        }
#pragma omp parallel for schedule(static)
        for (int64_t a = 0; a < N; ++a) z[a] = dinv[a] * r[a];
        double rz_new = or_dot(N, r, z);
        double beta = rz_new / rz;
        rz = rz_new;
        if (alpha_out && st->n_coef < coef_cap) {
            alpha_out[st->n_coef] = alpha;
            beta_out[st->n_coef] = beta;
            st->n_coef++;
        }
#pragma omp parallel for schedule(static)
        for (int64_t a = 0; a < N; ++a) p[a] = z[a] + beta * p[a];
    }
    /* final true residual */
    or_spmv(N, rowptr, colind, val, x, q);
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < N; ++a) q[a] = b[a] - q[a];
    st->rel_residual = sqrt(or_dot(N, q, q)) / bnorm;
    if (st->rel_residual <= tol) st->converged = 1;
done:
    st->iterations = it;
    free(r); free(z); free(p); free(q); free(dinv);
    return status;
}

/*
 * A fixed number of Jacobi-PCG iterations from x = 0 on the CSR matrix, with no convergence
 * test: the unit of work timed as the CPU baseline on sizes where a full solve takes hours.
 */
double or_pcg_fixed(int64_t N, const int64_t* rowptr, const int64_t* colind, const double* val,
                    const double* b, double* x, int iters) {
    or_stats st;
    /* tol = 0 never converges, no stagnation checks: exactly `iters` iterations */
    or_pcg(N, rowptr, colind, val, b, x, 0.0, iters, 0, NULL, NULL, 0, &st);
    return st.rel_residual;
}

int or_max_threads(void) { return omp_get_max_threads(); }
