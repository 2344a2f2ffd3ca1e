/*
 * FP64 CPU oracle of the SPH neighbour-interaction path.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code,
 * header, table or helper with the GPU library; the product path never
 * calls it.
 *
 * What it computes (Schaller et al., "SWIFT: Using task-based parallelism,
 * fully asynchronous communication, and graph partition-based domain
 * decomposition for strong scaling on more than 100 000 cores", PASC'16):
 *
 *   Sec. 2, eq. (rho):   rho_i = sum_{j, r_ij < h_i} m_j W(r_ij, h_i)
 *   Sec. 2, text after eqs. (dvdt)/(dudt):
 *                        P_i = (gamma-1) rho_i u_i,
 *                        Omega_i = 1 + h_i/(3 rho_i) d rho_i / d h_i
 *   Sec. 2, eq. (dvdt):  dv_i/dt = - sum_{j, r_ij < max(h_i,h_j)} m_j
 *                           [ P_i/(Omega_i rho_i^2) grad W(r_ij,h_i)
 *                           + P_j/(Omega_j rho_j^2) grad W(r_ij,h_j) ]
 *   Sec. 2, eq. (dudt):  du_i/dt = P_i/(Omega_i rho_i^2)
 *                           sum_{j, r_ij < h_i} m_j (v_i - v_j) . grad W(r_ij,h_i)
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - W is the cubic spline with compact support h (the paper allows
 *     "several forms"): W = 8/(pi h^3) w(r/h), w = 1-6q^2+6q^3 (q<=1/2),
 *     2(1-q)^3 (1/2<q<1), 0 otherwise.  The variable called H below is the
 *     paper's h (support radius).
 *   - "Neighbour number kept more or less constant" is read as the smooth
 *     constraint rho_i H_i^3 = (kernel_gamma*eta)^3 m_i, whose H-derivative
 *     is 3 H^2 rho Omega (the paper's Omega), solved per particle by a
 *     bracketed Newton iteration.
 *   - The self term (r = 0) is part of the density sum.
 *   - Distances use the minimum image in the periodic box.
 *   - The integrator is kick-drift-kick leapfrog with a predicted v, u for
 *     the force evaluation (the paper only says that integrator tasks update
 *     positions and velocities).
 *
 * Two neighbour finders, both independent of the GPU cell structure:
 *   brute force O(N^2) (tree == NULL), and a median-split k-d tree with a
 *   per-node maximum of H for the symmetric force range.
 *
 * All arithmetic is IEEE double; no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORACLE_OK 0
#define ORACLE_ERR_INVALID (-1)
#define ORACLE_ERR_NOT_CONVERGED (-3)
#define ORACLE_ERR_BOX_TOO_SMALL (-5)
#define ORACLE_ERR_ALLOC (-6)

typedef struct {
    double box[3];       /* periodic box edge lengths */
    double gamma;        /* adiabatic index (5/3) */
    double eta;          /* resolution parameter, Dehnen-Aly convention */
    double kernel_gamma; /* H / h_DA for the cubic spline: sqrt(10/3) */
    double h_tol;        /* |rho H^3 - C| <= h_tol * C */
    int max_iter;        /* Newton iterations per particle */
    int pad;
    double h_limit;      /* largest admissible H (<= 0: min(box)/3) */
} oracle_params;

/* ------------------------------------------------------------------ */
/* Kernel, Sec. 2 (W(r,h) with compact support h; cubic spline reading) */
/* ------------------------------------------------------------------ */
static const double NORM3 = 8.0 / M_PI;

static double w_q(double q)
{
    if (q < 0.0) return 0.0;
    if (q <= 0.5) return 1.0 - 6.0 * q * q + 6.0 * q * q * q;
    if (q < 1.0) { double t = 1.0 - q; return 2.0 * t * t * t; }
    return 0.0;
}

static double dw_q(double q) /* d w / d q */
{
    if (q < 0.0) return 0.0;
    if (q <= 0.5) return -12.0 * q + 18.0 * q * q;
    if (q < 1.0) { double t = 1.0 - q; return -6.0 * t * t; }
    return 0.0;
}

double oracle_W(double r, double H) { return NORM3 / (H * H * H) * w_q(r / H); }
double oracle_dWdr(double r, double H) { return NORM3 / (H * H * H * H) * dw_q(r / H); }
double oracle_dWdH(double r, double H)
{
    double q = r / H;
    return -NORM3 / (H * H * H * H) * (3.0 * w_q(q) + q * dw_q(q));
}

static double h_limit_of(const oracle_params* p)
{
    if (p->h_limit > 0) return p->h_limit;
    double b = p->box[0];
    if (p->box[1] < b) b = p->box[1];
    if (p->box[2] < b) b = p->box[2];
    return b / 3.0;
}

/* ------------------------------------------------------------------ */
/* k-d tree (median split on the longest axis)                          */
/* ------------------------------------------------------------------ */
typedef struct {
    double lo[3], hi[3];
    double hmax;
    int64_t b, e;
    int64_t left, right; /* -1 for leaves */
} kd_node;

typedef struct {
    int64_t n;
    double box[3];
    int leaf;
    int64_t* perm;      /* tree order -> original index */
    double* p;          /* positions in tree order, xyz interleaved */
    kd_node* nodes;
    int64_t n_nodes;
} kd_tree;

static int64_t kd_count_nodes(int64_t c, int leaf)
{
    if (c <= leaf) return 1;
    return 1 + kd_count_nodes(c / 2, leaf) + kd_count_nodes(c - c / 2, leaf);
}

/* partial selection so that element k of idx[b,e) is in sorted place by
 * coordinate ax (Hoare partitioning, median of three) */
static void kd_select(int64_t* idx, const double* pos, int ax, int64_t b, int64_t e, int64_t k)
{
    int64_t lo = b, hi = e - 1;
    while (hi > lo) {
        int64_t mid = lo + (hi - lo) / 2;
        double a = pos[3 * idx[lo] + ax], c = pos[3 * idx[mid] + ax], d = pos[3 * idx[hi] + ax];
        double piv = (a < c) ? ((c < d) ? c : ((a < d) ? d : a)) : ((a < d) ? a : ((c < d) ? d : c));
        int64_t i = lo, j = hi;
        while (i <= j) {
            while (pos[3 * idx[i] + ax] < piv) i++;
            while (pos[3 * idx[j] + ax] > piv) j--;
            if (i <= j) { int64_t t = idx[i]; idx[i] = idx[j]; idx[j] = t; i++; j--; }
        }
        if (k <= j) hi = j;
        else if (k >= i) lo = i;
        else return;
    }
}

static void kd_build_rec(kd_tree* t, const double* pos, int64_t node, int64_t b, int64_t e)
{
    kd_node* nd = &t->nodes[node];
    nd->b = b; nd->e = e;
    for (int a = 0; a < 3; a++) { nd->lo[a] = INFINITY; nd->hi[a] = -INFINITY; }
    for (int64_t k = b; k < e; k++)
        for (int a = 0; a < 3; a++) {
            double v = pos[3 * t->perm[k] + a];
            if (v < nd->lo[a]) nd->lo[a] = v;
            if (v > nd->hi[a]) nd->hi[a] = v;
        }
    if (e - b <= t->leaf) { nd->left = nd->right = -1; return; }
    int ax = 0;
    double ext = nd->hi[0] - nd->lo[0];
    for (int a = 1; a < 3; a++) if (nd->hi[a] - nd->lo[a] > ext) { ext = nd->hi[a] - nd->lo[a]; ax = a; }
    int64_t c = e - b, m = b + c / 2;
    kd_select(t->perm, pos, ax, b, e, m);
    int64_t l = node + 1;
    int64_t r = node + 1 + kd_count_nodes(c / 2, t->leaf);
    nd->left = l; nd->right = r;
    if (c > 200000) {
#pragma omp task
        kd_build_rec(t, pos, l, b, m);
#pragma omp task
        kd_build_rec(t, pos, r, m, e);
#pragma omp taskwait
    } else {
        kd_build_rec(t, pos, l, b, m);
        kd_build_rec(t, pos, r, m, e);
    }
}

void oracle_tree_free(void* h)
{
    kd_tree* t = (kd_tree*)h;
    if (!t) return;
    free(t->perm); free(t->p); free(t->nodes); free(t);
}

void* oracle_tree_new(int64_t n, const double* x, const double* y, const double* z,
                      const double* box, int leaf)
{
    if (n <= 0 || leaf < 1) return NULL;
    kd_tree* t = (kd_tree*)calloc(1, sizeof(kd_tree));
    double* pos = (double*)malloc(sizeof(double) * 3 * n);
    if (!t || !pos) { free(t); free(pos); return NULL; }
    t->n = n; t->leaf = leaf;
    memcpy(t->box, box, sizeof(double) * 3);
    t->perm = (int64_t*)malloc(sizeof(int64_t) * n);
    t->n_nodes = kd_count_nodes(n, leaf);
    t->nodes = (kd_node*)calloc(t->n_nodes, sizeof(kd_node));
    t->p = (double*)malloc(sizeof(double) * 3 * n);
    if (!t->perm || !t->nodes || !t->p) { free(pos); oracle_tree_free(t); return NULL; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        pos[3 * i] = x[i]; pos[3 * i + 1] = y[i]; pos[3 * i + 2] = z[i];
        t->perm[i] = i;
    }
#pragma omp parallel
#pragma omp single
    kd_build_rec(t, pos, 0, 0, n);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; k++) {
        int64_t i = t->perm[k];
        t->p[3 * k] = pos[3 * i]; t->p[3 * k + 1] = pos[3 * i + 1]; t->p[3 * k + 2] = pos[3 * i + 2];
    }
    free(pos);
    return t;
}

/* node-wise maximum of H (bottom-up; children have larger indices) */
static void kd_set_hmax(kd_tree* t, const double* H)
{
    for (int64_t k = t->n_nodes - 1; k >= 0; k--) {
        kd_node* nd = &t->nodes[k];
        if (nd->left < 0) {
            double hm = 0.0;
            for (int64_t q = nd->b; q < nd->e; q++) { double h = H[t->perm[q]]; if (h > hm) hm = h; }
            nd->hmax = hm;
        } else {
            double a = t->nodes[nd->left].hmax, b = t->nodes[nd->right].hmax;
            nd->hmax = a > b ? a : b;
        }
    }
}

static double box_dist2(const double* q, const double* lo, const double* hi)
{
    double s = 0.0;
    for (int a = 0; a < 3; a++) {
        double d = 0.0;
        if (q[a] < lo[a]) d = lo[a] - q[a];
        else if (q[a] > hi[a]) d = q[a] - hi[a];
        s += d * d;
    }
    return s;
}

/* Visitor over all j (with the periodic image giving r_ij < R_j) where
 * R_j = max(R, Hj) if use_hj, else R.  d = x_i - x_j (minimum image). */
typedef struct {
    double rho, drho;
    int64_t cnt;
    double ax, ay, az, du;
    int64_t fcnt;
    double sa, su;
} acc_t;

/* ------------------------------------------------------------------ */
/* Density at a given H for one particle (eq. (rho) and its H-derivative) */
/* ------------------------------------------------------------------ */
static void density_one_bf(const oracle_params* p, int64_t n, const double* x, const double* y,
                           const double* z, const double* m, int64_t i, double H, acc_t* a)
{
    double rho = 0.0, drho = 0.0;
    int64_t cnt = 0;
    const double H2 = H * H;
    for (int64_t j = 0; j < n; j++) {
        double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
        dx -= p->box[0] * nearbyint(dx / p->box[0]);
        dy -= p->box[1] * nearbyint(dy / p->box[1]);
        dz -= p->box[2] * nearbyint(dz / p->box[2]);
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < H2) {
            double r = sqrt(r2);
            rho += m[j] * oracle_W(r, H);
            drho += m[j] * oracle_dWdH(r, H);
            cnt++;
        }
    }
    a->rho = rho; a->drho = drho; a->cnt = cnt;
}

static void density_one_tree(const kd_tree* t, const double* m, const double* xi, double H, acc_t* a)
{
    double rho = 0.0, drho = 0.0;
    int64_t cnt = 0;
    const double H2 = H * H;
    int64_t stack[128];
    const kd_node* root = &t->nodes[0];
    for (int sx = -1; sx <= 1; sx++)
    for (int sy = -1; sy <= 1; sy++)
    for (int sz = -1; sz <= 1; sz++) {
        double q[3] = {xi[0] - sx * t->box[0], xi[1] - sy * t->box[1], xi[2] - sz * t->box[2]};
        if (box_dist2(q, root->lo, root->hi) >= H2) continue;
        int sp = 0;
        stack[sp++] = 0;
        while (sp) {
            const kd_node* nd = &t->nodes[stack[--sp]];
            if (box_dist2(q, nd->lo, nd->hi) >= H2) continue;
            if (nd->left < 0) {
                for (int64_t k = nd->b; k < nd->e; k++) {
                    double dx = q[0] - t->p[3 * k], dy = q[1] - t->p[3 * k + 1], dz = q[2] - t->p[3 * k + 2];
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 < H2) {
                        int64_t j = t->perm[k];
                        double r = sqrt(r2);
                        rho += m[j] * oracle_W(r, H);
                        drho += m[j] * oracle_dWdH(r, H);
                        cnt++;
                    }
                }
            } else {
                stack[sp++] = nd->right;
                stack[sp++] = nd->left;
            }
        }
    }
    a->rho = rho; a->drho = drho; a->cnt = cnt;
}

static void density_eval(const oracle_params* p, const kd_tree* t, int64_t n, const double* x,
                         const double* y, const double* z, const double* m, int64_t i, double H,
                         acc_t* a)
{
    if (t) {
        double xi[3] = {x[i], y[i], z[i]};
        density_one_tree(t, m, xi, H, a);
    } else {
        density_one_bf(p, n, x, y, z, m, i, H, a);
    }
}

/* Density at the given H for particles idx (all if idx == NULL). */
int oracle_density(const oracle_params* p, void* tree, int64_t n, const double* x, const double* y,
                   const double* z, const double* m, const double* H, int64_t n_idx,
                   const int64_t* idx, double* rho, double* drho, int64_t* cnt)
{
    if (!p || n <= 0) return ORACLE_ERR_INVALID;
    int64_t nn = idx ? n_idx : n;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < nn; k++) {
        int64_t i = idx ? idx[k] : k;
        acc_t a;
        density_eval(p, (const kd_tree*)tree, n, x, y, z, m, i, H[i], &a);
        rho[i] = a.rho; drho[i] = a.drho; cnt[i] = a.cnt;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* Smoothing-length solve: f(H) = rho(H) H^3 - C, C = (kernel_gamma eta)^3 m.
 * f is non-decreasing in H (each term m_j (8/pi) w(r_ij/H) grows with H),
 * f(0+) < 0, so a bracket [lo, hi] around the unique root is kept and every
 * Newton step that leaves it is replaced by bisection (or doubling while no
 * upper bound is known).  The returned rho, drho are those evaluated at the
 * returned H.  Status: 0 converged, 1 stalled at round-off, -1 failed. */
/* ------------------------------------------------------------------ */
static int solve_one(const oracle_params* p, const kd_tree* t, int64_t n, const double* x,
                     const double* y, const double* z, const double* m, int64_t i, double H0,
                     double* Hout, acc_t* aout, int* iters)
{
    const double C = pow(p->kernel_gamma * p->eta, 3.0) * m[i];
    const double hlim = h_limit_of(p);
    double lo = 0.0, hi = INFINITY, H = H0;
    if (!(H > 0.0) || !isfinite(H)) H = hlim * 0.5;
    if (H > hlim) H = hlim;
    int status = -1;
    acc_t a;
    memset(&a, 0, sizeof(a));
    int it;
    for (it = 1; it <= p->max_iter; it++) {
        density_eval(p, t, n, x, y, z, m, i, H, &a);
        double H3 = H * H * H;
        double f = a.rho * H3 - C;
        double fp = 3.0 * H * H * a.rho + H3 * a.drho;
        if (fabs(f) <= p->h_tol * C) { status = 0; break; }
        if (f < 0.0) lo = H; else hi = H;
        if (f < 0.0 && H >= hlim) { status = -2; break; }
        double Hn = H - f / fp;
        if (!(Hn > lo && Hn < hi) || !isfinite(Hn))
            Hn = isinf(hi) ? 2.0 * H : 0.5 * (lo + hi);
        if (Hn > hlim) Hn = (H < hlim) ? hlim : Hn;
        if (fabs(Hn - H) <= 4.0 * 2.220446049250313e-16 * H) { status = 1; break; }
        H = Hn;
    }
    if (it > p->max_iter) it = p->max_iter;
    *Hout = H; *aout = a; *iters = it;
    return status;
}

/* Solve H for particles idx (all if NULL).  H is in/out (initial guess in).
 * iters[i] receives the number of density evaluations; n_fail the number of
 * particles that did not converge. */
int oracle_solve_h(const oracle_params* p, void* tree, int64_t n, const double* x, const double* y,
                   const double* z, const double* m, double* H, int64_t n_idx, const int64_t* idx,
                   double* rho, double* drho, int64_t* cnt, int32_t* iters, int64_t* n_fail)
{
    if (!p || n <= 0) return ORACLE_ERR_INVALID;
    int64_t nn = idx ? n_idx : n;
    int64_t fails = 0, toolarge = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : fails, toolarge)
    for (int64_t k = 0; k < nn; k++) {
        int64_t i = idx ? idx[k] : k;
        acc_t a;
        double Hn;
        int it;
        int s = solve_one(p, (const kd_tree*)tree, n, x, y, z, m, i, H[i], &Hn, &a, &it);
        if (s < 0) fails++;
        if (s == -2) toolarge++;
        H[i] = Hn; rho[i] = a.rho; drho[i] = a.drho; cnt[i] = a.cnt;
        if (iters) iters[i] = it;
    }
    if (n_fail) *n_fail = fails;
    if (toolarge) return ORACLE_ERR_BOX_TOO_SMALL;
    return fails ? ORACLE_ERR_NOT_CONVERGED : ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* Ghost: close Omega, P and A = P/(Omega rho^2) (Sec. 2, after eq. (dudt)) */
/* ------------------------------------------------------------------ */
int oracle_ghost(const oracle_params* p, int64_t n, const double* rho, const double* drho,
                 const double* H, const double* u, double* omega, double* P, double* A, double* cs)
{
    if (!p || n < 0) return ORACLE_ERR_INVALID;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double om = 1.0 + H[i] / (3.0 * rho[i]) * drho[i];
        double pr = (p->gamma - 1.0) * rho[i] * u[i];
        omega[i] = om;
        P[i] = pr;
        A[i] = pr / (om * rho[i] * rho[i]);
        if (cs) cs[i] = sqrt(p->gamma * (p->gamma - 1.0) * u[i]);
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* Force, eqs. (dvdt) and (dudt), evaluated as a gather over the union set
 * {j : r_ij < max(H_i, H_j)}.  A_i = P_i/(Omega_i rho_i^2).            */
/* ------------------------------------------------------------------ */
static void force_pair(int64_t i, int64_t j, double dx, double dy, double dz, double r2,
                       const double* vx, const double* vy, const double* vz, const double* m,
                       const double* H, const double* A, acc_t* a)
{
    double Hi = H[i], Hj = H[j];
    a->fcnt++;
    /* the kernel gradient vanishes at r = 0: coincident particles exert no force */
    if (r2 <= 0.0) return;
    double r = sqrt(r2);
    double dWi = (r < Hi) ? oracle_dWdr(r, Hi) : 0.0;
    double dWj = (r < Hj) ? oracle_dWdr(r, Hj) : 0.0;
    double f = m[j] * (A[i] * dWi + A[j] * dWj) / r;
    a->ax -= f * dx; a->ay -= f * dy; a->az -= f * dz;
    double dvdr = (vx[i] - vx[j]) * dx + (vy[i] - vy[j]) * dy + (vz[i] - vz[j]) * dz;
    a->du += A[i] * m[j] * dWi * dvdr / r;
    /* error scales: sums of term magnitudes (no cancellation) */
    a->sa += m[j] * fabs(A[i] * dWi + A[j] * dWj);
    a->su += fabs(A[i] * m[j] * dWi * dvdr / r);
}

static void force_one_bf(const oracle_params* p, int64_t n, const double* x, const double* y,
                         const double* z, const double* vx, const double* vy, const double* vz,
                         const double* m, const double* H, const double* A, int64_t i, acc_t* a)
{
    for (int64_t j = 0; j < n; j++) {
        if (j == i) continue;
        double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
        dx -= p->box[0] * nearbyint(dx / p->box[0]);
        dy -= p->box[1] * nearbyint(dy / p->box[1]);
        dz -= p->box[2] * nearbyint(dz / p->box[2]);
        double r2 = dx * dx + dy * dy + dz * dz;
        double R = H[i] > H[j] ? H[i] : H[j];
        if (r2 < R * R) force_pair(i, j, dx, dy, dz, r2, vx, vy, vz, m, H, A, a);
    }
}

static void force_one_tree(const kd_tree* t, const double* x, const double* y, const double* z,
                           const double* vx, const double* vy, const double* vz, const double* m,
                           const double* H, const double* A, int64_t i, acc_t* a)
{
    int64_t stack[128];
    const kd_node* root = &t->nodes[0];
    const double Hi = H[i];
    for (int sx = -1; sx <= 1; sx++)
    for (int sy = -1; sy <= 1; sy++)
    for (int sz = -1; sz <= 1; sz++) {
        double q[3] = {x[i] - sx * t->box[0], y[i] - sy * t->box[1], z[i] - sz * t->box[2]};
        double Rr = Hi > root->hmax ? Hi : root->hmax;
        if (box_dist2(q, root->lo, root->hi) >= Rr * Rr) continue;
        int sp = 0;
        stack[sp++] = 0;
        while (sp) {
            const kd_node* nd = &t->nodes[stack[--sp]];
            double R = Hi > nd->hmax ? Hi : nd->hmax;
            if (box_dist2(q, nd->lo, nd->hi) >= R * R) continue;
            if (nd->left < 0) {
                for (int64_t k = nd->b; k < nd->e; k++) {
                    int64_t j = t->perm[k];
                    if (j == i) continue;
                    double dx = q[0] - t->p[3 * k], dy = q[1] - t->p[3 * k + 1], dz = q[2] - t->p[3 * k + 2];
                    double r2 = dx * dx + dy * dy + dz * dz;
                    double Rj = Hi > H[j] ? Hi : H[j];
                    if (r2 < Rj * Rj) force_pair(i, j, dx, dy, dz, r2, vx, vy, vz, m, H, A, a);
                }
            } else {
                stack[sp++] = nd->right;
                stack[sp++] = nd->left;
            }
        }
    }
}

/* Accelerations and du/dt for particles idx (all if NULL).  fcnt[i] = number
 * of j != i with r_ij < max(H_i, H_j); sa[i] = sum_j m_j |A_i dW_i + A_j dW_j|
 * and su[i] = sum_j |A_i m_j dW_i (v_i - v_j).r_ij/r| are the per-particle
 * magnitude scales used to normalise force errors (optional, may be NULL). */
int oracle_force(const oracle_params* p, void* tree, int64_t n, const double* x, const double* y,
                 const double* z, const double* vx, const double* vy, const double* vz,
                 const double* m, const double* H, const double* A, int64_t n_idx,
                 const int64_t* idx, double* ax, double* ay, double* az, double* dudt,
                 int64_t* fcnt, double* sa, double* su)
{
    if (!p || n <= 0) return ORACLE_ERR_INVALID;
    kd_tree* t = (kd_tree*)tree;
    if (t) kd_set_hmax(t, H);
    int64_t nn = idx ? n_idx : n;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < nn; k++) {
        int64_t i = idx ? idx[k] : k;
        acc_t a;
        memset(&a, 0, sizeof(a));
        if (t) force_one_tree(t, x, y, z, vx, vy, vz, m, H, A, i, &a);
        else force_one_bf(p, n, x, y, z, vx, vy, vz, m, H, A, i, &a);
        ax[i] = a.ax; ay[i] = a.ay; az[i] = a.az; dudt[i] = a.du;
        if (fcnt) fcnt[i] = a.fcnt;
        if (sa) sa[i] = a.sa;
        if (su) su[i] = a.su;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* One kick-drift-kick step (integrator tasks, Sec. 3.1).               */
/* State arrays are updated in place; ax..dudt must hold the forces of the
 * current positions on entry and hold those of the new positions on exit.
 * rho, drho, omega, P, A, cnt receive the new density-stage values.     */
/* ------------------------------------------------------------------ */
int oracle_step(const oracle_params* p, int use_tree, int64_t n, double* x, double* y, double* z,
                double* vx, double* vy, double* vz, double* u, const double* m, double* H,
                double* ax, double* ay, double* az, double* dudt, double* rho, double* drho,
                double* omega, double* P, double* A, int64_t* cnt, int64_t* fcnt, double dt)
{
    if (!p || n <= 0) return ORACLE_ERR_INVALID;
    double* vs = (double*)malloc(sizeof(double) * 4 * n);
    if (!vs) return ORACLE_ERR_ALLOC;
    double *vxs = vs, *vys = vs + n, *vzs = vs + 2 * n, *us = vs + 3 * n;
    const double hdt = 0.5 * dt;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        vx[i] += ax[i] * hdt; vy[i] += ay[i] * hdt; vz[i] += az[i] * hdt;
        u[i] += dudt[i] * hdt;
        double* c[3] = {x, y, z};
        double v[3] = {vx[i], vy[i], vz[i]};
        for (int d = 0; d < 3; d++) {
            double q = c[d][i] + v[d] * dt;
            q -= p->box[d] * floor(q / p->box[d]);
            if (q >= p->box[d]) q -= p->box[d];
            if (q < 0.0) q = 0.0;
            c[d][i] = q;
        }
        vxs[i] = vx[i] + ax[i] * hdt; vys[i] = vy[i] + ay[i] * hdt; vzs[i] = vz[i] + az[i] * hdt;
        us[i] = u[i] + dudt[i] * hdt;
    }
    void* t = use_tree ? oracle_tree_new(n, x, y, z, p->box, 16) : NULL;
    int64_t nf = 0;
    int st = oracle_solve_h(p, t, n, x, y, z, m, H, 0, NULL, rho, drho, cnt, NULL, &nf);
    if (st == ORACLE_OK) {
        oracle_ghost(p, n, rho, drho, H, us, omega, P, A, NULL);
        oracle_force(p, t, n, x, y, z, vxs, vys, vzs, m, H, A, 0, NULL, ax, ay, az, dudt, fcnt,
                     NULL, NULL);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; i++) {
            vx[i] += ax[i] * hdt; vy[i] += ay[i] * hdt; vz[i] += az[i] * hdt;
            u[i] += dudt[i] * hdt;
        }
    }
    oracle_tree_free(t);
    free(vs);
    return st;
}

/* FP64 conservation sums: mass, momentum (3), kinetic + thermal energy. */
void oracle_conserved(int64_t n, const double* m, const double* vx, const double* vy,
                      const double* vz, const double* u, double* out5)
{
    double M = 0, px = 0, py = 0, pz = 0, E = 0;
    for (int64_t i = 0; i < n; i++) {
        M += m[i];
        px += m[i] * vx[i]; py += m[i] * vy[i]; pz += m[i] * vz[i];
        E += m[i] * (0.5 * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]) + u[i]);
    }
    out5[0] = M; out5[1] = px; out5[2] = py; out5[3] = pz; out5[4] = E;
}

int oracle_num_threads(void) { return omp_get_max_threads(); }
