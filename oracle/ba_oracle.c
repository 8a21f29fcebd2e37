/*
 * Plain, slow, obviously-correct FP64 CPU oracle for one Levenberg-Marquardt
 * iteration of majorization-minimization LiDAR bundle adjustment
 * (Cai et al., "Accelerating Large-scale Bundle Adjustment for LiDAR Mapping
 * via Parallel Computing").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry and the
 * benchmark's CPU-baseline leg may load this code.  It shares no source with
 * the GPU library and is compiled separately by gcc without fast-math.
 *
 * What it computes (paper Sec. III, Eq. 1-3; Sec. IV-C, Alg. 2):
 *   - point clusters (N, mu, S) per (voxel, scan) from raw points  [Eq. 2]
 *   - transformed clusters under poses T_j = (R_j, t_j)              [Eq. 2]
 *   - voxel covariance A_i = P_i/N_i - v_i v_i^T / N_i^2, written with the
 *     parallel-axis theorem from centred clusters                    [Eq. 1]
 *   - cost c = sum_i lambda_min(A_i)                                 [Eq. 1]
 *   - the MM surrogate of Eq. 3 (plane form) and its gradient/Hessian in the
 *     chart  T (+) x = (Exp(phi) R, t + dt),  x = [phi; dt]
 *     (derivatives: the paper defers them to BALM3; derived here)
 *   - the coupled Hessian H_C of the first-stage majorizer u^T A(T) u
 *   - the exact Hessian H_E of Eq. 1 (diagnostic)
 *   - the damped increment solve (Alg. 2, Solver): per-pose 6x6 LDL^T of
 *     H_jj + mu Diag(H_jj) (MM), or a dense Cholesky of H + mu D (coupled)
 *   - LM control: trial point, gain ratio, Nielsen damping update.
 *
 * Readings of silent / ambiguous passages are listed in the design notes;
 * each function below names the one it uses.
 *
 * Conventions: a pose is 12 doubles [R00 R01 R02 R10 R11 R12 R20 R21 R22 t0 t1 t2];
 * a symmetric 3x3 is 6 doubles [xx xy xz yy yz zz]; an increment is
 * [phi0 phi1 phi2 dt0 dt1 dt2] per pose.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MM 0
#define ORC_COUPLED 1
#define ORC_EXACT 2

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */

static void sym_to_full(const double *s, double a[3][3]) {
    a[0][0] = s[0]; a[0][1] = s[1]; a[0][2] = s[2];
    a[1][0] = s[1]; a[1][1] = s[3]; a[1][2] = s[4];
    a[2][0] = s[2]; a[2][1] = s[4]; a[2][2] = s[5];
}

static void matmul3(const double a[3][3], const double b[3][3], double c[3][3]) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += a[i][k] * b[k][j];
            c[i][j] = s;
        }
}

static void transpose3(const double a[3][3], double b[3][3]) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) b[i][j] = a[j][i];
}

static void pose_R(const double *pose, double r[3][3]) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r[i][j] = pose[3 * i + j];
}

static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* [u]_x, the matrix with [u]_x v = u x v */
static void skew(const double *u, double k[3][3]) {
    k[0][0] = 0.0;   k[0][1] = -u[2]; k[0][2] = u[1];
    k[1][0] = u[2];  k[1][1] = 0.0;   k[1][2] = -u[0];
    k[2][0] = -u[1]; k[2][1] = u[0];  k[2][2] = 0.0;
}

/* ------------------------------------------------------------------ */
/* point clusters (Eq. 2)                                              */
/* ------------------------------------------------------------------ */

typedef struct { int32_t voxel, scan; int64_t idx; } orc_key;

static int key_cmp(const void *pa, const void *pb) {
    const orc_key *a = (const orc_key *)pa, *b = (const orc_key *)pb;
    if (a->voxel != b->voxel) return a->voxel < b->voxel ? -1 : 1;
    if (a->scan != b->scan) return a->scan < b->scan ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

/*
 * Group raw body-frame points by (voxel, scan) and return one cluster per
 * group, sorted by (voxel, scan): count N, centroid mu = (1/N) sum p and
 * centred scatter S = sum (p - mu)(p - mu)^T.  Eq. 2 defines the cluster by
 * the raw sums (sum p, sum p p^T); (N, mu, S) carries the same information
 * (sum p = N mu, sum p p^T = S + N mu mu^T) without the cancellation that
 * forming P/N - v v^T/N^2 from raw sums suffers at large coordinates.
 * Both passes accumulate in long double and round once.
 * Outputs must hold n entries (upper bound on clusters).  Returns C.
 */
int64_t orc_points_to_clusters(int64_t n, const double *x, const double *y, const double *z,
                               const int32_t *scan, const int32_t *voxel,
                               int32_t *cl_voxel, int32_t *cl_scan, int64_t *cl_n,
                               double *cl_mu, double *cl_S) {
    if (n <= 0) return 0;
    orc_key *keys = (orc_key *)malloc(sizeof(orc_key) * (size_t)n);
    if (!keys) return -1;
    for (int64_t i = 0; i < n; i++) { keys[i].voxel = voxel[i]; keys[i].scan = scan[i]; keys[i].idx = i; }
    qsort(keys, (size_t)n, sizeof(orc_key), key_cmp);
    int64_t c = 0, a = 0;
    while (a < n) {
        int64_t b = a;
        while (b < n && keys[b].voxel == keys[a].voxel && keys[b].scan == keys[a].scan) b++;
        long double sx = 0, sy = 0, sz = 0;
        for (int64_t k = a; k < b; k++) {
            int64_t i = keys[k].idx;
            sx += x[i]; sy += y[i]; sz += z[i];
        }
        long double cnt = (long double)(b - a);
        long double mx = sx / cnt, my = sy / cnt, mz = sz / cnt;
        long double sxx = 0, sxy = 0, sxz = 0, syy = 0, syz = 0, szz = 0;
        for (int64_t k = a; k < b; k++) {
            int64_t i = keys[k].idx;
            long double dx = (long double)x[i] - mx, dy = (long double)y[i] - my, dz = (long double)z[i] - mz;
            sxx += dx * dx; sxy += dx * dy; sxz += dx * dz;
            syy += dy * dy; syz += dy * dz; szz += dz * dz;
        }
        cl_voxel[c] = keys[a].voxel;
        cl_scan[c] = keys[a].scan;
        cl_n[c] = b - a;
        cl_mu[3 * c + 0] = (double)mx; cl_mu[3 * c + 1] = (double)my; cl_mu[3 * c + 2] = (double)mz;
        cl_S[6 * c + 0] = (double)sxx; cl_S[6 * c + 1] = (double)sxy; cl_S[6 * c + 2] = (double)sxz;
        cl_S[6 * c + 3] = (double)syy; cl_S[6 * c + 4] = (double)syz; cl_S[6 * c + 5] = (double)szz;
        c++;
        a = b;
    }
    free(keys);
    return c;
}

/*
 * The paper's interchange form of a cluster (Eq. 2): N, v_f = sum p,
 * P_f = sum p p^T, per (voxel, scan), sorted by (voxel, scan).  Sums in long
 * double, rounded once to double.  Returns C.
 */
int64_t orc_points_to_raw_sums(int64_t n, const double *x, const double *y, const double *z,
                               const int32_t *scan, const int32_t *voxel,
                               int32_t *cl_voxel, int32_t *cl_scan, int64_t *cl_n,
                               double *cl_sum, double *cl_sumsq) {
    if (n <= 0) return 0;
    orc_key *keys = (orc_key *)malloc(sizeof(orc_key) * (size_t)n);
    if (!keys) return -1;
    for (int64_t i = 0; i < n; i++) { keys[i].voxel = voxel[i]; keys[i].scan = scan[i]; keys[i].idx = i; }
    qsort(keys, (size_t)n, sizeof(orc_key), key_cmp);
    int64_t c = 0, a = 0;
    while (a < n) {
        int64_t b = a;
        while (b < n && keys[b].voxel == keys[a].voxel && keys[b].scan == keys[a].scan) b++;
        long double s[3] = {0, 0, 0}, q[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t k = a; k < b; k++) {
            int64_t i = keys[k].idx;
            long double px = x[i], py = y[i], pz = z[i];
            s[0] += px; s[1] += py; s[2] += pz;
            q[0] += px * px; q[1] += px * py; q[2] += px * pz;
            q[3] += py * py; q[4] += py * pz; q[5] += pz * pz;
        }
        cl_voxel[c] = keys[a].voxel;
        cl_scan[c] = keys[a].scan;
        cl_n[c] = b - a;
        for (int k = 0; k < 3; k++) cl_sum[3 * c + k] = (double)s[k];
        for (int k = 0; k < 6; k++) cl_sumsq[6 * c + k] = (double)q[k];
        c++;
        a = b;
    }
    free(keys);
    return c;
}

/*
 * Centre raw-sum clusters once: mu = v_f / N, S = P_f - v_f v_f^T / N,
 * evaluated in IEEE binary128 (software) and rounded once, so that the only
 * loss is the one already present in the double-precision raw sums.
 */
void orc_center_raw_sums(int64_t C, const int64_t *cl_n, const double *cl_sum, const double *cl_sumsq,
                         double *cl_mu, double *cl_S) {
    for (int64_t c = 0; c < C; c++) {
        __float128 nn = (__float128)cl_n[c];
        __float128 s0 = cl_sum[3 * c + 0], s1 = cl_sum[3 * c + 1], s2 = cl_sum[3 * c + 2];
        cl_mu[3 * c + 0] = (double)(s0 / nn);
        cl_mu[3 * c + 1] = (double)(s1 / nn);
        cl_mu[3 * c + 2] = (double)(s2 / nn);
        const double *q = cl_sumsq + 6 * c;
        cl_S[6 * c + 0] = (double)((__float128)q[0] - s0 * s0 / nn);
        cl_S[6 * c + 1] = (double)((__float128)q[1] - s0 * s1 / nn);
        cl_S[6 * c + 2] = (double)((__float128)q[2] - s0 * s2 / nn);
        cl_S[6 * c + 3] = (double)((__float128)q[3] - s1 * s1 / nn);
        cl_S[6 * c + 4] = (double)((__float128)q[4] - s1 * s2 / nn);
        cl_S[6 * c + 5] = (double)((__float128)q[5] - s2 * s2 / nn);
    }
}

/* ------------------------------------------------------------------ */
/* symmetric 3x3 eigen-decomposition: cyclic Jacobi (Golub & Van Loan,  */
/* Matrix Computations, Sec. 8.5)                                      */
/* ------------------------------------------------------------------ */

/* lam ascending; U columns are the matching unit eigenvectors (U[row][col]). */
void orc_eig3(const double *sym6, double *lam, double *Uout) {
    double a[3][3], v[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    sym_to_full(sym6, a);
    for (int sweep = 0; sweep < 50; sweep++) {
        double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
        if (off == 0.0) break;
        for (int p = 0; p < 2; p++)
            for (int q = p + 1; q < 3; q++) {
                double apq = a[p][q];
                if (apq == 0.0) continue;
                if (fabs(apq) < 1e-18 * (fabs(a[p][p]) + fabs(a[q][q]))) {
                    a[p][q] = a[q][p] = 0.0;
                    continue;
                }
                double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
                double t;
                if (fabs(theta) > 1e150)
                    t = 0.5 / theta;
                else
                    t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* A <- J^T A J with J the rotation in the (p, q) plane */
                for (int k = 0; k < 3; k++) {
                    double akp = a[k][p], akq = a[k][q];
                    a[k][p] = c * akp - s * akq;
                    a[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; k++) {
                    double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = c * apk - s * aqk;
                    a[q][k] = s * apk + c * aqk;
                }
                a[p][q] = a[q][p] = 0.0;
                for (int k = 0; k < 3; k++) {
                    double vkp = v[k][p], vkq = v[k][q];
                    v[k][p] = c * vkp - s * vkq;
                    v[k][q] = s * vkp + c * vkq;
                }
            }
    }
    int idx[3] = {0, 1, 2};
    double d[3] = {a[0][0], a[1][1], a[2][2]};
    for (int i = 0; i < 3; i++)
        for (int j = i + 1; j < 3; j++)
            if (d[idx[j]] < d[idx[i]]) { int t = idx[i]; idx[i] = idx[j]; idx[j] = t; }
    for (int c = 0; c < 3; c++) {
        lam[c] = d[idx[c]];
        for (int r = 0; r < 3; r++) Uout[3 * r + c] = v[r][idx[c]];
    }
}

/* ------------------------------------------------------------------ */
/* per-voxel statistics under poses (Eq. 1, Eq. 2)                     */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t C;
    const int32_t *vox, *scan;
    const int64_t *n;
    const double *mu, *S;
    int32_t V, Np;
    int64_t *vptr; /* V+1, clusters grouped by voxel via order[] */
    int64_t *order;
} orc_problem;

static int problem_init(orc_problem *p, int64_t C, const int32_t *vox, const int32_t *scan, const int64_t *n,
                        const double *mu, const double *S, int32_t V, int32_t Np) {
    p->C = C; p->vox = vox; p->scan = scan; p->n = n; p->mu = mu; p->S = S; p->V = V; p->Np = Np;
    p->vptr = (int64_t *)calloc((size_t)V + 1, sizeof(int64_t));
    p->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C > 0 ? C : 1));
    if (!p->vptr || !p->order) return -1;
    for (int64_t c = 0; c < C; c++) {
        if (vox[c] < 0 || vox[c] >= V || scan[c] < 0 || scan[c] >= Np || n[c] <= 0) return -2;
        p->vptr[vox[c] + 1]++;
    }
    for (int32_t v = 0; v < V; v++) p->vptr[v + 1] += p->vptr[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)V + 1));
    memcpy(fill, p->vptr, sizeof(int64_t) * ((size_t)V + 1));
    for (int64_t c = 0; c < C; c++) p->order[fill[vox[c]]++] = c;
    free(fill);
    return 0;
}

static void problem_free(orc_problem *p) { free(p->vptr); free(p->order); }

/* transformed cluster: ybar = R mu, m = ybar + t, St = R S R^T  (Eq. 2) */
static void transform_cluster(const double *pose, const double *mu, const double *S6, double *ybar, double *m,
                              double St[3][3]) {
    double r[3][3], s[3][3], rs[3][3], rt[3][3];
    pose_R(pose, r);
    for (int i = 0; i < 3; i++) {
        ybar[i] = r[i][0] * mu[0] + r[i][1] * mu[1] + r[i][2] * mu[2];
        m[i] = ybar[i] + pose[9 + i];
    }
    sym_to_full(S6, s);
    matmul3(r, s, rs);
    transpose3(r, rt);
    matmul3(rs, rt, St);
}

typedef struct {
    double Ni;       /* total points of the voxel */
    double mbar[3];  /* voxel centroid */
    double A[6];     /* covariance (1/N_i) sum_k (q_k - mbar)(q_k - mbar)^T */
    double lam[3];
    double U[9];     /* U[3*r + c], column c = eigenvector of lam[c] */
} orc_voxel;

/*
 * Voxel statistics at poses T (Eq. 1): N_i = sum_j N_ij,
 * mbar = sum_j N_ij m_ij / N_i and
 * A_i = (1/N_i) sum_j [ St_ij + N_ij (m_ij - mbar)(m_ij - mbar)^T ],
 * which equals P_i/N_i - v_i v_i^T/N_i^2 of Eq. 1 (parallel-axis theorem).
 */
static void voxel_stats(const orc_problem *p, const double *poses, int32_t v, orc_voxel *out) {
    double Ni = 0.0, sm[3] = {0, 0, 0};
    for (int64_t k = p->vptr[v]; k < p->vptr[v + 1]; k++) {
        int64_t c = p->order[k];
        double yb[3], m[3], St[3][3];
        transform_cluster(poses + 12 * p->scan[c], p->mu + 3 * c, p->S + 6 * c, yb, m, St);
        double nc = (double)p->n[c];
        Ni += nc;
        for (int i = 0; i < 3; i++) sm[i] += nc * m[i];
    }
    out->Ni = Ni;
    for (int i = 0; i < 3; i++) out->mbar[i] = sm[i] / Ni;
    double acc[3][3] = {{0}};
    for (int64_t k = p->vptr[v]; k < p->vptr[v + 1]; k++) {
        int64_t c = p->order[k];
        double yb[3], m[3], St[3][3];
        transform_cluster(poses + 12 * p->scan[c], p->mu + 3 * c, p->S + 6 * c, yb, m, St);
        double nc = (double)p->n[c];
        double d[3] = {m[0] - out->mbar[0], m[1] - out->mbar[1], m[2] - out->mbar[2]};
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) acc[i][j] += St[i][j] + nc * d[i] * d[j];
    }
    out->A[0] = acc[0][0] / Ni; out->A[1] = acc[0][1] / Ni; out->A[2] = acc[0][2] / Ni;
    out->A[3] = acc[1][1] / Ni; out->A[4] = acc[1][2] / Ni; out->A[5] = acc[2][2] / Ni;
    orc_eig3(out->A, out->lam, out->U);
}

/* ------------------------------------------------------------------ */
/* public: voxel statistics and cost (Eq. 1)                           */
/* ------------------------------------------------------------------ */

/* Per-voxel N_i, mbar (3), A (6), lambda (3 ascending), U (9).  Any output may
 * be NULL.  Voxels with no cluster get zeros.  Returns 0 or a negative error. */
int orc_voxel_stats(int64_t C, const int32_t *vox, const int32_t *scan, const int64_t *n, const double *mu,
                    const double *S, int32_t V, int32_t Np, const double *poses, double *out_N, double *out_mbar,
                    double *out_A, double *out_lam, double *out_U) {
    orc_problem p;
    int rc = problem_init(&p, C, vox, scan, n, mu, S, V, Np);
    if (rc) { problem_free(&p); return rc; }
    for (int32_t v = 0; v < V; v++) {
        orc_voxel vs;
        memset(&vs, 0, sizeof vs);
        if (p.vptr[v + 1] > p.vptr[v]) voxel_stats(&p, poses, v, &vs);
        if (out_N) out_N[v] = vs.Ni;
        if (out_mbar) memcpy(out_mbar + 3 * v, vs.mbar, sizeof vs.mbar);
        if (out_A) memcpy(out_A + 6 * v, vs.A, sizeof vs.A);
        if (out_lam) memcpy(out_lam + 3 * v, vs.lam, sizeof vs.lam);
        if (out_U) memcpy(out_U + 9 * v, vs.U, sizeof vs.U);
    }
    problem_free(&p);
    return 0;
}

/* c(T) = sum_i lambda_min(A_i(T)), summed serially in voxel order (Eq. 1). */
double orc_cost(int64_t C, const int32_t *vox, const int32_t *scan, const int64_t *n, const double *mu,
                const double *S, int32_t V, int32_t Np, const double *poses) {
    orc_problem p;
    if (problem_init(&p, C, vox, scan, n, mu, S, V, Np)) { problem_free(&p); return NAN; }
    double cost = 0.0;
    for (int32_t v = 0; v < V; v++) {
        if (p.vptr[v + 1] == p.vptr[v]) continue;
        orc_voxel vs;
        voxel_stats(&p, poses, v, &vs);
        cost += vs.lam[0];
    }
    problem_free(&p);
    return cost;
}

/*
 * Majorizers at poses T, built at the expansion point T_l (u and mbar frozen
 * there).
 *   kind 0: the MM surrogate of Eq. 3.  With u = u_min(T_l), mbar_l the voxel
 *           centroid at T_l and z = 1/2 sum_j u^T v_ij(T_l) = N_i u^T mbar_l / 2
 *           (reading: the sum of z runs over every scan observing the voxel),
 *           Eq. 3 equals (1/N_i) sum_k (u^T (q_k(T) - mbar_l))^2, i.e.
 *           (1/N_i) sum_j [u^T St_ij u + N_ij (u^T (m_ij - mbar_l))^2].
 *   kind 1: the first-stage majorizer u^T A_i(T) u (u frozen, centroid free).
 */
double orc_majorizer(int kind, int64_t C, const int32_t *vox, const int32_t *scan, const int64_t *n,
                     const double *mu, const double *S, int32_t V, int32_t Np, const double *poses,
                     const double *poses_l) {
    orc_problem p;
    if (problem_init(&p, C, vox, scan, n, mu, S, V, Np)) { problem_free(&p); return NAN; }
    double total = 0.0;
    for (int32_t v = 0; v < V; v++) {
        if (p.vptr[v + 1] == p.vptr[v]) continue;
        orc_voxel vl, vt;
        voxel_stats(&p, poses_l, v, &vl);
        double u[3] = {vl.U[0], vl.U[3], vl.U[6]};
        if (kind == 1) {
            voxel_stats(&p, poses, v, &vt);
            double a[3][3], au[3];
            sym_to_full(vt.A, a);
            for (int i = 0; i < 3; i++) au[i] = a[i][0] * u[0] + a[i][1] * u[1] + a[i][2] * u[2];
            total += dot3(u, au);
            continue;
        }
        double acc = 0.0;
        for (int64_t k = p.vptr[v]; k < p.vptr[v + 1]; k++) {
            int64_t c = p.order[k];
            double yb[3], m[3], St[3][3], su[3];
            transform_cluster(poses + 12 * p.scan[c], p.mu + 3 * c, p.S + 6 * c, yb, m, St);
            for (int i = 0; i < 3; i++) su[i] = St[i][0] * u[0] + St[i][1] * u[1] + St[i][2] * u[2];
            double d[3] = {m[0] - vl.mbar[0], m[1] - vl.mbar[1], m[2] - vl.mbar[2]};
            double e = dot3(u, d);
            acc += dot3(u, su) + (double)p.n[c] * e * e;
        }
        total += acc / vl.Ni;
    }
    problem_free(&p);
    return total;
}

/* ------------------------------------------------------------------ */
/* derivatives in the chart T (+) x = (Exp(phi) R, t + dt)            */
/* ------------------------------------------------------------------ */

static void add_block(double *H, int64_t ld, int64_t r0, int64_t c0, const double blk[6][6], double scale) {
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 6; j++) H[(r0 + i) * ld + (c0 + j)] += scale * blk[i][j];
}

/*
 * cost, gradient (6 Np) and Hessian at poses.
 *   mode ORC_MM:      hess is [Np][6][6], the block-diagonal Hessian of the
 *                     Eq. 3 surrogate (poses decouple: Sec. IV-C).
 *   mode ORC_COUPLED: hess is dense [6Np][6Np] row-major, the Hessian of the
 *                     first-stage majorizer u^T A(T) u (u frozen): H_MM blocks
 *                     minus 2 h_j h_k^T for every scan pair of every voxel.
 *   mode ORC_EXACT:   dense, the exact Hessian of Eq. 1:
 *                     H_C + sum_{l=1,2} 2/(lam0 - lam_l) F^l F^l^T
 *                     (terms with lam_l - lam0 <= 1e-12 lam2 are dropped).
 * The gradient is the same in every mode (the majorizers touch c at T_l).
 * Per cluster (voxel i, scan j), with u = u_min, ybar = R_j mu, m = ybar + t_j,
 * St = R_j S R_j^T, e = u^T (m - mbar), w = N_ij e ybar + St u:
 *   g_ij = (2/N_i) [ w x u ; N_ij e u ]
 *   H_ij = (2/N_i) [[ [u]x (N_ij ybar ybar^T + St) [u]x^T + (u w^T + w u^T)/2 - (u^T w) I,
 *                     N_ij (ybar x u) u^T ],
 *                   [ N_ij u (ybar x u)^T, N_ij u u^T ]]
 * Returns 0, or a negative error.  n_degenerate (may be NULL) counts voxels
 * whose EXACT term was dropped.
 */
/*
 * Evaluation at `poses` (Alg. 2 CalRes and CalJH; cost Eq. 1, gradient and
 * Hessian of the Eq. 3 surrogate or of its refinements, see the file header).
 * When gabs / habs are given (same layouts as grad / hess) they receive the
 * sums of the absolute values of every per-cluster (and, for the dense modes,
 * per-pair) contribution: the magnitude any summation order's rounding error
 * is proportional to, used by the tests as the scale of each pose block.
 */
static int eval_impl(int mode, int64_t C, const int32_t *vox, const int32_t *scan, const int64_t *n,
                     const double *mu, const double *S, int32_t V, int32_t Np, const double *poses,
                     double *cost_out, double *grad, double *hess, int64_t *n_degenerate, double *gabs,
                     double *habs) {
    orc_problem p;
    int rc = problem_init(&p, C, vox, scan, n, mu, S, V, Np);
    if (rc) { problem_free(&p); return rc; }
    int64_t D = 6 * (int64_t)Np;
    memset(grad, 0, sizeof(double) * (size_t)D);
    const size_t hsize = (mode == ORC_MM) ? 36 * (size_t)Np : (size_t)(D * D);
    memset(hess, 0, sizeof(double) * hsize);
    if (gabs) memset(gabs, 0, sizeof(double) * (size_t)D);
    if (habs) memset(habs, 0, sizeof(double) * hsize);
    double cost = 0.0;
    int64_t ndeg = 0;
    int maxm = 0;
    for (int32_t v = 0; v < V; v++) {
        int64_t mm = p.vptr[v + 1] - p.vptr[v];
        if (mm > maxm) maxm = (int)mm;
    }
    double *hv = (double *)malloc(sizeof(double) * 6 * (size_t)(maxm > 0 ? maxm : 1));
    double *f1 = (double *)malloc(sizeof(double) * 6 * (size_t)(maxm > 0 ? maxm : 1));
    double *f2 = (double *)malloc(sizeof(double) * 6 * (size_t)(maxm > 0 ? maxm : 1));
    for (int32_t v = 0; v < V; v++) {
        if (p.vptr[v + 1] == p.vptr[v]) continue;
        orc_voxel vs;
        voxel_stats(&p, poses, v, &vs);
        cost += vs.lam[0];
        double u[3] = {vs.U[0], vs.U[3], vs.U[6]};
        double u1[3] = {vs.U[1], vs.U[4], vs.U[7]};
        double u2[3] = {vs.U[2], vs.U[5], vs.U[8]};
        double w0 = 2.0 / vs.Ni;
        double ux[3][3], uxT[3][3];
        skew(u, ux);
        transpose3(ux, uxT);
        int use_l[3] = {0, 0, 0};
        if (mode == ORC_EXACT) {
            double tol = 1e-12 * fabs(vs.lam[2]);
            use_l[1] = (vs.lam[1] - vs.lam[0]) > tol;
            use_l[2] = (vs.lam[2] - vs.lam[0]) > tol;
            if (!use_l[1] || !use_l[2]) ndeg++;
        }
        int64_t k0 = p.vptr[v];
        for (int64_t k = p.vptr[v]; k < p.vptr[v + 1]; k++) {
            int64_t c = p.order[k];
            int32_t j = p.scan[c];
            double nc = (double)p.n[c];
            double yb[3], m[3], St[3][3];
            transform_cluster(poses + 12 * j, p.mu + 3 * c, p.S + 6 * c, yb, m, St);
            double d[3] = {m[0] - vs.mbar[0], m[1] - vs.mbar[1], m[2] - vs.mbar[2]};
            double e = dot3(u, d);
            double su[3], w[3];
            for (int i = 0; i < 3; i++) {
                su[i] = St[i][0] * u[0] + St[i][1] * u[1] + St[i][2] * u[2];
                w[i] = nc * e * yb[i] + su[i];
            }
            double wxu[3], a[3];
            cross3(w, u, wxu);
            cross3(yb, u, a);
            for (int i = 0; i < 3; i++) {
                grad[6 * j + i] += w0 * wxu[i];
                grad[6 * j + 3 + i] += w0 * nc * e * u[i];
            }
            if (gabs)
                for (int i = 0; i < 3; i++) {
                    gabs[6 * j + i] += fabs(w0 * wxu[i]);
                    gabs[6 * j + 3 + i] += fabs(w0 * nc * e * u[i]);
                }
            /* H_ij */
            double M[3][3], t1[3][3], t2[3][3];
            for (int r = 0; r < 3; r++)
                for (int s = 0; s < 3; s++) M[r][s] = nc * yb[r] * yb[s] + St[r][s];
            matmul3(ux, M, t1);
            matmul3(t1, uxT, t2);
            double uw = dot3(u, w);
            double blk[6][6];
            for (int r = 0; r < 3; r++)
                for (int s = 0; s < 3; s++) {
                    blk[r][s] = t2[r][s] + 0.5 * (u[r] * w[s] + w[r] * u[s]) - (r == s ? uw : 0.0);
                    blk[r][3 + s] = nc * a[r] * u[s];
                    blk[3 + r][s] = nc * u[r] * a[s];
                    blk[3 + r][3 + s] = nc * u[r] * u[s];
                }
            if (mode == ORC_MM)
                add_block(hess + 36 * (int64_t)j, 6, 0, 0, blk, w0);
            else
                add_block(hess, D, 6 * (int64_t)j, 6 * (int64_t)j, blk, w0);
            if (habs) {
                double ab[6][6];
                for (int r = 0; r < 6; r++)
                    for (int s2 = 0; s2 < 6; s2++) ab[r][s2] = fabs(w0 * blk[r][s2]);
                if (mode == ORC_MM)
                    add_block(habs + 36 * (int64_t)j, 6, 0, 0, ab, 1.0);
                else
                    add_block(habs, D, 6 * (int64_t)j, 6 * (int64_t)j, ab, 1.0);
            }
            if (mode != ORC_MM) {
                double *h = hv + 6 * (k - k0);
                for (int i = 0; i < 3; i++) { h[i] = nc / vs.Ni * a[i]; h[3 + i] = nc / vs.Ni * u[i]; }
            }
            if (mode == ORC_EXACT) {
                /* F^l = (1/N_i) [ (N e0 ybar + St u0) x u_l + (N e_l ybar + St u_l) x u0 ;
                 *                 N (e0 u_l + e_l u0) ] */
                for (int l = 1; l <= 2; l++) {
                    const double *ul = (l == 1) ? u1 : u2;
                    double *F = ((l == 1) ? f1 : f2) + 6 * (k - k0);
                    double el = dot3(ul, d);
                    double sul[3], wl[3], x1[3], x2[3];
                    for (int i = 0; i < 3; i++) {
                        sul[i] = St[i][0] * ul[0] + St[i][1] * ul[1] + St[i][2] * ul[2];
                        wl[i] = nc * el * yb[i] + sul[i];
                    }
                    cross3(w, ul, x1);
                    cross3(wl, u, x2);
                    for (int i = 0; i < 3; i++) {
                        F[i] = (x1[i] + x2[i]) / vs.Ni;
                        F[3 + i] = nc * (e * ul[i] + el * u[i]) / vs.Ni;
                    }
                }
            }
        }
        if (mode != ORC_MM) {
            int64_t mv = p.vptr[v + 1] - k0;
            for (int64_t a1 = 0; a1 < mv; a1++)
                for (int64_t b1 = 0; b1 < mv; b1++) {
                    int64_t ja = p.scan[p.order[k0 + a1]], jb = p.scan[p.order[k0 + b1]];
                    const double *ha = hv + 6 * a1, *hb = hv + 6 * b1;
                    for (int r = 0; r < 6; r++)
                        for (int s = 0; s < 6; s++) {
                            double val = -2.0 * ha[r] * hb[s];
                            if (mode == ORC_EXACT) {
                                for (int l = 1; l <= 2; l++) {
                                    if (!use_l[l]) continue;
                                    const double *Fa = ((l == 1) ? f1 : f2) + 6 * a1;
                                    const double *Fb = ((l == 1) ? f1 : f2) + 6 * b1;
                                    val += 2.0 / (vs.lam[0] - vs.lam[l]) * Fa[r] * Fb[s];
                                }
                            }
                            hess[(6 * ja + r) * D + 6 * jb + s] += val;
                            if (habs) habs[(6 * ja + r) * D + 6 * jb + s] += fabs(val);
                        }
                }
        }
    }
    free(hv); free(f1); free(f2);
    problem_free(&p);
    *cost_out = cost;
    if (n_degenerate) *n_degenerate = ndeg;
    return 0;
}

int orc_eval(int mode, int64_t C, const int32_t *vox, const int32_t *scan, const int64_t *n, const double *mu,
             const double *S, int32_t V, int32_t Np, const double *poses, double *cost_out, double *grad,
             double *hess, int64_t *n_degenerate) {
    return eval_impl(mode, C, vox, scan, n, mu, S, V, Np, poses, cost_out, grad, hess, n_degenerate, NULL, NULL);
}

int orc_eval_abs(int mode, int64_t C, const int32_t *vox, const int32_t *scan, const int64_t *n, const double *mu,
                 const double *S, int32_t V, int32_t Np, const double *poses, double *cost_out, double *grad,
                 double *hess, double *gabs, double *habs) {
    return eval_impl(mode, C, vox, scan, n, mu, S, V, Np, poses, cost_out, grad, hess, NULL, gabs, habs);
}

/* ------------------------------------------------------------------ */
/* increment solve (Alg. 2, Solver)                                    */
/* ------------------------------------------------------------------ */

/*
 * Damping matrix (reading of "mu Diag(H)"): D_kk = max(H_kk, 1e-12 max_k H_kk)
 * over the whole problem, so that poses no voxel constrains (zero rows) still
 * get a positive pivot and a zero increment.
 */
static double diag_floor(int mode, int32_t Np, const double *hess) {
    double mx = 0.0;
    int64_t D = 6 * (int64_t)Np;
    for (int64_t k = 0; k < D; k++) {
        double hk = (mode == ORC_MM) ? hess[36 * (k / 6) + 7 * (k % 6)] : hess[k * D + k];
        if (hk > mx) mx = hk;
    }
    return 1e-12 * mx;
}

/* LDL^T of a dense symmetric n x n (row-major, full), in place in L and dd.
 * Returns 0 or the 1-based index of the first non-positive pivot. */
static int ldlt_solve(int n, const double *A, const double *b, double *x) {
    double *L = (double *)calloc((size_t)n * n, sizeof(double));
    double *dd = (double *)calloc((size_t)n, sizeof(double));
    double *y = (double *)calloc((size_t)n, sizeof(double));
    int info = 0;
    for (int j = 0; j < n && !info; j++) {
        double s = A[j * n + j];
        for (int k = 0; k < j; k++) s -= L[j * n + k] * L[j * n + k] * dd[k];
        if (!(s > 0.0)) { info = j + 1; break; }
        dd[j] = s;
        L[j * n + j] = 1.0;
        for (int i = j + 1; i < n; i++) {
            double t = A[i * n + j];
            for (int k = 0; k < j; k++) t -= L[i * n + k] * L[j * n + k] * dd[k];
            L[i * n + j] = t / s;
        }
    }
    if (!info) {
        for (int i = 0; i < n; i++) {
            double t = b[i];
            for (int k = 0; k < i; k++) t -= L[i * n + k] * y[k];
            y[i] = t;
        }
        for (int i = 0; i < n; i++) y[i] /= dd[i];
        for (int i = n - 1; i >= 0; i--) {
            double t = y[i];
            for (int k = i + 1; k < n; k++) t -= L[k * n + i] * x[k];
            x[i] = t;
        }
    }
    free(L); free(dd); free(y);
    return info;
}

/* Dense Cholesky A = L L^T and solve; returns 0 or 1-based failing pivot. */
static int cholesky_solve(int64_t n, const double *A, const double *b, double *x) {
    if (n <= 0) return 0;
    double *L = (double *)calloc((size_t)(n * n), sizeof(double));
    double *y = (double *)calloc((size_t)n, sizeof(double));
    int info = 0;
    for (int64_t j = 0; j < n && !info; j++) {
        double s = A[j * n + j];
        for (int64_t k = 0; k < j; k++) s -= L[j * n + k] * L[j * n + k];
        if (!(s > 0.0)) { info = (int)(j + 1); break; }
        double ljj = sqrt(s);
        L[j * n + j] = ljj;
        for (int64_t i = j + 1; i < n; i++) {
            double t = A[i * n + j];
            for (int64_t k = 0; k < j; k++) t -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = t / ljj;
        }
    }
    if (!info) {
        for (int64_t i = 0; i < n; i++) {
            double t = b[i];
            for (int64_t k = 0; k < i; k++) t -= L[i * n + k] * y[k];
            y[i] = t / L[i * n + i];
        }
        for (int64_t i = n - 1; i >= 0; i--) {
            double t = y[i];
            for (int64_t k = i + 1; k < n; k++) t -= L[k * n + i] * x[k];
            x[i] = t / L[i * n + i];
        }
    }
    free(L); free(y);
    return info;
}

/*
 * Solve (H + mu D) dx = -g.  MM: Np independent 6x6 LDL^T (Alg. 2, Solver).
 * COUPLED/EXACT: one dense 6Np x 6Np Cholesky.  Returns 0, or the 1-based
 * index of the first failing pivot (dx then zeroed).
 */
int orc_solve(int mode, int32_t Np, const double *hess, const double *grad, double mu, double *dx) {
    double fl = diag_floor(mode, Np, hess);
    int64_t D = 6 * (int64_t)Np;
    if (mode == ORC_MM) {
        int info_all = 0;
        for (int32_t j = 0; j < Np; j++) {
            double A[36], b[6], x[6] = {0, 0, 0, 0, 0, 0};
            for (int r = 0; r < 6; r++) {
                for (int s = 0; s < 6; s++) A[6 * r + s] = hess[36 * j + 6 * r + s];
                double hk = A[7 * r];
                A[7 * r] += mu * (hk > fl ? hk : fl);
                b[r] = -grad[6 * j + r];
            }
            int info = ldlt_solve(6, A, b, x);
            if (info && !info_all) info_all = 6 * j + info;
            for (int r = 0; r < 6; r++) dx[6 * j + r] = info ? 0.0 : x[r];
        }
        if (info_all) memset(dx, 0, sizeof(double) * (size_t)D);
        return info_all;
    }
    double *A = (double *)malloc(sizeof(double) * (size_t)(D * D));
    double *b = (double *)malloc(sizeof(double) * (size_t)D);
    memcpy(A, hess, sizeof(double) * (size_t)(D * D));
    for (int64_t k = 0; k < D; k++) {
        double hk = A[k * D + k];
        A[k * D + k] += mu * (hk > fl ? hk : fl);
        b[k] = -grad[k];
    }
    int info = cholesky_solve(D, A, b, dx);
    if (info) memset(dx, 0, sizeof(double) * (size_t)D);
    free(A); free(b);
    return info;
}

/* ------------------------------------------------------------------ */
/* SE(3) update in the chart (reading of "T_i <- T_i + Delta T")       */
/* ------------------------------------------------------------------ */

/* Exp(phi) by Rodrigues' formula; second-order series below 1e-8 rad. */
void orc_so3_exp(const double *phi, double *R9) {
    double th2 = dot3(phi, phi), th = sqrt(th2), a, b;
    if (th < 1e-8) { a = 1.0 - th2 / 6.0; b = 0.5 - th2 / 24.0; }
    else { a = sin(th) / th; b = (1.0 - cos(th)) / th2; }
    double K[3][3], K2[3][3];
    skew(phi, K);
    matmul3(K, K, K2);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) R9[3 * i + j] = (i == j ? 1.0 : 0.0) + a * K[i][j] + b * K2[i][j];
}

/* T_j (+) x_j = (Exp(phi_j) R_j, t_j + dt_j) for every pose. */
void orc_apply_increment(int32_t Np, const double *poses, const double *dx, double *out) {
    for (int32_t j = 0; j < Np; j++) {
        double E[9], r[3][3], e[3][3], nr[3][3];
        orc_so3_exp(dx + 6 * j, E);
        pose_R(poses + 12 * j, r);
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < 3; k++) e[i][k] = E[3 * i + k];
        matmul3(e, r, nr);
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < 3; k++) out[12 * j + 3 * i + k] = nr[i][k];
        for (int i = 0; i < 3; i++) out[12 * j + 9 + i] = poses[12 * j + 9 + i] + dx[6 * j + 3 + i];
    }
}

/* ------------------------------------------------------------------ */
/* Levenberg-Marquardt (Fig. 1 LM box; damping rule not printed)       */
/* ------------------------------------------------------------------ */

/*
 * Reading of the unprinted LM control (PredResReduction / Adjust):
 *   q = -(g^T dx + 1/2 dx^T H dx), rho = (c - c_trial) / q;
 *   rho > 0 (and q > 0): accept, mu <- mu max(1/3, 1 - (2 rho - 1)^3), nu <- 2;
 *   otherwise (including a failed factorization): mu <- mu nu, nu <- 2 nu.
 * One iteration = one solve, accepted or not.  The loop stops after
 * max_iters iterations, or earlier when ||g||_2 < tol_g at an accepted point
 * (tol_g <= 0 disables that), or after max_rejects rejections in a row
 * (max_rejects <= 0 disables that): near the optimum the predicted reduction
 * falls below the resolution of the cost and no step can be confirmed.
 * Coupled mode with exact_below > 0: wherever the gradient norm at the
 * current poses is below exact_below, the step uses the exact Hessian of
 * Eq. 1 at those poses instead of the coupled one (a hybrid near
 * convergence, where the exact Hessian is positive semi-definite).
 * report (may be NULL) holds 8 doubles per iteration:
 *   [cost, cost_trial, rho, mu_used, accepted, gnorm, info, q]
 * Returns the number of iterations run; final cost in *cost_final.
 */
int orc_lm(int mode, int64_t C, const int32_t *vox, const int32_t *scan, const int64_t *n, const double *mu_c,
           const double *S, int32_t V, int32_t Np, double *poses, int max_iters, double mu0, double nu0,
           double tol_g, int max_rejects, double exact_below, double *report, double *cost_final) {
    int64_t D = 6 * (int64_t)Np;
    size_t hsz = (mode == ORC_MM) ? 36 * (size_t)Np : (size_t)(D * D);
    double *g = (double *)malloc(sizeof(double) * (size_t)D);
    double *H = (double *)malloc(sizeof(double) * hsz);
    double *dx = (double *)malloc(sizeof(double) * (size_t)D);
    double *trial = (double *)malloc(sizeof(double) * 12 * (size_t)Np);
    double lm_mu = mu0, nu = nu0, cost = 0.0;
    int need_eval = 1, it, rejects = 0;
    for (it = 0; it < max_iters; it++) {
        if (max_rejects > 0 && rejects >= max_rejects) break;
        double gn = 0.0;
        if (need_eval) {
            if (orc_eval(mode, C, vox, scan, n, mu_c, S, V, Np, poses, &cost, g, H, NULL)) break;
            for (int64_t k = 0; k < D; k++) gn += g[k] * g[k];
            gn = sqrt(gn);
            /* near convergence (coupled mode): the exact Hessian of Eq. 1 at
             * the same poses; its gradient is the same */
            if (mode == ORC_COUPLED && exact_below > 0.0 && gn < exact_below)
                if (orc_eval(ORC_EXACT, C, vox, scan, n, mu_c, S, V, Np, poses, &cost, g, H, NULL)) break;
            need_eval = 0;
        } else {
            for (int64_t k = 0; k < D; k++) gn += g[k] * g[k];
            gn = sqrt(gn);
        }
        if (tol_g > 0 && gn < tol_g) break;
        int info = orc_solve(mode, Np, H, g, lm_mu, dx);
        double q = 0.0, ct = cost, rho = 0.0;
        int acc = 0;
        if (!info) {
            double gdx = 0.0, dhd = 0.0;
            for (int64_t k = 0; k < D; k++) gdx += g[k] * dx[k];
            if (mode == ORC_MM) {
                for (int32_t j = 0; j < Np; j++)
                    for (int r = 0; r < 6; r++)
                        for (int s = 0; s < 6; s++) dhd += dx[6 * j + r] * H[36 * j + 6 * r + s] * dx[6 * j + s];
            } else {
                for (int64_t r = 0; r < D; r++)
                    for (int64_t s = 0; s < D; s++) dhd += dx[r] * H[r * D + s] * dx[s];
            }
            q = -(gdx + 0.5 * dhd);
            orc_apply_increment(Np, poses, dx, trial);
            ct = orc_cost(C, vox, scan, n, mu_c, S, V, Np, trial);
            rho = (q > 0.0) ? (cost - ct) / q : -1.0;
            acc = rho > 0.0;
        }
        if (report) {
            double *rp = report + 8 * it;
            rp[0] = cost; rp[1] = ct; rp[2] = rho; rp[3] = lm_mu; rp[4] = acc; rp[5] = gn; rp[6] = info; rp[7] = q;
        }
        if (acc) {
            memcpy(poses, trial, sizeof(double) * 12 * (size_t)Np);
            double f = 2.0 * rho - 1.0, fac = 1.0 - f * f * f;
            lm_mu *= (fac > 1.0 / 3.0 ? fac : 1.0 / 3.0);
            nu = 2.0;
            need_eval = 1;
            rejects = 0;
        } else {
            lm_mu *= nu;
            nu *= 2.0;
            rejects++;
        }
    }
    if (need_eval) cost = orc_cost(C, vox, scan, n, mu_c, S, V, Np, poses);
    if (cost_final) *cost_final = cost;
    free(g); free(H); free(dx); free(trial);
    return it;
}
