/*
 * Test infrastructure: a stand-alone driver that runs every entry point of
 * the CPU oracle (ba_oracle.c) once on a scene read from a binary file, so
 * that the oracle can be built and exercised under the host's address and
 * undefined-behaviour sanitizers (gcc -fsanitize=address,undefined).  It
 * prints the values the Python side compares with the uninstrumented oracle.
 *
 * Scene file (little endian): int64 n_points, int32 n_scans, int32 n_voxels,
 * then x, y, z (n doubles each), scan, voxel (n int32 each), initial poses
 * (12 n_scans doubles).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t orc_points_to_clusters(int64_t n, const double *x, const double *y, const double *z,
                               const int32_t *scan, const int32_t *voxel, int32_t *cl_voxel, int32_t *cl_scan,
                               int64_t *cl_n, double *cl_mu, double *cl_S);
int64_t orc_points_to_raw_sums(int64_t n, const double *x, const double *y, const double *z,
                               const int32_t *scan, const int32_t *voxel, int32_t *cl_voxel, int32_t *cl_scan,
                               int64_t *cl_n, double *cl_sum, double *cl_sumsq);
void orc_center_raw_sums(int64_t C, const int64_t *cl_n, const double *cl_sum, const double *cl_sumsq,
                         double *cl_mu, double *cl_S);
void orc_eig3(const double *sym6, double *lam, double *Uout);
int orc_voxel_stats(int64_t C, const int32_t *vox, const int32_t *scan, const int64_t *n, const double *mu,
                    const double *S, int32_t V, int32_t Np, const double *poses, double *out_N, double *out_mbar,
                    double *out_A, double *out_lam, double *out_U);
double orc_cost(int64_t C, const int32_t *vox, const int32_t *scan, const int64_t *n, const double *mu,
                const double *S, int32_t V, int32_t Np, const double *poses);
double orc_majorizer(int kind, int64_t C, const int32_t *vox, const int32_t *scan, const int64_t *n,
                     const double *mu, const double *S, int32_t V, int32_t Np, const double *poses,
                     const double *poses_l);
int orc_eval(int mode, int64_t C, const int32_t *vox, const int32_t *scan, const int64_t *n, const double *mu,
             const double *S, int32_t V, int32_t Np, const double *poses, double *cost_out, double *grad,
             double *hess, int64_t *n_degenerate);
int orc_eval_abs(int mode, int64_t C, const int32_t *vox, const int32_t *scan, const int64_t *n, const double *mu,
                 const double *S, int32_t V, int32_t Np, const double *poses, double *cost_out, double *grad,
                 double *hess, double *gabs, double *habs);
int orc_solve(int mode, int32_t Np, const double *hess, const double *grad, double mu, double *dx);
void orc_apply_increment(int32_t Np, const double *poses, const double *dx, double *out);
int orc_lm(int mode, int64_t C, const int32_t *vox, const int32_t *scan, const int64_t *n, const double *mu_c,
           const double *S, int32_t V, int32_t Np, double *poses, int max_iters, double mu0, double nu0,
           double tol_g, int max_rejects, double exact_below, double *report, double *cost_final);

static void *xmalloc(size_t n) {
    void *p = malloc(n ? n : 1);
    if (!p) {
        fprintf(stderr, "allocation of %zu bytes failed\n", n);
        exit(2);
    }
    return p;
}

static int read_all(FILE *f, void *dst, size_t size, size_t count) {
    return fread(dst, size, count, f) == count;
}

int main(int argc, char **argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s scene.bin\n", argv[0]);
        return 2;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) {
        fprintf(stderr, "cannot open %s\n", argv[1]);
        return 2;
    }
    int64_t n;
    int32_t Np, V;
    if (!read_all(f, &n, sizeof n, 1) || !read_all(f, &Np, sizeof Np, 1) || !read_all(f, &V, sizeof V, 1) ||
        n < 1 || Np < 1 || V < 1) {
        fprintf(stderr, "bad header\n");
        return 2;
    }
    double *x = xmalloc(8 * (size_t)n), *y = xmalloc(8 * (size_t)n), *z = xmalloc(8 * (size_t)n);
    int32_t *scan = xmalloc(4 * (size_t)n), *vox = xmalloc(4 * (size_t)n);
    double *poses = xmalloc(8 * 12 * (size_t)Np);
    if (!read_all(f, x, 8, (size_t)n) || !read_all(f, y, 8, (size_t)n) || !read_all(f, z, 8, (size_t)n) ||
        !read_all(f, scan, 4, (size_t)n) || !read_all(f, vox, 4, (size_t)n) ||
        !read_all(f, poses, 8, 12 * (size_t)Np)) {
        fprintf(stderr, "short file\n");
        return 2;
    }
    fclose(f);

    int32_t *cv = xmalloc(4 * (size_t)n), *cs = xmalloc(4 * (size_t)n);
    int64_t *cn = xmalloc(8 * (size_t)n);
    double *mu = xmalloc(8 * 3 * (size_t)n), *S = xmalloc(8 * 6 * (size_t)n);
    int64_t C = orc_points_to_clusters(n, x, y, z, scan, vox, cv, cs, cn, mu, S);
    int32_t *rv = xmalloc(4 * (size_t)n), *rs = xmalloc(4 * (size_t)n);
    int64_t *rn = xmalloc(8 * (size_t)n);
    double *s1 = xmalloc(8 * 3 * (size_t)n), *s2 = xmalloc(8 * 6 * (size_t)n);
    int64_t C2 = orc_points_to_raw_sums(n, x, y, z, scan, vox, rv, rs, rn, s1, s2);
    double *mu2 = xmalloc(8 * 3 * (size_t)C2), *S2 = xmalloc(8 * 6 * (size_t)C2);
    orc_center_raw_sums(C2, rn, s1, s2, mu2, S2);
    printf("clusters %lld %lld\n", (long long)C, (long long)C2);

    double lam[3], U[9];
    orc_eig3(S, lam, U);
    double *oN = xmalloc(8 * (size_t)V), *omb = xmalloc(8 * 3 * (size_t)V), *oA = xmalloc(8 * 6 * (size_t)V);
    double *olam = xmalloc(8 * 3 * (size_t)V), *oU = xmalloc(8 * 9 * (size_t)V);
    int rc = orc_voxel_stats(C, cv, cs, cn, mu, S, V, Np, poses, oN, omb, oA, olam, oU);
    double c0 = orc_cost(C, cv, cs, cn, mu, S, V, Np, poses);
    double cm = orc_majorizer(0, C, cv, cs, cn, mu, S, V, Np, poses, poses);
    printf("stats %d cost %.17g majorizer %.17g\n", rc, c0, cm);

    const int64_t D = 6 * (int64_t)Np;
    double *g = xmalloc(8 * (size_t)D), *ga = xmalloc(8 * (size_t)D), *dx = xmalloc(8 * (size_t)D);
    double *H = xmalloc(8 * (size_t)(D * D)), *Ha = xmalloc(8 * (size_t)(D * D));
    double *P2 = xmalloc(8 * 12 * (size_t)Np);
    for (int mode = 0; mode < 3; mode++) {
        double c = 0.0;
        int64_t nd = 0;
        int e = orc_eval(mode, C, cv, cs, cn, mu, S, V, Np, poses, &c, g, H, &nd);
        int e2 = orc_eval_abs(mode, C, cv, cs, cn, mu, S, V, Np, poses, &c, g, H, ga, Ha);
        int info = orc_solve(mode, Np, H, g, 1e-2, dx);
        orc_apply_increment(Np, poses, dx, P2);
        printf("eval mode %d: rc %d %d cost %.17g solve info %d dx0 %.17g\n", mode, e, e2, c, info, dx[0]);
    }
    double *rep = xmalloc(8 * 8 * 12);
    for (int mode = 0; mode < 2; mode++) {
        double cf = 0.0;
        for (int64_t k = 0; k < 12 * (int64_t)Np; k++) P2[k] = poses[k];
        int it = orc_lm(mode, C, cv, cs, cn, mu, S, V, Np, P2, 12, 1e-2, 2.0, 1e-9, 10,
                        mode == 1 ? 0.1 : 0.0, rep, &cf);
        printf("lm mode %d: iters %d cost %.17g\n", mode, it, cf);
    }
    free(x); free(y); free(z); free(scan); free(vox); free(poses);
    free(cv); free(cs); free(cn); free(mu); free(S);
    free(rv); free(rs); free(rn); free(s1); free(s2); free(mu2); free(S2);
    free(oN); free(omb); free(oA); free(olam); free(oU);
    free(g); free(ga); free(dx); free(H); free(Ha); free(P2); free(rep);
    return 0;
}
