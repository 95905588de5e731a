/*
 * CPU oracle for the hypothesis-tested progressive kernel estimator
 * ("Hypothesis Testing for Progressive Kernel Estimation and VCM Framework", arXiv 2504.04411).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library. It shares no code with the GPU library.
 *
 * This file holds the per-pair part of one iteration: for every kernel (eye vertex) it visits
 * every light vertex (all-pairs mode) or the light vertices of the 3x3x3 neighbouring cells of a
 * plain uniform grid (grid mode), and accumulates in float64:
 *   count       number of light vertices inside the disk,
 *   S[g], Q[g]  sum and sum of squares of the test sample of group g (Sec. 3.2.1-3.2.2, Sec. 5.1
 *               step 2), 12 groups = 2 equi-areal annuli x 6 equi-angular sectors (Sec. 6.1.1);
 *               with one test per RGB channel (Sec. 5.1, chromatic light), 3 x 12 sums,
 *   flux[c]     sum of the photon flux (PPM) or of w * throughput (vertex merging).
 *
 * Per-pair decisions (inside the disk, normal consistency, group) and the per-pair test sample are
 * evaluated in float32 with an explicit operation order, because these decide integers that the
 * GPU path must reproduce exactly. Everything summed is promoted to float64.
 *
 * The statistic, the critical value and the radius/estimate update live in oracle.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NG 12

/* Orthonormal tangent frame (u, v) of unit normal n: the branchless construction of Duff et al.,
 * "Building an Orthonormal Basis, Revisited", JCGT 6(1), 2017. The paper only asks for two
 * orthogonal tangent directions at the eye vertex (Eq. map-function). */
void oracle_frame(int64_t n, const float *nx, const float *ny, const float *nz,
                  float *ux, float *uy, float *uz, float *vx, float *vy, float *vz)
{
    for (int64_t i = 0; i < n; ++i) {
        float x = nx[i], y = ny[i], z = nz[i];
        float sgn = copysignf(1.0f, z);
        float a = -1.0f / (sgn + z);
        float b = (x * y) * a;
        ux[i] = 1.0f + ((sgn * x) * x) * a;
        uy[i] = sgn * b;
        uz[i] = -(sgn * x);
        vx[i] = b;
        vy[i] = sgn + (y * y) * a;
        vz[i] = -y;
    }
}

/* Group of a point y = (yu, yv) of the disk (Sec. 3.2.1; n_a = 2, n_s = 6, Sec. 6.1.1).
 * Annulus 1 holds 2 d2 >= r2 (outer half of the area, boundary radius r / sqrt 2).
 * Sector s covers polar angles [60 s, 60 (s+1)) degrees counter-clockwise from +u; the centre is
 * in sector 0. */
int oracle_group(float yu, float yv, float d2, float r2)
{
    const float s3 = 1.7320508075688772f;
    int ann = (d2 + d2 >= r2) ? 1 : 0;
    int upper = (yv > 0.0f) || (yv == 0.0f && yu >= 0.0f);
    float a = fmaf(-s3, yu, yv);           /* sign of yv - sqrt3 yu: left of the 60 degree line */
    float b = fmaf(s3, yu, yv);            /* sign of yv + sqrt3 yu: left of the 120 degree line */
    int s;
    if (yu == 0.0f && yv == 0.0f)
        s = 0;                             /* the centre is given to sector 0 */
    else if (upper)
        s = (a < 0.0f) ? 0 : ((b > 0.0f) ? 1 : 2);
    else
        s = 3 + ((a > 0.0f) ? 0 : ((b < 0.0f) ? 1 : 2));
    return 6 * ann + s;
}

typedef struct {
    /* kernels */
    int64_t H;
    const float *kx, *ky, *kz;
    const float *knx, *kny, *knz;          /* NULL: no normal test */
    const float *ux, *uy, *uz, *vx, *vy, *vz;
    const float *r;
    const float *cbR, *cbG, *cbB;          /* vertex merging: camera throughput */
    const float *cdvcm, *cdvm;             /* vertex merging: camera partials */
    /* photons */
    int64_t J;                             /* stored light vertices */
    int64_t J_emitted;
    const float *px, *py, *pz;
    const float *pnx, *pny, *pnz;          /* NULL: no normal test */
    const float *fR, *fG, *fB;             /* flux (PPM) or throughput (merging) */
    const float *pdvcm, *pdvm;             /* vertex merging: light partials */
    int vcm;
    float cos_min;
    int rgb;                               /* 1: one test sample per RGB channel (3 x 12 groups) */
    /* outputs */
    uint32_t *count;
    double *S, *Q, *flux;
} oracle_args;

/* Per-pair work for kernel h and photon j (S, Q: the kernel's 12 or, per channel, 3 x 12 sums). */
static inline void pair(const oracle_args *A, int64_t h, int64_t j, float r2, float inv_eta, float wc,
                        uint32_t *cnt, double *S, double *Q, double *fl)
{
    float dx = A->kx[h] - A->px[j];
    float dy = A->ky[h] - A->py[j];
    float dz = A->kz[h] - A->pz[j];
    float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    if (!(d2 < r2)) return;
    if (A->knx && A->pnx) {
        float c = fmaf(A->knz[h], A->pnz[j], fmaf(A->kny[h], A->pny[j], A->knx[h] * A->pnx[j]));
        if (!(c >= A->cos_min)) return;
    }
    /* unified 2-D coordinates y = (<x - x*, u>, <x - x*, v>)  (Eq. map-function) */
    float yu = fmaf(dz, A->uz[h], fmaf(dy, A->uy[h], dx * A->ux[h]));
    float yv = fmaf(dz, A->vz[h], fmaf(dy, A->vy[h], dx * A->vx[h]));
    int g = oracle_group(yu, yv, d2, r2);
    float R = A->fR[j], G = A->fG[j], B = A->fB[j];
    float psi;
    if (!A->vcm) {
        /* luminance of the photon flux (Sec. 5.1: test on the luminance channel) */
        psi = fmaf(0.0722f, B, fmaf(0.7152f, G, 0.2126f * R));
        fl[0] += (double)R;
        fl[1] += (double)G;
        fl[2] += (double)B;
    } else {
        /* balance-heuristic merge weight (Eq. mis-weight, beta = 1) */
        const float p_dir = 0.31830988618379067f;  /* Lambertian pdf at normal incidence, 1/pi */
        float wl = fmaf(A->pdvm[j], p_dir, A->pdvcm[j] * inv_eta);
        float w = 1.0f / ((1.0f + wl) + wc);
        float y = fmaf(0.0722f, A->cbB[h] * B, fmaf(0.7152f, A->cbG[h] * G, 0.2126f * (A->cbR[h] * R)));
        psi = w * y;
        fl[0] += (double)(w * R);
        fl[1] += (double)(w * G);
        fl[2] += (double)(w * B);
    }
    *cnt += 1;
    if (A->rgb) {
        /* one test per channel (Sec. 5.1: chromatic light): the channel itself replaces the
         * luminance, weighted as the luminance would be in vertex merging */
        float pc[3];
        if (!A->vcm) {
            pc[0] = R;
            pc[1] = G;
            pc[2] = B;
        } else {
            const float p_dir = 0.31830988618379067f;
            float wl = fmaf(A->pdvm[j], p_dir, A->pdvcm[j] * inv_eta);
            float w = 1.0f / ((1.0f + wl) + wc);
            pc[0] = w * (A->cbR[h] * R);
            pc[1] = w * (A->cbG[h] * G);
            pc[2] = w * (A->cbB[h] * B);
        }
        for (int c = 0; c < 3; ++c) {
            S[c * NG + g] += (double)pc[c];
            Q[c * NG + g] += (double)pc[c] * (double)pc[c];
        }
        return;
    }
    S[g] += (double)psi;
    Q[g] += (double)psi * (double)psi;
}

static void kernel_consts(const oracle_args *A, int64_t h, float *r2, float *inv_eta, float *wc)
{
    float r = A->r[h];
    *r2 = r * r;
    *inv_eta = 0.0f;
    *wc = 0.0f;
    if (A->vcm) {
        const float pi = 3.14159265358979323846f;
        const float p_dir = 0.31830988618379067f;
        float eta = (float)A->J_emitted * (pi * *r2);      /* n_VM / n_VC * pi r^2 with n_VC = 1 */
        *inv_eta = 1.0f / eta;
        *wc = fmaf(A->cdvm[h], p_dir, A->cdvcm[h] * *inv_eta);
    }
}

static int64_t sq_width(const oracle_args *A) { return A->rgb ? 3 * NG : NG; }

static void zero_out(const oracle_args *A, int64_t h)
{
    const int64_t w = sq_width(A);
    A->count[h] = 0;
    memset(A->S + h * w, 0, (size_t)w * sizeof(double));
    memset(A->Q + h * w, 0, (size_t)w * sizeof(double));
    memset(A->flux + h * 3, 0, 3 * sizeof(double));
}

/* All-pairs gather: every kernel against every stored light vertex, in photon order. */
int oracle_gather_allpairs(const oracle_args *A, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t h = 0; h < A->H; ++h) {
        float r2, inv_eta, wc;
        kernel_consts(A, h, &r2, &inv_eta, &wc);
        zero_out(A, h);
        for (int64_t j = 0; j < A->J; ++j)
            pair(A, h, j, r2, inv_eta, wc, A->count + h, A->S + h * sq_width(A), A->Q + h * sq_width(A),
                 A->flux + h * 3);
    }
    return 0;
}

/* Grid gather: photons bucketed in a uniform grid of cell size h >= max radius (1 + 1e-6); each
 * kernel visits the 27 cells around its own, so every photon with |x - p| < r is visited. */
int oracle_gather_grid(const oracle_args *A, int nthreads)
{
    double rmax = 0.0;
    for (int64_t h = 0; h < A->H; ++h)
        if (A->r[h] > rmax) rmax = A->r[h];
    if (A->J == 0 || A->H == 0 || !(rmax > 0.0)) return oracle_gather_allpairs(A, nthreads);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const float *P[3] = {A->px, A->py, A->pz};
    for (int a = 0; a < 3; ++a)
        for (int64_t j = 0; j < A->J; ++j) {
            double v = P[a][j];
            if (v < lo[a]) lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    double cell = rmax * (1.0 + 1e-6);
    int64_t dim[3];
    for (;;) {
        int64_t tot = 1;
        for (int a = 0; a < 3; ++a) {
            dim[a] = (int64_t)floor((hi[a] - lo[a]) / cell) + 1;
            tot *= dim[a];
        }
        if (tot <= (int64_t)1 << 22) break;
        cell *= 1.5;
    }
    int64_t ncell = dim[0] * dim[1] * dim[2];
    int64_t *start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *cid = (int64_t *)malloc((size_t)A->J * sizeof(int64_t));
    int64_t *order = (int64_t *)malloc((size_t)A->J * sizeof(int64_t));
    if (!start || !cid || !order) { free(start); free(cid); free(order); return -1; }
    for (int64_t j = 0; j < A->J; ++j) {
        int64_t c[3];
        for (int a = 0; a < 3; ++a) {
            int64_t q = (int64_t)floor(((double)P[a][j] - lo[a]) / cell);
            c[a] = q < 0 ? 0 : (q >= dim[a] ? dim[a] - 1 : q);
        }
        cid[j] = (c[2] * dim[1] + c[1]) * dim[0] + c[0];
        start[cid[j] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    {
        int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
        if (!fill) { free(start); free(cid); free(order); return -1; }
        memcpy(fill, start, (size_t)ncell * sizeof(int64_t));
        for (int64_t j = 0; j < A->J; ++j) order[fill[cid[j]]++] = j;
        free(fill);
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t h = 0; h < A->H; ++h) {
        float r2, inv_eta, wc;
        kernel_consts(A, h, &r2, &inv_eta, &wc);
        zero_out(A, h);
        double K[3] = {A->kx[h], A->ky[h], A->kz[h]};
        int64_t c0[3], c1[3];
        for (int a = 0; a < 3; ++a) {
            int64_t q = (int64_t)floor((K[a] - lo[a]) / cell);
            c0[a] = q - 1 < 0 ? 0 : q - 1;
            c1[a] = q + 1 >= dim[a] ? dim[a] - 1 : q + 1;
        }
        for (int64_t cz = c0[2]; cz <= c1[2]; ++cz)
            for (int64_t cy = c0[1]; cy <= c1[1]; ++cy)
                for (int64_t cx = c0[0]; cx <= c1[0]; ++cx) {
                    int64_t c = (cz * dim[1] + cy) * dim[0] + cx;
                    for (int64_t q = start[c]; q < start[c + 1]; ++q)
                        pair(A, h, order[q], r2, inv_eta, wc, A->count + h, A->S + h * sq_width(A),
                             A->Q + h * sq_width(A), A->flux + h * 3);
                }
    }
    free(start);
    free(cid);
    free(order);
    return 0;
}

/* Features of the learned radius proposal (not part of the paper's method): for each kernel, the
 * light vertices inside the disks of radius R_s = r1 / 2^s, s = 0..3, counted in 8 equi-areal
 * rings per scale. Ring b of scale s holds b/8 <= d2 / R_s^2 < (b+1)/8, decided in float32 against
 * the thresholds R_s^2 * (k / 8), k = 1..7. Inside-disk and normal tests as in the gather.
 * counts: H x 32, row-major (scale-major within a row). All pairs, in photon order. */
int oracle_features(int64_t H, const float *kx, const float *ky, const float *kz, const float *knx,
                    const float *kny, const float *knz, int64_t J, const float *px, const float *py,
                    const float *pz, const float *pnx, const float *pny, const float *pnz, float r1,
                    float cos_min, uint32_t *counts, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t h = 0; h < H; ++h) {
        float R2[4], T[4][8];
        for (int s = 0; s < 4; ++s) {
            float R = r1 * (1.0f / (float)(1 << s));
            R2[s] = R * R;
            for (int k = 1; k < 8; ++k) T[s][k] = R2[s] * (0.125f * (float)k);
        }
        uint32_t *c = counts + h * 32;
        memset(c, 0, 32 * sizeof(uint32_t));
        for (int64_t j = 0; j < J; ++j) {
            float dx = kx[h] - px[j];
            float dy = ky[h] - py[j];
            float dz = kz[h] - pz[j];
            float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            if (!(d2 < R2[0])) continue;
            if (knx && pnx) {
                float cs = fmaf(knz[h], pnz[j], fmaf(kny[h], pny[j], knx[h] * pnx[j]));
                if (!(cs >= cos_min)) continue;
            }
            for (int s = 0; s < 4; ++s) {
                if (!(d2 < R2[s])) break;
                int b = 0;
                for (int k = 1; k < 8; ++k) b += (d2 >= T[s][k]) ? 1 : 0;
                c[s * 8 + b] += 1;
            }
        }
    }
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
