#define _GNU_SOURCE
/*
 * raster_oracle.c -- FP64 CPU oracle for the query-map renderer and its adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library.  It shares no code with the GPU path and
 * the product never routes through it.
 *
 * What it computes (paper Sec. III-A/III-B):
 *   - Eq. 1 / Eq. 3: each Gaussian carries position p, orientation quaternion,
 *     scale, opacity and a query vector f_i (here "queries", dimension d).
 *   - Eq. 2 / Eq. 4: the query map Q is the depth-ordered alpha blend of the
 *     queries of the Gaussians that intersect each pixel ray.  The paper defers
 *     the projection and blending details to 3D Gaussian Splatting (Kerbl et al.);
 *     the 3DGS conventions used here are the named constants below.
 *
 * Readings taken where the paper is silent (all named constants, mirrored by
 * the GPU library as a specification, not as shared code):
 *   - a Gaussian is culled when its camera-space depth z <= ORC_NEAR;
 *   - the screen covariance gets ORC_DILATION added on its diagonal;
 *   - x/z and y/z entering the projection Jacobian are clamped to
 *     +-ORC_FOV_CLAMP * tan(fov/2), tan(fovx/2) = width / (2 fx);
 *   - radius r = ceil(3 sqrt(lambda_max)), lambda_max floored through
 *     max(ORC_EIG_FLOOR, mid^2 - det);
 *   - a Gaussian intersects pixel (px, py) iff |px - u| <= r and |py - v| <= r,
 *     i.e. px in [ceil(u - r), floor(u + r)] (the footprint); pixels sit at
 *     integer coordinates;
 *   - alpha = min(ORC_ALPHA_MAX, o * exp(power)); pairs with alpha < ORC_ALPHA_MIN
 *     are skipped; blending stops before a Gaussian that would bring the
 *     transmittance below ORC_T_STOP;
 *   - "sorted by increasing depth" (Eq. 2) orders by the float32 value of the
 *     camera-space z of the Gaussian centre, ties by record index.
 *
 * Everything that decides an integer (culling, radius, footprint, depth key) is
 * taken in float32 (decide_f32): the projection that decides them is float32
 * and, where floating point decides an integer, the oracle takes the decision
 * in that same precision, with every operation written out in a fixed order
 * and rounded on its own (no contraction; correctly rounded division, square
 * root and fused multiply-add; exp by the Cody-Waite reduction and Taylor
 * polynomial of exp_cw).  The continuous values the blend and the adjoint use
 * (screen mean, conic, opacity, Jacobian) stay FP64 (project_f64), which also
 * takes the same decisions in FP64 so that tests can compare the two.
 *
 * Records: r = cam * N + i (camera-major).  Pixels: views concatenated in
 * camera order, row-major inside a view.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_NEAR 0.2
#define ORC_DILATION 0.3
#define ORC_FOV_CLAMP 1.3
#define ORC_EIG_FLOOR 0.1
#define ORC_SIGMA 3.0
#define ORC_ALPHA_MAX 0.99
#define ORC_ALPHA_MIN (1.0 / 255.0)
#define ORC_T_STOP 1e-4

#define CAM_FLOATS 22

typedef struct {
    int w, h;
    double fx, fy, cx, cy;
    double vm[16];
} cam_t;

typedef struct {
    int vis;
    double x, y, z;          /* camera-space centre */
    double s[3];             /* scales */
    double qraw[4];          /* input quaternion (w, x, y, z) */
    double qn[4];            /* normalised quaternion */
    double qnorm;
    double R[3][3];          /* rotation of the Gaussian */
    double S3[3][3];         /* world covariance */
    double Sc[3][3];         /* camera covariance */
    double limx, limy, rx, ry;  /* x/z, y/z before clamping, and clamp limits */
    int clx, cly;            /* clamp active */
    double J[2][3];
    double a, b, c;          /* screen covariance incl. dilation: [[a, b], [b, c]] */
    double det;
    double A, B, C;          /* conic = inverse of the screen covariance */
    double u, v, o, radius;
    int px0, px1, py0, py1;  /* footprint, inclusive, clipped to the image */
    uint32_t depth_key;      /* bit pattern of the float32 z */
    int ok;                  /* the FP64 values are defined (z > 0, |q| > 0, det > 0) */
    /* the same decisions taken in FP64, and how far they are from flipping:
     * margin = min(distance of u - r, u + r, v - r, v + r, 3 sqrt(lambda_max)
     * from the nearest integer in pixels, z - near) */
    int vis64, r64x0, r64x1, r64y0, r64y1;
    double radius64, margin64;
    uint32_t key64;
} proj_t;

/* Integer decisions of one record, taken in float32. */
typedef struct {
    int vis;
    float radius, u, v, z;
    int px0, px1, py0, py1;
    uint32_t key;
} dec32_t;

static void load_cam(const float* row, cam_t* c)
{
    c->w = (int)row[0];
    c->h = (int)row[1];
    c->fx = row[2];
    c->fy = row[3];
    c->cx = row[4];
    c->cy = row[5];
    for (int k = 0; k < 16; ++k) c->vm[k] = row[6 + k];
}

/* Rotation matrix of a unit quaternion (w, x, y, z), standard formula. */
static void quat_to_rot(const double q[4], double R[3][3])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1.0 - 2.0 * (y * y + z * z);
    R[0][1] = 2.0 * (x * y - w * z);
    R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z);
    R[1][1] = 1.0 - 2.0 * (x * x + z * z);
    R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y);
    R[2][1] = 2.0 * (y * z + w * x);
    R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

static uint32_t f32_bits(double z)
{
    float f = (float)z;
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

/* exp(x) in float32: k = rint(x log2 e), r = (x - k ln2_hi) - k ln2_lo (ln2_hi
 * with 15 significant bits, so k ln2_hi is exact), the degree-7 Taylor
 * polynomial of exp(r) by Horner with fused multiply-adds, times 2^k (the
 * Cody-Waite reduction).  Each step is one correctly rounded float32
 * operation, so the value is a fixed function of x. */
static float exp_cw(float x)
{
    x = fminf(fmaxf(x, -87.0f), 88.0f);
    const float k = rintf(x * 1.44269504f);
    const float r = (x - k * 0.693145751953125f) - k * 1.42860677e-06f;
    float p = 1.0f / 5040.0f;
    p = fmaf(p, r, 1.0f / 720.0f);
    p = fmaf(p, r, 1.0f / 120.0f);
    p = fmaf(p, r, 1.0f / 24.0f);
    p = fmaf(p, r, 1.0f / 6.0f);
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    return ldexpf(p, (int)k);
}

static uint32_t f32_bits_f(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

/* The integer decisions of one record from its float32 inputs, in float32:
 * view transform, scales, normalised quaternion, world and camera covariance,
 * clamped Jacobian, screen covariance with dilation, radius from the larger
 * eigenvalue, screen mean, culling and the inclusive pixel footprint, with
 * every sum taken left to right and every product as written. */
static void decide_f32(const float* mean, const float* ls, const float* quat, const cam_t* cam, dec32_t* D)
{
    memset(D, 0, sizeof *D);
    float W[3][3], t[3];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) W[i][j] = (float)cam->vm[4 * i + j];
        t[i] = (float)cam->vm[4 * i + 3];
    }
    const float mx = mean[0], my = mean[1], mz = mean[2];
    const float x = ((W[0][0] * mx + W[0][1] * my) + W[0][2] * mz) + t[0];
    const float y = ((W[1][0] * mx + W[1][1] * my) + W[1][2] * mz) + t[1];
    const float z = ((W[2][0] * mx + W[2][1] * my) + W[2][2] * mz) + t[2];
    D->z = z;
    if (!(z > 0.2f)) return;
    float s[3];
    for (int k = 0; k < 3; ++k) s[k] = exp_cw(ls[k]);
    const float q0 = quat[0], q1 = quat[1], q2 = quat[2], q3 = quat[3];
    const float nrm = sqrtf(((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3);
    if (!(nrm > 0.0f)) return;
    const float w = q0 / nrm, qx = q1 / nrm, qy = q2 / nrm, qz = q3 / nrm;
    const float R[3][3] = {
        {1.0f - 2.0f * (qy * qy + qz * qz), 2.0f * (qx * qy - w * qz), 2.0f * (qx * qz + w * qy)},
        {2.0f * (qx * qy + w * qz), 1.0f - 2.0f * (qx * qx + qz * qz), 2.0f * (qy * qz - w * qx)},
        {2.0f * (qx * qz - w * qy), 2.0f * (qy * qz + w * qx), 1.0f - 2.0f * (qx * qx + qy * qy)}};
    float S3[3][3], Sc[3][3];
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            float acc = 0.0f;
            for (int k = 0; k < 3; ++k) acc = acc + ((R[p][k] * s[k]) * s[k]) * R[q][k];
            S3[p][q] = acc;
        }
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            float acc = 0.0f;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc = acc + (W[p][k] * S3[k][l]) * W[q][l];
            Sc[p][q] = acc;
        }
    const float fx = (float)cam->fx, fy = (float)cam->fy;
    const float limx = 1.3f * ((float)cam->w / (2.0f * fx));
    const float limy = 1.3f * ((float)cam->h / (2.0f * fy));
    float tx = x / z, ty = y / z;
    tx = tx < -limx ? -limx : (tx > limx ? limx : tx);
    ty = ty < -limy ? -limy : (ty > limy ? limy : ty);
    const float J[2][3] = {{fx / z, 0.0f, (-fx * tx) / z}, {0.0f, fy / z, (-fy * ty) / z}};
    float cov[2][2];
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q) {
            float acc = 0.0f;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc = acc + (J[p][k] * Sc[k][l]) * J[q][l];
            cov[p][q] = acc;
        }
    const float a = cov[0][0] + 0.3f, b = cov[0][1], c = cov[1][1] + 0.3f;
    const float det = a * c - b * b;
    if (!(det > 0.0f)) return;
    const float mid = 0.5f * (a + c);
    const float lam = mid + sqrtf(fmaxf(0.1f, mid * mid - det));
    const float r = ceilf(3.0f * sqrtf(lam));
    const float u = (fx * x) / z + (float)cam->cx;
    const float v = (fy * y) / z + (float)cam->cy;
    D->radius = r;
    D->u = u;
    D->v = v;
    if (!(u + r >= 0.0f) || !(u - r <= (float)(cam->w - 1)) || !(v + r >= 0.0f) || !(v - r <= (float)(cam->h - 1)))
        return;
    const float fx0 = ceilf(u - r), fx1 = floorf(u + r);
    const float fy0 = ceilf(v - r), fy1 = floorf(v + r);
    D->px0 = fx0 < 0.0f ? 0 : (int)fx0;
    D->px1 = fx1 > (float)(cam->w - 1) ? cam->w - 1 : (int)fx1;
    D->py0 = fy0 < 0.0f ? 0 : (int)fy0;
    D->py1 = fy1 > (float)(cam->h - 1) ? cam->h - 1 : (int)fy1;
    if (D->px0 > D->px1 || D->py0 > D->py1) return;
    D->key = f32_bits_f(z);
    D->vis = 1;
}

static double frac_dist(double x) { return fabs(x - nearbyint(x)); }

/* FP64 values of one record (screen mean, conic, opacity and the intermediate
 * quantities of the adjoint) wherever they are defined, and the same integer
 * decisions taken in FP64 with their margin. */
static void project_f64(const float* mean, const float* ls, const float* quat, float logit,
                        const cam_t* cam, proj_t* P)
{
    memset(P, 0, sizeof *P);
    P->margin64 = INFINITY;
    const double* V = cam->vm;
    double mx = mean[0], my = mean[1], mz = mean[2];
    P->x = ((V[0] * mx + V[1] * my) + V[2] * mz) + V[3];
    P->y = ((V[4] * mx + V[5] * my) + V[6] * mz) + V[7];
    P->z = ((V[8] * mx + V[9] * my) + V[10] * mz) + V[11];
    P->margin64 = fabs(P->z - ORC_NEAR);
    if (!(P->z > 0.0)) return;

    for (int k = 0; k < 3; ++k) P->s[k] = exp((double)ls[k]);
    for (int k = 0; k < 4; ++k) P->qraw[k] = quat[k];
    double nrm = sqrt(P->qraw[0] * P->qraw[0] + P->qraw[1] * P->qraw[1] +
                      P->qraw[2] * P->qraw[2] + P->qraw[3] * P->qraw[3]);
    if (!(nrm > 0.0)) return;
    P->qnorm = nrm;
    for (int k = 0; k < 4; ++k) P->qn[k] = P->qraw[k] / nrm;
    quat_to_rot(P->qn, P->R);

    /* world covariance: R diag(s^2) R^T */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += P->R[i][k] * P->s[k] * P->s[k] * P->R[j][k];
            P->S3[i][j] = acc;
        }
    /* camera covariance: W S3 W^T with W the rotation block of the view matrix */
    double W[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) W[i][j] = V[4 * i + j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc += W[i][k] * P->S3[k][l] * W[j][l];
            P->Sc[i][j] = acc;
        }
    /* projection Jacobian with clamped x/z, y/z */
    P->limx = ORC_FOV_CLAMP * (cam->w / (2.0 * cam->fx));
    P->limy = ORC_FOV_CLAMP * (cam->h / (2.0 * cam->fy));
    P->rx = P->x / P->z;
    P->ry = P->y / P->z;
    double txc = P->rx, tyc = P->ry;
    if (txc < -P->limx) { txc = -P->limx; P->clx = 1; }
    if (txc > P->limx) { txc = P->limx; P->clx = 1; }
    if (tyc < -P->limy) { tyc = -P->limy; P->cly = 1; }
    if (tyc > P->limy) { tyc = P->limy; P->cly = 1; }
    P->J[0][0] = cam->fx / P->z;
    P->J[0][1] = 0.0;
    P->J[0][2] = -cam->fx * txc / P->z;
    P->J[1][0] = 0.0;
    P->J[1][1] = cam->fy / P->z;
    P->J[1][2] = -cam->fy * tyc / P->z;
    double cov[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc += P->J[i][k] * P->Sc[k][l] * P->J[j][l];
            cov[i][j] = acc;
        }
    P->a = cov[0][0] + ORC_DILATION;
    P->b = cov[0][1];
    P->c = cov[1][1] + ORC_DILATION;
    P->det = P->a * P->c - P->b * P->b;
    if (!(P->det > 0.0)) return;
    P->A = P->c / P->det;
    P->B = -P->b / P->det;
    P->C = P->a / P->det;
    P->u = (cam->fx * P->x) / P->z + cam->cx;
    P->v = (cam->fy * P->y) / P->z + cam->cy;
    P->o = 1.0 / (1.0 + exp(-(double)logit));
    P->ok = 1;

    /* the integer decisions in FP64 */
    double mid = 0.5 * (P->a + P->c);
    double lam = mid + sqrt(fmax(ORC_EIG_FLOOR, mid * mid - P->det));
    double r3 = ORC_SIGMA * sqrt(lam);
    double r = ceil(r3);
    P->radius64 = r;
    double m = fmin(P->margin64, frac_dist(r3));
    m = fmin(m, fmin(frac_dist(P->u - r), frac_dist(P->u + r)));
    m = fmin(m, fmin(frac_dist(P->v - r), frac_dist(P->v + r)));
    P->margin64 = m;
    if (!(P->z > ORC_NEAR)) return;
    if (!(P->u + r >= 0.0) || !(P->u - r <= cam->w - 1) || !(P->v + r >= 0.0) ||
        !(P->v - r <= cam->h - 1))
        return;
    double fx0 = ceil(P->u - r), fx1 = floor(P->u + r);
    double fy0 = ceil(P->v - r), fy1 = floor(P->v + r);
    P->r64x0 = fx0 < 0.0 ? 0 : (int)fx0;
    P->r64x1 = fx1 > cam->w - 1 ? cam->w - 1 : (int)fx1;
    P->r64y0 = fy0 < 0.0 ? 0 : (int)fy0;
    P->r64y1 = fy1 > cam->h - 1 ? cam->h - 1 : (int)fy1;
    if (P->r64x0 > P->r64x1 || P->r64y0 > P->r64y1) return;
    P->key64 = f32_bits(P->z);
    P->vis64 = 1;
}

/* One record: FP64 values, float32 decisions. */
static void project_one(const float* mean, const float* ls, const float* quat, float logit,
                        const cam_t* cam, proj_t* P)
{
    project_f64(mean, ls, quat, logit, cam, P);
    dec32_t D;
    decide_f32(mean, ls, quat, cam, &D);
    P->radius = D.radius;
    /* the FP64 values exist wherever the float32 decision keeps a record: z >
     * 0.2 in float32 means z > 0 in FP64, and the dilated screen covariance is
     * positive definite */
    if (!D.vis || !P->ok) {
        P->vis = 0;
        return;
    }
    P->vis = 1;
    P->px0 = D.px0;
    P->px1 = D.px1;
    P->py0 = D.py0;
    P->py1 = D.py1;
    P->depth_key = D.key;
}

typedef struct {
    int n, n_cams, d;
    cam_t* cams;
    proj_t* proj;            /* [n_cams * n] */
    int64_t* pix_off;        /* [n_cams + 1] */
    int64_t* tile_off;       /* [n_cams + 1] */
    int* tiles_x;            /* [n_cams] */
    int tw, th;
} scene_t;

static void scene_project(scene_t* S, int n, const float* means, const float* log_scales,
                          const float* quats, const float* logits, int n_cams, const float* cams,
                          int tw, int th)
{
    S->n = n;
    S->n_cams = n_cams;
    S->tw = tw;
    S->th = th;
    S->cams = (cam_t*)calloc((size_t)n_cams, sizeof(cam_t));
    S->pix_off = (int64_t*)calloc((size_t)n_cams + 1, sizeof(int64_t));
    S->tile_off = (int64_t*)calloc((size_t)n_cams + 1, sizeof(int64_t));
    S->tiles_x = (int*)calloc((size_t)n_cams, sizeof(int));
    for (int c = 0; c < n_cams; ++c) {
        load_cam(cams + (size_t)c * CAM_FLOATS, &S->cams[c]);
        int tx = tw > 0 ? (S->cams[c].w + tw - 1) / tw : 0;
        int ty = th > 0 ? (S->cams[c].h + th - 1) / th : 0;
        S->tiles_x[c] = tx;
        S->pix_off[c + 1] = S->pix_off[c] + (int64_t)S->cams[c].w * S->cams[c].h;
        S->tile_off[c + 1] = S->tile_off[c] + (int64_t)tx * ty;
    }
    int64_t R = (int64_t)n_cams * n;
    S->proj = (proj_t*)malloc((size_t)(R > 0 ? R : 1) * sizeof(proj_t));
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < R; ++r) {
        int c = (int)(r / n);
        int64_t i = r % n;
        project_one(means + 3 * i, log_scales + 3 * i, quats + 4 * i, logits[i], &S->cams[c],
                    &S->proj[r]);
    }
}

static void scene_free(scene_t* S)
{
    free(S->cams);
    free(S->proj);
    free(S->pix_off);
    free(S->tile_off);
    free(S->tiles_x);
}

/* ---------------------------------------------------------------- binning */

typedef struct {
    uint32_t tile, depth, rec;
} inst_t;

static int inst_cmp(const void* pa, const void* pb)
{
    const inst_t* a = (const inst_t*)pa;
    const inst_t* b = (const inst_t*)pb;
    if (a->tile != b->tile) return a->tile < b->tile ? -1 : 1;
    if (a->depth != b->depth) return a->depth < b->depth ? -1 : 1;
    if (a->rec != b->rec) return a->rec < b->rec ? -1 : 1;
    return 0;
}

typedef struct {
    int64_t count;
    inst_t* inst;
    uint32_t* ranges; /* [tiles, 2] */
} bins_t;

/* One instance per (record, tile touched by its footprint); sort by
 * (tile, depth key, record); per-tile [start, end). */
static void scene_bin(const scene_t* S, bins_t* B)
{
    int64_t R = (int64_t)S->n_cams * S->n;
    int64_t total = 0;
    for (int64_t r = 0; r < R; ++r) {
        const proj_t* P = &S->proj[r];
        if (!P->vis) continue;
        int64_t nx = P->px1 / S->tw - P->px0 / S->tw + 1;
        int64_t ny = P->py1 / S->th - P->py0 / S->th + 1;
        total += nx * ny;
    }
    B->count = total;
    B->inst = (inst_t*)malloc((size_t)(total > 0 ? total : 1) * sizeof(inst_t));
    int64_t k = 0;
    for (int64_t r = 0; r < R; ++r) {
        const proj_t* P = &S->proj[r];
        if (!P->vis) continue;
        int c = (int)(r / S->n);
        for (int ty = P->py0 / S->th; ty <= P->py1 / S->th; ++ty)
            for (int tx = P->px0 / S->tw; tx <= P->px1 / S->tw; ++tx) {
                B->inst[k].tile = (uint32_t)(S->tile_off[c] + (int64_t)ty * S->tiles_x[c] + tx);
                B->inst[k].depth = P->depth_key;
                B->inst[k].rec = (uint32_t)r;
                ++k;
            }
    }
    qsort(B->inst, (size_t)total, sizeof(inst_t), inst_cmp);
    int64_t T = S->tile_off[S->n_cams];
    B->ranges = (uint32_t*)calloc((size_t)(2 * T + 2), sizeof(uint32_t));
    for (int64_t i = 0; i < total; ++i) {
        uint32_t t = B->inst[i].tile;
        if (i == 0 || B->inst[i - 1].tile != t) B->ranges[2 * t] = (uint32_t)i;
        if (i == total - 1 || B->inst[i + 1].tile != t) B->ranges[2 * t + 1] = (uint32_t)(i + 1);
    }
}

static void bins_free(bins_t* B)
{
    free(B->inst);
    free(B->ranges);
}

/* ------------------------------------------------------------- compositing */

typedef struct {
    int64_t rec;
    double alpha, a, G, T, dx, dy;
} contrib_t;

typedef struct {
    double* Q;          /* [P, d] */
    double* T_final;    /* [P] */
    int32_t* n_contrib; /* [P]: list position + 1 of the last blended Gaussian */
    int32_t* n_blended; /* [P] */
    int32_t* n_pairs;   /* [P]: pairs passing the footprint test before termination */
    double* margin;     /* [P]: min relative distance of a threshold decision; for the
                           termination test divided by the error amplification along the walk */
    uint64_t* hash;     /* [P]: decision signature */
} fwd_out_t;

static inline double rel_gap(double x, double thr) { return fabs(x - thr) / thr; }

static inline uint64_t mix64(uint64_t h, uint64_t v)
{
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    return h * 0xBF58476D1CE4E5B9ull;
}

/* Blend one pixel over an ordered candidate list.  ``list`` holds record ids;
 * when ``contribs`` is non-NULL the blended pairs are recorded for the adjoint.
 * With Zp non-NULL the same weights blend the camera-space depth of each
 * record's centre (Sec. III-A: depth is rendered by the same alpha blending). */
static void blend_pixel(const scene_t* S, const float* queries, int px, int py,
                        const uint32_t* list, int64_t len, double* Q, double* Zp, double* Tfin,
                        int32_t* ncontrib, int32_t* nblend, int32_t* npairs, double* margin,
                        uint64_t* hash, contrib_t* contribs)
{
    int d = S->d;
    for (int k = 0; k < d; ++k) Q[k] = 0.0;
    double Z = 0.0;
    double T = 1.0, mg = INFINITY;
    /* amp bounds how a relative error in each alpha grows in T: d(ln T) = -sum alpha/(1-alpha) d(ln alpha) */
    double amp = 1.0;
    int32_t last = 0, nb = 0, np = 0;
    uint64_t h = 0x1234567ull;
    for (int64_t k = 0; k < len; ++k) {
        const proj_t* P = &S->proj[list[k]];
        if (px < P->px0 || px > P->px1 || py < P->py0 || py > P->py1) continue;
        ++np;
        double dx = P->u - px, dy = P->v - py;
        double power = -0.5 * (P->A * dx * dx + P->C * dy * dy) - P->B * dx * dy;
        double G = exp(power);
        double a = P->o * G;
        double alpha = a < ORC_ALPHA_MAX ? a : ORC_ALPHA_MAX;
        mg = fmin(mg, rel_gap(a, ORC_ALPHA_MIN));
        mg = fmin(mg, rel_gap(a, ORC_ALPHA_MAX));
        if (alpha < ORC_ALPHA_MIN) continue;
        double Tn = T * (1.0 - alpha);
        mg = fmin(mg, rel_gap(Tn, ORC_T_STOP) / (amp + alpha / (1.0 - alpha)));
        if (Tn < ORC_T_STOP) break;
        int64_t gi = list[k] % S->n;
        const float* q = queries + gi * d;
        for (int j = 0; j < d; ++j) Q[j] += alpha * T * (double)q[j];
        Z += alpha * T * P->z;
        if (contribs) {
            contribs[nb].rec = list[k];
            contribs[nb].alpha = alpha;
            contribs[nb].a = a;
            contribs[nb].G = G;
            contribs[nb].T = T;
            contribs[nb].dx = dx;
            contribs[nb].dy = dy;
        }
        h = mix64(h, (uint64_t)list[k] * 2u + (a < ORC_ALPHA_MAX ? 0u : 1u));
        T = Tn;
        amp += alpha / (1.0 - alpha);
        last = (int32_t)(k + 1);
        ++nb;
    }
    *Tfin = T;
    if (Zp) *Zp = Z;
    if (ncontrib) *ncontrib = last;
    if (nblend) *nblend = nb;
    if (npairs) *npairs = np;
    if (margin) *margin = mg;
    if (hash) *hash = h;
}

/* pixel p of the concatenated views -> (camera, x, y) */
static void pixel_coords(const scene_t* S, int64_t p, int* c, int* x, int* y)
{
    int cc = 0;
    while (p >= S->pix_off[cc + 1]) ++cc;
    int64_t q = p - S->pix_off[cc];
    *c = cc;
    *x = (int)(q % S->cams[cc].w);
    *y = (int)(q / S->cams[cc].w);
}

static uint32_t* tile_list(const scene_t* S, const bins_t* B, uint32_t** store)
{
    uint32_t* ids = (uint32_t*)malloc((size_t)(B->count > 0 ? B->count : 1) * sizeof(uint32_t));
    for (int64_t i = 0; i < B->count; ++i) ids[i] = B->inst[i].rec;
    *store = ids;
    (void)S;
    return ids;
}

/* ================================================================ exports */

/* Projection of every (camera, Gaussian) record.  Returns the number of
 * visible records.  Outputs may be NULL. */
int64_t orc_project(int n, const float* means, const float* log_scales, const float* quats,
                    const float* logits, int n_cams, const float* cams, double* uv,
                    double* conic, double* opac, double* radius, int32_t* rect,
                    uint32_t* depth_key, uint8_t* vis, double* zcam)
{
    scene_t S;
    memset(&S, 0, sizeof S);
    scene_project(&S, n, means, log_scales, quats, logits, n_cams, cams, 16, 16);
    int64_t R = (int64_t)n_cams * n, nv = 0;
    for (int64_t r = 0; r < R; ++r) {
        const proj_t* P = &S.proj[r];
        nv += P->vis;
        if (uv) { uv[2 * r] = P->u; uv[2 * r + 1] = P->v; }
        if (conic) { conic[3 * r] = P->A; conic[3 * r + 1] = P->B; conic[3 * r + 2] = P->C; }
        if (opac) opac[r] = P->o;
        if (radius) radius[r] = P->radius;
        if (rect) {
            rect[4 * r] = P->vis ? P->px0 : -1;
            rect[4 * r + 1] = P->vis ? P->px1 : -1;
            rect[4 * r + 2] = P->vis ? P->py0 : -1;
            rect[4 * r + 3] = P->vis ? P->py1 : -1;
        }
        if (depth_key) depth_key[r] = P->vis ? P->depth_key : 0xFFFFFFFFu;
        if (vis) vis[r] = (uint8_t)P->vis;
        if (zcam) zcam[r] = P->z;
    }
    scene_free(&S);
    return nv;
}

/* The integer decisions of every record taken in FP64 (rect64 [R, 4] with -1
 * rows for culled records, key64, vis64) with their margin (margin64: the
 * smallest distance, in pixels, of u - r, u + r, v - r, v + r or 3 sqrt(lambda)
 * from an integer, or of z from the near plane), beside the float32 screen
 * mean the float32 decisions used (uv32 [R, 2]).  For tests that compare the
 * float32 decisions with the FP64 ones away from their thresholds.  Outputs may
 * be NULL. */
int64_t orc_project_decisions64(int n, const float* means, const float* log_scales, const float* quats,
                                const float* logits, int n_cams, const float* cams, int32_t* rect64,
                                uint32_t* key64, uint8_t* vis64, double* margin64, float* uv32)
{
    int64_t R = (int64_t)n_cams * n, nv = 0;
    cam_t* cs = (cam_t*)calloc((size_t)(n_cams > 0 ? n_cams : 1), sizeof(cam_t));
    for (int c = 0; c < n_cams; ++c) load_cam(cams + (size_t)c * CAM_FLOATS, &cs[c]);
#pragma omp parallel for schedule(static) reduction(+ : nv)
    for (int64_t r = 0; r < R; ++r) {
        const int c = (int)(r / n);
        const int64_t i = r % n;
        proj_t P;
        dec32_t D;
        project_f64(means + 3 * i, log_scales + 3 * i, quats + 4 * i, logits[i], &cs[c], &P);
        decide_f32(means + 3 * i, log_scales + 3 * i, quats + 4 * i, &cs[c], &D);
        nv += P.vis64;
        if (rect64) {
            rect64[4 * r] = P.vis64 ? P.r64x0 : -1;
            rect64[4 * r + 1] = P.vis64 ? P.r64x1 : -1;
            rect64[4 * r + 2] = P.vis64 ? P.r64y0 : -1;
            rect64[4 * r + 3] = P.vis64 ? P.r64y1 : -1;
        }
        if (key64) key64[r] = P.vis64 ? P.key64 : 0xFFFFFFFFu;
        if (vis64) vis64[r] = (uint8_t)P.vis64;
        if (margin64) margin64[r] = P.margin64;
        if (uv32) { uv32[2 * r] = D.u; uv32[2 * r + 1] = D.v; }
    }
    free(cs);
    return nv;
}

/* exp_cw of each input (for the tests that pin it against a reference exp). */
void orc_exp_cw(int64_t n, const float* x, float* y)
{
    for (int64_t i = 0; i < n; ++i) y[i] = exp_cw(x[i]);
}

/* Tile binning.  Returns the instance count; the arrays are filled only when
 * capacity >= count (tiles: global tile id, recs: record id, ranges: [tiles, 2]). */
int64_t orc_bin(int n, const float* means, const float* log_scales, const float* quats,
                const float* logits, int n_cams, const float* cams, int tw, int th,
                int64_t capacity, uint32_t* tiles, uint32_t* depths, uint32_t* recs,
                uint32_t* ranges)
{
    scene_t S;
    memset(&S, 0, sizeof S);
    scene_project(&S, n, means, log_scales, quats, logits, n_cams, cams, tw, th);
    bins_t B;
    scene_bin(&S, &B);
    int64_t cnt = B.count;
    if (capacity >= cnt) {
        for (int64_t i = 0; i < cnt; ++i) {
            if (tiles) tiles[i] = B.inst[i].tile;
            if (depths) depths[i] = B.inst[i].depth;
            if (recs) recs[i] = B.inst[i].rec;
        }
        if (ranges) memcpy(ranges, B.ranges, (size_t)S.tile_off[n_cams] * 2 * sizeof(uint32_t));
    }
    bins_free(&B);
    scene_free(&S);
    return cnt;
}

int64_t orc_num_tiles(int n_cams, const float* cams, int tw, int th)
{
    int64_t t = 0;
    for (int c = 0; c < n_cams; ++c) {
        int w = (int)cams[c * CAM_FLOATS], h = (int)cams[c * CAM_FLOATS + 1];
        t += (int64_t)((w + tw - 1) / tw) * ((h + th - 1) / th);
    }
    return t;
}

/* Tile-binned forward render (Eq. 4).  Outputs may be NULL except Q, T_final. */
int orc_render_forward(int n, int d, const float* means, const float* log_scales,
                       const float* quats, const float* logits, const float* queries,
                       int n_cams, const float* cams, int tw, int th, double* Q,
                       double* T_final, int32_t* n_contrib, int32_t* n_blended,
                       int32_t* n_pairs, double* margin, uint64_t* hash, double* Z)
{
    scene_t S;
    memset(&S, 0, sizeof S);
    scene_project(&S, n, means, log_scales, quats, logits, n_cams, cams, tw, th);
    S.d = d;
    bins_t B;
    scene_bin(&S, &B);
    uint32_t* ids;
    tile_list(&S, &B, &ids);
    int64_t P = S.pix_off[n_cams];
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t p = 0; p < P; ++p) {
        int c, x, y;
        pixel_coords(&S, p, &c, &x, &y);
        int64_t t = S.tile_off[c] + (int64_t)(y / th) * S.tiles_x[c] + x / tw;
        uint32_t s0 = B.ranges[2 * t], s1 = B.ranges[2 * t + 1];
        blend_pixel(&S, queries, x, y, ids + s0, (int64_t)s1 - s0, Q + p * d, Z ? Z + p : NULL, T_final + p,
                    n_contrib ? n_contrib + p : NULL, n_blended ? n_blended + p : NULL,
                    n_pairs ? n_pairs + p : NULL, margin ? margin + p : NULL,
                    hash ? hash + p : NULL, NULL);
    }
    free(ids);
    bins_free(&B);
    scene_free(&S);
    return 0;
}

/* The definition without tiles: per pixel, every visible record of its camera
 * in (depth key, record) order.  O(pixels x Gaussians): tiny scenes only. */
static int rec_cmp_depth(const void* pa, const void* pb, void* ctx)
{
    const proj_t* pr = (const proj_t*)ctx;
    uint32_t a = *(const uint32_t*)pa, b = *(const uint32_t*)pb;
    if (pr[a].depth_key != pr[b].depth_key) return pr[a].depth_key < pr[b].depth_key ? -1 : 1;
    return a < b ? -1 : (a > b);
}

int orc_render_bruteforce(int n, int d, const float* means, const float* log_scales,
                          const float* quats, const float* logits, const float* queries,
                          int n_cams, const float* cams, double* Q, double* T_final,
                          int32_t* n_blended, double* Z)
{
    scene_t S;
    memset(&S, 0, sizeof S);
    scene_project(&S, n, means, log_scales, quats, logits, n_cams, cams, 16, 16);
    S.d = d;
    for (int c = 0; c < n_cams; ++c) {
        uint32_t* order = (uint32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
        int64_t m = 0;
        for (int64_t i = 0; i < n; ++i)
            if (S.proj[(int64_t)c * n + i].vis) order[m++] = (uint32_t)((int64_t)c * n + i);
        qsort_r(order, (size_t)m, sizeof(uint32_t), rec_cmp_depth, S.proj);
        int W = S.cams[c].w, H = S.cams[c].h;
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t q = 0; q < (int64_t)W * H; ++q) {
            int64_t p = S.pix_off[c] + q;
            blend_pixel(&S, queries, (int)(q % W), (int)(q / W), order, m, Q + p * d,
                        Z ? Z + p : NULL, T_final + p, NULL, n_blended ? n_blended + p : NULL, NULL, NULL, NULL,
                        NULL);
        }
        free(order);
    }
    scene_free(&S);
    return 0;
}

/* ------------------------------------------------------------- the adjoint */

/* Chain the screen-space gradient of one record (du, dv, dA, dB, dC, dopacity)
 * back to the Gaussian's parameters.  Written by differentiating each forward
 * formula of project_one with respect to its scalar inputs. */
static void adjoint_record(const proj_t* P, const cam_t* cam, const double g[6], double dmean[3],
                           double dls[3], double dquat[4], double* dlogit)
{
    double du = g[0], dv = g[1], dA = g[2], dB = g[3], dC = g[4], dop = g[5];
    /* opacity o = sigmoid(logit) */
    *dlogit += dop * P->o * (1.0 - P->o);

    /* conic (A, B, C) = (c, -b, a) / det with det = a c - b^2 */
    double a = P->a, b = P->b, c = P->c, det = P->det, det2 = det * det;
    double da = dA * (-c * c / det2) + dB * (b * c / det2) + dC * (-b * b / det2);
    double db = dA * (2.0 * b * c / det2) + dB * (-(a * c + b * b) / det2) + dC * (2.0 * a * b / det2);
    double dc = dA * (-b * b / det2) + dB * (a * b / det2) + dC * (-a * a / det2);

    /* a = sum_kl J0k Sc_kl J0l (+dilation), b = sum J0k Sc_kl J1l, c = sum J1k Sc_kl J1l */
    double dSc[3][3], dJ[2][3];
    memset(dJ, 0, sizeof dJ);
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l)
            dSc[k][l] = da * P->J[0][k] * P->J[0][l] + db * P->J[0][k] * P->J[1][l] +
                        dc * P->J[1][k] * P->J[1][l];
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
            /* d/dJ0k of a: Sc_kl J0l (as left factor) and J0l Sc_lk (as right factor) */
            dJ[0][k] += da * (P->Sc[k][l] * P->J[0][l] + P->J[0][l] * P->Sc[l][k]);
            dJ[0][k] += db * (P->Sc[k][l] * P->J[1][l]);
            dJ[1][k] += db * (P->J[0][l] * P->Sc[l][k]);
            dJ[1][k] += dc * (P->Sc[k][l] * P->J[1][l] + P->J[1][l] * P->Sc[l][k]);
        }

    double x = P->x, y = P->y, z = P->z, fx = cam->fx, fy = cam->fy;
    double dx = 0.0, dy = 0.0, dz = 0.0;
    /* J00 = fx / z ; J11 = fy / z */
    dz += dJ[0][0] * (-fx / (z * z)) + dJ[1][1] * (-fy / (z * z));
    /* J02 = -fx * txc / z with txc = clamp(x / z) */
    double txc = P->clx ? (P->rx < 0 ? -P->limx : P->limx) : P->rx;
    double tyc = P->cly ? (P->ry < 0 ? -P->limy : P->limy) : P->ry;
    double dtxc = dJ[0][2] * (-fx / z);
    double dtyc = dJ[1][2] * (-fy / z);
    dz += dJ[0][2] * (fx * txc / (z * z)) + dJ[1][2] * (fy * tyc / (z * z));
    if (!P->clx) { dx += dtxc / z; dz += dtxc * (-x / (z * z)); }
    if (!P->cly) { dy += dtyc / z; dz += dtyc * (-y / (z * z)); }
    /* u = fx x / z + cx ; v = fy y / z + cy */
    dx += du * fx / z;
    dz += du * (-fx * x / (z * z));
    dy += dv * fy / z;
    dz += dv * (-fy * y / (z * z));
    /* camera centre (x, y, z) = W p + t */
    const double* V = cam->vm;
    for (int k = 0; k < 3; ++k) dmean[k] += V[k] * dx + V[4 + k] * dy + V[8 + k] * dz;

    /* Sc = W S3 W^T  ->  dS3_kl = sum_ij W_ik dSc_ij W_jl */
    double dS3[3][3];
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
            double acc = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) acc += V[4 * i + k] * dSc[i][j] * V[4 * j + l];
            dS3[k][l] = acc;
        }
    /* S3_ij = sum_k R_ik s_k^2 R_jk */
    double dR[3][3];
    memset(dR, 0, sizeof dR);
    double ds[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) {
                double s2 = P->s[k] * P->s[k];
                dR[i][k] += dS3[i][j] * s2 * P->R[j][k];
                dR[j][k] += dS3[i][j] * s2 * P->R[i][k];
                ds[k] += dS3[i][j] * P->R[i][k] * P->R[j][k] * 2.0 * P->s[k];
            }
    for (int k = 0; k < 3; ++k) dls[k] += ds[k] * P->s[k];

    /* rotation entries as functions of the unit quaternion (w, x, y, z) */
    double w = P->qn[0], qx = P->qn[1], qy = P->qn[2], qz = P->qn[3];
    double dq[4] = {0, 0, 0, 0};
    /* R00 = 1 - 2(y^2 + z^2) */
    dq[2] += dR[0][0] * (-4.0 * qy); dq[3] += dR[0][0] * (-4.0 * qz);
    /* R01 = 2(xy - wz) */
    dq[0] += dR[0][1] * (-2.0 * qz); dq[1] += dR[0][1] * (2.0 * qy);
    dq[2] += dR[0][1] * (2.0 * qx); dq[3] += dR[0][1] * (-2.0 * w);
    /* R02 = 2(xz + wy) */
    dq[0] += dR[0][2] * (2.0 * qy); dq[1] += dR[0][2] * (2.0 * qz);
    dq[2] += dR[0][2] * (2.0 * w); dq[3] += dR[0][2] * (2.0 * qx);
    /* R10 = 2(xy + wz) */
    dq[0] += dR[1][0] * (2.0 * qz); dq[1] += dR[1][0] * (2.0 * qy);
    dq[2] += dR[1][0] * (2.0 * qx); dq[3] += dR[1][0] * (2.0 * w);
    /* R11 = 1 - 2(x^2 + z^2) */
    dq[1] += dR[1][1] * (-4.0 * qx); dq[3] += dR[1][1] * (-4.0 * qz);
    /* R12 = 2(yz - wx) */
    dq[0] += dR[1][2] * (-2.0 * qx); dq[1] += dR[1][2] * (-2.0 * w);
    dq[2] += dR[1][2] * (2.0 * qz); dq[3] += dR[1][2] * (2.0 * qy);
    /* R20 = 2(xz - wy) */
    dq[0] += dR[2][0] * (-2.0 * qy); dq[1] += dR[2][0] * (2.0 * qz);
    dq[2] += dR[2][0] * (-2.0 * w); dq[3] += dR[2][0] * (2.0 * qx);
    /* R21 = 2(yz + wx) */
    dq[0] += dR[2][1] * (2.0 * qx); dq[1] += dR[2][1] * (2.0 * w);
    dq[2] += dR[2][1] * (2.0 * qz); dq[3] += dR[2][1] * (2.0 * qy);
    /* R22 = 1 - 2(x^2 + y^2) */
    dq[1] += dR[2][2] * (-4.0 * qx); dq[2] += dR[2][2] * (-4.0 * qy);
    /* normalisation qn = q / |q| */
    double dot = 0.0;
    for (int k = 0; k < 4; ++k) dot += dq[k] * P->qn[k];
    for (int k = 0; k < 4; ++k) dquat[k] += (dq[k] - P->qn[k] * dot) / P->qnorm;
}

/* Adjoint of the tile-binned render for a given upstream gradient dQ [P, d]
 * and, when dZ [P] is non-NULL, of the depth render.
 * Transmittance is re-derived forward (products), not by division.
 * Outputs are overwritten.  d_rec (nullable) receives the per-record
 * screen-space gradient [R, 6] = (du, dv, dA, dB, dC, dopacity).  The depth of
 * a record is z = row 3 of the world->camera transform applied to the mean,
 * so its gradient reaches the mean through that row. */
int orc_render_backward(int n, int d, const float* means, const float* log_scales,
                        const float* quats, const float* logits, const float* queries,
                        int n_cams, const float* cams, int tw, int th, const double* dQ,
                        double* d_means, double* d_log_scales, double* d_quats,
                        double* d_logits, double* d_queries, double* d_rec, const double* dZ)
{
    scene_t S;
    memset(&S, 0, sizeof S);
    scene_project(&S, n, means, log_scales, quats, logits, n_cams, cams, tw, th);
    S.d = d;
    bins_t B;
    scene_bin(&S, &B);
    uint32_t* ids;
    tile_list(&S, &B, &ids);
    int64_t Ptot = S.pix_off[n_cams];
    int64_t R = (int64_t)n_cams * n;
    int nth = omp_get_max_threads();
    double* acc_rec = (double*)calloc((size_t)nth * (size_t)(R > 0 ? R : 1) * 6, sizeof(double));
    double* acc_q = (double*)calloc((size_t)nth * (size_t)(n > 0 ? n : 1) * d, sizeof(double));
    double* acc_z = (double*)calloc((size_t)nth * (size_t)(R > 0 ? R : 1), sizeof(double));
    int64_t maxlen = 0;
    for (int64_t t = 0; t < S.tile_off[n_cams]; ++t) {
        int64_t len = (int64_t)B.ranges[2 * t + 1] - B.ranges[2 * t];
        if (len > maxlen) maxlen = len;
    }
#pragma omp parallel
    {
        int tid = omp_get_thread_num();
        double* my_rec = acc_rec + (size_t)tid * R * 6;
        double* my_q = acc_q + (size_t)tid * n * d;
        double* my_z = acc_z + (size_t)tid * R;
        contrib_t* cs = (contrib_t*)malloc((size_t)(maxlen > 0 ? maxlen : 1) * sizeof(contrib_t));
        double* Qp = (double*)malloc((size_t)d * sizeof(double));
        double* suffix = (double*)malloc((size_t)d * sizeof(double));
#pragma omp for schedule(dynamic, 256)
        for (int64_t p = 0; p < Ptot; ++p) {
            int c, x, y;
            pixel_coords(&S, p, &c, &x, &y);
            int64_t t = S.tile_off[c] + (int64_t)(y / th) * S.tiles_x[c] + x / tw;
            uint32_t s0 = B.ranges[2 * t], s1 = B.ranges[2 * t + 1];
            double Tf;
            int32_t nb;
            blend_pixel(&S, queries, x, y, ids + s0, (int64_t)s1 - s0, Qp, NULL, &Tf, NULL, &nb, NULL,
                        NULL, NULL, cs);
            const double* g = dQ + p * d;
            const double gz = dZ ? dZ[p] : 0.0;
            /* suffix = sum over later blended m of alpha_m T_m q_m (and of z_m) */
            for (int j = 0; j < d; ++j) suffix[j] = 0.0;
            double suffix_z = 0.0;
            for (int k = nb - 1; k >= 0; --k) {
                const contrib_t* e = &cs[k];
                int64_t gi = e->rec % n;
                const float* q = queries + gi * d;
                /* dQ/dalpha_k = T_k q_k - suffix / (1 - alpha_k) */
                double dal = 0.0;
                for (int j = 0; j < d; ++j) {
                    dal += (e->T * (double)q[j] - suffix[j] / (1.0 - e->alpha)) * g[j];
                    my_q[gi * d + j] += e->alpha * e->T * g[j];
                }
                for (int j = 0; j < d; ++j) suffix[j] += e->alpha * e->T * (double)q[j];
                if (dZ) {
                    const double z = S.proj[e->rec].z;
                    dal += (e->T * z - suffix_z / (1.0 - e->alpha)) * gz;
                    my_z[e->rec] += e->alpha * e->T * gz;
                    suffix_z += e->alpha * e->T * z;
                }
                if (e->a < ORC_ALPHA_MAX) {
                    const proj_t* P = &S.proj[e->rec];
                    double dpow = dal * e->a; /* alpha = o exp(power) */
                    double* gr = my_rec + e->rec * 6;
                    gr[0] += dpow * (-(P->A * e->dx + P->B * e->dy));
                    gr[1] += dpow * (-(P->C * e->dy + P->B * e->dx));
                    gr[2] += dpow * (-0.5 * e->dx * e->dx);
                    gr[3] += dpow * (-e->dx * e->dy);
                    gr[4] += dpow * (-0.5 * e->dy * e->dy);
                    gr[5] += dal * e->G;
                }
            }
        }
        free(cs);
        free(Qp);
        free(suffix);
    }
    /* reduce the per-thread partial sums */
    double* rec_g = (double*)calloc((size_t)(R > 0 ? R : 1) * 6, sizeof(double));
    for (int t = 0; t < nth; ++t)
        for (int64_t k = 0; k < R * 6; ++k) rec_g[k] += acc_rec[(size_t)t * R * 6 + k];
    double* rec_z = (double*)calloc((size_t)(R > 0 ? R : 1), sizeof(double));
    for (int t = 0; t < nth; ++t)
        for (int64_t k = 0; k < R; ++k) rec_z[k] += acc_z[(size_t)t * R + k];
    memset(d_queries, 0, (size_t)n * d * sizeof(double));
    for (int t = 0; t < nth; ++t)
        for (int64_t k = 0; k < (int64_t)n * d; ++k) d_queries[k] += acc_q[(size_t)t * n * d + k];
    if (d_rec) memcpy(d_rec, rec_g, (size_t)R * 6 * sizeof(double));
    /* chain to the parameters; cameras summed in order per Gaussian */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double dm[3] = {0, 0, 0}, dl[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dlg = 0.0;
        for (int c = 0; c < n_cams; ++c) {
            const proj_t* P = &S.proj[(int64_t)c * n + i];
            if (!P->vis) continue;
            adjoint_record(P, &S.cams[c], rec_g + ((int64_t)c * n + i) * 6, dm, dl, dq, &dlg);
            const double gzr = rec_z[(int64_t)c * n + i];
            for (int k = 0; k < 3; ++k) dm[k] += gzr * S.cams[c].vm[8 + k];
        }
        for (int k = 0; k < 3; ++k) d_means[3 * i + k] = dm[k];
        for (int k = 0; k < 3; ++k) d_log_scales[3 * i + k] = dl[k];
        for (int k = 0; k < 4; ++k) d_quats[4 * i + k] = dq[k];
        d_logits[i] = dlg;
    }
    free(rec_g);
    free(rec_z);
    free(acc_rec);
    free(acc_q);
    free(acc_z);
    free(ids);
    bins_free(&B);
    scene_free(&S);
    return 0;
}

int orc_num_threads(void) { return omp_get_max_threads(); }

/* ======================================================= pixel windows
 *
 * Test helpers over a rectangular window of pixels of ONE camera: the
 * tile-free definition (every visible record in (depth key, record) order,
 * the per-pixel footprint test inside blend_pixel), which the tile-binned
 * render equals bitwise (pinned on tiny scenes).  Used to take central finite
 * differences at realistic list lengths without re-rendering a whole frame. */

typedef struct {
    const proj_t* proj;
    const uint32_t* order; /* visible records by (depth key, record) */
    int64_t m;
} worder_t;

static int cmp_rec_key(const proj_t* pr, uint32_t a, uint32_t b)
{
    if (pr[a].depth_key != pr[b].depth_key) return pr[a].depth_key < pr[b].depth_key ? -1 : 1;
    return a < b ? -1 : (a > b);
}

/* Blend every window pixel; returns sum_p w_p . Q_p (w may be NULL: 0) and
 * writes Q [npx, d], T [npx] and the decision signatures [npx] when non-NULL. */
static double window_eval(const scene_t* S, const float* queries, const uint32_t* order, int64_t m,
                          int x0, int y0, int ww, int wh, const double* w, double* Qbuf, double* Tbuf,
                          uint64_t* hash, double* Qout)
{
    double acc = 0.0;
    const int d = S->d;
    for (int yy = 0; yy < wh; ++yy)
        for (int xx = 0; xx < ww; ++xx) {
            const int64_t p = (int64_t)yy * ww + xx;
            double T;
            uint64_t h;
            blend_pixel(S, queries, x0 + xx, y0 + yy, order, m, Qbuf, NULL, &T, NULL, NULL, NULL, NULL, &h,
                        NULL);
            if (hash) hash[p] = h;
            if (Tbuf) Tbuf[p] = T;
            if (Qout) memcpy(Qout + p * d, Qbuf, (size_t)d * sizeof(double));
            if (w)
                for (int j = 0; j < d; ++j) acc += w[p * d + j] * Qbuf[j];
        }
    return acc;
}

static int64_t visible_order(const scene_t* S, uint32_t* order)
{
    int64_t m = 0;
    for (int64_t i = 0; i < S->n; ++i)
        if (S->proj[i].vis) order[m++] = (uint32_t)i;
    qsort_r(order, (size_t)m, sizeof(uint32_t), rec_cmp_depth, (void*)S->proj);
    return m;
}

/* Query map, transmittance and decision signatures of the pixels
 * [x0, x0 + ww) x [y0, y0 + wh) of the camera ``cam`` (one row). */
int orc_render_window(int n, int d, const float* means, const float* log_scales, const float* quats,
                      const float* logits, const float* queries, const float* cam, int x0, int y0, int ww,
                      int wh, double* Q, double* T_final, uint64_t* hash)
{
    scene_t S;
    memset(&S, 0, sizeof S);
    scene_project(&S, n, means, log_scales, quats, logits, 1, cam, 16, 16);
    S.d = d;
    uint32_t* order = (uint32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
    const int64_t m = visible_order(&S, order);
    double* Qbuf = (double*)malloc((size_t)d * sizeof(double));
    window_eval(&S, queries, order, m, x0, y0, ww, wh, NULL, Qbuf, T_final, hash, Q);
    free(Qbuf);
    free(order);
    scene_free(&S);
    return 0;
}

/* Central finite differences of L(theta) = sum_p w_p . Q_p(theta) over the
 * window for a list of probes (Gaussian pg[j], parameter pk[j]); parameter
 * index k: 0-2 mean, 3-5 log-scale, 6-9 quaternion, 10 opacity logit,
 * 11 .. 10 + d query.  The perturbed value x +- h (h = hrel max(1, |x|)) is
 * rounded to float32, as the inputs are float32, and the realised step is
 * the exact difference of the two rounded values.  ok[j] = 1 when no pixel's
 * decision signature (which records blend, in which order, which are clamped)
 * changes inside the stencil, i.e. the functional is differentiable there. */
int orc_fd_window(int n, int d, const float* means, const float* log_scales, const float* quats,
                  const float* logits, const float* queries, const float* cam, int x0, int y0, int ww, int wh,
                  const double* w, int nprobe, const int32_t* pg, const int32_t* pk, double hrel, double* fd,
                  int32_t* ok)
{
    scene_t S;
    memset(&S, 0, sizeof S);
    scene_project(&S, n, means, log_scales, quats, logits, 1, cam, 16, 16);
    S.d = d;
    const int64_t npx = (int64_t)ww * wh;
    uint32_t* order = (uint32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
    const int64_t m = visible_order(&S, order);
    uint64_t* h0 = (uint64_t*)malloc((size_t)(npx > 0 ? npx : 1) * sizeof(uint64_t));
    {
        double* Qbuf = (double*)malloc((size_t)d * sizeof(double));
        window_eval(&S, queries, order, m, x0, y0, ww, wh, NULL, Qbuf, NULL, h0, NULL);
        free(Qbuf);
    }
#pragma omp parallel
    {
        scene_t L = S;
        proj_t* pr = (proj_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(proj_t));
        memcpy(pr, S.proj, (size_t)n * sizeof(proj_t));
        L.proj = pr;
        float* qloc = (float*)malloc((size_t)(n > 0 ? n : 1) * d * sizeof(float));
        memcpy(qloc, queries, (size_t)n * d * sizeof(float));
        uint32_t* ord = (uint32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
        uint64_t* hh = (uint64_t*)malloc((size_t)(npx > 0 ? npx : 1) * sizeof(uint64_t));
        double* Qbuf = (double*)malloc((size_t)d * sizeof(double));
#pragma omp for schedule(dynamic, 4)
        for (int j = 0; j < nprobe; ++j) {
            const int i = pg[j], k = pk[j];
            float mu[3], ls[3], qt[4], lg = logits[i];
            memcpy(mu, means + 3 * (size_t)i, sizeof mu);
            memcpy(ls, log_scales + 3 * (size_t)i, sizeof ls);
            memcpy(qt, quats + 4 * (size_t)i, sizeof qt);
            float* slot = k < 3 ? &mu[k] : k < 6 ? &ls[k - 3] : k < 10 ? &qt[k - 6] : k == 10 ? &lg
                                                                                      : &qloc[(size_t)i * d + (k - 11)];
            const float xv = *slot;
            const double h = hrel * fmax(1.0, fabs((double)xv));
            double val[2], step[2];
            int good = 1;
            for (int sgn = 0; sgn < 2; ++sgn) {
                const float xp = (float)((double)xv + (sgn == 0 ? h : -h));
                step[sgn] = fabs((double)xp - (double)xv);
                *slot = xp;
                project_one(mu, ls, qt, lg, &S.cams[0], &pr[i]);
                /* the order with record i at the place its (new) depth key takes */
                int64_t mm = 0;
                for (int64_t t = 0; t < m; ++t)
                    if (order[t] != (uint32_t)i) ord[mm++] = order[t];
                if (pr[i].vis) {
                    int64_t pos = mm;
                    for (int64_t t = 0; t < mm; ++t)
                        if (cmp_rec_key(pr, (uint32_t)i, ord[t]) < 0) { pos = t; break; }
                    memmove(ord + pos + 1, ord + pos, (size_t)(mm - pos) * sizeof(uint32_t));
                    ord[pos] = (uint32_t)i;
                    ++mm;
                }
                val[sgn] = window_eval(&L, qloc, ord, mm, x0, y0, ww, wh, w, Qbuf, NULL, hh, NULL);
                for (int64_t p = 0; p < npx; ++p)
                    if (hh[p] != h0[p]) { good = 0; break; }
                *slot = xv;
            }
            pr[i] = S.proj[i];
            fd[j] = (val[0] - val[1]) / (step[0] + step[1]);
            ok[j] = good && step[0] > 0.0 && step[1] > 0.0;
        }
        free(pr);
        free(qloc);
        free(ord);
        free(hh);
        free(Qbuf);
    }
    free(h0);
    free(order);
    scene_free(&S);
    return 0;
}

/* The walk of each listed pixel p (concatenated pixel order) through its
 * tile's list: for the k-th blended record, its id, its alpha and the
 * transmittance before it (T_k), at most max_len entries per pixel; count[i]
 * the number blended and T_final[i] the transmittance left. */
int orc_pixel_walks(int n, int d, const float* means, const float* log_scales, const float* quats,
                    const float* logits, const float* queries, int n_cams, const float* cams, int tw, int th,
                    int npix, const int64_t* pixels, int max_len, int64_t* recs, double* alpha,
                    double* T_before, int32_t* count, double* T_final)
{
    scene_t S;
    memset(&S, 0, sizeof S);
    scene_project(&S, n, means, log_scales, quats, logits, n_cams, cams, tw, th);
    S.d = d;
    bins_t B;
    scene_bin(&S, &B);
    uint32_t* ids;
    tile_list(&S, &B, &ids);
    int64_t maxlen = 1;
    for (int64_t t = 0; t < S.tile_off[n_cams]; ++t) {
        int64_t len = (int64_t)B.ranges[2 * t + 1] - B.ranges[2 * t];
        if (len > maxlen) maxlen = len;
    }
    contrib_t* cs = (contrib_t*)malloc((size_t)maxlen * sizeof(contrib_t));
    double* Qp = (double*)malloc((size_t)(d > 0 ? d : 1) * sizeof(double));
    for (int i = 0; i < npix; ++i) {
        int c, x, y;
        pixel_coords(&S, pixels[i], &c, &x, &y);
        int64_t t = S.tile_off[c] + (int64_t)(y / th) * S.tiles_x[c] + x / tw;
        uint32_t s0 = B.ranges[2 * t], s1 = B.ranges[2 * t + 1];
        int32_t nb = 0;
        blend_pixel(&S, queries, x, y, ids + s0, (int64_t)s1 - s0, Qp, NULL, &T_final[i], NULL, &nb, NULL, NULL,
                    NULL, cs);
        count[i] = nb;
        for (int k = 0; k < nb && k < max_len; ++k) {
            recs[(int64_t)i * max_len + k] = cs[k].rec;
            alpha[(int64_t)i * max_len + k] = cs[k].alpha;
            T_before[(int64_t)i * max_len + k] = cs[k].T;
        }
    }
    free(cs);
    free(Qp);
    free(ids);
    bins_free(&B);
    scene_free(&S);
    return 0;
}

/* Threads of the OpenMP regions above (for timing the oracle on one core). */
void orc_set_num_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}
