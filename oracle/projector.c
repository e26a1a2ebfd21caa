/*
 * FP64 CPU oracle: ray-driven Joseph projector and its scatter adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference the
 * HIP library is checked against; it shares no code with the library and the library
 * never calls it.
 *
 * What it computes: the geometric part G of the projection operator P = diag(mult) G
 * of the PET forward model (Section 1.2, "PET Reconstruction via Optimization": P
 * "includes geometric factors, attenuation and normalization").  The paper delegates
 * the geometry to its projector package; the reading implemented here is Joseph's
 * method (P. M. Joseph, IEEE TMI 1982) for parallel-beam rays with oblique planes:
 *
 *   ray (a, q, k):   phi = a*pi/n_ang,  s = (k - (n_rad-1)/2) d_rad,
 *                    plane q = local plane p of segment g,
 *                    z_p = (p - (N_g-1)/2) pitch_g vz  (pitch_g = 1, or 2 for ring pairs),
 *   points           (s cos phi - t sin phi,  s sin phi + t cos phi,  z_p + tau_g t).
 *
 * Scanner model (a ring of radius R): with `nonarc` the radial bins are equal steps of
 * the angle on the ring, s = R sin((k - (n_rad-1)/2) d_rad / R); with `oblique_s` a line
 * of response between two rings spans the chord 2 sqrt(R^2 - s^2) between its detectors,
 * so its slope is tau_g R / sqrt(R^2 - s^2) (tau_g: the slope at s = 0).
 *
 * If |cos phi| >= |sin phi| (decided by the integer test 4a <= n_ang or 4a >= 3 n_ang,
 * ties go to rows) the ray is sampled at every image row y_j; otherwise at every column
 * x_i.  At each sample the image slice is interpolated bilinearly in the two remaining
 * axes (zero outside the image) and weighted by the 3-D path length per sample,
 * v/|cos phi| * sqrt(1 + tau^2) (or v/|sin phi| * ...).
 *
 * The adjoint is computed by scattering the very same weights (ray-driven), which is a
 * different algorithm from the GPU's voxel-driven gather.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define ORC_MAX_SEG 128

typedef struct {
    int32_t nx, ny, nz;
    double vx, vy, vz;
    int32_t n_rad;
    double d_rad;
    int32_t n_ang;
    int32_t n_seg;
    int32_t seg_planes[ORC_MAX_SEG];
    double seg_tan[ORC_MAX_SEG];
    int32_t seg_pitch[ORC_MAX_SEG]; /* axial spacing of the segment's planes in image planes
                                     * (0 or 1: every plane; 2: every other plane, the ring
                                     * pairs of span 1 with a ring pitch of two planes) */
    double det_radius;              /* scanner model: detector ring radius R (mm) */
    int32_t nonarc;                 /* radial bins at R sin(...) instead of equal steps */
    int32_t oblique_s;              /* slope tau_g R / sqrt(R^2 - s^2) */
} orc_geom;

static int32_t n_planes(const orc_geom* G) {
    int32_t n = 0;
    for (int g = 0; g < G->n_seg; g++) n += G->seg_planes[g];
    return n;
}

static void plane_seg(const orc_geom* G, int32_t q, int32_t* g_out, int32_t* p_out) {
    int32_t g = 0;
    while (q >= G->seg_planes[g]) {
        q -= G->seg_planes[g];
        g++;
    }
    *g_out = g;
    *p_out = q;
}

static int row_dominant(const orc_geom* G, int32_t a) {
    return (4 * a <= G->n_ang) || (4 * a >= 3 * G->n_ang);
}

/* One sample of a ray: the primary index (row j or column i), the continuous index in
 * the secondary in-plane axis (u) and in z (w), and the path length per sample. */
typedef struct {
    double u, w;
} sample_t;

/* Radial position (mm) of bin k. */
static double radial_pos(const orc_geom* G, int32_t k) {
    double t = ((double)k - 0.5 * (G->n_rad - 1)) * G->d_rad;
    return G->nonarc ? G->det_radius * sin(t / G->det_radius) : t;
}

/* Axial slope of the rays of segment g in radial bin k. */
static double ray_slope(const orc_geom* G, int32_t g, int32_t k) {
    double tau = G->seg_tan[g];
    if (G->oblique_s) {
        double r = radial_pos(G, k), R = G->det_radius;
        tau *= R / sqrt(R * R - r * r);
    }
    return tau;
}

static sample_t ray_sample(const orc_geom* G, int32_t a, int32_t p, int32_t g,
                           int32_t k, int32_t prim) {
    double phi = M_PI * (double)a / (double)G->n_ang;
    double c = cos(phi), s = sin(phi);
    double r = radial_pos(G, k);
    int32_t Ng = G->seg_planes[g];
    int32_t pitch = G->seg_pitch[g] > 1 ? G->seg_pitch[g] : 1;
    double zp = ((double)p - 0.5 * (Ng - 1)) * pitch * G->vz;
    double tau = ray_slope(G, g, k);
    sample_t out;
    if (row_dominant(G, a)) {
        double Y = ((double)prim - 0.5 * (G->ny - 1)) * G->vy;
        double t = (Y - r * s) / c;
        double X = (r - Y * s) / c;
        double Z = zp + tau * t;
        out.u = X / G->vx + 0.5 * (G->nx - 1);
        out.w = Z / G->vz + 0.5 * (G->nz - 1);
    } else {
        double X = ((double)prim - 0.5 * (G->nx - 1)) * G->vx;
        double t = (r * c - X) / s;
        double Y = (r - X * c) / s;
        double Z = zp + tau * t;
        out.u = Y / G->vy + 0.5 * (G->ny - 1);
        out.w = Z / G->vz + 0.5 * (G->nz - 1);
    }
    return out;
}

static double step_length(const orc_geom* G, int32_t a, int32_t g, int32_t k) {
    double phi = M_PI * (double)a / (double)G->n_ang;
    double tau = ray_slope(G, g, k);
    if (row_dominant(G, a)) return G->vy / fabs(cos(phi)) * sqrt(1.0 + tau * tau);
    return G->vx / fabs(sin(phi)) * sqrt(1.0 + tau * tau);
}

/* Value of voxel (x index xi, y index yi, z index zi) or 0 outside the image. */
static double voxel(const orc_geom* G, const double* img, int64_t xi, int64_t yi, int64_t zi) {
    if (xi < 0 || xi >= G->nx || yi < 0 || yi >= G->ny || zi < 0 || zi >= G->nz) return 0.0;
    return img[(zi * G->ny + yi) * G->nx + xi];
}

static void voxel_add(const orc_geom* G, double* img, int64_t xi, int64_t yi, int64_t zi,
                      double v) {
    if (xi < 0 || xi >= G->nx || yi < 0 || yi >= G->ny || zi < 0 || zi >= G->nz) return;
    img[(zi * G->ny + yi) * G->nx + xi] += v;
}

/* Sum over samples of the bilinear interpolant: the ray sum of G. */
static double ray_sum(const orc_geom* G, const double* img, int32_t a, int32_t q, int32_t k) {
    int32_t g, p;
    plane_seg(G, q, &g, &p);
    int rowdom = row_dominant(G, a);
    int32_t n_prim = rowdom ? G->ny : G->nx;
    double acc = 0.0;
    for (int32_t j = 0; j < n_prim; j++) {
        sample_t sm = ray_sample(G, a, p, g, k, j);
        double u0 = floor(sm.u), w0 = floor(sm.w);
        double fu = sm.u - u0, fw = sm.w - w0;
        int64_t iu = (int64_t)u0, iw = (int64_t)w0;
        double v00, v10, v01, v11;
        if (rowdom) {
            v00 = voxel(G, img, iu, j, iw);
            v10 = voxel(G, img, iu + 1, j, iw);
            v01 = voxel(G, img, iu, j, iw + 1);
            v11 = voxel(G, img, iu + 1, j, iw + 1);
        } else {
            v00 = voxel(G, img, j, iu, iw);
            v10 = voxel(G, img, j, iu + 1, iw);
            v01 = voxel(G, img, j, iu, iw + 1);
            v11 = voxel(G, img, j, iu + 1, iw + 1);
        }
        acc += (1 - fu) * (1 - fw) * v00 + fu * (1 - fw) * v10 + (1 - fu) * fw * v01 +
               fu * fw * v11;
    }
    return acc * step_length(G, a, g, k);
}

/* out[ia][q][k] = (G img)[angles[ia]][q][k]: the rows of the listed angles, packed. */
void orc_forward(const orc_geom* G, const int32_t* angles, int32_t n_angles,
                 const double* img, double* out) {
    int32_t np_ = n_planes(G);
    int64_t per_angle = (int64_t)np_ * G->n_rad;
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int32_t ia = 0; ia < n_angles; ia++) {
        for (int32_t q = 0; q < np_; q++) {
            int32_t a = angles[ia];
            for (int32_t k = 0; k < G->n_rad; k++)
                out[ia * per_angle + (int64_t)q * G->n_rad + k] = ray_sum(G, img, a, q, k);
        }
    }
}

/* Single ray sum (for sampled checks at full size). */
double orc_ray(const orc_geom* G, const double* img, int32_t a, int32_t q, int32_t k) {
    return ray_sum(G, img, a, q, k);
}

/* img_out = G^T y for y packed as y[ia][q][k] over the listed angles (overwrites).
 * Ray-driven scatter; for each angle the work is split over the primary index, so each
 * thread writes only its own image row (or column): no races, fixed summation order. */
void orc_backward(const orc_geom* G, const int32_t* angles, int32_t n_angles,
                  const double* y, double* img_out) {
    int32_t np_ = n_planes(G);
    int64_t per_angle = (int64_t)np_ * G->n_rad;
    memset(img_out, 0, sizeof(double) * (size_t)G->nx * G->ny * G->nz);
    for (int32_t ia = 0; ia < n_angles; ia++) {
        int32_t a = angles[ia];
        int rowdom = row_dominant(G, a);
        int32_t n_prim = rowdom ? G->ny : G->nx;
#pragma omp parallel for schedule(dynamic, 1)
        for (int32_t j = 0; j < n_prim; j++) {
            for (int32_t q = 0; q < np_; q++) {
                int32_t g, p;
                plane_seg(G, q, &g, &p);
                for (int32_t k = 0; k < G->n_rad; k++) {
                    double val = y[ia * per_angle + (int64_t)q * G->n_rad + k];
                    if (val == 0.0) continue;
                    val *= step_length(G, a, g, k);
                    sample_t sm = ray_sample(G, a, p, g, k, j);
                    double u0 = floor(sm.u), w0 = floor(sm.w);
                    double fu = sm.u - u0, fw = sm.w - w0;
                    int64_t iu = (int64_t)u0, iw = (int64_t)w0;
                    if (rowdom) {
                        voxel_add(G, img_out, iu, j, iw, (1 - fu) * (1 - fw) * val);
                        voxel_add(G, img_out, iu + 1, j, iw, fu * (1 - fw) * val);
                        voxel_add(G, img_out, iu, j, iw + 1, (1 - fu) * fw * val);
                        voxel_add(G, img_out, iu + 1, j, iw + 1, fu * fw * val);
                    } else {
                        voxel_add(G, img_out, j, iu, iw, (1 - fu) * (1 - fw) * val);
                        voxel_add(G, img_out, j, iu + 1, iw, fu * (1 - fw) * val);
                        voxel_add(G, img_out, j, iu, iw + 1, (1 - fu) * fw * val);
                        voxel_add(G, img_out, j, iu + 1, iw + 1, fu * fw * val);
                    }
                }
            }
        }
    }
}

int32_t orc_max_seg(void) { return ORC_MAX_SEG; }
