// HIP kernels of the SPDHG subset step for gfx950 (wave64).
//
//   fwd_*   ray-driven Joseph forward projection of a subset (one thread per ray, the
//           thread walks the primary axis); variants fuse the per-bin epilogues:
//           plain output, preconditioner sigma = gamma rho / (A 1), the KL-dual prox of
//           Algorithm 2 line 5, or the FP64 data term of the objective.
//   bwd_*   voxel-driven gather backprojection A_i^T (one thread per voxel, loops over the
//           subset's angles and the rays that touch the voxel; same weights as fwd_*, no
//           atomics); variants fuse: plain output, running minimum for the primal step
//           T, or the primal epilogue of Algorithm 2 lines 7-8 and line 3 of the next
//           iteration.
//   tv_*    prior block of TV / dTV (eq. setting TV, Section 4.3): dual ascent with the
//           l2-ball projection, its adjoint, and the same primal epilogue.
//   reduce  deterministic FP64 block partials + ordered final sum.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "geom.hpp"

#define BLOCK 256

namespace spdhg {

// ---------------------------------------------------------------- ray walk
// Range of primary indices [j0, j1) outside of which every tap of the ray is zero
// (conservative by two samples; the loop still tests every tap).
__device__ __forceinline__ void ray_range(const GeomDev& G, const AngleDev& A,
                                          const SegAngleDev& S, double u0, double kk, int zb,
                                          int& j0, int& j1) {
    double lo = -1e30, hi = 1e30;
    // secondary: need -1 < u < n_sec, u = du_dj * jj + u0
    if (A.du_dj != 0.0) {
        const double t0 = (-1.0 - u0) / A.du_dj, t1 = ((double)A.n_sec - u0) / A.du_dj;
        lo = fmax(lo, fmin(t0, t1));
        hi = fmin(hi, fmax(t0, t1));
    } else if (!(u0 > -1.0 && u0 < (double)A.n_sec)) {
        j0 = j1 = 0;
        return;
    }
    // axial: need -1 < zb + e < nz, e = ez_dj * jj + ez_dk * kk
    const double ek = S.ez_dk * kk;
    if (S.ez_dj != 0.0) {
        const double t0 = (-1.0 - (double)zb - ek) / S.ez_dj;
        const double t1 = ((double)G.nz - (double)zb - ek) / S.ez_dj;
        lo = fmax(lo, fmin(t0, t1));
        hi = fmin(hi, fmax(t0, t1));
    } else {
        const double z = (double)zb + ek;
        if (!(z > -1.0 && z < (double)G.nz)) {
            j0 = j1 = 0;
            return;
        }
    }
    const double a = fmax(lo + A.cj - 2.0, 0.0);
    const double b = fmin(hi + A.cj + 3.0, (double)A.n_prim);
    if (!(a < b)) {
        j0 = j1 = 0;
        return;
    }
    j0 = (int)a;
    j1 = (int)b;
}

// Sum over samples of the bilinear interpolant times the segment step length: (G x) of
// ray (a, q, k).  ONES: the image is 1 everywhere inside (sensitivities).
template <bool ONES>
__device__ float ray_sum(const GeomDev& G, const float* __restrict__ x, int a, int q, int k) {
    const AngleDev A = G.ang[a];
    const int g = G.plane_seg[q];
    const int p = q - G.seg_base[g];
    const SegAngleDev S = G.sa[a * G.n_seg + g];
    const double kk = (double)k - G.ck;
    const int zb = p + G.seg_off[g];
    const int64_t s_sec = A.rowdom ? 1 : G.nx;
    const int64_t s_prim = A.rowdom ? G.nx : 1;
    const int64_t s_z = (int64_t)G.nx * G.ny;
    const double u0 = __builtin_fma(A.du_dk, kk, A.cu);
    int j0, j1;
    ray_range(G, A, S, u0, kk, zb, j0, j1);
    float acc = 0.0f;
    for (int j = j0; j < j1; ++j) {
        const double jj = (double)j - A.cj;
        const Sample s = split(sec_coord(A, kk, jj));
        const Sample sz = split(ax_offset(S, kk, jj));
        const float fz = sz.fu;
        const int iz = zb + sz.i0;
        const bool x0ok = (unsigned)s.i0 < (unsigned)A.n_sec;
        const bool x1ok = (unsigned)(s.i0 + 1) < (unsigned)A.n_sec;
        const bool z0ok = (unsigned)iz < (unsigned)G.nz;
        const bool z1ok = (unsigned)(iz + 1) < (unsigned)G.nz;
        const int64_t base = (int64_t)iz * s_z + (int64_t)j * s_prim + (int64_t)s.i0 * s_sec;
        float v00 = 0.f, v10 = 0.f, v01 = 0.f, v11 = 0.f;
        if (ONES) {
            v00 = (x0ok && z0ok) ? 1.f : 0.f;
            v10 = (x1ok && z0ok) ? 1.f : 0.f;
            v01 = (x0ok && z1ok) ? 1.f : 0.f;
            v11 = (x1ok && z1ok) ? 1.f : 0.f;
        } else {
            if (x0ok && z0ok) v00 = x[base];
            if (x1ok && z0ok) v10 = x[base + s_sec];
            if (x0ok && z1ok) v01 = x[base + s_z];
            if (x1ok && z1ok) v11 = x[base + s_z + s_sec];
        }
        const float wx0 = 1.0f - s.fu, wx1 = s.fu;
        const float wz0 = 1.0f - fz, wz1 = fz;
        acc += wz0 * (wx0 * v00 + wx1 * v10) + wz1 * (wx0 * v01 + wx1 * v11);
    }
    return acc * S.L;
}

// Number of taps of ray (a, q, k) with a nonzero weight inside the image: the ray's
// nonzeros in the system matrix (each tap is one voxel; voxels hit twice along a ray
// are counted per tap, as the projector evaluates them).
__device__ double ray_taps(const GeomDev& G, int a, int q, int k) {
    const AngleDev A = G.ang[a];
    const int g = G.plane_seg[q];
    const int p = q - G.seg_base[g];
    const SegAngleDev S = G.sa[a * G.n_seg + g];
    const double kk = (double)k - G.ck;
    const int zb = p + G.seg_off[g];
    const double u0 = __builtin_fma(A.du_dk, kk, A.cu);
    int j0, j1;
    ray_range(G, A, S, u0, kk, zb, j0, j1);
    double n = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double jj = (double)j - A.cj;
        const Sample s = split(sec_coord(A, kk, jj));
        const Sample sz = split(ax_offset(S, kk, jj));
        const int iz = zb + sz.i0;
        const float wx[2] = {1.0f - s.fu, s.fu};
        const float wz[2] = {1.0f - sz.fu, sz.fu};
        for (int dz = 0; dz < 2; ++dz)
            for (int dx = 0; dx < 2; ++dx)
                if ((unsigned)(s.i0 + dx) < (unsigned)A.n_sec &&
                    (unsigned)(iz + dz) < (unsigned)G.nz && wx[dx] * wz[dz] != 0.0f)
                    n += 1.0;
    }
    return n;
}

struct RayIdx {
    int ia, q, k;
};

__device__ __forceinline__ bool ray_index(const GeomDev& G, int n_ang_sub, int64_t t, RayIdx& r) {
    const int64_t per_ang = (int64_t)G.n_planes * G.n_rad;
    if (t >= per_ang * n_ang_sub) return false;
    r.ia = (int)(t / per_ang);
    const int64_t rem = t - (int64_t)r.ia * per_ang;
    r.q = (int)(rem / G.n_rad);
    r.k = (int)(rem - (int64_t)r.q * G.n_rad);
    return true;
}

// out[packed] = mult? * (G x) over the angles ang0 + ia * ang_step.
__global__ void __launch_bounds__(BLOCK)
fwd_plain(GeomDev G, const float* __restrict__ x, const float* __restrict__ mult,
          float* __restrict__ out, int ang0, int ang_step, int n_ang_sub) {
    RayIdx r;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (!ray_index(G, n_ang_sub, t, r)) return;
    const int a = ang0 + r.ia * ang_step;
    float v = ray_sum<false>(G, x, a, r.q, r.k);
    if (mult) v *= mult[((int64_t)a * G.n_planes + r.q) * G.n_rad + r.k];
    out[t] = v;
}

// sigma[full] = gamma rho / (A 1) where A 1 > 0, else 0 (eq. STEPSIZE:PRECOND).
__global__ void __launch_bounds__(BLOCK)
fwd_sens(GeomDev G, const float* __restrict__ mult, float* __restrict__ sigma, float gr) {
    RayIdx r;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (!ray_index(G, G.n_ang, t, r)) return;
    const float a1 = mult[t] * ray_sum<true>(G, nullptr, r.ia, r.q, r.k);
    sigma[t] = a1 > 0.0f ? gr / a1 : 0.0f;
}

// prox^sigma_{phi*}(v) = (w + 1 - sqrt((w - 1)^2 + 4 sigma b)) / 2, w = v + sigma r, in
// the cancellation-free form obtained by rationalising the surd when w > 1.
__device__ __forceinline__ float prox_kl_dual(float v, float sigma, float b, float r) {
    const float w = __builtin_fmaf(sigma, r, v);
    const float q = w - 1.0f;
    const float c = 4.0f * sigma * b;
    const float root = __builtin_sqrtf(__builtin_fmaf(q, q, c));
    return q > 0.0f ? 1.0f - c / (2.0f * (q + root)) : 1.0f + 0.5f * (q - root);
}

// Algorithm 2 line 5 for data block i (and the dual change for line 6):
//   y+ = prox(y + S_i A_i x),  d = mult (y+ - y)  (packed),  y <- y+.
// sigma: per-bin array (preconditioned) or NULL with the scalar sig_s.
__global__ void __launch_bounds__(BLOCK)
fwd_dual(GeomDev G, const float* __restrict__ x, const float* __restrict__ mult,
         const float* __restrict__ b, const float* __restrict__ r,
         const float* __restrict__ sigma, float sig_s, float* __restrict__ y,
         float* __restrict__ d, int ang0, int ang_step, int n_ang_sub) {
    RayIdx ri;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (!ray_index(G, n_ang_sub, t, ri)) return;
    const int a = ang0 + ri.ia * ang_step;
    const int64_t j = ((int64_t)a * G.n_planes + ri.q) * G.n_rad + ri.k;
    const float sg = sigma ? sigma[j] : sig_s;
    const float m = mult[j];
    const float yo = y[j];
    float yn = yo;
    if (sg > 0.0f) {
        const float ax = m * ray_sum<false>(G, x, a, ri.q, ri.k);
        yn = prox_kl_dual(__builtin_fmaf(sg, ax, yo), sg, b[j], r[j]);
    }
    y[j] = yn;
    d[t] = m * (yn - yo);
}

// ---------------------------------------------------------------- FP64 reductions
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Deterministic block sum: fixed shuffle tree per wave, waves added in order.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double part[BLOCK / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) part[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < BLOCK / 64; ++i) s += part[i];
    return s;  // valid in thread 0
}

// Per-bin Poisson distance phi(u) = u + r - b log(u + r) - b + b log b, FP64
// (eq. LOCALDISTANCE; 0 log 0 = 0, -log 0 = inf).
__device__ __forceinline__ double phi64(double u, double b, double r) {
    const double s = u + r;
    if (s < 0.0) return INFINITY;
    if (b > 0.0) {
        if (s <= 0.0) return INFINITY;
        return s - b - b * log(s) + b * log(b);
    }
    return s;
}

// Data term of the objective: per-block FP64 partial sums of phi((A x)_j) over all bins.
__global__ void __launch_bounds__(BLOCK)
fwd_obj(GeomDev G, const float* __restrict__ x, const float* __restrict__ mult,
        const float* __restrict__ b, const float* __restrict__ r, double* __restrict__ part) {
    RayIdx ri;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double v = 0.0;
    if (ray_index(G, G.n_ang, t, ri)) {
        const float ax = mult[t] * ray_sum<false>(G, x, ri.ia, ri.q, ri.k);
        v = phi64((double)ax, (double)b[t], (double)r[t]);
    }
    const double s = block_sum(v);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Per-block partial counts of nonzero taps over the rays of the listed angles.
__global__ void __launch_bounds__(BLOCK)
fwd_count(GeomDev G, int ang0, int ang_step, int n_ang_sub, double* __restrict__ part) {
    RayIdx r;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double v = 0.0;
    if (ray_index(G, n_ang_sub, t, r)) v = ray_taps(G, ang0 + r.ia * ang_step, r.q, r.k);
    const double s = block_sum(v);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Sum of n partials in index order by one block: each thread sums a strided slice in
// order, then the fixed block tree.  out[slot] = scale * total (+ out[add_slot] if >= 0).
__global__ void __launch_bounds__(BLOCK)
reduce_final(const double* __restrict__ part, int64_t n, double* __restrict__ out, int slot,
             double scale) {
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += BLOCK) v += part[i];
    const double s = block_sum(v);
    if (threadIdx.x == 0) out[slot] = scale * s;
}

__global__ void combine_objective(double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        out[0] = out[1] + out[2];
        out[3] = 0.0;
    }
}

// ---------------------------------------------------------------- gather backprojection
// (A_i^T d) at voxel (ix, iy, iz): every ray of the listed angles whose bilinear taps
// include the voxel, with the weights of ray_sum.  d rows: d_ang0 + ia * d_step.
// MULT: each d value is multiplied by mult at the full-sinogram position of the ray.
template <bool MULT>
__device__ float voxel_gather(const GeomDev& G, const float* __restrict__ d, int d_ang0,
                              int d_step, int ang0, int ang_step, int n_ang_sub, int ix,
                              int iy, int iz, const float* __restrict__ mult = nullptr) {
    float acc = 0.0f;
    const int64_t per_ang = (int64_t)G.n_planes * G.n_rad;
    for (int ia = 0; ia < n_ang_sub; ++ia) {
        const int a = ang0 + ia * ang_step;
        const AngleDev A = G.ang[a];
        const int j = A.rowdom ? iy : ix;
        const int isec = A.rowdom ? ix : iy;
        const double jj = (double)j - A.cj;
        // candidate radial bins: u(k) in [isec - 1, isec + 1]
        const double base = __builtin_fma(A.du_dj, jj, A.cu);
        const double k_a = ((double)(isec - 1) - base) / A.du_dk + G.ck;
        const double k_b = ((double)(isec + 1) - base) / A.du_dk + G.ck;
        const int k0 = max(0, (int)__builtin_floor(fmin(k_a, k_b)) - 1);
        const int k1 = min(G.n_rad - 1, (int)__builtin_ceil(fmax(k_a, k_b)) + 1);
        const float* drow = d + (int64_t)(d_ang0 + ia * d_step) * per_ang;
        const float* mrow = MULT ? mult + (int64_t)a * per_ang : nullptr;
        for (int k = k0; k <= k1; ++k) {
            const double kk = (double)k - G.ck;
            const Sample s = split(sec_coord(A, kk, jj));
            float wx;
            if (s.i0 == isec)
                wx = 1.0f - s.fu;
            else if (s.i0 + 1 == isec)
                wx = s.fu;
            else
                continue;
            float accr = 0.0f;
            for (int g = 0; g < G.n_seg; ++g) {
                const SegAngleDev S = G.sa[a * G.n_seg + g];
                const Sample sz = split(ax_offset(S, kk, jj));
                const float fz = sz.fu;
                const int p0 = iz - G.seg_off[g] - sz.i0;  // voxel is the lower tap
                const int p1 = p0 - 1;                      // voxel is the upper tap
                const int ng = G.seg_planes[g];
                const int64_t o = (int64_t)G.seg_base[g] * G.n_rad + k;
                const float* dr = drow + o;
                float sg = 0.0f;
                if ((unsigned)p0 < (unsigned)ng) {
                    float v = dr[(int64_t)p0 * G.n_rad];
                    if (MULT) v *= mrow[o + (int64_t)p0 * G.n_rad];
                    sg += (1.0f - fz) * v;
                }
                if ((unsigned)p1 < (unsigned)ng) {
                    float v = dr[(int64_t)p1 * G.n_rad];
                    if (MULT) v *= mrow[o + (int64_t)p1 * G.n_rad];
                    sg += fz * v;
                }
                accr += S.L * sg;
            }
            acc += wx * accr;
        }
    }
    return acc;
}

__device__ __forceinline__ bool voxel_index(const GeomDev& G, int64_t t, int& ix, int& iy,
                                            int& iz) {
    const int64_t nxy = (int64_t)G.nx * G.ny;
    if (t >= nxy * G.nz) return false;
    iz = (int)(t / nxy);
    const int64_t rem = t - (int64_t)iz * nxy;
    iy = (int)(rem / G.nx);
    ix = (int)(rem - (int64_t)iy * G.nx);
    return true;
}

// out = G^T d, or G^T diag(mult) d when mult is given (full sinogram of factors).
__global__ void __launch_bounds__(BLOCK)
bwd_plain(GeomDev G, const float* __restrict__ d, int d_ang0, int d_step, int ang0,
          int ang_step, int n_ang_sub, float* __restrict__ out, const float* __restrict__ mult) {
    int ix, iy, iz;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (!voxel_index(G, t, ix, iy, iz)) return;
    out[t] = mult ? voxel_gather<true>(G, d, d_ang0, d_step, ang0, ang_step, n_ang_sub, ix, iy,
                                       iz, mult)
                  : voxel_gather<false>(G, d, d_ang0, d_step, ang0, ang_step, n_ang_sub, ix, iy,
                                        iz);
}

// T = min(T, scale / (A_i^T 1)) where A_i^T 1 > 0 (eq. STEPSIZE:PRECOND, Theorem 1).
__global__ void __launch_bounds__(BLOCK)
bwd_sens_min(GeomDev G, const float* __restrict__ mult, int ang0, int ang_step,
             int n_ang_sub, float scale, float* __restrict__ T) {
    int ix, iy, iz;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (!voxel_index(G, t, ix, iy, iz)) return;
    const float s = voxel_gather<false>(G, mult, ang0, ang_step, ang0, ang_step, n_ang_sub, ix, iy, iz);
    if (s > 0.0f) T[t] = fminf(T[t], scale / s);
}

// Algorithm 2 lines 6-8 for a data block, fused with line 3 of the next iteration:
//   dz = A_i^T d;  z += dz;  x = max(x - T (z + dz / p_i), 0).
__global__ void __launch_bounds__(BLOCK)
bwd_iter(GeomDev G, const float* __restrict__ d, int ang0, int ang_step, int n_ang_sub,
         float inv_p, float* __restrict__ z, float* __restrict__ x, const float* __restrict__ T) {
    int ix, iy, iz;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (!voxel_index(G, t, ix, iy, iz)) return;
    const float dz = voxel_gather<false>(G, d, 0, 1, ang0, ang_step, n_ang_sub, ix, iy, iz);
    const float zn = z[t] + dz;
    z[t] = zn;
    const float zbar = __builtin_fmaf(dz, inv_p, zn);
    x[t] = fmaxf(x[t] - T[t] * zbar, 0.0f);
}

// ---------------------------------------------------------------- TV / dTV prior block
struct PriorArgs {
    int nx, ny, nz;
    float sigma;  // scalar dual step of the prior block
    float alpha;  // ball radius
    float inv_p;
    float gamma_d;
    int dtv;
};

__device__ __forceinline__ float ld(const float* a, int64_t i) { return a[i]; }

// Dual update of the prior block at voxel c: q = P_alpha(y(c) + sigma A_n x (c)); returns
// dy = q - y(c) (for dTV the D-weighted change D dy, i.e. the input of grad^T).
__device__ __forceinline__ void prior_dual_at(const PriorArgs& P, const float* __restrict__ x,
                                              const float* __restrict__ y,
                                              const float* __restrict__ xi, int cx, int cy,
                                              int cz, float q[3], float dy[3]) {
    const int64_t nxy = (int64_t)P.nx * P.ny;
    const int64_t nv = nxy * P.nz;
    const int64_t c = (int64_t)cz * nxy + (int64_t)cy * P.nx + cx;
    const float xc = ld(x, c);
    float g0 = cx < P.nx - 1 ? ld(x, c + 1) - xc : 0.0f;
    float g1 = cy < P.ny - 1 ? ld(x, c + P.nx) - xc : 0.0f;
    float g2 = cz < P.nz - 1 ? ld(x, c + nxy) - xc : 0.0f;
    float x0 = 0.f, x1 = 0.f, x2 = 0.f;
    if (P.dtv) {
        x0 = ld(xi, c);
        x1 = ld(xi, c + nv);
        x2 = ld(xi, c + 2 * nv);
        const float dot = x0 * g0 + x1 * g1 + x2 * g2;
        g0 -= P.gamma_d * dot * x0;
        g1 -= P.gamma_d * dot * x1;
        g2 -= P.gamma_d * dot * x2;
    }
    const float y0 = ld(y, c), y1 = ld(y, c + nv), y2 = ld(y, c + 2 * nv);
    q[0] = __builtin_fmaf(P.sigma, g0, y0);
    q[1] = __builtin_fmaf(P.sigma, g1, y1);
    q[2] = __builtin_fmaf(P.sigma, g2, y2);
    const float nrm = __builtin_sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    if (nrm > P.alpha) {
        const float sc = P.alpha / nrm;
        q[0] *= sc;
        q[1] *= sc;
        q[2] *= sc;
    }
    dy[0] = q[0] - y0;
    dy[1] = q[1] - y1;
    dy[2] = q[2] - y2;
    if (P.dtv) {
        const float dot = x0 * dy[0] + x1 * dy[1] + x2 * dy[2];
        dy[0] -= P.gamma_d * dot * x0;
        dy[1] -= P.gamma_d * dot * x1;
        dy[2] -= P.gamma_d * dot * x2;
    }
}

// Algorithm 2 lines 5-8 for the prior block, fused with line 3 of the next iteration.
// The dual changes of the three backward neighbours are recomputed locally (they enter
// grad^T at this voxel), so x and y are read from one buffer and written to the other.
__global__ void __launch_bounds__(BLOCK)
tv_iter(PriorArgs P, const float* __restrict__ x_in, float* __restrict__ x_out,
        const float* __restrict__ y_in, float* __restrict__ y_out, float* __restrict__ z,
        const float* __restrict__ T, const float* __restrict__ xi) {
    const int64_t nxy = (int64_t)P.nx * P.ny;
    const int64_t nv = nxy * P.nz;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t >= nv) return;
    const int cz = (int)(t / nxy);
    const int cy = (int)((t - (int64_t)cz * nxy) / P.nx);
    const int cx = (int)(t - (int64_t)cz * nxy - (int64_t)cy * P.nx);
    float q[3], dy[3], qn[3], dn[3];
    prior_dual_at(P, x_in, y_in, xi, cx, cy, cz, q, dy);
    // grad^T p (v) = sum_d [v_d > 0] p_d(v - e_d) - [v_d < N_d - 1] p_d(v)
    float dz = 0.0f;
    if (cx < P.nx - 1) dz -= dy[0];
    if (cy < P.ny - 1) dz -= dy[1];
    if (cz < P.nz - 1) dz -= dy[2];
    if (cx > 0) {
        prior_dual_at(P, x_in, y_in, xi, cx - 1, cy, cz, qn, dn);
        dz += dn[0];
    }
    if (cy > 0) {
        prior_dual_at(P, x_in, y_in, xi, cx, cy - 1, cz, qn, dn);
        dz += dn[1];
    }
    if (cz > 0) {
        prior_dual_at(P, x_in, y_in, xi, cx, cy, cz - 1, qn, dn);
        dz += dn[2];
    }
    y_out[t] = q[0];
    y_out[t + nv] = q[1];
    y_out[t + 2 * nv] = q[2];
    const float zn = z[t] + dz;
    z[t] = zn;
    const float zbar = __builtin_fmaf(dz, P.inv_p, zn);
    x_out[t] = fmaxf(x_in[t] - T[t] * zbar, 0.0f);
}

// Prior term alpha sum_v |(A_n x)_v|_2 (FP64 partials; 0 when use_grad is 0) plus the
// non-negativity indicator: a negative voxel makes the term +inf.
__global__ void __launch_bounds__(BLOCK)
tv_obj(PriorArgs P, const float* __restrict__ x, const float* __restrict__ xi,
       double* __restrict__ part, int use_grad) {
    const int64_t nxy = (int64_t)P.nx * P.ny;
    const int64_t nv = nxy * P.nz;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double v = 0.0;
    if (t < nv) {
        const int cz = (int)(t / nxy);
        const int cy = (int)((t - (int64_t)cz * nxy) / P.nx);
        const int cx = (int)(t - (int64_t)cz * nxy - (int64_t)cy * P.nx);
        const double xc = x[t];
        double g0 = cx < P.nx - 1 ? (double)x[t + 1] - xc : 0.0;
        double g1 = cy < P.ny - 1 ? (double)x[t + P.nx] - xc : 0.0;
        double g2 = cz < P.nz - 1 ? (double)x[t + nxy] - xc : 0.0;
        if (P.dtv) {
            const double x0 = xi[t], x1 = xi[t + nv], x2 = xi[t + 2 * nv];
            const double dot = x0 * g0 + x1 * g1 + x2 * g2;
            g0 -= P.gamma_d * dot * x0;
            g1 -= P.gamma_d * dot * x1;
            g2 -= P.gamma_d * dot * x2;
        }
        v = use_grad ? (double)P.alpha * sqrt(g0 * g0 + g1 * g1 + g2 * g2) : 0.0;
        if (xc < 0.0) v = INFINITY;
    }
    const double s = block_sum(v);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// xi = grad s / sqrt(|grad s|^2 + eta^2) for the dTV side image s.
__global__ void __launch_bounds__(BLOCK)
dtv_field(int nx, int ny, int nz, const float* __restrict__ s, float eta, float* __restrict__ xi) {
    const int64_t nxy = (int64_t)nx * ny;
    const int64_t nv = nxy * nz;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t >= nv) return;
    const int cz = (int)(t / nxy);
    const int cy = (int)((t - (int64_t)cz * nxy) / nx);
    const int cx = (int)(t - (int64_t)cz * nxy - (int64_t)cy * nx);
    const double sc = s[t];
    const double g0 = cx < nx - 1 ? (double)s[t + 1] - sc : 0.0;
    const double g1 = cy < ny - 1 ? (double)s[t + nx] - sc : 0.0;
    const double g2 = cz < nz - 1 ? (double)s[t + nxy] - sc : 0.0;
    const double nrm = sqrt(g0 * g0 + g1 * g1 + g2 * g2 + (double)eta * eta);
    xi[t] = (float)(g0 / nrm);
    xi[t + nv] = (float)(g1 / nrm);
    xi[t + 2 * nv] = (float)(g2 / nrm);
}

// ---------------------------------------------------------------- small helpers
__global__ void fill_f32(float* __restrict__ a, int64_t n, float v) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t < n) a[t] = v;
}

__global__ void clip_nonneg(float* __restrict__ a, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t < n) a[t] = fmaxf(a[t], 0.0f);
}

// T = min(T, t_prior); +inf (no block constrains the voxel) -> 0.
__global__ void finalize_T(float* __restrict__ T, int64_t n, float t_prior) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t >= n) return;
    float v = fminf(T[t], t_prior);
    T[t] = isinf(v) ? 0.0f : v;
}

// Domain check partials: counts of bins with b < 0 or r < 0 or mult <= 0 or non-finite
// values (slot 0), and of bins whose objective term is infinite for every image:
// b > 0, r = 0 and no voxel reaches the bin (sigma = 0 there) (slot 1).
__global__ void __launch_bounds__(BLOCK)
domain_check(const float* __restrict__ b, const float* __restrict__ r,
             const float* __restrict__ mult, const float* __restrict__ a1, int64_t n,
             double* __restrict__ part, int64_t nblocks) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double bad = 0.0, inf = 0.0;
    if (t < n) {
        const float bb = b[t], rr = r[t], mm = mult[t];
        if (!(bb >= 0.0f) || !(rr >= 0.0f) || !(mm > 0.0f) || isinf(bb) || isinf(rr) ||
            isinf(mm))
            bad = 1.0;
        if (bb > 0.0f && rr == 0.0f && !(a1[t] > 0.0f)) inf = 1.0;
    }
    const double s0 = block_sum(bad);
    __syncthreads();
    const double s1 = block_sum(inf);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0;
        part[nblocks + blockIdx.x] = s1;
    }
}

// Sum of squares of an image in FP64 (power iteration), and scaling by 1/sqrt(norm2).
__global__ void __launch_bounds__(BLOCK)
sumsq(const float* __restrict__ a, int64_t n, double* __restrict__ part) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double v = 0.0;
    if (t < n) v = (double)a[t] * (double)a[t];
    const double s = block_sum(v);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void scale_by_rnorm(const float* __restrict__ in, float* __restrict__ out, int64_t n,
                               const double* __restrict__ norm2) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t < n) {
        const double s = norm2[0];
        out[t] = s > 0.0 ? (float)((double)in[t] / sqrt(s)) : 0.0f;
    }
}

}  // namespace spdhg
