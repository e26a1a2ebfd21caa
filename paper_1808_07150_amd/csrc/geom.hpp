// Device-side geometry of the ray-driven Joseph projector.
//
// A ray (angle a, plane q = plane p of segment g, radial bin k) is sampled at every
// "primary" index j (image rows when 4a <= n_ang or 4a >= 3 n_ang, else columns).  At a
// sample it needs two continuous indices, both affine in the centred integers
// kk = k - (n_rad-1)/2 and jj = j - (n_prim-1)/2:
//
//   u = du_dj * jj + (du_dk * kk + cu)       secondary in-plane index (fma, fma)
//   e = ez_dj[g] * jj + ez_dk[g] * kk        axial offset in voxels from the plane centre
//   z index = off_g + pitch_g p + e,  off_g = (nz - 1 - pitch_g (N_g - 1)) / 2
//
// Bilinear interpolation in (u, z) with zero padding; each sample carries the 3-D path
// length L_g = v_prim / |cos or sin| * sqrt(1 + tau_g^2).
//
// Scanner model (tables, NULL when off): radial bin k sits at the centred coordinate
// kpos[k] = s_k / d_rad instead of k - (n_rad-1)/2 (non-arc-corrected bins, s_k = R sin(..)),
// and the slope of every segment at s_k is scaled by kobl[k] = R / sqrt(R^2 - s_k^2), so
// both axial coefficients take that factor and the step length the factor
// kL[g][k] = sqrt(1 + tau_g^2 kobl^2) / sqrt(1 + tau_g^2).  u and e stay affine in the
// centred radial coordinate, so every formula below reads kk = kappa(G, k).  The coordinates are evaluated
// in FP64 from FP64 coefficients (an FP32 index near 300 would carry ~2e-5 absolute
// error) and only the interpolation fractions are rounded to FP32.  The forward walk and
// the gather backprojector call the same inline functions below with the same integer
// inputs, so the interpolation weights they use are bit-identical: the backprojector is
// the transpose of the forward projector up to the order of the FP32 sums.
#pragma once

#include <stdint.h>

#define SPDHG_DEV_MAX_SEG 128

struct AngleDev {
    double du_dk;  // secondary index per radial bin
    double du_dj;  // secondary index per primary index
    double cu;     // (n_sec - 1) / 2
    double cj;     // (n_prim - 1) / 2
    int32_t rowdom;  // 1: primary = rows (y), secondary = columns (x)
    int32_t n_prim;
    int32_t n_sec;
    int32_t pad;
};

struct SegAngleDev {  // per (angle, segment)
    double ez_dj;
    double ez_dk;
    float L;
    float pad[3];
};

struct GeomDev {
    int32_t nx, ny, nz;
    int32_t n_rad, n_ang, n_seg, n_planes;  // n_planes: the projector's (ray) planes
    int32_t n_dplanes;  // planes of a data (sinogram) row: n_planes, or the span-compressed count
    int32_t dstride;    // data elements between consecutive planes of a segment (1; 2 compressed)
    double ck;          // (n_rad - 1) / 2
    double krho;        // non-arc-corrected bins: R / d_rad (0: equal steps)
    int32_t seg_planes[SPDHG_DEV_MAX_SEG];
    int32_t seg_base[SPDHG_DEV_MAX_SEG];  // first projector plane of the segment
    int32_t seg_off[SPDHG_DEV_MAX_SEG];   // image plane of the first plane: (nz - 1 - pitch (N_g - 1)) / 2
    int32_t seg_pitch[SPDHG_DEV_MAX_SEG]; // image planes between consecutive planes (1 or 2)
    int32_t seg_dbase[SPDHG_DEV_MAX_SEG]; // data element of the segment's plane 0 in a data row
    const AngleDev* ang;                  // [n_ang]
    const SegAngleDev* sa;                // [n_ang][n_seg]
    const int32_t* plane_seg;             // [n_planes] segment of each plane
    const double* kpos;                   // [n_rad] centred radial coordinate (NULL: k - ck)
    const double* kobl;                   // [n_rad] slope factor (NULL: 1)
    const float* kL;                      // [n_seg][n_rad] step-length factor (NULL: 1)
    const int32_t* cstart;                // [n_dplanes + 1] span compression: the ring-pair
    const int32_t* clist;                 // planes clist[cstart[q] ..] of data plane q (NULL: none)
};

struct Sample {
    int32_t i0;  // lower secondary index
    float fu;    // weight of i0 + 1 (i0 gets 1 - fu)
};

// Secondary in-plane coordinate of radial bin kk at primary index jj (canonical order).
__device__ __forceinline__ double sec_coord(const AngleDev& A, double kk, double jj) {
    return __builtin_fma(A.du_dj, jj, __builtin_fma(A.du_dk, kk, A.cu));
}

// Integer cell and FP32 fraction of a continuous index.
__device__ __forceinline__ Sample split(double u) {
    const double f0 = __builtin_floor(u);
    Sample s;
    s.i0 = (int32_t)f0;
    s.fu = (float)(u - f0);
    return s;
}

// Centred radial coordinate of bin k.  SCAN = false: the caller guarantees that there are
// no scanner tables (kpos, kobl, kL NULL), so the lookups compile away.
template <bool SCAN = true>
__device__ __forceinline__ double kappa(const GeomDev& G, int k) {
    if (SCAN && G.kpos) return G.kpos[k];
    return (double)k - G.ck;
}

// Continuous radial bin of the centred coordinate kk (inverse of kappa; for ray ranges).
template <bool SCAN = true>
__device__ __forceinline__ double bin_of(const GeomDev& G, double kk) {
    if (SCAN && G.krho > 0.0) return G.ck + G.krho * asin(fmin(fmax(kk / G.krho, -1.0), 1.0));
    return kk + G.ck;
}

// Axial coefficients and step length of the rays of segment g, angle a, radial bin k
// (centred coordinate kk): axial offset fma(ezj, jj, ezk) voxels at primary index jj.
struct SegRay {
    double ezj, ezk;
    float L;
};

template <bool SCAN = true>
__device__ __forceinline__ SegRay seg_ray(const GeomDev& G, int a, int g, int k, double kk) {
    const SegAngleDev S = G.sa[a * G.n_seg + g];
    SegRay r;
    if (SCAN && G.kobl) {
        const double f = G.kobl[k];
        r.ezj = S.ez_dj * f;
        r.ezk = (S.ez_dk * f) * kk;
    } else {
        r.ezj = S.ez_dj;
        r.ezk = S.ez_dk * kk;
    }
    r.L = (SCAN && G.kL) ? S.L * G.kL[g * G.n_rad + k] : S.L;
    return r;
}
