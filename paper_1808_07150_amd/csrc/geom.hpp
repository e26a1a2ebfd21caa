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
// length L_g = v_prim / |cos or sin| * sqrt(1 + tau_g^2).  The coordinates are evaluated
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
    int32_t n_rad, n_ang, n_seg, n_planes;
    double ck;  // (n_rad - 1) / 2
    int32_t seg_planes[SPDHG_DEV_MAX_SEG];
    int32_t seg_base[SPDHG_DEV_MAX_SEG];  // first sinogram plane of the segment
    int32_t seg_off[SPDHG_DEV_MAX_SEG];   // image plane of the first plane: (nz - 1 - pitch (N_g - 1)) / 2
    int32_t seg_pitch[SPDHG_DEV_MAX_SEG]; // image planes between consecutive planes (1 or 2)
    const AngleDev* ang;                  // [n_ang]
    const SegAngleDev* sa;                // [n_ang][n_seg]
    const int32_t* plane_seg;             // [n_planes] segment of each plane
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

// Axial offset (in voxels) of the ray of radial bin kk at primary index jj.
__device__ __forceinline__ double ax_offset(const SegAngleDev& S, double kk, double jj) {
    return __builtin_fma(S.ez_dj, jj, S.ez_dk * kk);
}
