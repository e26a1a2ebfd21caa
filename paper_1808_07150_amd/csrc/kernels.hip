// HIP kernels of the SPDHG subset step for gfx950 (wave64).
//
// Internal layouts (the caller's layouts are converted at the boundary):
//   image     z-fastest [y][x][z]:  voxel (ix, iy, iz) at (iy * nx + ix) * nz + iz
//   sinogram  [angle][radial][plane]: bin (a, q, k) at (a * n_rad + k) * n_planes + q
// In these layouts every stream of the hot loop is contiguous across the 64 lanes of a
// wavefront for both angle classes (row- and column-sampled rays).
//
//   fwd_wave   forward projection, one workgroup of 1, 2, 4 or 8 wavefronts per (angle,
//              radial bin), each walking its share of the primary steps: at every step
//              the lanes form the in-plane interpolated axial column
//              G(z) = (1 - fu) x[j][i0][z] + fu x[j][i0 + 1][z] in LDS, then each ray of
//              the bin (all planes of all segments) adds its axial interpolation of G.
//              Epilogues: plain output, preconditioner sigma, KL-dual prox (the dual
//              step of Algorithm 2), FP64 data term of the objective.
//   fwd_bundle the same with the planes of a bin split over 2 or 4 wavefronts that
//              share each step's axial column (an autotuner candidate).
//   bwd_strip  gather backprojection for 32 <= nz <= 127: one wavefront per strip of 10
//              voxel columns and angle class, rays' tap tables in LDS, lanes along z
//              reading the dual change contiguously, accumulators in registers.
//   bwd_col    gather backprojection, one workgroup per group of voxel columns: the
//              interpolation coordinates of every candidate ray are computed once per
//              column and angle (FP64, shared through LDS), lanes run along z and read
//              the dual change d[angle][k][plane] contiguously.  No atomics.  Epilogues:
//              plain output, running minimum for T, primal epilogue (the z updates, extrapolation
//              and the next primal step).
//   tv_wave    TV / dTV prior block (dual ascent, l2-ball projection, adjoint, epilogue),
//              one wavefront per 64-voxel run of a column marching along y (nz >= 32);
//   tv_iter    the same on column tiles of one workgroup (thin volumes).
//   tgv1_wave / tgv2_wave (tgv1_iter / tgv2_iter on tiles): the two TGV prior blocks.
//   reductions deterministic FP64 block partials + ordered final sum.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "geom.hpp"

#define BLOCK 256

namespace spdhg {

// ---------------------------------------------------------------- helpers
// Blocks are dispatched round-robin over the 8 XCDs; map them so that consecutive
// logical blocks (neighbouring radial bins / voxel columns, which read overlapping data)
// run on the same XCD and share its L2.  Bijective on [0, nb).
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
    const int per = nb >> 3;
    if (bid >= (per << 3)) return bid;
    return (bid & 7) * per + (bid >> 3);
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Deterministic block sum: fixed shuffle tree per wave, waves added in order.
template <int NT>
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double part[NT / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) part[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) s += part[i];
    __syncthreads();
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

// prox^sigma_{phi*}(v) = (w + 1 - sqrt((w - 1)^2 + 4 sigma b)) / 2, w = v + sigma r
// (Section 2.2), rationalised so that no branch subtracts nearly equal numbers: with
// root = sqrt((w - 1)^2 + 4 sigma b),
//   w > 1:   1 - 2 sigma b / (w - 1 + root)        (the result is close to 1)
//   w <= 1:  2 (w - sigma b) / (w + 1 + root)      (denominator >= 2; the printed form
//            loses the result's low bits to 1 + ... when it is small, as in most bins)
__device__ __forceinline__ float prox_kl_dual(float v, float sigma, float b, float r) {
    const float w = __builtin_fmaf(sigma, r, v);
    const float q = w - 1.0f;
    const float sb = sigma * b;
    const float root = __builtin_sqrtf(__builtin_fmaf(q, q, 4.0f * sb));
    return q > 0.0f ? 1.0f - (2.0f * sb) / (q + root) : (2.0f * (w - sb)) / (w + 1.0f + root);
}

// Primary-index range [j0, j1) outside which the ray's in-plane taps are all outside the
// image (conservative by two samples; the samples themselves test every tap).
__device__ __forceinline__ void sec_range(const AngleDev& A, double u0, int& j0, int& j1) {
    double lo = -1e30, hi = 1e30;
    if (A.du_dj != 0.0) {
        const double t0 = (-1.0 - u0) / A.du_dj, t1 = ((double)A.n_sec - u0) / A.du_dj;
        lo = fmin(t0, t1);
        hi = fmax(t0, t1);
    } else if (!(u0 > -1.0 && u0 < (double)A.n_sec)) {
        j0 = j1 = 0;
        return;
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

// ---------------------------------------------------------------- forward projection
enum FwdMode { F_PLAIN_QK = 0, F_POWER = 1, F_SENS = 2, F_DUAL = 3, F_OBJ = 4, F_EM = 5 };

// Row layout of the dual change read by the backprojectors: per (angle of the list,
// radial bin) the n_dplanes values of the data bins; projector segment g's plane p at
// element seg_dbase[g] + dstride p (without span compression: the ray bundle's planes,
// segment g at seg_base[g] ..).
__device__ __forceinline__ int64_t dual_row(const GeomDev& G, int ia, int k) {
    return ((int64_t)ia * G.n_rad + k) * G.n_dplanes;
}

struct FwdArgs {
    GeomDev G;
    const float* x;  // z-fastest image (unused for F_SENS)
    int ang0, ang_step, n_ang_sub;
    int pad, gsize;  // zero padding of the axial column, padded column length
    const float* mult;   // F_PLAIN_QK: caller layout, full; others: internal, full
    float* out;          // F_PLAIN_QK: packed output; F_SENS: sigma; F_POWER: padded
    const float* b;      // internal, full
    const float* r;      // internal, full
    const float* sigma;  // internal, full, or NULL (scalar sig_s)
    float sig_s;
    float* y;            // internal, full
    float* d;            // F_DUAL: dual change, padded layout
    double* part;        // F_OBJ partials (one per block)
    float gr;            // F_SENS: gamma * rho
    int split;           // host only: wavefronts per ray bundle (0: chosen from the size)
    int interleave;      // host only: 1 keeps the interleaved rays where RUN instances apply
    float* raw;          // span compression: ray sums [angle of the chunk][k][ray plane]
    int raw_kq;          // 1: the walk writes its ray sums times L to raw (no epilogue)
    int ia0;             // index of the launch's first angle in the output lists
    int raw_angles;      // host only: angles the raw buffer holds
};

// Epilogue of one data bin (a, k, data plane q) with geometric projection v; ia indexes
// the launch's list of angles.
template <int MODE>
__device__ __forceinline__ void fwd_bin(const FwdArgs& P, int a, int ia, int k, int q, float v,
                                        double& obj) {
    const GeomDev& G = P.G;
    const int64_t full = ((int64_t)a * G.n_rad + k) * G.n_dplanes + q;
    if (MODE == F_PLAIN_QK) {
        const float m = P.mult ? P.mult[((int64_t)a * G.n_dplanes + q) * G.n_rad + k] : 1.0f;
        P.out[((int64_t)ia * G.n_dplanes + q) * G.n_rad + k] = v * m;
    } else if (MODE == F_POWER) {
        // A_i^T A_i needs mult (G x) times mult again: write mult^2 G x
        const float m = P.mult[full];
        P.out[dual_row(G, ia, k) + q] = m * m * v;
    } else if (MODE == F_SENS) {
        const float a1 = P.mult[full] * v;
        P.out[full] = a1 > 0.0f ? P.gr / a1 : 0.0f;
    } else if (MODE == F_DUAL) {
        const float sg = P.sigma ? P.sigma[full] : P.sig_s;
        const float m = P.mult[full];
        const float yo = P.y[full];
        float yn = yo;
        if (sg > 0.0f) yn = prox_kl_dual(__builtin_fmaf(sg, m * v, yo), sg, P.b[full], P.r[full]);
        P.y[full] = yn;
        P.d[dual_row(G, ia, k) + q] = m * (yn - yo);
    } else if (MODE == F_OBJ) {
        obj += phi64((double)(P.mult[full] * v), (double)P.b[full], (double)P.r[full]);
    } else if (MODE == F_EM) {
        // EM-type update (eq. MLEM / OSEM): the ratio b / (A x + r) of the bin, times mult
        // (the row factor of the backprojection A^T = G^T diag(mult)); 0 where b = 0
        const float m = P.mult[full];
        const float b = P.b[full];
        P.d[dual_row(G, ia, k) + q] = b > 0.0f ? m * (b / __builtin_fmaf(m, v, P.r[full])) : 0.0f;
    }
}

// Per-ray epilogue of the forward walk (sum acc of ray (a, k, plane q) in segment g): the
// data bin's epilogue, or with span compression (raw_kq) the ray's sum times its step
// length into the raw rows, which fwd_compress adds up per data bin.
template <int MODE>
__device__ __forceinline__ void fwd_epilogue(const FwdArgs& P, int a, int ia, int k, int q, int g,
                                             float acc, double& obj) {
    const GeomDev& G = P.G;
    const float L = G.kL ? G.sa[a * G.n_seg + g].L * G.kL[g * G.n_rad + k] : G.sa[a * G.n_seg + g].L;
    const float v = acc * L;
    if (P.raw_kq) {
        P.raw[((int64_t)ia * G.n_rad + k) * G.n_planes + q] = v;
        return;
    }
    fwd_bin<MODE>(P, a, ia, k, q, v, obj);
}

// The F_DUAL epilogue of fwd_bin for N rays of a lane (no raw rows): every table and
// data load is issued before the first store (the stores to y and d may alias the next
// ray's loads, so ray by ray each waited for its own loads).  A slot with q[e] < 0 loads
// plane 0 of segment 0 and stores nothing.
template <int N>
__device__ __forceinline__ void fwd_dual_batch(const FwdArgs& P, int a, int ia, int k,
                                               const int (&q)[N], const int (&g)[N],
                                               const float (&acc)[N]) {
    const GeomDev& G = P.G;
    float v[N], sg[N], m[N], yo[N], bb[N], rr[N];
    int64_t full[N];
#pragma unroll
    for (int e = 0; e < N; ++e) {
        const int qc = q[e] < 0 ? 0 : q[e];
        const int gc = q[e] < 0 ? 0 : g[e];
        const float L = G.kL ? G.sa[a * G.n_seg + gc].L * G.kL[gc * G.n_rad + k]
                             : G.sa[a * G.n_seg + gc].L;
        v[e] = acc[e] * L;
        full[e] = ((int64_t)a * G.n_rad + k) * G.n_dplanes + qc;
        sg[e] = P.sigma ? P.sigma[full[e]] : P.sig_s;
        m[e] = P.mult[full[e]];
        yo[e] = P.y[full[e]];
        bb[e] = P.b[full[e]];
        rr[e] = P.r[full[e]];
    }
#pragma unroll
    for (int e = 0; e < N; ++e) {
        if (q[e] < 0) continue;
        float yn = yo[e];
        if (sg[e] > 0.0f)
            yn = prox_kl_dual(__builtin_fmaf(sg[e], m[e] * v[e], yo[e]), sg[e], bb[e], rr[e]);
        P.y[full[e]] = yn;
        P.d[dual_row(G, ia, k) + q[e]] = m[e] * (yn - yo[e]);
    }
}

// Span compression (eq. of the forward model with the scanner's data planes): every data
// bin of the chunk's angles is the sum of its ring-pair rays (clist order, fixed), then
// the mode's epilogue.  One block per (angle of the chunk, radial bin), so the objective's
// partial of bin row (ia0 + ia, k) lands where the walks put theirs.
template <int MODE>
__global__ void __launch_bounds__(256) fwd_compress(FwdArgs P) {
    const GeomDev& G = P.G;
    const int bid = blockIdx.x;
    const int ia = bid / G.n_rad;
    const int k = bid - ia * G.n_rad;
    const int a = P.ang0 + ia * P.ang_step;
    const float* raw = P.raw + (int64_t)bid * G.n_planes;
    double obj = 0.0;
    for (int q = threadIdx.x; q < G.n_dplanes; q += 256) {
        float v = 0.0f;
        for (int i = G.cstart[q]; i < G.cstart[q + 1]; ++i) v += raw[G.clist[i]];
        fwd_bin<MODE>(P, a, P.ia0 + ia, k, q, v, obj);
    }
    if (MODE == F_OBJ) {
        const double t = block_sum<256>(obj);
        if (threadIdx.x == 0) P.part[(int64_t)(P.ia0 + ia) * G.n_rad + k] = t;
    }
}

// One workgroup of NW wavefronts per (angle, radial bin); RPL = rays per lane (planes / 64,
// rounded up to a power of two, or 14 for the iteration and the objective).  Wavefront w walks the w-th of NW consecutive parts of the primary steps
// with its own LDS buffers; the partial ray sums are added in a fixed order by wavefront 0
// (several wavefronts per ray bundle give small subsets enough parallelism).
// The iteration's projection (F_DUAL) with up to 16 rays per lane is held to five waves
// per SIMD (at most 96 VGPRs, no spills): room for the reads of FWD_RG rays in flight
// together.  The objective's projection (F_OBJ), which the autotuner times in its place,
// is held the same way.
constexpr int FWD_RG = 8;  // rays per lane whose LDS reads are issued together
// RUN instances (pitch-1 geometries whose segments split into at most 64 runs of FWD_RUN
// consecutive planes: 61 for the 837 planes of span 11): lane L walks the rays of run L,
// which lie in one segment on consecutive image planes, so per step a lane reads one
// segment entry and the FWD_RUN + 1 column values its rays' two taps cover (in pairs),
// instead of an entry and a pair per ray.  Each ray's arithmetic and the order of the
// partial sums are those of the interleaved instances, so the sums are bitwise the same;
// they pass through LDS into plane order before the epilogue.  An odd run length keeps
// the lanes of a segment, FWD_RUN planes apart, on distinct LDS banks (a power-of-two
// length puts every other lane on the same bank).
constexpr int FWD_RUN = 15;

// Per step and segment: byte offset of the axial cell and the axial fraction (one 8-byte
// LDS read per ray and step).
struct __align__(8) SegStep {
    int c4;
    float fz;
};

template <int RPL, int MODE, int NW, bool RUN = false>
__global__ void __launch_bounds__(64 * NW, ((MODE == F_DUAL || MODE == F_OBJ) && RPL <= 16) ? 5 : 1)
fwd_wave(FwdArgs P) {
    static_assert(!RUN || RPL == FWD_RUN, "a run is FWD_RUN rays");
    extern __shared__ float smem[];
    const GeomDev& G = P.G;
    const int ns = G.n_seg;
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    // each wavefront's LDS region (floats; even, so the 8-byte entries stay aligned)
    const int wstride = max(2 * P.gsize + 8 * ns, 64);
    float* Gb = smem + w * wstride;                        // [gsize] axial column (+ gsize spare)
    SegStep* segt = (SegStep*)(Gb + 2 * P.gsize);          // [ns] this step's axial samples
    double* segk = (double*)(Gb + 2 * P.gsize + 4 * ns);   // [ns] ez_dk * kk of the segment
    double* segj = segk + ns;                              // [ns] ez_dj of the segment
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int ia = bid / G.n_rad;
    const int k = bid - ia * G.n_rad;
    const int a = P.ang0 + ia * P.ang_step;
    const AngleDev A = G.ang[a];
    const double kk = kappa(G, k);
    const int nz = G.nz;
    const int64_t s_prim = A.rowdom ? G.nx : 1;
    const int64_t s_sec = A.rowdom ? 1 : G.nx;

    // Per ray of the lane: LDS byte offsets of its segment's entry and of its padded axial
    // base in the column.  A plane beyond the last takes plane 0's (in range; its sum is
    // never written), so every step handles all rows without per-lane branches.
    int toff[RPL], boff[RPL];
    float acc[RPL];
    int run_q0 = 0, run_n = 0;  // RUN: first plane and ray count of the lane's run
    int run_g = 0;              // RUN: the run's segment
    if (RUN) {
        // runs in segment order, FWD_RUN planes each (the last of a segment shorter); a
        // lane without a run walks segment 0's first planes and writes nothing
        int g = 0, first = 0, o = 0;
        for (int sg = 0; sg < ns; ++sg) {
            const int cnt = (G.seg_planes[sg] + FWD_RUN - 1) / FWD_RUN;
            if (lane >= first && lane < first + cnt) {
                g = sg;
                o = (lane - first) * FWD_RUN;
                run_n = min(FWD_RUN, G.seg_planes[sg] - o);
            }
            first += cnt;
        }
        run_q0 = G.seg_base[g] + o;
        run_g = g;
        toff[0] = (int)((const char*)(segt + g) - (const char*)smem);
        boff[0] = (int)((const char*)(Gb + o + G.seg_off[g] + P.pad) - (const char*)smem);
#pragma unroll
        for (int r = 0; r < RPL; ++r) acc[r] = 0.0f;
    } else {
        const int g0 = G.plane_seg[0];
        const int base0 = G.seg_off[g0] - G.seg_pitch[g0] * G.seg_base[g0] + P.pad;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int q = lane + 64 * r;
            acc[r] = 0.0f;
            int g = g0, base = base0;
            if (q < G.n_planes) {
                g = G.plane_seg[q];
                base = G.seg_pitch[g] * (q - G.seg_base[g]) + G.seg_off[g] + P.pad;
            }
            toff[r] = (int)((const char*)(segt + g) - (const char*)smem);
            boff[r] = (int)((const char*)(Gb + base) - (const char*)smem);
        }
    }
    for (int i = lane; i < P.gsize; i += 64) Gb[i] = 0.0f;
    // the axial offset of segment g at step j is fma(ezj, jj, ezk) (seg_ray):
    // its two step-independent parts are read once, so the step loop loads nothing from
    // global memory but the image columns (only lane g % 64 touches entry g)
    for (int sg = lane; sg < ns; sg += 64) {
        const SegRay S = seg_ray(G, a, sg, k, kk);
        segk[sg] = S.ezk;
        segj[sg] = S.ezj;
    }
    // RUN: the run's own segment coefficients in registers (its axial sample per step is
    // then computed by the lane, with the expression the table uses)
    double run_ezj = 0.0, run_ezk = 0.0;
    if (RUN) {
        __builtin_amdgcn_wave_barrier();
        run_ezk = segk[run_g];
        run_ezj = segj[run_g];
    }
    int j0, j1;
    sec_range(A, __builtin_fma(A.du_dk, kk, A.cu), j0, j1);
    if (NW > 1 && j0 < j1) {  // this wavefront's part of the steps
        const int n = j1 - j0;
        j1 = j0 + (n * (w + 1)) / NW;
        j0 = j0 + (n * w) / NW;
    }
    // A wavefront's LDS accesses execute in issue order, so one axial column and one
    // segment table serve every step: the next step's writes cannot overtake this step's
    // reads, and code-motion barriers keep the compiler to that order.  The image columns
    // of step j + 1 are in flight while the rays consume step j (loads through a
    // range-checked buffer resource: an offset of 1 GiB or more reads zero, which covers
    // samples outside the image and z beyond nz without branches).  Deeper prefetch costs
    // more registers than it hides latency on gfx950.
    constexpr int NZL = 2;  // z values per lane (nz <= 128)
    constexpr int OUT = 1 << 30;
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
        (void*)P.x, (short)0, (int)(P.G.nx * (int64_t)P.G.ny * nz * 4), 0x00020000);
    int zoff[NZL];
#pragma unroll
    for (int u = 0; u < NZL; ++u) zoff[u] = lane + 64 * u < nz ? (lane + 64 * u) * 4 : OUT;
    float v0[NZL], v1[NZL];
    Sample sm;
    auto issue = [&](int j) {
        const Sample q = split(sec_coord(A, kk, (double)j - A.cj));
        sm = q;
        if (MODE == F_SENS) return;
        const bool ok0 = (unsigned)q.i0 < (unsigned)A.n_sec;
        const bool ok1 = (unsigned)(q.i0 + 1) < (unsigned)A.n_sec;
        const int c0 = ok0 ? (int)(((int64_t)j * s_prim + (int64_t)q.i0 * s_sec) * nz * 4) : OUT;
        const int c1 = ok1 ? (int)(((int64_t)j * s_prim + (int64_t)(q.i0 + 1) * s_sec) * nz * 4) : OUT;
#pragma unroll
        for (int u = 0; u < NZL; ++u) {
            v0[u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(xr, c0 + zoff[u], 0, 0));
            v1[u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(xr, c1 + zoff[u], 0, 0));
        }
    };
    if (j0 < j1) issue(j0);
    float* Gc = Gb + P.pad;
    const char* lds = (const char*)smem;
    for (int j = j0; j < j1; ++j) {
        const double jj = (double)j - A.cj;
        const Sample s = sm;
        const float w0 = 1.0f - s.fu, w1 = s.fu;
        if (MODE == F_SENS) {
            const bool ok0 = (unsigned)s.i0 < (unsigned)A.n_sec;
            const bool ok1 = (unsigned)(s.i0 + 1) < (unsigned)A.n_sec;
            const float v = (ok0 ? w0 : 0.0f) + (ok1 ? w1 : 0.0f);
            for (int iz = lane; iz < nz; iz += 64) Gc[iz] = v;
        } else {
#pragma unroll
            for (int u = 0; u < NZL; ++u) {
                const int iz = lane + 64 * u;
                if (iz < nz) Gc[iz] = __builtin_fmaf(w1, v1[u], w0 * v0[u]);
            }
        }
        if (j + 1 < j1) issue(j + 1);
        if (RUN) {
            // the run's axial sample, then its rays r read taps r and r + 1 of one window
            // of the column
            const Sample sz = split(__builtin_fma(run_ezj, jj, run_ezk));
            SegStep e;
            e.c4 = sz.i0 * 4;
            e.fz = sz.fu;
            __builtin_amdgcn_wave_barrier();
            const float* gp = (const float*)(lds + boff[0] + e.c4);
            float v[RPL + 1];
#pragma unroll
            for (int r = 0; r <= RPL; ++r) v[r] = gp[r];
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                acc[r] = __builtin_fmaf(1.0f - e.fz, v[r], acc[r]);
                acc[r] = __builtin_fmaf(e.fz, v[r + 1], acc[r]);
            }
            __builtin_amdgcn_wave_barrier();
            continue;
        }
        for (int sg = lane; sg < ns; sg += 64) {
            const Sample sz = split(__builtin_fma(segj[sg], jj, segk[sg]));
            SegStep e;
            e.c4 = sz.i0 * 4;
            e.fz = sz.fu;
            segt[sg] = e;
        }
        __builtin_amdgcn_wave_barrier();
        // rays in groups of RG: the table reads of a group, then its column reads, then
        // its sums, so a group costs two LDS round trips instead of two per ray
        constexpr int RG = RPL < FWD_RG ? RPL : FWD_RG;
#pragma unroll
        for (int r0 = 0; r0 < RPL; r0 += RG) {
            SegStep e[RG];
            float ga[RG], gb[RG];
#pragma unroll
            for (int i = 0; i < RG; ++i)
                if (r0 + i < RPL) e[i] = *(const SegStep*)(lds + toff[r0 + i]);
#pragma unroll
            for (int i = 0; i < RG; ++i) {
                if (r0 + i < RPL) {
                    const float* gp = (const float*)(lds + boff[r0 + i] + e[i].c4);
                    ga[i] = gp[0];
                    gb[i] = gp[1];
                }
            }
#pragma unroll
            for (int i = 0; i < RG; ++i) {
                if (r0 + i < RPL) {
                    acc[r0 + i] = __builtin_fmaf(1.0f - e[i].fz, ga[i], acc[r0 + i]);
                    acc[r0 + i] = __builtin_fmaf(e[i].fz, gb[i], acc[r0 + i]);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (NW > 1) {
        // partial ray sums pass through each wavefront's own LDS region (its axial columns
        // are no longer needed), `per` rays at a time; wavefront 0 adds them in wavefront
        // order, so the sum is the same for any number of passes
        const int per = min(RPL, wstride / 64);
#pragma unroll 1
        for (int r0 = 0; r0 < RPL; r0 += per) {
            __syncthreads();  // the walks (first pass) or wavefront 0's reads are done
            if (w > 0) {
#pragma unroll
                for (int r = 0; r < RPL; ++r)
                    if (r >= r0 && r < r0 + per) Gb[(r - r0) * 64 + lane] = acc[r];
            }
            __syncthreads();
            if (w == 0) {
#pragma unroll 1
                for (int v = 1; v < NW; ++v) {
                    const float* pv = smem + v * wstride;
#pragma unroll
                    for (int r = 0; r < RPL; ++r)
                        if (r >= r0 && r < r0 + per) acc[r] += pv[(r - r0) * 64 + lane];
                }
            }
        }
        if (w > 0) return;
    }

    // epilogues
    double obj = 0.0;
    if (RUN) {
        // the run's sums into plane order, then plane q = lane + 64 r per lane; the walk's
        // LDS reads are done (a wavefront's LDS accesses execute in issue order)
        float* T = smem;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int r = 0; r < RPL; ++r)
            if (r < run_n) T[run_q0 + r] = acc[r];
        __builtin_amdgcn_wave_barrier();
        if (MODE == F_DUAL && !P.raw_kq) {
            // five planes per lane at a time (60 VGPRs, eight waves; seven needed 78)
            constexpr int EB = 5;
            const int nq = G.n_planes;
            for (int q0 = 0; q0 < nq; q0 += 64 * EB) {
                int qs[EB], gs[EB];
                float vs[EB];
#pragma unroll
                for (int e = 0; e < EB; ++e) {
                    const int q = q0 + lane + 64 * e;
                    qs[e] = q < nq ? q : -1;
                    gs[e] = q < nq ? G.plane_seg[q] : 0;
                    vs[e] = q < nq ? T[q] : 0.0f;
                }
                fwd_dual_batch<EB>(P, a, ia, k, qs, gs, vs);
            }
        } else {
            for (int q = lane; q < G.n_planes; q += 64)
                fwd_epilogue<MODE>(P, a, ia, k, q, G.plane_seg[q], T[q], obj);
        }
    } else if (MODE == F_DUAL && !P.raw_kq) {
        // four rays per lane at a time through fwd_dual_batch
        constexpr int EB = RPL < 4 ? RPL : 4;
#pragma unroll
        for (int r0 = 0; r0 < RPL; r0 += EB) {
            int qs[EB], gs[EB];
            float vs[EB];
#pragma unroll
            for (int e = 0; e < EB; ++e) {
                const int q = lane + 64 * (r0 + e);
                const bool ok = r0 + e < RPL && q < G.n_planes;
                qs[e] = ok ? q : -1;
                gs[e] = ok ? G.plane_seg[q] : 0;
                vs[e] = r0 + e < RPL ? acc[r0 + e < RPL ? r0 + e : 0] : 0.0f;
            }
            fwd_dual_batch<EB>(P, a, ia, k, qs, gs, vs);
        }
    } else {
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int q = lane + 64 * r;
            if (q < G.n_planes) fwd_epilogue<MODE>(P, a, ia, k, q, G.plane_seg[q], acc[r], obj);
        }
    }
    if (MODE == F_OBJ && !P.raw_kq) {  // raw rows: fwd_compress writes the partials
        obj = wave_sum(obj);
        if (lane == 0) P.part[bid] = obj;
    }
}

// Plane-split variant: PS wavefronts per (angle, radial bin) share every step's axial
// column (built cooperatively, double-buffered in LDS, one workgroup barrier per step)
// and each walks the whole ray bundle for its own contiguous share of the planes.  Fewer
// rays per lane than fwd_wave, so fewer registers and more resident wavefronts.
template <int RPL, int MODE, int PS>
__global__ void __launch_bounds__(64 * PS) fwd_bundle(FwdArgs P) {
    extern __shared__ float smem[];
    __shared__ double wsum[PS];
    const GeomDev& G = P.G;
    const int ns = G.n_seg;
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63;
    float* Gb = smem;                        // [2][gsize] axial columns
    int* segc = (int*)(Gb + 2 * P.gsize);    // [2][ns] axial cell offsets
    float* segf = (float*)(segc + 2 * ns);   // [2][ns] axial fractions
    double* segk = (double*)(segf + 2 * ns); // [ns] ez_dk * kk of the segment
    double* segj = segk + ns;                // [ns] ez_dj of the segment
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int ia = bid / G.n_rad;
    const int k = bid - ia * G.n_rad;
    const int a = P.ang0 + ia * P.ang_step;
    const AngleDev A = G.ang[a];
    const double kk = kappa(G, k);
    const int nz = G.nz;
    const int64_t s_prim = A.rowdom ? G.nx : 1;
    const int64_t s_sec = A.rowdom ? 1 : G.nx;
    const int q0 = w * 64 * RPL;  // first plane of this wavefront

    int pinfo[RPL];  // (padded axial base of the plane) << 7 | segment
    float acc[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int q = q0 + lane + 64 * r;
        acc[r] = 0.0f;
        pinfo[r] = 0;
        if (q < G.n_planes) {
            const int g = G.plane_seg[q];
            pinfo[r] = ((G.seg_pitch[g] * (q - G.seg_base[g]) + G.seg_off[g] + P.pad) << 7) | g;
        }
    }
    for (int i = tid; i < 2 * P.gsize; i += 64 * PS) Gb[i] = 0.0f;
    // step-independent parts of the axial offset (seg_ray; only one thread touches entry g)
    for (int sg = tid; sg < ns; sg += 64 * PS) {
        const SegRay S = seg_ray(G, a, sg, k, kk);
        segk[sg] = S.ezk;
        segj[sg] = S.ezj;
    }
    int j0, j1;
    sec_range(A, __builtin_fma(A.du_dk, kk, A.cu), j0, j1);
    // image columns through a range-checked buffer resource (see fwd_wave)
    constexpr int ZPT = PS >= 2 ? 1 : 2;  // z values per thread (nz <= 128)
    constexpr int OUT = 1 << 30;
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
        (void*)P.x, (short)0, (int)(P.G.nx * (int64_t)P.G.ny * nz * 4), 0x00020000);
    int zoff[ZPT];
#pragma unroll
    for (int u = 0; u < ZPT; ++u) {
        const int iz = tid + 64 * PS * u;
        zoff[u] = iz < nz ? iz * 4 : OUT;
    }
    float v0[ZPT], v1[ZPT];
    Sample s{0, 0.0f};
    auto issue = [&](int j) {
        s = split(sec_coord(A, kk, (double)j - A.cj));
        if (MODE == F_SENS) return;
        const bool ok0 = (unsigned)s.i0 < (unsigned)A.n_sec;
        const bool ok1 = (unsigned)(s.i0 + 1) < (unsigned)A.n_sec;
        const int c0 = ok0 ? (int)(((int64_t)j * s_prim + (int64_t)s.i0 * s_sec) * nz * 4) : OUT;
        const int c1 = ok1 ? (int)(((int64_t)j * s_prim + (int64_t)(s.i0 + 1) * s_sec) * nz * 4) : OUT;
#pragma unroll
        for (int u = 0; u < ZPT; ++u) {
            v0[u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(xr, c0 + zoff[u], 0, 0));
            v1[u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(xr, c1 + zoff[u], 0, 0));
        }
    };
    if (j0 < j1) issue(j0);
    int buf = 0;
    for (int j = j0; j < j1; ++j) {
        const double jj = (double)j - A.cj;
        float* Gc = Gb + buf * P.gsize + P.pad;
        const float w0 = 1.0f - s.fu, w1 = s.fu;
        if (MODE == F_SENS) {
            const bool ok0 = (unsigned)s.i0 < (unsigned)A.n_sec;
            const bool ok1 = (unsigned)(s.i0 + 1) < (unsigned)A.n_sec;
            const float v = (ok0 ? w0 : 0.0f) + (ok1 ? w1 : 0.0f);
            for (int iz = tid; iz < nz; iz += 64 * PS) Gc[iz] = v;
        } else {
#pragma unroll
            for (int u = 0; u < ZPT; ++u) {
                const int iz = tid + 64 * PS * u;
                if (iz < nz) Gc[iz] = __builtin_fmaf(w1, v1[u], w0 * v0[u]);
            }
        }
        if (j + 1 < j1) issue(j + 1);
        for (int sg = tid; sg < ns; sg += 64 * PS) {
            const Sample sz = split(__builtin_fma(segj[sg], jj, segk[sg]));
            segc[buf * ns + sg] = sz.i0;
            segf[buf * ns + sg] = sz.fu;
        }
        // the other buffer was last read before this barrier's predecessor
        __syncthreads();
        const float* Gr = Gb + buf * P.gsize;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            if (q0 + lane + 64 * r < G.n_planes) {
                const int g = pinfo[r] & 127;
                const int idx = (pinfo[r] >> 7) + segc[buf * ns + g];
                const float fz = segf[buf * ns + g];
                acc[r] = __builtin_fmaf(1.0f - fz, Gr[idx], acc[r]);
                acc[r] = __builtin_fmaf(fz, Gr[idx + 1], acc[r]);
            }
        }
        buf ^= 1;
    }
    double obj = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int q = q0 + lane + 64 * r;
        if (q < G.n_planes) fwd_epilogue<MODE>(P, a, ia, k, q, pinfo[r] & 127, acc[r], obj);
    }
    if (MODE == F_OBJ && !P.raw_kq) {  // raw rows: fwd_compress writes the partials
        obj = wave_sum(obj);
        if (lane == 0) wsum[w] = obj;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int v = 0; v < PS; ++v) t += wsum[v];
            P.part[bid] = t;
        }
    }
}

// ---------------------------------------------------------------- gather backprojection
enum BwdMode { B_PLAIN = 0, B_SENS = 1, B_ITER = 2, B_PARTIAL = 3, B_ACCUM = 4, B_EM = 5,
               B_PAIR = 6 };
#define BWD_THREADS 128
#define BWD_KC 4  // candidate radial bins per column and angle

struct BwdArgs {
    GeomDev G;
    const float* d;  // dual change / sinogram rows of the listed angles (see dual_row)
    int ang0, ang_step, n_ang_sub;
    int cols;        // per-column kernel: voxel columns per block
    float* out;      // B_PLAIN / B_PARTIAL: z-fastest image; B_ACCUM: added to
    float scale;     // B_SENS: rho p_i / gamma
    float* T;
    float inv_p;
    float* z;
    float* x;
    float* zlo;      // B_PAIR: low parts of z and x (see primal_pair)
    float* xlo;
};

// Per (candidate ray, segment): voxel z reads planes p = z + off (weight wa) and p - 1
// (weight wb) of the segment, zero outside 0 .. N_g - 1; the weights carry the segment's
// step length.
struct TapCoef {
    int off;
    float wa, wb;
};

template <bool SCAN = true>
__device__ __forceinline__ TapCoef tap_coef(const GeomDev& G, int a, int g, int k, double kk,
                                            double jj) {
    const SegRay S = seg_ray<SCAN>(G, a, g, k, kk);
    const Sample sz = split(__builtin_fma(S.ezj, jj, S.ezk));
    TapCoef t;
    t.off = -(G.seg_off[g] + sz.i0);
    t.wa = S.L * (1.0f - sz.fu);
    t.wb = S.L * sz.fu;
    return t;
}

// Per-lane bounds (per-column gather).  Pitch 1: voxel z takes plane
// p = z + off (weight wa) and p - 1 (wb).  Pitch 2 (a segment on every other image plane):
// with u = z + off, plane p sits at image plane off_g + 2p + i0 (weight wa) and reaches the
// next one with weight wb, so voxel z takes one plane, u / 2 with wa if u is even, else
// (u - 1) / 2 with wb (u >> 1 in both cases).  Plane pp is data element pp * ds (ds = 2:
// a span-compressed data row).
__device__ __forceinline__ float tap_sum_masked(const float* __restrict__ seg, int n, int pitch,
                                                int ds, const TapCoef& t, int z, float h) {
    const int p = z + t.off;
    if (pitch == 2) {
        const int pp = p >> 1;
        if ((unsigned)pp < (unsigned)n) h = __builtin_fmaf((p & 1) ? t.wb : t.wa, seg[pp * ds], h);
        return h;
    }
    if ((unsigned)p < (unsigned)n) h = __builtin_fmaf(t.wa, seg[p], h);
    if ((unsigned)(p - 1) < (unsigned)n) h = __builtin_fmaf(t.wb, seg[p - 1], h);
    return h;
}

// Buffer resource over segment g of a dual-change row (raw, byte offsets, range checked):
// its planes at elements 0, ds, .., (N_g - 1) ds (ds = dstride).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t seg_rsrc(const GeomDev& G, const float* row,
                                                           int g) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)(row + (uint32_t)G.seg_dbase[g]), (short)0,
                                             ((G.seg_planes[g] - 1) * G.dstride + 1) * 4,
                                             0x00020000);
}

// The primal part of Algorithm 2 (z += dz; x = max(x - T (z + dz / p_i), 0)) on a state
// held as FP32 pairs, x = xh + xl and z = zh + zl with |lo| at most half an ulp of hi,
// evaluated in FP64 on the sums: a change smaller than half an ulp of the FP32 value
// accumulates in the low part instead of being rounded away (with many subsets each
// iteration moves x and z by a small fraction of their size).  The projector reads xh.
__device__ __forceinline__ void primal_pair(float& xh, float& xl, float& zh, float& zl,
                                            float T, float dz, float inv_p) {
    const double z = ((double)zh + (double)zl) + (double)dz;
    zh = (float)z;
    zl = (float)(z - (double)zh);
    const double zbar = __builtin_fma((double)dz, (double)inv_p, z);
    double x = ((double)xh + (double)xl) - (double)T * zbar;
    x = x > 0.0 ? x : 0.0;
    xh = (float)x;
    xl = (float)(x - (double)xh);
}

__device__ __forceinline__ void bwd_epilogue(const BwdArgs& P, int MODE, int64_t t, float dz) {
    if (MODE == B_PLAIN || MODE == B_PARTIAL) {
        P.out[t] = dz;
    } else if (MODE == B_ACCUM) {
        P.out[t] += dz;
    } else if (MODE == B_SENS) {
        if (dz > 0.0f) P.T[t] = fminf(P.T[t], P.scale / dz);
    } else if (MODE == B_EM) {
        // eq. OSEM: x = x / (A_i^T 1) * A_i^T (b / (A_i x + r)); T holds 1 / (A_i^T 1) (0 off
        // the subset's support)
        P.x[t] = P.x[t] * (dz * P.T[t]);
    } else if (MODE == B_PAIR) {
        float xh = P.x[t], xl = P.xlo[t], zh = P.z[t], zl = P.zlo[t];
        primal_pair(xh, xl, zh, zl, P.T[t], dz, P.inv_p);
        P.z[t] = zh;
        P.zlo[t] = zl;
        P.x[t] = xh;
        P.xlo[t] = xl;
    } else {
        // Algorithm 2: dual and z updates, extrapolation and the next iteration's primal step:
        // z += dz;  x = max(x - T (z + dz / p_i), 0)
        const float zn = P.z[t] + dz;
        P.z[t] = zn;
        const float zbar = __builtin_fmaf(dz, P.inv_p, zn);
        P.x[t] = fmaxf(P.x[t] - P.T[t] * zbar, 0.0f);
    }
}

// A candidate ray of a column for one angle: radial bin and in-plane weight (0: none).
struct ColCoord {
    int k;
    float wx;
};

// Per-column gather (any nz <= 256 and radial spacing >= half a voxel): one block per
// group of voxel columns; the candidate rays of each column and their tap coefficients
// are computed once per column and angle (FP64) and shared through LDS; lanes run
// along z.
template <int MODE>
__global__ void __launch_bounds__(BWD_THREADS) bwd_col(BwdArgs P, const float* __restrict__ partial) {
    const GeomDev& G = P.G;
    const int ns = G.n_seg;
    const int nz = G.nz;
    extern __shared__ float smem[];
    const int cols = P.cols;
    ColCoord* cc = (ColCoord*)smem;                 // [cols][KC]
    TapCoef* tc = (TapCoef*)(cc + cols * BWD_KC);   // [cols][KC][ns]
    const int ncol = G.nx * G.ny;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int col0 = blk * cols;
    const int zchunk = nz < BWD_THREADS ? nz : BWD_THREADS;
    const int cl = threadIdx.x / zchunk;
    const int z0 = threadIdx.x - cl * zchunk;
    const int col = col0 + cl;
    const bool active = cl < cols && col < ncol;
    const int nzz = (nz + zchunk - 1) / zchunk;  // z values per thread (<= 2, nz <= 256)
    float acc[2] = {0.f, 0.f};

    for (int ia = 0; ia < P.n_ang_sub; ++ia) {
        const int a = P.ang0 + ia * P.ang_step;
        const AngleDev A = G.ang[a];
        __syncthreads();  // the previous angle's coordinates are no longer read
        for (int t = threadIdx.x; t < cols * BWD_KC; t += BWD_THREADS) {
            const int c = t / BWD_KC, kc = t - c * BWD_KC;
            const int cq = col0 + c;
            ColCoord o{0, 0.0f};
            if (cq < ncol) {
                const int qy = cq / G.nx, qx = cq - qy * G.nx;
                const int j = A.rowdom ? qy : qx;
                const int isec = A.rowdom ? qx : qy;
                const double jj = (double)j - A.cj;
                const double base = __builtin_fma(A.du_dj, jj, A.cu);
                const double ka = bin_of(G, ((double)(isec - 1) - base) / A.du_dk);
                const double kb = bin_of(G, ((double)(isec + 1) - base) / A.du_dk);
                const int klo = max(0, (int)__builtin_floor(fmin(ka, kb)) - 1);
                const int khi = min(G.n_rad - 1, (int)__builtin_ceil(fmax(ka, kb)) + 1);
                int found = 0;
                for (int k = klo; k <= khi; ++k) {
                    const Sample sm = split(sec_coord(A, kappa(G, k), jj));
                    float w = -1.0f;
                    if (sm.i0 == isec)
                        w = 1.0f - sm.fu;
                    else if (sm.i0 + 1 == isec)
                        w = sm.fu;
                    if (w > 0.0f) {
                        if (found == kc) {
                            o.k = k;
                            o.wx = w;
                        }
                        ++found;
                    }
                }
            }
            cc[t] = o;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < cols * BWD_KC * ns; t += BWD_THREADS) {
            const int c = t / (BWD_KC * ns);
            const int rem = t - c * BWD_KC * ns;
            const int kc = rem / ns, g = rem - kc * ns;
            const int cq = col0 + c;
            const ColCoord o = cc[c * BWD_KC + kc];
            TapCoef v{0, 0.0f, 0.0f};
            if (cq < ncol && o.wx != 0.0f) {
                const int qy = cq / G.nx, qx = cq - qy * G.nx;
                const int j = A.rowdom ? qy : qx;
                v = tap_coef(G, a, g, o.k, kappa(G, o.k), (double)j - A.cj);
            }
            tc[t] = v;
        }
        __syncthreads();
        if (!active) continue;
        for (int kc = 0; kc < BWD_KC; ++kc) {
            const ColCoord o = cc[cl * BWD_KC + kc];
            if (o.wx == 0.0f) continue;
            const float* dk = P.d + dual_row(G, ia, o.k);
            const TapCoef* tk = tc + (cl * BWD_KC + kc) * ns;
            for (int zz = 0; zz < nzz; ++zz) {
                const int iz = z0 + zz * zchunk;
                if (iz >= nz) break;
                float h = 0.0f;
                for (int g = 0; g < ns; ++g)
                    h = tap_sum_masked(dk + G.seg_dbase[g], G.seg_planes[g], G.seg_pitch[g],
                                       G.dstride, tk[g], iz, h);
                acc[zz] = __builtin_fmaf(o.wx, h, acc[zz]);
            }
        }
    }
    if (!active) return;
    for (int zz = 0; zz < nzz; ++zz) {
        const int iz = z0 + zz * zchunk;
        if (iz >= nz) break;
        const int64_t t = (int64_t)col * nz + iz;
        bwd_epilogue(P, MODE, t, acc[zz] + (partial ? partial[t] : 0.0f));
    }
}

// ---------------------------------------------------------------- strip gather backprojection
// One wavefront per strip of BS_W voxel columns that lie along the secondary axis at one
// primary index j, for the angles of one sampling class (rows or columns), nz <= 127
// (lane holds z = lane and z = lane + 64 of every strip column).  Per angle:
//   1. the radial bins of the rays touching the strip (consecutive, at most KR), each
//      ray's in-plane cell / fraction and per segment its tap coefficients (FP64, the
//      same inline functions as the forward walk), into LDS; then, per in-plane cell
//      c = -1 .. BS_W - 1 of the strip, the range of rays whose cell it is (the cell is
//      monotonic in the radial bin, so the range is contiguous);
//   2. per cell (unrolled) and ray of its range (a wave-uniform loop) the axial gather
//      h(z) = sum_g wa_g d(z + off_g) + wb_g d(z + off_g - 1), lanes along z reading the
//      dual change contiguously (each plane is loaded once: the second tap comes from
//      the next lane by a wavefront shift), added with the in-plane weights 1 - fu and
//      fu to the strip columns c and c + 1.
// Every ray's axial gather is computed once per strip and angle and serves both columns
// it touches; the accumulators stay in registers with static indices.  The row-sampled
// angles of a subset write a partial image that the column-sampled launch adds before its
// epilogue.  Deterministic, no atomics.  The workgroup is one wavefront, whose LDS
// accesses execute in order: code-motion barriers separate the phases.
#define BS_W 10
#define SEG_CHUNK 11  // segments whose tap tables the strip gather holds at a time

// N consecutive segments of one ray: all 2N loads, then all sums (in segment order).
// PITCH 1 (consecutive planes): lanes hold z = lane - 1 and z = lane + 63 and load
// c(z) = d(z + off) of each segment.  With h(z) = sum_g wa_g d(z + off_g) + wb_g d(z - 1 +
// off_g) = A(z) + B(z - 1), A = sum wa c and B = sum wb c, every lane uses only its own
// loaded value; the one-voxel shift of B is taken once per ray (ray_sum).  PITCH 2 (planes
// on every other image plane): la, lb = lane, lane + 64; each voxel takes one plane of
// the segment, u >> 1 with u = z + off, weighted wa (u even) or wb (u odd), so
// neighbouring voxels share planes (with span-compressed rows one load covers both
// halves, below); s[0] and s[2] are the two halves' sums.
template <int N, int PITCH, int DS = 1>
__device__ __forceinline__ void strip_batch(const GeomDev& G, const float* dk, const TapCoef* tk,
                                            int g, int la, int lb, float (&s)[4]) {
    float v[N][2];
    if constexpr (PITCH == 1) {
#pragma unroll
        for (int u = 0; u < N; ++u) {
            const __amdgpu_buffer_rsrc_t rs = seg_rsrc(G, dk, g + u);
            const int off = tk[g + u].off;
            v[u][0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (la + off) * 4, 0, 0));
            v[u][1] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (lb + off) * 4, 0, 0));
        }
#pragma unroll
        for (int u = 0; u < N; ++u) {
            const TapCoef& t = tk[g + u];
            s[0] = __builtin_fmaf(t.wa, v[u][0], s[0]);
            s[1] = __builtin_fmaf(t.wb, v[u][0], s[1]);
            s[2] = __builtin_fmaf(t.wa, v[u][1], s[2]);
            s[3] = __builtin_fmaf(t.wb, v[u][1], s[3]);
        }
    } else {
        // DS = 1, the generic instance, tests the stride at run time (dense rows take two
        // loads, compressed ones the permutes below); DS = 2 is specialised to compressed
        // rows.  (Measured: the generic instance runs dense rows 9% faster than an instance
        // compiled for dense rows alone, 6.5 against 7.15 ms for span 1 at mMR size, a
        // code-generation effect; the specialised one runs compressed rows 7% faster.)
        if (DS == 1 && G.dstride == 1) {
#pragma unroll
            for (int u = 0; u < N; ++u) {
                const __amdgpu_buffer_rsrc_t rs = seg_rsrc(G, dk, g + u);
                const int off = tk[g + u].off;
                v[u][0] = __uint_as_float(
                    __builtin_amdgcn_raw_buffer_load_b32(rs, ((la + off) >> 1) << 2, 0, 0));
                v[u][1] = __uint_as_float(
                    __builtin_amdgcn_raw_buffer_load_b32(rs, ((lb + off) >> 1) << 2, 0, 0));
            }
#pragma unroll
            for (int u = 0; u < N; ++u) {
                const TapCoef& t = tk[g + u];
                s[0] = __builtin_fmaf(((la + t.off) & 1) ? t.wb : t.wa, v[u][0], s[0]);
                s[2] = __builtin_fmaf(((lb + t.off) & 1) ? t.wb : t.wa, v[u][1], s[2]);
            }
            return;
        }
        // Span-compressed rows (a plane every 8 bytes): the two halves' voxels (z = la, lb)
        // take planes (z + off) >> 1, 64 consecutive planes from off >> 1, which one load
        // brings in (lane L holds plane (off >> 1) + L) where two loads spanning the same
        // 512 bytes each did before.  Voxel z = L then takes lane (L + (off & 1)) >> 1's
        // value and z = L + 64 the lane 32 above it, moved by LDS crossbar permutes (no
        // memory access; z = 127, beyond the image, takes lane 0's).  With dense rows the
        // two permutes cost more than the load they save, so those keep two loads.
        constexpr int sh = 3;  // bytes per plane: 4 dstride
        float w[N];
#pragma unroll
        for (int u = 0; u < N; ++u) {
            const __amdgpu_buffer_rsrc_t rs = seg_rsrc(G, dk, g + u);
            const int off = tk[g + u].off;
            w[u] = __uint_as_float(
                __builtin_amdgcn_raw_buffer_load_b32(rs, (la + (off >> 1)) << sh, 0, 0));
        }
#pragma unroll
        for (int u = 0; u < N; ++u) {
            const TapCoef& t = tk[g + u];
            const int src = ((la + (t.off & 1)) >> 1) << 2;
            const float v0 = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(w[u])));
            const float v1 =
                __int_as_float(__builtin_amdgcn_ds_bpermute(src + 128, __float_as_int(w[u])));
            s[0] = __builtin_fmaf(((la + t.off) & 1) ? t.wb : t.wa, v0, s[0]);
            s[2] = __builtin_fmaf(((lb + t.off) & 1) ? t.wb : t.wa, v1, s[2]);
        }
    }
}

// The axial gathers of the two halves from the sums of strip_batch.  PITCH 1: h(z) = A(z)
// + B(z - 1); B(z - 1) is the previous lane's value (wavefront shift right by one lane,
// checked on the GPU like the left shift), and for the upper half's lane 0 (z = 63) the
// lower half's lane 63 (z = 62).  The lower half's lane 0 (z = -1) is never written out.
template <int PITCH>
__device__ __forceinline__ void ray_sum(const float (&s)[4], float& h0, float& h1) {
    if constexpr (PITCH == 1) {
        const int top = __builtin_amdgcn_readlane(__float_as_int(s[1]), 63);
        const float b0 = __int_as_float(
            __builtin_amdgcn_update_dpp(0, __float_as_int(s[1]), 0x138 /* wave_shr:1 */, 0xF, 0xF, false));
        const float b1 = __int_as_float(
            __builtin_amdgcn_update_dpp(top, __float_as_int(s[3]), 0x138 /* wave_shr:1 */, 0xF, 0xF, false));
        h0 = s[0] + b0;
        h1 = s[2] + b1;
    } else {
        h0 = s[0];
        h1 = s[2];
    }
}

// NS = 11: every launch has exactly 11 segments (span 11) and no scanner tables, so the
// segment table's entries are compile-time indices the compiler keeps in scalar
// registers and the scanner model's lookups compile away; NS = 0: any count, any model.
template <int MODE, int PITCH, int NS, int DS = 1>
// Seven waves per SIMD (at most 72 VGPRs): room for the loads of a whole ray (span 11:
// 22 values) next to the 20 accumulators, so a ray costs one memory round trip.  A wave's
// time is set by the latency of its rays, so narrow strips (fewer rays per wave, more
// waves) finish sooner: at 344 x 344 the 12040 strips take 1.7 rounds of the chip's wave
// slots where 16-column strips took 1.2 rounds of longer waves.
//
// A workgroup holds wj = blockDim.x / 64 wavefronts (1 or 4), the strips of wj consecutive
// primary indices at one strip position: they read nearly the same rays, which the
// workgroup's shared L1 then serves.  Each wavefront has its own LDS tables; there is no
// workgroup barrier.
__global__ void __launch_bounds__(256, 7) bwd_strip(BwdArgs P, int KR, int rowdom,
                                                const float* __restrict__ partial) {
    const GeomDev& G = P.G;
    const int ns = G.n_seg;
    const int nz = G.nz;
    const int sc = NS ? NS : min(ns, SEG_CHUNK);  // the table's entries per ray (host: bwd_plan)
    extern __shared__ float smem[];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    float* wsm = smem + wv * (2 * KR + 2 * (BS_W + 1) + 3 * KR * sc);
    int* ri0 = (int*)wsm;                     // [KR] in-plane cell relative to the strip
    float* rfu = (float*)(ri0 + KR);          // [KR] in-plane fraction
    int* cfirst = (int*)(rfu + KR);           // [BS_W + 1] first ray of cell c (index c + 1)
    int* clast = cfirst + (BS_W + 1);         // [BS_W + 1] last ray of cell c
    TapCoef* tc = (TapCoef*)(clast + (BS_W + 1));  // [KR][sc]: one chunk of segments

    const int lane = threadIdx.x & 63;
    const int wj = blockDim.x >> 6;
    const int n_sec = rowdom ? G.nx : G.ny;
    const int n_prim = rowdom ? G.ny : G.nx;
    // consecutive blocks (one XCD's share) walk along the primary axis at one strip
    // position: neighbouring strips read nearly the same rays
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int njb = (n_prim + wj - 1) / wj;
    const int sidx = blk / njb;
    const int j = (blk - sidx * njb) * wj + wv;
    if (j >= n_prim) return;
    const int s0 = sidx * BS_W;
    // the lane offsets of strip_batch (lane - 1 and lane + 63, or lane and lane + 64: the
    // z of the lane's two halves) through register copies the compiler cannot fold into an
    // immediate buffer offset (the hardware range check must see the whole offset)
    const int zl = PITCH == 1 ? lane - 1 : lane;
    int lane_a, lane_b;
    asm volatile("v_mov_b32 %0, %1" : "=v"(lane_a) : "v"(PITCH == 1 ? lane - 1 : lane));
    asm volatile("v_mov_b32 %0, %1" : "=v"(lane_b) : "v"(PITCH == 1 ? lane + 63 : lane + 64));
    float acc[BS_W][2];
#pragma unroll
    for (int c = 0; c < BS_W; ++c) acc[c][0] = acc[c][1] = 0.0f;

    for (int ia = 0; ia < P.n_ang_sub; ++ia) {
        const int a = P.ang0 + ia * P.ang_step;
        const AngleDev A = G.ang[a];
        if (A.rowdom != rowdom) continue;  // the other class has its own launch
        const double jj = (double)j - A.cj;
        // 1. rays touching the strip: u in [s0 - 1, s0 + BS_W)  (wave-uniform)
        const double base = __builtin_fma(A.du_dj, jj, A.cu);
        constexpr bool SCAN = NS == 0;
        const double ka = bin_of<SCAN>(G, ((double)(s0 - 1) - base) / A.du_dk);
        const double kb = bin_of<SCAN>(G, ((double)(s0 + BS_W) - base) / A.du_dk);
        const int klo = max(0, (int)__builtin_floor(fmin(ka, kb)) - 1);
        const int khi = min(G.n_rad - 1, (int)__builtin_ceil(fmax(ka, kb)) + 1);
        const int nr = min(max(khi - klo + 1, 0), KR);
        __builtin_amdgcn_wave_barrier();  // the previous angle's tables are consumed
        for (int kr = lane; kr < nr; kr += 64) {
            const Sample sm = split(sec_coord(A, kappa<SCAN>(G, klo + kr), jj));
            ri0[kr] = sm.i0 - s0;
            rfu[kr] = sm.fu;
        }
        if (lane <= BS_W) {
            cfirst[lane] = 0;
            clast[lane] = -1;
        }
        __builtin_amdgcn_wave_barrier();
        for (int kr = lane; kr < nr; kr += 64) {
            const int ci = ri0[kr];
            if (ci >= -1 && ci < BS_W) {
                if (kr == 0 || ri0[kr - 1] != ci) cfirst[ci + 1] = kr;
                if (kr == nr - 1 || ri0[kr + 1] != ci) clast[ci + 1] = kr;
            }
        }
        // 2. per chunk of up to SEG_CHUNK segments (all of them for span 11): the chunk's
        // tap coefficients of every ray, then the axial gather of the rays of each cell,
        // added to the cell's two columns
        for (int gc = 0; gc < ns; gc += SEG_CHUNK) {
            const int nsc = NS ? NS : min(SEG_CHUNK, ns - gc);
            __builtin_amdgcn_wave_barrier();  // the previous chunk's taps are consumed
            for (int t = lane; t < nr * nsc; t += 64) {
                const int kr = t / nsc, gl = t - kr * nsc;
                tc[kr * sc + gl] = tap_coef<SCAN>(G, a, gc + gl, klo + kr, kappa<SCAN>(G, klo + kr), jj);
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int c = -1; c < BS_W; ++c) {
                const int r0 = __builtin_amdgcn_readfirstlane(cfirst[c + 1]);
                const int r1 = __builtin_amdgcn_readfirstlane(clast[c + 1]);
                for (int kr = r0; kr <= r1; ++kr) {
                    const float fu =
                        __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(rfu[kr])));
                    const float* dk = P.d + dual_row(G, ia, klo + kr);
                    const TapCoef* tk = tc + kr * sc - gc;  // tk[g]: segment g of the chunk
                    float sm[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                    // segments in batches of 11, then 4, then 1: every load of a batch is
                    // issued before any tap is summed, so a span-11 ray costs one memory
                    // round trip (batches with per-slot guards lose this overlap)
                    if constexpr (NS == 11) {
                        strip_batch<11, PITCH, DS>(G, dk, tk, 0, lane_a, lane_b, sm);
                    } else {
                        int g = gc;
                        const int ge = gc + nsc;
                        for (; g + 11 <= ge; g += 11)
                            strip_batch<11, PITCH, DS>(G, dk, tk, g, lane_a, lane_b, sm);
                        for (; g + 4 <= ge; g += 4)
                            strip_batch<4, PITCH, DS>(G, dk, tk, g, lane_a, lane_b, sm);
                        for (; g < ge; ++g)
                            strip_batch<1, PITCH, DS>(G, dk, tk, g, lane_a, lane_b, sm);
                    }
                    float h0, h1;
                    ray_sum<PITCH>(sm, h0, h1);
                    if (c >= 0) {
                        acc[c][0] = __builtin_fmaf(1.0f - fu, h0, acc[c][0]);
                        acc[c][1] = __builtin_fmaf(1.0f - fu, h1, acc[c][1]);
                    }
                    if (c + 1 < BS_W) {
                        acc[c + 1][0] = __builtin_fmaf(fu, h0, acc[c + 1][0]);
                        acc[c + 1][1] = __builtin_fmaf(fu, h1, acc[c + 1][1]);
                    }
                }
            }
        }
    }
    if constexpr (MODE == B_ITER || MODE == B_PAIR) {
        // The epilogue of Algorithm 2 (z += dz; x = max(x - T (z + dz / p_i), 0)) in
        // batches of columns (five; two for the compensated state, whose low parts of z
        // and x add two loads per voxel): all loads of a batch (z, x, T, the partial image
        // and the low parts) are issued before its first store, so a wavefront waits for
        // one round trip per batch instead of two per voxel.  The loads go through
        // range-checked buffer resources, so lanes outside the image (z = -1, z >= nz,
        // columns past the edge) read a neighbouring voxel or zero; only lanes inside it
        // store.  The arithmetic is that of bwd_epilogue.
        constexpr bool PAIR = MODE == B_PAIR;
        const int nvb = 4 * G.nx * G.ny * nz;  // below 1 GiB
        const auto rz = __builtin_amdgcn_make_buffer_rsrc(P.z, (short)0, nvb, 0x00020000);
        const auto rx = __builtin_amdgcn_make_buffer_rsrc(P.x, (short)0, nvb, 0x00020000);
        const auto rt = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(P.T), (short)0,
                                                          nvb, 0x00020000);
        const auto rp = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(partial ? partial : P.T), (short)0, nvb, 0x00020000);
        const auto rzl = __builtin_amdgcn_make_buffer_rsrc(PAIR ? P.zlo : P.z, (short)0, nvb,
                                                           0x00020000);
        const auto rxl = __builtin_amdgcn_make_buffer_rsrc(PAIR ? P.xlo : P.x, (short)0, nvb,
                                                           0x00020000);
        constexpr int CB = PAIR ? 2 : 5;
        static_assert(BS_W % CB == 0, "whole batches of columns");
#pragma unroll
        for (int cb = 0; cb < BS_W; cb += CB) {
            float zv[CB][2], xv[CB][2], tv[CB][2], pv[CB][2], zlv[CB][2], xlv[CB][2];
            uint32_t off[CB][2];
#pragma unroll
            for (int u = 0; u < CB; ++u) {
                const int sec = s0 + cb + u;
                const int ix = rowdom ? sec : j, iy = rowdom ? j : sec;
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    off[u][hh] = 4u * (uint32_t)((iy * G.nx + ix) * nz + zl + 64 * hh);
                    zv[u][hh] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rz, off[u][hh], 0, 0));
                    xv[u][hh] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rx, off[u][hh], 0, 0));
                    tv[u][hh] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rt, off[u][hh], 0, 0));
                    pv[u][hh] = partial ? __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                                              rp, off[u][hh], 0, 0))
                                        : 0.0f;
                    zlv[u][hh] = xlv[u][hh] = 0.0f;
                    if constexpr (PAIR) {
                        zlv[u][hh] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rzl, off[u][hh], 0, 0));
                        xlv[u][hh] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rxl, off[u][hh], 0, 0));
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < CB; ++u) {
                if (s0 + cb + u >= n_sec) continue;
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    const int iz = zl + 64 * hh;
                    if (iz < 0 || iz >= nz) continue;
                    const float dz = acc[cb + u][hh] + pv[u][hh];
                    if constexpr (PAIR) {
                        float xh = xv[u][hh], xl = xlv[u][hh], zh = zv[u][hh], zlo = zlv[u][hh];
                        primal_pair(xh, xl, zh, zlo, tv[u][hh], dz, P.inv_p);
                        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(zh), rz, off[u][hh], 0, 0);
                        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(zlo), rzl, off[u][hh], 0, 0);
                        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(xh), rx, off[u][hh], 0, 0);
                        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(xl), rxl, off[u][hh], 0, 0);
                    } else {
                        const float zn = zv[u][hh] + dz;
                        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(zn), rz, off[u][hh], 0, 0);
                        const float zbar = __builtin_fmaf(dz, P.inv_p, zn);
                        __builtin_amdgcn_raw_buffer_store_b32(
                            __float_as_uint(fmaxf(xv[u][hh] - tv[u][hh] * zbar, 0.0f)), rx,
                            off[u][hh], 0, 0);
                    }
                }
            }
        }
        return;
    }
#pragma unroll
    for (int c = 0; c < BS_W; ++c) {
        const int sec = s0 + c;
        if (sec >= n_sec) continue;
        const int ix = rowdom ? sec : j, iy = rowdom ? j : sec;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int iz = zl + 64 * hh;
            if (iz < 0 || iz >= nz) continue;
            const int64_t t = ((int64_t)iy * G.nx + ix) * nz + iz;
            bwd_epilogue(P, MODE, t, acc[c][hh] + (partial ? partial[t] : 0.0f));
        }
    }
}

// Rows of a sinogram (internal full [a][k][q] layout at angles ang0 + ia * step, or the
// caller's packed [ia][q][k] layout times an optional full caller mult) -> dual_row layout.
__global__ void __launch_bounds__(BLOCK)
to_rows(GeomDev G, const float* __restrict__ src, int caller, const float* __restrict__ mult,
        int ang0, int step, int n_ang_sub, float* __restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t per = (int64_t)G.n_dplanes * G.n_rad;
    if (t >= per * n_ang_sub) return;
    const int ia = (int)(t / per);
    const int64_t rem = t - ia * per;
    if (caller) {  // packed [ia][q][k]: consecutive threads run along k
        const int q = (int)(rem / G.n_rad);
        const int k = (int)(rem - (int64_t)q * G.n_rad);
        float v = src[t];
        if (mult) v *= mult[(int64_t)(ang0 + ia * step) * per + rem];
        dst[dual_row(G, ia, k) + q] = v;
    } else {  // internal [a][k][q]: the same order
        dst[t] = src[(int64_t)(ang0 + ia * step) * per + rem];
    }
}

// ---------------------------------------------------------------- layout transposes
// caller image [z][y][x] <-> internal [y][x][z]: per row y a 2-D transpose of (z, x).
#define TT 32
__global__ void __launch_bounds__(TT * 8)
img_to_zf(int nx, int ny, int nz, const float* __restrict__ src, float* __restrict__ dst) {
    __shared__ float tile[TT][TT + 1];
    const int x0 = blockIdx.x * TT, z0 = blockIdx.y * TT, y = blockIdx.z;
    const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
    for (int i = ty; i < TT; i += 8) {
        const int z = z0 + i, x = x0 + tx;
        if (z < nz && x < nx) tile[i][tx] = src[((int64_t)z * ny + y) * nx + x];
    }
    __syncthreads();
    for (int i = ty; i < TT; i += 8) {
        const int x = x0 + i, z = z0 + tx;
        if (z < nz && x < nx) dst[((int64_t)y * nx + x) * nz + z] = tile[tx][i];
    }
}

__global__ void __launch_bounds__(TT * 8)
img_from_zf(int nx, int ny, int nz, const float* __restrict__ src, float* __restrict__ dst) {
    __shared__ float tile[TT][TT + 1];
    const int x0 = blockIdx.x * TT, z0 = blockIdx.y * TT, y = blockIdx.z;
    const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
    for (int i = ty; i < TT; i += 8) {
        const int x = x0 + i, z = z0 + tx;
        if (z < nz && x < nx) tile[i][tx] = src[((int64_t)y * nx + x) * nz + z];
    }
    __syncthreads();
    for (int i = ty; i < TT; i += 8) {
        const int z = z0 + i, x = x0 + tx;
        if (z < nz && x < nx) dst[((int64_t)z * ny + y) * nx + x] = tile[tx][i];
    }
}

// caller sinogram [a][q][k] -> internal [a][k][q] (per angle a 2-D transpose).
__global__ void __launch_bounds__(TT * 8)
sino_to_kq(int n_planes, int n_rad, const float* __restrict__ src, float* __restrict__ dst) {
    __shared__ float tile[TT][TT + 1];
    const int k0 = blockIdx.x * TT, q0 = blockIdx.y * TT;
    const int64_t a = blockIdx.z;
    const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
    const float* s = src + a * n_planes * (int64_t)n_rad;
    float* dd = dst + a * n_planes * (int64_t)n_rad;
    for (int i = ty; i < TT; i += 8) {
        const int q = q0 + i, k = k0 + tx;
        if (q < n_planes && k < n_rad) tile[i][tx] = s[(int64_t)q * n_rad + k];
    }
    __syncthreads();
    for (int i = ty; i < TT; i += 8) {
        const int k = k0 + i, q = q0 + tx;
        if (q < n_planes && k < n_rad) dd[(int64_t)k * n_planes + q] = tile[tx][i];
    }
}

// internal [a][k][q] -> caller [a][q][k]
__global__ void __launch_bounds__(TT * 8)
sino_to_qk(int n_planes, int n_rad, const float* __restrict__ src, float* __restrict__ dst) {
    __shared__ float tile[TT][TT + 1];
    const int q0 = blockIdx.x * TT, k0 = blockIdx.y * TT;
    const int64_t a = blockIdx.z;
    const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
    const float* s = src + a * n_planes * (int64_t)n_rad;
    float* dd = dst + a * n_planes * (int64_t)n_rad;
    for (int i = ty; i < TT; i += 8) {
        const int k = k0 + i, q = q0 + tx;
        if (q < n_planes && k < n_rad) tile[i][tx] = s[(int64_t)k * n_planes + q];
    }
    __syncthreads();
    for (int i = ty; i < TT; i += 8) {
        const int q = q0 + i, k = k0 + tx;
        if (q < n_planes && k < n_rad) dd[(int64_t)q * n_rad + k] = tile[tx][i];
    }
}

// ---------------------------------------------------------------- FP64 reductions
__global__ void __launch_bounds__(BLOCK)
reduce_final(const double* __restrict__ part, int64_t n, double* __restrict__ out, int slot,
             double scale) {
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += BLOCK) v += part[i];
    const double s = block_sum<BLOCK>(v);
    if (threadIdx.x == 0) out[slot] = scale * s;
}

__global__ void combine_objective(double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = out[1] + out[2];
}

// FP64 partials of the number of non-finite entries of a (the failure flag of the
// objective: an iterate stays finite unless an input or a step overflowed).
__global__ void __launch_bounds__(BLOCK)
count_nonfinite(const float* __restrict__ a, int64_t n, double* __restrict__ part) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const double v = (t < n && !isfinite(a[t])) ? 1.0 : 0.0;
    const double s = block_sum<BLOCK>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ---------------------------------------------------------------- TV / dTV prior block
struct PriorArgs {
    int nx, ny, nz;
    float sigma;  // scalar dual step of the prior block
    float alpha;  // ball radius
    float inv_p;
    float gamma_d;
    int dtv;
    int atv;      // anisotropic TV: f_n = alpha ||.||_{1,1}, dual prox = clip to [-alpha, alpha]
    // PDHG (Algorithm 1): the data blocks' backprojected dual change of the same iteration
    // (z-fastest image), added to the prior's before the z update and the primal step;
    // NULL in SPDHG, where each iteration updates one block
    const float* dz_add;
    // compensated primal (the PAIR instances): low parts of z and x (see primal_pair),
    // updated in place at the voxel's own lane
    float* zlo;
    float* xlo;
};

__device__ __forceinline__ void zf_coords(const PriorArgs& P, int64_t t, int& cx, int& cy,
                                          int& cz) {
    const int64_t col = t / P.nz;
    cz = (int)(t - col * P.nz);
    cy = (int)(col / P.nx);
    cx = (int)(col - (int64_t)cy * P.nx);
}

// Dual update of the prior block at one voxel from its forward differences g (zero on
// the high faces), duals y and (dTV) field xi: q = P_alpha(y + sigma A_n x); returns
// dy = q - y (for dTV the D-weighted change D dy, i.e. the input of grad^T).
__device__ __forceinline__ void prior_dual_vals(const PriorArgs& P, float g0, float g1, float g2,
                                                float y0, float y1, float y2, float x0, float x1,
                                                float x2, float q[3], float dy[3]) {
    if (P.dtv) {
        const float dot = x0 * g0 + x1 * g1 + x2 * g2;
        g0 -= P.gamma_d * dot * x0;
        g1 -= P.gamma_d * dot * x1;
        g2 -= P.gamma_d * dot * x2;
    }
    q[0] = __builtin_fmaf(P.sigma, g0, y0);
    q[1] = __builtin_fmaf(P.sigma, g1, y1);
    q[2] = __builtin_fmaf(P.sigma, g2, y2);
    if (P.atv) {  // conjugate of alpha ||.||_1: the box [-alpha, alpha]^3
        q[0] = fminf(fmaxf(q[0], -P.alpha), P.alpha);
        q[1] = fminf(fmaxf(q[1], -P.alpha), P.alpha);
        q[2] = fminf(fmaxf(q[2], -P.alpha), P.alpha);
    } else {  // conjugate of alpha ||.||_2 per voxel: the l2 ball of radius alpha
        const float nrm = __builtin_sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        if (nrm > P.alpha) {
            const float sc = P.alpha / nrm;
            q[0] *= sc;
            q[1] *= sc;
            q[2] *= sc;
        }
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

// The same at voxel (cx, cy, cz), loading everything it needs.
__device__ __forceinline__ void prior_dual_at(const PriorArgs& P, const float* __restrict__ x,
                                              const float* __restrict__ y,
                                              const float* __restrict__ xi, int cx, int cy,
                                              int cz, float q[3], float dy[3]) {
    const int64_t sz = 1, sx = P.nz, sy = (int64_t)P.nz * P.nx;
    const int64_t nv = sy * P.ny;
    const int64_t c = (int64_t)cy * sy + (int64_t)cx * sx + cz;
    const float xc = x[c];
    const float g0 = cx < P.nx - 1 ? x[c + sx] - xc : 0.0f;
    const float g1 = cy < P.ny - 1 ? x[c + sy] - xc : 0.0f;
    const float g2 = cz < P.nz - 1 ? x[c + sz] - xc : 0.0f;
    float x0 = 0.f, x1 = 0.f, x2 = 0.f;
    if (P.dtv) {
        x0 = xi[c];
        x1 = xi[c + nv];
        x2 = xi[c + 2 * nv];
    }
    prior_dual_vals(P, g0, g1, g2, y[c], y[c + nv], y[c + 2 * nv], x0, x1, x2, q, dy);
}

// Column tiles of the prior kernels: a workgroup holds TX x TY voxel columns of nz
// threads each (z fastest), at most 1024 threads.  Every thread computes its own dual
// update and leaves the change in LDS, where the x-, y- and z-neighbours inside the tile
// read it; only the tile's low faces recompute a neighbour's update.
struct PriorTile {
    int tx, ty;  // columns per tile along x and y
};

__device__ __forceinline__ bool tile_voxel(const PriorTile& TL, int nx, int ny, int nz, int bid,
                                           int& cx, int& cy, int& cz, int& lx, int& ly) {
    const int ntx = (nx + TL.tx - 1) / TL.tx;
    const int by = bid / ntx, bx = bid - by * ntx;
    const int l = threadIdx.x;
    const int col = l / nz;
    cz = l - col * nz;
    ly = col / TL.tx;
    lx = col - ly * TL.tx;
    cx = bx * TL.tx + lx;
    cy = by * TL.ty + ly;
    return ly < TL.ty && cx < nx && cy < ny;
}

// Algorithm 2 from the dual step to the extrapolation for the prior block, fused with the
// next iteration's primal step.
// x and y are read from one buffer and written to the other (a recomputing neighbour
// reads the old values).  PAIR: the compensated primal step (primal_pair).
template <bool PAIR>
__global__ void __launch_bounds__(1024)
tv_iter(PriorArgs P, PriorTile TL, const float* __restrict__ x_in, float* __restrict__ x_out,
        const float* __restrict__ y_in, float* __restrict__ y_out, float* __restrict__ z,
        const float* __restrict__ T, const float* __restrict__ xi) {
    __shared__ float sdq[3][1024];
    const int64_t nv = (int64_t)P.nx * P.ny * P.nz;
    int cx, cy, cz, lx, ly;
    const bool act = tile_voxel(TL, P.nx, P.ny, P.nz, xcd_remap(blockIdx.x, gridDim.x), cx, cy,
                                cz, lx, ly);
    const int l = threadIdx.x;
    float q[3], dy[3] = {0.0f, 0.0f, 0.0f};
    if (act) prior_dual_at(P, x_in, y_in, xi, cx, cy, cz, q, dy);
    sdq[0][l] = dy[0];
    sdq[1][l] = dy[1];
    sdq[2][l] = dy[2];
    __syncthreads();
    if (!act) return;
    // grad^T p (v) = sum_d [v_d > 0] p_d(v - e_d) - [v_d < N_d - 1] p_d(v)
    float dz = 0.0f;
    if (cx < P.nx - 1) dz -= dy[0];
    if (cy < P.ny - 1) dz -= dy[1];
    if (cz < P.nz - 1) dz -= dy[2];
    float qn[3], dn[3];
    if (cx > 0) {
        if (lx > 0) {
            dz += sdq[0][l - P.nz];
        } else {
            prior_dual_at(P, x_in, y_in, xi, cx - 1, cy, cz, qn, dn);
            dz += dn[0];
        }
    }
    if (cy > 0) {
        if (ly > 0) {
            dz += sdq[1][l - TL.tx * P.nz];
        } else {
            prior_dual_at(P, x_in, y_in, xi, cx, cy - 1, cz, qn, dn);
            dz += dn[1];
        }
    }
    if (cz > 0) dz += sdq[2][l - 1];
    const int64_t t = ((int64_t)cy * P.nx + cx) * P.nz + cz;
    if (P.dz_add) dz += P.dz_add[t];
    y_out[t] = q[0];
    y_out[t + nv] = q[1];
    y_out[t + 2 * nv] = q[2];
    if (PAIR) {
        float xh = x_in[t], xl = P.xlo[t], zh = z[t], zl = P.zlo[t];
        primal_pair(xh, xl, zh, zl, T[t], dz, P.inv_p);
        z[t] = zh;
        P.zlo[t] = zl;
        x_out[t] = xh;
        P.xlo[t] = xl;
        return;
    }
    const float zn = z[t] + dz;
    z[t] = zn;
    const float zbar = __builtin_fmaf(dz, P.inv_p, zn);
    x_out[t] = fmaxf(x_in[t] - T[t] * zbar, 0.0f);
}

// Buffer-resource access to an array of at most 4 GiB: a 32-bit byte offset per lane
// plus a wave-uniform one (plain vector loads and stores through the vector cache).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t vol_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                             0x00020000);
}
__device__ __forceinline__ float vol_ld(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}
__device__ __forceinline__ void vol_st(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff,
                                       float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, soff, 0);
}

// The same update with one wavefront per run of 64 consecutive voxels of a column,
// marching along y through the rows of a chunk and never waiting on another wavefront
// (no LDS, no barrier).  Runs overlap by one voxel: run h covers z = 63h .. 63h + 63, and
// its first lane (h > 0) computes the dual update below the run only to pass it on.  In
// the same way the chunk starts one row early (below y0) without writing that row.  The
// z-neighbour's change then comes from the next-lower lane, the y-neighbour's from the
// previous row (a register), and the x-neighbour's is recomputed from its inputs, which
// the neighbouring column's wavefront reads at about the same time (cache hits).  Each
// row's loads are issued before the previous row's stores.  Requires nz <= 128.

// The wavefront march's mapping: wavefront gw (XCD-ordered) takes run h = gw % nh of
// column (cx, chunk) = (gw / nh) % nx, (gw / nh) / nx; lane covers z = 63 h + lane.
struct WaveMap {
    int cx, cz, y0, y1, lane;
    bool act, own;
};

__device__ __forceinline__ bool wave_map(int nx, int ny, int nz, int ly, WaveMap& m) {
    const int nh = nz <= 64 ? 1 : (nz + 61) / 63;  // ceil((nz - 1) / 63)
    m.lane = threadIdx.x & 63;
    const int gw = xcd_remap(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int h = gw % nh;
    const int rest = gw / nh;
    m.cx = rest % nx;
    m.y0 = (rest / nx) * ly;
    if (m.y0 >= ny) return false;
    m.y1 = min(ny, m.y0 + ly);
    m.cz = 63 * h + m.lane;
    m.act = m.cz < nz;
    m.own = m.act && (h == 0 || m.lane > 0);
    return true;
}

struct TvRow {
    // x(c + e_x), x(c + e_y), x(c + e_z), y(c), z(c), T(c); the x(. + e_z) values only on
    // the lane that loads them (the run's last: the others take the next lane's x)
    float xp, xn, xz, y0, y1, y2, z, t;
    float lxn, lxz, ly0, ly1, ly2;       // x-neighbour: x(c - e_x + e_y), x(c - e_x + e_z), y
    float i0, i1, i2, li0, li1, li2;     // dTV field at c and c - e_x
};

template <bool DTV>
__device__ __forceinline__ void tv_row_load(TvRow& r, __amdgpu_buffer_rsrc_t rx,
                                            __amdgpu_buffer_rsrc_t ry, __amdgpu_buffer_rsrc_t rz,
                                            __amdgpu_buffer_rsrc_t rt, __amdgpu_buffer_rsrc_t rxi,
                                            uint32_t c, uint32_t sx, uint32_t sy, uint32_t nvb,
                                            bool hx, bool hy, bool hz, bool lx) {
    r.xp = hx ? vol_ld(rx, c + sx, 0) : 0.0f;
    r.xn = hy ? vol_ld(rx, c + sy, 0) : 0.0f;
    r.xz = hz ? vol_ld(rx, c + 4, 0) : 0.0f;
    r.y0 = vol_ld(ry, c, 0);
    r.y1 = vol_ld(ry, c, nvb);
    r.y2 = vol_ld(ry, c, 2 * nvb);
    r.z = vol_ld(rz, c, 0);
    r.t = vol_ld(rt, c, 0);
    r.i0 = r.i1 = r.i2 = r.li0 = r.li1 = r.li2 = 0.0f;
    r.lxn = r.lxz = r.ly0 = r.ly1 = r.ly2 = 0.0f;
    if (DTV) {
        r.i0 = vol_ld(rxi, c, 0);
        r.i1 = vol_ld(rxi, c, nvb);
        r.i2 = vol_ld(rxi, c, 2 * nvb);
    }
    if (lx) {
        const uint32_t cl = c - sx;
        r.lxn = hy ? vol_ld(rx, cl + sy, 0) : 0.0f;
        r.lxz = hz ? vol_ld(rx, cl + 4, 0) : 0.0f;
        r.ly0 = vol_ld(ry, cl, 0);
        r.ly1 = vol_ld(ry, cl, nvb);
        r.ly2 = vol_ld(ry, cl, 2 * nvb);
        if (DTV) {
            r.li0 = vol_ld(rxi, cl, 0);
            r.li1 = vol_ld(rxi, cl, nvb);
            r.li2 = vol_ld(rxi, cl, 2 * nvb);
        }
    }
}

template <bool DTV, bool PAIR>
__global__ void __launch_bounds__(256)
tv_wave(PriorArgs P, int ly, const float* __restrict__ x_in, float* __restrict__ x_out,
        const float* __restrict__ y_in, float* __restrict__ y_out, float* __restrict__ z,
        const float* __restrict__ T, const float* __restrict__ xi) {
    // byte strides; 3 nv floats stay below 4 GiB (images are limited to 1 GiB)
    const uint32_t sx = 4u * P.nz, sy = 4u * P.nz * P.nx;
    const uint32_t nvb = sy * P.ny;
    const auto rx = vol_rsrc(x_in, nvb), rxo = vol_rsrc(x_out, nvb);
    const auto ry = vol_rsrc(y_in, 3 * nvb), ryo = vol_rsrc(y_out, 3 * nvb);
    const auto rz = vol_rsrc(z, nvb), rt = vol_rsrc(T, nvb);
    const auto rxi = vol_rsrc(DTV ? xi : x_in, DTV ? 3 * nvb : nvb);
    WaveMap m;
    if (!wave_map(P.nx, P.ny, P.nz, ly, m)) return;  // whole wavefront beyond the last chunk
    const int cx = m.cx, cz = m.cz, y0 = m.y0, y1 = m.y1;
    const bool act = m.act, own = m.own;  // own: writes its voxel
    const bool hx = cx < P.nx - 1, lx = cx > 0, hz = cz < P.nz - 1;
    const bool hz_ld = hz && m.lane == 63;  // loads its own +z neighbours
    int cy = y0 > 0 ? y0 - 1 : y0;
    uint32_t c = 4u * (((uint32_t)cy * P.nx + cx) * P.nz + min(cz, P.nz - 1));
    TvRow cur = {}, nxt = {};
    float xc = 0.0f, xl = 0.0f, dprev = 0.0f;
    // PAIR: low parts of x and z at the voxel (this row and the prefetched next one)
    const auto rxl = vol_rsrc(PAIR ? P.xlo : x_in, nvb), rzl = vol_rsrc(PAIR ? P.zlo : z, nvb);
    float lo_x = 0.0f, lo_z = 0.0f, lo_xn = 0.0f, lo_zn = 0.0f;
    if (act) {
        tv_row_load<DTV>(cur, rx, ry, rz, rt, rxi, c, sx, sy, nvb, hx, cy < P.ny - 1, hz_ld, lx);
        xc = vol_ld(rx, c, 0);
        if (lx) xl = vol_ld(rx, c - sx, 0);
        if (PAIR) {
            lo_x = vol_ld(rxl, c, 0);
            lo_z = vol_ld(rzl, c, 0);
        }
    }
    for (; cy < y1; ++cy, c += sy) {
        const bool hy = cy < P.ny - 1;
        if (act && cy + 1 < y1) {
            tv_row_load<DTV>(nxt, rx, ry, rz, rt, rxi, c + sy, sx, sy, nvb, hx, cy + 1 < P.ny - 1,
                             hz_ld, lx);
            if (PAIR) {
                lo_xn = vol_ld(rxl, c + sy, 0);
                lo_zn = vol_ld(rzl, c + sy, 0);
            }
        }
        // +z neighbours: the next lane's x and x-neighbour (wavefront shift left by one
        // lane, all lanes taking part); the last lane keeps the values it loaded
        const float xz = __int_as_float(__builtin_amdgcn_update_dpp(
            __float_as_int(cur.xz), __float_as_int(xc), 0x130 /* wave_shl:1 */, 0xF, 0xF, false));
        const float lxz = __int_as_float(__builtin_amdgcn_update_dpp(
            __float_as_int(cur.lxz), __float_as_int(xl), 0x130 /* wave_shl:1 */, 0xF, 0xF, false));
        float q[3], dy[3] = {0.0f, 0.0f, 0.0f}, qn[3], dn[3] = {0.0f, 0.0f, 0.0f};
        if (act) {
            prior_dual_vals(P, hx ? cur.xp - xc : 0.0f, hy ? cur.xn - xc : 0.0f,
                            hz ? xz - xc : 0.0f, cur.y0, cur.y1, cur.y2, cur.i0, cur.i1,
                            cur.i2, q, dy);
            // x-neighbour (cx - 1, cy, cz): its +x difference is x(c) - x(c - e_x)
            if (lx)
                prior_dual_vals(P, xc - xl, hy ? cur.lxn - xl : 0.0f, hz ? lxz - xl : 0.0f,
                                cur.ly0, cur.ly1, cur.ly2, cur.li0, cur.li1, cur.li2, qn, dn);
        }
        const float dzn = __shfl_up(dy[2], 1, 64);  // all lanes take part
        if (own && cy >= y0) {
            // grad^T p (v) = sum_d [v_d > 0] p_d(v - e_d) - [v_d < N_d - 1] p_d(v)
            float dz = 0.0f;
            if (hx) dz -= dy[0];
            if (hy) dz -= dy[1];
            if (hz) dz -= dy[2];
            if (lx) dz += dn[0];
            if (cy > 0) dz += dprev;
            if (cz > 0) dz += dzn;
            if (P.dz_add) dz += vol_ld(vol_rsrc(P.dz_add, nvb), c, 0);
            vol_st(ryo, c, 0, q[0]);
            vol_st(ryo, c, nvb, q[1]);
            vol_st(ryo, c, 2 * nvb, q[2]);
            if (PAIR) {
                float xh = xc, zh = cur.z;
                primal_pair(xh, lo_x, zh, lo_z, cur.t, dz, P.inv_p);
                vol_st(rz, c, 0, zh);
                vol_st(rzl, c, 0, lo_z);
                vol_st(rxo, c, 0, xh);
                vol_st(rxl, c, 0, lo_x);
            } else {
                const float zn = cur.z + dz;
                vol_st(rz, c, 0, zn);
                const float zbar = __builtin_fmaf(dz, P.inv_p, zn);
                vol_st(rxo, c, 0, fmaxf(xc - cur.t * zbar, 0.0f));
            }
        }
        dprev = dy[1];
        xc = cur.xn;
        xl = cur.lxn;
        cur = nxt;
        lo_x = lo_xn;
        lo_z = lo_zn;
    }
}

// Prior term alpha sum_v |(A_n x)_v|_2 (FP64 partials; 0 when use_grad is 0) plus the
// non-negativity indicator: a negative voxel makes the term +inf.
__global__ void __launch_bounds__(BLOCK)
tv_obj(PriorArgs P, const float* __restrict__ x, const float* __restrict__ xi,
       double* __restrict__ part, int use_grad) {
    const int64_t sx = P.nz, sy = (int64_t)P.nz * P.nx;
    const int64_t nv = sy * P.ny;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double v = 0.0;
    if (t < nv) {
        int cx, cy, cz;
        zf_coords(P, t, cx, cy, cz);
        const double xc = x[t];
        double g0 = cx < P.nx - 1 ? (double)x[t + sx] - xc : 0.0;
        double g1 = cy < P.ny - 1 ? (double)x[t + sy] - xc : 0.0;
        double g2 = cz < P.nz - 1 ? (double)x[t + 1] - xc : 0.0;
        if (P.dtv) {
            const double x0 = xi[t], x1 = xi[t + nv], x2 = xi[t + 2 * nv];
            const double dot = x0 * g0 + x1 * g1 + x2 * g2;
            g0 -= P.gamma_d * dot * x0;
            g1 -= P.gamma_d * dot * x1;
            g2 -= P.gamma_d * dot * x2;
        }
        const double r = P.atv ? fabs(g0) + fabs(g1) + fabs(g2) : sqrt(g0 * g0 + g1 * g1 + g2 * g2);
        v = use_grad ? (double)P.alpha * r : 0.0;
        if (xc < 0.0) v = INFINITY;
    }
    const double s = block_sum<BLOCK>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// xi = grad s / sqrt(|grad s|^2 + eta^2) for the dTV side image s (z-fastest).
__global__ void __launch_bounds__(BLOCK)
dtv_field(PriorArgs P, const float* __restrict__ s, float eta, float* __restrict__ xi) {
    const int64_t sx = P.nz, sy = (int64_t)P.nz * P.nx;
    const int64_t nv = sy * P.ny;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t >= nv) return;
    int cx, cy, cz;
    zf_coords(P, t, cx, cy, cz);
    const double sc = s[t];
    const double g0 = cx < P.nx - 1 ? (double)s[t + sx] - sc : 0.0;
    const double g1 = cy < P.ny - 1 ? (double)s[t + sy] - sc : 0.0;
    const double g2 = cz < P.nz - 1 ? (double)s[t + 1] - sc : 0.0;
    const double nrm = sqrt(g0 * g0 + g1 * g1 + g2 * g2 + (double)eta * eta);
    xi[t] = (float)(g0 / nrm);
    xi[t + nv] = (float)(g1 / nrm);
    xi[t + 2 * nv] = (float)(g2 / nrm);
}

// ---------------------------------------------------------------- TGV (two prior blocks)
// x = (u, w) with w a 3-component field; block n-1: f = alpha0 ||.||_{2,1}, A = (grad, -I)
// (dual q1, 3 components); block n: f = alpha1 ||.||_{2,1}, A = (0, E) with
// E w = sym(J w) stored as (J00, J11, J22, (J01+J10)/sqrt2, (J02+J20)/sqrt2,
// (J12+J21)/sqrt2), J_kl = forward difference of w_k along axis l (Section 4.3, eq.
// setting TGV).  Components 0, 1, 2 are the x, y, z axes.  w has no prox (g is the
// non-negativity of u only), and its step T_w is the scalar minimum of the two blocks'.
struct TgvArgs {
    int nx, ny, nz;
    float sigma;  // dual step of the block
    float alpha;  // ball radius of the block
    float inv_p;
    float tw;     // T_w
};

#define TGV_SQRT_HALF 0.70710678118654752f

struct ZfStrides {
    int64_t sx, sy, nv;
};

__device__ __forceinline__ ZfStrides zf_strides(int nx, int ny, int nz) {
    ZfStrides S;
    S.sx = nz;
    S.sy = (int64_t)nz * nx;
    S.nv = S.sy * ny;
    return S;
}

// Block n-1 dual update from the forward differences g of u (zero on the high faces),
// w and q1 at one voxel: q = P_alpha0(q1 + sigma (grad u - w)), dq = q - q1.
__device__ __forceinline__ void tgv1_dual_vals(const TgvArgs& P, float g0, float g1, float g2,
                                               float w0, float w1, float w2, float y0, float y1,
                                               float y2, float q[3], float dq[3]) {
    q[0] = __builtin_fmaf(P.sigma, g0 - w0, y0);
    q[1] = __builtin_fmaf(P.sigma, g1 - w1, y1);
    q[2] = __builtin_fmaf(P.sigma, g2 - w2, y2);
    const float nrm = __builtin_sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    if (nrm > P.alpha) {
        const float sc = P.alpha / nrm;
        q[0] *= sc;
        q[1] *= sc;
        q[2] *= sc;
    }
    dq[0] = q[0] - y0;
    dq[1] = q[1] - y1;
    dq[2] = q[2] - y2;
}

// The same at voxel (cx, cy, cz), loading everything it needs.
__device__ __forceinline__ void tgv1_dual_at(const TgvArgs& P, const float* __restrict__ u,
                                             const float* __restrict__ w,
                                             const float* __restrict__ q1, int cx, int cy,
                                             int cz, float q[3], float dq[3]) {
    const ZfStrides S = zf_strides(P.nx, P.ny, P.nz);
    const int64_t c = (int64_t)cy * S.sy + (int64_t)cx * S.sx + cz;
    const float uc = u[c];
    const float g0 = cx < P.nx - 1 ? u[c + S.sx] - uc : 0.0f;
    const float g1 = cy < P.ny - 1 ? u[c + S.sy] - uc : 0.0f;
    const float g2 = cz < P.nz - 1 ? u[c + 1] - uc : 0.0f;
    tgv1_dual_vals(P, g0, g1, g2, w[c], w[c + S.nv], w[c + 2 * S.nv], q1[c], q1[c + S.nv],
                   q1[c + 2 * S.nv], q, dq);
}

// Algorithm 2 from the dual step to the extrapolation for block n-1, fused with the next
// iteration's primal step:
// dz_u = grad^T dq, dz_w = -dq; u, w, q1 ping-pong, z_u and z_w in place.  Column tiles as
// in tv_iter: the dual changes of the tile's voxels are shared through LDS and only the
// tile's low faces recompute a neighbour's update.
__global__ void __launch_bounds__(1024)
tgv1_iter(TgvArgs P, PriorTile TL, const float* __restrict__ u_in, float* __restrict__ u_out,
          const float* __restrict__ w_in, float* __restrict__ w_out,
          const float* __restrict__ q_in, float* __restrict__ q_out, float* __restrict__ zu,
          float* __restrict__ zw, const float* __restrict__ Tu) {
    __shared__ float sdq[3][1024];
    const ZfStrides S = zf_strides(P.nx, P.ny, P.nz);
    int cx, cy, cz, lx, ly;
    const bool act = tile_voxel(TL, P.nx, P.ny, P.nz, xcd_remap(blockIdx.x, gridDim.x), cx, cy,
                                cz, lx, ly);
    const int l = threadIdx.x;
    float q[3], dq[3] = {0.0f, 0.0f, 0.0f};
    if (act) tgv1_dual_at(P, u_in, w_in, q_in, cx, cy, cz, q, dq);
    sdq[0][l] = dq[0];
    sdq[1][l] = dq[1];
    sdq[2][l] = dq[2];
    __syncthreads();
    if (!act) return;
    float qn[3], dn[3];
    float dzu = 0.0f;
    if (cx < P.nx - 1) dzu -= dq[0];
    if (cy < P.ny - 1) dzu -= dq[1];
    if (cz < P.nz - 1) dzu -= dq[2];
    if (cx > 0) {
        if (lx > 0) {
            dzu += sdq[0][l - P.nz];
        } else {
            tgv1_dual_at(P, u_in, w_in, q_in, cx - 1, cy, cz, qn, dn);
            dzu += dn[0];
        }
    }
    if (cy > 0) {
        if (ly > 0) {
            dzu += sdq[1][l - TL.tx * P.nz];
        } else {
            tgv1_dual_at(P, u_in, w_in, q_in, cx, cy - 1, cz, qn, dn);
            dzu += dn[1];
        }
    }
    if (cz > 0) dzu += sdq[2][l - 1];
    const int64_t t = ((int64_t)cy * P.nx + cx) * P.nz + cz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int64_t i = t + k * S.nv;
        q_out[i] = q[k];
        const float dzw = -dq[k];
        const float zn = zw[i] + dzw;
        zw[i] = zn;
        w_out[i] = w_in[i] - P.tw * __builtin_fmaf(dzw, P.inv_p, zn);
    }
    const float zn = zu[t] + dzu;
    zu[t] = zn;
    u_out[t] = fmaxf(u_in[t] - Tu[t] * __builtin_fmaf(dzu, P.inv_p, zn), 0.0f);
}

// E w from the forward differences J[k][l] of w_k along axis l.
__device__ __forceinline__ void sym_grad_vals(const float J[3][3], float e[6]) {
    e[0] = J[0][0];
    e[1] = J[1][1];
    e[2] = J[2][2];
    e[3] = TGV_SQRT_HALF * (J[0][1] + J[1][0]);
    e[4] = TGV_SQRT_HALF * (J[0][2] + J[2][0]);
    e[5] = TGV_SQRT_HALF * (J[1][2] + J[2][1]);
}

// E w at voxel (cx, cy, cz), 6 components.
__device__ __forceinline__ void sym_grad_at(int nx, int ny, int nz, const float* __restrict__ w,
                                            int cx, int cy, int cz, float e[6]) {
    const ZfStrides S = zf_strides(nx, ny, nz);
    const int64_t c = (int64_t)cy * S.sy + (int64_t)cx * S.sx + cz;
    const int64_t step[3] = {S.sx, S.sy, 1};
    const bool in[3] = {cx < nx - 1, cy < ny - 1, cz < nz - 1};
    float J[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float* wk = w + k * S.nv;
        const float wc = wk[c];
#pragma unroll
        for (int l = 0; l < 3; ++l) J[k][l] = in[l] ? wk[c + step[l]] - wc : 0.0f;
    }
    sym_grad_vals(J, e);
}

// Block n dual update from e = E w and q2 at one voxel: q = P_alpha1(q2 + sigma e),
// dq = q - q2.
__device__ __forceinline__ void tgv2_dual_vals(const TgvArgs& P, const float e[6],
                                               const float y[6], float q[6], float dq[6]) {
    float ss = 0.0f;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        q[k] = __builtin_fmaf(P.sigma, e[k], y[k]);
        ss = __builtin_fmaf(q[k], q[k], ss);
    }
    const float nrm = __builtin_sqrtf(ss);
    const float sc = nrm > P.alpha ? P.alpha / nrm : 1.0f;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        if (nrm > P.alpha) q[k] *= sc;
        dq[k] = q[k] - y[k];
    }
}

// Block n dual update at voxel (cx, cy, cz), loading everything it needs.
__device__ __forceinline__ void tgv2_dual_at(const TgvArgs& P, const float* __restrict__ w,
                                             const float* __restrict__ q2, int cx, int cy,
                                             int cz, float q[6], float dq[6]) {
    const ZfStrides S = zf_strides(P.nx, P.ny, P.nz);
    const int64_t c = (int64_t)cy * S.sy + (int64_t)cx * S.sx + cz;
    float e[6], y[6];
    sym_grad_at(P.nx, P.ny, P.nz, w, cx, cy, cz, e);
#pragma unroll
    for (int k = 0; k < 6; ++k) y[k] = q2[c + k * S.nv];
    tgv2_dual_vals(P, e, y, q, dq);
}

// Algorithm 2 from the dual step to the extrapolation for block n, fused with the next
// iteration's primal step:
// dz_w = E^T dq (E^T p)_k = sum_l D_l^T of the (k, l) entry, D_l^T p (v) = [v_l > 0]
// p(v - e_l) - [v_l < N_l - 1] p(v); dz_u = 0, so u = max(u - T_u z_u, 0).  Column tiles
// with the 6-component dual changes shared through LDS, as in tgv1_iter.
__global__ void __launch_bounds__(1024)
tgv2_iter(TgvArgs P, PriorTile TL, const float* __restrict__ u_in, float* __restrict__ u_out,
          const float* __restrict__ w_in, float* __restrict__ w_out,
          const float* __restrict__ q_in, float* __restrict__ q_out, const float* __restrict__ zu,
          float* __restrict__ zw, const float* __restrict__ Tu) {
    __shared__ float sdq[6][1024];
    const ZfStrides S = zf_strides(P.nx, P.ny, P.nz);
    int cx, cy, cz, lx, ly;
    const bool act = tile_voxel(TL, P.nx, P.ny, P.nz, xcd_remap(blockIdx.x, gridDim.x), cx, cy,
                                cz, lx, ly);
    const int l = threadIdx.x;
    float q[6], dq[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (act) tgv2_dual_at(P, w_in, q_in, cx, cy, cz, q, dq);
#pragma unroll
    for (int k = 0; k < 6; ++k) sdq[k][l] = dq[k];
    __syncthreads();
    if (!act) return;
    const int cc[3] = {cx, cy, cz};
    const int nn[3] = {P.nx, P.ny, P.nz};
    const bool inner[3] = {lx > 0, ly > 0, true};  // backward neighbour inside the tile
    const int lstep[3] = {P.nz, TL.tx * P.nz, 1};
    // entry (k, l) of the symmetric matrix -> component
    const int ent[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    float dzw[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        float dn[6];
        const bool back = cc[ax] > 0;
        if (back) {
            if (inner[ax]) {
#pragma unroll
                for (int k = 0; k < 6; ++k) dn[k] = sdq[k][l - lstep[ax]];
            } else {
                float qn[6];
                tgv2_dual_at(P, w_in, q_in, cx - (ax == 0), cy - (ax == 1), cz - (ax == 2), qn, dn);
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int e = ent[k][ax];
            const float wgt = (k == ax) ? 1.0f : TGV_SQRT_HALF;
            float v = 0.0f;
            if (back) v += dn[e];
            if (cc[ax] < nn[ax] - 1) v -= dq[e];
            dzw[k] = __builtin_fmaf(wgt, v, dzw[k]);
        }
    }
    const int64_t t = ((int64_t)cy * P.nx + cx) * P.nz + cz;
#pragma unroll
    for (int k = 0; k < 6; ++k) q_out[t + k * S.nv] = q[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int64_t i = t + k * S.nv;
        const float zn = zw[i] + dzw[k];
        zw[i] = zn;
        w_out[i] = w_in[i] - P.tw * __builtin_fmaf(dzw[k], P.inv_p, zn);
    }
    u_out[t] = fmaxf(u_in[t] - Tu[t] * zu[t], 0.0f);
}

// Wavefront forms of tgv1_iter and tgv2_iter for volumes with 32 <= nz <= 128, laid out
// as tv_wave: one wavefront per run of 64 voxels of a column (runs overlap by one voxel,
// the first lane of a run above the first only passes its dual change on), marching
// along y through a chunk of rows that starts one row early, the y-neighbour's change
// carried in registers, the z-neighbour's taken from the next-lower lane and the
// x-neighbour's recomputed.  In tgv1_wave each row's loads are issued before the
// previous row's stores; tgv2_wave, with twice the inputs per row, loads its row when it
// gets there (the prefetching form needed 103 registers and was no faster).  Every
// 6-component field stays below 4 GiB (checked by the host).
struct Tgv1Row {
    float up, un, uz;     // u(c + e_x), u(c + e_y), u(c + e_z)
    float w[3], y[3], zw[3], zu, t;
    float lun, luz;       // x-neighbour: u(c - e_x + e_y), u(c - e_x + e_z)
    float lw[3], ly[3];   // w(c - e_x), q1(c - e_x)
};

__device__ __forceinline__ void tgv1_row_load(Tgv1Row& r, __amdgpu_buffer_rsrc_t ru,
                                              __amdgpu_buffer_rsrc_t rw, __amdgpu_buffer_rsrc_t rq,
                                              __amdgpu_buffer_rsrc_t rzu, __amdgpu_buffer_rsrc_t rzw,
                                              __amdgpu_buffer_rsrc_t rt, uint32_t c, uint32_t sx,
                                              uint32_t sy, uint32_t nvb, bool hx, bool hy, bool hz,
                                              bool lx) {
    r.up = hx ? vol_ld(ru, c + sx, 0) : 0.0f;
    r.un = hy ? vol_ld(ru, c + sy, 0) : 0.0f;
    r.uz = hz ? vol_ld(ru, c + 4, 0) : 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r.w[k] = vol_ld(rw, c, k * nvb);
        r.y[k] = vol_ld(rq, c, k * nvb);
        r.zw[k] = vol_ld(rzw, c, k * nvb);
    }
    r.zu = vol_ld(rzu, c, 0);
    r.t = vol_ld(rt, c, 0);
    r.lun = r.luz = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) r.lw[k] = r.ly[k] = 0.0f;
    if (lx) {
        const uint32_t cl = c - sx;
        r.lun = hy ? vol_ld(ru, cl + sy, 0) : 0.0f;
        r.luz = hz ? vol_ld(ru, cl + 4, 0) : 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            r.lw[k] = vol_ld(rw, cl, k * nvb);
            r.ly[k] = vol_ld(rq, cl, k * nvb);
        }
    }
}

__global__ void __launch_bounds__(256)
tgv1_wave(TgvArgs P, int ly, const float* __restrict__ u_in, float* __restrict__ u_out,
          const float* __restrict__ w_in, float* __restrict__ w_out,
          const float* __restrict__ q_in, float* __restrict__ q_out, float* __restrict__ zu,
          float* __restrict__ zw, const float* __restrict__ Tu) {
    const uint32_t sx = 4u * P.nz, sy = 4u * P.nz * P.nx;
    const uint32_t nvb = sy * P.ny;
    const auto ru = vol_rsrc(u_in, nvb), ruo = vol_rsrc(u_out, nvb);
    const auto rw = vol_rsrc(w_in, 3 * nvb), rwo = vol_rsrc(w_out, 3 * nvb);
    const auto rq = vol_rsrc(q_in, 3 * nvb), rqo = vol_rsrc(q_out, 3 * nvb);
    const auto rzu = vol_rsrc(zu, nvb), rzw = vol_rsrc(zw, 3 * nvb), rt = vol_rsrc(Tu, nvb);
    WaveMap m;
    if (!wave_map(P.nx, P.ny, P.nz, ly, m)) return;
    const int cx = m.cx, cz = m.cz;
    const bool hx = cx < P.nx - 1, lx = cx > 0, hz = cz < P.nz - 1;
    int cy = m.y0 > 0 ? m.y0 - 1 : m.y0;
    uint32_t c = 4u * (((uint32_t)cy * P.nx + cx) * P.nz + min(cz, P.nz - 1));
    Tgv1Row cur = {}, nxt = {};
    float uc = 0.0f, ul = 0.0f, dprev = 0.0f;
    if (m.act) {
        tgv1_row_load(cur, ru, rw, rq, rzu, rzw, rt, c, sx, sy, nvb, hx, cy < P.ny - 1, hz, lx);
        uc = vol_ld(ru, c, 0);
        if (lx) ul = vol_ld(ru, c - sx, 0);
    }
    for (; cy < m.y1; ++cy, c += sy) {
        const bool hy = cy < P.ny - 1;
        if (m.act && cy + 1 < m.y1)
            tgv1_row_load(nxt, ru, rw, rq, rzu, rzw, rt, c + sy, sx, sy, nvb, hx,
                          cy + 1 < P.ny - 1, hz, lx);
        float q[3], dq[3] = {0.0f, 0.0f, 0.0f}, qn[3], dn[3] = {0.0f, 0.0f, 0.0f};
        if (m.act) {
            tgv1_dual_vals(P, hx ? cur.up - uc : 0.0f, hy ? cur.un - uc : 0.0f,
                           hz ? cur.uz - uc : 0.0f, cur.w[0], cur.w[1], cur.w[2], cur.y[0],
                           cur.y[1], cur.y[2], q, dq);
            if (lx)  // x-neighbour: its +x difference of u is u(c) - u(c - e_x)
                tgv1_dual_vals(P, uc - ul, hy ? cur.lun - ul : 0.0f, hz ? cur.luz - ul : 0.0f,
                               cur.lw[0], cur.lw[1], cur.lw[2], cur.ly[0], cur.ly[1], cur.ly[2],
                               qn, dn);
        }
        const float dzn = __shfl_up(dq[2], 1, 64);
        if (m.own && cy >= m.y0) {
            float dzu = 0.0f;
            if (hx) dzu -= dq[0];
            if (hy) dzu -= dq[1];
            if (hz) dzu -= dq[2];
            if (lx) dzu += dn[0];
            if (cy > 0) dzu += dprev;
            if (cz > 0) dzu += dzn;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                vol_st(rqo, c, k * nvb, q[k]);
                const float dzw = -dq[k];
                const float zn = cur.zw[k] + dzw;
                vol_st(rzw, c, k * nvb, zn);
                vol_st(rwo, c, k * nvb, cur.w[k] - P.tw * __builtin_fmaf(dzw, P.inv_p, zn));
            }
            const float zn = cur.zu + dzu;
            vol_st(rzu, c, 0, zn);
            vol_st(ruo, c, 0, fmaxf(uc - cur.t * __builtin_fmaf(dzu, P.inv_p, zn), 0.0f));
        }
        dprev = dq[1];
        uc = cur.un;
        ul = cur.lun;
        cur = nxt;
    }
}

struct Tgv2Row {
    float wp[3], wn[3], wz[3];  // w_k(c + e_x), w_k(c + e_y), w_k(c + e_z)
    float y[6];                 // q2(c)
    float zw[3], u, t, zu;      // z_w(c), u(c), T_u(c), z_u(c)
    float lwn[3], lwz[3];       // x-neighbour: w_k(c - e_x + e_y), w_k(c - e_x + e_z)
    float ly[6];                // q2(c - e_x)
};

__device__ __forceinline__ void tgv2_row_load(Tgv2Row& r, __amdgpu_buffer_rsrc_t ru,
                                              __amdgpu_buffer_rsrc_t rw, __amdgpu_buffer_rsrc_t rq,
                                              __amdgpu_buffer_rsrc_t rzu, __amdgpu_buffer_rsrc_t rzw,
                                              __amdgpu_buffer_rsrc_t rt, uint32_t c, uint32_t sx,
                                              uint32_t sy, uint32_t nvb, bool hx, bool hy, bool hz,
                                              bool lx) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r.wp[k] = hx ? vol_ld(rw, c + sx, k * nvb) : 0.0f;
        r.wn[k] = hy ? vol_ld(rw, c + sy, k * nvb) : 0.0f;
        r.wz[k] = hz ? vol_ld(rw, c + 4, k * nvb) : 0.0f;
        r.zw[k] = vol_ld(rzw, c, k * nvb);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) r.y[k] = vol_ld(rq, c, k * nvb);
    r.u = vol_ld(ru, c, 0);
    r.t = vol_ld(rt, c, 0);
    r.zu = vol_ld(rzu, c, 0);
#pragma unroll
    for (int k = 0; k < 3; ++k) r.lwn[k] = r.lwz[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < 6; ++k) r.ly[k] = 0.0f;
    if (lx) {
        const uint32_t cl = c - sx;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            r.lwn[k] = hy ? vol_ld(rw, cl + sy, k * nvb) : 0.0f;
            r.lwz[k] = hz ? vol_ld(rw, cl + 4, k * nvb) : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) r.ly[k] = vol_ld(rq, cl, k * nvb);
    }
}

__global__ void __launch_bounds__(256)
tgv2_wave(TgvArgs P, int ly, const float* __restrict__ u_in, float* __restrict__ u_out,
          const float* __restrict__ w_in, float* __restrict__ w_out,
          const float* __restrict__ q_in, float* __restrict__ q_out, const float* __restrict__ zu,
          float* __restrict__ zw, const float* __restrict__ Tu) {
    const uint32_t sx = 4u * P.nz, sy = 4u * P.nz * P.nx;
    const uint32_t nvb = sy * P.ny;
    const auto ru = vol_rsrc(u_in, nvb), ruo = vol_rsrc(u_out, nvb);
    const auto rw = vol_rsrc(w_in, 3 * nvb), rwo = vol_rsrc(w_out, 3 * nvb);
    const auto rq = vol_rsrc(q_in, 6 * nvb), rqo = vol_rsrc(q_out, 6 * nvb);
    const auto rzu = vol_rsrc(zu, nvb), rzw = vol_rsrc(zw, 3 * nvb), rt = vol_rsrc(Tu, nvb);
    WaveMap m;
    if (!wave_map(P.nx, P.ny, P.nz, ly, m)) return;
    const int cx = m.cx, cz = m.cz;
    const bool hx = cx < P.nx - 1, lx = cx > 0, hz = cz < P.nz - 1;
    int cy = m.y0 > 0 ? m.y0 - 1 : m.y0;
    uint32_t c = 4u * (((uint32_t)cy * P.nx + cx) * P.nz + min(cz, P.nz - 1));
    Tgv2Row cur = {};
    float wc[3] = {0.0f, 0.0f, 0.0f}, wl[3] = {0.0f, 0.0f, 0.0f};
    float dprev[3] = {0.0f, 0.0f, 0.0f};  // y-neighbour's changes of entries (k, y)
    if (m.act) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            wc[k] = vol_ld(rw, c, k * nvb);
            if (lx) wl[k] = vol_ld(rw, c - sx, k * nvb);
        }
    }
    // entry (k, l) of the symmetric matrix -> component
    constexpr int ent[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    for (; cy < m.y1; ++cy, c += sy) {
        const bool hy = cy < P.ny - 1;
        if (m.act) tgv2_row_load(cur, ru, rw, rq, rzu, rzw, rt, c, sx, sy, nvb, hx, hy, hz, lx);
        float q[6], dq[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, qn[6];
        float dn[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (m.act) {
            float J[3][3], e[6];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                J[k][0] = hx ? cur.wp[k] - wc[k] : 0.0f;
                J[k][1] = hy ? cur.wn[k] - wc[k] : 0.0f;
                J[k][2] = hz ? cur.wz[k] - wc[k] : 0.0f;
            }
            sym_grad_vals(J, e);
            tgv2_dual_vals(P, e, cur.y, q, dq);
            if (lx) {  // x-neighbour: its +x differences are w_k(c) - w_k(c - e_x)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    J[k][0] = wc[k] - wl[k];
                    J[k][1] = hy ? cur.lwn[k] - wl[k] : 0.0f;
                    J[k][2] = hz ? cur.lwz[k] - wl[k] : 0.0f;
                }
                sym_grad_vals(J, e);
                tgv2_dual_vals(P, e, cur.ly, qn, dn);
            }
        }
        float dzn[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) dzn[k] = __shfl_up(dq[ent[k][2]], 1, 64);
        if (m.own && cy >= m.y0) {
            // dz_w = E^T dq: (E^T p)_k = sum_l wgt(k, l) D_l^T p_(k, l)
            const bool back[3] = {lx, cy > 0, cz > 0};
            const bool fwd[3] = {hx, hy, hz};
            float dzw[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int e = ent[k][ax];
                    const float wgt = (k == ax) ? 1.0f : TGV_SQRT_HALF;
                    const float nb = ax == 0 ? dn[e] : (ax == 1 ? dprev[k] : dzn[k]);
                    float v = 0.0f;
                    if (back[ax]) v += nb;
                    if (fwd[ax]) v -= dq[e];
                    dzw[k] = __builtin_fmaf(wgt, v, dzw[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) vol_st(rqo, c, k * nvb, q[k]);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float zn = cur.zw[k] + dzw[k];
                vol_st(rzw, c, k * nvb, zn);
                vol_st(rwo, c, k * nvb, wc[k] - P.tw * __builtin_fmaf(dzw[k], P.inv_p, zn));
            }
            vol_st(ruo, c, 0, fmaxf(cur.u - cur.t * cur.zu, 0.0f));
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            dprev[k] = dq[ent[k][1]];
            wc[k] = cur.wn[k];
            wl[k] = cur.lwn[k];
        }
    }
}

// The primal step for the w component over k data iterations (their dz_w is 0, so z_w is
// unchanged and every one of them subtracts T_w z_w): w -= k T_w z_w.
__global__ void w_catchup(float* __restrict__ w, const float* __restrict__ zw, int64_t n, float s) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t < n) w[t] = w[t] - s * zw[t];
}

// TGV prior term alpha0 sum |grad u - w|_2 + alpha1 sum |E w|_2 (FP64 partials) plus the
// non-negativity indicator of u.
__global__ void __launch_bounds__(BLOCK)
tgv_obj(int nx, int ny, int nz, double alpha0, double alpha1, const float* __restrict__ u,
        const float* __restrict__ w, double* __restrict__ part) {
    const ZfStrides S = zf_strides(nx, ny, nz);
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double v = 0.0;
    if (t < S.nv) {
        const int64_t col = t / nz;
        const int cz = (int)(t - col * nz);
        const int cy = (int)(col / nx), cx = (int)(col - (int64_t)cy * nx);
        const double uc = u[t];
        const double g0 = (cx < nx - 1 ? (double)u[t + S.sx] - uc : 0.0) - w[t];
        const double g1 = (cy < ny - 1 ? (double)u[t + S.sy] - uc : 0.0) - w[t + S.nv];
        const double g2 = (cz < nz - 1 ? (double)u[t + 1] - uc : 0.0) - w[t + 2 * S.nv];
        double J[3][3];
        const int64_t step[3] = {S.sx, S.sy, 1};
        const bool in[3] = {cx < nx - 1, cy < ny - 1, cz < nz - 1};
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l)
                J[k][l] = in[l] ? (double)w[t + k * S.nv + step[l]] - (double)w[t + k * S.nv] : 0.0;
        const double h = 0.5;  // (1/sqrt2)^2
        const double e2 = J[0][0] * J[0][0] + J[1][1] * J[1][1] + J[2][2] * J[2][2] +
                          h * ((J[0][1] + J[1][0]) * (J[0][1] + J[1][0]) +
                               (J[0][2] + J[2][0]) * (J[0][2] + J[2][0]) +
                               (J[1][2] + J[2][1]) * (J[1][2] + J[2][1]));
        v = alpha0 * sqrt(g0 * g0 + g1 * g1 + g2 * g2) + alpha1 * sqrt(e2);
        if (uc < 0.0) v = INFINITY;
    }
    const double s = block_sum<BLOCK>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ---------------------------------------------------------------- normalised backprojection
// out = atb / at1 where at1 > 0, else 0 (out may alias atb: each thread reads its element
// before writing it); FP64 partials per block of the sum of the positive outputs (part_s)
// and of their count (part_n).
__global__ void __launch_bounds__(BLOCK)
ratio_on_support(const float* atb, const float* __restrict__ at1, int64_t n, float* out,
                 double* __restrict__ part_s, double* __restrict__ part_n) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double v = 0.0, c = 0.0;
    if (t < n) {
        const float a = at1[t];
        const float r = a > 0.0f ? atb[t] / a : 0.0f;
        out[t] = r;
        if (r > 0.0f) {
            v = r;
            c = 1.0;
        }
    }
    const double s = block_sum<BLOCK>(v);
    const double k = block_sum<BLOCK>(c);
    if (threadIdx.x == 0) {
        part_s[blockIdx.x] = s;
        part_n[blockIdx.x] = k;
    }
}

// stats = [sum, count] of the positive voxels -> [sum, count, count / sum] (1 if none):
// the scale that brings the mean over the support to one.
__global__ void support_scale(double* stats) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        stats[2] = (stats[1] > 0.0 && stats[0] > 0.0) ? stats[1] / stats[0] : 1.0;
}

// ---------------------------------------------------------------- small helpers
// inv = 1 / s where s > 0, else 0 (the EM update's 1 / (A_i^T 1), zero off the support).
__global__ void reciprocal_on_support(const float* __restrict__ s, int64_t n,
                                      float* __restrict__ inv) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t < n) inv[t] = s[t] > 0.0f ? 1.0f / s[t] : 0.0f;
}

__global__ void fill_f64(double* __restrict__ a, int64_t n, double v) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t < n) a[t] = v;
}

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

// Domain check partials: counts of bins with b < 0 or r < 0 or mult < 0 or non-finite
// values (slot 0), and of bins whose objective term is infinite for every image:
// b > 0, r = 0 and no voxel reaches the bin (a1 = 0 there, also where mult = 0: a bin of
// zero efficiency such as a detector gap has a zero row of A) (slot 1).
__global__ void __launch_bounds__(BLOCK)
domain_check(const float* __restrict__ b, const float* __restrict__ r,
             const float* __restrict__ mult, const float* __restrict__ a1, int64_t n,
             double* __restrict__ part, int64_t nblocks) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double bad = 0.0, inf = 0.0;
    if (t < n) {
        const float bb = b[t], rr = r[t], mm = mult[t];
        if (!(bb >= 0.0f) || !(rr >= 0.0f) || !(mm >= 0.0f) || isinf(bb) || isinf(rr) ||
            isinf(mm))
            bad = 1.0;
        if (bb > 0.0f && rr == 0.0f && !(a1[t] > 0.0f)) inf = 1.0;
    }
    const double s0 = block_sum<BLOCK>(bad);
    const double s1 = block_sum<BLOCK>(inf);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0;
        part[nblocks + blockIdx.x] = s1;
    }
}

// Sum of phi_j(0) over the bins no voxel reaches ((A 1)_j = 0, given in a1): a constant
// of the objective that the duality gap leaves out (those rows are masked).
__global__ void __launch_bounds__(BLOCK)
masked_phi0(const float* __restrict__ b, const float* __restrict__ r,
            const float* __restrict__ a1, int64_t n, double* __restrict__ part) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double v = 0.0;
    if (t < n && !(a1[t] > 0.0f)) v = phi64(0.0, (double)b[t], (double)r[t]);
    const double s = block_sum<BLOCK>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Duality-gap pieces (FP64 partials): phi*(y_j) = -y r - b log(1 - y) (y <= 1; +inf
// beyond the domain) over the bins (eq. PET:CVX), and U max(0, -z_v) over the voxels.
__global__ void __launch_bounds__(BLOCK)
gap_dual(const float* __restrict__ y, const float* __restrict__ b, const float* __restrict__ r,
         int64_t n, double* __restrict__ part) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double v = 0.0;
    if (t < n) {
        const double yy = y[t], bb = b[t], rr = r[t];
        const double om = 1.0 - yy;
        if (yy > 1.0 || (bb > 0.0 && om <= 0.0))
            v = INFINITY;
        else
            v = -yy * rr - (bb > 0.0 ? bb * log(om) : 0.0);
    }
    const double s = block_sum<BLOCK>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(BLOCK)
gap_box(const float* __restrict__ z, int64_t n, double U, double* __restrict__ part) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double v = 0.0;
    if (t < n) v = U * fmax(0.0, -(double)z[t]);
    const double s = block_sum<BLOCK>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Prior dual feasibility (the conjugate of alpha ||.|| is the indicator of its dual
// ball): +inf for a voxel outside the ball by more than FP32 rounding of the projection.
__global__ void __launch_bounds__(BLOCK)
gap_prior(const float* __restrict__ q, int64_t nv, double alpha, int atv, double* __restrict__ part) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double v = 0.0;
    if (t < nv) {
        const double q0 = q[t], q1 = q[t + nv], q2 = q[t + 2 * nv];
        const double lim = alpha * (1.0 + 1e-6);
        const bool out = atv ? (fabs(q0) > lim || fabs(q1) > lim || fabs(q2) > lim)
                             : sqrt(q0 * q0 + q1 * q1 + q2 * q2) > lim;
        if (out) v = INFINITY;
    }
    const double s = block_sum<BLOCK>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out = [gap, primal, dual, box] from the objective psi = obj[0], the masked constant,
// the dual sum, the prior feasibility term and the box term.
__global__ void combine_gap(double* out, const double* obj, double c_mask, const double* dual,
                            const double* feas, const double* box) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        out[1] = obj[0] - c_mask;
        out[2] = dual[0] + feas[0];
        out[3] = box[0];
        out[0] = out[1] + out[2] + out[3];
    }
}

// Sum of squares of an image in FP64 (power iteration), and scaling by 1/sqrt(norm2).
__global__ void __launch_bounds__(BLOCK)
sumsq(const float* __restrict__ a, int64_t n, double* __restrict__ part) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double v = 0.0;
    if (t < n) v = (double)a[t] * (double)a[t];
    const double s = block_sum<BLOCK>(v);
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

// ---------------------------------------------------------------- tap counting
// Number of taps of ray (a, q, k) with a nonzero weight inside the image: the ray's
// nonzeros in the system matrix (measurement helper).
__device__ double ray_taps(const GeomDev& G, int a, int q, int k) {
    const AngleDev A = G.ang[a];
    const int g = G.plane_seg[q];
    const int p = q - G.seg_base[g];
    const double kk = kappa(G, k);
    const SegRay S = seg_ray(G, a, g, k, kk);
    const int zb = G.seg_pitch[g] * p + G.seg_off[g];
    int j0, j1;
    sec_range(A, __builtin_fma(A.du_dk, kk, A.cu), j0, j1);
    double n = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double jj = (double)j - A.cj;
        const Sample s = split(sec_coord(A, kk, jj));
        const Sample sz = split(__builtin_fma(S.ezj, jj, S.ezk));
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

__global__ void __launch_bounds__(BLOCK)
fwd_count(GeomDev G, int ang0, int ang_step, int n_ang_sub, double* __restrict__ part) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t per_ang = (int64_t)G.n_planes * G.n_rad;
    double v = 0.0;
    if (t < per_ang * n_ang_sub) {
        const int ia = (int)(t / per_ang);
        const int64_t rem = t - (int64_t)ia * per_ang;
        const int q = (int)(rem / G.n_rad);
        const int k = (int)(rem - (int64_t)q * G.n_rad);
        v = ray_taps(G, ang0 + ia * ang_step, q, k);
    }
    const double s = block_sum<BLOCK>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

}  // namespace spdhg

namespace spdhg {
// ---------------------------------------------------------------- dTV operator norm
// (-1)^(ix + iy + iz): start vector of the power iteration for difference operators.
__global__ void checkerboard_zf(PriorArgs P, float* __restrict__ out) {
    const int64_t nv = (int64_t)P.nx * P.ny * P.nz;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t >= nv) return;
    int cx, cy, cz;
    zf_coords(P, t, cx, cy, cz);
    out[t] = ((cx + cy + cz) & 1) ? -1.0f : 1.0f;
}

// out[3][v] = D_v grad x (v)
__global__ void __launch_bounds__(BLOCK)
dgrad_apply(PriorArgs P, const float* __restrict__ x, const float* __restrict__ xi,
            float* __restrict__ out) {
    const int64_t sx = P.nz, sy = (int64_t)P.nz * P.nx;
    const int64_t nv = sy * P.ny;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t >= nv) return;
    int cx, cy, cz;
    zf_coords(P, t, cx, cy, cz);
    const float xc = x[t];
    float g0 = cx < P.nx - 1 ? x[t + sx] - xc : 0.0f;
    float g1 = cy < P.ny - 1 ? x[t + sy] - xc : 0.0f;
    float g2 = cz < P.nz - 1 ? x[t + 1] - xc : 0.0f;
    const float x0 = xi[t], x1 = xi[t + nv], x2 = xi[t + 2 * nv];
    const float dot = x0 * g0 + x1 * g1 + x2 * g2;
    out[t] = g0 - P.gamma_d * dot * x0;
    out[t + nv] = g1 - P.gamma_d * dot * x1;
    out[t + 2 * nv] = g2 - P.gamma_d * dot * x2;
}

// out[v] = grad^T (D p) (v)
__global__ void __launch_bounds__(BLOCK)
dgrad_adj(PriorArgs P, const float* __restrict__ p, const float* __restrict__ xi,
          float* __restrict__ out) {
    const int64_t sx = P.nz, sy = (int64_t)P.nz * P.nx;
    const int64_t nv = sy * P.ny;
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t >= nv) return;
    int cx, cy, cz;
    zf_coords(P, t, cx, cy, cz);
    auto dp = [&](int64_t c, int comp) {
        const float x0 = xi[c], x1 = xi[c + nv], x2 = xi[c + 2 * nv];
        const float p0 = p[c], p1 = p[c + nv], p2 = p[c + 2 * nv];
        const float dot = x0 * p0 + x1 * p1 + x2 * p2;
        const float xs = comp == 0 ? x0 : (comp == 1 ? x1 : x2);
        const float ps = comp == 0 ? p0 : (comp == 1 ? p1 : p2);
        return ps - P.gamma_d * dot * xs;
    };
    float v = 0.0f;
    if (cx < P.nx - 1) v -= dp(t, 0);
    if (cy < P.ny - 1) v -= dp(t, 1);
    if (cz < P.nz - 1) v -= dp(t, 2);
    if (cx > 0) v += dp(t - sx, 0);
    if (cy > 0) v += dp(t - sy, 1);
    if (cz > 0) v += dp(t - 1, 2);
    out[t] = v;
}
}  // namespace spdhg

namespace spdhg {
}  // namespace spdhg
