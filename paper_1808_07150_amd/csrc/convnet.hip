// Warm-start network kernels: 3-D convolutions (3x3x3, zero padding) on BF16 activations
// and weights with FP32 accumulation on the MFMA units, and the element-wise pieces of
// an encoder-decoder (ReLU, 2x2x2 average pooling, nearest 2x upsampling, skip sums,
// squared-error loss, Adam).  C ABI in include/spdhg_net.h.
//
// Layouts.  Activations are channel-last [y][x][z][C] BF16 (C a multiple of 16; z is the
// fastest spatial axis, as in the reconstruction's images).  Convolution weights are
// packed as [tap][ci / 16][co][16] BF16 (tap = (dy + 1) * 9 + (dx + 1) * 3 + (dz + 1)),
// so that one MFMA B operand (16 input channels x 16 output channels of one tap) is 16
// rows of 32 contiguous bytes.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>

#include "../../include/spdhg_net.h"

namespace wsnet {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

#define NET_BLOCK 256

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Round to nearest even (finite inputs; NaN stays NaN).
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

struct Dims {
    int ny, nx, nz;
};

__device__ __forceinline__ int64_t vox(const Dims& D, int y, int x, int z) {
    return ((int64_t)y * D.nx + x) * D.nz + z;
}

typedef int i32x2 __attribute__((ext_vector_type(2)));

// v moved by one lane within each row of 16 lanes (CTRL 0x101: from the next lane, 0x111:
// from the previous one); the row's end lane that has no source takes `edge`.
template <int CTRL>
__device__ __forceinline__ bf16x4 row_shift(bf16x4 v, bf16x4 edge) {
    const i32x2 vi = __builtin_bit_cast(i32x2, v), ei = __builtin_bit_cast(i32x2, edge);
    i32x2 r;
    r.x = __builtin_amdgcn_update_dpp(ei.x, vi.x, CTRL, 0xF, 0xF, false);
    r.y = __builtin_amdgcn_update_dpp(ei.y, vi.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(bf16x4, r);
}

// ---------------------------------------------------------------- convolution forward
// One wavefront per output tile of 16 consecutive z x 4 consecutive x at one y, all COUT
// channels: four M blocks (one per x) times COUT / 16 N blocks of 16x16 FP32 accumulators.
// For every tap and 16-channel input chunk, A (16 voxels x 16 input channels) comes
// straight from the channel-last activations (8 bytes per lane; each input column is read
// once per (dy, dz) for all three dx) and B from the packed weights; both are cached
// reads shared by neighbouring tiles.  Epilogue: + bias, optional
// ReLU, BF16 store.
template <int CIN, int COUT>
__global__ void __launch_bounds__(NET_BLOCK)
conv3d_fwd(Dims D, const uint16_t* __restrict__ in, const uint16_t* __restrict__ w,
           const float* __restrict__ bias, int relu, uint16_t* __restrict__ out) {
    constexpr int NB = COUT / 16, KC = CIN / 16;
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * (NET_BLOCK / 64)) + (threadIdx.x >> 6);
    const int nzt = (D.nz + 15) / 16, nxt = (D.nx + 3) / 4;
    const int ntiles = D.ny * nxt * nzt;
    if (wave >= ntiles) return;
    const int zt = wave % nzt;
    const int rest = wave / nzt;
    const int xt = rest % nxt, y = rest / nxt;
    const int z0 = zt * 16, x0 = xt * 4;
    const int i = lane & 15;         // voxel row of A (z offset) / output channel column
    const int kq = (lane >> 4) * 4;  // first of the four K entries this lane holds
    f32x4 acc[4][NB];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int n = 0; n < NB; ++n) acc[s][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    // per dy: the six input columns x0 - 1 .. x0 + 4 are loaded once (the tile's 16 z,
    // plus z0 - 1 and z0 + 16 in the first and last lane of each 16-lane row) and serve
    // all nine (dz, dx) taps of the four output columns: the dz = -1 / +1 operands are the
    // centre ones moved by one lane within each row (DPP row shifts), whose end lanes take
    // the extra voxel
    for (int dy = -1; dy <= 1; ++dy) {
        const int yy = y + dy;
        const bool oky = yy >= 0 && yy < D.ny;
        const int zc = z0 + i;
        const int ze = i == 0 ? z0 - 1 : z0 + 16;  // used by lanes with i == 0 or i == 15
        const bool edge = i == 0 || i == 15;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            bf16x4 ac[6], ae[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const int xx = x0 + q - 1;
                const bool okx = oky && xx >= 0 && xx < D.nx;
                ac[q] = bf16x4{0, 0, 0, 0};
                ae[q] = bf16x4{0, 0, 0, 0};
                if (okx && zc < D.nz)
                    ac[q] = *(const bf16x4*)(in + vox(D, yy, xx, zc) * CIN + kc * 16 + kq);
                if (okx && edge && ze >= 0 && ze < D.nz)
                    ae[q] = *(const bf16x4*)(in + vox(D, yy, xx, ze) * CIN + kc * 16 + kq);
            }
#pragma unroll
            for (int dz = -1; dz <= 1; ++dz) {
                bf16x4 a[6];
#pragma unroll
                for (int q = 0; q < 6; ++q)
                    a[q] = dz == 0 ? ac[q] : dz > 0 ? row_shift<0x101>(ac[q], ae[q])
                                                    : row_shift<0x111>(ac[q], ae[q]);
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int t = (dy + 1) * 9 + (dx + 1) * 3 + (dz + 1);
                    bf16x4 b[NB];
#pragma unroll
                    for (int n = 0; n < NB; ++n) {
                        const uint16_t* wp =
                            w + (((int64_t)(t * KC + kc) * COUT + n * 16 + i) * 16 + kq);
                        b[n] = *(const bf16x4*)wp;
                    }
#pragma unroll
                    for (int s = 0; s < 4; ++s)
#pragma unroll
                        for (int n = 0; n < NB; ++n)
                            acc[s][n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                                a[s + dx + 1], b[n], acc[s][n], 0, 0, 0);
                }
            }
        }
    }
    // D[i][n] of a 16x16 block: lane holds rows kq .. kq + 3 (z) of column i (channel)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int x = x0 + s;
        if (x >= D.nx) continue;
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const int co = n * 16 + i;
            const float bb = bias ? bias[co] : 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int z = z0 + kq + j;
                if (z >= D.nz) continue;
                float v = acc[s][n][j] + bb;
                if (relu) v = fmaxf(v, 0.0f);
                out[vox(D, y, x, z) * COUT + co] = f2bf(v);
            }
        }
    }
}

// Packed weights of the input-gradient convolution: the adjoint of a 3x3x3 convolution
// is the convolution with the channel roles exchanged and the taps mirrored.
__global__ void conv3d_adjoint_weights(int cin, int cout, const uint16_t* __restrict__ w,
                                       uint16_t* __restrict__ wt) {
    const int64_t n = 27LL * cin * cout;
    const int64_t e = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    if (e >= n) return;
    // destination [t'][co / 16][ci][co % 16] of the (cin' = cout, cout' = cin) convolution
    const int cq = (int)(e % 16);
    int64_t r = e / 16;
    const int ci = (int)(r % cin);
    r /= cin;
    const int cchunk = (int)(r % (cout / 16));
    const int tp = (int)(r / (cout / 16));
    const int co = cchunk * 16 + cq;
    const int t = 26 - tp;  // mirrored tap
    wt[e] = w[(((int64_t)t * (cin / 16) + ci / 16) * cout + co) * 16 + ci % 16];
}

// ---------------------------------------------------------------- weight gradient
// dW[t][ci][co] = sum_v dout[v][co] in[v + off_t][ci]: per (tap, voxel chunk) one
// wavefront accumulates the COUT x CIN block with MFMA over 16 voxels per step
// (A = dout^T: 16 output channels x 16 voxels, B = in: 16 voxels x 16 input channels)
// and writes its FP32 partial; a second kernel adds the chunks in a fixed order.
template <int CIN, int COUT>
__global__ void __launch_bounds__(64)
conv3d_wgrad_part(Dims D, const uint16_t* __restrict__ in, const uint16_t* __restrict__ dout,
                  int chunk, float* __restrict__ part) {
    constexpr int MB = COUT / 16, NB = CIN / 16;
    const int lane = threadIdx.x;
    const int t = blockIdx.x % 27;
    const int c = blockIdx.x / 27;
    const int dy = t / 9 - 1, dx = (t / 3) % 3 - 1, dz = t % 3 - 1;
    const int64_t nv = (int64_t)D.ny * D.nx * D.nz;
    const int64_t v0 = (int64_t)c * chunk;
    const int64_t v1 = v0 + chunk < nv ? v0 + chunk : nv;
    const int i = lane & 15, kq = (lane >> 4) * 4;
    f32x4 acc[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t vb = v0; vb < v1; vb += 16) {
        // the four voxels of this lane's K entries and their shifted input voxels
        int64_t vv[4], vin[4];
        bool ok[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t v = vb + kq + j;
            vv[j] = v;
            ok[j] = v < v1;
            int64_t r = v < v1 ? v : v0;
            const int z = (int)(r % D.nz);
            r /= D.nz;
            const int x = (int)(r % D.nx), y = (int)(r / D.nx);
            const int yy = y + dy, xx = x + dx, zz = z + dz;
            ok[j] = ok[j] && yy >= 0 && yy < D.ny && xx >= 0 && xx < D.nx && zz >= 0 && zz < D.nz;
            vin[j] = ok[j] ? vox(D, yy, xx, zz) : 0;
        }
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            bf16x4 a;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                a[j] = ok[j] ? (short)dout[vv[j] * COUT + m * 16 + i] : (short)0;
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                bf16x4 b;
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = ok[j] ? (short)in[vin[j] * CIN + n * 16 + i] : (short)0;
                acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[m][n], 0, 0, 0);
            }
        }
    }
    // acc[m][n] holds rows (co) m*16 + kq + j, column (ci) n*16 + i
    float* p = part + ((int64_t)c * 27 + t) * COUT * CIN;
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int j = 0; j < 4; ++j) p[(m * 16 + kq + j) * CIN + n * 16 + i] = acc[m][n][j];
}

// Sum of the chunk partials in chunk order; dW in FP32 [t][co][ci].
__global__ void conv3d_wgrad_sum(int nchunk, int64_t per, const float* __restrict__ part,
                                 float* __restrict__ dw) {
    const int64_t e = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    if (e >= per) return;
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * per + e];
    dw[e] = s;
}

// Bias gradient: sum over voxels of dout[v][co] (FP32 partials per block, then fixed-order sum).
__global__ void bias_grad_part(int64_t nv, int cout, const uint16_t* __restrict__ dout,
                               float* __restrict__ part) {
    // block b sums voxels [b * 1024, (b + 1) * 1024) for every channel: thread = channel lane
    const int64_t v0 = (int64_t)blockIdx.x * 1024;
    for (int co = threadIdx.x; co < cout; co += NET_BLOCK) {
        float s = 0.0f;
        for (int64_t v = v0; v < v0 + 1024 && v < nv; ++v) s += bf2f(dout[v * cout + co]);
        part[(int64_t)blockIdx.x * cout + co] = s;
    }
}

__global__ void bias_grad_sum(int nblk, int cout, const float* __restrict__ part, float* __restrict__ db) {
    const int co = blockIdx.x * NET_BLOCK + threadIdx.x;
    if (co >= cout) return;
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * cout + co];
    db[co] = s;
}

// ---------------------------------------------------------------- element-wise pieces
// dy *= (y > 0): the ReLU derivative taken from the layer's output.
__global__ void relu_bwd(int64_t n, const uint16_t* __restrict__ y, uint16_t* __restrict__ dy) {
    const int64_t e = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    if (e < n && !(bf2f(y[e]) > 0.0f)) dy[e] = 0;
}

// out = a + b (BF16, rounded once).
__global__ void add_bf16(int64_t n, const uint16_t* __restrict__ a, const uint16_t* __restrict__ b,
                         uint16_t* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    if (e < n) out[e] = f2bf(bf2f(a[e]) + bf2f(b[e]));
}

// The same eight elements (16 bytes) per thread, for 16-byte aligned arrays; elements
// from 8 * n8 on are left to add_bf16.
__global__ void add_bf16_v8(int64_t n8, const uint4* __restrict__ a, const uint4* __restrict__ b,
                            uint4* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    if (e >= n8) return;
    const uint4 va = a[e], vb = b[e];
    const uint32_t* pa = (const uint32_t*)&va;
    const uint32_t* pb = (const uint32_t*)&vb;
    uint4 vo;
    uint32_t* po = (uint32_t*)&vo;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint16_t lo = f2bf(bf2f((uint16_t)(pa[k] & 0xFFFFu)) + bf2f((uint16_t)(pb[k] & 0xFFFFu)));
        const uint16_t hi = f2bf(bf2f((uint16_t)(pa[k] >> 16)) + bf2f((uint16_t)(pb[k] >> 16)));
        po[k] = (uint32_t)lo | ((uint32_t)hi << 16);
    }
    out[e] = vo;
}

// 2x2x2 average pooling (the fine grid has even sizes) and its adjoint (each fine voxel
// receives 1/8 of its coarse voxel's gradient).
__global__ void pool2_fwd(Dims F, int C, const uint16_t* __restrict__ in, uint16_t* __restrict__ out) {
    const Dims Cd{F.ny / 2, F.nx / 2, F.nz / 2};
    const int64_t n = (int64_t)Cd.ny * Cd.nx * Cd.nz * C;
    const int64_t e = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    if (e >= n) return;
    const int c = (int)(e % C);
    int64_t r = e / C;
    const int z = (int)(r % Cd.nz);
    r /= Cd.nz;
    const int x = (int)(r % Cd.nx), y = (int)(r / Cd.nx);
    float s = 0.0f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int d = 0; d < 2; ++d) s += bf2f(in[vox(F, 2 * y + a, 2 * x + b, 2 * z + d) * C + c]);
    out[e] = f2bf(0.125f * s);
}

__global__ void pool2_bwd(Dims F, int C, const uint16_t* __restrict__ dout, uint16_t* __restrict__ din) {
    const Dims Cd{F.ny / 2, F.nx / 2, F.nz / 2};
    const int64_t n = (int64_t)F.ny * F.nx * F.nz * C;
    const int64_t e = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    if (e >= n) return;
    const int c = (int)(e % C);
    int64_t r = e / C;
    const int z = (int)(r % F.nz);
    r /= F.nz;
    const int x = (int)(r % F.nx), y = (int)(r / F.nx);
    din[e] = f2bf(0.125f * bf2f(dout[vox(Cd, y / 2, x / 2, z / 2) * C + c]));
}

// Nearest 2x upsampling and its adjoint (sum of the eight fine voxels).
// Eight channels (16 bytes) per thread: C is a multiple of 16 and channel-last rows are
// 16-byte aligned.
__global__ void up2_fwd(Dims F, int C, const uint16_t* __restrict__ in, uint16_t* __restrict__ out) {
    const Dims Cd{F.ny / 2, F.nx / 2, F.nz / 2};
    const int C8 = C / 8;
    const int64_t n = (int64_t)F.ny * F.nx * F.nz * C8;
    const int64_t e = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    if (e >= n) return;
    const int c8 = (int)(e % C8);
    int64_t r = e / C8;
    const int z = (int)(r % F.nz);
    r /= F.nz;
    const int x = (int)(r % F.nx), y = (int)(r / F.nx);
    ((uint4*)out)[e] = ((const uint4*)in)[vox(Cd, y / 2, x / 2, z / 2) * C8 + c8];
}

__global__ void up2_bwd(Dims F, int C, const uint16_t* __restrict__ dout, uint16_t* __restrict__ din) {
    const Dims Cd{F.ny / 2, F.nx / 2, F.nz / 2};
    const int64_t n = (int64_t)Cd.ny * Cd.nx * Cd.nz * C;
    const int64_t e = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    if (e >= n) return;
    const int c = (int)(e % C);
    int64_t r = e / C;
    const int z = (int)(r % Cd.nz);
    r /= Cd.nz;
    const int x = (int)(r % Cd.nx), y = (int)(r / Cd.nx);
    float s = 0.0f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int d = 0; d < 2; ++d) s += bf2f(dout[vox(F, 2 * y + a, 2 * x + b, 2 * z + d) * C + c]);
    din[e] = f2bf(s);
}

// Image (z-fastest FP32, one channel) -> 16-channel BF16 activations (channel 0 = scale *
// image, the rest zero), and channel 0 of the network output + the input image -> image.
__global__ void image_to_act(int64_t nv, float scale, const float* __restrict__ img,
                             uint16_t* __restrict__ act) {
    const int64_t e = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    if (e >= nv * 16) return;
    const int c = (int)(e % 16);
    act[e] = c == 0 ? f2bf(scale * img[e / 16]) : (uint16_t)0;
}

// The same, one voxel (16 channels, 32 bytes) per thread for a 16-byte aligned `act`.
__global__ void image_to_act_v(int64_t nv, float scale, const float* __restrict__ img,
                               uint4* __restrict__ act) {
    const int64_t v = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    if (v >= nv) return;
    act[2 * v] = make_uint4((uint32_t)f2bf(scale * img[v]), 0u, 0u, 0u);
    act[2 * v + 1] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void act_to_image(int64_t nv, float scale, const uint16_t* __restrict__ act, int cact,
                             const float* __restrict__ skip, float* __restrict__ img) {
    const int64_t v = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    if (v >= nv) return;
    img[v] = (bf2f(act[v * cact]) + (skip ? skip[v] * scale : 0.0f)) / scale;
}

// Squared-error loss 0.5 sum (pred - target)^2 over channel 0 (FP64 partials) and its
// gradient written into channel 0 of a zeroed C-channel BF16 tensor.
__global__ void mse_grad(int64_t nv, int cact, const uint16_t* __restrict__ pred,
                         const float* __restrict__ skip, const float* __restrict__ target,
                         float scale, uint16_t* __restrict__ grad, double* __restrict__ part) {
    __shared__ double red[NET_BLOCK];
    const int64_t v = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    double l = 0.0;
    if (v < nv) {
        const float p = bf2f(pred[v * cact]) + (skip ? scale * skip[v] : 0.0f);
        const float r = p - scale * target[v];
        l = 0.5 * (double)r * (double)r;
        grad[v * cact] = f2bf(r);
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = NET_BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Adam on FP32 master parameters, with the BF16 copy of the weights refreshed.
__global__ void adam_step(int64_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                          float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                          const float* __restrict__ g, uint16_t* __restrict__ p16) {
    const int64_t e = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    if (e >= n) return;
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.0f - b1) * gg;
    const float vv = b2 * v[e] + (1.0f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    const float pn = p[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    p[e] = pn;
    if (p16) p16[e] = f2bf(pn);
}

// FP32 [t][co][ci] <-> packed BF16 [t][ci/16][co][16].
__global__ void pack_weights(int cin, int cout, const float* __restrict__ w32, uint16_t* __restrict__ w16) {
    const int64_t n = 27LL * cin * cout;
    const int64_t e = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    if (e >= n) return;
    const int ci = (int)(e % cin);
    int64_t r = e / cin;
    const int co = (int)(r % cout);
    const int t = (int)(r / cout);
    w16[(((int64_t)t * (cin / 16) + ci / 16) * cout + co) * 16 + ci % 16] = f2bf(w32[e]);
}

// Zero fill of n 16-bit values (a kernel rather than a memset node: safe under graph capture).
__global__ void fill_zero_u16(int64_t n, uint16_t* __restrict__ a) {
    const int64_t t = (int64_t)blockIdx.x * NET_BLOCK + threadIdx.x;
    if (t < n) a[t] = 0;
}

// out[0] = sum of n FP64 partials in a fixed order (one block: strided per-thread sums,
// then the threads' sums in index order).
__global__ void sum_parts(const double* __restrict__ part, int64_t n, double* __restrict__ out) {
    __shared__ double s[256];
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) v += part[i];
    s[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < 256; ++i) t += s[i];
        out[0] = t;
    }
}

}  // namespace wsnet

// ====================================================================== C ABI
namespace {
using namespace wsnet;

thread_local char net_err[256] = "";
int net_fail(int code, const char* msg) {
    snprintf(net_err, sizeof(net_err), "%s", msg);
    return code;
}
int64_t nblk(int64_t n) { return (n + NET_BLOCK - 1) / NET_BLOCK; }

bool channels_ok(int c) { return c == 16 || c == 32 || c == 64; }

#define NET_CHECK()                                                     \
    do {                                                                \
        hipError_t e_ = hipGetLastError();                              \
        if (e_ != hipSuccess) return net_fail(-4, hipGetErrorString(e_)); \
    } while (0)

template <int CI, int CO>
void fwd_launch(Dims D, const uint16_t* in, const uint16_t* w, const float* b, int relu,
                uint16_t* out, hipStream_t st) {
    const int64_t tiles = (int64_t)D.ny * ((D.nx + 3) / 4) * ((D.nz + 15) / 16);
    conv3d_fwd<CI, CO><<<(tiles + 3) / 4, NET_BLOCK, 0, st>>>(D, in, w, b, relu, out);
}

template <int CI, int CO>
void wgrad_launch(Dims D, const uint16_t* in, const uint16_t* dout, int chunk, int nchunk,
                  float* part, hipStream_t st) {
    conv3d_wgrad_part<CI, CO><<<27 * nchunk, 64, 0, st>>>(D, in, dout, chunk, part);
}

#define NET_DISPATCH(CI, CO, CALL)                                                 \
    switch (CI * 1000 + CO) {                                                      \
        case 16016: CALL(16, 16); break;                                           \
        case 16032: CALL(16, 32); break;                                           \
        case 32016: CALL(32, 16); break;                                           \
        case 32032: CALL(32, 32); break;                                           \
        case 32064: CALL(32, 64); break;                                           \
        case 64032: CALL(64, 32); break;                                           \
        case 64064: CALL(64, 64); break;                                           \
        case 16064: CALL(16, 64); break;                                           \
        case 64016: CALL(64, 16); break;                                           \
        default: return net_fail(-2, "unsupported channel pair");                  \
    }

}  // namespace

extern "C" {

const char* spdhg_net_last_error(void) { return net_err; }

int spdhg_conv3d_fwd(const int32_t dims[3], int32_t cin, int32_t cout, const uint16_t* in,
                     const uint16_t* w, const float* bias, int32_t relu, uint16_t* out, void* stream) {
    if (!dims || !in || !w || !out) return net_fail(-1, "NULL argument");
    if (!channels_ok(cin) || !channels_ok(cout)) return net_fail(-2, "channels must be 16, 32 or 64");
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return net_fail(-2, "empty volume");
    const Dims D{dims[0], dims[1], dims[2]};
    hipStream_t st = (hipStream_t)stream;
#define FWD_CALL(A, B) fwd_launch<A, B>(D, in, w, bias, relu, out, st)
    NET_DISPATCH(cin, cout, FWD_CALL)
#undef FWD_CALL
    NET_CHECK();
    return 0;
}

int spdhg_conv3d_adjoint_weights(int32_t cin, int32_t cout, const uint16_t* w, uint16_t* wt,
                                 void* stream) {
    if (!w || !wt) return net_fail(-1, "NULL argument");
    if (!channels_ok(cin) || !channels_ok(cout)) return net_fail(-2, "channels must be 16, 32 or 64");
    conv3d_adjoint_weights<<<nblk(27LL * cin * cout), NET_BLOCK, 0, (hipStream_t)stream>>>(cin, cout, w, wt);
    NET_CHECK();
    return 0;
}

int spdhg_conv3d_wgrad(const int32_t dims[3], int32_t cin, int32_t cout, const uint16_t* in,
                       const uint16_t* dout, int32_t chunk, float* part, int64_t part_floats,
                       float* dw, float* dbias, void* stream) {
    if (!dims || !in || !dout || !part || !dw) return net_fail(-1, "NULL argument");
    if (!channels_ok(cin) || !channels_ok(cout)) return net_fail(-2, "channels must be 16, 32 or 64");
    if (chunk < 16 || chunk % 16) return net_fail(-1, "chunk must be a positive multiple of 16");
    const Dims D{dims[0], dims[1], dims[2]};
    const int64_t nv = (int64_t)D.ny * D.nx * D.nz;
    const int64_t nchunk = (nv + chunk - 1) / chunk;
    const int64_t per = 27LL * cin * cout;
    const int64_t bblk = (nv + 1023) / 1024;
    if (nchunk * per > part_floats || bblk * cout > part_floats)
        return net_fail(-5, "partials buffer too small");
    if (nchunk > 65535) return net_fail(-2, "too many voxel chunks");
    hipStream_t st = (hipStream_t)stream;
#define WG_CALL(A, B) wgrad_launch<A, B>(D, in, dout, chunk, (int)nchunk, part, st)
    NET_DISPATCH(cin, cout, WG_CALL)
#undef WG_CALL
    conv3d_wgrad_sum<<<nblk(per), NET_BLOCK, 0, st>>>((int)nchunk, per, part, dw);
    if (dbias) {
        bias_grad_part<<<bblk, NET_BLOCK, 0, st>>>(nv, cout, dout, part);
        bias_grad_sum<<<nblk(cout), NET_BLOCK, 0, st>>>((int)bblk, cout, part, dbias);
    }
    NET_CHECK();
    return 0;
}

int spdhg_net_relu_bwd(int64_t n, const uint16_t* y, uint16_t* dy, void* stream) {
    if (!y || !dy || n < 0) return net_fail(-1, "bad argument");
    if (n) relu_bwd<<<nblk(n), NET_BLOCK, 0, (hipStream_t)stream>>>(n, y, dy);
    NET_CHECK();
    return 0;
}

int spdhg_net_add(int64_t n, const uint16_t* a, const uint16_t* b, uint16_t* out, void* stream) {
    if (!a || !b || !out || n < 0) return net_fail(-1, "bad argument");
    const bool aligned = (((uintptr_t)a | (uintptr_t)b | (uintptr_t)out) & 15) == 0;
    const int64_t n8 = aligned ? n / 8 : 0;
    if (n8)
        add_bf16_v8<<<nblk(n8), NET_BLOCK, 0, (hipStream_t)stream>>>(
            n8, (const uint4*)a, (const uint4*)b, (uint4*)out);
    if (n > 8 * n8)
        add_bf16<<<nblk(n - 8 * n8), NET_BLOCK, 0, (hipStream_t)stream>>>(
            n - 8 * n8, a + 8 * n8, b + 8 * n8, out + 8 * n8);
    NET_CHECK();
    return 0;
}

int spdhg_net_pool2(const int32_t fine[3], int32_t c, int32_t adjoint, const uint16_t* src,
                    uint16_t* dst, void* stream) {
    if (!fine || !src || !dst) return net_fail(-1, "NULL argument");
    if (fine[0] % 2 || fine[1] % 2 || fine[2] % 2) return net_fail(-2, "fine grid must be even");
    const Dims F{fine[0], fine[1], fine[2]};
    const int64_t nf = (int64_t)F.ny * F.nx * F.nz * c;
    hipStream_t st = (hipStream_t)stream;
    if (adjoint)
        pool2_bwd<<<nblk(nf), NET_BLOCK, 0, st>>>(F, c, src, dst);
    else
        pool2_fwd<<<nblk(nf / 8), NET_BLOCK, 0, st>>>(F, c, src, dst);
    NET_CHECK();
    return 0;
}

int spdhg_net_up2(const int32_t fine[3], int32_t c, int32_t adjoint, const uint16_t* src,
                  uint16_t* dst, void* stream) {
    if (!fine || !src || !dst) return net_fail(-1, "NULL argument");
    if (fine[0] % 2 || fine[1] % 2 || fine[2] % 2) return net_fail(-2, "fine grid must be even");
    const Dims F{fine[0], fine[1], fine[2]};
    const int64_t nf = (int64_t)F.ny * F.nx * F.nz * c;
    hipStream_t st = (hipStream_t)stream;
    if (c <= 0 || c % 16) return net_fail(-2, "channel count must be a multiple of 16");
    if (adjoint)
        up2_bwd<<<nblk(nf / 8), NET_BLOCK, 0, st>>>(F, c, src, dst);
    else
        up2_fwd<<<nblk(nf / 8), NET_BLOCK, 0, st>>>(F, c, src, dst);
    NET_CHECK();
    return 0;
}

int spdhg_net_image_to_act(int64_t nv, float scale, const float* img, uint16_t* act, void* stream) {
    if (!img || !act) return net_fail(-1, "NULL argument");
    if (((uintptr_t)act & 15) == 0)
        image_to_act_v<<<nblk(nv), NET_BLOCK, 0, (hipStream_t)stream>>>(nv, scale, img, (uint4*)act);
    else
        image_to_act<<<nblk(nv * 16), NET_BLOCK, 0, (hipStream_t)stream>>>(nv, scale, img, act);
    NET_CHECK();
    return 0;
}

int spdhg_net_act_to_image(int64_t nv, float scale, const uint16_t* act, int32_t cact,
                           const float* skip, float* img, void* stream) {
    if (!act || !img || !(scale > 0)) return net_fail(-1, "bad argument");
    act_to_image<<<nblk(nv), NET_BLOCK, 0, (hipStream_t)stream>>>(nv, scale, act, cact, skip, img);
    NET_CHECK();
    return 0;
}

int spdhg_net_mse_grad(int64_t nv, int32_t cact, const uint16_t* pred, const float* skip,
                       const float* target, float scale, uint16_t* grad, double* part,
                       void* stream) {
    if (!pred || !target || !grad || !part) return net_fail(-1, "NULL argument");
    mse_grad<<<nblk(nv), NET_BLOCK, 0, (hipStream_t)stream>>>(nv, cact, pred, skip, target, scale,
                                                             grad, part);
    NET_CHECK();
    return 0;
}

int spdhg_net_adam(int64_t n, float lr, float b1, float b2, float eps, int64_t step, float* p,
                   float* m, float* v, const float* g, uint16_t* p16, void* stream) {
    if (!p || !m || !v || !g || step < 1) return net_fail(-1, "bad argument");
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    adam_step<<<nblk(n), NET_BLOCK, 0, (hipStream_t)stream>>>(n, lr, b1, b2, eps, c1, c2, p, m, v, g, p16);
    NET_CHECK();
    return 0;
}

int spdhg_net_pack_weights(int32_t cin, int32_t cout, const float* w32, uint16_t* w16, void* stream) {
    if (!w32 || !w16) return net_fail(-1, "NULL argument");
    if (!channels_ok(cin) || !channels_ok(cout)) return net_fail(-2, "channels must be 16, 32 or 64");
    pack_weights<<<nblk(27LL * cin * cout), NET_BLOCK, 0, (hipStream_t)stream>>>(cin, cout, w32, w16);
    NET_CHECK();
    return 0;
}

// ---------------------------------------------------------------- the network as a whole
// Encoder-decoder of 11 3x3x3 convolutions (channels 16/32/64, three resolutions):
//   e1 = relu(c2(relu(c1(in))));  e2 = relu(c4(relu(c3(pool e1))));
//   b = relu(c6(relu(c5(pool e2))));  d2 = relu(c8(relu(c7(up b)) + e2));
//   d1 = relu(c10(relu(c9(up d2)) + e1));  image = in + channel 0 of c11(d1) (linear).
static const int WS_CI[11] = {16, 16, 16, 32, 32, 64, 64, 32, 32, 16, 16};
static const int WS_CO[11] = {16, 16, 32, 32, 64, 64, 32, 32, 16, 16, 16};
static const int WS_RELU[11] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 0};
static const int WS_LEVEL[11] = {0, 0, 1, 1, 2, 2, 1, 1, 0, 0, 0};  // resolution of the layer's input
constexpr int WS_CHUNK = 4096;  // voxel chunk of the weight-gradient partials

}  // extern "C"

namespace {

// Offsets (in elements) of layer l's FP32 weights [27][co][ci] and bias [co] in the FP32
// parameter blob, and of its packed BF16 weights in the BF16 blob.
struct WsParams {
    int64_t w32[11], b32[11], w16[11], n32 = 0, n16 = 0;
    WsParams() {
        for (int l = 0; l < 11; ++l) {
            const int64_t nw = 27LL * WS_CI[l] * WS_CO[l];
            w32[l] = n32;
            b32[l] = n32 + nw;
            n32 += nw + WS_CO[l];
            w16[l] = n16;
            n16 += nw;
        }
    }
};

// Workspace carving: activations (and with train, gradients and partials), 256-byte aligned.
struct WsLayout {
    // activations: in c1 e1 p1 c3 e2 p2 c5 b u2 c7 s2 d2 u1 c9 s1 d1 out
    size_t act[18];
    // gradients
    size_t gout, g10, g9in, g9, g9u, g8, g7in, g7, g7u, g6, g5, g5p, g5s, g4, g3, g3p, g3s, g2;
    size_t wt, part, grads, lparts, total;
    int64_t part_floats, nv;
    int32_t dims[3][3];  // per level: ny, nx, nz
};

int ws_dims_ok(const int32_t d[3]) {
    return d && d[0] >= 4 && d[1] >= 4 && d[2] >= 4 && d[0] % 4 == 0 && d[1] % 4 == 0 &&
           d[2] % 4 == 0;
}

WsLayout ws_layout(const int32_t dims[3], bool train) {
    WsLayout L{};
    for (int lv = 0; lv < 3; ++lv)
        for (int a = 0; a < 3; ++a) L.dims[lv][a] = dims[a] >> lv;
    const int64_t nv = (int64_t)dims[0] * dims[1] * dims[2];
    L.nv = nv;
    const int64_t n[3] = {nv, nv / 8, nv / 64};
    size_t off = 0;
    auto take = [&](int64_t elems, int bytes_each) {
        const size_t o = off;
        off += ((size_t)elems * bytes_each + 255) & ~(size_t)255;
        return o;
    };
    // level and channels of each activation, in the order of the comment above
    const int lvl[18] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 1, 1, 1, 1, 0, 0, 0, 0, 0};
    const int ch[18] = {16, 16, 16, 16, 32, 32, 32, 64, 64, 64, 32, 32, 32, 32, 16, 16, 16, 16};
    for (int i = 0; i < 18; ++i) L.act[i] = take(n[lvl[i]] * ch[i], 2);
    if (train) {
        L.gout = take(n[0] * 16, 2);
        L.g10 = take(n[0] * 16, 2);
        L.g9in = take(n[0] * 16, 2);
        L.g9 = take(n[0] * 32, 2);
        L.g9u = take(n[1] * 32, 2);
        L.g8 = take(n[1] * 32, 2);
        L.g7in = take(n[1] * 32, 2);
        L.g7 = take(n[1] * 64, 2);
        L.g7u = take(n[2] * 64, 2);
        L.g6 = take(n[2] * 64, 2);
        L.g5 = take(n[2] * 32, 2);
        L.g5p = take(n[1] * 32, 2);
        L.g5s = take(n[1] * 32, 2);
        L.g4 = take(n[1] * 32, 2);
        L.g3 = take(n[1] * 16, 2);
        L.g3p = take(n[0] * 16, 2);
        L.g3s = take(n[0] * 16, 2);
        L.g2 = take(n[0] * 16, 2);
        L.wt = take(27LL * 64 * 64, 2);
        int64_t pf = 0;
        for (int l = 0; l < 11; ++l) {
            const int64_t nvl = n[WS_LEVEL[l]];
            pf = std::max<int64_t>(pf, std::max<int64_t>((nvl + WS_CHUNK - 1) / WS_CHUNK * 27 *
                                                             WS_CI[l] * WS_CO[l],
                                                         (nvl + 1023) / 1024 * WS_CO[l]));
        }
        L.part_floats = pf;
        L.part = take(pf, 4);
        L.grads = take(WsParams().n32, 4);
        L.lparts = take((nv + 255) / 256, 8);
    }
    L.total = off;
    return L;
}

#define WS_TRY(call)                \
    do {                            \
        const int rc_ = (call);     \
        if (rc_ != 0) return rc_;   \
    } while (0)

// The forward pass into the workspace's activations (A[i] as in WsLayout::act).
int ws_forward(const WsLayout& L, char* w, const uint16_t* w16, const float* p32, float scale,
               const float* img, float* out, hipStream_t st) {
    static const WsParams PR;
    uint16_t* A[18];
    for (int i = 0; i < 18; ++i) A[i] = (uint16_t*)(w + L.act[i]);
    const int32_t* D0 = L.dims[0];
    const int32_t* D1 = L.dims[1];
    const int32_t* D2 = L.dims[2];
    auto conv = [&](int l, const int32_t* D, const uint16_t* in, uint16_t* o) {
        return spdhg_conv3d_fwd(D, WS_CI[l], WS_CO[l], in, w16 + PR.w16[l], p32 + PR.b32[l],
                                WS_RELU[l], o, st);
    };
    WS_TRY(spdhg_net_image_to_act(L.nv, scale, img, A[0], st));
    WS_TRY(conv(0, D0, A[0], A[1]));
    WS_TRY(conv(1, D0, A[1], A[2]));
    WS_TRY(spdhg_net_pool2(D0, 16, 0, A[2], A[3], st));
    WS_TRY(conv(2, D1, A[3], A[4]));
    WS_TRY(conv(3, D1, A[4], A[5]));
    WS_TRY(spdhg_net_pool2(D1, 32, 0, A[5], A[6], st));
    WS_TRY(conv(4, D2, A[6], A[7]));
    WS_TRY(conv(5, D2, A[7], A[8]));
    WS_TRY(spdhg_net_up2(D1, 64, 0, A[8], A[9], st));
    WS_TRY(conv(6, D1, A[9], A[10]));
    WS_TRY(spdhg_net_add(L.nv / 8 * 32, A[10], A[5], A[11], st));
    WS_TRY(conv(7, D1, A[11], A[12]));
    WS_TRY(spdhg_net_up2(D0, 32, 0, A[12], A[13], st));
    WS_TRY(conv(8, D0, A[13], A[14]));
    WS_TRY(spdhg_net_add(L.nv * 16, A[14], A[2], A[15], st));
    WS_TRY(conv(9, D0, A[15], A[16]));
    WS_TRY(conv(10, D0, A[16], A[17]));
    if (out) WS_TRY(spdhg_net_act_to_image(L.nv, scale, A[17], 16, img, out, st));
    return 0;
}

}  // namespace

extern "C" {

int spdhg_ws_param_count(int64_t* n32, int64_t* n16) {
    if (!n32 || !n16) return net_fail(-1, "NULL argument");
    static const WsParams PR;
    *n32 = PR.n32;
    *n16 = PR.n16;
    return 0;
}

int spdhg_ws_param_offsets(int32_t layer, int64_t* w32, int64_t* b32, int64_t* w16) {
    if (layer < 0 || layer > 10 || !w32 || !b32 || !w16) return net_fail(-1, "bad argument");
    static const WsParams PR;
    *w32 = PR.w32[layer];
    *b32 = PR.b32[layer];
    *w16 = PR.w16[layer];
    return 0;
}

int spdhg_ws_workspace_bytes(const int32_t dims[3], int32_t train, size_t* bytes) {
    if (!bytes) return net_fail(-1, "NULL argument");
    if (!ws_dims_ok(dims)) return net_fail(-2, "volume sizes must be positive multiples of 4");
    *bytes = ws_layout(dims, train != 0).total;
    return 0;
}

int spdhg_ws_pack(const float* p32, uint16_t* w16, void* stream) {
    if (!p32 || !w16) return net_fail(-1, "NULL argument");
    static const WsParams PR;
    for (int l = 0; l < 11; ++l)
        WS_TRY(spdhg_net_pack_weights(WS_CI[l], WS_CO[l], p32 + PR.w32[l], w16 + PR.w16[l], stream));
    return 0;
}

int spdhg_ws_infer(const int32_t dims[3], const float* p32, const uint16_t* w16, float scale,
                   const float* img, float* out, void* ws, size_t ws_bytes, void* stream) {
    if (!p32 || !w16 || !img || !out || !ws) return net_fail(-1, "NULL argument");
    if (!ws_dims_ok(dims)) return net_fail(-2, "volume sizes must be positive multiples of 4");
    if (!(scale > 0)) return net_fail(-1, "scale must be positive");
    if ((uintptr_t)ws & 255) return net_fail(-1, "workspace must be 256-byte aligned");
    const WsLayout L = ws_layout(dims, false);
    if (ws_bytes < L.total) return net_fail(-5, "workspace too small");
    return ws_forward(L, (char*)ws, w16, p32, scale, img, out, (hipStream_t)stream);
}

}  // extern "C"

namespace {

// Loss 0.5 |net(img) - scale target|^2 (into loss, if not NULL) and its gradient with
// respect to every parameter (FP32 blob layout, into grads): the forward pass, then
// backpropagation through the layers in reverse order with the kernels' adjoints.
int ws_grads(const WsLayout& L, char* w, const float* p32, const uint16_t* w16, float scale,
             const float* img, const float* target, float* grads, double* loss, hipStream_t st) {
    static const WsParams PR;
    WS_TRY(ws_forward(L, w, w16, p32, scale, img, nullptr, st));
    uint16_t* A[18];
    for (int i = 0; i < 18; ++i) A[i] = (uint16_t*)(w + L.act[i]);
    auto G = [&](size_t o) { return (uint16_t*)(w + o); };
    float* part = (float*)(w + L.part);
    uint16_t* wt = G(L.wt);
    const int32_t* D[3] = {L.dims[0], L.dims[1], L.dims[2]};
    const int64_t nv = L.nv;
    // loss and its gradient in channel 0 of the output (the other channels zero)
    wsnet::fill_zero_u16<<<nblk(nv * 16), NET_BLOCK, 0, st>>>(nv * 16, G(L.gout));
    NET_CHECK();
    WS_TRY(spdhg_net_mse_grad(nv, 16, A[17], img, target, scale, G(L.gout),
                              (double*)(w + L.lparts), st));
    // back(l): relu derivative (from the layer's output), weight and bias gradients, and
    // the input gradient through the adjoint convolution (not needed for the first layer)
    auto back = [&](int l, const uint16_t* in, const uint16_t* outp, uint16_t* gout,
                    uint16_t* gin) -> int {
        const int32_t* Dl = D[WS_LEVEL[l]];
        const int64_t nvl = (int64_t)Dl[0] * Dl[1] * Dl[2];
        if (WS_RELU[l]) WS_TRY(spdhg_net_relu_bwd(nvl * WS_CO[l], outp, gout, st));
        WS_TRY(spdhg_conv3d_wgrad(Dl, WS_CI[l], WS_CO[l], in, gout, WS_CHUNK, part, L.part_floats,
                                  grads + PR.w32[l], grads + PR.b32[l], st));
        if (!gin) return 0;
        WS_TRY(spdhg_conv3d_adjoint_weights(WS_CI[l], WS_CO[l], w16 + PR.w16[l], wt, st));
        return spdhg_conv3d_fwd(Dl, WS_CO[l], WS_CI[l], gout, wt, nullptr, 0, gin, st);
    };
    auto copy = [&](uint16_t* dst, const uint16_t* src, int64_t n) -> int {
        const hipError_t e = hipMemcpyAsync(dst, src, n * 2, hipMemcpyDeviceToDevice, st);
        return e == hipSuccess ? 0 : net_fail(-4, hipGetErrorString(e));
    };
    WS_TRY(back(10, A[16], A[17], G(L.gout), G(L.g10)));          // c11: d1 -> out
    WS_TRY(back(9, A[15], A[16], G(L.g10), G(L.g9in)));           // c10: s1 -> d1
    WS_TRY(copy(G(L.g2), G(L.g9in), nv * 16));                    // d s1 / d e1: the skip
    WS_TRY(back(8, A[13], A[14], G(L.g9in), G(L.g9)));            // c9: u1 -> c9
    WS_TRY(spdhg_net_up2(D[0], 32, 1, G(L.g9), G(L.g9u), st));    // up(d2) adjoint
    WS_TRY(back(7, A[11], A[12], G(L.g9u), G(L.g8)));             // c8: s2 -> d2
    WS_TRY(copy(G(L.g7in), G(L.g8), nv / 8 * 32));                // d s2 / d e2: the skip
    WS_TRY(back(6, A[9], A[10], G(L.g7in), G(L.g7)));             // c7: u2 -> c7
    WS_TRY(spdhg_net_up2(D[1], 64, 1, G(L.g7), G(L.g7u), st));    // up(b) adjoint
    WS_TRY(back(5, A[7], A[8], G(L.g7u), G(L.g6)));               // c6: c5 -> b
    WS_TRY(back(4, A[6], A[7], G(L.g6), G(L.g5)));                // c5: p2 -> c5
    WS_TRY(spdhg_net_pool2(D[1], 32, 1, G(L.g5), G(L.g5p), st));  // pool(e2) adjoint
    WS_TRY(spdhg_net_add(nv / 8 * 32, G(L.g5p), G(L.g8), G(L.g5s), st));
    WS_TRY(back(3, A[4], A[5], G(L.g5s), G(L.g4)));               // c4: c3 -> e2
    WS_TRY(back(2, A[3], A[4], G(L.g4), G(L.g3)));                // c3: p1 -> c3
    WS_TRY(spdhg_net_pool2(D[0], 16, 1, G(L.g3), G(L.g3p), st));  // pool(e1) adjoint
    WS_TRY(spdhg_net_add(nv * 16, G(L.g3p), G(L.g2), G(L.g3s), st));
    WS_TRY(back(1, A[1], A[2], G(L.g3s), G(L.g9in)));             // c2: c1 -> e1
    WS_TRY(back(0, A[0], A[1], G(L.g9in), nullptr));              // c1: in -> c1
    if (loss) {
        wsnet::sum_parts<<<1, 256, 0, st>>>((const double*)(w + L.lparts), (nv + 255) / 256, loss);
        NET_CHECK();
    }
    return 0;
}

int ws_train_checks(const int32_t dims[3], float scale, const void* ws, size_t ws_bytes,
                    WsLayout& L) {
    if (!ws_dims_ok(dims)) return net_fail(-2, "volume sizes must be positive multiples of 4");
    if (!(scale > 0)) return net_fail(-1, "scale must be positive");
    if ((uintptr_t)ws & 255) return net_fail(-1, "workspace must be 256-byte aligned");
    L = ws_layout(dims, true);
    if (ws_bytes < L.total) return net_fail(-5, "workspace too small");
    return 0;
}

}  // namespace

extern "C" {

int spdhg_ws_gradients(const int32_t dims[3], const float* p32, const uint16_t* w16, float scale,
                       const float* img, const float* target, float* grads, double* loss,
                       void* ws, size_t ws_bytes, void* stream) {
    if (!p32 || !w16 || !img || !target || !grads || !ws) return net_fail(-1, "NULL argument");
    WsLayout L;
    WS_TRY(ws_train_checks(dims, scale, ws, ws_bytes, L));
    return ws_grads(L, (char*)ws, p32, w16, scale, img, target, grads, loss, (hipStream_t)stream);
}

int spdhg_ws_train_step(const int32_t dims[3], float* p32, uint16_t* w16, float* adam_m,
                        float* adam_v, int64_t step, float lr, float scale, const float* img,
                        const float* target, double* loss, void* ws, size_t ws_bytes,
                        void* stream) {
    if (!p32 || !w16 || !adam_m || !adam_v || !img || !target || !ws)
        return net_fail(-1, "NULL argument");
    if (step < 1) return net_fail(-1, "step must be >= 1");
    WsLayout L;
    WS_TRY(ws_train_checks(dims, scale, ws, ws_bytes, L));
    static const WsParams PR;
    hipStream_t st = (hipStream_t)stream;
    float* grads = (float*)((char*)ws + L.grads);
    WS_TRY(ws_grads(L, (char*)ws, p32, w16, scale, img, target, grads, loss, st));
    // one Adam step over the whole blob (elementwise: the same as a step per tensor), then
    // the packed BF16 copies of the new weights
    WS_TRY(spdhg_net_adam(PR.n32, lr, 0.9f, 0.999f, 1e-8f, step, p32, adam_m, adam_v, grads,
                          nullptr, st));
    return spdhg_ws_pack(p32, w16, st);
}

}  // extern "C"
