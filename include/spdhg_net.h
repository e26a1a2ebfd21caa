/* Warm-start network kernels (C ABI of libspdhg.so).
 *
 * Not part of the paper's method: a small 3-D convolutional encoder-decoder maps the
 * normalised backprojection of the data to an initial image for SPDHG (Algorithm 2 then
 * runs from it unchanged).  These entry points are its building blocks; the network,
 * its training on SPDHG MAP solutions and the warm-started reconstruction are assembled
 * from them by the Python binding (paper_1808_07150_amd/warmstart.py).
 *
 * Conventions.  All pointers are device pointers on the current HIP device; nothing is
 * allocated and nothing is freed.  Volumes are dims = {ny, nx, nz}.  Activations are
 * channel-last BF16 ([y][x][z][C], C in {16, 32, 64}; BF16 passed as uint16_t bit
 * patterns).  Convolutions are 3x3x3 with zero padding ("same" size); their weights are
 * packed BF16 [tap][ci / 16][co][16] with tap = (dy+1)*9 + (dx+1)*3 + (dz+1), and the
 * FP32 master weights [tap][co][ci].  Products run on the MFMA units in BF16 with FP32
 * accumulation.  Calls are asynchronous on `stream`; errors are negative codes
 * (-1 argument, -2 shape, -4 HIP, -5 buffer too small) with a thread-local message. */
#ifndef SPDHG_NET_H
#define SPDHG_NET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

const char* spdhg_net_last_error(void);

/* out[v][co] = relu?(bias[co] + sum_{tap, ci} W[tap][co][ci] in[v + off(tap)][ci]);
 * bias may be NULL, relu 0 or 1.  in (cin channels) and out (cout) must not overlap. */
int spdhg_conv3d_fwd(const int32_t dims[3], int32_t cin, int32_t cout, const uint16_t* in,
                     const uint16_t* w, const float* bias, int32_t relu, uint16_t* out, void* stream);

/* Packed weights wt of the adjoint convolution (cout -> cin channels, taps mirrored):
 * spdhg_conv3d_fwd(dims, cout, cin, dout, wt, NULL, 0, din) is the input gradient. */
int spdhg_conv3d_adjoint_weights(int32_t cin, int32_t cout, const uint16_t* w, uint16_t* wt,
                                 void* stream);

/* Weight gradient dw[tap][co][ci] = sum_v dout[v][co] in[v + off(tap)][ci] (FP32) and,
 * if dbias is not NULL, dbias[co] = sum_v dout[v][co].  Deterministic: voxel chunks of
 * `chunk` (a multiple of 16) are summed into FP32 partials `part` (at least
 * ceil(nv / chunk) * 27 * cin * cout and ceil(nv / 1024) * cout floats) and then added in
 * chunk order. */
int spdhg_conv3d_wgrad(const int32_t dims[3], int32_t cin, int32_t cout, const uint16_t* in,
                       const uint16_t* dout, int32_t chunk, float* part, int64_t part_floats,
                       float* dw, float* dbias, void* stream);

/* dy[e] = 0 where y[e] <= 0 (ReLU derivative from the layer output), n elements. */
int spdhg_net_relu_bwd(int64_t n, const uint16_t* y, uint16_t* dy, void* stream);

/* out = a + b element-wise (BF16). */
int spdhg_net_add(int64_t n, const uint16_t* a, const uint16_t* b, uint16_t* out, void* stream);

/* 2x2x2 average pooling from the fine grid `fine` (even sizes) to half size, or with
 * adjoint != 0 its adjoint (coarse gradient -> fine). */
int spdhg_net_pool2(const int32_t fine[3], int32_t c, int32_t adjoint, const uint16_t* src,
                    uint16_t* dst, void* stream);

/* Nearest 2x upsampling to the fine grid `fine`, or with adjoint != 0 its adjoint (sum of
 * the eight fine voxels of each coarse voxel); c a multiple of 16 (else -2). */
int spdhg_net_up2(const int32_t fine[3], int32_t c, int32_t adjoint, const uint16_t* src,
                  uint16_t* dst, void* stream);

/* FP32 image (nv voxels, z-fastest) -> 16-channel activations, channel 0 = scale * image. */
int spdhg_net_image_to_act(int64_t nv, float scale, const float* img, uint16_t* act, void* stream);

/* image = (channel 0 of act (cact channels) + scale * skip) / scale; skip may be NULL. */
int spdhg_net_act_to_image(int64_t nv, float scale, const uint16_t* act, int32_t cact,
                           const float* skip, float* img, void* stream);

/* Squared error 0.5 sum_v (p_v - scale * target_v)^2 with p = channel 0 of pred plus
 * scale * skip (skip may be NULL): FP64 partials per 256 voxels into part, and dL/dp
 * written to channel 0 of grad (the other channels are left untouched). */
int spdhg_net_mse_grad(int64_t nv, int32_t cact, const uint16_t* pred, const float* skip,
                       const float* target, float scale, uint16_t* grad, double* part,
                       void* stream);

/* One Adam step (bias-corrected, step >= 1) on n FP32 parameters p with moments m, v and
 * gradient g; p16 (may be NULL) receives the BF16 copy of the new p. */
int spdhg_net_adam(int64_t n, float lr, float b1, float b2, float eps, int64_t step, float* p,
                   float* m, float* v, const float* g, uint16_t* p16, void* stream);

/* FP32 weights [tap][co][ci] -> packed BF16 [tap][ci / 16][co][16]. */
int spdhg_net_pack_weights(int32_t cin, int32_t cout, const float* w32, uint16_t* w16, void* stream);

#ifdef __cplusplus
}
#endif

#endif
