/* Warm-start network kernels (C ABI of libspdhg.so).
 *
 * Not part of the paper's method: a small 3-D convolutional encoder-decoder maps the
 * normalised backprojection of the data to an initial image for SPDHG (Algorithm 2 then
 * runs from it unchanged).  spdhg_ws_infer / spdhg_ws_gradients / spdhg_ws_train_step
 * run the whole network (forward, backpropagation, Adam) from parameter blobs and a
 * caller-owned workspace; the single-kernel entry points below them are its building
 * blocks.  The input image comes from spdhg_normalised_backprojection (spdhg.h).
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

/* ---- the whole network ------------------------------------------------------------
 * Layers c1 .. c11 (cin -> cout, ReLU): 16->16, 16->16 (ReLU, full resolution, e1);
 * 16->32, 32->32 (half, e2); 32->64, 64->64 (quarter, b); 64->32 after nearest 2x up,
 * then + e2, 32->32 (half, d2); 32->16 after up, then + e1, 16->16 (full, d1); 16->16
 * linear (c11).  Pooling is 2x2x2 averaging.  Output image = input + channel 0 of c11
 * (divided by scale).  Volumes dims = {ny, nx, nz}, each a positive multiple of 4; images
 * are FP32 [ny][nx][nz].
 * Parameters: an FP32 blob of n32 values (per layer in order: weights [27][cout][cin],
 * then bias [cout]) and a packed BF16 blob of n16 values (per layer: the weights packed as
 * by spdhg_net_pack_weights); spdhg_ws_param_offsets gives layer l's offsets (elements). */
int spdhg_ws_param_count(int64_t* n32, int64_t* n16);
int spdhg_ws_param_offsets(int32_t layer, int64_t* w32, int64_t* b32, int64_t* w16);

/* The packed BF16 blob from the FP32 blob (every layer). */
int spdhg_ws_pack(const float* p32, uint16_t* w16, void* stream);

/* Bytes of device workspace for a volume: train = 0 for spdhg_ws_infer (activations),
 * 1 for spdhg_ws_gradients / spdhg_ws_train_step (also gradients and partials).  -2 if
 * dims are not positive multiples of 4. */
int spdhg_ws_workspace_bytes(const int32_t dims[3], int32_t train, size_t* bytes);

/* out = network(img) (scale: brings img to order one, e.g. 1 / its mean over the
 * support).  ws: device workspace (256-byte aligned, at least the train = 0 size), owned
 * by the caller, nothing allocated; -5 if too small. */
int spdhg_ws_infer(const int32_t dims[3], const float* p32, const uint16_t* w16, float scale,
                   const float* img, float* out, void* ws, size_t ws_bytes, void* stream);

/* Loss 0.5 sum_v (net(img)_v - target_v)^2 scale^2 (FP64, device scalar *loss, or NULL)
 * and its gradient with respect to every parameter (grads: n32 FP32, blob layout).  BF16
 * activations and gradients, FP32 accumulation; deterministic.  ws: at least the
 * train = 1 size. */
int spdhg_ws_gradients(const int32_t dims[3], const float* p32, const uint16_t* w16, float scale,
                       const float* img, const float* target, float* grads, double* loss,
                       void* ws, size_t ws_bytes, void* stream);

/* One training step: spdhg_ws_gradients, one Adam step (lr, beta 0.9 / 0.999, eps 1e-8,
 * bias-corrected at `step` >= 1) on p32 with moments adam_m, adam_v (n32 each), and the
 * new packed w16. */
int spdhg_ws_train_step(const int32_t dims[3], float* p32, uint16_t* w16, float* adam_m,
                        float* adam_v, int64_t step, float lr, float scale, const float* img,
                        const float* target, double* loss, void* ws, size_t ws_bytes,
                        void* stream);

#ifdef __cplusplus
}
#endif

#endif
