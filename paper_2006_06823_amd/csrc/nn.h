// Small 3D convolutional network of the learned warm start (see nn.hip).
#pragma once

#include "common.h"

namespace lddmm {

struct ConvLayer {
  int cin = 0, cout = 0, k = 3, stride = 1, pad = 1, relu = 1;
  float *w = nullptr, *b = nullptr;    // float masters [cout][cin][k^3], [cout]
  float *dw = nullptr, *db = nullptr;  // gradients
  float *mw = nullptr, *vw = nullptr, *mb = nullptr, *vb = nullptr;  // Adam moments
  int64_t nw() const { return (int64_t)cout * cin * k * k * k; }
};

void conv_forward(const ConvLayer& L, const float* x, float* y, int B, int Di, hipStream_t s);
// g: scratch of y's size; dx may be null (first layer)
void conv_backward(const ConvLayer& L, const float* x, const float* y, const float* dy, float* g, float* dx, int B,
                   int Di, hipStream_t s);
void adam_step(float* w, float* m, float* v, const float* g, int64_t n, float lr, int t, hipStream_t s);
void fill(float* p, int64_t n, float v, hipStream_t s);
// box-average an image pair of n[0] x n[1] x n[2] voxels (each divisible by S) into a [2][S^3] input
void pool_pair(const float* I0, const float* I1, const int n[3], int S, float* out, hipStream_t s);
// coarse samples -> band coefficients [B][3][k0][k1][k2] through the projection P [sz][sz]; group b
// of three sample channels starts at channel 3 gs b of samp ([B][3 gs][sz^3])
void samples_to_bl(const float* samp, const float* P, int B, int gs, int sz, const int k[3], float* v,
                   hipStream_t s);
// ds = scale * (projection block)^T (w * diff), diff [B][3][k0][k1][k2], w [k0 k1 k2] (double), written
// to the channels 3 gs b .. 3 gs b + 2 of ds ([B][3 gs][sz^3]); other channels are left untouched
void block_grad(const float* diff, const double* w, const float* P, int B, int gs, int sz, const int k[3],
                float scale, float* ds, hipStream_t s);

}  // namespace lddmm
