// The learned surrogate of the AIM grid convolution (the FFT step of the
// four-step AIM, Sec. 3.2.2): a network of 3x3x3 convolution layers that maps
// the grid charges Q to the grid potential U on the same [nz][ny][nx] grid of
// a film, circular along the periodic x and y axes and zero-padded across the
// thickness. Device kernels and the host-side network object; internal to the
// library.
//
// Network: layer 0 maps 1 -> kSgC channels, layers 1 .. depth-2 map kSgC ->
// kSgC, layer depth-1 maps kSgC -> 1; ReLU after every layer but the last.
// Parameters (FP32 master, the order of the public parameter vector): for each
// layer W[co][ci][3][3][3] then b[co]; offset o = (dz+1)*9 + (dy+1)*3 + (dx+1).
// The kernels use the weights rounded to BF16 (biases stay FP32) and
// accumulate in FP32. The middle layers run on the matrix cores: activations
// are FP32 in HBM, split into a BF16 high part and a BF16 remainder when
// staged, both multiplied by the BF16 weights, so that the layer keeps FP32
// accuracy. Activations are channels-last, [voxel][kSgC].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace pmfem {

constexpr int kSgC = 32;                      // hidden channels
constexpr int kSgMaxDepth = 12;
constexpr int kSgTX = 32, kSgTY = 8;          // output tile of one z-plane
constexpr int kSgHX = kSgTX + 2, kSgHY = kSgTY + 2;
constexpr int kSgHalo = kSgHX * kSgHY;        // staged points of one plane
constexpr int kSgWPart = 512;                 // partial sums of the weight-gradient pass

struct SgGrid {
  int nx, ny, nz;
};

// Parameters of the synthetic training textures (host-drawn per texture).
struct SgTexture {
  int kind;            // 0 random, 1 vortex, 2 domain-wall pair
  uint32_t seed;
  double Lx, Ly;       // periods
  double cx, cy;       // vortex centre / wall offset along the normal
  double rc;           // vortex core radius / wall width
  double chir, pol;    // vortex chirality and polarity (+-1)
  double nx, ny;       // in-plane wall normal (unit, along x or y)
  double ed[3], er[3]; // wall: domain direction and the direction the wall turns through
};

struct Surrogate {
  int depth = 0;
  int64_t nparam = 0;
  std::vector<int64_t> woff, boff;   // offsets of W and b of each layer
  SgGrid gd{};
  int64_t nvox = 0, n = 0;           // grid points, unknowns of the context
  float s_in = 0.f, s_out = 0.f;     // network input = Q s_in, U = output s_out (0: unset)
  bool split = true;                 // BF16 high part + remainder (else BF16 activations)
  bool trained_buffers = false;
  // parameters: FP32 master, gradient and Adam moments
  float *p = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
  int64_t adam_t = 0;
  // packed weights for the kernels
  uint16_t *wmid = nullptr, *wmidt = nullptr;  // [depth-2][27][C][C] BF16 (forward; transposed+flipped)
  float *win = nullptr, *wout = nullptr, *woutt = nullptr;  // [C][27] (BF16 values)
  // work buffers
  float* act = nullptr;   // inference: 2 x [nvox][C]; training: (depth-1) x [nvox][C]
  float *gA = nullptr, *gB = nullptr, *xpad = nullptr, *gpad = nullptr;  // [nvox][C]
  float *y = nullptr, *gy = nullptr;   // [nvox]
  float *qbuf = nullptr, *ubuf = nullptr;  // a training pair's Q and U grids
  float* part = nullptr;                // weight-gradient partial sums [kSgWPart][C*C*27]
  double* dred = nullptr;               // reduction partials
  double* loss = nullptr;               // per training pair
  int loss_cap = 0;
  double *pos = nullptr, *m64 = nullptr;  // unknown positions, a texture
  float *m32 = nullptr, *ha = nullptr, *hs = nullptr;  // [n][3]
};

// All functions return a hipError_t from the launches or allocations.
hipError_t sg_create(Surrogate* s, int depth, SgGrid gd, int64_t n_unknowns, const double* pos_host,
                     bool split);
void sg_destroy(Surrogate* s);
hipError_t sg_set_params(Surrogate* s, const float* host, hipStream_t st);
hipError_t sg_pack(Surrogate* s, hipStream_t st);   // master -> kernel weight forms
hipError_t sg_get_params(const Surrogate* s, float* host, hipStream_t st);
void sg_default_params(const Surrogate* s, uint64_t seed, std::vector<float>& out);
// U = surrogate(Q) on the grid (inference). Q and U may be one buffer: the
// first layer has read Q before the last layer writes U.
hipError_t sg_apply(Surrogate* s, hipStream_t st, const float* Q, float* U);
// reps forward passes with events around every layer; ms[depth] = mean
// milliseconds of each layer (synchronises)
hipError_t sg_profile(Surrogate* s, hipStream_t st, const float* Q, float* U, int reps, double* ms);
// One forward and backward pass for the pair (Q, t): the network's input is
// Q s_in; the loss is the mean over the grid of (y - t tscale)^2; the
// gradient goes to s->grad, the loss to s->loss[slot].
hipError_t sg_loss_grad(Surrogate* s, hipStream_t st, const float* Q, const float* t, float tscale,
                        int slot);
hipError_t sg_adam(Surrogate* s, hipStream_t st, double lr);
hipError_t sg_texture(Surrogate* s, hipStream_t st, const SgTexture& tx, double* m_dev);
hipError_t sg_to_f32(Surrogate* s, hipStream_t st, const double* m64, float* m32);
// sum of |a - b|^2 and |b|^2 over [n][3] on the device -> host (synchronises)
hipError_t sg_field_error(Surrogate* s, hipStream_t st, const float* a, const float* b, double* out2);
// sum of squares of a grid (synchronises)
hipError_t sg_sumsq(Surrogate* s, hipStream_t st, const float* x, int64_t count, double* out);
hipError_t sg_ensure_training(Surrogate* s, int n_loss);

}  // namespace pmfem
