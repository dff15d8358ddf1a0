// Learned preconditioner stage: a small 1D convolutional network along the
// interface coordinate, trained on the GPU with hand-written forward and
// backward kernels, used inside flexible GMRES as z = GS(v) + N(v).
//
// Network: 4 convolutions 8 -> 32 -> 32 -> 32 -> 8 (kernel 5, zero padding 2,
// stride 1), ReLU after the first three.  Weights are kept as float32 master
// copies (Adam) and as bfloat16 copies that the forward and backward kernels
// read; activations, accumulation and gradients are float32.
#include <cstdio>
#include <fstream>

#include "solver_internal.h"

namespace polar_impl {
namespace {

constexpr int kLayers = 4;
constexpr int kK = 5;
constexpr int kPad = 2;
constexpr int kCin[kLayers] = {8, 32, 32, 32};
constexpr int kCout[kLayers] = {32, 32, 32, 8};
// dilation of each layer: taps at offsets (k - kPad) d, so the network sees
// 1 + 2 kPad (1 + 2 + 4 + 8) = 61 interface points around each output point
constexpr int kDil[kLayers] = {1, 2, 4, 8};
constexpr int kThreadsL = 256;

constexpr int64_t w_size(int l) { return (int64_t)kCout[l] * kCin[l] * kK; }
constexpr int64_t layer_size(int l) { return w_size(l) + kCout[l]; }
int64_t w_off(int l) {
  int64_t o = 0;
  for (int q = 0; q < l; ++q) o += layer_size(q);
  return o;
}
int64_t nparams() {
  int64_t o = 0;
  for (int q = 0; q < kLayers; ++q) o += layer_size(q);
  return o;
}

__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f_to_bf16(float f) {  // round to nearest even (finite inputs)
  const uint32_t u = __float_as_uint(f);
  const uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

// y[b][o][i] = bias[o] + sum_{c,k} w[o][c][k] x[b][c][i+(k-2)d], optional ReLU.
// grid (ceil(n/256), Cout, B)
__global__ __launch_bounds__(kThreadsL) void conv_fwd_kernel(const float* __restrict__ x, const uint16_t* __restrict__ w,
                                                              const float* __restrict__ bias, float* __restrict__ y,
                                                              int Cin, int Cout, int n, int relu, int d) {
  __shared__ float ws[32 * kK];
  const int o = blockIdx.y, b = blockIdx.z;
  for (int q = threadIdx.x; q < Cin * kK; q += kThreadsL) ws[q] = bf16_to_f(w[(size_t)o * Cin * kK + q]);
  __syncthreads();
  const int i = blockIdx.x * kThreadsL + threadIdx.x;
  if (i >= n) return;
  float acc = bias[o];
  const float* xb = x + (size_t)b * Cin * n;
  for (int c = 0; c < Cin; ++c)
#pragma unroll
    for (int k = 0; k < kK; ++k) {
      const int j = i + (k - kPad) * d;
      if (j >= 0 && j < n) acc = fmaf(ws[c * kK + k], xb[(size_t)c * n + j], acc);
    }
  if (relu) acc = fmaxf(acc, 0.f);
  y[((size_t)b * Cout + o) * n + i] = acc;
}

__device__ __forceinline__ float masked(const float* g, const float* yl, size_t e) {
  return (yl == nullptr || yl[e] > 0.f) ? g[e] : 0.f;
}

// dx[b][c][j] = sum_{o,k} w[o][c][k] gm[b][o][j-(k-2)d], gm = g masked by ReLU'(layer output yl)
// grid (ceil(n/256), Cin, B)
__global__ __launch_bounds__(kThreadsL) void conv_bwd_data_kernel(const float* __restrict__ g,
                                                                   const float* __restrict__ yl,
                                                                   const uint16_t* __restrict__ w,
                                                                   float* __restrict__ dx, int Cin, int Cout, int n,
                                                                   int d) {
  __shared__ float ws[32 * kK];
  const int c = blockIdx.y, b = blockIdx.z;
  for (int q = threadIdx.x; q < Cout * kK; q += kThreadsL) {
    const int o = q / kK, k = q % kK;
    ws[q] = bf16_to_f(w[((size_t)o * Cin + c) * kK + k]);
  }
  __syncthreads();
  const int j = blockIdx.x * kThreadsL + threadIdx.x;
  if (j >= n) return;
  float acc = 0.f;
  for (int o = 0; o < Cout; ++o) {
    const size_t base = ((size_t)b * Cout + o) * n;
#pragma unroll
    for (int k = 0; k < kK; ++k) {
      const int i = j - (k - kPad) * d;
      if (i >= 0 && i < n) acc = fmaf(ws[o * kK + k], masked(g, yl, base + i), acc);
    }
  }
  dx[((size_t)b * Cin + c) * n + j] = acc;
}

// dw[o][c][k] = sum_{b,i} gm[b][o][i] x[b][c][i+(k-2)d];  db[o] = sum gm[b][o][i] (written by c == 0)
// grid (Cout, Cin), fixed-order reduction
__global__ __launch_bounds__(kThreadsL) void conv_bwd_weight_kernel(const float* __restrict__ g,
                                                                     const float* __restrict__ yl,
                                                                     const float* __restrict__ x,
                                                                     float* __restrict__ dw, float* __restrict__ db,
                                                                     int B, int Cin, int Cout, int n, int d) {
  __shared__ float red[kK + 1][kThreadsL];
  const int o = blockIdx.x, c = blockIdx.y;
  float acc[kK + 1] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const int total = B * n;
  for (int e = threadIdx.x; e < total; e += kThreadsL) {
    const int b = e / n, i = e - b * n;
    const float gv = masked(g, yl, ((size_t)b * Cout + o) * n + i);
    const float* xb = x + ((size_t)b * Cin + c) * n;
#pragma unroll
    for (int k = 0; k < kK; ++k) {
      const int j = i + (k - kPad) * d;
      if (j >= 0 && j < n) acc[k] = fmaf(gv, xb[j], acc[k]);
    }
    acc[kK] += gv;
  }
#pragma unroll
  for (int k = 0; k <= kK; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = kThreadsL / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
#pragma unroll
      for (int k = 0; k <= kK; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < kK) dw[((size_t)o * Cin + c) * kK + threadIdx.x] = red[threadIdx.x][0];
  if (threadIdx.x == kK && c == 0) db[o] = red[kK][0];
}

// per sample b: loss_b = ||y-t||^2 / (||t||^2 + tiny), dy = 2 (y - t) / (||t||^2 + tiny) / B
__global__ __launch_bounds__(kThreadsL) void loss_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                          float* __restrict__ dy, float* __restrict__ lossv, int B,
                                                          int m) {
  __shared__ float s_num[kThreadsL], s_den[kThreadsL];
  const int b = blockIdx.x;
  const float* yb = y + (size_t)b * m;
  const float* tb = t + (size_t)b * m;
  float num = 0.f, den = 0.f;
  for (int e = threadIdx.x; e < m; e += kThreadsL) {
    const float d = yb[e] - tb[e];
    num = fmaf(d, d, num);
    den = fmaf(tb[e], tb[e], den);
  }
  s_num[threadIdx.x] = num;
  s_den[threadIdx.x] = den;
  __syncthreads();
  for (int s = kThreadsL / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      s_num[threadIdx.x] += s_num[threadIdx.x + s];
      s_den[threadIdx.x] += s_den[threadIdx.x + s];
    }
    __syncthreads();
  }
  const float D = s_den[0] + 1e-30f;
  if (threadIdx.x == 0) lossv[b] = s_num[0] / D;
  const float sc = 2.f / D / (float)B;
  for (int e = threadIdx.x; e < m; e += kThreadsL) dy[(size_t)b * m + e] = sc * (yb[e] - tb[e]);
}

__global__ void adam_kernel(float* __restrict__ w, uint16_t* __restrict__ w16, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int64_t np, float lr, float b1, float b2,
                            float eps, float bc1, float bc2) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= np) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.f - b1) * gq;
  const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  const float wq = w[q] - lr * (mq / bc1) / (sqrtf(vq / bc2) + eps);
  w[q] = wq;
  w16[q] = f_to_bf16(wq);
}

__global__ void to_bf16_kernel(const float* __restrict__ w, uint16_t* __restrict__ w16, int64_t np) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < np) w16[q] = f_to_bf16(w[q]);
}

// batch gather: dst[b] = src[idx[b]] (m floats per sample)
__global__ void gather_kernel(const float* __restrict__ src, const int32_t* __restrict__ idx, float* __restrict__ dst,
                              int B, int m) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)B * m) return;
  const int b = (int)(e / m), q = (int)(e % m);
  dst[e] = src[(size_t)idx[b] * m + q];
}

// polarized trace vectors (nrhs, 2, L1, 2, n) complex -> samples (nrhs*L1, 8, n)
// channel (h*2 + a)*2 + {0: re, 1: im}; sample b = r*L1 + k.  mode 0: compute the
// per-sample RMS into scale and store v / scale; mode 1: store v / scale with
// the given scale (targets).  grid: B workgroups.
__global__ __launch_bounds__(kThreadsL) void pack_kernel(const double2* __restrict__ v, float* __restrict__ X,
                                                          float* __restrict__ scale, int L1, int n, int mode) {
  __shared__ double s_sum[kThreadsL];
  const int b = blockIdx.x;
  const int r = b / L1, k = b % L1;
  const int64_t Nt = (int64_t)4 * L1 * n;
  const double2* vr = v + (int64_t)r * Nt;
  double sc;
  if (mode == 0) {
    double acc = 0.0;
    for (int e = threadIdx.x; e < 4 * n; e += kThreadsL) {
      const int ha = e / n, i = e % n;
      const int h = ha >> 1, a = ha & 1;
      const double2 z = vr[((int64_t)(h * L1 + k) * 2 + a) * n + i];
      acc += z.x * z.x + z.y * z.y;
    }
    s_sum[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kThreadsL / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) s_sum[threadIdx.x] += s_sum[threadIdx.x + s];
      __syncthreads();
    }
    sc = sqrt(s_sum[0] / (8.0 * n));
    if (threadIdx.x == 0) scale[b] = (float)sc;
  } else {
    sc = scale[b];
  }
  const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
  for (int e = threadIdx.x; e < 4 * n; e += kThreadsL) {
    const int ha = e / n, i = e % n;
    const int h = ha >> 1, a = ha & 1;
    const double2 z = vr[((int64_t)(h * L1 + k) * 2 + a) * n + i];
    X[((size_t)b * 8 + ha * 2) * n + i] = (float)(z.x * inv);
    X[((size_t)b * 8 + ha * 2 + 1) * n + i] = (float)(z.y * inv);
  }
}

// z += scale * Y for samples (nrhs*L1, 8, n) -> polarized vectors; non-finite entries are skipped
__global__ __launch_bounds__(kThreadsL) void unpack_add_kernel(const float* __restrict__ Y,
                                                                const float* __restrict__ scale,
                                                                double2* __restrict__ z, int L1, int n,
                                                                int32_t* __restrict__ flag) {
  const int b = blockIdx.x;
  const int r = b / L1, k = b % L1;
  const int64_t Nt = (int64_t)4 * L1 * n;
  double2* zr = z + (int64_t)r * Nt;
  const double sc = scale[b];
  for (int e = threadIdx.x; e < 4 * n; e += kThreadsL) {
    const int ha = e / n, i = e % n;
    const int h = ha >> 1, a = ha & 1;
    const float re = Y[((size_t)b * 8 + ha * 2) * n + i];
    const float im = Y[((size_t)b * 8 + ha * 2 + 1) * n + i];
    if (!isfinite(re) || !isfinite(im)) {
      atomicOr(flag, 1);
      continue;
    }
    double2& t = zr[((int64_t)(h * L1 + k) * 2 + a) * n + i];
    t.x += sc * (double)re;
    t.y += sc * (double)im;
  }
}

// per RHS r: keep the correction if ||r - A c|| (nt) < ||r|| (nr); then z += c, w += A c
__global__ void select_kernel(double2* __restrict__ z, double2* __restrict__ w, const double2* __restrict__ c,
                              const double2* __restrict__ ac, const double* __restrict__ nr,
                              const double* __restrict__ nt, const int32_t* __restrict__ done,
                              int32_t* __restrict__ kept, int nrhs, int64_t N) {
  const int64_t total = (int64_t)nrhs * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / N);
    if (!(nt[r] < nr[r])) continue;  // also rejects NaN
    const double2 cv = c[e], av = ac[e];
    z[e].x += cv.x;
    z[e].y += cv.y;
    w[e].x += av.x;
    w[e].y += av.y;
    if (e == (int64_t)r * N && !done[r]) kept[r] += 1;
  }
}

__global__ void count_kernel(const int32_t* __restrict__ done, int32_t* __restrict__ kept, int nrhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrhs && !done[r]) kept[r] += 1;
}

__global__ void zero_i32_kernel(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// SplitMix64 -> uniform / normal (host side)
struct HRng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double u1 = uniform(), u2 = uniform();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

inline unsigned blocks_for(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace
}  // namespace polar_impl

using namespace polar_impl;

struct pt_learned {
  hipStream_t st = nullptr;
  int64_t np = 0;
  DevBuf<float> w32, grad, m, v;
  DevBuf<uint16_t> w16;
  int64_t adam_t = 0;
  // training samples (capacity x 8 x n)
  int capacity = 0, count = 0, n = 0;
  DevBuf<float> X, T;
  // workspace: activations act[0..4] (batch x 32 x n), gradients g0/g1, targets
  int wsB = 0, wsn = 0;
  DevBuf<float> act[kLayers + 1], g0, g1, tgt, lossv, scale;
  DevBuf<int32_t> idx, flag;
  // online stage vectors: residual, correction, its image under A (nrhs x Nt)
  int64_t vec_n = 0;
  int vec_rhs = 0;
  DevBuf<double2> rh, cv, ac;
  DevBuf<double> nr, nt;
  DevBuf<int32_t> kept;
  HRng rng{0};
};

namespace polar_impl {
namespace {

pt_status ensure_ws(pt_learned* N, int B, int n) {
  if (B <= N->wsB && n <= N->wsn) return PT_OK;
  const int Bm = std::max(B, N->wsB), nm = std::max(n, N->wsn);
  const size_t e = (size_t)Bm * 32 * nm;
  for (auto& a : N->act) {
    a.release();
    HIPCHK(a.alloc(e));
  }
  N->g0.release();
  N->g1.release();
  N->tgt.release();
  N->lossv.release();
  N->scale.release();
  N->idx.release();
  HIPCHK(N->g0.alloc(e));
  HIPCHK(N->g1.alloc(e));
  HIPCHK(N->tgt.alloc((size_t)Bm * 8 * nm));
  HIPCHK(N->lossv.alloc(Bm));
  HIPCHK(N->scale.alloc(Bm));
  HIPCHK(N->idx.alloc(Bm));
  N->wsB = Bm;
  N->wsn = nm;
  return PT_OK;
}

// forward through the 4 layers: act[0] -> act[4]
pt_status net_forward(pt_learned* N, int B, int n) {
  for (int l = 0; l < kLayers; ++l) {
    hipLaunchKernelGGL(conv_fwd_kernel, dim3(blocks_for(n), kCout[l], B), dim3(kThreadsL), 0, N->st, N->act[l].p,
                       N->w16.p + w_off(l), N->w32.p + w_off(l) + w_size(l), N->act[l + 1].p, kCin[l], kCout[l], n,
                       l < kLayers - 1 ? 1 : 0, kDil[l]);
    HIPCHK(hipGetLastError());
  }
  return PT_OK;
}

// loss against tgt, gradients of every parameter into N->grad; per-sample loss in lossv
pt_status net_backward(pt_learned* N, int B, int n) {
  hipLaunchKernelGGL(loss_kernel, dim3(B), dim3(kThreadsL), 0, N->st, N->act[kLayers].p, N->tgt.p, N->g0.p,
                     N->lossv.p, B, 8 * n);
  HIPCHK(hipGetLastError());
  float* g = N->g0.p;
  float* gn = N->g1.p;
  for (int l = kLayers - 1; l >= 0; --l) {
    const float* mask = l < kLayers - 1 ? N->act[l + 1].p : nullptr;
    hipLaunchKernelGGL(conv_bwd_weight_kernel, dim3(kCout[l], kCin[l]), dim3(kThreadsL), 0, N->st, g, mask,
                       N->act[l].p, N->grad.p + w_off(l), N->grad.p + w_off(l) + w_size(l), B, kCin[l], kCout[l], n,
                       kDil[l]);
    HIPCHK(hipGetLastError());
    if (l > 0) {
      hipLaunchKernelGGL(conv_bwd_data_kernel, dim3(blocks_for(n), kCin[l], B), dim3(kThreadsL), 0, N->st, g, mask,
                         N->w16.p + w_off(l), gn, kCin[l], kCout[l], n, kDil[l]);
      HIPCHK(hipGetLastError());
      std::swap(g, gn);
    }
  }
  return PT_OK;
}

pt_status refresh_bf16(pt_learned* N) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(N->np)), dim3(256), 0, N->st, N->w32.p, N->w16.p, N->np);
  HIPCHK(hipGetLastError());
  return PT_OK;
}

}  // namespace

pt_status ensure_vec(pt_learned* N, int nrhs, int64_t Nt) {
  const int64_t tot = (int64_t)nrhs * Nt;
  if (tot <= N->vec_n && nrhs <= N->vec_rhs) return PT_OK;
  for (auto* b : {&N->rh, &N->cv, &N->ac}) {
    b->release();
    HIPCHK(b->alloc((size_t)tot));
  }
  N->nr.release();
  N->nt.release();
  N->kept.release();
  HIPCHK(N->nr.alloc(nrhs));
  HIPCHK(N->nt.alloc(nrhs));
  HIPCHK(N->kept.alloc(nrhs));
  N->vec_n = tot;
  N->vec_rhs = nrhs;
  return PT_OK;
}

pt_status learned_begin(pt_solver* S, int nrhs) {
  pt_learned* N = S->learned;
  PTCHK(ensure_vec(N, nrhs, S->Nt));
  PTCHK(ensure_ws(N, nrhs * (S->L - 1), S->NX));
  hipLaunchKernelGGL(zero_i32_kernel, dim3(blocks_for(nrhs)), dim3(256), 0, S->st, N->kept.p, nrhs);
  HIPCHK(hipGetLastError());
  return PT_OK;
}

pt_status learned_step(pt_solver* S, const double2* v, double2* z, double2* w, int nrhs) {
  pt_learned* N = S->learned;
  const int L1 = S->L - 1, n = S->NX, B = nrhs * L1;
  const int64_t tot = (int64_t)nrhs * S->Nt;
  hipStream_t st = S->st;
  PTCHK(system_A(S, z, w, nrhs));                      // w = A z
  HIPCHK(launch_add(N->rh.p, v, w, -1.0, tot, st));    // r = v - A z
  hipLaunchKernelGGL(pack_kernel, dim3(B), dim3(kThreadsL), 0, st, (const double2*)N->rh.p, N->act[0].p, N->scale.p,
                     L1, n, 0);
  HIPCHK(hipGetLastError());
  hipStream_t keep = N->st;
  N->st = st;
  const pt_status rc = net_forward(N, B, n);
  N->st = keep;
  PTCHK(rc);
  HIPCHK(launch_zero(N->cv.p, tot, st));
  hipLaunchKernelGGL(unpack_add_kernel, dim3(B), dim3(kThreadsL), 0, st, N->act[kLayers].p, N->scale.p, N->cv.p, L1,
                     n, N->flag.p);
  HIPCHK(hipGetLastError());
  PTCHK(system_A(S, N->cv.p, N->ac.p, nrhs));          // A c
  HIPCHK(launch_knorm(N->rh.p, N->nr.p, nrhs, S->Nt, st));
  HIPCHK(launch_add(N->rh.p, N->rh.p, N->ac.p, -1.0, tot, st));  // r - A c
  HIPCHK(launch_knorm(N->rh.p, N->nt.p, nrhs, S->Nt, st));
  hipLaunchKernelGGL(select_kernel, dim3((unsigned)std::min<int64_t>(blocks_for(tot), 4096)), dim3(256), 0, st, z, w,
                     (const double2*)N->cv.p, (const double2*)N->ac.p, (const double*)N->nr.p,
                     (const double*)N->nt.p, (const int32_t*)S->done.p, N->kept.p, nrhs, S->Nt);
  HIPCHK(hipGetLastError());
  return PT_OK;
}

pt_status learned_residual(pt_solver* S, const double2* v, const double2* w, int nrhs) {
  HIPCHK(launch_add(S->learned->rh.p, v, w, -1.0, (int64_t)nrhs * S->Nt, S->st));
  return PT_OK;
}

pt_status learned_direction(pt_solver* S, double2* z, int nrhs) {
  pt_learned* N = S->learned;
  const int L1 = S->L - 1, n = S->NX, B = nrhs * L1;
  hipStream_t st = S->st;
  hipLaunchKernelGGL(pack_kernel, dim3(B), dim3(kThreadsL), 0, st, (const double2*)N->rh.p, N->act[0].p, N->scale.p,
                     L1, n, 0);
  HIPCHK(hipGetLastError());
  hipStream_t keep = N->st;
  N->st = st;
  const pt_status rc = net_forward(N, B, n);
  N->st = keep;
  PTCHK(rc);
  HIPCHK(launch_zero(z, (int64_t)nrhs * S->Nt, st));
  hipLaunchKernelGGL(unpack_add_kernel, dim3(B), dim3(kThreadsL), 0, st, N->act[kLayers].p, N->scale.p, z, L1, n,
                     N->flag.p);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(count_kernel, dim3(blocks_for(nrhs)), dim3(256), 0, st, (const int32_t*)S->done.p, N->kept.p,
                     nrhs);
  HIPCHK(hipGetLastError());
  return PT_OK;
}

pt_status learned_kept(pt_solver* S, int nrhs, int32_t* host) {
  HIPCHK(hipMemcpyAsync(host, S->learned->kept.p, nrhs * sizeof(int32_t), hipMemcpyDeviceToHost, S->st));
  return PT_OK;
}

}  // namespace polar_impl

extern "C" {

int64_t pt_learned_num_params(void) { return nparams(); }

void pt_learned_free(pt_learned* N) {
  if (!N) return;
  (void)hipStreamSynchronize(N->st);
  for (auto* b : {&N->w32, &N->grad, &N->m, &N->v, &N->X, &N->T, &N->g0, &N->g1, &N->tgt, &N->lossv, &N->scale})
    b->release();
  for (auto& a : N->act) a.release();
  for (auto* b : {&N->rh, &N->cv, &N->ac}) b->release();
  N->nr.release();
  N->nt.release();
  N->kept.release();
  N->w16.release();
  N->idx.release();
  N->flag.release();
  delete N;
}

pt_status pt_learned_create(int32_t capacity, uint64_t seed, void* hip_stream, pt_learned** out) {
  if (!out || capacity < 1) return fail(PT_EINVAL, "bad arguments");
  *out = nullptr;
  pt_learned* N = new pt_learned();
  N->st = (hipStream_t)hip_stream;
  N->np = nparams();
  N->capacity = capacity;
  N->rng.s = seed ^ 0xC0FFEE1234567ull;
  auto bail = [&](pt_status s) {
    pt_learned_free(N);
    return s;
  };
  if (N->w32.alloc(N->np) != hipSuccess || N->grad.alloc(N->np) != hipSuccess || N->m.alloc(N->np) != hipSuccess ||
      N->v.alloc(N->np) != hipSuccess || N->w16.alloc(N->np) != hipSuccess || N->flag.alloc(1) != hipSuccess)
    return bail(fail(PT_ENOMEM, "network parameters"));
  // He initialisation of the weights, zero biases
  std::vector<float> h(N->np, 0.f);
  for (int l = 0; l < kLayers; ++l) {
    const double sd = std::sqrt(2.0 / (kCin[l] * kK));
    for (int64_t q = 0; q < w_size(l); ++q) h[w_off(l) + q] = (float)(sd * N->rng.normal());
  }
  if (hipMemcpy(N->w32.p, h.data(), N->np * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(N->m.p, 0, N->np * 4) != hipSuccess || hipMemset(N->v.p, 0, N->np * 4) != hipSuccess ||
      hipMemset(N->flag.p, 0, 4) != hipSuccess)
    return bail(fail(PT_EHIP, "network init"));
  if (refresh_bf16(N) != PT_OK || hipStreamSynchronize(N->st) != hipSuccess) return bail(fail(PT_EHIP, "bf16 copy"));
  *out = N;
  return PT_OK;
}

pt_status pt_learned_get_params(const pt_learned* N, float* out) {
  if (!N || !out) return fail(PT_EINVAL, "null argument");
  HIPCHK(hipStreamSynchronize(N->st));
  HIPCHK(hipMemcpy(out, N->w32.p, N->np * 4, hipMemcpyDeviceToHost));
  return PT_OK;
}

pt_status pt_learned_set_params(pt_learned* N, const float* in) {
  if (!N || !in) return fail(PT_EINVAL, "null argument");
  HIPCHK(hipStreamSynchronize(N->st));
  HIPCHK(hipMemcpy(N->w32.p, in, N->np * 4, hipMemcpyHostToDevice));
  PTCHK(refresh_bf16(N));
  HIPCHK(hipStreamSynchronize(N->st));
  return PT_OK;
}

pt_status pt_learned_forward(pt_learned* N, int32_t B, int32_t n, const float* x, float* y) {
  if (!N || !x || !y || B < 1 || n < 1) return fail(PT_EINVAL, "bad arguments");
  PTCHK(ensure_ws(N, B, n));
  HIPCHK(hipMemcpyAsync(N->act[0].p, x, (size_t)B * 8 * n * 4, hipMemcpyHostToDevice, N->st));
  PTCHK(net_forward(N, B, n));
  HIPCHK(hipMemcpyAsync(y, N->act[kLayers].p, (size_t)B * 8 * n * 4, hipMemcpyDeviceToHost, N->st));
  HIPCHK(hipStreamSynchronize(N->st));
  return PT_OK;
}

pt_status pt_learned_gradient(pt_learned* N, int32_t B, int32_t n, const float* x, const float* t, double* loss,
                              float* grad) {
  if (!N || !x || !t || B < 1 || n < 1) return fail(PT_EINVAL, "bad arguments");
  PTCHK(ensure_ws(N, B, n));
  HIPCHK(hipMemcpyAsync(N->act[0].p, x, (size_t)B * 8 * n * 4, hipMemcpyHostToDevice, N->st));
  HIPCHK(hipMemcpyAsync(N->tgt.p, t, (size_t)B * 8 * n * 4, hipMemcpyHostToDevice, N->st));
  PTCHK(net_forward(N, B, n));
  PTCHK(net_backward(N, B, n));
  std::vector<float> lv(B);
  HIPCHK(hipMemcpyAsync(lv.data(), N->lossv.p, B * 4, hipMemcpyDeviceToHost, N->st));
  if (grad) HIPCHK(hipMemcpyAsync(grad, N->grad.p, N->np * 4, hipMemcpyDeviceToHost, N->st));
  HIPCHK(hipStreamSynchronize(N->st));
  if (loss) {
    double s = 0;
    for (float v : lv) s += v;
    *loss = s / B;
  }
  return PT_OK;
}

pt_status pt_learned_samples(const pt_learned* N, int32_t* count, int32_t* n) {
  if (!N) return fail(PT_EINVAL, "null network");
  if (count) *count = N->count;
  if (n) *n = N->n;
  return PT_OK;
}

pt_status pt_learned_collect(pt_learned* N, pt_solver* S, int32_t nrhs, const double* f, int32_t on_device,
                             int32_t* added) {
  if (!N || !S || !f) return fail(PT_EINVAL, "null argument");
  if (S->L < 2) return fail(PT_EINVAL, "no interfaces (L = 1)");
  if (nrhs < 1 || nrhs > S->opt.max_nrhs) return fail(PT_EINVAL, "nrhs must be in 1..max_nrhs");
  if (N->n && N->n != S->NX) return fail(PT_EINVAL, "all samples of a network must share the interface length");
  const int n = S->NX, L1 = S->L - 1;
  const int64_t Nt = S->Nt;
  if (!N->X.p) {
    N->n = n;
    if (N->X.alloc((size_t)N->capacity * 8 * n) != hipSuccess || N->T.alloc((size_t)N->capacity * 8 * n) != hipSuccess)
      return fail(PT_ENOMEM, "training samples");
  }
  hipStream_t st = S->st;
  const double2* fd = (const double2*)f;
  if (!on_device) {
    HIPCHK(hipMemcpyAsync(S->fio.p, f, (size_t)nrhs * S->NZ * S->NX * 16, hipMemcpyHostToDevice, st));
    fd = S->fio.p;
  }
  // Krylov vectors of the sweep-only trace solve
  PTCHK(trace_rhs(S, fd, S->s.p, nrhs));
  bool conv = false;
  PTCHK(fgmres(S, nrhs, conv, S->opt.tol, false));
  std::vector<int32_t> it(nrhs);
  HIPCHK(hipMemcpyAsync(it.data(), S->iters.p, nrhs * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  int J = S->opt.maxit;
  for (int r = 0; r < nrhs; ++r) J = std::min(J, (int)it[r]);
  J = std::min(J, (N->capacity - N->count) / (nrhs * L1));
  if (added) *added = 0;
  if (J <= 0) return PT_OK;
  DevBuf<double2> vs, gs;
  if (vs.alloc((size_t)J * nrhs * Nt) != hipSuccess || gs.alloc((size_t)nrhs * Nt) != hipSuccess) {
    vs.release();
    return fail(PT_ENOMEM, "collection workspace");
  }
  pt_status rc = PT_OK;
  auto hchk = [&](hipError_t e) {
    if (e != hipSuccess && rc == PT_OK) rc = fail(PT_EHIP, hipGetErrorString(e));
    return rc == PT_OK;
  };
  hchk(hipMemcpyAsync(vs.p, S->V.p, (size_t)J * nrhs * Nt * 16, hipMemcpyDeviceToDevice, st));
  if (rc == PT_OK) rc = ensure_ws(N, nrhs * L1, n);
  for (int j = 0; j < J && rc == PT_OK; ++j) {
    const double2* vj = vs.p + (size_t)j * nrhs * Nt;
    // r = v - A GS(v) becomes the right-hand side of a tight trace solve for e = A^-1 r
    rc = system_M(S, vj, gs.p, nrhs);
    if (rc == PT_OK) rc = system_A(S, gs.p, S->tmp.p, nrhs);
    if (rc != PT_OK) break;
    if (!hchk(launch_add(S->s.p, vj, S->tmp.p, -1.0, (int64_t)nrhs * Nt, st))) break;
    float* Xo = N->X.p + (size_t)N->count * 8 * n;
    float* To = N->T.p + (size_t)N->count * 8 * n;
    hipLaunchKernelGGL(pack_kernel, dim3(nrhs * L1), dim3(kThreadsL), 0, st, (const double2*)S->s.p, Xo, N->scale.p,
                       L1, n, 0);
    if (!hchk(hipGetLastError())) break;
    bool c2 = false;
    rc = fgmres(S, nrhs, c2, std::min(S->opt.tol, 1e-11), false);
    if (rc != PT_OK) break;
    hipLaunchKernelGGL(pack_kernel, dim3(nrhs * L1), dim3(kThreadsL), 0, st, (const double2*)S->x.p, To, N->scale.p,
                       L1, n, 1);
    if (!hchk(hipGetLastError())) break;
    N->count += nrhs * L1;
    if (added) *added += nrhs * L1;
  }
  hchk(hipStreamSynchronize(st));
  vs.release();
  gs.release();
  return rc;
}

pt_status pt_learned_train(pt_learned* N, int32_t steps, int32_t batch, double lr, double* loss_per_step) {
  if (!N || steps < 0 || batch < 1 || !(lr > 0)) return fail(PT_EINVAL, "bad arguments");
  if (N->count < 1) return fail(PT_EINVAL, "no training samples");
  const int n = N->n, m = 8 * n;
  PTCHK(ensure_ws(N, batch, n));
  std::vector<int32_t> idx(batch);
  std::vector<float> lv(batch);
  const float b1 = 0.9f, b2 = 0.999f;
  for (int s = 0; s < steps; ++s) {
    for (int b = 0; b < batch; ++b) idx[b] = (int32_t)(N->rng.next() % (uint64_t)N->count);
    HIPCHK(hipMemcpyAsync(N->idx.p, idx.data(), batch * 4, hipMemcpyHostToDevice, N->st));
    hipLaunchKernelGGL(gather_kernel, dim3(blocks_for((int64_t)batch * m)), dim3(256), 0, N->st, N->X.p, N->idx.p,
                       N->act[0].p, batch, m);
    hipLaunchKernelGGL(gather_kernel, dim3(blocks_for((int64_t)batch * m)), dim3(256), 0, N->st, N->T.p, N->idx.p,
                       N->tgt.p, batch, m);
    HIPCHK(hipGetLastError());
    PTCHK(net_forward(N, batch, n));
    PTCHK(net_backward(N, batch, n));
    ++N->adam_t;
    const float bc1 = 1.f - std::pow(b1, (float)N->adam_t), bc2 = 1.f - std::pow(b2, (float)N->adam_t);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(N->np)), dim3(256), 0, N->st, N->w32.p, N->w16.p, N->grad.p,
                       N->m.p, N->v.p, N->np, (float)lr, b1, b2, 1e-8f, bc1, bc2);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(lv.data(), N->lossv.p, batch * 4, hipMemcpyDeviceToHost, N->st));
    HIPCHK(hipStreamSynchronize(N->st));  // the index vector is reused next step
    if (loss_per_step) {
      double a = 0;
      for (float v : lv) a += v;
      loss_per_step[s] = a / batch;
    }
  }
  return PT_OK;
}

pt_status pt_solver_set_learned(pt_solver* S, pt_learned* N, int32_t mode) {
  if (!S) return fail(PT_EINVAL, "null solver");
  if (N && S->L < 2) return fail(PT_EINVAL, "no interfaces (L = 1)");
  if (mode != PT_LEARN_CORRECT && mode != PT_LEARN_AUGMENT) return fail(PT_EINVAL, "unknown learned mode");
  S->learned = N;
  S->learned_mode = mode;
  return PT_OK;
}

pt_status pt_learned_save(const pt_learned* N, const char* path) {
  if (!N || !path) return fail(PT_EINVAL, "null argument");
  std::vector<float> h(N->np);
  PTCHK(pt_learned_get_params(N, h.data()));
  std::ofstream o(path, std::ios::binary);
  if (!o) return fail(PT_EINVAL, "cannot open file");
  const char magic[8] = {'P', 'T', 'C', 'N', 'N', '2', 0, 0};  // 2: the dilated layers
  o.write(magic, 8);
  const int64_t np = N->np;
  o.write(reinterpret_cast<const char*>(&np), 8);
  o.write(reinterpret_cast<const char*>(h.data()), np * 4);
  return o ? PT_OK : fail(PT_EINVAL, "write failed");
}

pt_status pt_learned_load(pt_learned* N, const char* path) {
  if (!N || !path) return fail(PT_EINVAL, "null argument");
  std::ifstream in(path, std::ios::binary);
  if (!in) return fail(PT_EINVAL, "cannot open file");
  char magic[8];
  int64_t np = 0;
  in.read(magic, 8);
  in.read(reinterpret_cast<char*>(&np), 8);
  if (!in || std::memcmp(magic, "PTCNN2", 6) != 0 || np != N->np) return fail(PT_EINVAL, "not a network file");
  std::vector<float> h(np);
  in.read(reinterpret_cast<char*>(h.data()), np * 4);
  if (!in) return fail(PT_EINVAL, "truncated network file");
  return pt_learned_set_params(N, h.data());
}

}  // extern "C"
