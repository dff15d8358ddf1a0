// Split-bfloat16 block apply on MFMA (gfx950): Y = P + alpha sum_t M_t (Q_t + beta_t S_t)
// with every complex block M_t held as four bfloat16 planes, M = (Mr_hi + Mr_lo) + i (Mi_hi + Mi_lo),
// and the float64 input X = Q + beta S split the same way when it is staged.  Each real
// product is formed as hi*hi + hi*lo + lo*hi with float32 accumulation (the lo*lo term,
// 2^-16 below the result, is dropped), about 16 significant bits, which is what a
// preconditioner needs: flexible GMRES restores full accuracy from float64 operators.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "polar_kernels.h"

namespace polar {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kSpK = 32;  // block columns (k) per chunk: the MFMA depth of v_mfma_f32_16x16x32_bf16

__device__ __forceinline__ double2* sp_base(const Bases& b, int buf) {
  return buf == 0 ? b.b[0] : buf == 1 ? b.b[1] : buf == 2 ? b.b[2] : buf == 3 ? b.b[3] : nullptr;
}

// global-memory views: loads through them compile to global_load, not flat_load
typedef __attribute__((address_space(1))) const bf16x8 gbf16x8;
typedef double d2v __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const d2v gdouble2;
__device__ __forceinline__ const gdouble2* to_global(const double2* p) {
  return reinterpret_cast<const gdouble2*>(reinterpret_cast<uintptr_t>(p));
}
__device__ __forceinline__ double2 ldg(const gdouble2* p, int64_t i) {
  const d2v v = p[i];
  return make_double2(v.x, v.y);
}

// hi = bf16(x), lo = bf16(x - hi), both rounded to nearest
__device__ __forceinline__ void split2(double x, __bf16& hi, __bf16& lo) {
  hi = static_cast<__bf16>(static_cast<float>(x));
  lo = static_cast<__bf16>(static_cast<float>(x - static_cast<double>(static_cast<float>(hi))));
}

// ----------------------------------------------------------------------------
// setup: float64 row-major blocks -> swizzled split planes
// ----------------------------------------------------------------------------
// Tile (rt, kt) of a block covers rows 16 rt .. 16 rt + 15 and columns
// 32 kt .. 32 kt + 31; it stores 4 planes (re hi, re lo, im hi, im lo) of 64
// lanes x 8 values: lane l holds row 16 rt + l % 16, columns 32 kt + 8 (l / 16)
// + 0..7, exactly the A operand of the MFMA, so a wave reads each plane of a
// tile as one contiguous KiB.  Entries beyond n are zero.
__global__ void split_planes_kernel(const double2* __restrict__ src, __bf16* __restrict__ dst, int n, int nrt16,
                                    int nkt) {
  const int b = blockIdx.y;
  const int64_t tiles = (int64_t)nrt16 * nkt;
  const int64_t lanes = tiles * 64;
  const double2* M = src + (size_t)b * n * n;
  __bf16* D = dst + (size_t)b * tiles * 4 * 512;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < lanes; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t tile = e >> 6;
    const int l = (int)(e & 63);
    const int rt = (int)(tile / nkt), kt = (int)(tile % nkt);
    const int row = rt * 16 + (l & 15);
    const int k0 = kt * kSpK + 8 * (l >> 4);
    bf16x8 rh, rl, ih, il;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + u;
      const double2 v = (row < n && k < n) ? M[(size_t)row * n + k] : make_double2(0.0, 0.0);
      __bf16 h, lo;
      split2(v.x, h, lo);
      rh[u] = h;
      rl[u] = lo;
      split2(v.y, h, lo);
      ih[u] = h;
      il[u] = lo;
    }
    bf16x8* T = reinterpret_cast<bf16x8*>(D + tile * 4 * 512);
    T[0 * 64 + l] = rh;
    T[1 * 64 + l] = rl;
    T[2 * 64 + l] = ih;
    T[3 * 64 + l] = il;
  }
}

// ----------------------------------------------------------------------------
// block apply
// ----------------------------------------------------------------------------
// One workgroup = KS waves = one 16-row x 16 NB-right-hand-side output tile of
// one job; wave w takes the chunks w, w + KS, ... of the job's (term, 32-column)
// chunk sequence, so short sweeps still put several waves per SIMD in flight.
// A wave reads its A operands straight from the swizzled planes and loads its
// B operands straight into registers: lane l of a 16-column tile needs rows
// 8 (l / 16) + 0..7 of column l % 16 of the input chunk, i.e. 8 consecutive
// float64 pairs, which it combines (Q + beta S), splits and feeds to the MFMA;
// the next chunk's loads are in flight during the current chunk's MFMAs.  Four
// float32 accumulators per column tile (Mr Xr, Mi Xi, Mr Xi, Mi Xr), three
// MFMAs each per chunk, are interleaved so consecutive MFMAs are independent.
// The KS partial tiles are summed through LDS in a fixed order by wave 0: no
// atomics, deterministic results.
template <int NB, int KS>
__global__ __launch_bounds__(64 * KS) void block_split_kernel(const Job* __restrict__ jobs, int n, int nrt16,
                                                              int nct, int nrhs, int64_t ld, Bases bases) {
  __shared__ f32x4 red[KS > 1 ? KS - 1 : 1][4][NB][64];
  const int lane = threadIdx.x & 63;
  // wave-uniform, so chunk and term indices, job fields and base pointers stay scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int bid = blockIdx.x;
  const int ct = bid % nct;
  bid /= nct;
  const int rt = bid % nrt16;
  const Job& J = jobs[bid / nrt16];
  const int nkt = (n + kSpK - 1) / kSpK;
  const int col0 = ct * 16 * NB;
  const int kl = 8 * (lane >> 4);  // first of the 8 chunk columns (k) this lane feeds

  f32x4 acc[4][NB];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int nchunks = J.nterms * nkt;
  bf16x8 pa[4];
  double2 xq[NB][8], xs[NB][8];  // raw input of the chunk in flight: Q and S rows
  bool has_q = false, has_s = false;
  double2 beta = make_double2(0.0, 0.0);
  int kfetch = 0;  // first input row of the chunk in flight for this lane
  // Loads only, all unconditional (indices clamped into the vectors): the
  // combination Q + beta S and the masking of rows >= n or columns >= nrhs
  // wait until the values are consumed, so every load of a chunk is in flight
  // together and no branch splits them.
  auto fetch = [&](int q) {
    const int t = q / nkt;
    const int kt = q - t * nkt;
    const gbf16x8* T = reinterpret_cast<const gbf16x8*>(
        reinterpret_cast<uintptr_t>(static_cast<const __bf16*>(J.M[t]) + ((size_t)rt * nkt + kt) * 4 * 512));
#pragma unroll
    for (int p = 0; p < 4; ++p) pa[p] = T[p * 64 + lane];
    const VecRef qr = J.Q[t];
    const VecRef svr = J.S[t];
    has_q = qr.buf >= 0;
    has_s = svr.buf >= 0;
    beta = J.beta[t];
    kfetch = kt * kSpK + kl;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int rhs = min(col0 + b * 16 + (lane & 15), nrhs - 1);
      if (has_q) {
        const gdouble2* __restrict__ qp = to_global(sp_base(bases, qr.buf) + qr.off + (int64_t)rhs * ld);
#pragma unroll
        for (int u = 0; u < 8; ++u) xq[b][u] = ldg(qp, min(kfetch + u, n - 1));
      }
      if (has_s) {
        const gdouble2* __restrict__ sp = to_global(sp_base(bases, svr.buf) + svr.off + (int64_t)rhs * ld);
#pragma unroll
        for (int u = 0; u < 8; ++u) xs[b][u] = ldg(sp, min(kfetch + u, n - 1));
      }
    }
  };
  if (wave < nchunks) fetch(wave);
  for (int q = wave; q < nchunks; q += KS) {
    const bf16x8 ar_h = pa[0], ar_l = pa[1], ai_h = pa[2], ai_l = pa[3];
    bf16x8 xr_h[NB], xr_l[NB], xi_h[NB], xi_l[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const bool col_ok = col0 + b * 16 + (lane & 15) < nrhs;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        double2 v = has_q ? xq[b][u] : make_double2(0.0, 0.0);
        if (has_s) {
          const double2 w = xs[b][u];
          v.x += beta.x * w.x - beta.y * w.y;
          v.y += beta.x * w.y + beta.y * w.x;
        }
        if (!(col_ok && kfetch + u < n)) v = make_double2(0.0, 0.0);
        __bf16 h, lo;
        split2(v.x, h, lo);
        xr_h[b][u] = h;
        xr_l[b][u] = lo;
        split2(v.y, h, lo);
        xi_h[b][u] = h;
        xi_l[b][u] = lo;
      }
    }
    if (q + KS < nchunks) fetch(q + KS);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      acc[0][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar_h, xr_h[b], acc[0][b], 0, 0, 0);
      acc[1][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai_h, xi_h[b], acc[1][b], 0, 0, 0);
      acc[2][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar_h, xi_h[b], acc[2][b], 0, 0, 0);
      acc[3][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai_h, xr_h[b], acc[3][b], 0, 0, 0);
      acc[0][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar_h, xr_l[b], acc[0][b], 0, 0, 0);
      acc[1][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai_h, xi_l[b], acc[1][b], 0, 0, 0);
      acc[2][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar_h, xi_l[b], acc[2][b], 0, 0, 0);
      acc[3][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai_h, xr_l[b], acc[3][b], 0, 0, 0);
      acc[0][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar_l, xr_h[b], acc[0][b], 0, 0, 0);
      acc[1][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai_l, xi_h[b], acc[1][b], 0, 0, 0);
      acc[2][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar_l, xi_h[b], acc[2][b], 0, 0, 0);
      acc[3][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai_l, xr_h[b], acc[3][b], 0, 0, 0);
    }
  }

  if constexpr (KS > 1) {
    if (wave > 0)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) red[wave - 1][a][b][lane] = acc[a][b];
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int w = 0; w < KS - 1; ++w)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] += red[w][a][b][lane];
  }

  double2* __restrict__ Yb = sp_base(bases, J.Y.buf) + J.Y.off;
  const double2* __restrict__ Pb = J.P.buf >= 0 ? sp_base(bases, J.P.buf) + J.P.off : nullptr;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = rt * 16 + 4 * (lane >> 4) + i;
      const int rhs = col0 + b * 16 + (lane & 15);
      if (row < n && rhs < nrhs) {
        const double yr = (double)acc[0][b][i] - (double)acc[1][b][i];
        const double yi = (double)acc[2][b][i] + (double)acc[3][b][i];
        double2 y = make_double2(J.alpha.x * yr - J.alpha.y * yi, J.alpha.x * yi + J.alpha.y * yr);
        if (Pb) {
          const double2 p = Pb[(int64_t)rhs * ld + row];
          y.x += p.x;
          y.y += p.y;
        }
        Yb[(int64_t)rhs * ld + row] = y;
      }
    }
}

template <int NB, int KS>
hipError_t launch_sp(const Job* jobs, int njobs, int n, int nrhs, int64_t ld, Bases bases, hipStream_t st,
                     hipEvent_t ev0, hipEvent_t ev1) {
  const int nrt16 = (n + 15) / 16;
  const int nct = (nrhs + 16 * NB - 1) / (16 * NB);
  const dim3 grid((unsigned)njobs * nrt16 * nct);
  hipExtLaunchKernelGGL((block_split_kernel<NB, KS>), grid, dim3(64 * KS), 0, st, ev0, ev1, 0, jobs, n, nrt16, nct,
                        nrhs, ld, bases);
  return hipGetLastError();
}

template <int NB>
hipError_t launch_sp_ks(int ks, const Job* jobs, int njobs, int n, int nrhs, int64_t ld, Bases bases, hipStream_t st,
                        hipEvent_t ev0, hipEvent_t ev1) {
  if (ks >= 4) return launch_sp<NB, 4>(jobs, njobs, n, nrhs, ld, bases, st, ev0, ev1);
  if (ks == 2) return launch_sp<NB, 2>(jobs, njobs, n, nrhs, ld, bases, st, ev0, ev1);
  return launch_sp<NB, 1>(jobs, njobs, n, nrhs, ld, bases, st, ev0, ev1);
}

}  // namespace

size_t split_block_elems(int n) {
  const size_t nrt16 = (n + 15) / 16, nkt = (n + kSpK - 1) / kSpK;
  return nrt16 * nkt * 4 * 512;
}

hipError_t launch_split_planes(const double2* src, void* dst, int nblk, int n, hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  const int nrt16 = (n + 15) / 16, nkt = (n + kSpK - 1) / kSpK;
  const int64_t lanes = (int64_t)nrt16 * nkt * 64;
  const unsigned gx = (unsigned)std::min<int64_t>((lanes + 255) / 256, 1024);
  hipLaunchKernelGGL(split_planes_kernel, dim3(gx, nblk), dim3(256), 0, st, src, static_cast<__bf16*>(dst), n, nrt16,
                     nkt);
  return hipGetLastError();
}

hipError_t launch_block_apply_split(const Job* jobs, int njobs, int n, int nrhs, int64_t ld, Bases bases,
                                    hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (njobs <= 0) return hipSuccess;
  // 16-column tiles; the chunks of a tile are split over up to 4 waves until
  // the launch has about 4 waves per SIMD
  constexpr long kSimds = 1024;
  const long tasks = (long)njobs * ((n + 15) / 16) * ((nrhs + 15) / 16);
  const int ks = tasks >= 4 * kSimds ? 1 : tasks >= 2 * kSimds ? 2 : 4;
  return launch_sp_ks<1>(ks, jobs, njobs, n, nrhs, ld, bases, st, ev0, ev1);
}

}  // namespace polar
