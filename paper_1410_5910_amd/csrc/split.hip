// Split block apply on MFMA (gfx950): Y = P + alpha sum_t M_t (Q_t + beta_t S_t) with every
// complex block M_t held as four 16-bit planes, M = (Mr_hi + Mr_lo) + i (Mi_hi + Mi_lo), and the
// float64 input X = Q + beta S split the same way when it is staged.  Each real product is
// formed as hi*hi + hi*lo + lo*hi with float32 accumulation (the lo*lo term is dropped).
// Two element types: bfloat16 (about 16 significant bits per pair; float32's exponent range,
// no scaling) and float16 (about 22 significant bits; a 5-bit exponent, so the blocks are
// stored scaled by a power of two chosen at setup, the inputs are multiplied by 2^12 as they
// are split, and both factors are folded into the jobs' alpha).  Either is what a
// preconditioner needs: flexible GMRES restores full accuracy from float64 operators.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>

#include "polar_kernels.h"

namespace polar {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// The element type of the split planes and the MFMA that consumes them.
struct SpBf16 {
  typedef __bf16 E;
  typedef __bf16 v8 __attribute__((ext_vector_type(8)));
  typedef __bf16 v2 __attribute__((ext_vector_type(2)));
  static constexpr double kX = 1.0;  // input scale at the split
  static __device__ __forceinline__ f32x4 mfma(v8 a, v8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  // hi = bf16(x), lo = bf16(x - hi), both rounded to nearest
  static __device__ __forceinline__ void split(double x, E& hi, E& lo) {
    hi = static_cast<__bf16>(static_cast<float>(x));
    lo = static_cast<__bf16>(static_cast<float>(x - static_cast<double>(static_cast<float>(hi))));
  }
  // the same from a float32 value (x - hi is exact in float32: at most 17 significant bits)
  static __device__ __forceinline__ void splitf(float x, E& hi, E& lo) {
    hi = static_cast<__bf16>(x);
    lo = static_cast<__bf16>(x - static_cast<float>(hi));
  }
};
struct SpF16 {
  typedef _Float16 E;
  typedef _Float16 v8 __attribute__((ext_vector_type(8)));
  typedef _Float16 v2 __attribute__((ext_vector_type(2)));
  static constexpr double kX = 4096.0;
  static __device__ __forceinline__ f32x4 mfma(v8 a, v8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ void split(double x, E& hi, E& lo) {
    hi = static_cast<_Float16>(static_cast<float>(x));
    lo = static_cast<_Float16>(static_cast<float>(x - static_cast<double>(static_cast<float>(hi))));
  }
  static __device__ __forceinline__ void splitf(float x, E& hi, E& lo) {
    hi = static_cast<_Float16>(x);
    lo = static_cast<_Float16>(x - static_cast<float>(hi));
  }
};

// a 16-byte vector at element i of a global array (a global_load, not a flat_load)
template <typename V>
__device__ __forceinline__ V gload(const void* p, int64_t i) {
  typedef __attribute__((address_space(1))) const V gv;
  return reinterpret_cast<const gv*>(reinterpret_cast<uintptr_t>(p))[i];
}

constexpr int kSpK = 32;  // block columns (k) per chunk: the MFMA depth of v_mfma_f32_16x16x32_{bf16,f16}

__device__ __forceinline__ double2* sp_base(const Bases& b, int buf) {
  return buf == 0 ? b.b[0] : buf == 1 ? b.b[1] : buf == 2 ? b.b[2] : buf == 3 ? b.b[3] : nullptr;
}

// global-memory views of the float64 inputs
typedef double d2v __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const d2v gdouble2;
__device__ __forceinline__ const gdouble2* to_global(const double2* p) {
  return reinterpret_cast<const gdouble2*>(reinterpret_cast<uintptr_t>(p));
}
__device__ __forceinline__ double2 ldg(const gdouble2* p, int64_t i) {
  const d2v v = p[i];
  return make_double2(v.x, v.y);
}

// Workgroup ids are dealt round-robin to the 8 XCDs, each with its own L2.
// Renumber so that every XCD gets one contiguous range of logical ids: tiles
// next to each other in logical order (sharing block rows or input columns)
// then meet in the same L2.
__device__ __forceinline__ int xcd_logical(int i, int G) {
  constexpr int kXcd = 8;
  const int x = i % kXcd, local = i / kXcd;
  const int per = G / kXcd, rem = G % kXcd;
  return x < rem ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

// Workgroup barrier that orders LDS only: waits for this wave's LDS operations,
// not for its global loads, so loads issued for later chunks stay in flight
// across it (a full __syncthreads() also drains the vector-memory counter).
__device__ __forceinline__ void lds_barrier() { __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Slot of B-operand lane l in a staged 16-column plane tile (64 slots of 16 bytes).  The staging
// stores write 4-byte pairs: the 16 lanes of a column put row pairs into slots l, l + 16, l + 32 and
// l + 48, which share LDS banks; XORing bits 1-2 of the slot with bits 4-5 spreads one 32-lane
// store over all 32 banks, and any 8 consecutive operand reads still cover the 8 bank groups.
__device__ __forceinline__ int sp_swz(int l) { return l ^ (2 * ((l >> 4) & 3)); }

// Q + beta S of one complex input entry, in float32 (the split pair keeps at most 22 bits of it)
__device__ __forceinline__ float2 combine_f(double2 q, double2 sv, double2 beta, bool has_q, bool has_s) {
  float2 v = has_q ? make_float2(static_cast<float>(q.x), static_cast<float>(q.y)) : make_float2(0.f, 0.f);
  if (has_s) {
    const float wx = static_cast<float>(sv.x), wy = static_cast<float>(sv.y);
    const float bx = static_cast<float>(beta.x), by = static_cast<float>(beta.y);
    v.x = fmaf(bx, wx, fmaf(-by, wy, v.x));
    v.y = fmaf(bx, wy, fmaf(by, wx, v.y));
  }
  return v;
}

// ----------------------------------------------------------------------------
// setup: float64 row-major blocks -> swizzled split planes
// ----------------------------------------------------------------------------
// Tile (rt, kt) of a block covers rows 16 rt .. 16 rt + 15 and columns
// 32 kt .. 32 kt + 31; it stores 4 planes (re hi, re lo, im hi, im lo) of 64
// lanes x 8 values: lane l holds row 16 rt + l % 16, columns 32 kt + 8 (l / 16)
// + 0..7, exactly the A operand of the MFMA, so a wave reads each plane of a
// tile as one contiguous KiB.  Entries beyond n are zero; entries are
// multiplied by `scale` (a power of two: exact) before the split.
template <typename T>
__global__ void split_planes_kernel(const double2* __restrict__ src, typename T::E* __restrict__ dst, int n,
                                    int nrt16, int nkt, double scale) {
  typedef typename T::v8 v8;
  const int b = blockIdx.y;
  const int64_t tiles = (int64_t)nrt16 * nkt;
  const int64_t lanes = tiles * 64;
  const double2* M = src + (size_t)b * n * n;
  typename T::E* D = dst + (size_t)b * tiles * 4 * 512;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < lanes; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t tile = e >> 6;
    const int l = (int)(e & 63);
    const int rt = (int)(tile / nkt), kt = (int)(tile % nkt);
    const int row = rt * 16 + (l & 15);
    const int k0 = kt * kSpK + 8 * (l >> 4);
    v8 rh, rl, ih, il;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + u;
      const double2 v = (row < n && k < n) ? M[(size_t)row * n + k] : make_double2(0.0, 0.0);
      typename T::E h, lo;
      T::split(v.x * scale, h, lo);
      rh[u] = h;
      rl[u] = lo;
      T::split(v.y * scale, h, lo);
      ih[u] = h;
      il[u] = lo;
    }
    v8* P = reinterpret_cast<v8*>(D + tile * 4 * 512);
    P[0 * 64 + l] = rh;
    P[1 * 64 + l] = rl;
    P[2 * 64 + l] = ih;
    P[3 * 64 + l] = il;
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
template <typename T, int NB, int KS, int NS>
__global__ __launch_bounds__(64 * KS) void block_split_kernel(const SegTableT<NS> tab,
                                                              const Job* __restrict__ jobs1) {
  typedef typename T::v8 bf16x8;
  __shared__ f32x4 red[KS > 1 ? KS - 1 : 1][4][NB][64];
  const int lane = threadIdx.x & 63;
  // wave-uniform, so chunk and term indices, job fields and base pointers stay scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int bid = blockIdx.x;
  // segment of this block: a0 = 16-row tiles, a1 = column tiles
  const int seg = seg_of(tab, bid);
  const Job* __restrict__ jobs = NS == 1 ? jobs1 : tab.jobs[seg];
  const int n = tab.n[seg], nrt16 = tab.a0[seg], nct = tab.a1[seg], nrhs = tab.nrhs[seg];
  const int64_t ld = tab.ld[seg];
  const Bases bases = tab.bases[seg];
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
    const typename T::E* tp = static_cast<const typename T::E*>(J.M[t]) + ((size_t)rt * nkt + kt) * 4 * 512;
#pragma unroll
    for (int p = 0; p < 4; ++p) pa[p] = gload<bf16x8>(tp, p * 64 + lane);
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
        float2 v = combine_f(xq[b][u], xs[b][u], beta, has_q, has_s);
        if (!(col_ok && kfetch + u < n)) v = make_float2(0.f, 0.f);
        typename T::E h, lo;
        T::splitf(v.x * static_cast<float>(T::kX), h, lo);
        xr_h[b][u] = h;
        xr_l[b][u] = lo;
        T::splitf(v.y * static_cast<float>(T::kX), h, lo);
        xi_h[b][u] = h;
        xi_l[b][u] = lo;
      }
    }
    if (q + KS < nchunks) fetch(q + KS);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      acc[0][b] = T::mfma(ar_h, xr_h[b], acc[0][b]);
      acc[1][b] = T::mfma(ai_h, xi_h[b], acc[1][b]);
      acc[2][b] = T::mfma(ar_h, xi_h[b], acc[2][b]);
      acc[3][b] = T::mfma(ai_h, xr_h[b], acc[3][b]);
      acc[0][b] = T::mfma(ar_h, xr_l[b], acc[0][b]);
      acc[1][b] = T::mfma(ai_h, xi_l[b], acc[1][b]);
      acc[2][b] = T::mfma(ar_h, xi_l[b], acc[2][b]);
      acc[3][b] = T::mfma(ai_h, xr_l[b], acc[3][b]);
      acc[0][b] = T::mfma(ar_l, xr_h[b], acc[0][b]);
      acc[1][b] = T::mfma(ai_l, xi_h[b], acc[1][b]);
      acc[2][b] = T::mfma(ar_l, xi_h[b], acc[2][b]);
      acc[3][b] = T::mfma(ai_l, xr_h[b], acc[3][b]);
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

// Wide form for many right-hand sides: one group of 4 waves = a 64-row x
// 16 NB-right-hand-side output tile; wave w owns the 16-row tile 4 tile + w
// and all NB 16-column tiles (12 NB MFMAs per chunk).  The 32 x 16 NB input
// chunk is loaded once per group and shared by the 4 waves through LDS, so
// each input element is read once per 64 output rows.  The loads run down the
// columns: thread t takes row pairs (2 (p % 16), 2 (p % 16) + 1) of column
// p / 16 for p = t + 256 i, i < NB, so a wave reads 4 columns x 512
// contiguous bytes per instruction; each pair is combined (Q + beta S), split and written into the
// B operand layout (lane l: rows 8 (l / 16) + 0..7 of column l % 16) as 4-byte
// words.  KS groups split the chunk sequence of the tile (KS = 1, 2); their
// partial tiles are summed through LDS one group at a time, in a fixed order.
constexpr int kWideRows = 64;

template <typename T, int NB, int KS, int NS>
__global__ __launch_bounds__(256 * KS) void block_split_wide_kernel(const SegTableT<NS> tab, int kslices,
                                                                    const Job* __restrict__ jobs1) {
  typedef typename T::v8 bf16x8;
  constexpr int kWideCols = 16 * NB;
  constexpr int PPT = kSpK * kWideCols / 2 / 256;                          // row pairs per thread: NB
  constexpr size_t kPlane = (size_t)NB * 64 * sizeof(bf16x8);              // one plane of a chunk
  constexpr size_t kStage = (size_t)KS * 4 * kPlane;                       // split input planes of every group
  constexpr size_t kRed = KS > 1 ? (size_t)4 * 64 * 4 * NB * sizeof(f32x4) : 0;  // one group's partial tiles
  __shared__ __align__(16) unsigned char smem[kStage > kRed ? kStage : kRed];
  const int tid = threadIdx.x & 255;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x >> 8);
  unsigned char* gst = smem + (size_t)grp * 4 * kPlane;  // this group's planes
  // logical order, fastest first: column tile, row tile, k-slice, job -- so an
  // XCD's range shares block rows (across column tiles) and input rows (across
  // row tiles) in its L2
  int bid = xcd_logical(blockIdx.x, gridDim.x);
  // segment of this block (segments stay contiguous in the logical order):
  // a0 = 64-row tiles, a1 = column tiles, part = its k-slice partial tiles
  const int seg = seg_of(tab, bid);
  const Job* __restrict__ jobs = NS == 1 ? jobs1 : tab.jobs[seg];
  const int n = tab.n[seg], ntiles = tab.a0[seg], nct = tab.a1[seg], nrhs = tab.nrhs[seg], njobs = tab.njobs[seg];
  const int64_t ld = tab.ld[seg];
  const Bases bases = tab.bases[seg];
  float2* __restrict__ part = tab.part[seg];
  const int ct = bid % nct;
  bid /= nct;
  const int tile = bid % ntiles;
  bid /= ntiles;
  const int slice = bid % kslices;  // k-slice of the tile (kslices > 1: partial tile to `part`)
  const int job = bid / kslices;
  const Job& J = jobs[job];
  const int nkt = (n + kSpK - 1) / kSpK;
  const int nrt16 = (n + 15) / 16;
  const int rt = tile * 4 + wave;
  const bool rt_ok = rt < nrt16;
  const int rtc = rt_ok ? rt : nrt16 - 1;  // clamped: loads stay inside the block
  const int col0 = ct * kWideCols;

  f32x4 acc[4][NB];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  // chunk range of this k-slice: [qbeg, qend)
  const int nall = J.nterms * nkt;
  const int cps = (nall + kslices - 1) / kslices;
  const int qbeg = min(slice * cps, nall);
  const int nchunks = min(nall, qbeg + cps) - qbeg;
  const int rounds = (nchunks + KS - 1) / KS;  // the same for every group: barriers stay uniform
  bf16x8 pa[4];
  double2 xq[PPT][2], xs[PPT][2];
  bool live = false, has_q = false, has_s = false;
  double2 beta = make_double2(0.0, 0.0);
  int kbase = 0;
  auto fetch = [&](int qi) {
    live = qi < nchunks;
    if (!live) return;
    const int q = qbeg + qi;
    const int t = q / nkt;
    const int kt = q - t * nkt;
    const typename T::E* tp = static_cast<const typename T::E*>(J.M[t]) + ((size_t)rtc * nkt + kt) * 4 * 512;
#pragma unroll
    for (int p = 0; p < 4; ++p) pa[p] = gload<bf16x8>(tp, p * 64 + lane);
    const VecRef qr = J.Q[t];
    const VecRef svr = J.S[t];
    has_q = qr.buf >= 0;
    has_s = svr.buf >= 0;
    beta = J.beta[t];
    kbase = kt * kSpK;
    const double2* qb = has_q ? sp_base(bases, qr.buf) + qr.off : nullptr;
    const double2* sb = has_s ? sp_base(bases, svr.buf) + svr.off : nullptr;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int pr = tid + 256 * i;
      const int k = kbase + 2 * (pr & 15);
      const int64_t e = (int64_t)min(col0 + (pr >> 4), nrhs - 1) * ld;
      const int k0c = min(k, n - 1), k1c = min(k + 1, n - 1);
      if (has_q) {
        const gdouble2* qp = to_global(qb + e);
        xq[i][0] = ldg(qp, k0c);
        xq[i][1] = ldg(qp, k1c);
      }
      if (has_s) {
        const gdouble2* sp = to_global(sb + e);
        xs[i][0] = ldg(sp, k0c);
        xs[i][1] = ldg(sp, k1c);
      }
    }
  };
  fetch(grp);
  for (int i = 0; i < rounds; ++i) {
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int pr = tid + 256 * j;
      const int kp = pr & 15, c = pr >> 4;  // row pair within the chunk, column within the tile
      const bool col_ok = live && col0 + c < nrhs;
      typename T::E h[4][2];  // [plane][row of the pair]
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        float2 v = combine_f(xq[j][u], xs[j][u], beta, has_q, has_s);
        if (!(col_ok && kbase + 2 * kp + u < n)) v = make_float2(0.f, 0.f);
        T::splitf(v.x * static_cast<float>(T::kX), h[0][u], h[1][u]);
        T::splitf(v.y * static_cast<float>(T::kX), h[2][u], h[3][u]);
      }
      // rows 2 kp, 2 kp + 1 sit at positions (2 kp) % 8, +1 of lane (2 kp / 8) * 16 + c % 16 of tile c / 16
      const int l = sp_swz(((2 * kp) >> 3) * 16 + (c & 15));
      const size_t off = ((size_t)(c >> 4) * 64 + l) * sizeof(bf16x8) + (size_t)((2 * kp) & 7) * 2;
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) {
        typename T::v2 w;
        w[0] = h[pl][0];
        w[1] = h[pl][1];
        *reinterpret_cast<typename T::v2*>(gst + pl * kPlane + off) = w;
      }
    }
    const bool mult = live;
    const bf16x8 ar_h = pa[0], ar_l = pa[1], ai_h = pa[2], ai_l = pa[3];
    lds_barrier();
    fetch((i + 1) * KS + grp);
    if (mult) {
      const bf16x8* P0 = reinterpret_cast<const bf16x8*>(gst);
      const bf16x8* P1 = reinterpret_cast<const bf16x8*>(gst + kPlane);
      const bf16x8* P2 = reinterpret_cast<const bf16x8*>(gst + 2 * kPlane);
      const bf16x8* P3 = reinterpret_cast<const bf16x8*>(gst + 3 * kPlane);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int sl = b * 64 + sp_swz(lane);
        const bf16x8 xr_h = P0[sl], xr_l = P1[sl];
        const bf16x8 xi_h = P2[sl], xi_l = P3[sl];
        acc[0][b] = T::mfma(ar_h, xr_h, acc[0][b]);
        acc[1][b] = T::mfma(ai_h, xi_h, acc[1][b]);
        acc[2][b] = T::mfma(ar_h, xi_h, acc[2][b]);
        acc[3][b] = T::mfma(ai_h, xr_h, acc[3][b]);
        acc[0][b] = T::mfma(ar_h, xr_l, acc[0][b]);
        acc[1][b] = T::mfma(ai_h, xi_l, acc[1][b]);
        acc[2][b] = T::mfma(ar_h, xi_l, acc[2][b]);
        acc[3][b] = T::mfma(ai_h, xr_l, acc[3][b]);
        acc[0][b] = T::mfma(ar_l, xr_h, acc[0][b]);
        acc[1][b] = T::mfma(ai_l, xi_h, acc[1][b]);
        acc[2][b] = T::mfma(ar_l, xi_h, acc[2][b]);
        acc[3][b] = T::mfma(ai_l, xr_h, acc[3][b]);
      }
    }
    lds_barrier();  // the next chunk's loads stay in flight
  }

  if constexpr (KS > 1) {
    f32x4* red = reinterpret_cast<f32x4*>(smem);  // [wave][a][b][lane]
#pragma unroll
    for (int g = 1; g < KS; ++g) {
      if (grp == g)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) red[((wave * 4 + a) * NB + b) * 64 + lane] = acc[a][b];
      __syncthreads();
      if (grp == 0)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) acc[a][b] += red[((wave * 4 + a) * NB + b) * 64 + lane];
      __syncthreads();
    }
    if (grp > 0) return;
  }

  if (!rt_ok) return;
  if (kslices > 1) {
    // partial tile of this k-slice: part[((slice * njobs + job) * nrhs + rhs) * n + row]
    float2* __restrict__ pt = part + ((size_t)slice * njobs + job) * nrhs * n;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rt * 16 + 4 * (lane >> 4) + i;
        const int rhs = col0 + b * 16 + (lane & 15);
        if (row < n && rhs < nrhs)
          pt[(size_t)rhs * n + row] = make_float2(acc[0][b][i] - acc[1][b][i], acc[2][b][i] + acc[3][b][i]);
      }
    return;
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

// The wide form specialised for launches whose jobs all have two terms with
// an input Q each and, when HAS_S, an S each (the Gauss-Seidel sweep steps and
// the reflection terms).  Every fetch of a chunk inside the slice issues the
// same loads with no branches (term pointers picked by selects), so two chunks
// can be in flight while a third is multiplied; the arithmetic and its order
// are those of block_split_wide_kernel<NB, 1>.
template <typename T, int NB, bool HAS_S, int NS>
__global__ __launch_bounds__(256) void block_split_stream_kernel(const SegTableT<NS> tab, int kslices,
                                                                 const Job* __restrict__ jobs1) {
  typedef typename T::v8 bf16x8;
  constexpr int kWideCols = 16 * NB;
  constexpr int PPT = kSpK * kWideCols / 2 / 256;              // row pairs per thread: NB
  constexpr size_t kPlane = (size_t)NB * 64 * sizeof(bf16x8);  // one plane of a chunk
  __shared__ __align__(16) unsigned char gst[4 * kPlane];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  int bid = xcd_logical(blockIdx.x, gridDim.x);
  // segment of this block (segments stay contiguous in the logical order):
  // a0 = 64-row tiles, a1 = column tiles, part = its k-slice partial tiles
  const int seg = seg_of(tab, bid);
  const Job* __restrict__ jobs = NS == 1 ? jobs1 : tab.jobs[seg];
  const int n = tab.n[seg], ntiles = tab.a0[seg], nct = tab.a1[seg], nrhs = tab.nrhs[seg], njobs = tab.njobs[seg];
  const int64_t ld = tab.ld[seg];
  const Bases bases = tab.bases[seg];
  float2* __restrict__ part = tab.part[seg];
  const int ct = bid % nct;
  bid /= nct;
  const int tile = bid % ntiles;
  bid /= ntiles;
  const int slice = bid % kslices;
  const int job = bid / kslices;
  const Job& J = jobs[job];
  const int nkt = (n + kSpK - 1) / kSpK;
  const int nrt16 = (n + 15) / 16;
  const int rt = tile * 4 + wave;
  const bool rt_ok = rt < nrt16;
  const int rtc = rt_ok ? rt : nrt16 - 1;
  const int col0 = ct * kWideCols;
  const typename T::E* const M0 = static_cast<const typename T::E*>(J.M[0]);
  const typename T::E* const M1 = static_cast<const typename T::E*>(J.M[1]);
  const double2* const q0 = sp_base(bases, J.Q[0].buf) + J.Q[0].off;
  const double2* const q1 = sp_base(bases, J.Q[1].buf) + J.Q[1].off;
  const double2* const s0 = HAS_S ? sp_base(bases, J.S[0].buf) + J.S[0].off : q0;
  const double2* const s1 = HAS_S ? sp_base(bases, J.S[1].buf) + J.S[1].off : q1;
  const double2 be0 = J.beta[0], be1 = J.beta[1];

  f32x4 acc[4][NB];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int nall = 2 * nkt;
  const int cps = (nall + kslices - 1) / kslices;
  const int qbeg = min(slice * cps, nall);
  const int nchunks = min(nall, qbeg + cps) - qbeg;
  struct InFlight {
    bf16x8 pa[4];
    double2 xq[PPT][2];
    double2 xs[HAS_S ? PPT : 1][2];
    int qi;
  };
  auto fetch = [&](InFlight& F, int qi) {
    F.qi = qi;
    if (qi >= nchunks) return;  // past the slice (workgroup-uniform): staged as zeros, not multiplied
    const int q = qbeg + qi;
    const bool t1 = q >= nkt;
    const int kt = t1 ? q - nkt : q;
    const typename T::E* Mt = (t1 ? M1 : M0) + ((size_t)rtc * nkt + kt) * 4 * 512;
#pragma unroll
    for (int p = 0; p < 4; ++p) F.pa[p] = gload<bf16x8>(Mt, p * 64 + lane);
    const double2* qb = t1 ? q1 : q0;
    const double2* sb = t1 ? s1 : s0;
    const int kbase = kt * kSpK;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int pr = tid + 256 * i;
      const int k = kbase + 2 * (pr & 15);
      const int64_t e = (int64_t)min(col0 + (pr >> 4), nrhs - 1) * ld;
      const int k0c = min(k, n - 1), k1c = min(k + 1, n - 1);
      const gdouble2* qp = to_global(qb + e);
      F.xq[i][0] = ldg(qp, k0c);
      F.xq[i][1] = ldg(qp, k1c);
      if constexpr (HAS_S) {
        const gdouble2* sp = to_global(sb + e);
        F.xs[i][0] = ldg(sp, k0c);
        F.xs[i][1] = ldg(sp, k1c);
      }
    }
  };
  auto stage = [&](const InFlight& F) {
    const bool live = F.qi < nchunks;
    const int q = qbeg + min(F.qi, nchunks - 1);
    const bool t1 = q >= nkt;
    const int kbase = (t1 ? q - nkt : q) * kSpK;
    const double2 beta = t1 ? be1 : be0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int pr = tid + 256 * j;
      const int kp = pr & 15, c = pr >> 4;
      const bool col_ok = live && col0 + c < nrhs;
      typename T::E h[4][2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        float2 v = combine_f(F.xq[j][u], F.xs[HAS_S ? j : 0][u], beta, true, HAS_S);
        if (!(col_ok && kbase + 2 * kp + u < n)) v = make_float2(0.f, 0.f);
        T::splitf(v.x * static_cast<float>(T::kX), h[0][u], h[1][u]);
        T::splitf(v.y * static_cast<float>(T::kX), h[2][u], h[3][u]);
      }
      const int l = sp_swz(((2 * kp) >> 3) * 16 + (c & 15));
      const size_t off = ((size_t)(c >> 4) * 64 + l) * sizeof(bf16x8) + (size_t)((2 * kp) & 7) * 2;
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) {
        typename T::v2 w;
        w[0] = h[pl][0];
        w[1] = h[pl][1];
        *reinterpret_cast<typename T::v2*>(gst + pl * kPlane + off) = w;
      }
    }
  };
  auto multiply = [&](const bf16x8& ar_h, const bf16x8& ar_l, const bf16x8& ai_h, const bf16x8& ai_l) {
    const bf16x8* P0 = reinterpret_cast<const bf16x8*>(gst);
    const bf16x8* P1 = reinterpret_cast<const bf16x8*>(gst + kPlane);
    const bf16x8* P2 = reinterpret_cast<const bf16x8*>(gst + 2 * kPlane);
    const bf16x8* P3 = reinterpret_cast<const bf16x8*>(gst + 3 * kPlane);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int sl = b * 64 + sp_swz(lane);
      const bf16x8 xr_h = P0[sl], xr_l = P1[sl];
      const bf16x8 xi_h = P2[sl], xi_l = P3[sl];
      acc[0][b] = T::mfma(ar_h, xr_h, acc[0][b]);
      acc[1][b] = T::mfma(ai_h, xi_h, acc[1][b]);
      acc[2][b] = T::mfma(ar_h, xi_h, acc[2][b]);
      acc[3][b] = T::mfma(ai_h, xr_h, acc[3][b]);
      acc[0][b] = T::mfma(ar_h, xr_l, acc[0][b]);
      acc[1][b] = T::mfma(ai_h, xi_l, acc[1][b]);
      acc[2][b] = T::mfma(ar_h, xi_l, acc[2][b]);
      acc[3][b] = T::mfma(ai_h, xr_l, acc[3][b]);
      acc[0][b] = T::mfma(ar_l, xr_h, acc[0][b]);
      acc[1][b] = T::mfma(ai_l, xi_h, acc[1][b]);
      acc[2][b] = T::mfma(ar_l, xi_h, acc[2][b]);
      acc[3][b] = T::mfma(ai_l, xr_h, acc[3][b]);
    }
  };
  auto round = [&](InFlight& F, int ahead) {
    stage(F);
    const bool mult = F.qi < nchunks;
    const bf16x8 ar_h = F.pa[0], ar_l = F.pa[1], ai_h = F.pa[2], ai_l = F.pa[3];
    lds_barrier();
    fetch(F, ahead);
    if (mult) multiply(ar_h, ar_l, ai_h, ai_l);
    lds_barrier();
  };
  // DEPTH chunks in flight: three for the 32-column form with S terms (the
  // sweep steps: 48 registers a chunk still fit two workgroups per CU), two
  // otherwise
  constexpr int DEPTH = (NB == 2 && HAS_S) ? 3 : 2;
  if (nchunks > 0) {  // workgroup-uniform
    InFlight f[DEPTH] = {};
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) fetch(f[d], d);
    for (int i = 0; i < nchunks; i += DEPTH) {
#pragma unroll
      for (int d = 0; d < DEPTH; ++d)
        if (d == 0 || i + d < nchunks) round(f[d], i + d + DEPTH);
    }
  }

  if (!rt_ok) return;
  if (kslices > 1) {
    float2* __restrict__ pt = part + ((size_t)slice * njobs + job) * nrhs * n;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rt * 16 + 4 * (lane >> 4) + i;
        const int rhs = col0 + b * 16 + (lane & 15);
        if (row < n && rhs < nrhs)
          pt[(size_t)rhs * n + row] = make_float2(acc[0][b][i] - acc[1][b][i], acc[2][b][i] + acc[3][b][i]);
      }
    return;
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

// Y = P + alpha sum_s part[s] over the k-slices of every job, slices summed in order
// (blk0 of the table counts jobs: blockIdx.y is a job of the launch)
template <int NS>
__global__ void split_reduce_kernel(const SegTableT<NS> tab, int kslices, const Job* __restrict__ jobs1) {
  int job = blockIdx.y;
  const int seg = seg_of(tab, job);
  const Job* __restrict__ jobs = NS == 1 ? jobs1 : tab.jobs[seg];
  const int n = tab.n[seg], nrhs = tab.nrhs[seg], njobs = tab.njobs[seg];
  const int64_t ld = tab.ld[seg];
  const Bases bases = tab.bases[seg];
  const float2* __restrict__ part = tab.part[seg];
  const Job& J = jobs[job];
  double2* __restrict__ Yb = sp_base(bases, J.Y.buf) + J.Y.off;
  const double2* __restrict__ Pb = J.P.buf >= 0 ? sp_base(bases, J.P.buf) + J.P.off : nullptr;
  const size_t per = (size_t)nrhs * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < per; e += (size_t)gridDim.x * blockDim.x) {
    const int rhs = (int)(e / n), row = (int)(e % n);
    double yr = 0.0, yi = 0.0;
    for (int sl = 0; sl < kslices; ++sl) {
      const float2 v = part[((size_t)sl * njobs + job) * per + e];
      yr += (double)v.x;
      yi += (double)v.y;
    }
    double2 y = make_double2(J.alpha.x * yr - J.alpha.y * yi, J.alpha.x * yi + J.alpha.y * yr);
    if (Pb) {
      const double2 p = Pb[(int64_t)rhs * ld + row];
      y.x += p.x;
      y.y += p.y;
    }
    Yb[(int64_t)rhs * ld + row] = y;
  }
}

template <int NS>
SegTableT<NS> seg_table(const ApplySeg* segs, int nseg) {
  SegTableT<NS> t;
  std::memset(&t, 0, sizeof(t));
  t.nseg = nseg;
  for (int i = 0; i < nseg; ++i) {
    t.n[i] = segs[i].n;
    t.nrhs[i] = segs[i].nrhs;
    t.njobs[i] = segs[i].njobs;
    t.ld[i] = segs[i].ld;
    t.jobs[i] = segs[i].jobs;
    t.bases[i] = segs[i].bases;
    t.part[i] = segs[i].part;
  }
  return t;
}

// Per-segment tiles and block offsets of the 64-row forms (wide, stream); the
// launch's block count, or -1 if it does not fit the grid
template <int NB, int NS>
long wide_blocks(SegTableT<NS>& t, int kslices) {
  long blk = 0;
  for (int i = 0; i < t.nseg; ++i) {
    t.a0[i] = (t.n[i] + kWideRows - 1) / kWideRows;
    t.a1[i] = (t.nrhs[i] + 16 * NB - 1) / (16 * NB);
    t.blk0[i] = (int32_t)blk;
    blk += (long)t.njobs[i] * t.a0[i] * t.a1[i] * kslices;
  }
  t.blk0[t.nseg] = (int32_t)blk;
  return blk > INT32_MAX ? -1 : blk;
}

// The k-slice sum: one row of blocks per job of the launch (blk0 counts jobs)
template <int NS>
hipError_t launch_reduce(SegTableT<NS> t, int kslices, hipStream_t st, hipEvent_t ev1) {
  int jobs = 0;
  size_t per = 0;
  for (int i = 0; i < t.nseg; ++i) {
    t.blk0[i] = jobs;
    jobs += t.njobs[i];
    per = std::max(per, (size_t)t.nrhs[i] * t.n[i]);
  }
  t.blk0[t.nseg] = jobs;
  const dim3 rgrid((unsigned)std::min<size_t>((per + 255) / 256, 256), (unsigned)jobs);
  hipExtLaunchKernelGGL(split_reduce_kernel<NS>, rgrid, dim3(256), 0, st, nullptr, ev1, 0, t, kslices,
                        t.jobs[0]);
  return hipGetLastError();
}

template <typename T, int NB, int KS, int NS>
hipError_t launch_wide(SegTableT<NS> t, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, int kslices = 1) {
  const long blk = wide_blocks<NB, NS>(t, kslices);
  if (blk < 0) return hipErrorInvalidValue;
  if (blk == 0) return hipSuccess;
  const dim3 grid((unsigned)blk);
  if (kslices > 1) {
    // the stop event goes on the reduction, so a timed launch covers both kernels
    hipExtLaunchKernelGGL((block_split_wide_kernel<T, NB, KS, NS>), grid, dim3(256 * KS), 0, st, ev0, nullptr, 0, t,
                          kslices, t.jobs[0]);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(t, kslices, st, ev1);
  }
  hipExtLaunchKernelGGL((block_split_wide_kernel<T, NB, KS, NS>), grid, dim3(256 * KS), 0, st, ev0, ev1, 0, t, 1,
                        t.jobs[0]);
  return hipGetLastError();
}

template <typename T, int NB, bool HAS_S, int NS>
hipError_t launch_stream(SegTableT<NS> t, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, int kslices) {
  const long blk = wide_blocks<NB, NS>(t, kslices);
  if (blk < 0) return hipErrorInvalidValue;
  if (blk == 0) return hipSuccess;
  const dim3 grid((unsigned)blk);
  if (kslices > 1) {
    hipExtLaunchKernelGGL((block_split_stream_kernel<T, NB, HAS_S, NS>), grid, dim3(256), 0, st, ev0, nullptr, 0, t,
                          kslices, t.jobs[0]);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(t, kslices, st, ev1);
  }
  hipExtLaunchKernelGGL((block_split_stream_kernel<T, NB, HAS_S, NS>), grid, dim3(256), 0, st, ev0, ev1, 0, t, 1,
                        t.jobs[0]);
  return hipGetLastError();
}

template <typename T, int NB, int KS, int NS>
hipError_t launch_sp(SegTableT<NS> t, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  long blk = 0;
  for (int i = 0; i < t.nseg; ++i) {
    t.a0[i] = (t.n[i] + 15) / 16;
    t.a1[i] = (t.nrhs[i] + 16 * NB - 1) / (16 * NB);
    t.blk0[i] = (int32_t)blk;
    blk += (long)t.njobs[i] * t.a0[i] * t.a1[i];
  }
  t.blk0[t.nseg] = (int32_t)blk;
  if (blk > INT32_MAX) return hipErrorInvalidValue;
  if (blk == 0) return hipSuccess;
  hipExtLaunchKernelGGL((block_split_kernel<T, NB, KS, NS>), dim3((unsigned)blk), dim3(64 * KS), 0, st, ev0, ev1, 0,
                        t, t.jobs[0]);
  return hipGetLastError();
}

template <typename T, int NB, int NS>
hipError_t launch_sp_ks(int ks, const SegTableT<NS>& t, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (ks >= 4) return launch_sp<T, NB, 4, NS>(t, st, ev0, ev1);
  if (ks == 2) return launch_sp<T, NB, 2, NS>(t, st, ev0, ev1);
  return launch_sp<T, NB, 1, NS>(t, st, ev0, ev1);
}

}  // namespace

size_t split_block_elems(int n) {
  const size_t nrt16 = (n + 15) / 16, nkt = (n + kSpK - 1) / kSpK;
  return nrt16 * nkt * 4 * 512;
}

hipError_t launch_split_planes(const double2* src, void* dst, int nblk, int n, hipStream_t st, int f16,
                               double scale) {
  if (nblk <= 0) return hipSuccess;
  const int nrt16 = (n + 15) / 16, nkt = (n + kSpK - 1) / kSpK;
  const int64_t lanes = (int64_t)nrt16 * nkt * 64;
  const unsigned gx = (unsigned)std::min<int64_t>((lanes + 255) / 256, 1024);
  if (f16)
    hipLaunchKernelGGL(split_planes_kernel<SpF16>, dim3(gx, nblk), dim3(256), 0, st, src, static_cast<_Float16*>(dst),
                       n, nrt16, nkt, scale);
  else
    hipLaunchKernelGGL(split_planes_kernel<SpBf16>, dim3(gx, nblk), dim3(256), 0, st, src, static_cast<__bf16*>(dst),
                       n, nrt16, nkt, 1.0);
  return hipGetLastError();
}

double split_input_scale(int f16) { return f16 ? SpF16::kX : SpBf16::kX; }


// right-hand sides per tile of the wide form (rule)
constexpr int kWideColsRule = 32;

int split_kslices(int njobs, int n, int nrhs, int tile_rhs) {
  if (nrhs <= 16) return 1;
  if (tile_rhs <= 0) tile_rhs = kWideColsRule;
  constexpr long kCUs = 256;
  const long tiles = (long)njobs * ((n + kWideRows - 1) / kWideRows) * ((nrhs + tile_rhs - 1) / tile_rhs);
  int ks = 1;
  while (ks < 16 && tiles * ks < 4 * kCUs) ks *= 2;
  return ks;
}

namespace {

template <typename T>
hipError_t apply_split(const Job* jobs, int njobs, int n, int nrhs, int64_t ld, Bases bases, hipStream_t st,
                       hipEvent_t ev0, hipEvent_t ev1, float2* part, SplitCfg cfg) {
  constexpr long kSimds = 1024;
  const ApplySeg sg{jobs, njobs, n, nrhs, ld, bases, part, 0};
  const SegTableT<1> t = seg_table<1>(&sg, 1);
  if (nrhs > 16) {
    // 64 x 32 (or 64 x 64) tiles; launches with fewer than four tiles per CU
    // split the chunk sequence over k-slices (partial tiles in `part`, summed
    // by a second kernel)
    const int tr = cfg.tile_rhs == 64 ? 64 : kWideColsRule;
    const int ks = cfg.kslices > 0 ? cfg.kslices : split_kslices(njobs, n, nrhs, tr);
    if (cfg.stream) {  // every job: two terms with Q (and S iff stream == 2)
      const int k = part ? ks : 1;
      if (cfg.stream == 2)
        return tr == 64 ? launch_stream<T, 4, true, 1>(t, st, ev0, ev1, k)
                        : launch_stream<T, 2, true, 1>(t, st, ev0, ev1, k);
      return tr == 64 ? launch_stream<T, 4, false, 1>(t, st, ev0, ev1, k)
                      : launch_stream<T, 2, false, 1>(t, st, ev0, ev1, k);
    }
    const int k = ks > 1 && part ? ks : 1;
    return tr == 64 ? launch_wide<T, 4, 1, 1>(t, st, ev0, ev1, k) : launch_wide<T, 2, 1, 1>(t, st, ev0, ev1, k);
  }
  // 16-column tiles; the chunks of a tile are split over up to 4 waves until
  // the launch has about 4 waves per SIMD
  const long tasks = (long)njobs * ((n + 15) / 16) * ((nrhs + 15) / 16);
  const int ks = cfg.kslices > 0 ? cfg.kslices : tasks >= 4 * kSimds ? 1 : tasks >= 2 * kSimds ? 2 : 4;
  return launch_sp_ks<T, 1, 1>(ks, t, st, ev0, ev1);
}

// The rule's shapes for a merged launch, from the segments' total size.
template <typename T>
hipError_t apply_split_segs(const ApplySeg* segs, int nseg, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  constexpr long kSimds = 1024, kCUs = 256;
  int rmax = 0;
  long tiles = 0, tasks = 0;
  for (int i = 0; i < nseg; ++i) {
    if (segs[i].njobs <= 0 || segs[i].n <= 0 || segs[i].nrhs <= 0) return hipErrorInvalidValue;
    rmax = std::max(rmax, segs[i].nrhs);
    tiles += (long)segs[i].njobs * ((segs[i].n + kWideRows - 1) / kWideRows) *
             ((segs[i].nrhs + kWideColsRule - 1) / kWideColsRule);
    tasks += (long)segs[i].njobs * ((segs[i].n + 15) / 16) * ((segs[i].nrhs + 15) / 16);
  }
  const SegTableT<kMaxSeg> t = seg_table<kMaxSeg>(segs, nseg);
  if (rmax > 16) {
    int ks = 1;
    while (ks < 16 && tiles * ks < 4 * kCUs) ks *= 2;
    for (int i = 0; i < nseg && ks > 1; ++i)  // every segment's workspace must hold its partial tiles
      if (!segs[i].part || (size_t)ks * segs[i].njobs * segs[i].nrhs * segs[i].n > segs[i].part_n) ks = 1;
    return launch_wide<T, 2, 1, kMaxSeg>(t, st, ev0, ev1, ks);
  }
  const int ks = tasks >= 4 * kSimds ? 1 : tasks >= 2 * kSimds ? 2 : 4;
  return launch_sp_ks<T, 1, kMaxSeg>(ks, t, st, ev0, ev1);
}

}  // namespace

hipError_t launch_block_apply_split(const Job* jobs, int njobs, int n, int nrhs, int64_t ld, Bases bases,
                                    hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, float2* part, SplitCfg cfg) {
  if (njobs <= 0) return hipSuccess;
  return cfg.f16 ? apply_split<SpF16>(jobs, njobs, n, nrhs, ld, bases, st, ev0, ev1, part, cfg)
                 : apply_split<SpBf16>(jobs, njobs, n, nrhs, ld, bases, st, ev0, ev1, part, cfg);
}

hipError_t launch_block_apply_split_segs(const ApplySeg* segs, int nseg, int f16, hipStream_t st, hipEvent_t ev0,
                                         hipEvent_t ev1) {
  if (nseg <= 0) return hipSuccess;
  if (nseg > kMaxSeg) return hipErrorInvalidValue;
  return f16 ? apply_split_segs<SpF16>(segs, nseg, st, ev0, ev1) : apply_split_segs<SpBf16>(segs, nseg, st, ev0, ev1);
}

}  // namespace polar
