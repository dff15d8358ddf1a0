// HIP kernels of libpolar (gfx950 / CDNA4, 64-wide wavefronts).
//
// The hot kernel is block_apply: a batched complex block matrix-vector
// (matrix-matrix for several right-hand sides) product with fused input
// combination and output epilogue,
//     Y = P + alpha * sum_t M_t (Q_t + beta_t S_t),
// which covers every dense operation of the online path: one step of a
// layer's forward/backward block sweep with the stored inverse Schur
// complements, one step of the down/up Gauss-Seidel sweeps through the
// transfer blocks, the reflection terms, and the polarized operator itself.
// The matrices are streamed from HBM once per launch (column-major blocks,
// coalesced along rows), the input slice is staged in LDS, and every
// reduction happens inside one workgroup in a fixed order.
#include "polar_kernels.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <type_traits>

namespace polar {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm for a / b
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    double r = b.x / b.y, d = b.y + b.x * r;
    return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}

template <typename T>
struct Cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ void cfma(Cx<T>& acc, Cx<T> m, Cx<T> v) {
  acc.x = fma(m.x, v.x, acc.x);
  acc.x = fma(-m.y, v.y, acc.x);
  acc.y = fma(m.x, v.y, acc.y);
  acc.y = fma(m.y, v.x, acc.y);
}

template <bool F32>
struct MatT;
template <>
struct MatT<false> {
  using vec = double2;
  using real = double;
};
template <>
struct MatT<true> {
  using vec = float2;
  using real = float;
};

// ----------------------------------------------------------------------------
// block_apply, few right-hand sides (NR <= 4): the HBM-streaming form
// ----------------------------------------------------------------------------
// Blocks are stored row-major, so every output row is a contiguous stream.
// One workgroup = kGvWaves waves = kGvWaves output rows (one per wave); lane l
// of a wave reads columns l, l+64, ... of its row, one contiguous 1 KiB
// segment per load instruction for float64.  The job's (term, column chunk)
// steps are walked in a workgroup-uniform loop, software-pipelined: the matrix
// loads and the input loads of step q+1 are in flight while step q is
// multiplied, and the inputs go through a double-buffered LDS slice.  The
// whole job record is fetched with loads issued back to back before any of
// it is used, so a launch pays one scalar round trip, not one per field.  The
// row's partial sums are reduced by a fixed butterfly of cross-lane shuffles:
// no atomics or fences, deterministic results.
constexpr int kGvWaves = 8;                 // rows per workgroup
constexpr int kGvThreads = kGvWaves * 64;

// global-memory views of float64 data: loads through them compile to global_load
// (not flat_load) and may be scheduled across LDS stores
typedef double d2v __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const d2v gd2;
__device__ __forceinline__ const gd2* to_gd2(const double2* p) {
  return reinterpret_cast<const gd2*>(reinterpret_cast<uintptr_t>(p));
}

// Workgroup ids are dealt round-robin to the 8 XCDs, each with its own L2.
// Renumber so that every XCD gets one contiguous range of logical ids: tiles
// next to each other in logical order (the right-hand-side tiles of one block
// row range) then meet in the same L2 and the block is fetched from HBM once.
__device__ __forceinline__ int xcd_logical(int i, int G) {
  constexpr int kXcd = 8;
  const int x = i % kXcd, local = i / kXcd;
  const int per = G / kXcd, rem = G % kXcd;
  return x < rem ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

// base pointer of a VecRef without dynamic indexing of the by-value kernel argument
__device__ __forceinline__ double2* base_of(const Bases& b, int buf) {
  return buf == 0 ? b.b[0] : buf == 1 ? b.b[1] : buf == 2 ? b.b[2] : buf == 3 ? b.b[3] : nullptr;
}

// columns per step of the streaming form: one load per lane and in-flight slot
template <int NR>
constexpr int gemv_u() { return NR >= 4 ? 4 : 8; }

// PIPE: the launch has jobs of more than one step (several terms or column
// chunks); without it every job is one step and one register set suffices.
template <int NR, bool F32, bool PIPE, int NS>
__global__ __launch_bounds__(kGvThreads) void block_gemv_kernel(const SegTableT<NS> tab,
                                                                const Job* __restrict__ jobs1) {
  // segment of this block: a0 = row tiles per job, a1 = columns per chunk
  int bx = blockIdx.x;
  const int seg = seg_of(tab, bx);
  const Job* __restrict__ jobs = NS == 1 ? jobs1 : tab.jobs[seg];
  const int n = tab.n[seg], ntiles = tab.a0[seg], kc = tab.a1[seg], nrhs = tab.nrhs[seg];
  const int64_t ld = tab.ld[seg];
  const Bases bases = tab.bases[seg];
  if constexpr (NS > 1)
    if ((int)blockIdx.y * NR >= nrhs) return;  // right-hand-side tiles beyond this segment's
  using MV = typename MatT<F32>::vec;
  using T = typename MatT<F32>::real;
  constexpr int U = gemv_u<NR>();  // kc <= 64 U: every lane has at most U columns of a step
  extern __shared__ unsigned char smem_raw[];
  Cx<T>* xs = reinterpret_cast<Cx<T>*>(smem_raw);  // 2 buffers of kc * NR

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int tile = bx % ntiles;
  // every field of the job, read into scalars up front (independent loads, one round trip)
  const Job* __restrict__ Jp = jobs + bx / ntiles;
  const int nterms = Jp->nterms;
  const void* const M0 = Jp->M[0];
  const void* const M1 = Jp->M[1];
  const void* const M2 = Jp->M[2];
  const void* const M3 = Jp->M[3];
  const VecRef Q0 = Jp->Q[0], Q1 = Jp->Q[1], Q2 = Jp->Q[2], Q3 = Jp->Q[3];
  const VecRef S0 = Jp->S[0], S1 = Jp->S[1], S2 = Jp->S[2], S3 = Jp->S[3];
  const double2 B0 = Jp->beta[0], B1 = Jp->beta[1], B2 = Jp->beta[2], B3 = Jp->beta[3];
  const VecRef Pr = Jp->P, Yr = Jp->Y;
  const double2 alpha = Jp->alpha;
  const int K0 = Jp->kw[0] > 0 ? Jp->kw[0] : n, K1 = Jp->kw[1] > 0 ? Jp->kw[1] : n;
  const int K2 = Jp->kw[2] > 0 ? Jp->kw[2] : n, K3 = Jp->kw[3] > 0 ? Jp->kw[3] : n;
  const int L0 = Jp->ldm[0] > 0 ? Jp->ldm[0] : K0, L1 = Jp->ldm[1] > 0 ? Jp->ldm[1] : K1;
  const int L2 = Jp->ldm[2] > 0 ? Jp->ldm[2] : K2, L3 = Jp->ldm[3] > 0 ? Jp->ldm[3] : K3;
  const int r0 = blockIdx.y * NR;
  const int row = tile * kGvWaves + wave;
  const int rowc = row < n ? row : n - 1;
  // steps (term, column chunk of kc): chunks per term, cumulative
  const int C0 = nterms > 0 ? (K0 + kc - 1) / kc : 0, C1 = nterms > 1 ? (K1 + kc - 1) / kc : 0;
  const int C2 = nterms > 2 ? (K2 + kc - 1) / kc : 0, C3 = nterms > 3 ? (K3 + kc - 1) / kc : 0;
  const int nq = C0 + C1 + C2 + C3;

  // fields of term t (workgroup-uniform selects)
  auto sel_k = [&](int t) { return t == 0 ? K0 : t == 1 ? K1 : t == 2 ? K2 : K3; };
  auto sel_l = [&](int t) { return t == 0 ? L0 : t == 1 ? L1 : t == 2 ? L2 : L3; };
  auto sel_m = [&](int t) { return t == 0 ? M0 : t == 1 ? M1 : t == 2 ? M2 : M3; };
  auto sel_q = [&](int t) { return t == 0 ? Q0 : t == 1 ? Q1 : t == 2 ? Q2 : Q3; };
  auto sel_s = [&](int t) { return t == 0 ? S0 : t == 1 ? S1 : t == 2 ? S2 : S3; };
  auto sel_b = [&](int t) { return t == 0 ? B0 : t == 1 ? B1 : t == 2 ? B2 : B3; };

  Cx<T> acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = Cx<T>{(T)0, (T)0};

  // raw loads of one step: U matrix entries of this lane's row, one input column per thread
  struct Step {
    MV m[U];
    d2v vq[NR], vs[NR];
    double2 be;
    int kw;
    bool has_q, has_s;
  };
  auto fetch = [&](Step& F, int q) {
    int t = 0;
    if (q >= C0) {
      q -= C0;
      t = 1;
      if (q >= C1) {
        q -= C1;
        t = 2;
        if (q >= C2) {
          q -= C2;
          t = 3;
        }
      }
    }
    const int c0 = q * kc;
    F.kw = min(kc, sel_k(t) - c0);
    const MV* __restrict__ Mrow = reinterpret_cast<const MV*>(sel_m(t)) + (size_t)rowc * sel_l(t) + c0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = lane + 64 * u;
      F.m[u] = c < F.kw ? Mrow[c] : MV{};
    }
    const VecRef qr = sel_q(t), sr = sel_s(t);
    F.has_q = qr.buf >= 0;
    F.has_s = sr.buf >= 0;
    F.be = sel_b(t);
    const int cj = c0 + min(tid, F.kw - 1);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int64_t e = (int64_t)min(r0 + r, nrhs - 1) * ld + cj;
      F.vq[r] = F.has_q ? to_gd2(base_of(bases, qr.buf) + qr.off)[e] : d2v{0.0, 0.0};
      F.vs[r] = F.has_s ? to_gd2(base_of(bases, sr.buf) + sr.off)[e] : d2v{0.0, 0.0};
    }
  };
  // input column tid of a step: X = Q + beta S into LDS buffer b
  auto stage = [&](const Step& F, int b) {
    if (tid < F.kw) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        double2 v = make_double2(F.vq[r].x, F.vq[r].y);
        if (F.has_s) v = cadd(v, cmul(F.be, make_double2(F.vs[r].x, F.vs[r].y)));
        if (r0 + r >= nrhs) v = make_double2(0.0, 0.0);
        xs[((size_t)b * kc + tid) * NR + r] = Cx<T>{(T)v.x, (T)v.y};
      }
    }
  };
  auto multiply = [&](const Step& F, int b) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = lane + 64 * u;
      if (c < F.kw) {
        const Cx<T> mm{(T)F.m[u].x, (T)F.m[u].y};
        const Cx<T>* xp = xs + ((size_t)b * kc + c) * NR;
#pragma unroll
        for (int r = 0; r < NR; ++r) cfma(acc[r], mm, xp[r]);
      }
    }
  };

  if constexpr (!PIPE) {
    if (nq > 0) {
      Step f0;
      fetch(f0, 0);
      stage(f0, 0);
      __syncthreads();
      multiply(f0, 0);
    }
  } else {
  Step f0, f1;
  if (nq > 0) {
    fetch(f0, 0);
    stage(f0, 0);
  }
  __syncthreads();
#pragma unroll 1
  for (int q = 0; q < nq; q += 2) {
    // step q from f0 / buffer 0 while step q+1 is fetched into f1
    if (q + 1 < nq) fetch(f1, q + 1);
    multiply(f0, 0);
    if (q + 1 < nq) stage(f1, 1);
    __syncthreads();
    if (q + 1 >= nq) break;
    // step q+1 from f1 / buffer 1 while step q+2 is fetched into f0
    if (q + 2 < nq) fetch(f0, q + 2);
    multiply(f1, 1);
    if (q + 2 < nq) stage(f0, 0);
    __syncthreads();
  }
  }

  // reduce the row over the 64 lanes (fixed butterfly), lanes 0..NR-1 write
#pragma unroll
  for (int r = 0; r < NR; ++r) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      acc[r].x += __shfl_xor(acc[r].x, off, 64);
      acc[r].y += __shfl_xor(acc[r].y, off, 64);
    }
  }
  if (lane < NR && row < n && r0 + lane < nrhs) {
    Cx<T> a = acc[0];
#pragma unroll
    for (int r = 1; r < NR; ++r)
      if (lane == r) a = acc[r];
    const int r = lane;
    double2 y = cmul(alpha, make_double2((double)a.x, (double)a.y));
    if (Pr.buf >= 0) y = cadd(y, base_of(bases, Pr.buf)[Pr.off + (int64_t)(r0 + r) * ld + row]);
    base_of(bases, Yr.buf)[Yr.off + (int64_t)(r0 + r) * ld + row] = y;
  }
}

// ----------------------------------------------------------------------------
// block_apply, many right-hand sides, float64 or float32 blocks: MFMA form
// ----------------------------------------------------------------------------
// One workgroup = KS groups of 4 waves = a 64-row x TN-right-hand-side output
// tile of one job (TN = 16, 32 or 64), or with kslices > 1 the partial tile of
// one contiguous share of the job's chunk sequence (mfma_reduce_kernel sums
// the shares).  The job's columns are walked in chunks
// of 16 (term by term); k-group g takes chunks g, g + KS, ..., so a launch with
// few tiles (a local-solve step with few right-hand sides, a sweep step) still
// has KS times the waves in flight.  Each group stages the 64 x 16 slice of the
// (row-major) block and the 16 x TN slice of the combined input Q + beta S in
// its own LDS buffers; all loads of the next chunk are issued before the
// current chunk's MFMAs, and the combination and tail masking wait until
// staging.  Wave w of a group accumulates rows 16w..16w+15 for all TN
// right-hand sides as TN/16 tiles of v_mfma_f64_16x16x4 (lane l holds
// A[l%16][l/16] and B[l/16][l%16]; accumulator register i of lane l holds
// C[4i + l/16][l%16]).  A complex product is four real MFMAs, Cr += Ar Br -
// Ai Bi, Ci += Ar Bi + Ai Br, issued so that consecutive MFMAs update different
// accumulators.  Groups 1..KS-1 hand their partial tiles to group 0 through
// LDS, summed in a fixed order: deterministic, no atomics.
//
// The staging stores write one row (A) or right-hand side (B) from several
// lanes at k rows 1 KiB apart, which would all land in the same LDS banks; the
// row / column index within a staged k row is therefore XORed with a function
// of k (stg_swz_a / stg_swz_b) that spreads every 8 consecutive lanes of a
// store over the 8 16-byte bank groups.  The XOR only permutes indices within
// aligned groups of 16, so the fragment reads (16 consecutive rows or columns
// of one k row) stay conflict-free.
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int kMmRows = 64;  // rows per workgroup tile
constexpr int kMmK = 16;     // columns per staged chunk
static_assert(kMmK == kNzChunk, "nonzero-chunk lists count MFMA staging chunks");

// A is staged by 4 lanes per row, each taking 4 consecutive k: lanes 4 i + j
// write row i at k = 4 j + u.
__device__ __forceinline__ int stg_swz_a(int k) { return 2 * ((k >> 2) & 3); }
// B is staged by 16 / BPT lanes per right-hand side, each taking BPT
// consecutive k (BPT = TN / 16).
template <int TN>
__device__ __forceinline__ int stg_swz_b(int k) {
  constexpr int BPT = kMmK * TN / 256;
  constexpr int G = kMmK / BPT;  // lanes per right-hand side
  return G >= 16 ? k : (k / BPT) * (8 / G);
}

// The same tiles for float32 blocks (the float32 form's preconditioner blocks)
// on v_mfma_f32_16x16x4f32: its operand layout is that of the float64
// instruction (one real per lane and operand), its four accumulator entries of
// lane l are rows 4 (l / 16) + 0..3 instead of 4 i + l / 16.
template <bool F32>
struct MmT;
template <>
struct MmT<false> {
  using acc = d4v;
  static __device__ __forceinline__ d4v mfma(double a, double b, d4v c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct MmT<true> {
  using acc = f4v;
  static __device__ __forceinline__ f4v mfma(float a, float b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

template <int TN, int KS, int NS, bool F32>
__global__ __launch_bounds__(256 * KS, 2) void block_mfma64_kernel(const SegTableT<NS> tab,
                                                                 const Job* __restrict__ jobs1, int kslices,
                                                                 double2* __restrict__ mpart) {
  using R = typename MatT<F32>::real;   // element type of the blocks and of the MFMA
  using R2 = typename MatT<F32>::vec;
  using Acc = typename MmT<F32>::acc;
  constexpr int NB = TN / 16;           // MFMA tiles per wave
  constexpr int BPT = kMmK * TN / 256;  // staged B entries per thread of a group
  __shared__ R2 As[KS][kMmK][kMmRows];  // k-major: fragment reads are 16 consecutive rows
  __shared__ R2 Bs[KS][kMmK][TN];
  __shared__ int32_t kls[kKlMax];
  const int tid = threadIdx.x & 255;    // thread within its k-group
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x >> 8);  // k-group (wave-uniform)
  int bid = xcd_logical(blockIdx.x, gridDim.x);
  // segment of this block (segments stay contiguous in the logical order): a0 =
  // right-hand-side tiles, a1 = row tiles per job
  const int seg = seg_of(tab, bid);
  const Job* __restrict__ jobs = NS == 1 ? jobs1 : tab.jobs[seg];
  const int n = tab.n[seg], nrt = tab.a0[seg], ntiles = tab.a1[seg], nrhs = tab.nrhs[seg];
  const int64_t ld = tab.ld[seg];
  const Bases bases = tab.bases[seg];
  const int ct = bid % nrt;  // right-hand-side tile (fastest: tiles sharing block rows stay on one XCD)
  bid /= nrt;
  const int tile = bid % ntiles;
  bid /= ntiles;
  const int slice = bid % kslices;  // k-slice of the tile (kslices > 1: its partial tile goes to mpart)
  const int job = bid / kslices;
  const Job& J = jobs[job];
  const int row0 = tile * kMmRows;
  const int col0 = ct * TN;

  // A staging: row tid/4, 4 consecutive columns (tid%4)*4
  const int sr = tid >> 2;
  const int sc = (tid & 3) * 4;
  const int arow = min(row0 + sr, n - 1);
  const bool arow_ok = row0 + sr < n;
  // B staging: BPT consecutive columns of one right-hand side
  const int bq = tid / (kMmK / BPT);
  const int bc = (tid % (kMmK / BPT)) * BPT;
  const int brhs = col0 + bq;
  const bool brhs_ok = brhs < nrhs;

  // float64: three real products per complex one (Gauss): p1 = Re A Re B,
  // p2 = Im A Im B, p3 = (Re A + Im A)(Re B + Im B); then Re = p1 - p2,
  // Im = p3 - p1 - p2.  A quarter fewer MFMAs than the four-product form; the
  // error stays within a small multiple of the unit roundoff times |A||B|
  // (normwise).  float32: the four products (p3 = Re A Im B, p4 = Im A Re B,
  // Im = p3 + p4), since in single precision the cancellation in p3 - p1 - p2
  // costs the imaginary part digits whenever it is much smaller than the real.
  Acc p1[NB], p2[NB], p3[NB], p4[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    p1[b] = Acc{};
    p2[b] = Acc{};
    p3[b] = Acc{};
    p4[b] = Acc{};
  }
  const int wr = wave * 16;
  auto r2 = [](R x, R y) -> R2 {
    if constexpr (F32)
      return make_float2(x, y);
    else
      return make_double2(x, y);
  };

  // columns and row stride of each term (wide terms: kw > 0), chunks of kMmK per term
  // chunks of term 0 with nonzero inputs (null: all), copied to LDS once so
  // that looking one up waits on LDS only, not on the chunk loads in flight
  typedef __attribute__((address_space(1))) const int32_t gi32;
  const bool kl = J.kl != nullptr;
  int kl_cnt = 0;
  if (kl) {
    gi32* __restrict__ src = reinterpret_cast<gi32*>(reinterpret_cast<uintptr_t>(J.kl));
    kl_cnt = min((int)src[0], kKlMax);
    for (int i = threadIdx.x; i < kl_cnt; i += 256 * KS) kls[i] = src[1 + i];
    __syncthreads();
  }
  int kt[4], lt[4], nct[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    kt[t] = J.kw[t] > 0 ? J.kw[t] : n;
    lt[t] = J.ldm[t] > 0 ? J.ldm[t] : kt[t];
    nct[t] = t < J.nterms ? (t == 0 && kl ? kl_cnt : (kt[t] + kMmK - 1) / kMmK) : 0;
  }
  // this slice's chunks of the job's (term, chunk) sequence: qbeg .. qbeg + nchunks - 1
  const int nall = nct[0] + nct[1] + nct[2] + nct[3];
  const int cps = (nall + kslices - 1) / kslices;
  const int qbeg = min(slice * cps, nall);
  const int nchunks = min(nall, qbeg + cps) - qbeg;
  const int rounds = (nchunks + KS - 1) / KS;  // the same for every group: barriers stay uniform
  // Raw loads of a chunk, all unconditional (indices clamped into the block and
  // vectors): masking and the combination Q + beta S wait until the chunk is
  // staged, so all its loads are in flight together.
  struct Stage {
    R2 pa[4];
    double2 pq[BPT], ps[BPT];
    double2 be;
    int c0, kc;
    bool live, has_q, has_s;
  };
  auto fetch = [&](Stage& S, int q) {
    S.live = q < nchunks;
    if (!S.live) return;
    q += qbeg;
    // term t of chunk q and the chunk within it (array indices stay compile-time constants)
    int t = 0, K = kt[0], ldm = lt[0];
#pragma unroll
    for (int u = 0; u < 3; ++u)
      if (t == u && q >= nct[u]) {
        q -= nct[u];
        t = u + 1;
        K = kt[u + 1];
        ldm = lt[u + 1];
      }
    S.c0 = (kl && t == 0 ? kls[q] : q) * kMmK;
    S.kc = K;
    typedef R rv2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(1))) const rv2 grv2;
    const grv2* __restrict__ M =
        reinterpret_cast<const grv2*>(reinterpret_cast<uintptr_t>(J.M[t])) + (size_t)arow * ldm;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const rv2 a = M[min(S.c0 + sc + u, K - 1)];
      S.pa[u] = r2(a.x, a.y);
    }
    const VecRef qr = J.Q[t];
    const VecRef svr = J.S[t];
    S.has_q = qr.buf >= 0;
    S.has_s = svr.buf >= 0;
    S.be = J.beta[t];
    const int64_t cb = (int64_t)min(brhs, nrhs - 1) * ld;
    if (S.has_q) {
      const gd2* __restrict__ qp = to_gd2(base_of(bases, qr.buf) + qr.off + cb);
#pragma unroll
      for (int u = 0; u < BPT; ++u) {
        const d2v v = qp[min(S.c0 + bc + u, K - 1)];
        S.pq[u] = make_double2(v.x, v.y);
      }
    }
    if (S.has_s) {
      const gd2* __restrict__ sp = to_gd2(base_of(bases, svr.buf) + svr.off + cb);
#pragma unroll
      for (int u = 0; u < BPT; ++u) {
        const d2v v = sp[min(S.c0 + bc + u, K - 1)];
        S.ps[u] = make_double2(v.x, v.y);
      }
    }
  };
  auto stage = [&](const Stage& S) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      As[grp][sc + u][sr ^ stg_swz_a(sc + u)] =
          (S.live && arow_ok && S.c0 + sc + u < S.kc) ? S.pa[u] : r2((R)0, (R)0);
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
      double2 v = S.has_q ? S.pq[u] : make_double2(0.0, 0.0);
      if (S.has_s) v = cadd(v, cmul(S.be, S.ps[u]));
      Bs[grp][bc + u][bq ^ stg_swz_b<TN>(bc + u)] =
          (S.live && brhs_ok && S.c0 + bc + u < S.kc) ? r2((R)v.x, (R)v.y) : r2((R)0, (R)0);
    }
  };
  auto multiply = [&]() {
#pragma unroll
    for (int kk = 0; kk < kMmK; kk += 4) {
      const int kr = kk + (lane >> 4);
      const R2 av = As[grp][kr][wr + ((lane & 15) ^ stg_swz_a(kr))];
      const R as = av.x + av.y;
      R2 bv[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) bv[b] = Bs[grp][kr][b * 16 + ((lane & 15) ^ stg_swz_b<TN>(kr))];
#pragma unroll
      for (int b = 0; b < NB; ++b) p1[b] = MmT<F32>::mfma(av.x, bv[b].x, p1[b]);
#pragma unroll
      for (int b = 0; b < NB; ++b) p2[b] = MmT<F32>::mfma(av.y, bv[b].y, p2[b]);
      if constexpr (F32) {
#pragma unroll
        for (int b = 0; b < NB; ++b) p3[b] = MmT<F32>::mfma(av.x, bv[b].y, p3[b]);
#pragma unroll
        for (int b = 0; b < NB; ++b) p4[b] = MmT<F32>::mfma(av.y, bv[b].x, p4[b]);
      } else {
#pragma unroll
        for (int b = 0; b < NB; ++b) p3[b] = MmT<F32>::mfma(as, bv[b].x + bv[b].y, p3[b]);
      }
    }
  };
  Stage s0;
  fetch(s0, grp);
  for (int i = 0; i < rounds; ++i) {
    stage(s0);
    __syncthreads();
    fetch(s0, (i + 1) * KS + grp);  // next chunk in flight during the MFMAs
    multiply();
    __syncthreads();
  }
  Acc cr[NB], ci[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    cr[b] = p1[b] - p2[b];
    if constexpr (F32)
      ci[b] = p3[b] + p4[b];
    else
      ci[b] = p3[b] - p1[b] - p2[b];
  }

  if constexpr (KS > 1) {
    // partial tiles of groups 1..KS-1 through the (now idle) staging buffers
    static_assert((KS - 1) * 4 * 64 * NB * 8 * sizeof(R) <= sizeof(As) + sizeof(Bs) || KS == 1,
                  "reduction does not fit the staging buffers");
    R* red = reinterpret_cast<R*>(&As[0][0][0]);
    auto at = [&](int g, int b, int j) -> R& {
      return red[((((size_t)(g - 1) * 4 + wave) * NB + b) * 8 + j) * 64 + lane];
    };
    if (grp > 0)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          at(grp, b, j) = cr[b][j];
          at(grp, b, 4 + j) = ci[b][j];
        }
    __syncthreads();
    if (grp > 0) return;
#pragma unroll
    for (int g = 1; g < KS; ++g)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cr[b][j] += at(g, b, j);
          ci[b][j] += at(g, b, 4 + j);
        }
  }

  if (kslices > 1) {
    // this slice's partial tile, before alpha and P: mpart[((slice * njobs + job) * nrhs + rhs) * n + row];
    // mfma_reduce_kernel sums the slices in order and finishes the rows
    double2* __restrict__ pt = mpart + ((size_t)slice * tab.njobs[seg] + job) * nrhs * n;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = row0 + wr + (F32 ? 4 * (lane >> 4) + i : 4 * i + (lane >> 4));
        const int rhs = col0 + b * 16 + (lane & 15);
        if (row < n && rhs < nrhs) pt[(size_t)rhs * n + row] = make_double2((double)cr[b][i], (double)ci[b][i]);
      }
    return;
  }
  double2* __restrict__ Yb = base_of(bases, J.Y.buf) + J.Y.off;
  const double2* __restrict__ Pb = J.P.buf >= 0 ? base_of(bases, J.P.buf) + J.P.off : nullptr;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      // accumulator entry i of lane l: row 4 i + l / 16 (float64), 4 (l / 16) + i (float32)
      const int row = row0 + wr + (F32 ? 4 * (lane >> 4) + i : 4 * i + (lane >> 4));
      const int rhs = col0 + b * 16 + (lane & 15);
      if (row < n && rhs < nrhs) {
        double2 y = cmul(J.alpha, make_double2((double)cr[b][i], (double)ci[b][i]));
        if (Pb) y = cadd(y, Pb[(int64_t)rhs * ld + row]);
        Yb[(int64_t)rhs * ld + row] = y;
      }
    }
}

// Y = P + alpha * (the k-slice partial tiles of block_mfma64_kernel summed in
// slice order) for every job of a single-problem launch; grid: (<= 256, jobs)
__global__ void mfma_reduce_kernel(const Job* __restrict__ jobs, int n, int nrhs, int njobs, int64_t ld, Bases bases,
                                   int kslices, const double2* __restrict__ mpart) {
  const int job = blockIdx.y;
  const Job& J = jobs[job];
  double2* __restrict__ Yb = base_of(bases, J.Y.buf) + J.Y.off;
  const double2* __restrict__ Pb = J.P.buf >= 0 ? base_of(bases, J.P.buf) + J.P.off : nullptr;
  const size_t per = (size_t)nrhs * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < per; e += (size_t)gridDim.x * blockDim.x) {
    const int rhs = (int)(e / n), row = (int)(e % n);
    double2 s = mpart[(size_t)job * per + e];
    for (int sl = 1; sl < kslices; ++sl) s = cadd(s, mpart[((size_t)sl * njobs + job) * per + e]);
    double2 y = cmul(J.alpha, s);
    if (Pb) y = cadd(y, Pb[(int64_t)rhs * ld + row]);
    Yb[(int64_t)rhs * ld + row] = y;
  }
}

// G[x'][e] for e = (r - r0) NX + x: row x' of the trace-row block j of the
// inverse, from column q NX + x' of the extraction solve, rescaled (see
// launch_pack_green).  grid.x covers nrows NX entries, grid.y = x'.
__global__ __launch_bounds__(256) void pack_green_kernel(const double2* __restrict__ W, int64_t ld, int q, int j,
                                                         int r0, int nrows, int NX, const double2* __restrict__ ax,
                                                         const double2* __restrict__ az, double2* __restrict__ G) {
  const int xp = blockIdx.y;
  const int64_t cnt = (int64_t)nrows * NX;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= cnt) return;
  const int r = r0 + (int)(e / NX), x = (int)(e % NX);
  const double2 w = W[((int64_t)q * NX + xp) * ld + (int64_t)r * NX + x];
  const double2 sc = cdiv(cmul(ax[xp], az[j]), cmul(ax[x], az[r]));
  G[(int64_t)xp * cnt + e] = cmul(w, sc);
}

// W[c][dst[e]] = sum over s < cnt[e] of W[c][src0[e] + s] (rows of NX entries,
// column stride ld), the partial rows summed in order.  grid: (NX / 256, entries, columns).
__global__ __launch_bounds__(256) void sum_rows_kernel(double2* __restrict__ W, int64_t ld, int NX,
                                                       const int32_t* __restrict__ dst,
                                                       const int32_t* __restrict__ src0,
                                                       const int32_t* __restrict__ cnt) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= NX) return;
  const int e = blockIdx.y;
  double2* col = W + (int64_t)blockIdx.z * ld;
  const int s0 = src0[e], n = cnt[e];
  double2 acc = make_double2(0.0, 0.0);
  for (int k = 0; k < n; ++k) acc = cadd(acc, col[(int64_t)(s0 + k) * NX + x]);
  col[(int64_t)dst[e] * NX + x] = acc;
}

// One workgroup per input e: flags its chunks (one per thread and pass), then
// writes the flagged indices in ascending order through a ballot prefix.
__global__ __launch_bounds__(256) void nonzero_chunks_kernel(const double2* __restrict__ B, int64_t ld, int ncols,
                                                             const int64_t* __restrict__ off,
                                                             const int32_t* __restrict__ kk,
                                                             int32_t* __restrict__ list, int stride) {
  __shared__ int wcnt[4];
  const int e = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t o = off[e];
  const int K = kk[e];
  const int nch = (K + kNzChunk - 1) / kNzChunk;
  int32_t* __restrict__ out = list + (int64_t)e * stride;
  int base = 0;
  for (int c0 = 0; c0 < nch; c0 += 256) {
    const int c = c0 + tid;
    bool nz = false;
    if (c < nch) {
      const int lim = min(kNzChunk, K - c * kNzChunk);
      for (int col = 0; col < ncols && !nz; ++col) {
        const double2* __restrict__ p = B + (int64_t)col * ld + o + (int64_t)c * kNzChunk;
        for (int i = 0; i < lim; ++i) {
          const double2 v = p[i];
          nz = nz || !(v.x == 0.0 && v.y == 0.0);
        }
      }
    }
    const uint64_t m = __ballot(nz);
    if (lane == 0) wcnt[wave] = __popcll(m);
    __syncthreads();
    int pos = base + __popcll(m & ((1ull << lane) - 1ull));
    for (int w = 0; w < wave; ++w) pos += wcnt[w];
    if (nz) out[1 + pos] = c;
    base += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
  if (tid == 0) out[0] = base;
}

// Kernel form and shape of one (possibly merged) block-apply launch.
struct ApplyForm {
  int kind;  // 0: row-streaming (<= 4 right-hand sides), 1: MFMA tiles
  int nr;    // right-hand sides per pass (streaming)
  int tn;    // MFMA tile width
  int ks;    // MFMA wave groups (0: rule)
  bool pipe; // streaming: jobs of more than one step
  int mks = 1;                // MFMA k-slices over workgroups (single-problem launches)
  double2* mpart = nullptr;   // their partial tiles
};

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

// Fills the per-segment tile counts and block offsets of `t` for form f and
// launches it; ev0/ev1: optional events stamped by the dispatch itself.
template <int NR, bool F32, int NS>
hipError_t launch_apply_form(SegTableT<NS> t, const ApplyForm& f, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  using T = typename MatT<F32>::real;
  long blk = 0;
  int ymax = 1, kcmax = 1;
  for (int i = 0; i < t.nseg; ++i) {
    const int n = t.n[i];
    t.blk0[i] = (int32_t)blk;
    if (f.kind == 0) {
      t.a0[i] = (n + kGvWaves - 1) / kGvWaves;
      t.a1[i] = std::min(n, NR >= 4 ? 256 : 512);  // <= 64 columns per in-flight load slot
      blk += (long)t.njobs[i] * t.a0[i];
      ymax = std::max(ymax, (t.nrhs[i] + NR - 1) / NR);
    } else {
      t.a0[i] = (t.nrhs[i] + f.tn - 1) / f.tn;
      t.a1[i] = (n + kMmRows - 1) / kMmRows;
      blk += (long)t.njobs[i] * t.a1[i] * t.a0[i];
    }
    kcmax = std::max(kcmax, t.a1[i]);
  }
  t.blk0[t.nseg] = (int32_t)blk;
  if (blk <= 0) return hipSuccess;
  if (blk > INT32_MAX) return hipErrorInvalidValue;
  if (f.kind == 0) {
    const size_t lds = 2 * (size_t)kcmax * NR * sizeof(Cx<T>);
    const dim3 grid((unsigned)blk, (unsigned)ymax);
    if (!f.pipe)  // every job one step: one LDS buffer
      hipExtLaunchKernelGGL((block_gemv_kernel<NR, F32, false, NS>), grid, dim3(kGvThreads), (uint32_t)lds / 2, st, ev0,
                            ev1, 0, t, t.jobs[0]);
    else
      hipExtLaunchKernelGGL((block_gemv_kernel<NR, F32, true, NS>), grid, dim3(kGvThreads), (uint32_t)lds, st, ev0, ev1,
                            0, t, t.jobs[0]);
  } else {
    if (f.tn != 16 && f.tn != 32 && f.tn != 64) return hipErrorInvalidValue;  // the kernel's tile widths
    // k-split over 4 groups when the launch has fewer tiles than CUs, 2 below two per CU
    const int ks = f.ks > 0 ? f.ks : blk < 256 ? 4 : blk < 512 ? 2 : 1;
    // k-slices over workgroups (partial tiles summed by a second kernel): single-problem launches only
    const int mks = NS == 1 && f.mks > 1 && f.mpart ? f.mks : 1;
    if (blk * mks > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid2((unsigned)(blk * mks));
    hipEvent_t ev_end = mks > 1 ? nullptr : ev1;  // with k-slices the stop event goes on the sum
#define POLAR_MFMA64(TNV, KSV)                                                                               \
  hipExtLaunchKernelGGL((block_mfma64_kernel<TNV, KSV, NS, F32>), grid2, dim3(256 * KSV), 0, st, ev0, ev_end, 0, \
                        t, t.jobs[0], mks, f.mpart)
    // (32- and 64-column tiles take one wave group: the rules choose them for launches of >= 512
    // tiles, the tuner pairs them with k-slices over workgroups where the launch is smaller)
    if (f.tn == 64) {
      POLAR_MFMA64(64, 1);
    } else if (f.tn == 32) {
      POLAR_MFMA64(32, 1);
    } else {
      if (ks == 4) POLAR_MFMA64(16, 4); else if (ks == 2) POLAR_MFMA64(16, 2); else POLAR_MFMA64(16, 1);
    }
#undef POLAR_MFMA64
    if (mks > 1) {
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      const size_t per = (size_t)t.nrhs[0] * t.n[0];
      const dim3 rgrid((unsigned)std::min<size_t>((per + 255) / 256, 256), (unsigned)t.njobs[0]);
      hipExtLaunchKernelGGL(mfma_reduce_kernel, rgrid, dim3(256), 0, st, nullptr, ev1, 0, t.jobs[0], t.n[0], t.nrhs[0],
                            t.njobs[0], t.ld[0], t.bases[0], mks, f.mpart);
    }
  }
  return hipGetLastError();
}

template <bool F32, int NS>
hipError_t launch_apply_t(const SegTableT<NS>& t, const ApplyForm& f, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  switch (f.nr) {
    case 1: return launch_apply_form<1, F32, NS>(t, f, st, ev0, ev1);
    case 2: return launch_apply_form<2, F32, NS>(t, f, st, ev0, ev1);
    case 4: return launch_apply_form<4, F32, NS>(t, f, st, ev0, ev1);
    case 8: return launch_apply_form<8, F32, NS>(t, f, st, ev0, ev1);
    case 16: return launch_apply_form<16, F32, NS>(t, f, st, ev0, ev1);
    default: return hipErrorInvalidValue;
  }
}

// ----------------------------------------------------------------------------
// setup: Gauss-Jordan inversion with partial pivoting
// ----------------------------------------------------------------------------
// At step k the pivot is the largest |a_ik|^2 over rows i >= k (smallest index
// on ties), rows k and p are swapped, row k is divided by the pivot and
// eliminated from every other row, and column k takes the inverse's entries
// (in place: a zero or NaN column keeps its row order and raises the flag).
// Blocked: one panel of kGjBw columns at a time.  gj_panel_kernel runs
// the steps k0 .. k0+bw-1 on the panel columns alone, in place (one workgroup
// per matrix; the panel stays in L2): pivot search over rows >= k, the row
// swap within the panel, the elimination.  gj_update_kernel then brings every
// other column through the same steps at once: with the panel's row swaps
// applied to it (row source map), column j becomes
//   new[i][j] = [i outside the pivot rows] old[src(i)][j] + sum_t P[i][t] old[src(k0+t)][j],
// P the transformed panel, written out of place.  Columns are column-major.
constexpr int kGjBw = 16;   // panel width
constexpr int kGjCols = 16; // columns per workgroup of the update

__global__ __launch_bounds__(1024) void gj_panel_kernel(double2* const* __restrict__ A, int n, int k0, int bw,
                                                        int32_t* __restrict__ perm, int32_t* __restrict__ flag) {
  const int b = blockIdx.x;
  double2* __restrict__ a = A[b] + (size_t)k0 * n;  // panel column c at a + c n
  const int tid = threadIdx.x;
  __shared__ double sv[1024];
  __shared__ int si[1024];
  __shared__ double2 fi[4096];
  __shared__ double2 wj[kGjBw];
  for (int c = 0; c < bw; ++c) {
    const int k = k0 + c;
    // pivot: largest |a_ik|^2 over i >= k, smallest index on ties
    double bv = -1.0;
    int bi = n;
    for (int i = k + tid; i < n; i += 1024) {
      const double2 v = a[(size_t)c * n + i];
      const double m = v.x * v.x + v.y * v.y;
      if (m > bv) {
        bv = m;
        bi = i;
      }
    }
    sv[tid] = bv;
    si[tid] = bi;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
      if (tid < st) {
        const double v2 = sv[tid + st];
        const int i2 = si[tid + st];
        if (v2 > sv[tid] || (v2 == sv[tid] && i2 < si[tid])) {
          sv[tid] = v2;
          si[tid] = i2;
        }
      }
      __syncthreads();
    }
    const bool singular = !(sv[0] > 0.0) || si[0] >= n;
    const int p = singular ? k : si[0];
    if (tid == 0) {
      perm[(size_t)b * n + k] = p;
      if (singular) atomicOr(flag, 1);
    }
    // swap rows k and p of the panel
    if (tid < bw && p != k) {
      const double2 t = a[(size_t)tid * n + k];
      a[(size_t)tid * n + k] = a[(size_t)tid * n + p];
      a[(size_t)tid * n + p] = t;
    }
    __syncthreads();
    for (int i = tid; i < n; i += 1024) fi[i] = a[(size_t)c * n + i];
    if (tid < bw) wj[tid] = a[(size_t)tid * n + k];
    __syncthreads();
    const double2 piv = singular ? make_double2(1.0, 0.0) : fi[k];
    const double2 inv = cdiv(make_double2(1.0, 0.0), piv);
    for (int e = tid; e < n * bw; e += 1024) {
      const int t = e / n, i = e - t * n;
      double2 out;
      if (i == k) {
        out = (t == c) ? inv : cmul(wj[t], inv);
      } else if (t == c) {
        const double2 q = cmul(fi[i], inv);
        out = make_double2(-q.x, -q.y);
      } else {
        const double2 q = cmul(fi[i], cmul(wj[t], inv));
        const double2 v = a[(size_t)t * n + i];
        out = make_double2(v.x - q.x, v.y - q.y);
      }
      a[(size_t)t * n + i] = out;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void gj_update_kernel(double2* const* __restrict__ A, double2* const* __restrict__ B,
                                                        int n, int k0, int bw, const int32_t* __restrict__ perm) {
  const int b = blockIdx.y;
  const double2* __restrict__ a = A[b];
  double2* __restrict__ o = B[b];
  const int tid = threadIdx.x;
  __shared__ int src[4096];
  __shared__ double2 bv[kGjCols][kGjBw];
  for (int i = tid; i < n; i += 256) src[i] = i;
  __syncthreads();
  if (tid == 0)
    for (int c = 0; c < bw; ++c) {
      const int k = k0 + c, p = perm[(size_t)b * n + k];
      const int t = src[k];
      src[k] = src[p];
      src[p] = t;
    }
  __syncthreads();
  const int j0 = blockIdx.x * kGjCols;
  // every entry of bv is written: the product below runs over all kGjBw
  // panel columns, and LDS left over from an earlier workgroup may hold NaN
  // bit patterns that a zero factor would not cancel
  for (int e = tid; e < kGjCols * kGjBw; e += 256) {
    const int jj = e / kGjBw, t = e - jj * kGjBw, j = j0 + jj;
    bv[jj][t] = (j < n && t < bw) ? a[(size_t)j * n + src[k0 + t]] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int i = tid; i < n; i += 256) {
    double2 pn[kGjBw];
#pragma unroll
    for (int t = 0; t < kGjBw; ++t) pn[t] = t < bw ? a[(size_t)(k0 + t) * n + i] : make_double2(0.0, 0.0);
    const int si_ = src[i];
    const bool piv_row = i >= k0 && i < k0 + bw;
    for (int jj = 0; jj < kGjCols; ++jj) {
      const int j = j0 + jj;
      if (j >= n) break;
      if (j >= k0 && j < k0 + bw) {  // panel column: already final
        o[(size_t)j * n + i] = a[(size_t)j * n + i];
        continue;
      }
      double2 v = piv_row ? make_double2(0.0, 0.0) : a[(size_t)j * n + si_];
#pragma unroll
      for (int t = 0; t < kGjBw; ++t) v = cadd(v, cmul(pn[t], bv[jj][t]));
      o[(size_t)j * n + i] = v;
    }
  }
}

__global__ void gj_perm_kernel(const int32_t* __restrict__ perm, int32_t* __restrict__ pi, int nb, int n) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  int32_t* q = pi + (size_t)b * n;
  const int32_t* pm = perm + (size_t)b * n;
  for (int c = 0; c < n; ++c) q[c] = c;
  for (int k = n - 1; k >= 0; --k) {
    const int pk = pm[k];
    const int32_t t = q[k];
    q[k] = q[pk];
    q[pk] = t;
  }
}

__device__ __forceinline__ double2 tridiag_entry(int i, int c, const double2* diag, const double2* west,
                                                 const double2* east) {
  if (i == c) return diag[i];
  if (i == c + 1) return west[i];
  if (i + 1 == c) return east[i];
  return make_double2(0.0, 0.0);
}

// grid.x = ceil(n*n / 256), grid.y = matrix
__global__ void init_delta_kernel(double2* const* out, const double2* const* diag, const double2* west,
                                  const double2* east, int n) {
  const int b = blockIdx.y;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int c = (int)(e / n), i = (int)(e % n);
  out[b][e] = tridiag_entry(i, c, diag[b], west, east);
}

// G[b] += Y[b] - tridiag(A_m): the two halves of the middle Schur complement
// of a two-ended elimination, each of which already holds tridiag(A_m)
__global__ void twist_combine_kernel(double2* const* G, const double2* const* Y, const double2* const* diag,
                                     const double2* west, const double2* east, int n) {
  const int b = blockIdx.y;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int c = (int)(e / n), i = (int)(e % n);
  const double2 d = tridiag_entry(i, c, diag[b], west, east);
  const double2 g = G[b][e], y = Y[b][e];
  G[b][e] = make_double2(g.x + y.x - d.x, g.y + y.y - d.y);
}

__global__ void finish_row_kernel(double2* const* B, const int32_t* pi, double2* const* dinv64,
                                  double2* const* nextD, const double2* const* next_diag, const double2* coef,
                                  const double2* west, const double2* east, int n) {
  const int b = blockIdx.y;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int c = (int)(e / n), i = (int)(e % n);
  const double2 v = B[b][(size_t)pi[(size_t)b * n + c] * n + i];
  const size_t er = (size_t)i * n + c;  // stored factors are row-major
  if (dinv64[b]) dinv64[b][er] = v;
  if (next_diag[b]) {
    const double2 t = cmul(coef[b], v);
    const double2 d = tridiag_entry(i, c, next_diag[b], west, east);
    nextD[b][e] = make_double2(d.x - t.x, d.y - t.y);
  }
}

// ----------------------------------------------------------------------------
// field kernels
// ----------------------------------------------------------------------------
__global__ void scatter_source_kernel(const double2* __restrict__ f, double2* __restrict__ W,
                                      const int32_t* __restrict__ rowmap, int sumR, int NZ, int NX, int nrhs,
                                      double scale) {
  const size_t total = (size_t)nrhs * sumR * NX;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % NX);
    const size_t rg = e / NX;
    const int gr = (int)(rg % sumR);
    const int r = (int)(rg / sumR);
    const int src = rowmap[gr];
    double2 v = make_double2(0.0, 0.0);
    if (src >= 0) {
      const double2 fv = f[((size_t)r * NZ + src) * NX + i];
      v = make_double2(scale * fv.x, scale * fv.y);
    }
    W[e] = v;
  }
}

// amax[r * L + l] = max |f[r]|^2 over the owned rows of layer l (fixed-order tree, deterministic)
// 1024 threads per (layer, source): with one source a launch has only L workgroups
constexpr int kActThreads = 1024;
__global__ __launch_bounds__(kActThreads) void source_activity_kernel(const double2* __restrict__ f,
                                                                       double* __restrict__ amax,
                                                                       const int32_t* __restrict__ own_start,
                                                                       const int32_t* __restrict__ n_own, int L,
                                                                       int NZ, int NX) {
  __shared__ double red[kActThreads];
  const int l = blockIdx.x, r = blockIdx.y;
  const double2* fr = f + ((size_t)r * NZ + own_start[l]) * NX;
  const int64_t cnt = (int64_t)n_own[l] * NX;
  // a max that keeps NaN (fmax would drop it): a NaN source must reach every layer
  auto nmax = [](double a, double b) { return (b > a || b != b) ? b : a; };
  double mx = 0.0;
  for (int64_t e = threadIdx.x; e < cnt; e += kActThreads) {
    const double2 v = fr[e];
    mx = nmax(mx, v.x * v.x + v.y * v.y);
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = kActThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = nmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) amax[(size_t)r * L + l] = red[0];
}

// Layer-compacted sources: column slot j of layer l holds source slot_rhs[l * m + j] (-1: zero)
__global__ void scatter_slots_kernel(const double2* __restrict__ f, double2* __restrict__ W,
                                     const int32_t* __restrict__ rowmap, const int32_t* __restrict__ row_layer,
                                     const int32_t* __restrict__ slot_rhs, int m, int sumR, int NZ, int NX,
                                     double scale) {
  const size_t total = (size_t)m * sumR * NX;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % NX);
    const size_t rg = e / NX;
    const int gr = (int)(rg % sumR);
    const int j = (int)(rg / sumR);
    const int src = rowmap[gr];
    const int r = slot_rhs[row_layer[gr] * m + j];
    double2 v = make_double2(0.0, 0.0);
    if (src >= 0 && r >= 0) {
      const double2 fv = f[((size_t)r * NZ + src) * NX + i];
      v = make_double2(scale * fv.x, scale * fv.y);
    }
    W[e] = v;
  }
}

// s[r][seg] = W[slot of r in the row's layer][row] (zero where r does not touch that layer)
__global__ void gather_slots_kernel(const double2* __restrict__ W, double2* __restrict__ s,
                                    const int32_t* __restrict__ seg, const int32_t* __restrict__ row,
                                    const int32_t* __restrict__ row_layer, const int32_t* __restrict__ rhs_slot,
                                    int L, int sumR, int NX, int64_t ntrace) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NX) return;
  const int mi = blockIdx.y;
  const int r = blockIdx.z;
  const int g = row[mi];
  const int j = rhs_slot[(size_t)r * L + row_layer[g]];
  const int64_t si = (int64_t)r * ntrace + (int64_t)seg[mi] * NX + i;
  s[si] = j >= 0 ? W[((int64_t)j * sumR + g) * NX + i] : make_double2(0.0, 0.0);
}

__global__ void gather_owned_kernel(const double2* __restrict__ W, double2* __restrict__ u,
                                    const int32_t* __restrict__ rowmap, int sumR, int NZ, int NX, int nrhs) {
  const size_t total = (size_t)nrhs * sumR * NX;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % NX);
    const size_t rg = e / NX;
    const int gr = (int)(rg % sumR);
    const int r = (int)(rg / sumR);
    const int dst = rowmap[gr];
    if (dst >= 0) u[((size_t)r * NZ + dst) * NX + i] = W[e];
  }
}

// grid: x over NX, y over map entries, z over rhs
__global__ void trace_map_kernel(double2* W, double2* s, const double2* x, const int32_t* seg,
                                 const int32_t* row, const double* sign, int mode, int sumR, int NX,
                                 int64_t ntrace, int64_t half) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NX) return;
  const int m = blockIdx.y;
  const int r = blockIdx.z;
  const int64_t wi = ((int64_t)r * sumR + row[m]) * NX + i;
  const int64_t si = (int64_t)r * ntrace + (int64_t)seg[m] * NX + i;
  if (mode == 0) {
    s[si] = W[wi];
  } else {
    const double2 t = cadd(x[si], x[si + half]);
    const double sg = sign[m];
    const double2 w = W[wi];
    W[wi] = make_double2(w.x + sg * t.x, w.y + sg * t.y);
  }
}

__global__ void rec_rhs_kernel(double2* __restrict__ T, const double2* __restrict__ f, const double2* __restrict__ x,
                               const int32_t* __restrict__ dst, const int32_t* __restrict__ src,
                               const int32_t* __restrict__ seg, const double* __restrict__ sign, int NX, int64_t ld,
                               int64_t ntrace, int64_t half, double h2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NX) return;
  const int e = blockIdx.y;
  const int r = blockIdx.z;
  double2 v = make_double2(0.0, 0.0);
  if (src[e] >= 0) {
    const double2 fv = f[(int64_t)r * ld + (int64_t)src[e] * NX + i];
    v = make_double2(h2 * fv.x, h2 * fv.y);
  }
  const int64_t si = (int64_t)r * ntrace + (int64_t)seg[e] * NX + i;
  const double2 t = cadd(x[si], x[si + half]);
  const double sg = sign[e];
  T[(int64_t)r * ld + (int64_t)dst[e] * NX + i] = make_double2(v.x + sg * t.x, v.y + sg * t.y);
}

__global__ void zero_extrap_rows_kernel(double2* __restrict__ v, int L, int NX, int64_t ntrace) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NX) return;
  const int k = blockIdx.y;
  double2* col = v + (int64_t)blockIdx.z * ntrace;
  col[(int64_t)((0 * (L - 1) + k) * 2 + 1) * NX + i] = make_double2(0.0, 0.0);  // down pair, row n+1
  col[(int64_t)((1 * (L - 1) + k) * 2 + 0) * NX + i] = make_double2(0.0, 0.0);  // up pair, row 0
}

__global__ void identity_rhs_kernel(double2* W, const int32_t* rows, int nq, int n, int64_t ld) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (c >= n || q >= nq) return;
  W[(int64_t)(q * n + c) * ld + (int64_t)rows[q] * n + c] = make_double2(1.0, 0.0);
}

__global__ void pack_block_kernel(const double2* __restrict__ W, int64_t ld, int q, int row, int n, double sign,
                                  double shift, double2* dst64, float2* dst32) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // row-major destination index
  if (e >= (size_t)n * n) return;
  const int i = (int)(e / n), c = (int)(e % n);
  const double2 v = W[(int64_t)(q * n + c) * ld + (int64_t)row * n + i];
  double2 o = make_double2(sign * v.x, sign * v.y);
  if (i == c) o.x += shift;
  if (dst64) dst64[e] = o;
  if (dst32) dst32[e] = make_float2((float)o.x, (float)o.y);
}

// C = alpha A (B + shift I) for row-major complex n x n blocks (setup only): 16 x 16 output tiles, the
// k-range walked in 16-wide LDS slices, each output summed in a fixed order
__global__ __launch_bounds__(256) void setup_gemm_kernel(const double2* __restrict__ A, const double2* __restrict__ B,
                                                         double2* __restrict__ C, int n, double2 alpha,
                                                         double shift) {
  __shared__ double2 As[16][17], Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
  double2 acc = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < n; k0 += 16) {
    const int ka = k0 + tx, kb = k0 + ty;
    As[ty][tx] = (row < n && ka < n) ? A[(size_t)row * n + ka] : make_double2(0.0, 0.0);
    double2 b = (kb < n && col < n) ? B[(size_t)kb * n + col] : make_double2(0.0, 0.0);
    if (kb == col && kb < n) b.x += shift;
    Bs[ty][tx] = b;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc = cadd(acc, cmul(As[ty][k], Bs[k][tx]));
    __syncthreads();
  }
  if (row < n && col < n) C[(size_t)row * n + col] = cmul(alpha, acc);
}

// dst = sign src + shift I (row-major n x n)
__global__ void sign_copy_kernel(const double2* __restrict__ src, double2* __restrict__ dst, int n, double sign,
                                 double shift) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const double2 v = src[e];
  double2 o = make_double2(sign * v.x, sign * v.y);
  if (e / n == e % n) o.x += shift;
  dst[e] = o;
}

__global__ void copy_kernel(double2* __restrict__ d, const double2* __restrict__ s, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    d[e] = s[e];
}
__global__ void zero_kernel(double2* __restrict__ d, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    d[e] = make_double2(0.0, 0.0);
}
__global__ void add_kernel(double2* y, const double2* x, const double2* z, double sign, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const double2 a = x[e], b = z[e];
    y[e] = make_double2(a.x + sign * b.x, a.y + sign * b.y);
  }
}

// ----------------------------------------------------------------------------
// Krylov kernels (float64)
// ----------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The Krylov reductions (one dot product or norm per workgroup: a few to a
// few hundred workgroups per launch) use 1024-thread workgroups, so that a
// launch for one or a few sources still has many loads in flight; the 16 wave
// sums are added in wave order.
constexpr int kRedThreads = 1024;
constexpr int kRedWaves = kRedThreads / 64;

// grid: (m, nrhs), kRedThreads threads
__global__ __launch_bounds__(kRedThreads) void kdot_kernel(const double2* __restrict__ V, const double2* __restrict__ w,
                                                           double2* __restrict__ hout, int nrhs, int64_t N) {
  const int i = blockIdx.x, r = blockIdx.y;
  const double2* v = V + ((int64_t)i * nrhs + r) * N;
  const double2* x = w + (int64_t)r * N;
  double re = 0.0, im = 0.0;
  for (int64_t e = threadIdx.x; e < N; e += kRedThreads) {
    const double2 t = cconjmul(v[e], x[e]);
    re += t.x;
    im += t.y;
  }
  __shared__ double sre[kRedWaves], sim[kRedWaves];
  re = wave_sum(re);
  im = wave_sum(im);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    sre[wv] = re;
    sim[wv] = im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = sre[0], b = sim[0];
    for (int k = 1; k < kRedWaves; ++k) {
      a += sre[k];
      b += sim[k];
    }
    hout[(int64_t)i * nrhs + r] = make_double2(a, b);
  }
}

__global__ void kupdate_kernel(const double2* __restrict__ V, double2* __restrict__ w, const double2* __restrict__ h,
                               double2* __restrict__ hacc, int m, int nrhs, int64_t N) {
  if (blockIdx.x == 0) {
    for (int t = threadIdx.x; t < m * nrhs; t += blockDim.x) hacc[t] = cadd(hacc[t], h[t]);
  }
  const int64_t total = (int64_t)nrhs * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / N);
    const int64_t k = e - (int64_t)r * N;
    double2 acc = w[e];
    for (int i = 0; i < m; ++i) {
      const double2 t = cmul(h[(int64_t)i * nrhs + r], V[((int64_t)i * nrhs + r) * N + k]);
      acc.x -= t.x;
      acc.y -= t.y;
    }
    w[e] = acc;
  }
}

__global__ __launch_bounds__(kRedThreads) void knorm_kernel(const double2* __restrict__ w, double* __restrict__ nrm,
                                                            int64_t N) {
  const int r = blockIdx.x;
  const double2* x = w + (int64_t)r * N;
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < N; e += kRedThreads) s += x[e].x * x[e].x + x[e].y * x[e].y;
  __shared__ double ss[kRedWaves];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) ss[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = ss[0];
    for (int k = 1; k < kRedWaves; ++k) t += ss[k];
    nrm[r] = sqrt(t);
  }
}

__global__ void kscale_kernel(double2* v, const double2* w, const double* nrm, int nrhs, int64_t N) {
  const int64_t total = (int64_t)nrhs * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / N);
    const double s = nrm[r];
    const double2 x = w[e];
    v[e] = s > 0.0 ? make_double2(x.x / s, x.y / s) : make_double2(0.0, 0.0);
  }
}

__global__ void kmulnorm_kernel(double2* v, const double* nrm, int nrhs, int64_t N) {
  const int64_t total = (int64_t)nrhs * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const double s = nrm[(int)(e / N)];
    v[e] = make_double2(v[e].x * s, v[e].y * s);
  }
}

__global__ void givens_kernel(double2* Hc, const double2* hacc, const double* nrm, double* cs, double2* sn,
                              double2* g, double* est, const double* beta, int32_t* iters, int32_t* done,
                              double tol, int j, int mdim, int nrhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double2* H = Hc + (size_t)r * (mdim + 1) * mdim + (size_t)j * (mdim + 1);
  for (int i = 0; i <= j; ++i) H[i] = hacc[(size_t)i * nrhs + r];
  H[j + 1] = make_double2(nrm[r], 0.0);
  double* c = cs + (size_t)r * mdim;
  double2* s = sn + (size_t)r * mdim;
  double2* gg = g + (size_t)r * (mdim + 1);
  for (int i = 0; i < j; ++i) {
    const double2 a = H[i], b = H[i + 1];
    const double2 sb = cmul(s[i], b);
    const double2 sa = cconjmul(s[i], a);  // conj(s) a
    H[i] = make_double2(c[i] * a.x + sb.x, c[i] * a.y + sb.y);
    H[i + 1] = make_double2(-sa.x + c[i] * b.x, -sa.y + c[i] * b.y);
  }
  const double2 a = H[j], b = H[j + 1];
  const double na = hypot(a.x, a.y), nb = hypot(b.x, b.y);
  double cj;
  double2 sj;
  if (nb == 0.0) {
    cj = 1.0;
    sj = make_double2(0.0, 0.0);
  } else if (na == 0.0) {
    cj = 0.0;
    sj = make_double2(1.0, 0.0);
  } else {
    const double t = hypot(na, nb);
    cj = na / t;
    const double2 ph = make_double2(a.x / na, a.y / na);
    sj = cmul(ph, make_double2(b.x / t, -b.y / t));
  }
  c[j] = cj;
  s[j] = sj;
  const double2 sb = cmul(sj, b);
  H[j] = make_double2(cj * a.x + sb.x, cj * a.y + sb.y);
  H[j + 1] = make_double2(0.0, 0.0);
  const double2 gj = gg[j];
  const double2 t = cconjmul(sj, gj);
  gg[j + 1] = make_double2(-t.x, -t.y);
  gg[j] = make_double2(cj * gj.x, cj * gj.y);
  const double e = hypot(gg[j + 1].x, gg[j + 1].y) / beta[r];
  if (!done[r]) {
    est[r] = e;
    iters[r] = j + 1;
    if (e < tol || !(nrm[r] > 0.0)) done[r] = 1;
  }
}

__global__ void ksolve_kernel(const double2* Hc, const double2* g, double2* y, const int32_t* iters, int mdim,
                              int nrhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const double2* H = Hc + (size_t)r * (mdim + 1) * mdim;
  const double2* gg = g + (size_t)r * (mdim + 1);
  double2* yy = y + (size_t)r * mdim;
  const int k = iters[r];
  for (int i = k - 1; i >= 0; --i) {
    double2 acc = gg[i];
    for (int c = i + 1; c < k; ++c) {
      const double2 t = cmul(H[(size_t)c * (mdim + 1) + i], yy[c]);
      acc.x -= t.x;
      acc.y -= t.y;
    }
    const double2 d = H[(size_t)i * (mdim + 1) + i];
    yy[i] = (d.x == 0.0 && d.y == 0.0) ? make_double2(0.0, 0.0) : cdiv(acc, d);
  }
}

__global__ void kcombine_kernel(const double2* __restrict__ Z, const double2* __restrict__ y,
                                const int32_t* __restrict__ iters, double2* __restrict__ x, int mdim, int nrhs,
                                int64_t N) {
  const int64_t total = (int64_t)nrhs * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / N);
    const int64_t k = e - (int64_t)r * N;
    double2 acc = make_double2(0.0, 0.0);
    const int m = iters[r];
    for (int j = 0; j < m; ++j) acc = cadd(acc, cmul(y[(size_t)r * mdim + j], Z[((int64_t)j * nrhs + r) * N + k]));
    x[e] = acc;
  }
}

__global__ void kinit_kernel(double2* g, const double* beta, int32_t* done, int32_t* iters, double* est, int mdim,
                             int nrhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double2* gg = g + (size_t)r * (mdim + 1);
  for (int i = 0; i <= mdim; ++i) gg[i] = make_double2(0.0, 0.0);
  gg[0] = make_double2(beta[r], 0.0);
  done[r] = beta[r] > 0.0 ? 0 : 1;  // zero, or not finite (NaN / Inf source): nothing to iterate
  iters[r] = 0;
  est[r] = beta[r] > 0.0 ? 1.0 : (beta[r] == 0.0 ? 0.0 : __builtin_nan(""));
}

__global__ void to_f32_kernel(float2* __restrict__ d, const double2* __restrict__ s, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    d[e] = make_float2((float)s[e].x, (float)s[e].y);
}

inline unsigned grid_for(int64_t n, int cap = 8192) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_nonzero_chunks(const double2* B, int64_t ld, int ncols, const int64_t* off, const int32_t* kk,
                                 int nentries, int32_t* list, int stride, hipStream_t st) {
  if (nentries <= 0) return hipSuccess;
  hipLaunchKernelGGL(nonzero_chunks_kernel, dim3(nentries), dim3(256), 0, st, B, ld, ncols, off, kk, list, stride);
  return hipGetLastError();
}


// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
hipError_t launch_block_apply(const Job* jobs, int njobs, const ApplyGeom& g, int nrhs, int64_t ld, Bases bases,
                              bool f32, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, double2* mpart,
                              size_t mpart_n) {
  if (njobs <= 0) return hipSuccess;
  const ApplySeg sg{jobs, njobs, g.n, nrhs, ld, bases, nullptr, 0};
  ApplyForm f{};
  if (!g.gemv && !g.mfma) return hipErrorInvalidValue;  // every shape is one of the two forms
  f.kind = g.gemv ? 0 : 1;
  f.nr = g.nr;
  f.tn = g.mfma;
  f.ks = g.ks;
  f.pipe = g.steps != 1;
  // MFMA k-slices only where the workspace holds every slice's partial tiles
  if (g.mks > 1 && mpart && (size_t)g.mks * njobs * nrhs * g.n <= mpart_n) {
    f.mks = g.mks;
    f.mpart = mpart;
  }
  const SegTableT<1> t = seg_table<1>(&sg, 1);
  return f32 ? launch_apply_t<true, 1>(t, f, st, ev0, ev1) : launch_apply_t<false, 1>(t, f, st, ev0, ev1);
}

hipError_t launch_block_apply_segs(const ApplySeg* segs, int nseg, int maxterms, bool wide, bool f32,
                                   hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (nseg <= 0) return hipSuccess;
  if (nseg > kMaxSeg) return hipErrorInvalidValue;
  int rmax = 0, rmin = INT32_MAX;
  long rows = 0;
  bool multi = wide || maxterms > 1;
  for (int i = 0; i < nseg; ++i) {
    if (segs[i].njobs <= 0 || segs[i].n <= 0 || segs[i].nrhs <= 0) return hipErrorInvalidValue;
    rmax = std::max(rmax, segs[i].nrhs);
    rmin = std::min(rmin, segs[i].nrhs);
    rows += (long)segs[i].njobs * ((segs[i].n + 63) / 64);
    multi = multi || segs[i].n > 256;  // a streaming chunk holds at most 256 columns
  }
  ApplyForm f{};
  f.nr = rmax <= 1 ? 1 : rmax <= 2 ? 2 : rmax <= 4 ? 4 : rmax <= 8 ? 8 : 16;
  f.pipe = multi;
  if (rmax <= 4) {
    f.kind = 0;
  } else {
    // the widest tile that still gives about two workgroups per CU, never wider
    // than the fewest right-hand sides rounded up to 16 (the single launch's rule)
    f.kind = 1;
    f.tn = 16;
    for (int tn : {64, 32})
      if (tn <= 16 * ((rmin + 15) / 16) && rows * ((rmax + tn - 1) / tn) >= 512) {
        f.tn = tn;
        break;
      }
  }
  const SegTableT<kMaxSeg> t = seg_table<kMaxSeg>(segs, nseg);
  return f32 ? launch_apply_t<true, kMaxSeg>(t, f, st, ev0, ev1) : launch_apply_t<false, kMaxSeg>(t, f, st, ev0, ev1);
}


hipError_t launch_gj_panel(double2* const* A, int nb, int n, int k0, int bw, int32_t* perm, int32_t* flag,
                           hipStream_t st) {
  if (n > 4096 || bw > kGjBw) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gj_panel_kernel, dim3(nb), dim3(1024), 0, st, A, n, k0, bw, perm, flag);
  return hipGetLastError();
}
hipError_t launch_gj_update(double2* const* A, double2* const* B, int nb, int n, int k0, int bw, const int32_t* perm,
                            hipStream_t st) {
  if (n > 4096 || bw > kGjBw) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gj_update_kernel, dim3((n + kGjCols - 1) / kGjCols, nb), dim3(256), 0, st, A, B, n, k0, bw,
                     perm);
  return hipGetLastError();
}
int gj_panel_width() { return kGjBw; }

hipError_t launch_gj_perm(const int32_t* perm, int32_t* pi, int nb, int n, hipStream_t st) {
  hipLaunchKernelGGL(gj_perm_kernel, dim3((nb + 63) / 64), dim3(64), 0, st, perm, pi, nb, n);
  return hipGetLastError();
}

hipError_t launch_init_delta(double2* const* out, const double2* const* diag, const double2* west,
                             const double2* east, int nb, int n, hipStream_t st) {
  const unsigned gx = (unsigned)(((size_t)n * n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(init_delta_kernel, dim3(gx, nb), dim3(kThreads), 0, st, out, diag, west, east, n);
  return hipGetLastError();
}

hipError_t launch_twist_combine(double2* const* G, const double2* const* Y, const double2* const* diag,
                                const double2* west, const double2* east, int nb, int n, hipStream_t st) {
  const unsigned gx = (unsigned)(((size_t)n * n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(twist_combine_kernel, dim3(gx, nb), dim3(kThreads), 0, st, G, Y, diag, west, east, n);
  return hipGetLastError();
}

hipError_t launch_finish_row(double2* const* B, const int32_t* pi, double2* const* dinv64, double2* const* nextD,
                             const double2* const* next_diag, const double2* coef, const double2* west,
                             const double2* east, int nb, int n, hipStream_t st) {
  const unsigned gx = (unsigned)(((size_t)n * n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(finish_row_kernel, dim3(gx, nb), dim3(kThreads), 0, st, B, pi, dinv64, nextD, next_diag, coef,
                     west, east, n);
  return hipGetLastError();
}

hipError_t launch_scatter_source(const double2* f, double2* W, const int32_t* rowmap, int sumR, int NZ, int NX,
                                 int nrhs, double scale, hipStream_t st) {
  hipLaunchKernelGGL(scatter_source_kernel, dim3(grid_for((int64_t)nrhs * sumR * NX)), dim3(kThreads), 0, st, f,
                     W, rowmap, sumR, NZ, NX, nrhs, scale);
  return hipGetLastError();
}

hipError_t launch_source_activity(const double2* f, double* amax, const int32_t* own_start, const int32_t* n_own,
                                  int L, int NZ, int NX, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(source_activity_kernel, dim3(L, nrhs), dim3(kActThreads), 0, st, f, amax, own_start, n_own, L,
                     NZ, NX);
  return hipGetLastError();
}

hipError_t launch_scatter_slots(const double2* f, double2* W, const int32_t* rowmap, const int32_t* row_layer,
                                const int32_t* slot_rhs, int m, int sumR, int NZ, int NX, double scale,
                                hipStream_t st) {
  hipLaunchKernelGGL(scatter_slots_kernel, dim3(grid_for((int64_t)m * sumR * NX)), dim3(kThreads), 0, st, f, W,
                     rowmap, row_layer, slot_rhs, m, sumR, NZ, NX, scale);
  return hipGetLastError();
}

hipError_t launch_gather_slots(const double2* W, double2* s, const int32_t* seg, const int32_t* row,
                               const int32_t* row_layer, const int32_t* rhs_slot, int nmap, int L, int sumR, int NX,
                               int64_t ntrace, int nrhs, hipStream_t st) {
  if (nmap <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_slots_kernel, dim3((NX + 255) / 256, nmap, nrhs), dim3(256), 0, st, W, s, seg, row,
                     row_layer, rhs_slot, L, sumR, NX, ntrace);
  return hipGetLastError();
}

hipError_t launch_gather_owned(const double2* W, double2* u, const int32_t* rowmap, int sumR, int NZ, int NX,
                               int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(gather_owned_kernel, dim3(grid_for((int64_t)nrhs * sumR * NX)), dim3(kThreads), 0, st, W, u,
                     rowmap, sumR, NZ, NX, nrhs);
  return hipGetLastError();
}

hipError_t launch_trace_map(double2* W, double2* s, const double2* x, const int32_t* seg, const int32_t* row,
                            const double* sign, int nmap, int mode, int sumR, int NX, int64_t ntrace, int nrhs,
                            int64_t half, hipStream_t st) {
  if (nmap <= 0) return hipSuccess;
  dim3 grid((NX + 127) / 128, nmap, nrhs);
  hipLaunchKernelGGL(trace_map_kernel, grid, dim3(128), 0, st, W, s, x, seg, row, sign, mode, sumR, NX, ntrace,
                     half);
  return hipGetLastError();
}

hipError_t launch_rec_rhs(double2* T, const double2* f, const double2* x, const int32_t* dst, const int32_t* src,
                          const int32_t* seg, const double* sign, int ne, int NX, int64_t ld, int64_t ntrace,
                          int64_t half, double h2, int nrhs, hipStream_t st) {
  if (ne <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(rec_rhs_kernel, dim3((NX + 127) / 128, ne, nrhs), dim3(128), 0, st, T, f, x, dst, src, seg, sign,
                     NX, ld, ntrace, half, h2);
  return hipGetLastError();
}

hipError_t launch_zero_extrap_rows(double2* v, int L, int NX, int64_t ntrace, int nrhs, hipStream_t st) {
  if (L < 2 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_extrap_rows_kernel, dim3((NX + 127) / 128, L - 1, nrhs), dim3(128), 0, st, v, L, NX,
                     ntrace);
  return hipGetLastError();
}

hipError_t launch_identity_rhs(double2* W, const int32_t* rows, int nq, int n, int64_t ld, hipStream_t st) {
  hipLaunchKernelGGL(identity_rhs_kernel, dim3((n + 127) / 128, nq), dim3(128), 0, st, W, rows, nq, n, ld);
  return hipGetLastError();
}

hipError_t launch_pack_block(const double2* W, int64_t ld, int q, int row, int n, double sign, double shift,
                             double2* dst64, float2* dst32, hipStream_t st) {
  const unsigned gx = (unsigned)(((size_t)n * n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(pack_block_kernel, dim3(gx), dim3(kThreads), 0, st, W, ld, q, row, n, sign, shift, dst64,
                     dst32);
  return hipGetLastError();
}

hipError_t launch_setup_gemm(const double2* A, const double2* B, double2* C, int n, double2 alpha, double shift,
                             hipStream_t st) {
  const unsigned t = (unsigned)((n + 15) / 16);
  hipLaunchKernelGGL(setup_gemm_kernel, dim3(t, t), dim3(256), 0, st, A, B, C, n, alpha, shift);
  return hipGetLastError();
}
hipError_t launch_sign_copy(const double2* src, double2* dst, int n, double sign, double shift, hipStream_t st) {
  const unsigned gx = (unsigned)(((size_t)n * n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(sign_copy_kernel, dim3(gx), dim3(kThreads), 0, st, src, dst, n, sign, shift);
  return hipGetLastError();
}

hipError_t launch_pack_green(const double2* W, int64_t ld, int q, int j, int r0, int nrows, int NX,
                             const double2* ax, const double2* az, double2* G, hipStream_t st) {
  if (nrows <= 0) return hipSuccess;
  const int64_t cnt = (int64_t)nrows * NX;
  const dim3 grid((unsigned)((cnt + 255) / 256), (unsigned)NX);
  hipLaunchKernelGGL(pack_green_kernel, grid, dim3(256), 0, st, W, ld, q, j, r0, nrows, NX, ax, az, G);
  return hipGetLastError();
}

hipError_t launch_sum_rows(double2* W, int64_t ld, int NX, const int32_t* dst, const int32_t* src0,
                           const int32_t* cnt, int nentries, int ncols, hipStream_t st) {
  if (nentries <= 0 || ncols <= 0) return hipSuccess;
  const dim3 grid((unsigned)((NX + 255) / 256), (unsigned)nentries, (unsigned)ncols);
  hipLaunchKernelGGL(sum_rows_kernel, grid, dim3(256), 0, st, W, ld, NX, dst, src0, cnt);
  return hipGetLastError();
}

hipError_t launch_copy(double2* dst, const double2* src, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(kThreads), 0, st, dst, src, n);
  return hipGetLastError();
}
hipError_t launch_zero(double2* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n)), dim3(kThreads), 0, st, dst, n);
  return hipGetLastError();
}
hipError_t launch_add(double2* y, const double2* x, const double2* z, double sign, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(add_kernel, dim3(grid_for(n)), dim3(kThreads), 0, st, y, x, z, sign, n);
  return hipGetLastError();
}

hipError_t launch_kdot(const double2* V, const double2* w, double2* hout, int m, int nrhs, int64_t N,
                       hipStream_t st) {
  hipLaunchKernelGGL(kdot_kernel, dim3(m, nrhs), dim3(kRedThreads), 0, st, V, w, hout, nrhs, N);
  return hipGetLastError();
}
hipError_t launch_kupdate(const double2* V, double2* w, const double2* h, double2* hacc, int m, int nrhs, int64_t N,
                          hipStream_t st) {
  hipLaunchKernelGGL(kupdate_kernel, dim3(grid_for((int64_t)nrhs * N)), dim3(kThreads), 0, st, V, w, h, hacc, m,
                     nrhs, N);
  return hipGetLastError();
}
hipError_t launch_knorm(const double2* w, double* nrm, int nrhs, int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(knorm_kernel, dim3(nrhs), dim3(kRedThreads), 0, st, w, nrm, N);
  return hipGetLastError();
}
hipError_t launch_kscale(double2* v, const double2* w, const double* nrm, int nrhs, int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(kscale_kernel, dim3(grid_for((int64_t)nrhs * N)), dim3(kThreads), 0, st, v, w, nrm, nrhs, N);
  return hipGetLastError();
}
hipError_t launch_kmulnorm(double2* v, const double* nrm, int nrhs, int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(kmulnorm_kernel, dim3(grid_for((int64_t)nrhs * N)), dim3(kThreads), 0, st, v, nrm, nrhs, N);
  return hipGetLastError();
}
hipError_t launch_givens(double2* Hc, const double2* hacc, const double* nrm, double* cs, double2* sn, double2* g,
                         double* est, const double* beta, int32_t* iters, int32_t* done, double tol, int j,
                         int mdim, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(givens_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, st, Hc, hacc, nrm, cs, sn, g, est, beta,
                     iters, done, tol, j, mdim, nrhs);
  return hipGetLastError();
}
hipError_t launch_ksolve(const double2* Hc, const double2* g, double2* y, const int32_t* iters, int mdim, int nrhs,
                         hipStream_t st) {
  hipLaunchKernelGGL(ksolve_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, st, Hc, g, y, iters, mdim, nrhs);
  return hipGetLastError();
}
hipError_t launch_kinit(double2* g, const double* beta, int32_t* done, int32_t* iters, double* est, int mdim,
                        int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(kinit_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, st, g, beta, done, iters, est, mdim, nrhs);
  return hipGetLastError();
}
hipError_t launch_to_f32(float2* d, const double2* s, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(to_f32_kernel, dim3(grid_for(n)), dim3(kThreads), 0, st, d, s, n);
  return hipGetLastError();
}
hipError_t launch_kcombine(const double2* Z, const double2* y, const int32_t* iters, double2* x, int mdim, int nrhs,
                           int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(kcombine_kernel, dim3(grid_for((int64_t)nrhs * N)), dim3(kThreads), 0, st, Z, y, iters, x,
                     mdim, nrhs, N);
  return hipGetLastError();
}

}  // namespace polar
