// Partitioned low-rank (PLR) trace blocks: compression at setup and the online
// apply kernel, both on the GPU.
//
// Compression follows the adaptive quadtree of the paper's Alg. 5: a block
// becomes a leaf when its (r_max+1)-th singular value is below eps (absolute),
// keeping the k <= r_max triplets with sigma >= eps; otherwise it is split
// into four (ceil/floor halves) and each quarter is compressed; a block whose
// smaller side is <= r_max is a dense leaf.  The singular values are those of
// a randomized sketch (Section 7: the compression uses a randomized SVD):
// Y = M Omega with s = r_max + 1 + 10 Gaussian columns (at most 70), one power
// iteration Y = M (M^H Q) with re-orthonormalisation, B = Q^H M, and the SVD
// of B from X = B^H = Q2 R and a one-sided (Hestenes) Jacobi SVD of the small
// factor R, which keeps the small singular values accurate.
// A candidate leaf is accepted only if four random probes see an error below
// eps.  The leaves are applied in the factored form y[rows] += U (V x[cols])
// of the paper's Alg. 6 / sparse-factorised product.
//
// The quadtree is processed one level at a time: every candidate node of a
// level (across all blocks) is one entry of a node table, and each step of the
// randomized SVD is one batched launch over that table (one workgroup per node,
// or per node and 64-row tile for the products).  The host reads back only the
// per-node decision (accepted, rank) to form the next level; the factors go
// from the staging buffer straight into the packed leaf data on the device.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "persist.h"
#include "plr.h"

namespace polar {

namespace {

__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double znorm(double2 a) { return a.x * a.x + a.y * a.y; }

// ----------------------------------------------------------------------------
// compression (setup)
// ----------------------------------------------------------------------------
// widest sketch: r_max + 1 + 10 columns, at most 70 so that the Jacobi SVD's
// two s x s factors fit the 160 KiB of LDS (the oversampling drops to 5 at r_max = 64)
constexpr int kSMax = 70;
constexpr int kCpw = (kSMax + 3) / 4;        // product columns per wave (4 waves)
constexpr int kKc = 16;                      // inner-dimension chunk of the products
constexpr int kGsq = 6;                      // Gram-Schmidt dot products per wave and pass

// per-node staging slots (complex entries, column-major unless noted)
enum Slot {
  S_OM = 0,  // Omega, n x s
  S_Y,       // Y = M Omega, then Q (m x s)
  S_T,       // M^H Q (n x s); at the end X = B^H, then Q2 of X = Q2 R
  S_R,       // R of X = Q2 R (column-major, leading dimension s)
  S_U,       // leaf U = Q W diag(sigma), m x k row-major
  S_V,       // leaf V^T, n x k row-major (V = Z^H)
  S_P4,      // probe vectors, n x 4
  S_Y4,      // M times the probes, m x 4
  S_NSLOT
};

struct CNode {
  int32_t blk, r0, c0, m, n, s;
  int64_t off[S_NSLOT];
};

// per-node results: r = orthonormal sketch rank, r2 = rank of X = B^H, k = leaf
// rank, ok = accepted
struct CRes {
  int32_t r, r2, k, ok;
};

// A leaf to copy into the packed data: k < 0 dense (from the block), else U
// and V^T from the staging buffer.
struct EmitRec {
  int32_t blk, r0, c0, m, n, k;
  int64_t srcU, srcV, dst;
};

// SplitMix64 finaliser (Steele, Lea, Flood 2014) as a counter-based generator;
// two uniforms -> one complex normal by Box-Muller.
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double2 cnormal(uint64_t key, uint64_t i) {
  const uint64_t a = mix64(key + (2 * i + 1) * 0x9E3779B97F4A7C15ull);
  const uint64_t b = mix64(key + (2 * i + 2) * 0x9E3779B97F4A7C15ull);
  const double u1 = ((double)(a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = ((double)(b >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double rr = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);
  return make_double2(rr * cs, rr * sn);
}

__device__ __forceinline__ double wave_sum(double v) {
  // xor butterfly: every lane ends with the same bits (each step adds a pair in both orders)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sum over an aligned group of 16 lanes (same bits in every lane of the group)
__device__ __forceinline__ double group16_sum(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 16);
  return v;
}

// sum over the 256 threads of a workgroup, in a fixed order; every thread gets it
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// slot `slot` of each node <- complex normals, n x s (four = 0) or n x 4 (four = 1)
__global__ __launch_bounds__(256) void plr_random_kernel(const CNode* __restrict__ nodes, double2* __restrict__ buf,
                                                         int slot, int four, uint64_t seed) {
  const CNode& nd = nodes[blockIdx.x];
  uint64_t key = mix64(seed ^ (uint64_t)nd.blk);
  key = mix64(key ^ ((uint64_t)nd.r0 << 32 | (uint32_t)nd.c0));
  key = mix64(key ^ ((uint64_t)nd.m << 32 | (uint32_t)nd.n));
  const int64_t cnt = (int64_t)nd.n * (four ? 4 : nd.s);
  double2* out = buf + nd.off[slot];
  for (int64_t i = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.y * blockDim.x)
    out[i] = cnormal(key, (uint64_t)i);
}

// out = op(M_node) P with op(M) = M (m x n, CONJ = false) or M^H (n x m, CONJ =
// true); P is inner x cols and out outer x cols, column-major with leading
// dimensions inner and outer.  cols: the node's sketch width s (cols_mode 0),
// its orthonormal rank r (1) or 4 (2).  grid = (nodes, 64-row tiles of the
// widest node); lane = output row, wave w takes the columns w, w + 4, ...; the
// operand tiles are staged in LDS with coalesced loads.
template <bool CONJ>
__global__ __launch_bounds__(256) void plr_panel_kernel(const CNode* __restrict__ nodes, const CRes* __restrict__ res,
                                                        const double2* __restrict__ blocks, int N,
                                                        double2* __restrict__ buf, int in_slot, int out_slot,
                                                        int cols_mode) {
  __shared__ double2 Ms[64][kKc + 1];
  __shared__ double2 Ps[kSMax][kKc + 1];
  const CNode& nd = nodes[blockIdx.x];
  const int outer = CONJ ? nd.n : nd.m, inner = CONJ ? nd.m : nd.n;
  const int tile0 = blockIdx.y * 64;
  if (tile0 >= outer) return;
  const int cols = cols_mode == 0 ? nd.s : (cols_mode == 1 ? res[blockIdx.x].r : 4);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const double2* M = blocks + (size_t)nd.blk * N * N + (size_t)nd.r0 * N + nd.c0;
  const double2* P = buf + nd.off[in_slot];
  double2 acc[kCpw];
#pragma unroll
  for (int jj = 0; jj < kCpw; ++jj) acc[jj] = make_double2(0.0, 0.0);
  for (int i0 = 0; i0 < inner; i0 += kKc) {
    __syncthreads();
    if (!CONJ) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {  // Ms[o][i] = M(tile0 + o, i0 + i): 16 consecutive columns per row
        const int o = (t >> 4) + 16 * q, i = t & 15;
        double2 v = make_double2(0.0, 0.0);
        if (tile0 + o < outer && i0 + i < inner) v = M[(size_t)(tile0 + o) * N + i0 + i];
        Ms[o][i] = v;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {  // Ms[o][i] = conj(M(i0 + i, tile0 + o)): 64 consecutive columns per row
        const int o = t & 63, i = (t >> 6) + 4 * q;
        double2 v = make_double2(0.0, 0.0);
        if (tile0 + o < outer && i0 + i < inner) {
          v = M[(size_t)(i0 + i) * N + tile0 + o];
          v.y = -v.y;
        }
        Ms[o][i] = v;
      }
    }
    for (int e = t; e < cols * kKc; e += 256) {
      const int j = e / kKc, i = e % kKc;
      Ps[j][i] = (i0 + i < inner) ? P[(size_t)j * inner + i0 + i] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int ni = min(kKc, inner - i0);
    for (int i = 0; i < ni; ++i) {
      const double2 a = Ms[lane][i];
#pragma unroll
      for (int jj = 0; jj < kCpw; ++jj) {
        const int j = w + 4 * jj;
        if (j < cols) acc[jj] = zadd(acc[jj], zmul(a, Ps[j][i]));
      }
    }
  }
  const int o = tile0 + lane;
  if (o < outer) {
    double2* O = buf + nd.off[out_slot];
#pragma unroll
    for (int jj = 0; jj < kCpw; ++jj) {
      const int j = w + 4 * jj;
      if (j < cols) O[(size_t)j * outer + o] = acc[jj];
    }
  }
}

// Orthonormalise the columns of slot `slot` (m x cols, m = the node's outer
// size `rows`, cols = s or the node's current r) in place: classical
// Gram-Schmidt applied twice per column, a column whose remaining norm is below
// 1e-14 of its original norm dropped, the kept ones compacted to the front.
// Without R (rslot < 0) res.r = the number kept; with R, res.r2 = that number
// and slot rslot holds R (column j: the coefficients of input column j on the
// kept columns, leading dimension s), so input = kept R.  One workgroup per
// node; the column being orthogonalised lives in global memory (L2-resident).
__global__ __launch_bounds__(256) void plr_orth_kernel(const CNode* __restrict__ nodes, CRes* __restrict__ res,
                                                       double2* __restrict__ buf, int slot, int use_r, int by_n,
                                                       int rslot) {
  __shared__ double2 d[kSMax];
  __shared__ double red[4];
  const CNode& nd = nodes[blockIdx.x];
  const int m = by_n ? nd.n : nd.m;
  const int cols = use_r ? res[blockIdx.x].r : nd.s;
  double2* Y = buf + nd.off[slot];
  double2* R = rslot >= 0 ? buf + nd.off[rslot] : nullptr;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int r = 0;
  for (int j = 0; j < cols; ++j) {
    double2* yj = Y + (size_t)j * m;
    if (R && t < nd.s) R[(size_t)j * nd.s + t] = make_double2(0.0, 0.0);
    double s0 = 0.0;
    for (int i = t; i < m; i += 256) s0 += znorm(yj[i]);
    const double n0 = sqrt(block_sum(s0, red));
    for (int pass = 0; pass < 2; ++pass) {
      // d[q] = q-th basis column^H y; wave w takes q = w, w + 4, ..., kGsq of them per pass over the rows
      for (int qb = 0; qb < r; qb += 4 * kGsq) {
        double re[kGsq], im[kGsq];
#pragma unroll
        for (int u = 0; u < kGsq; ++u) re[u] = im[u] = 0.0;
        for (int i = lane; i < m; i += 64) {
          const double2 b = yj[i];
#pragma unroll
          for (int u = 0; u < kGsq; ++u) {
            const int q = qb + w + 4 * u;
            if (q < r) {
              const double2 a = Y[(size_t)q * m + i];
              re[u] += a.x * b.x + a.y * b.y;
              im[u] += a.x * b.y - a.y * b.x;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kGsq; ++u) {
          const int q = qb + w + 4 * u;
          if (q < r) {  // uniform over the wave
            const double x = wave_sum(re[u]), y = wave_sum(im[u]);
            if (lane == 0) d[q] = make_double2(x, y);
          }
        }
      }
      __syncthreads();
      if (R && t < r) R[(size_t)j * nd.s + t] = zadd(R[(size_t)j * nd.s + t], d[t]);
      for (int i = t; i < m; i += 256) {
        double2 v = yj[i];
#pragma unroll 8
        for (int q = 0; q < r; ++q) v = zsub(v, zmul(Y[(size_t)q * m + i], d[q]));
        yj[i] = v;
      }
      __syncthreads();
    }
    double s1 = 0.0;
    for (int i = t; i < m; i += 256) s1 += znorm(yj[i]);
    const double nn = sqrt(block_sum(s1, red));
    if (!(nn > 1e-14 * fmax(n0, 1e-300))) continue;  // dependent column: dropped (uniform over the group)
    const double inv = 1.0 / nn;
    double2* dst = Y + (size_t)r * m;
    for (int i = t; i < m; i += 256) dst[i] = zscale(yj[i], inv);
    if (R && t == 0) R[(size_t)j * nd.s + r] = make_double2(nn, 0.0);
    __syncthreads();
    ++r;
  }
  if (t == 0) {
    if (R)
      res[blockIdx.x].r2 = r;
    else
      res[blockIdx.x].r = r;
  }
}

// SVD of B = Q^H M (r x n) from X = B^H = M^H Q = Q2 R (slots T and R; R is
// r2 x r): a one-sided Jacobi SVD of R, whose columns are rotated until
// mutually orthogonal, R W = Z' diag(sigma), so X W = (Q2 Z') diag(sigma) and
// B = W diag(sigma) (Q2 Z')^H.  R and W sit in LDS (leading dimension ld);
// disjoint pairs in round-robin order (16 lanes per pair, 16 pairs at a time,
// r - 1 rounds per sweep, a sweep without rotations ends it).  Then sigma = column norms sorted
// descending, the leaf decision of Alg. 5 (sigma_{r_max+1} < eps), k =
// #{sigma >= eps, first r_max}, and for a candidate leaf U = Q W(:, :k)
// diag(sigma) (slot U) and V^T = conj(Q2 Z'(:, :k)) (slot V).  One workgroup
// per node.
__global__ __launch_bounds__(256) void plr_svd_kernel(const CNode* __restrict__ nodes, CRes* __restrict__ res,
                                                      double2* __restrict__ buf, int ld, int rmax, double eps) {
  extern __shared__ double2 lds[];
  __shared__ double nrm[kSMax];
  __shared__ int ord[kSMax];
  __shared__ int rotated;
  double2* Xs = lds;            // R, then R W: column j at j * ld, rows < r2
  double2* Ws = lds + ld * ld;  // W: column j at j * ld, rows < r
  const CNode& nd = nodes[blockIdx.x];
  const int n = nd.n, m = nd.m, r = res[blockIdx.x].r, r2 = res[blockIdx.x].r2;
  const double2* Rg = buf + nd.off[S_R];
  const double2* Q = buf + nd.off[S_Y];
  const double2* Q2 = buf + nd.off[S_T];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int e = t; e < r * r; e += 256) {
    const int i = e % r, j = e / r;
    Xs[j * ld + i] = i < r2 ? Rg[(size_t)j * nd.s + i] : make_double2(0.0, 0.0);
    Ws[j * ld + i] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int rp = r + (r & 1);  // a phantom column when r is odd
  const double tol = 2.220446049250313e-16 * fmax(1.0, (double)r2);
  const int slot = t >> 4, sl = t & 15;  // 16 pair slots of 16 lanes
  for (int sweep = 0; sweep < 60 && r > 1; ++sweep) {
    if (t == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < rp - 1; ++round) {
      for (int pi = slot; pi < rp / 2; pi += 16) {
        // circle method: column 0 fixed, the others rotate by one position per round
        int p, q;
        if (pi == 0) {
          p = 0;
          q = 1 + round;
        } else {
          p = 1 + (round + pi) % (rp - 1);
          q = 1 + (round - pi + rp - 1) % (rp - 1);
        }
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        if (q >= r) continue;
        double2* xp = Xs + p * ld;
        double2* xq = Xs + q * ld;
        double a = 0.0, b = 0.0, gr = 0.0, gi = 0.0;
        for (int i = sl; i < r2; i += 16) {
          const double2 u = xp[i], v = xq[i];
          a += znorm(u);
          b += znorm(v);
          gr += u.x * v.x + u.y * v.y;
          gi += u.x * v.y - u.y * v.x;
        }
        a = group16_sum(a);
        b = group16_sum(b);
        gr = group16_sum(gr);
        gi = group16_sum(gi);
        const double ag = sqrt(gr * gr + gi * gi);
        // orthogonal to working accuracy: the rounding of a length-r2 inner product
        if (ag == 0.0 || ag <= tol * sqrt(a * b)) continue;
        if (sl == 0) rotated = 1;
        // x_q' = conj(ph) x_q makes the inner product real; then a real rotation
        const double2 phc = make_double2(gr / ag, -gi / ag);
        const double zeta = (b - a) / (2.0 * ag);
        const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
        for (int i = sl; i < r2; i += 16) {
          const double2 u = xp[i], v = zmul(phc, xq[i]);
          xp[i] = zsub(zscale(u, c), zscale(v, sn));
          xq[i] = zadd(zscale(u, sn), zscale(v, c));
        }
        double2* wp = Ws + p * ld;
        double2* wq = Ws + q * ld;
        for (int i = sl; i < r; i += 16) {
          const double2 u = wp[i], v = zmul(phc, wq[i]);
          wp[i] = zsub(zscale(u, c), zscale(v, sn));
          wq[i] = zadd(zscale(u, sn), zscale(v, c));
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  for (int j = w; j < r; j += 4) {
    double a = 0.0;
    for (int i = lane; i < r2; i += 64) a += znorm(Xs[j * ld + i]);
    a = wave_sum(a);
    if (lane == 0) nrm[j] = sqrt(a);
  }
  __syncthreads();
  if (t < r) {  // descending order, ties by index
    int rank = 0;
    for (int l = 0; l < r; ++l) rank += (nrm[l] > nrm[t] || (nrm[l] == nrm[t] && l < t)) ? 1 : 0;
    ord[rank] = t;
  }
  __syncthreads();
  const double s_next = rmax < r ? nrm[ord[rmax]] : 0.0;
  const int ok = s_next < eps ? 1 : 0;
  int k = 0;
  while (k < r && k < rmax && nrm[ord[k]] >= eps) ++k;
  if (t == 0) {
    res[blockIdx.x].k = k;
    res[blockIdx.x].ok = ok;
  }
  if (!ok) return;
  double2* U = buf + nd.off[S_U];
  double2* Vt = buf + nd.off[S_V];
  // one thread per row, 16 ranks at a time: the basis entries load coalesced
  // across the workgroup, the rotation columns are LDS broadcasts
  for (int c0 = 0; c0 < k; c0 += 16) {
    const int kc = min(16, k - c0);
    for (int i = t; i < m; i += 256) {  // U = Q W(:, ord) diag(sigma)
      double2 a[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) a[c] = make_double2(0.0, 0.0);
      for (int j = 0; j < r; ++j) {
        const double2 q = Q[(size_t)j * m + i];
#pragma unroll
        for (int c = 0; c < 16; ++c)
          if (c < kc) a[c] = zadd(a[c], zmul(q, Ws[ord[c0 + c] * ld + j]));
      }
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c < kc) U[(size_t)i * k + c0 + c] = zscale(a[c], nrm[ord[c0 + c]]);
    }
    for (int i = t; i < n; i += 256) {  // V^T = conj(Q2 Z'(:, ord)), Z' = R W diag(sigma)^-1
      double2 a[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) a[c] = make_double2(0.0, 0.0);
      for (int j = 0; j < r2; ++j) {
        const double2 q = Q2[(size_t)j * n + i];
#pragma unroll
        for (int c = 0; c < 16; ++c)
          if (c < kc) a[c] = zadd(a[c], zmul(q, Xs[ord[c0 + c] * ld + j]));
      }
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c < kc) {
          const double inv = 1.0 / nrm[ord[c0 + c]];
          Vt[(size_t)i * k + c0 + c] = make_double2(a[c].x * inv, -a[c].y * inv);
        }
    }
  }
}

// Posterior check of a candidate leaf with the four probes w_p (slot P4) and
// M w_p (slot Y4): accepted iff ||M w_p - U (V w_p)|| <= eps ||w_p|| for all p.
__global__ __launch_bounds__(256) void plr_probe_kernel(const CNode* __restrict__ nodes, CRes* __restrict__ res,
                                                        const double2* __restrict__ buf, double eps) {
  __shared__ double2 tv[kPlrMaxRank][4];
  __shared__ double red[4];
  const CNode& nd = nodes[blockIdx.x];
  if (!res[blockIdx.x].ok) return;
  const int m = nd.m, n = nd.n, k = res[blockIdx.x].k;
  const double2* U = buf + nd.off[S_U];
  const double2* Vt = buf + nd.off[S_V];
  const double2* P4 = buf + nd.off[S_P4];
  const double2* Y4 = buf + nd.off[S_Y4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int e = w; e < 4 * k; e += 4) {  // tv[c][p] = (V w_p)_c
    const int c = e >> 2, p = e & 3;
    double re = 0.0, im = 0.0;
    for (int i = lane; i < n; i += 64) {
      const double2 v = zmul(Vt[(size_t)i * k + c], P4[(size_t)p * n + i]);
      re += v.x;
      im += v.y;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) tv[c][p] = make_double2(re, im);
  }
  __syncthreads();
  int good = 1;
  for (int p = 0; p < 4; ++p) {
    double en = 0.0, wn = 0.0;
    for (int i = t; i < m; i += 256) {
      double2 a = Y4[(size_t)p * m + i];
      for (int c = 0; c < k; ++c) a = zsub(a, zmul(U[(size_t)i * k + c], tv[c][p]));
      en += znorm(a);
    }
    for (int i = t; i < n; i += 256) wn += znorm(P4[(size_t)p * n + i]);
    en = block_sum(en, red);
    wn = block_sum(wn, red);
    if (!(sqrt(en) <= eps * sqrt(wn))) good = 0;
  }
  if (t == 0) res[blockIdx.x].ok = good;
}

// Copy accepted leaves into the packed data: a dense leaf from its block
// (row-major m x n), a low-rank one as U (m x k) then V^T (n x k) from staging.
__global__ __launch_bounds__(256) void plr_emit_kernel(const EmitRec* __restrict__ recs,
                                                       const double2* __restrict__ blocks, int N,
                                                       const double2* __restrict__ stage, double2* __restrict__ out) {
  const EmitRec& e = recs[blockIdx.x];
  if (e.k < 0) {
    const double2* M = blocks + (size_t)e.blk * N * N + (size_t)e.r0 * N + e.c0;
    for (int64_t x = threadIdx.x; x < (int64_t)e.m * e.n; x += blockDim.x)
      out[e.dst + x] = M[(size_t)(x / e.n) * N + x % e.n];
  } else {
    const int64_t nu = (int64_t)e.m * e.k, nv = (int64_t)e.n * e.k;
    for (int64_t x = threadIdx.x; x < nu; x += blockDim.x) out[e.dst + x] = stage[e.srcU + x];
    for (int64_t x = threadIdx.x; x < nv; x += blockDim.x) out[e.dst + nu + x] = stage[e.srcV + x];
  }
}

// Dense N x N expansion of one compressed block (one workgroup per leaf; the
// leaves tile the block, so every entry is written once).
__global__ __launch_bounds__(256) void plr_expand_kernel(const PlrBlockDev* __restrict__ B, int N,
                                                         double2* __restrict__ out) {
  const PlrLeafDev L = B->leaves[blockIdx.x];
  for (int64_t x = threadIdx.x; x < (int64_t)L.m * L.n; x += blockDim.x) {
    const int i = (int)(x / L.n), j = (int)(x % L.n);
    double2 v = make_double2(0.0, 0.0);
    if (L.k < 0) {
      v = B->data[L.offU + x];
    } else {
      for (int c = 0; c < L.k; ++c)
        v = zadd(v, zmul(B->data[L.offU + (int64_t)i * L.k + c], B->data[L.offV + (int64_t)j * L.k + c]));
    }
    out[(size_t)(L.r0 + i) * N + L.c0 + j] = v;
  }
}

// ----------------------------------------------------------------------------
// online apply
// ----------------------------------------------------------------------------
__device__ __forceinline__ double2* zbase(const Bases& b, int buf) {
  return buf == 0 ? b.b[0] : buf == 1 ? b.b[1] : buf == 2 ? b.b[2] : buf == 3 ? b.b[3] : nullptr;
}

// grid.x = njobs * ntiles (64-row tiles), grid.y = right-hand side; 4 waves.
// Every job term is a PLR block; wave w of NW takes the leaves w, w + NW, ...
// of the tile's leaf list; lane = output row.  The leaf's input columns (Q + beta S)
// are staged in LDS in chunks of kXs, shared by the wave.  A low-rank leaf
// forms t = V x with V stored column by column (n x k): lane l takes rank
// l % k of the columns congruent to l / k modulo 64 / k, so one load
// instruction reads 64 consecutive entries, and the 64 / k partial sums of a
// rank are added in order through LDS; then U[row] t.  A dense leaf adds
// D[row] x.  Wave partials are summed in a fixed order through LDS.
constexpr int kXs = 128;

template <int NW>
__global__ __launch_bounds__(64 * NW) void plr_apply_kernel(const Job* __restrict__ jobs, int n, int ntiles,
                                                            int64_t ld, Bases bases, double2* __restrict__ out_part) {
  __shared__ double2 part[NW][64];
  __shared__ double2 tb[NW][kPlrMaxRank];
  __shared__ double2 xs[NW][kXs];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tile = blockIdx.x % ntiles;
  const Job& J = jobs[blockIdx.x / ntiles];
  const int r = blockIdx.y;
  const int slices = gridDim.z, slice = blockIdx.z;  // slice z takes leaves z NW + w, step slices NW
  const int row = tile * 64 + lane;
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll 1
  for (int t = 0; t < 4; ++t) {
    if (t >= J.nterms) break;
    const PlrBlockDev* B = reinterpret_cast<const PlrBlockDev*>(J.M[t]);
    const VecRef qr = J.Q[t];
    const VecRef sr = J.S[t];
    const double2* qp = qr.buf >= 0 ? zbase(bases, qr.buf) + qr.off + (int64_t)r * ld : nullptr;
    const double2* sp = sr.buf >= 0 ? zbase(bases, sr.buf) + sr.off + (int64_t)r * ld : nullptr;
    const double2 be = J.beta[t];
    const int l0 = B->tile_ptr[tile], l1 = B->tile_ptr[tile + 1];
    for (int li = l0 + slice * NW + wave; li < l1; li += slices * NW) {
      const PlrLeafDev L = B->leaves[B->tile_leaf[li]];
      if (L.k == 0) continue;  // a zero leaf
      const bool in = row >= L.r0 && row < L.r0 + L.m;
      const bool lowrank = L.k > 0;
      const int G = lowrank ? 64 / L.k : 1;           // column groups of a rank
      const int jr = lowrank ? lane % L.k : 0, cg = lowrank ? lane / L.k : 0;
      const bool act = lowrank && cg < G;
      const double2* Dr = B->data + L.offU + (size_t)(in ? row - L.r0 : 0) * L.n;  // dense leaf row
      const double2* Vt = B->data + L.offV;                                       // n x k
      double2 s = make_double2(0.0, 0.0);
      for (int c0 = 0; c0 < L.n; c0 += kXs) {
        const int cn = min(kXs, L.n - c0);
        for (int c = lane; c < cn; c += 64) {
          double2 x = qp ? qp[L.c0 + c0 + c] : make_double2(0.0, 0.0);
          if (sp) x = zadd(x, zmul(be, sp[L.c0 + c0 + c]));
          xs[wave][c] = x;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        if (act) {
#pragma unroll 4
          for (int c = cg; c < cn; c += G) s = zadd(s, zmul(Vt[(size_t)(c0 + c) * L.k + jr], xs[wave][c]));
        } else if (!lowrank && in) {
#pragma unroll 4
          for (int c = 0; c < cn; ++c) acc = zadd(acc, zmul(Dr[c0 + c], xs[wave][c]));
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      }
      if (lowrank) {
        part[wave][lane] = act ? s : make_double2(0.0, 0.0);  // (part is free until the end)
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        if (lane < L.k) {
          double2 tj = make_double2(0.0, 0.0);
          for (int g = 0; g < G; ++g) tj = zadd(tj, part[wave][g * L.k + lane]);
          tb[wave][lane] = tj;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        if (in) {
          const double2* U = B->data + L.offU + (size_t)(row - L.r0) * L.k;
#pragma unroll 4
          for (int j = 0; j < L.k; ++j) acc = zadd(acc, zmul(U[j], tb[wave][j]));
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      }
    }
  }
  __syncthreads();  // every wave is done with its LDS rows before they hold the partials
  part[wave][lane] = acc;
  __syncthreads();
  if (wave == 0) {
    double2 s = part[0][lane];
#pragma unroll
    for (int w = 1; w < NW; ++w) s = zadd(s, part[w][lane]);
    if (slices > 1) {  // this slice's partial tile; plr_reduce_kernel finishes the rows
      out_part[(((size_t)r * gridDim.x + blockIdx.x) * slices + slice) * 64 + lane] = s;
    } else if (row < n) {
      double2 y = zmul(J.alpha, s);
      if (J.P.buf >= 0) y = zadd(y, zbase(bases, J.P.buf)[J.P.off + (int64_t)r * ld + row]);
      zbase(bases, J.Y.buf)[J.Y.off + (int64_t)r * ld + row] = y;
    }
  }
}

// Y = P + alpha * (sum over the slices of a tile's partials, in slice order);
// grid: (jobs x tiles, right-hand sides), one 64-lane wave per tile
__global__ __launch_bounds__(64) void plr_reduce_kernel(const Job* __restrict__ jobs, int n, int ntiles, int64_t ld,
                                                        Bases bases, int slices, const double2* __restrict__ part) {
  const int lane = threadIdx.x;
  const int tile = blockIdx.x % ntiles;
  const Job& J = jobs[blockIdx.x / ntiles];
  const int r = blockIdx.y;
  const int row = tile * 64 + lane;
  if (row >= n) return;
  const double2* p = part + ((size_t)r * gridDim.x + blockIdx.x) * slices * 64 + lane;
  double2 s = p[0];
  for (int z = 1; z < slices; ++z) s = zadd(s, p[(size_t)z * 64]);
  double2 y = zmul(J.alpha, s);
  if (J.P.buf >= 0) y = zadd(y, zbase(bases, J.P.buf)[J.P.off + (int64_t)r * ld + row]);
  zbase(bases, J.Y.buf)[J.Y.off + (int64_t)r * ld + row] = y;
}

}  // namespace

size_t PlrSet::stored_entries(int b) const { return stored[b]; }

namespace {

// device buffer that grows by doubling, keeping its contents (stream-ordered)
struct Grow {
  double2* p = nullptr;
  size_t cap = 0;
  hipError_t reserve(size_t want, hipStream_t st) {
    if (want <= cap) return hipSuccess;
    size_t nc = std::max<size_t>(want, 2 * cap);
    double2* q = nullptr;
    hipError_t e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&q, nc * sizeof(double2))) != hipSuccess) return e;
    if (cap && (e = hipMemcpyAsync(q, p, cap * sizeof(double2), hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (p) (void)hipFree(p);
    p = q;
    cap = nc;
    return hipSuccess;
  }
  ~Grow() {
    if (p) (void)hipFree(p);
  }
};

template <typename T>
struct Tmp {
  T* p = nullptr;
  size_t cap = 0;
  hipError_t fit(size_t want) {
    if (want <= cap) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc((void**)&p, std::max<size_t>(1, want) * sizeof(T));
    if (e == hipSuccess) cap = want;
    return e;
  }
  ~Tmp() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

hipError_t PlrSet::build(const double2* blocks, int nb, int N, int rmax, double eps, hipStream_t st) {
  release();
  this->n = N;
  if (rmax < 1 || rmax > kPlrMaxRank) return hipErrorInvalidValue;
  struct HN {
    int blk, r0, c0, m, n;
  };
  struct HLeaf {
    int blk, r0, c0, m, n, k;
    int64_t off;
  };
  std::vector<HLeaf> hleaves;
  std::vector<HN> cur;
  for (int b = 0; b < nb; ++b) cur.push_back({b, 0, 0, N, N});
  Grow data;
  size_t used = 0;
  Tmp<CNode> dnodes;
  Tmp<CRes> dres;
  Tmp<double2> stage;
  Tmp<EmitRec> drec;
  constexpr int64_t kStageCap = (int64_t)1 << 25;  // staging entries per batch of nodes (512 MiB)
  const uint64_t seed = 0x5EED5EEDull;
  hipError_t e;

  // copy a list of leaves into the packed data (appending) and record them
  auto emit = [&](std::vector<EmitRec>& recs) -> hipError_t {
    if (recs.empty()) return hipSuccess;
    size_t need = used;
    for (EmitRec& r : recs) {
      r.dst = (int64_t)need;
      need += r.k < 0 ? (size_t)r.m * r.n : (size_t)(r.m + r.n) * r.k;
      hleaves.push_back({r.blk, r.r0, r.c0, r.m, r.n, r.k, r.dst});
    }
    hipError_t er;
    if ((er = data.reserve(need, st)) != hipSuccess) return er;
    if ((er = drec.fit(recs.size())) != hipSuccess) return er;
    if ((er = hipMemcpyAsync(drec.p, recs.data(), recs.size() * sizeof(EmitRec), hipMemcpyHostToDevice, st)) !=
        hipSuccess)
      return er;
    hipLaunchKernelGGL(plr_emit_kernel, dim3((unsigned)recs.size()), dim3(256), 0, st, drec.p, blocks, N, stage.p,
                       data.p);
    if ((er = hipGetLastError()) != hipSuccess) return er;
    used = need;
    // the record list and the staging buffer are reused by the next batch
    return hipStreamSynchronize(st);
  };

  while (!cur.empty()) {
    std::vector<HN> work, next;
    std::vector<EmitRec> dense;
    for (const HN& h : cur) {
      if (std::min(h.m, h.n) <= rmax)
        dense.push_back({h.blk, h.r0, h.c0, h.m, h.n, -1, 0, 0, 0});
      else
        work.push_back(h);
    }
    if ((e = emit(dense)) != hipSuccess) return e;
    size_t w0 = 0;
    while (w0 < work.size()) {
      std::vector<CNode> cn;
      int64_t so = 0;
      int wide = 0, smax = 1;
      size_t w1 = w0;
      for (; w1 < work.size(); ++w1) {
        const HN& h = work[w1];
        const int s = std::min(std::min(std::min(h.m, h.n), rmax + 1 + 10), kSMax);
        const int64_t need = (int64_t)(3 * h.n + 2 * h.m) * s + (int64_t)s * s + 4 * (int64_t)(h.m + h.n);
        if (!cn.empty() && so + need > kStageCap) break;
        CNode c{};
        c.blk = h.blk;
        c.r0 = h.r0;
        c.c0 = h.c0;
        c.m = h.m;
        c.n = h.n;
        c.s = s;
        const int64_t sz[S_NSLOT] = {(int64_t)h.n * s, (int64_t)h.m * s, (int64_t)h.n * s, (int64_t)s * s,
                                     (int64_t)h.m * s, (int64_t)h.n * s, 4 * (int64_t)h.n, 4 * (int64_t)h.m};
        for (int q = 0; q < S_NSLOT; ++q) {
          c.off[q] = so;
          so += sz[q];
        }
        wide = std::max(wide, std::max(h.m, h.n));
        smax = std::max(smax, s);
        cn.push_back(c);
      }
      const int cnt = (int)cn.size();
      if ((e = dnodes.fit(cnt)) != hipSuccess || (e = dres.fit(cnt)) != hipSuccess || (e = stage.fit(so)) != hipSuccess)
        return e;
      if ((e = hipMemcpyAsync(dnodes.p, cn.data(), cnt * sizeof(CNode), hipMemcpyHostToDevice, st)) != hipSuccess)
        return e;
      const dim3 g1(cnt), gr(cnt, 8), gt(cnt, (wide + 63) / 64), b(256);
      // range finder with one power iteration, then the SVD of B = Q^H M
      hipLaunchKernelGGL(plr_random_kernel, gr, b, 0, st, dnodes.p, stage.p, (int)S_OM, 0, seed);
      hipLaunchKernelGGL(plr_panel_kernel<false>, gt, b, 0, st, dnodes.p, dres.p, blocks, N, stage.p, (int)S_OM,
                         (int)S_Y, 0);
      hipLaunchKernelGGL(plr_orth_kernel, g1, b, 0, st, dnodes.p, dres.p, stage.p, (int)S_Y, 0, 0, -1);
      hipLaunchKernelGGL(plr_panel_kernel<true>, gt, b, 0, st, dnodes.p, dres.p, blocks, N, stage.p, (int)S_Y,
                         (int)S_T, 1);
      hipLaunchKernelGGL(plr_panel_kernel<false>, gt, b, 0, st, dnodes.p, dres.p, blocks, N, stage.p, (int)S_T,
                         (int)S_Y, 1);
      hipLaunchKernelGGL(plr_orth_kernel, g1, b, 0, st, dnodes.p, dres.p, stage.p, (int)S_Y, 1, 0, -1);
      hipLaunchKernelGGL(plr_panel_kernel<true>, gt, b, 0, st, dnodes.p, dres.p, blocks, N, stage.p, (int)S_Y,
                         (int)S_T, 1);
      hipLaunchKernelGGL(plr_orth_kernel, g1, b, 0, st, dnodes.p, dres.p, stage.p, (int)S_T, 1, 1, (int)S_R);
      const size_t svd_lds = (size_t)2 * smax * smax * sizeof(double2);
      if (svd_lds > 65536 &&
          (e = hipFuncSetAttribute(reinterpret_cast<const void*>(&plr_svd_kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)svd_lds)) != hipSuccess)
        return e;
      hipLaunchKernelGGL(plr_svd_kernel, g1, b, svd_lds, st, dnodes.p, dres.p, stage.p, smax, rmax, eps);
      // posterior probes
      hipLaunchKernelGGL(plr_random_kernel, gr, b, 0, st, dnodes.p, stage.p, (int)S_P4, 1, seed ^ 0xA5A5A5A5ull);
      hipLaunchKernelGGL(plr_panel_kernel<false>, gt, b, 0, st, dnodes.p, dres.p, blocks, N, stage.p, (int)S_P4,
                         (int)S_Y4, 2);
      hipLaunchKernelGGL(plr_probe_kernel, g1, b, 0, st, dnodes.p, dres.p, stage.p, eps);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      std::vector<CRes> hr(cnt);
      if ((e = hipMemcpyAsync(hr.data(), dres.p, cnt * sizeof(CRes), hipMemcpyDeviceToHost, st)) != hipSuccess ||
          (e = hipStreamSynchronize(st)) != hipSuccess)
        return e;
      std::vector<EmitRec> acc;
      for (int i = 0; i < cnt; ++i) {
        const CNode& c = cn[i];
        if (hr[i].ok) {
          acc.push_back({c.blk, c.r0, c.c0, c.m, c.n, hr[i].k, c.off[S_U], c.off[S_V], 0});
        } else {
          const int m1 = (c.m + 1) / 2, n1 = (c.n + 1) / 2;
          next.push_back({c.blk, c.r0, c.c0, m1, n1});
          next.push_back({c.blk, c.r0, c.c0 + n1, m1, c.n - n1});
          next.push_back({c.blk, c.r0 + m1, c.c0, c.m - m1, n1});
          next.push_back({c.blk, c.r0 + m1, c.c0 + n1, c.m - m1, c.n - n1});
        }
      }
      if ((e = emit(acc)) != hipSuccess) return e;
      w0 = w1;
    }
    cur.swap(next);
  }

  // per block: leaves (in the order found), per-tile leaf lists
  const int ntile = (N + 63) / 64;
  std::vector<std::vector<int>> per(nb);
  for (size_t i = 0; i < hleaves.size(); ++i) per[hleaves[i].blk].push_back((int)i);
  std::vector<PlrLeafDev> hl;
  std::vector<int32_t> hptr, hlist;
  std::vector<PlrBlockDev> hb(nb);
  std::vector<size_t> leaf0(nb), ptr0(nb), list0(nb);
  stored.assign(nb, 0);
  nleaves.assign(nb, 0);
  for (int bb = 0; bb < nb; ++bb) {
    leaf0[bb] = hl.size();
    for (int i : per[bb]) {
      const HLeaf& lf = hleaves[i];
      PlrLeafDev d{};
      d.r0 = lf.r0;
      d.c0 = lf.c0;
      d.m = lf.m;
      d.n = lf.n;
      d.k = lf.k;
      d.offU = lf.off;
      d.offV = lf.k < 0 ? 0 : lf.off + (int64_t)lf.m * lf.k;
      stored[bb] += lf.k < 0 ? (size_t)lf.m * lf.n : (size_t)(lf.m + lf.n) * lf.k;
      hl.push_back(d);
    }
    nleaves[bb] = (int)per[bb].size();
    ptr0[bb] = hptr.size();
    list0[bb] = hlist.size();
    hptr.push_back(0);
    for (int t = 0; t < ntile; ++t) {
      const int a = t * 64, z = std::min(N, a + 64);
      for (int i = 0; i < (int)per[bb].size(); ++i) {
        const PlrLeafDev& lf = hl[leaf0[bb] + i];
        if (lf.r0 < z && lf.r0 + lf.m > a) hlist.push_back(i);
      }
      hptr.push_back((int32_t)(hlist.size() - list0[bb]));
    }
    nleaves_total += per[bb].size();
  }
  d_data = data.p;  // owned from here on
  data.p = nullptr;
  if ((e = hipMalloc((void**)&d_leaves, std::max<size_t>(1, hl.size()) * sizeof(PlrLeafDev))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&d_ptr, std::max<size_t>(1, hptr.size()) * sizeof(int32_t))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&d_list, std::max<size_t>(1, hlist.size()) * sizeof(int32_t))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&d_blocks, std::max(1, nb) * sizeof(PlrBlockDev))) != hipSuccess) return e;
  for (int bb = 0; bb < nb; ++bb) {
    hb[bb].nleaves = nleaves[bb];
    hb[bb].ntile = ntile;
    hb[bb].leaves = d_leaves + leaf0[bb];
    hb[bb].tile_ptr = d_ptr + ptr0[bb];
    hb[bb].tile_leaf = d_list + list0[bb];
    hb[bb].data = d_data;  // leaf offsets are global
  }
  if ((e = hipMemcpy(d_leaves, hl.data(), hl.size() * sizeof(PlrLeafDev), hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(d_ptr, hptr.data(), hptr.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(d_list, hlist.data(), hlist.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(d_blocks, hb.data(), nb * sizeof(PlrBlockDev), hipMemcpyHostToDevice)) != hipSuccess) return e;
  data_entries = used;
  return hipSuccess;
}

hipError_t PlrSet::expand(int b, double2* out, hipStream_t st) const {
  if (b < 0 || b >= (int)nleaves.size()) return hipErrorInvalidValue;
  if (nleaves[b] == 0) return hipSuccess;
  hipLaunchKernelGGL(plr_expand_kernel, dim3((unsigned)nleaves[b]), dim3(256), 0, st, d_blocks + b, n, out);
  return hipGetLastError();
}

hipError_t PlrSet::adopt(PlrSet& o) {
  if (o.stored.size() != stored.size() || !d_blocks || !o.d_blocks) return hipErrorInvalidValue;
  const size_t nb = stored.size();
  hipError_t e = hipMemcpy(d_blocks, o.d_blocks, nb * sizeof(PlrBlockDev), hipMemcpyDeviceToDevice);
  if (e != hipSuccess) return e;
  PlrBlockDev* keep = d_blocks;
  d_blocks = nullptr;
  release();  // the old leaves, tile lists and data (not the descriptor array)
  d_blocks = keep;
  n = o.n;
  d_leaves = o.d_leaves;
  d_ptr = o.d_ptr;
  d_list = o.d_list;
  d_data = o.d_data;
  data_entries = o.data_entries;
  nleaves_total = o.nleaves_total;
  stored = std::move(o.stored);
  nleaves = std::move(o.nleaves);
  (void)hipFree(o.d_blocks);
  o.d_leaves = nullptr;
  o.d_ptr = o.d_list = nullptr;
  o.d_data = nullptr;
  o.d_blocks = nullptr;
  o.release();
  return hipSuccess;
}

void PlrSet::release() {
  if (d_leaves) (void)hipFree(d_leaves);
  if (d_ptr) (void)hipFree(d_ptr);
  if (d_list) (void)hipFree(d_list);
  if (d_data) (void)hipFree(d_data);
  if (d_blocks) (void)hipFree(d_blocks);
  d_leaves = nullptr;
  d_ptr = d_list = nullptr;
  d_data = nullptr;
  d_blocks = nullptr;
  data_entries = 0;
  nleaves_total = 0;
  stored.clear();
  nleaves.clear();
}

hipError_t launch_plr_apply(const Job* jobs, int njobs, int n, int nrhs, int64_t ld, Bases bases, hipStream_t st,
                            hipEvent_t ev0, hipEvent_t ev1, double2* part, size_t part_n) {
  if (njobs <= 0) return hipSuccess;
  const int ntiles = (n + 63) / 64;
  const long tiles = (long)njobs * ntiles * nrhs;
  const dim3 grid((unsigned)njobs * ntiles, (unsigned)nrhs);
  if (tiles >= 512) {
    hipExtLaunchKernelGGL(plr_apply_kernel<4>, grid, dim3(256), 0, st, ev0, ev1, 0, jobs, n, ntiles, ld, bases,
                          nullptr);
    return hipGetLastError();
  }
  // few tiles (one source; a sweep step has four blocks): a tile's leaves are
  // spread over up to 16 four-wave workgroups, about 1024 in the launch
  int slices = (int)std::min<long>(16, (1024 + tiles - 1) / tiles);
  while (slices > 1 && (size_t)slices * tiles * 64 > part_n) --slices;
  if (!part || slices < 2) {  // no workspace: 16 waves of one workgroup share a tile's leaves
    hipExtLaunchKernelGGL(plr_apply_kernel<16>, grid, dim3(1024), 0, st, ev0, ev1, 0, jobs, n, ntiles, ld, bases,
                          nullptr);
    return hipGetLastError();
  }
  hipExtLaunchKernelGGL(plr_apply_kernel<4>, dim3(grid.x, grid.y, (unsigned)slices), dim3(256), 0, st, ev0, nullptr,
                        0, jobs, n, ntiles, ld, bases, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipExtLaunchKernelGGL(plr_reduce_kernel, grid, dim3(64), 0, st, nullptr, ev1, 0, jobs, n, ntiles, ld, bases, slices,
                        part);
  return hipGetLastError();
}

}  // namespace polar

namespace polar {

bool PlrSet::save(FILE* fp) const {
  const int64_t nb = (int64_t)stored.size();
  const int64_t ntile = (n + 63) / 64;
  std::vector<PlrBlockDev> hb(nb);
  if (nb && hipMemcpy(hb.data(), d_blocks, nb * sizeof(PlrBlockDev), hipMemcpyDeviceToHost) != hipSuccess)
    return false;
  std::vector<int64_t> offs(3 * nb);
  for (int64_t b = 0; b < nb; ++b) {
    offs[3 * b] = hb[b].leaves - d_leaves;
    offs[3 * b + 1] = hb[b].tile_ptr - d_ptr;
    offs[3 * b + 2] = hb[b].tile_leaf - d_list;
  }
  const int64_t nptr = nb * (ntile + 1);
  int64_t nlist = 0;
  if (nb) {
    int32_t last = 0;
    if (hipMemcpy(&last, d_ptr + offs[3 * (nb - 1) + 1] + ntile, sizeof(int32_t), hipMemcpyDeviceToHost) !=
        hipSuccess)
      return false;
    nlist = offs[3 * (nb - 1) + 2] + last;
  }
  const int64_t head[7] = {n, nb, ntile, (int64_t)nleaves_total, nptr, nlist, (int64_t)data_entries};
  std::vector<uint64_t> st(stored.begin(), stored.end());
  return rec_write_host(fp, head, 7, sizeof(int64_t)) && rec_write_host(fp, offs.data(), offs.size(), 8) &&
         rec_write_host(fp, nleaves.data(), nb, sizeof(int)) && rec_write_host(fp, st.data(), nb, 8) &&
         rec_write_device(fp, d_leaves, nleaves_total, sizeof(PlrLeafDev)) &&
         rec_write_device(fp, d_ptr, nptr, sizeof(int32_t)) && rec_write_device(fp, d_list, nlist, sizeof(int32_t)) &&
         rec_write_device(fp, d_data, data_entries, sizeof(double2));
}

bool PlrSet::load(FILE* fp) {
  release();
  int64_t head[7];
  if (!rec_read_host(fp, head, 7, sizeof(int64_t))) return false;
  const int64_t nb = head[1], ntile = head[2], nlv = head[3], nptr = head[4], nlist = head[5], nd = head[6];
  if (nb < 0 || ntile != (head[0] + 63) / 64 || nlv < 0 || nptr != nb * (ntile + 1) || nlist < 0 || nd < 0)
    return false;
  n = (int)head[0];
  std::vector<int64_t> offs(3 * nb);
  std::vector<uint64_t> st(nb);
  nleaves.assign(nb, 0);
  if (!rec_read_host(fp, offs.data(), offs.size(), 8) || !rec_read_host(fp, nleaves.data(), nb, sizeof(int)) ||
      !rec_read_host(fp, st.data(), nb, 8))
    return false;
  stored.assign(st.begin(), st.end());
  nleaves_total = (size_t)nlv;
  data_entries = (size_t)nd;
  if (hipMalloc((void**)&d_leaves, std::max<int64_t>(1, nlv) * sizeof(PlrLeafDev)) != hipSuccess ||
      hipMalloc((void**)&d_ptr, std::max<int64_t>(1, nptr) * sizeof(int32_t)) != hipSuccess ||
      hipMalloc((void**)&d_list, std::max<int64_t>(1, nlist) * sizeof(int32_t)) != hipSuccess ||
      hipMalloc((void**)&d_data, std::max<int64_t>(1, nd) * sizeof(double2)) != hipSuccess ||
      hipMalloc((void**)&d_blocks, std::max<int64_t>(1, nb) * sizeof(PlrBlockDev)) != hipSuccess)
    return false;
  if (!rec_read_device(fp, d_leaves, nlv, sizeof(PlrLeafDev)) || !rec_read_device(fp, d_ptr, nptr, 4) ||
      !rec_read_device(fp, d_list, nlist, 4) || !rec_read_device(fp, d_data, nd, sizeof(double2)))
    return false;
  std::vector<PlrBlockDev> hb(nb);
  for (int64_t b = 0; b < nb; ++b) {
    if (offs[3 * b] < 0 || offs[3 * b] + nleaves[b] > nlv || offs[3 * b + 1] < 0 ||
        offs[3 * b + 1] + ntile + 1 > nptr || offs[3 * b + 2] < 0 || offs[3 * b + 2] > nlist)
      return false;
    hb[b].nleaves = nleaves[b];
    hb[b].ntile = (int)ntile;
    hb[b].leaves = d_leaves + offs[3 * b];
    hb[b].tile_ptr = d_ptr + offs[3 * b + 1];
    hb[b].tile_leaf = d_list + offs[3 * b + 2];
    hb[b].data = d_data;
  }
  return nb == 0 || hipMemcpy(d_blocks, hb.data(), nb * sizeof(PlrBlockDev), hipMemcpyHostToDevice) == hipSuccess;
}

}  // namespace polar
