// Partitioned low-rank (PLR) trace blocks: compression at setup (host) and
// the online apply kernel (GPU).
//
// Compression follows the adaptive quadtree of the paper's Alg. 5: a block
// becomes a leaf when its (r_max+1)-th singular value is below eps (absolute),
// keeping the k <= r_max triplets with sigma >= eps; otherwise it is split
// into four (ceil/floor halves) and each quarter is compressed; a block whose
// smaller side is <= r_max is a dense leaf.  The singular values are those of
// a randomized sketch: Y = (M M^H) M Omega with r_max + 1 + 10 columns (one
// power iteration, re-orthonormalised), B = Q^H M, and a one-sided Jacobi SVD
// of B (accurate small singular values, unlike an eigen-solve of B B^H).  A
// candidate leaf is accepted only if four random probes see an error below
// eps.  The leaves are applied in the factored form y[rows] += U (V x[cols])
// of the paper's Alg. 6 / sparse-factorised product.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <thread>
#include <vector>

#include "plr.h"

namespace polar {

namespace {

using cplx = std::complex<double>;

// SplitMix64 (Steele, Lea, Flood 2014) -> two uniforms -> Box-Muller normal pair
struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed) {}
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  cplx normal() {
    const double u1 = uniform(), u2 = uniform();
    const double r = std::sqrt(-2.0 * std::log(u1));
    return cplx(r * std::cos(6.283185307179586 * u2), r * std::sin(6.283185307179586 * u2));
  }
};

// view of a sub-block of a row-major matrix
struct View {
  const cplx* p;
  int m, n, ld;
  cplx at(int i, int j) const { return p[(size_t)i * ld + j]; }
};

// orthonormalise the columns of Y (m x s, column-major) in place by modified
// Gram-Schmidt applied twice; returns the number of independent columns
int orthonormalise(std::vector<cplx>& Y, int m, int s) {
  int r = 0;
  for (int j = 0; j < s; ++j) {
    cplx* y = &Y[(size_t)j * m];
    double n0 = 0;
    for (int i = 0; i < m; ++i) n0 += std::norm(y[i]);
    n0 = std::sqrt(n0);
    for (int pass = 0; pass < 2; ++pass)
      for (int q = 0; q < r; ++q) {
        const cplx* u = &Y[(size_t)q * m];
        cplx d = 0;
        for (int i = 0; i < m; ++i) d += std::conj(u[i]) * y[i];
        for (int i = 0; i < m; ++i) y[i] -= d * u[i];
      }
    double nn = 0;
    for (int i = 0; i < m; ++i) nn += std::norm(y[i]);
    nn = std::sqrt(nn);
    if (nn <= 1e-14 * std::max(n0, 1e-300)) continue;  // dependent column: dropped
    cplx* dst = &Y[(size_t)r * m];
    for (int i = 0; i < m; ++i) dst[i] = y[i] / nn;
    ++r;
  }
  return r;
}

// One-sided (Hestenes) Jacobi SVD of the s x n matrix B (row-major): returns
// sigma (descending), W (s x s, column-major) and Z (n x s, column-major) with
// B = W diag(sigma) Z^H.  Works on X = B^H (n x s) whose columns are rotated
// until mutually orthogonal: X W = Z diag(sigma).
void jacobi_svd(const std::vector<cplx>& B, int s, int n, std::vector<double>& sig, std::vector<cplx>& W,
                std::vector<cplx>& Z) {
  std::vector<cplx> X((size_t)n * s);
  for (int j = 0; j < s; ++j)
    for (int i = 0; i < n; ++i) X[(size_t)j * n + i] = std::conj(B[(size_t)j * n + i]);
  W.assign((size_t)s * s, 0.0);
  for (int j = 0; j < s; ++j) W[(size_t)j * s + j] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < s - 1; ++p)
      for (int q = p + 1; q < s; ++q) {
        cplx* xp = &X[(size_t)p * n];
        cplx* xq = &X[(size_t)q * n];
        double a = 0, b = 0;
        cplx g = 0;
        for (int i = 0; i < n; ++i) {
          a += std::norm(xp[i]);
          b += std::norm(xq[i]);
          g += std::conj(xp[i]) * xq[i];
        }
        const double ag = std::abs(g);
        if (ag <= 1e-15 * std::sqrt(a * b) || ag == 0.0) continue;
        rotated = true;
        const cplx ph = g / ag;  // x_q' = conj(ph) x_q makes the inner product real
        const double zeta = (b - a) / (2.0 * ag);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int i = 0; i < n; ++i) {
          const cplx u = xp[i], v = std::conj(ph) * xq[i];
          xp[i] = c * u - sn * v;
          xq[i] = sn * u + c * v;
        }
        cplx* wp = &W[(size_t)p * s];
        cplx* wq = &W[(size_t)q * s];
        for (int i = 0; i < s; ++i) {
          const cplx u = wp[i], v = std::conj(ph) * wq[i];
          wp[i] = c * u - sn * v;
          wq[i] = sn * u + c * v;
        }
      }
    if (!rotated) break;
  }
  std::vector<int> ord(s);
  std::vector<double> nrm(s);
  for (int j = 0; j < s; ++j) {
    double a = 0;
    for (int i = 0; i < n; ++i) a += std::norm(X[(size_t)j * n + i]);
    nrm[j] = std::sqrt(a);
    ord[j] = j;
  }
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return nrm[x] > nrm[y]; });
  sig.resize(s);
  Z.assign((size_t)n * s, 0.0);
  std::vector<cplx> W2((size_t)s * s);
  for (int jj = 0; jj < s; ++jj) {
    const int j = ord[jj];
    sig[jj] = nrm[j];
    for (int i = 0; i < s; ++i) W2[(size_t)jj * s + i] = W[(size_t)j * s + i];
    if (nrm[j] > 0)
      for (int i = 0; i < n; ++i) Z[(size_t)jj * n + i] = X[(size_t)j * n + i] / nrm[j];
  }
  W.swap(W2);
}

struct HostLeaf {
  int r0, c0, m, n, k;  // k < 0: dense
  std::vector<cplx> U, V, D;
};

struct Compressor {
  int rmax;
  double eps;
  Rng rng;
  std::vector<HostLeaf> out;

  void dense(const View& M, int r0, int c0) {
    HostLeaf lf{r0, c0, M.m, M.n, -1, {}, {}, {}};
    lf.D.resize((size_t)M.m * M.n);
    for (int i = 0; i < M.m; ++i)
      for (int j = 0; j < M.n; ++j) lf.D[(size_t)i * M.n + j] = M.at(i, j);
    out.push_back(std::move(lf));
  }

  // y = M x (x length n) and y = M^H x (x length m)
  static void mv(const View& M, const cplx* x, cplx* y) {
    for (int i = 0; i < M.m; ++i) {
      cplx a = 0;
      for (int j = 0; j < M.n; ++j) a += M.at(i, j) * x[j];
      y[i] = a;
    }
  }
  static void mhv(const View& M, const cplx* x, cplx* y) {
    for (int j = 0; j < M.n; ++j) y[j] = 0;
    for (int i = 0; i < M.m; ++i)
      for (int j = 0; j < M.n; ++j) y[j] += std::conj(M.at(i, j)) * x[i];
  }

  bool try_leaf(const View& M, int r0, int c0) {
    const int m = M.m, n = M.n;
    const int s = std::min(std::min(m, n), rmax + 1 + 10);
    std::vector<cplx> Y((size_t)m * s), T((size_t)n * s), om(n);
    for (int j = 0; j < s; ++j) {
      for (int i = 0; i < n; ++i) om[i] = rng.normal();
      mv(M, om.data(), &Y[(size_t)j * m]);
    }
    int r = orthonormalise(Y, m, s);
    // one power iteration: Y = M (M^H Q)
    for (int j = 0; j < r; ++j) mhv(M, &Y[(size_t)j * m], &T[(size_t)j * n]);
    std::vector<cplx> Y2((size_t)m * r);
    for (int j = 0; j < r; ++j) mv(M, &T[(size_t)j * n], &Y2[(size_t)j * m]);
    r = orthonormalise(Y2, m, r);
    // B = Q^H M (r x n, row-major)
    std::vector<cplx> B((size_t)r * n);
    for (int j = 0; j < r; ++j) {
      mhv(M, &Y2[(size_t)j * m], &T[0]);  // row j of Q^H M is conj(M^H q_j)
      for (int i = 0; i < n; ++i) B[(size_t)j * n + i] = std::conj(T[i]);
    }
    std::vector<double> sig;
    std::vector<cplx> W, Z;
    jacobi_svd(B, r, n, sig, W, Z);
    const double s_next = rmax < r ? sig[rmax] : 0.0;
    if (!(s_next < eps)) return false;
    int k = 0;
    while (k < r && k < rmax && sig[k] >= eps) ++k;
    HostLeaf lf{r0, c0, m, n, k, {}, {}, {}};
    lf.U.assign((size_t)m * k, 0.0);  // U = Q W(:, :k) diag(sigma), row-major m x k
    for (int i = 0; i < m; ++i)
      for (int c = 0; c < k; ++c) {
        cplx a = 0;
        for (int j = 0; j < r; ++j) a += Y2[(size_t)j * m + i] * W[(size_t)c * r + j];
        lf.U[(size_t)i * k + c] = a * sig[c];
      }
    lf.V.assign((size_t)k * n, 0.0);  // V = Z(:, :k)^H, row-major k x n
    for (int c = 0; c < k; ++c)
      for (int i = 0; i < n; ++i) lf.V[(size_t)c * n + i] = std::conj(Z[(size_t)c * n + i]);
    // posterior check with random probes: ||(M - U V) w|| <= eps ||w||
    std::vector<cplx> w(n), y(m), t(k > 0 ? k : 1);
    for (int probe = 0; probe < 4; ++probe) {
      double wn = 0;
      for (int i = 0; i < n; ++i) {
        w[i] = rng.normal();
        wn += std::norm(w[i]);
      }
      mv(M, w.data(), y.data());
      for (int c = 0; c < k; ++c) {
        cplx a = 0;
        for (int i = 0; i < n; ++i) a += lf.V[(size_t)c * n + i] * w[i];
        t[c] = a;
      }
      double en = 0;
      for (int i = 0; i < m; ++i) {
        cplx a = y[i];
        for (int c = 0; c < k; ++c) a -= lf.U[(size_t)i * k + c] * t[c];
        en += std::norm(a);
      }
      if (std::sqrt(en) > eps * std::sqrt(wn)) return false;
    }
    out.push_back(std::move(lf));
    return true;
  }

  void compress(const View& M, int r0, int c0) {
    if (std::min(M.m, M.n) <= rmax) {
      dense(M, r0, c0);
      return;
    }
    if (try_leaf(M, r0, c0)) return;
    const int m1 = (M.m + 1) / 2, n1 = (M.n + 1) / 2;
    compress(View{M.p, m1, n1, M.ld}, r0, c0);
    compress(View{M.p + n1, m1, M.n - n1, M.ld}, r0, c0 + n1);
    compress(View{M.p + (size_t)m1 * M.ld, M.m - m1, n1, M.ld}, r0 + m1, c0);
    compress(View{M.p + (size_t)m1 * M.ld + n1, M.m - m1, M.n - n1, M.ld}, r0 + m1, c0 + n1);
  }
};

// ----------------------------------------------------------------------------
// online apply
// ----------------------------------------------------------------------------
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
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
                                                            int64_t ld, Bases bases) {
  __shared__ double2 part[NW][64];
  __shared__ double2 tb[NW][kPlrMaxRank];
  __shared__ double2 xs[NW][kXs];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tile = blockIdx.x % ntiles;
  const Job& J = jobs[blockIdx.x / ntiles];
  const int r = blockIdx.y;
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
    for (int li = l0 + wave; li < l1; li += NW) {
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
  if (wave == 0 && row < n) {
    double2 s = part[0][lane];
#pragma unroll
    for (int w = 1; w < NW; ++w) s = zadd(s, part[w][lane]);
    double2 y = zmul(J.alpha, s);
    if (J.P.buf >= 0) y = zadd(y, zbase(bases, J.P.buf)[J.P.off + (int64_t)r * ld + row]);
    zbase(bases, J.Y.buf)[J.Y.off + (int64_t)r * ld + row] = y;
  }
}

}  // namespace

size_t PlrSet::stored_entries(int b) const { return stored[b]; }

hipError_t PlrSet::build(const std::vector<const std::complex<double>*>& blocks, int n, int rmax, double eps,
                         int nthreads) {
  release();
  this->n = n;
  const int nb = (int)blocks.size();
  std::vector<std::vector<HostLeaf>> res(nb);
  std::vector<std::thread> th;
  const int T = std::max(1, std::min(nthreads, nb));
  for (int w = 0; w < T; ++w)
    th.emplace_back([&, w]() {
      for (int b = w; b < nb; b += T) {
        Compressor c{rmax, eps, Rng(0x5EED0000ull + (uint64_t)b), {}};
        c.compress(View{reinterpret_cast<const cplx*>(blocks[b]), n, n, n}, 0, 0);
        res[b] = std::move(c.out);
      }
    });
  for (auto& t : th) t.join();

  // flatten: per block, leaves + per-tile leaf lists + data
  const int ntile = (n + 63) / 64;
  std::vector<PlrLeafDev> hl;
  std::vector<int32_t> hptr, hlist;
  std::vector<cplx> hdata;
  std::vector<PlrBlockDev> hb(nb);
  std::vector<size_t> leaf0(nb), ptr0(nb), list0(nb), data0(nb);
  stored.assign(nb, 0);
  for (int b = 0; b < nb; ++b) {
    leaf0[b] = hl.size();
    data0[b] = hdata.size();
    for (const HostLeaf& lf : res[b]) {
      PlrLeafDev d{};
      d.r0 = lf.r0;
      d.c0 = lf.c0;
      d.m = lf.m;
      d.n = lf.n;
      d.k = lf.k;
      if (lf.k < 0) {
        d.offU = (int64_t)(hdata.size() - data0[b]);
        hdata.insert(hdata.end(), lf.D.begin(), lf.D.end());
        stored[b] += lf.D.size();
      } else {
        d.offU = (int64_t)(hdata.size() - data0[b]);
        hdata.insert(hdata.end(), lf.U.begin(), lf.U.end());
        // V stored transposed (n x k): the apply reads one column's k values per step
        d.offV = (int64_t)(hdata.size() - data0[b]);
        for (int i = 0; i < lf.n; ++i)
          for (int c = 0; c < lf.k; ++c) hdata.push_back(lf.V[(size_t)c * lf.n + i]);
        stored[b] += lf.U.size() + lf.V.size();
      }
      hl.push_back(d);
    }
    ptr0[b] = hptr.size();
    list0[b] = hlist.size();
    hptr.push_back(0);
    for (int t = 0; t < ntile; ++t) {
      const int a = t * 64, e = std::min(n, a + 64);
      for (int i = 0; i < (int)res[b].size(); ++i) {
        const HostLeaf& lf = res[b][i];
        if (lf.r0 < e && lf.r0 + lf.m > a) hlist.push_back(i);
      }
      hptr.push_back((int32_t)(hlist.size() - list0[b]));
    }
    nleaves_total += res[b].size();
  }
  hipError_t e;
  if ((e = hipMalloc((void**)&d_leaves, std::max<size_t>(1, hl.size()) * sizeof(PlrLeafDev))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&d_ptr, std::max<size_t>(1, hptr.size()) * sizeof(int32_t))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&d_list, std::max<size_t>(1, hlist.size()) * sizeof(int32_t))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&d_data, std::max<size_t>(1, hdata.size()) * sizeof(double2))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&d_blocks, std::max(1, nb) * sizeof(PlrBlockDev))) != hipSuccess) return e;
  for (int b = 0; b < nb; ++b) {
    hb[b].nleaves = (int)res[b].size();
    hb[b].ntile = ntile;
    hb[b].leaves = d_leaves + leaf0[b];
    hb[b].tile_ptr = d_ptr + ptr0[b];
    hb[b].tile_leaf = d_list + list0[b];
    hb[b].data = d_data + data0[b];
  }
  if ((e = hipMemcpy(d_leaves, hl.data(), hl.size() * sizeof(PlrLeafDev), hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(d_ptr, hptr.data(), hptr.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(d_list, hlist.data(), hlist.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(d_data, hdata.data(), hdata.size() * sizeof(double2), hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(d_blocks, hb.data(), nb * sizeof(PlrBlockDev), hipMemcpyHostToDevice)) != hipSuccess) return e;
  data_entries = hdata.size();
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
}

hipError_t launch_plr_apply(const Job* jobs, int njobs, int n, int nrhs, int64_t ld, Bases bases, hipStream_t st,
                            hipEvent_t ev0, hipEvent_t ev1) {
  if (njobs <= 0) return hipSuccess;
  const int ntiles = (n + 63) / 64;
  // few workgroups (one source, a sweep step's four blocks): 16 waves share a tile's leaves
  if ((long)njobs * ntiles * nrhs < 512)
    hipExtLaunchKernelGGL(plr_apply_kernel<16>, dim3((unsigned)njobs * ntiles, (unsigned)nrhs), dim3(1024), 0, st, ev0,
                          ev1, 0, jobs, n, ntiles, ld, bases);
  else
    hipExtLaunchKernelGGL(plr_apply_kernel<4>, dim3((unsigned)njobs * ntiles, (unsigned)nrhs), dim3(256), 0, st, ev0,
                          ev1, 0, jobs, n, ntiles, ld, bases);
  return hipGetLastError();
}

}  // namespace polar
