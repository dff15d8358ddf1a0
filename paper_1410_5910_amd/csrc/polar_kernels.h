// Internal interface between the host orchestration (solver.hip) and the
// HIP kernels (kernels.hip) of libpolar.  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace polar {

// A reference to a complex float64 vector inside one of the four base buffers
// a launch receives: element (row i, right-hand side r) lives at
// base[buf] + off + r * ld + i.  buf < 0 means "absent".
struct VecRef {
  int32_t buf;
  int32_t pad;
  int64_t off;
};

// One output block of a batched block apply:
//   Y = P + alpha * sum_t M_t (Q_t + beta_t S_t)
// Each M_t is an n x n row-major matrix (complex float64 or complex float32),
// every vector has n rows and nrhs columns with the launch's column stride.
// A wide term (kw[t] > 0, float64 streaming and MFMA forms only) has an
// n x kw[t] matrix with row stride ldm[t] (0: kw[t]) and inputs of kw[t] rows.
struct Job {
  const void* M[4];
  VecRef Q[4];
  VecRef S[4];
  double2 beta[4];
  VecRef P;
  VecRef Y;
  double2 alpha;
  int32_t nterms;
  int32_t pad;
  int32_t kw[4];   // columns of M_t (0: n)
  int32_t ldm[4];  // row stride of M_t in entries (0: its column count)
  // float64 MFMA form: the column chunks (kNzChunk columns each) of term 0
  // whose inputs are not all zero, kl[0] = their count (at most kKlMax) and
  // kl[1..kl[0]] their indices in ascending order; the others add exact zeros
  // and are skipped (null: every chunk).  The other forms read every chunk.
  const int32_t* kl;
};

constexpr int kNzChunk = 16;
constexpr int kKlMax = 512;  // longest chunk list: terms of at most kKlMax * kNzChunk columns

struct Bases {
  double2* b[4];
};

// Launch geometry of one block-apply launch (host-computed).
constexpr int kMfmaSlicesMax = 8;  // most MFMA k-slices over workgroups

struct ApplyGeom {
  int n;        // block size NX
  int ntiles;   // row tiles per job: ceil(n / 8) for nr <= 4 (one row per wave), ceil(n / 64) otherwise
  int kc;       // columns staged in LDS per chunk
  int nr;       // right-hand sides per workgroup (template width)
  int mfma;     // float64 with more than 4 right-hand sides: MFMA kernel with this many
                // right-hand sides per workgroup tile (16, 32 or 64); 0: not used
  int gemv;     // 1: the row-streaming kernel (nr <= 4 right-hand sides per pass)
  int ks;       // float64 MFMA: wave groups splitting a tile's chunks (0: rule)
  int mks;      // MFMA: workgroups splitting a tile's chunks (k-slices; 0 or 1: none)
  int steps;    // streaming form: most (term, column chunk) steps of a job in the launch
};

// Shape override of a split-bfloat16 launch (0: rule).
struct SplitCfg {
  int tile_rhs;    // 32 or 64 right-hand sides per tile (more than 16 right-hand sides)
  int kslices;     // k-slices per tile
  int stream = 0;  // > 16 right-hand sides, every job two terms with Q: the branch-free
                   // two-chunks-in-flight form, 1 without S terms, 2 with (0: general form)
  int f16 = 0;     // planes and MFMA in float16 (1) or bfloat16 (0)
};

// One block-apply launch over up to NS segments: the job lists of several
// problems, each with its own block size n, right-hand sides, vector stride
// and base buffers, placed one after another along the grid's x dimension
// (blocks blk0[s] .. blk0[s+1]-1 serve segment s).  a0/a1 hold the
// per-segment tile counts of the kernel the table is built for.  Passed by
// value: a kernel reads the fields of its segment straight from its
// arguments.  Launches of one problem use NS = 1 (a small argument block, no
// segment search) and also pass their job list as a separate restrict-
// qualified argument, whose workgroup-uniform fields the compiler then reads
// with scalar loads; merged launches use NS = kMaxSeg.
constexpr int kMaxSeg = 8;
template <int NS>
struct SegTableT {
  int32_t nseg;
  int32_t blk0[NS + 1];
  int32_t n[NS];
  int32_t nrhs[NS];
  int32_t njobs[NS];
  int32_t a0[NS];
  int32_t a1[NS];
  int64_t ld[NS];
  const Job* jobs[NS];
  Bases bases[NS];
  float2* part[NS];  // split forms: k-slice partial tiles of the segment
};

// The segment of x block `bid` (blk0 ascending, blk0[0] = 0) and the block's
// index inside it.
template <int NS>
__device__ __forceinline__ int seg_of(const SegTableT<NS>& T, int& bid) {
  if constexpr (NS == 1) {
    return 0;
  } else {
    int s = 0;
    for (int i = 1; i < T.nseg; ++i)
      if (bid >= T.blk0[i]) s = i;
    bid -= T.blk0[s];
    return s;
  }
}

// Host description of one segment of a merged launch.
struct ApplySeg {
  const Job* jobs;
  int njobs;
  int n;
  int nrhs;
  int64_t ld;
  Bases bases;
  float2* part;  // split forms: k-slice workspace of the segment (null: none)
  size_t part_n; // its size in complex floats
};

// ---------------------------------------------------------------- block apply
// ev0/ev1 (may be null): events stamped with the kernel's own start and end.
// mpart (mpart_n complex doubles, may be null): workspace of MFMA k-slices
// (g.mks > 1), used only when it holds every slice's partial tiles.
hipError_t launch_block_apply(const Job* jobs, int njobs, const ApplyGeom& g, int nrhs, int64_t ld,
                              Bases bases, bool f32, hipStream_t st, hipEvent_t ev0 = nullptr,
                              hipEvent_t ev1 = nullptr, double2* mpart = nullptr, size_t mpart_n = 0);
// The same over nseg <= kMaxSeg segments in one launch (float64 or float32
// blocks).  The kernel form follows from the segments together: the
// row-streaming kernel when every segment has at most 4 right-hand sides
// (nr: the widest), otherwise the MFMA form (float64 or float32 blocks) with
// tiles chosen for the launch's total size.  Every
// segment's job arithmetic is that of a launch of the same form on its own.
hipError_t launch_block_apply_segs(const ApplySeg* segs, int nseg, int maxterms, bool wide, bool f32,
                                   hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Split-bfloat16 block apply (split.hip): the same job semantics as
// launch_block_apply, with every M_t pointing at the split planes of a block
// written by launch_split_planes.  part (may be null): workspace of
// split_kslices(njobs, n, nrhs) * njobs * nrhs * n complex floats for partial
// tiles of launches too small to fill the chip.
hipError_t launch_block_apply_split(const Job* jobs, int njobs, int n, int nrhs, int64_t ld, Bases bases,
                                    hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                                    float2* part = nullptr, SplitCfg cfg = SplitCfg{0, 0});
// The split block apply over nseg <= kMaxSeg segments in one launch: the
// rule's tile shape and k-slice count for the launch's total size (k-slices
// only when every segment's workspace holds its partial tiles).
hipError_t launch_block_apply_split_segs(const ApplySeg* segs, int nseg, int f16, hipStream_t st,
                                         hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Interface Green's function rows of one layer from its extraction solve:
// G[x'][(r - r0) NX + x] = W[(q NX + x') ld + r NX + x] * s(j, x') / s(r, x)
// for r in [r0, r0 + nrows), with s(r, x) = ax[x] az[r] the diagonal that
// makes the local operator symmetric (A = diag(s) A_sym): the rows of the
// inverse follow from its columns at the trace row j (solve column block q).
hipError_t launch_pack_green(const double2* W, int64_t ld, int q, int j, int r0, int nrows, int NX,
                             const double2* ax, const double2* az, double2* G, hipStream_t st);
// W[c][dst[e]] = sum_{s < cnt[e]} W[c][src0[e] + s] for entries e < nentries and columns c < ncols
// (rows of NX complex entries, column stride ld; the rows summed in order)
hipError_t launch_sum_rows(double2* W, int64_t ld, int NX, const int32_t* dst, const int32_t* src0,
                           const int32_t* cnt, int nentries, int ncols, hipStream_t st);
// list[e * stride] = number of kNzChunk-entry chunks of input e with an entry
// that is not zero (NaN and Inf count as not zero) in any of ncols columns,
// list[e * stride + 1 ..] = their indices in ascending order; input e holds
// entries off[e] .. off[e] + kk[e] - 1 of each column (stride ld) of B.
// stride >= 1 + ceil(kk[e] / kNzChunk) for every e.
hipError_t launch_nonzero_chunks(const double2* B, int64_t ld, int ncols, const int64_t* off, const int32_t* kk,
                                 int nentries, int32_t* list, int stride, hipStream_t st);
// Zeroes the extrapolation rows of polarized vectors (nrhs, 2, L-1, 2, NX),
// column stride ntrace: row n+1 of every down pair and row 0 of every up pair.
hipError_t launch_zero_extrap_rows(double2* v, int L, int NX, int64_t ntrace, int nrhs, hipStream_t st);
// Forced right-hand-side rows of an in-place reconstruction: for entries e <
// ne and right-hand sides r < nrhs, row dst[e] of T = h2 f(row src[e]) (0 if
// src[e] < 0) + sign[e] (x + x[half])(segment seg[e]); T and f have column
// stride ld, x column stride ntrace; rows of NX entries.
hipError_t launch_rec_rhs(double2* T, const double2* f, const double2* x, const int32_t* dst, const int32_t* src,
                          const int32_t* seg, const double* sign, int ne, int NX, int64_t ld, int64_t ntrace,
                          int64_t half, double h2, int nrhs, hipStream_t st);
// the rule's k-slice count of a split launch with the given tile width (0: the rule's width)
int split_kslices(int njobs, int n, int nrhs, int tile_rhs = 0);
// bfloat16 elements of the split planes of one n x n block
size_t split_block_elems(int n);
// nblk row-major complex float64 n x n blocks -> their split planes (dst: nblk * split_block_elems(n)
// 16-bit elements): bfloat16 (f16 = 0), or float16 of the entries times `scale` (a power of two)
hipError_t launch_split_planes(const double2* src, void* dst, int nblk, int n, hipStream_t st, int f16 = 0,
                               double scale = 1.0);
// the factor the float16 form multiplies its inputs by as it splits them (1 for bfloat16)
double split_input_scale(int f16);

// ---------------------------------------------------------- setup kernels
// Per-layer Gauss-Jordan inversion with partial pivoting of nb dense n x n
// column-major matrices.  One call performs elimination step k on every
// matrix: reads A[b], writes B[b], records perm[b*n + k], raises *flag on a
// zero pivot.
// blocked Gauss-Jordan: the steps k0 .. k0+bw-1 on the panel columns (in place), then every other column
// through the same steps, out of place (A -> B); bw <= gj_panel_width(), n <= 4096
hipError_t launch_gj_panel(double2* const* A, int nb, int n, int k0, int bw, int32_t* perm, int32_t* flag,
                           hipStream_t st);
hipError_t launch_gj_update(double2* const* A, double2* const* B, int nb, int n, int k0, int bw, const int32_t* perm,
                            hipStream_t st);
int gj_panel_width();
// Composes the column un-scrambling permutation of each matrix (pi[b*n + c]).
hipError_t launch_gj_perm(const int32_t* perm, int32_t* pi, int nb, int n, hipStream_t st);

// Delta_0 = tridiag(A_0) for nb layers: out[b] = west/east couplings + diag[b].
hipError_t launch_init_delta(double2* const* out, const double2* const* diag, const double2* west,
                             const double2* east, int nb, int n, hipStream_t st);

// Finishes local row r of nb layers: Dinv = B[:, pi] (stored row-major, where
// dinv64[b] != nullptr), and if next_diag[b] != nullptr also writes the next Schur complement
// Delta_{r+1} = tridiag(A_{r+1}) - coef[b] * Dinv into nextD[b].
hipError_t launch_finish_row(double2* const* B, const int32_t* pi, double2* const* dinv64, double2* const* nextD,
                             const double2* const* next_diag, const double2* coef, const double2* west,
                             const double2* east, int nb, int n, hipStream_t st);

// Middle Schur complement of a two-ended elimination: G[b] += Y[b] - tridiag(diag[b]),
// where G[b] and Y[b] (column-major) each hold tridiag(A_m) minus one side's term.
hipError_t launch_twist_combine(double2* const* G, const double2* const* Y, const double2* const* diag,
                                const double2* west, const double2* east, int nb, int n, hipStream_t st);

// --------------------------------------------------------- field kernels
// Local fields: (nrhs, sumR, NX); volume fields: (nrhs, NZ, NX).
// rowmap[g] for local row g in 0..sumR-1: the padded-grid row it copies from
// (owned rows) or -1 (extension rows).
hipError_t launch_scatter_source(const double2* f, double2* W, const int32_t* rowmap, int sumR, int NZ,
                                 int NX, int nrhs, double scale, hipStream_t st);
// u[own rows] = W[rows with rowmap >= 0]
hipError_t launch_gather_owned(const double2* W, double2* u, const int32_t* rowmap, int sumR, int NZ,
                               int NX, int nrhs, hipStream_t st);
// Sources that touch only some layers (the pre-solve needs only those layers):
// amax[r * L + l] = max |f[r]|^2 over rows own_start[l] .. own_start[l] + n_own[l] - 1.
hipError_t launch_source_activity(const double2* f, double* amax, const int32_t* own_start, const int32_t* n_own,
                                  int L, int NZ, int NX, int nrhs, hipStream_t st);
// W (m, sumR, NX): column slot j of the rows of layer l = scale * f[slot_rhs[l * m + j]] (zero for -1)
hipError_t launch_scatter_slots(const double2* f, double2* W, const int32_t* rowmap, const int32_t* row_layer,
                                const int32_t* slot_rhs, int m, int sumR, int NZ, int NX, double scale,
                                hipStream_t st);
// s[r][seg[i]] = W[rhs_slot[r * L + layer of row[i]]][row[i]] (zero for -1), for nmap entries
hipError_t launch_gather_slots(const double2* W, double2* s, const int32_t* seg, const int32_t* row,
                               const int32_t* row_layer, const int32_t* rhs_slot, int nmap, int L, int sumR, int NX,
                               int64_t ntrace, int nrhs, hipStream_t st);
// Trace exchange: for each of nmap (trace segment, local row, sign) triples:
// mode 0: s[seg] = W[row]              (trace right-hand side)
// mode 1: W[row] += sign * (x_d[seg] + x_a[seg])  (interface forcing)
hipError_t launch_trace_map(double2* W, double2* s, const double2* x, const int32_t* seg,
                            const int32_t* row, const double* sign, int nmap, int mode, int sumR,
                            int NX, int64_t ntrace, int nrhs, int64_t half, hipStream_t st);

// Extraction right-hand sides: W = 0 except W[c + q*n, row_q, c] = 1 for the
// nq source rows row_q (local rows of one layer, offset already applied).
hipError_t launch_identity_rhs(double2* W, const int32_t* rows, int nq, int n, int64_t ld, hipStream_t st);

// Copy with optional scale/identity shift of one n x n block out of a local
// field with nrhs = nq*n columns: dst(i, c) = sign * W[c + q*n, row, i] + shift*(i==c),
// stored row-major.
// C = alpha A (B + shift I), row-major complex n x n (setup)
hipError_t launch_setup_gemm(const double2* A, const double2* B, double2* C, int n, double2 alpha, double shift,
                             hipStream_t st);
// dst = sign src + shift I, row-major complex n x n
hipError_t launch_sign_copy(const double2* src, double2* dst, int n, double sign, double shift, hipStream_t st);
hipError_t launch_pack_block(const double2* W, int64_t ld, int q, int row, int n, double sign,
                             double shift, double2* dst64, float2* dst32, hipStream_t st);

// ---------------------------------------------------------- vector kernels
hipError_t launch_copy(double2* dst, const double2* src, int64_t n, hipStream_t st);
hipError_t launch_zero(double2* dst, int64_t n, hipStream_t st);
// y[e] = x[e] + sign * z[e]
hipError_t launch_add(double2* y, const double2* x, const double2* z, double sign, int64_t n, hipStream_t st);

// ---------------------------------------------------------- Krylov kernels
// Basis vectors are (nrhs, N) blocks, basis i at V + i * nrhs * N.
// hout[i * nrhs + r] = <V_i[r], w[r]> = sum conj(V_i[r]) w[r], i < m
hipError_t launch_kdot(const double2* V, const double2* w, double2* hout, int m, int nrhs, int64_t N,
                       hipStream_t st);
// w[r] -= sum_i h[i * nrhs + r] V_i[r]; hacc[i * nrhs + r] += h[...]
hipError_t launch_kupdate(const double2* V, double2* w, const double2* h, double2* hacc, int m, int nrhs,
                          int64_t N, hipStream_t st);
// nrm[r] = ||w[r]||_2
hipError_t launch_knorm(const double2* w, double* nrm, int nrhs, int64_t N, hipStream_t st);
// v[r] *= nrm[r] for each of the nrhs vectors of length N
hipError_t launch_kmulnorm(double2* v, const double* nrm, int nrhs, int64_t N, hipStream_t st);
// v[r] = w[r] / nrm[r] (zero if nrm == 0)
hipError_t launch_kscale(double2* v, const double2* w, const double* nrm, int nrhs, int64_t N,
                         hipStream_t st);
// Per right-hand side: Hessenberg column j from hacc (j+1 entries) and nrm, the
// previous Givens rotations, a new rotation, the rotated residual vector g and
// the residual estimate |g[j+1]| / beta.  State arrays are per-RHS strided by mdim.
hipError_t launch_givens(double2* Hc, const double2* hacc, const double* nrm, double* cs, double2* sn,
                         double2* g, double* est, const double* beta, int32_t* iters, int32_t* done,
                         double tol, int j, int mdim, int nrhs, hipStream_t st);
// y = H(0:k,0:k)^{-1} g(0:k) per RHS with k = iters[r]
hipError_t launch_ksolve(const double2* Hc, const double2* g, double2* y, const int32_t* iters, int mdim,
                         int nrhs, hipStream_t st);
// x[r] = sum_{j < iters[r]} y[r*mdim + j] Z_j[r]
hipError_t launch_kcombine(const double2* Z, const double2* y, const int32_t* iters, double2* x, int mdim,
                           int nrhs, int64_t N, hipStream_t st);

// g[r] = (beta[r], 0, ...), done[r] = (beta[r] == 0), iters[r] = 0, est[r] = 1 (0 if beta == 0)
hipError_t launch_kinit(double2* g, const double* beta, int32_t* done, int32_t* iters, double* est, int mdim,
                        int nrhs, hipStream_t st);
// d = (complex float32) s
hipError_t launch_to_f32(float2* d, const double2* s, int64_t n, hipStream_t st);

}  // namespace polar
