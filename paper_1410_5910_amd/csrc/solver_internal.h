// Internal state of a libpolar solver, shared by the host translation units
// (solver.hip, learned.hip).  Not part of the public C-ABI.
#pragma once

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "../../include/polar.h"
#include "plr.h"
#include "polar_kernels.h"

using namespace polar;

namespace polar_impl {

inline thread_local std::string g_err;

inline pt_status fail(pt_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(PT_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// GPU(S, expr): expr issued on S's stream (written st_ in expr), or recorded
#define GPU(S, expr)                                                                                        \
  do {                                                                                                      \
    pt_status g_ = gpu_op((S)->rec, (S)->st, #expr, [=](hipStream_t st_) -> hipError_t { return expr; }); \
    if (g_ != PT_OK) return g_;                                                                             \
  } while (0)

#define PTCHK(expr)               \
  do {                            \
    pt_status s_ = (expr);        \
    if (s_ != PT_OK) return s_;   \
  } while (0)

struct cd {
  double re, im;
};
inline cd cmk(double r, double i) { return {r, i}; }
inline cd operator*(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline cd operator+(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
inline cd operator-(cd a) { return {-a.re, -a.im}; }
inline double2 d2(cd a) { return make_double2(a.re, a.im); }
inline double2 cdiv_h(cd a, cd b) {  // a / b on the host
  const double den = b.re * b.re + b.im * b.im;
  return make_double2((a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den);
}

// alpha = 1 / (1 + i sigma / omega), sigma = (C/delta)(d/delta)^2
inline cd pml_alpha(double d_len, double C, double delta, double omega) {
  const double s = d_len > 0.0 ? (C / delta) * (d_len / delta) * (d_len / delta) : 0.0;
  const double t = s / omega;  // 1/(1 + i t) = (1 - i t)/(1 + t^2)
  return {1.0 / (1.0 + t * t), -t / (1.0 + t * t)};
}

// distance (in units of h) of a grid position beyond the physical segment [0, n+1]
inline double beyond(double pos, int n) { return std::max(0.0, std::max(-pos, pos - (n + 1))); }

struct Layer {
  int own_start, n, top_ext, bot_ext, R, rowbase;
  int r0, r1, rn, rn1;  // local rows of the paper's j = 0, 1, n, n+1 (-1 if absent)
  int mid;              // middle row of the two-ended elimination (floor(R / 2))
};

struct Launch {
  int job0 = 0, njobs = 0, maxterms = 0;
  int cls = PT_CLS_LOCAL;    // pt_launch_class
  bool plr = false;          // job terms point at compressed blocks
  bool split = false;        // job terms point at split planes
  bool f32 = false;          // job terms point at float32 blocks
  double mat_elems = 0;      // matrix entries streamed by one launch
  double vec_elems_rhs = 0;  // vector entries read + written per right-hand side
  std::vector<int> lay_off;  // local-solve launches: first job of each layer (L + 1 entries; jobs in layer order)
  bool wide = false;         // some job has a wide term (columns != n)
  int two_term = 0;          // split launches: every job two terms with Q and (2) every S or (1) no S
  bool klist = false;        // jobs carry nonzero-chunk lists: float64 MFMA form only
};

struct ProfPending {
  int ev;  // index of the event pair
  int cls;
  double bytes, flops;
};

// One GPU operation of a recorded stage (a merged solve of several problems
// records each problem's operations, then issues them together): a block
// apply, which may share one launch with other problems' applies, or any
// other stream operation (fn).
struct Rec {
  std::function<hipError_t(hipStream_t)> fn;  // empty: a block apply
  Launch Lc;
  int nrhs = 0;
  int64_t ld = 0;
  Bases b{};
};

// Issue a stream operation on the solver's stream, or record it while the
// solver records a stage; `f` takes the stream to issue on.
template <typename F>
inline pt_status gpu_op(std::vector<Rec>* rec, hipStream_t st, const char* what, F&& f) {
  if (rec) {
    Rec r;
    r.fn = std::forward<F>(f);
    rec->push_back(std::move(r));
    return PT_OK;
  }
  const hipError_t e = f(st);
  if (e != hipSuccess) return fail(PT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return PT_OK;
}

// a tuned launch shape (0: the built-in rule)
struct TuneCfg {
  int tn = 0, ks = 0;         // MFMA tile width and wave groups
  int mks = 0;                // MFMA k-slices over workgroups (0, 1: none)
  SplitCfg sp{0, 0};          // split-bfloat16 tile width and k-slices
  int njobs = 0;              // jobs of the launch the shape was timed on
};

// block types per layer; each is a 2x2 arrangement of NX x NX blocks
enum { T_DN = 0, B_UP = 1, T_UP = 2, B_DN = 3 };

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  hipError_t alloc(size_t count) {
    n = count;
    if (count == 0) return hipSuccess;
    return hipMalloc((void**)&p, count * sizeof(T));
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

}  // namespace polar_impl

using namespace polar_impl;

struct pt_solver {
  // problem
  int nx = 0, nz = 0, npml = 0, NX = 0, NZ = 0, L = 0;
  double h = 0, omega = 0, C = 0;
  pt_options opt{};
  hipStream_t st = nullptr;
  int device = 0;
  std::vector<Layer> lay;
  int sumR = 0, Rmax = 0;
  int64_t Nt = 0;  // complex entries of one polarized vector
  bool f32 = false;  // float32 form: the Gauss-Seidel preconditioner's blocks in float32 (blk32)
  double plr_ms = 0;
  double setup_ms = 0;

  // coefficients
  std::vector<cd> lcoef, ucoef;  // z couplings of each local row (sumR)
  std::vector<double> c_host;    // the velocity on the padded grid (kept for pt_save)

  // device data
  PlrSet plr;
  bool use_plr = false;
  int plr_rmax = 0;  // leaf rank limit of the compressed blocks in use
  DevBuf<double2> dinv64, blk64;
  DevBuf<float2> blk32;
  DevBuf<uint16_t> blkbf;  // split-bfloat16 planes of every block (preconditioner of the mixed form)
  bool split = false;
  bool split_f16 = false;    // the split planes are float16 (PT_SPLIT_F16), else bfloat16
  double split_alpha = 1.0;  // factor folded into the jobs of split launches (float16: 1 / both scales)
  DevBuf<float2> part;     // k-slice partial tiles of small split launches
  DevBuf<double2> plr_part;  // leaf-slice partial tiles of small compressed-block launches
  DevBuf<double2> mpart;     // k-slice partial tiles of MFMA sweep launches (float64 and float32 forms)
  // interface Green's functions of the pre-solve: per layer, rows 1 and n of
  // (A^l)^-1 over the owned rows, NX x (n NX) each (null: line-by-line)
  DevBuf<double2> green;
  std::vector<size_t> green_off;  // [layer * 4 + trace-row slot] -> offset in green (SIZE_MAX: absent)
  Launch green_launch;            // one job per (layer, kept row 1 / n), layer order
  Launch green_ext;               // rows 0 and n+1 by extrapolation from rows 1 and n, layer order
  // the same products with each row block split over K ranges (wide passes):
  // partial rows in free rows of each layer, summed into the trace rows
  Launch green_split;
  DevBuf<int32_t> gsum_dst, gsum_src, gsum_cnt;  // per (layer, trace row), layer order
  std::vector<int> gsum_off;                     // first entry of each layer (L + 1)
  // nonzero-chunk lists of the split products' inputs, per (layer, row range)
  DevBuf<int32_t> nz_list, nz_in_k;
  DevBuf<int64_t> nz_in_off;
  std::vector<int> nz_off;  // first list of each layer (L + 1)
  int nz_stride = 1;
  std::vector<cd> ax_host;        // x-direction PML alphas at the nodes
  int nblk = 0;
  std::vector<int> bidx;  // [layer][type][a][b] -> block number, -1 absent
  DevBuf<int32_t> rowmap;
  // layers touched by each source (pre-solve only where a source is nonzero)
  DevBuf<int32_t> row_layer, lay_own_start, lay_n_own, slot_rhs, rhs_slot;
  DevBuf<double> act;         // per (source, layer): largest |f|^2 on the layer's owned rows
  double* h_act = nullptr;    // pinned, L * max_nrhs
  int32_t* h_slot = nullptr;  // pinned, 2 * L * max_nrhs: slot_rhs then rhs_slot
  int last_slots = 0;         // column slots of the last pre-solve (nrhs when dense)
  DevBuf<int32_t> g_seg, g_row, f_seg, f_row;
  DevBuf<double> f_sign, g_sign;
  int n_gather = 0, n_force = 0;

  // job lists
  std::vector<Job> hjobs;
  DevBuf<Job> jobs;
  std::vector<Launch> fwd, bwd, sweep;
  std::vector<Launch> bwd_pre, bwd_rec;  // backward passes stopped at the trace rows / the owned rows
  std::vector<Launch> fwd_win;           // forward passes of right-hand sides zero outside the trace rows 0..n+1
  // reconstruction on the volume fields in place (no layer-local copies)
  std::vector<Launch> fwd_rec, bwd_rec2;
  bool rec_direct = false;
  int n_rec_rhs = 0;  // forced right-hand-side rows
  DevBuf<int32_t> rr_dst, rr_src, rr_seg;
  DevBuf<double> rr_sign;
  Launch bterm, opA, opR;
  Launch opA2;  // second launch of A in the extrapolated form (njobs 0: A is one launch)
  // the system closed by extrapolation relations (closure 1)
  Launch opX, opX2, opRX, gsRX, tX;
  DevBuf<uint16_t> xbf;  // split-bfloat16 planes of the extrapolators' factors (mixed form)

  // captured GMRES iterations: (nrhs, iteration) -> executable graph
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  bool graph_failed = false;  // capture did not work on this stream: plain launches
  std::vector<Rec>* rec = nullptr;  // set: stream operations are recorded here instead of issued

  // learned preconditioner stage (null: sweeps only)
  pt_learned* learned = nullptr;
  int learned_mode = PT_LEARN_CORRECT;

  // live timing of block-apply launches
  bool prof = false;
  std::vector<hipEvent_t> ev;  // 2 per slot
  int ev_next = 0;
  std::vector<ProfPending> pend;
  pt_kernel_stats stats{};
  pt_kernel_stats cstats[PT_CLS_COUNT]{};
  std::map<int, TuneCfg> tune[PT_CLS_COUNT];  // per class: nrhs -> shape

  // work
  DevBuf<double2> W, Bw, fio, uio, s, V, Z, U1, U2, tmp, zeros, x;
  DevBuf<double2> hbuf, hacc, Hc, sn, g, y;
  DevBuf<double> nrm, cs, est, beta;
  DevBuf<int32_t> iters, done, flag;
  int32_t* h_done = nullptr;  // pinned

  size_t block_elems() const { return (size_t)NX * NX; }
  const void* blk(int l, int type, int a, int b) const {
    const int id = bidx[((l * 4 + type) * 2 + a) * 2 + b];
    return id < 0 ? nullptr : (const void*)(blk64.p + (size_t)id * block_elems());
  }
  // the float32 copy of a block (float32 form: the preconditioner's blocks)
  const void* blk_f32(int l, int type, int a, int b) const {
    const int id = bidx[((l * 4 + type) * 2 + a) * 2 + b];
    return id < 0 ? nullptr : (const void*)(blk32.p + (size_t)id * block_elems());
  }
  // what a trace-block job term points at: the dense block or its compressed form
  const void* blk_term(int l, int type, int a, int b) const {
    if (!use_plr) return blk(l, type, a, b);
    const int id = bidx[((l * 4 + type) * 2 + a) * 2 + b];
    return id < 0 ? nullptr : (const void*)plr.block(id);
  }
  const void* blk_split(int l, int type, int a, int b) const {
    const int id = bidx[((l * 4 + type) * 2 + a) * 2 + b];
    return id < 0 ? nullptr : (const void*)(blkbf.p + (size_t)id * split_block_elems(NX));
  }
  // block term of a preconditioner job: the split planes or the float32 copy
  // in the reduced-precision forms
  const void* blk_pre(int l, int type, int a, int b) const {
    return split ? blk_split(l, type, a, b) : f32 ? blk_f32(l, type, a, b) : blk_term(l, type, a, b);
  }
  int blk_id(const void* term) const {
    if (!use_plr) return -1;
    return (int)((const PlrBlockDev*)term - plr.d_blocks);
  }
  const void* dinv(int l, int r) const {
    return (const void*)(dinv64.p + (size_t)(lay[l].rowbase + r) * block_elems());
  }
  // offset of trace segment (half h: 0 down, 1 up; interface k; row a)
  int64_t seg(int hh, int k, int a) const { return ((int64_t)(hh * (L - 1) + k) * 2 + a) * NX; }
};


namespace polar_impl {

// A saved solver being read back (pt_load): setup takes the factors, blocks,
// Green's functions and compressed blocks from fp, in the order it needs them,
// instead of computing them.
struct LoadSrc {
  FILE* fp = nullptr;
  bool green = false;  // interface Green's functions stored
  bool plr = false;    // compressed blocks stored
};
pt_status setup_impl(const pt_problem* prob, const pt_options* opt, void* hip_stream, pt_solver** out,
                     const LoadSrc* src);

// stages of the online path (solver.hip)
pt_status precondition(pt_solver* S, const double2* v, double2* z, int nrhs);
pt_status apply_op(pt_solver* S, const Launch& op, const double2* x, double2* y, int nrhs);
pt_status trace_rhs(pt_solver* S, const double2* f, double2* s, int nrhs);
// the operator and preconditioner of the system GMRES solves (closure 0: jump, 1: extrapolation)
pt_status system_A(pt_solver* S, const double2* x, double2* y, int nrhs);
pt_status system_M(pt_solver* S, const double2* v, double2* z, int nrhs);
pt_status precondition_extrap(pt_solver* S, const double2* v, double2* z, int nrhs);
pt_status dinv_extrap_inplace(pt_solver* S, double2* c, int nrhs);
// flexible GMRES on A x = S->s for nrhs columns; result in S->x.  With
// `learned`, every preconditioner output goes through the learned stage.
pt_status fgmres(pt_solver* S, int nrhs, bool& all_conv, double tol, bool learned);

// learned stage (learned.hip)
// clears the per-RHS counters of steps that kept the correction
pt_status learned_begin(pt_solver* S, int nrhs);
// z = GS(v) on entry.  Computes w = A z, r = v - w, c = N(r), A c, and per RHS
// keeps z += c, w += A c where ||r - A c|| < ||r||.  On return w = A z.
pt_status learned_step(pt_solver* S, const double2* v, double2* z, double2* w, int nrhs);
// augmenting form: r = v - w after a sweep step (w = A GS(v)), then z = N(r)
// as the direction of the next step (counted per RHS not yet converged)
pt_status learned_residual(pt_solver* S, const double2* v, const double2* w, int nrhs);
pt_status learned_direction(pt_solver* S, double2* z, int nrhs);
// per-RHS step counters to the host (asynchronous on the solver stream)
pt_status learned_kept(pt_solver* S, int nrhs, int32_t* host);

}  // namespace polar_impl
