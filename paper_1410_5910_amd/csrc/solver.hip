// libpolar host side: validation, layer layout, coefficient assembly, the
// offline factorisation / trace-block extraction on the GPU (Alg. 1), the
// online solve (Alg. 2 with flexible GMRES on the jump-closed polarized
// system, Def. 9, preconditioned by Gauss-Seidel sweeps, Alg. 4), and the
// C-ABI of include/polar.h.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "persist.h"
#include "solver_internal.h"

namespace polar_impl {

// ---------------------------------------------------------------------------
// geometry of one block-apply launch
// ---------------------------------------------------------------------------
ApplyGeom geom_for(int n, int maxterms, int nrhs, int njobs = 1) {
  ApplyGeom g{};
  g.n = n;
  g.nr = nrhs <= 1 ? 1 : nrhs <= 2 ? 2 : nrhs <= 4 ? 4 : nrhs <= 8 ? 8 : 16;
  const int K = std::max(1, maxterms * n);
  // column chunks are taken inside one term (block) at a time
  (void)K;
  // MFMA tile width: the widest that still gives about two workgroups per CU
  g.mfma = 0;
  if (nrhs > 4) {
    const long rows = (long)njobs * ((n + 63) / 64);
    g.mfma = 16;
    for (int tn : {64, 32})  // never wider than the right-hand sides rounded up to 16
      if (tn <= 16 * ((nrhs + 15) / 16) && rows * ((nrhs + tn - 1) / tn) >= 512) {
        g.mfma = tn;
        break;
      }
  }
  // up to 4 right-hand sides the matrix is streamed row by row at HBM speed
  g.gemv = nrhs <= 4 ? 1 : 0;
  if (g.gemv) {
    g.ntiles = (n + 7) / 8;
    g.kc = std::min(n, g.nr >= 4 ? 256 : 512);  // <= 64 columns per in-flight load slot; LDS 2 kc nr complex
    g.steps = std::max(1, maxterms) * ((n + g.kc - 1) / g.kc);
  } else {
    g.ntiles = (n + 63) / 64;
    g.kc = std::min(n, 2048 / g.nr);  // LDS = max(kc, 128) * nr complex doubles <= 32 KiB
  }
  return g;
}

VecRef vr(int buf, int64_t off) { return VecRef{buf, 0, off}; }
VecRef none() { return VecRef{-1, 0, 0}; }

Job empty_job() {
  Job j;
  std::memset(&j, 0, sizeof(j));
  for (int t = 0; t < 4; ++t) {
    j.Q[t] = none();
    j.S[t] = none();
    j.beta[t] = make_double2(0.0, 0.0);
  }
  j.P = none();
  j.Y = none();
  j.alpha = make_double2(1.0, 0.0);
  return j;
}

void add_term(Job& j, const void* M, VecRef q, VecRef s = VecRef{-1, 0, 0}, double2 beta = make_double2(1.0, 0.0)) {
  const int t = j.nterms++;
  j.M[t] = M;
  j.Q[t] = q;
  j.S[t] = s;
  j.beta[t] = beta;
}

constexpr int kEventSlots = 2048;

pt_status prof_harvest(pt_solver* S) {
  if (S->pend.empty()) return PT_OK;
  HIPCHK(hipStreamSynchronize(S->st));
  for (const ProfPending& p : S->pend) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, S->ev[2 * p.ev], S->ev[2 * p.ev + 1]));
    for (pt_kernel_stats* k : {&S->stats, &S->cstats[p.cls]}) {
      k->launches += 1;
      k->kernel_ms += ms;
      k->alg_bytes += p.bytes;
      k->alg_flops += p.flops;
    }
  }
  S->pend.clear();
  S->ev_next = 0;
  return PT_OK;
}

// the shape of a launch: the tuned one for its class and nrhs, else the rules
const TuneCfg* tuned(const pt_solver* S, const Launch& Lc, int nrhs) {
  const auto& m = S->tune[Lc.cls];
  const auto it = m.find(nrhs);
  if (it == m.end()) return nullptr;
  // a launch with far fewer jobs than the timed one (the tail rows of the
  // longest layers) fills few CUs: the rules' k-split serves it better
  if (4 * Lc.njobs < it->second.njobs) return nullptr;
  return &it->second;
}

// complex floats of k-slice partial tiles a split-bfloat16 launch writes (0: one slice)
size_t split_part_need(const pt_solver* S, const Launch& Lc, int nrhs, const TuneCfg* tc) {
  const SplitCfg sc = tc ? tc->sp : SplitCfg{0, 0};
  const int ks = sc.kslices > 0 ? sc.kslices : split_kslices(Lc.njobs, S->NX, nrhs, sc.tile_rhs);
  return ks > 1 ? (size_t)ks * Lc.njobs * nrhs * S->NX : 0;
}

pt_status run_apply_cfg(pt_solver* S, const Launch& Lc, int nrhs, int64_t ld, Bases b, const TuneCfg* tc) {
  if (Lc.njobs == 0) return PT_OK;
  if (S->rec) {  // recorded: issued later, possibly in one launch with other problems'
    Rec r;
    r.Lc = Lc;
    r.nrhs = nrhs;
    r.ld = ld;
    r.b = b;
    S->rec->push_back(std::move(r));
    return PT_OK;
  }
  ApplyGeom g = geom_for(S->NX, Lc.maxterms, nrhs, Lc.njobs);
  if (Lc.wide) g.steps = 0;  // wide terms: the streaming form's general (pipelined) variant
  if (tc && g.mfma && tc->tn) {
    g.mfma = tc->tn;
    g.ks = tc->ks;
    g.mks = tc->mks;
  }
  int slot = -1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (S->prof) {
    if (S->ev_next >= kEventSlots) PTCHK(prof_harvest(S));
    slot = S->ev_next++;
    e0 = S->ev[2 * slot];
    e1 = S->ev[2 * slot + 1];
  }
  // with profiling on, the dispatch itself stamps e0 / e1 at kernel start / end
  if (Lc.plr)
    HIPCHK(launch_plr_apply(S->jobs.p + Lc.job0, Lc.njobs, S->NX, nrhs, ld, b, S->st, e0, e1, S->plr_part.p,
                            S->plr_part.n));
  else if (Lc.split) {
    SplitCfg sc = tc ? tc->sp : SplitCfg{0, 0};
    if (sc.stream && sc.stream != Lc.two_term) sc.stream = 0;  // the form only serves launches it fits
    sc.f16 = S->split_f16 ? 1 : 0;
    const size_t need = split_part_need(S, Lc, nrhs, tc);
    float2* part = need <= S->part.n ? S->part.p : nullptr;  // null: no k-slices
    HIPCHK(launch_block_apply_split(S->jobs.p + Lc.job0, Lc.njobs, S->NX, nrhs, ld, b, S->st, e0, e1, part, sc));
  }
  else {
    HIPCHK(launch_block_apply(S->jobs.p + Lc.job0, Lc.njobs, g, nrhs, ld, b, Lc.f32, S->st, e0, e1, S->mpart.p,
                              S->mpart.n));
  }
  if (S->prof) {
    // bytes per stored complex entry: 4 bfloat16 planes, float32 or float64 pairs
    const double es = Lc.split ? 8.0 : Lc.f32 ? 8.0 : 16.0;
    S->pend.push_back(ProfPending{slot, Lc.cls, Lc.mat_elems * es + Lc.vec_elems_rhs * nrhs * 16.0,
                                  8.0 * Lc.mat_elems * nrhs});
  }
  return PT_OK;
}

pt_status run_apply(pt_solver* S, const Launch& Lc, int nrhs, int64_t ld, Bases b) {
  return run_apply_cfg(S, Lc, nrhs, ld, b, tuned(S, Lc, nrhs));
}

Launch push_launch(pt_solver* S, const std::vector<Job>& js, int cls, bool plr_terms = false,
                   bool split_terms = false) {
  Launch Lc;
  Lc.cls = cls;
  Lc.split = split_terms && S->split;
  Lc.f32 = split_terms && S->f32 && !S->split;  // the float32 form's preconditioner blocks
  if (Lc.split || Lc.f32) plr_terms = false;
  Lc.job0 = (int)S->hjobs.size();
  Lc.njobs = (int)js.size();
  for (const Job& j : js) Lc.maxterms = std::max(Lc.maxterms, j.nterms);
  const double n = S->NX;
  for (const Job& j : js) {
    if (S->use_plr && plr_terms) {
      for (int t = 0; t < j.nterms; ++t) Lc.mat_elems += (double)S->plr.stored_entries(S->blk_id(j.M[t]));
      Lc.plr = true;
    } else {
      for (int t = 0; t < j.nterms; ++t) Lc.mat_elems += n * (j.kw[t] > 0 ? (double)j.kw[t] : n);
    }
    double v = (j.P.buf >= 0 ? n : 0) + n;  // epilogue read + output write
    for (int t = 0; t < j.nterms; ++t) {
      const double k = j.kw[t] > 0 ? (double)j.kw[t] : n;
      v += (j.Q[t].buf >= 0 ? k : 0) + (j.S[t].buf >= 0 ? k : 0);
      if (j.kw[t] > 0) Lc.wide = true;
    }
    Lc.vec_elems_rhs += v;
  }
  if (Lc.split && !js.empty()) {
    bool all_s = true, no_s = true, ok = true;
    for (const Job& j : js) {
      ok = ok && j.nterms == 2 && j.Q[0].buf >= 0 && j.Q[1].buf >= 0;
      for (int t = 0; t < 2; ++t) {
        all_s = all_s && j.S[t].buf >= 0;
        no_s = no_s && j.S[t].buf < 0;
      }
    }
    Lc.two_term = !ok ? 0 : all_s ? 2 : no_s ? 1 : 0;
  }
  S->hjobs.insert(S->hjobs.end(), js.begin(), js.end());
  return Lc;
}

// ---------------------------------------------------------------------------
// layout and coefficients
// ---------------------------------------------------------------------------
pt_status validate(const pt_problem* p, const pt_options* o) {
  if (!p || !o) return fail(PT_EINVAL, "null problem or options");
  if (p->nx < 1 || p->nz < 1 || p->npml < 1) return fail(PT_EINVAL, "nx, nz, npml must be >= 1");
  if (!(p->h > 0) || !(p->omega > 0) || !std::isfinite(p->h) || !std::isfinite(p->omega))
    return fail(PT_EINVAL, "h and omega must be positive and finite");
  if (!(p->pml_C >= 0) || !std::isfinite(p->pml_C)) return fail(PT_EINVAL, "pml_C must be >= 0 and finite");
  if (p->L < 1) return fail(PT_EINVAL, "L must be >= 1");
  if (p->nz / p->L < 2) return fail(PT_EINVAL, "every layer needs at least 2 physical rows (nz >= 2L)");
  if (p->nx + 2 * p->npml > 4096) return fail(PT_EINVAL, "NX > 4096 is not supported");
  if (!p->c) return fail(PT_EINVAL, "null velocity");
  const size_t N = (size_t)(p->nx + 2 * p->npml) * (p->nz + 2 * p->npml);
  for (size_t e = 0; e < N; ++e)
    if (!(p->c[e] > 0) || !std::isfinite(p->c[e])) return fail(PT_EINVAL, "velocity must be positive and finite");
  if (o->precision != PT_F64 && o->precision != PT_F32 && o->precision != PT_SPLIT_BF16 &&
      o->precision != PT_SPLIT_F16)
    return fail(PT_EINVAL, "unknown precision");
  if (o->gs_iters < 0 || o->gs_iters > 8) return fail(PT_EINVAL, "gs_iters must be in 0..8");
  if (o->maxit < 1 || o->maxit > 200) return fail(PT_EINVAL, "maxit must be in 1..200");
  if (!(o->tol >= 0)) return fail(PT_EINVAL, "tol must be >= 0");
  if (o->max_nrhs < 1) return fail(PT_EINVAL, "max_nrhs must be >= 1");
  if (o->plr) {
    if (o->precision != PT_F64) return fail(PT_EINVAL, "PLR blocks are float64 only");
    if (!(o->plr_eps > 0)) return fail(PT_EINVAL, "plr_eps must be > 0");
    if (o->plr_rmax < 0 || o->plr_rmax > kPlrMaxRank) return fail(PT_EINVAL, "plr_rmax must be in 0..64");
  }
  if (o->presolve < 0 || o->presolve > 2) return fail(PT_EINVAL, "presolve must be 0, 1 or 2");
  if (o->closure < 0 || o->closure > 1) return fail(PT_EINVAL, "closure must be 0 (jump) or 1 (extrapolation)");
  if (o->closure == 1 && (o->precision == PT_F32 || o->plr))
    return fail(PT_EINVAL, "the extrapolation closure needs float64 factors without PLR blocks");
  return PT_OK;
}

void make_layout(pt_solver* S) {
  const int L = S->L, nz = S->nz, npml = S->npml;
  const int base = nz / L, extra = nz % L;
  int start = 0, rowbase = 0;
  S->lay.clear();
  for (int l = 0; l < L; ++l) {
    Layer y{};
    y.n = base + (l < extra ? 1 : 0) + (l == 0 ? npml : 0) + (l == L - 1 ? npml : 0);
    y.own_start = start;
    y.top_ext = l > 0 ? npml : 0;
    y.bot_ext = l < L - 1 ? npml : 0;
    y.R = y.top_ext + y.n + y.bot_ext;
    y.rowbase = rowbase;
    y.r0 = y.top_ext ? y.top_ext - 1 : -1;
    y.r1 = y.top_ext ? y.top_ext : -1;
    y.rn = y.bot_ext ? y.top_ext + y.n - 1 : -1;
    y.rn1 = y.bot_ext ? y.top_ext + y.n : -1;
    // middle of the rows where the online right-hand sides can be nonzero
    // (trace rows 0..n+1, or the layer's own end without an extension), so
    // both chains of a solve that starts at them are equally long
    y.mid = ((y.top_ext ? y.r0 : 0) + (y.bot_ext ? y.rn1 : y.R - 1)) / 2;
    start += y.n;
    rowbase += y.R;
    S->lay.push_back(y);
  }
  S->sumR = rowbase;
  S->Rmax = 0;
  for (auto& y : S->lay) S->Rmax = std::max(S->Rmax, y.R);
  S->Nt = (int64_t)4 * (L - 1) * S->NX;
}

// Local z data of every local row: alpha at the node and both half nodes
// (owned rows use the global profile; extension rows a profile measured from
// the first extension node), and the padded-grid row of the (normally
// extended) model.
struct RowZ {
  cd a, am, ap;
  int mrow;
};

std::vector<RowZ> local_rows(const pt_solver* S, const Layer& y) {
  const double delta = S->npml * S->h;
  const int q_start = y.own_start - S->npml + 1;  // global q of local j = 1
  auto dist = [&](double zeta) -> double {
    if (y.top_ext && zeta < 1) return std::max(0.0, -zeta);
    if (y.bot_ext && zeta > y.n) return std::max(0.0, zeta - (y.n + 1));
    return beyond(q_start + zeta - 1, S->nz);
  };
  std::vector<RowZ> out(y.R);
  for (int r = 0; r < y.R; ++r) {
    const double j = r - y.top_ext + 1;
    out[r].a = pml_alpha(dist(j) * S->h, S->C, delta, S->omega);
    out[r].am = pml_alpha(dist(j - 0.5) * S->h, S->C, delta, S->omega);
    out[r].ap = pml_alpha(dist(j + 0.5) * S->h, S->C, delta, S->omega);
    const int jj = std::min(std::max((int)j, 1), y.n);
    out[r].mrow = y.own_start + jj - 1;
  }
  return out;
}

// ---------------------------------------------------------------------------
// local solves (forward/backward block sweeps with the stored inverses)
// ---------------------------------------------------------------------------
// Local-solve jobs of the layers ls (row bases rb), two-ended (matching the
// factorisation): forward launch f eliminates row f top-down and row R-1-f
// bottom-up in every layer, y_r = Delta_r^-1 (b_r - l_r y_{r-1}) and
// z_r = Sigma_r^-1 (b_r - u_r z_{r+1}); the last forward launch solves the
// middle row, x_m = Gamma_m^-1 (b_m - l_m y_{m-1} - u_m z_{m+1}); backward
// launches run outward, x_r = y_r - u_r Delta_r^-1 x_{r+1} above the middle and
// x_r = z_r - l_r Sigma_r^-1 x_{r-1} below it, only as far as rows
// rmin[q]..rmax[q] (empty: all rows): rows beyond the ones a caller reads are
// never needed, since the backward recurrences run outward.
//
// zlo[q]..zhi[q] (empty: all rows) is where the right-hand side may be nonzero.
// Above zlo the top-down recurrence gives y_r = 0 and below zhi the bottom-up
// one z_r = 0, so both chains start at the window's ends (launch f then holds
// rows zlo + f and zhi - f) and the backward steps outside it take y_r = 0.
//
// Addresses default to a layer-local field: row r of layer q is row rb[q] + r
// of base 0 (solution) and of base 1 (right-hand side).  `ad` overrides them:
// ad->w(q, r) is the solution row, ad->b(q, r) the right-hand-side row and
// ad->s(q, r) a scale the right-hand side is taken with (the forward step then
// reads y_r = s Delta_r^-1 (b_r - (l_r / s) y_{r-1})).
struct LocalAddr {
  std::function<VecRef(size_t, int)> w, b;
  std::function<double(size_t, int)> s;
};

void build_local_jobs(pt_solver* S, const std::vector<int>& ls, const std::vector<int>& rb,
                      std::vector<std::vector<Job>>& fw, std::vector<std::vector<Job>>& bw,
                      const std::vector<int>& rmin = {}, const std::vector<int>& rmax = {},
                      const std::vector<int>& zlo = {}, const std::vector<int>& zhi = {},
                      const LocalAddr* ad = nullptr) {
  const int NX = S->NX;
  int F = 0, G = 0;
  auto win = [&](size_t q, const Layer& y, int& a, int& b) {  // the window, widened to hold the middle row
    a = zlo.empty() ? 0 : std::min(std::max(0, zlo[q]), y.mid);
    b = zhi.empty() ? y.R - 1 : std::max(std::min(y.R - 1, zhi[q]), y.mid);
  };
  for (size_t q = 0; q < ls.size(); ++q) {
    const Layer& y = S->lay[ls[q]];
    const int lo = rmin.empty() ? 0 : rmin[q], hi = rmax.empty() ? y.R - 1 : rmax[q];
    int a, b;
    win(q, y, a, b);
    F = std::max(F, std::max(y.mid - a, b - y.mid));
    G = std::max(G, std::max(y.mid - std::min(lo, y.mid), std::max(hi, y.mid) - y.mid));
  }
  fw.assign(F + 1, {});
  bw.assign(G, {});
  auto W = [&](size_t q, int r) { return ad ? ad->w(q, r) : vr(0, (int64_t)(rb[q] + r) * NX); };
  auto B = [&](size_t q, int r) { return ad ? ad->b(q, r) : vr(1, (int64_t)(rb[q] + r) * NX); };
  auto sc = [&](size_t q, int r) { return ad ? ad->s(q, r) : 1.0; };
  // beta -c / s of a coupling c on a right-hand side taken with scale s
  auto cb = [&](cd c, double sv) { return make_double2(-c.re / sv, -c.im / sv); };
  for (size_t q = 0; q < ls.size(); ++q) {
    const int l = ls[q];
    const Layer& y = S->lay[l];
    const int m = y.mid;
    const int lo = rmin.empty() ? 0 : rmin[q], hi = rmax.empty() ? y.R - 1 : rmax[q];
    int a, b;
    win(q, y, a, b);
    for (int r = a; r < m; ++r) {  // top-down from the window's top
      Job j = empty_job();
      j.Y = W(q, r);
      const double sv = sc(q, r);
      j.alpha = make_double2(sv, 0.0);
      if (r > a)
        add_term(j, S->dinv(l, r), B(q, r), W(q, r - 1), cb(S->lcoef[y.rowbase + r], sv));
      else
        add_term(j, S->dinv(l, r), B(q, r));
      fw[r - a].push_back(j);
    }
    for (int r = b; r > m; --r) {  // bottom-up from the window's bottom
      Job j = empty_job();
      j.Y = W(q, r);
      const double sv = sc(q, r);
      j.alpha = make_double2(sv, 0.0);
      if (r < b)
        add_term(j, S->dinv(l, r), B(q, r), W(q, r + 1), cb(S->ucoef[y.rowbase + r], sv));
      else
        add_term(j, S->dinv(l, r), B(q, r));
      fw[b - r].push_back(j);
    }
    {  // middle row
      Job j = empty_job();
      j.Y = W(q, m);
      const double sv = sc(q, m);
      j.alpha = make_double2(sv, 0.0);
      if (m > a)
        add_term(j, S->dinv(l, m), B(q, m), W(q, m - 1), cb(S->lcoef[y.rowbase + m], sv));
      else
        add_term(j, S->dinv(l, m), B(q, m));
      if (m < b) add_term(j, S->dinv(l, m), none(), W(q, m + 1), cb(S->ucoef[y.rowbase + m], sv));
      fw[F].push_back(j);
    }
    for (int r = m - 1; r >= lo; --r) {  // outward, upper part
      Job j = empty_job();
      j.Y = W(q, r);
      if (r >= a) j.P = j.Y;  // y_r = 0 above the window
      j.alpha = d2(-S->ucoef[y.rowbase + r]);
      add_term(j, S->dinv(l, r), W(q, r + 1));
      bw[m - 1 - r].push_back(j);
    }
    for (int r = m + 1; r <= hi; ++r) {  // outward, lower part
      Job j = empty_job();
      j.Y = W(q, r);
      if (r <= b) j.P = j.Y;  // z_r = 0 below the window
      j.alpha = d2(-S->lcoef[y.rowbase + r]);
      add_term(j, S->dinv(l, r), W(q, r - 1));
      bw[r - m - 1].push_back(j);
    }
  }
}

// Rows where the right-hand sides of the pre-solve, the reconstruction and the
// extraction can be nonzero: the trace rows 0..n+1 of the layer (a layer
// without an extension on one side: its own end there).
void rhs_window(const pt_solver* S, std::vector<int>& zlo, std::vector<int>& zhi) {
  zlo.resize(S->L);
  zhi.resize(S->L);
  for (int l = 0; l < S->L; ++l) {
    const Layer& y = S->lay[l];
    zlo[l] = y.top_ext ? y.r0 : 0;
    zhi[l] = y.bot_ext ? y.rn1 : y.R - 1;
  }
}

pt_status run_local(pt_solver* S, const std::vector<Launch>& fw, const std::vector<Launch>& bw, int nrhs, int64_t ld,
                    double2* Wsol, double2* Brhs) {
  Bases b{{Wsol, Brhs, nullptr, nullptr}};
  for (const Launch& Lc : fw) PTCHK(run_apply(S, Lc, nrhs, ld, b));
  for (const Launch& Lc : bw) PTCHK(run_apply(S, Lc, nrhs, ld, b));
  return PT_OK;
}

// Record where each layer's jobs start in a local-solve launch (its jobs are
// built layer by layer, each job's output row names its layer).
void index_layers(pt_solver* S, Launch& Lc) {
  const int L = S->L;
  Lc.lay_off.assign(L + 1, 0);
  int prev = 0;
  for (int i = 0; i < Lc.njobs; ++i) {
    const int64_t row = S->hjobs[Lc.job0 + i].Y.off / S->NX;
    int l = 0;
    while (l + 1 < L && row >= S->lay[l + 1].rowbase) ++l;
    if (l < prev) {  // not in layer order: no sub-ranges for this launch
      Lc.lay_off.clear();
      return;
    }
    prev = l;
    ++Lc.lay_off[l + 1];
  }
  for (int l = 0; l < L; ++l) Lc.lay_off[l + 1] += Lc.lay_off[l];
}

// The part of a local-solve launch on layers la..lb (njobs 0: nothing to do).
Launch layer_range(const pt_solver* S, const Launch& Lc, int la, int lb) {
  if (Lc.lay_off.empty() || (la == 0 && lb == S->L - 1)) return Lc;
  Launch sub = Lc;
  sub.job0 = Lc.job0 + Lc.lay_off[la];
  sub.njobs = Lc.lay_off[lb + 1] - Lc.lay_off[la];
  sub.lay_off.clear();
  sub.maxterms = 0;
  sub.mat_elems = 0;
  sub.vec_elems_rhs = 0;
  const double n = S->NX;
  for (int i = 0; i < sub.njobs; ++i) {
    const Job& j = S->hjobs[sub.job0 + i];
    sub.maxterms = std::max(sub.maxterms, j.nterms);
    double v = (j.P.buf >= 0 ? n : 0) + n;
    for (int t = 0; t < j.nterms; ++t) {
      const double k = j.kw[t] > 0 ? (double)j.kw[t] : n;
      sub.mat_elems += n * k;
      v += (j.Q[t].buf >= 0 ? k : 0) + (j.S[t].buf >= 0 ? k : 0);
    }
    sub.vec_elems_rhs += v;
  }
  return sub;
}

// run_local restricted to the contiguous layers la..lb
pt_status run_local_layers(pt_solver* S, const std::vector<Launch>& fw, const std::vector<Launch>& bw, int la, int lb,
                           int nrhs, int64_t ld, double2* Wsol, double2* Brhs) {
  Bases b{{Wsol, Brhs, nullptr, nullptr}};
  for (const auto* list : {&fw, &bw})
    for (const Launch& Lc : *list) {
      const Launch sub = layer_range(S, Lc, la, lb);
      if (sub.njobs > 0) PTCHK(run_apply(S, sub, nrhs, ld, b));
    }
  return PT_OK;
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
// Two-ended line-by-line factorisation of every layer (appendix B's
// recurrence run from both ends).  Rows 0..m-1 are eliminated top-down,
// Delta_0 = A_0, Delta_{r+1} = A_{r+1} - l_{r+1} u_r Delta_r^-1; rows R-1..m+1
// bottom-up, Sigma_{R-1} = A_{R-1}, Sigma_{r-1} = A_{r-1} - u_{r-1} l_r Sigma_r^-1;
// the middle row gets Gamma_m = A_m - l_m u_{m-1} Delta_{m-1}^-1 - u_m l_{m+1}
// Sigma_{m+1}^-1.  The inverses are stored in the slot of their row.  Both
// chains of all layers advance together, one pivoted Gauss-Jordan inversion
// (FP64) per step; each chain's last step leaves its half of Gamma_m, and the
// halves are combined and inverted last.
pt_status factorize(pt_solver* S, const std::vector<cd>& diag_all, const std::vector<cd>& west,
                    const std::vector<cd>& east) {
  const int NX = S->NX, L = S->L;
  const int NC = 2 * L;  // chains: 2l top-down, 2l+1 bottom-up
  const size_t E = S->block_elems();
  hipStream_t st = S->st;
  DevBuf<double2> dg, dw, de, gjA, gjB, coef;
  DevBuf<int32_t> perm, pi;
  DevBuf<double2*> pA, pB, pD, pN, pDiag, pY;
  pt_status rc = PT_OK;
  auto cleanup = [&]() {
    for (auto* b : {&dg, &dw, &de, &gjA, &gjB, &coef}) b->release();
    perm.release();
    pi.release();
    for (auto* b : {&pA, &pB, &pD, &pN, &pDiag, &pY}) b->release();
  };
  auto chk = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && rc == PT_OK) rc = fail(e == hipErrorOutOfMemory ? PT_ENOMEM : PT_EHIP,
                                                  std::string(what) + ": " + hipGetErrorString(e));
    return rc == PT_OK;
  };
  if (!chk(dg.alloc(diag_all.size()), "alloc diag") || !chk(dw.alloc(NX), "alloc") || !chk(de.alloc(NX), "alloc") ||
      !chk(gjA.alloc(E * NC), "alloc gj") || !chk(gjB.alloc(E * NC), "alloc gj") || !chk(coef.alloc(NC), "alloc") ||
      !chk(perm.alloc((size_t)NC * NX), "alloc") || !chk(pi.alloc((size_t)NC * NX), "alloc") ||
      !chk(pA.alloc(NC), "alloc") || !chk(pB.alloc(NC), "alloc") || !chk(pD.alloc(NC), "alloc") ||
      !chk(pN.alloc(NC), "alloc") || !chk(pDiag.alloc(NC), "alloc") || !chk(pY.alloc(NC), "alloc")) {
    cleanup();
    return rc;
  }
  chk(hipMemcpy(dg.p, diag_all.data(), diag_all.size() * sizeof(double2), hipMemcpyHostToDevice), "copy");
  chk(hipMemcpy(dw.p, west.data(), NX * sizeof(double2), hipMemcpyHostToDevice), "copy");
  chk(hipMemcpy(de.p, east.data(), NX * sizeof(double2), hipMemcpyHostToDevice), "copy");
  chk(hipMemsetAsync(S->flag.p, 0, sizeof(int32_t), st), "memset");
  if (rc != PT_OK) {
    cleanup();
    return rc;
  }
  auto diag_of = [&](int l, int r) { return (double2*)dg.p + (size_t)(S->lay[l].rowbase + r) * NX; };
  auto buf = [&](int c, int which) { return (which ? gjB.p : gjA.p) + (size_t)c * E; };
  // chain c: its layer, direction, length and the local row of its step f
  auto chain_len = [&](int c) {
    const Layer& y = S->lay[c / 2];
    return (c & 1) ? y.R - 1 - y.mid : y.mid;
  };
  auto chain_row = [&](int c, int f) { return (c & 1) ? S->lay[c / 2].R - 1 - f : f; };
  int F = 0;
  for (int c = 0; c < NC; ++c) F = std::max(F, chain_len(c));
  std::vector<int> cur(NC, 0);  // which of the chain's two buffers holds its current matrix

  // Invert the nb matrices whose pointers are in pA (scratch in pB); returns whether the result is in pB.
  // Blocked: one panel of columns per pair of launches (panel steps in place, then the other columns
  // out of place), instead of one launch per pivot.
  auto gj_invert = [&](int nb) {
    const int bw = gj_panel_width();
    int np = 0;
    for (int k0 = 0; k0 < NX && rc == PT_OK; k0 += bw, ++np) {
      const int w = std::min(bw, NX - k0);
      DevBuf<double2*>& from = (np % 2 == 0) ? pA : pB;
      DevBuf<double2*>& to = (np % 2 == 0) ? pB : pA;
      chk(launch_gj_panel(from.p, nb, NX, k0, w, perm.p, S->flag.p, st), "gj_panel");
      chk(launch_gj_update(from.p, to.p, nb, NX, k0, w, perm.p, st), "gj_update");
    }
    chk(launch_gj_perm(perm.p, pi.p, nb, NX, st), "gj_perm");
    return (np % 2) == 1;
  };
  auto upload = [&](DevBuf<double2*>& d, const std::vector<double2*>& h) {
    return chk(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(double2*), hipMemcpyHostToDevice, st), "copy");
  };
  // first matrix of every non-empty chain: tridiag of its first row; an empty
  // chain's half of Gamma_m is tridiag(A_m) itself
  {
    std::vector<double2*> out, dia;
    for (int c = 0; c < NC; ++c) {
      const int l = c / 2;
      out.push_back(buf(c, 0));
      dia.push_back(chain_len(c) > 0 ? diag_of(l, chain_row(c, 0)) : diag_of(l, S->lay[l].mid));
    }
    upload(pA, out);
    upload(pDiag, dia);
    chk(launch_init_delta(pA.p, (const double2* const*)pDiag.p, dw.p, de.p, NC, NX, st), "init_delta");
    chk(hipStreamSynchronize(st), "sync");
  }
  for (int f = 0; f < F && rc == PT_OK; ++f) {
    std::vector<int> act;
    for (int c = 0; c < NC; ++c)
      if (f < chain_len(c)) act.push_back(c);
    const int nb = (int)act.size();
    std::vector<double2*> hA(nb), hB(nb), hD(nb), hN(nb), hDiag(nb), hRes(nb);
    std::vector<double2> hcoef(nb);
    for (int q = 0; q < nb; ++q) {
      hA[q] = buf(act[q], cur[act[q]]);
      hB[q] = buf(act[q], 1 - cur[act[q]]);
    }
    upload(pA, hA);
    upload(pB, hB);
    const bool inB = gj_invert(nb);
    for (int q = 0; q < nb; ++q) {
      const int c = act[q], l = c / 2;
      const Layer& y = S->lay[l];
      const int r = chain_row(c, f);
      hRes[q] = inB ? hB[q] : hA[q];
      double2* other = inB ? hA[q] : hB[q];
      hD[q] = S->dinv64.p + (size_t)(y.rowbase + r) * E;
      // next matrix of the chain: the next row's Schur complement, or after the
      // last step this chain's half of Gamma_m (the next row is then m)
      const int rn = (c & 1) ? r - 1 : r + 1;
      hN[q] = other;
      hDiag[q] = diag_of(l, rn);
      const cd cf = (c & 1) ? S->ucoef[y.rowbase + rn] * S->lcoef[y.rowbase + r]
                            : S->lcoef[y.rowbase + rn] * S->ucoef[y.rowbase + r];
      hcoef[q] = d2(cf);
      cur[c] = (other == buf(c, 0)) ? 0 : 1;
    }
    // pB may still be read by the last elimination steps: the copy is stream-ordered after them
    upload(pB, hRes);
    upload(pD, hD);
    upload(pN, hN);
    upload(pDiag, hDiag);
    chk(hipMemcpyAsync(coef.p, hcoef.data(), nb * sizeof(double2), hipMemcpyHostToDevice, st), "copy");
    chk(launch_finish_row(pB.p, pi.p, pD.p, pN.p, (const double2* const*)pDiag.p, coef.p, dw.p, de.p, nb, NX, st),
        "finish_row");
    chk(hipStreamSynchronize(st), "sync");
  }
  // Gamma_m = (top half) + (bottom half) - tridiag(A_m), inverted into the slot of row m
  if (rc == PT_OK) {
    std::vector<double2*> hG(L), hY(L), hDiag(L), hS(L), hD(L), hN(L, nullptr), hRes(L);
    for (int l = 0; l < L; ++l) {
      hG[l] = buf(2 * l, cur[2 * l]);
      hY[l] = buf(2 * l + 1, cur[2 * l + 1]);
      hDiag[l] = diag_of(l, S->lay[l].mid);
      hS[l] = buf(2 * l, 1 - cur[2 * l]);
      hD[l] = S->dinv64.p + (size_t)(S->lay[l].rowbase + S->lay[l].mid) * E;
    }
    upload(pA, hG);
    upload(pY, hY);
    upload(pDiag, hDiag);
    chk(launch_twist_combine(pA.p, (const double2* const*)pY.p, (const double2* const*)pDiag.p, dw.p, de.p, L, NX,
                             st),
        "twist_combine");
    upload(pB, hS);
    const bool inB = gj_invert(L);
    for (int l = 0; l < L; ++l) hRes[l] = inB ? hS[l] : hG[l];
    upload(pB, hRes);
    upload(pD, hD);
    upload(pN, hN);
    for (auto& d : hDiag) d = nullptr;
    upload(pDiag, hDiag);
    chk(launch_finish_row(pB.p, pi.p, pD.p, pN.p, (const double2* const*)pDiag.p, coef.p, dw.p, de.p, L, NX, st),
        "finish_row");
    chk(hipStreamSynchronize(st), "sync");
  }
  int32_t flag = 0;
  if (rc == PT_OK) chk(hipMemcpy(&flag, S->flag.p, sizeof(int32_t), hipMemcpyDeviceToHost), "copy");
  cleanup();
  if (rc == PT_OK && flag) rc = fail(PT_ESINGULAR, "zero pivot in a local Schur complement");
  return rc;
}

// device bytes of interface Green's functions held by all solvers of the process
std::atomic<size_t> g_green_total{0};

void release_green(pt_solver* S) {
  if (S->green.p) g_green_total -= S->green.n * sizeof(double2);
  S->green.release();
}

// Rows of a layer's inverse kept as interface Green's functions: row 1 (with
// a top interface) and row n (with a bottom one).  Rows 0 and n+1 of the
// pre-solve follow from them by one-sided extrapolation: the sources lie on
// the owned rows, where G(z_0, z_j) = E_up G(z_1, z_j) and
// G(z_{n+1}, z_j) = E_down G(z_n, z_j) (Lemma extrapolator_def), with
// E_up = -u Delta_0^-1 and E_down = -l Sigma_{n+1}^-1 from the factors.
std::vector<int> green_rows(const Layer& y) {
  std::vector<int> g;
  if (y.top_ext) g.push_back(y.r1);
  if (y.bot_ext) g.push_back(y.rn);
  return g;
}

pt_status extract_blocks(pt_solver* S, const LoadSrc* src) {
  const int NX = S->NX, L = S->L;
  const size_t E = S->block_elems();
  hipStream_t st = S->st;
  // block numbering
  S->bidx.assign((size_t)L * 16, -1);
  int nb = 0;
  for (int l = 0; l < L; ++l) {
    const bool top = S->lay[l].top_ext > 0, bot = S->lay[l].bot_ext > 0;
    const bool has[4] = {top && bot, bot, top && bot, top};
    for (int t = 0; t < 4; ++t)
      if (has[t])
        for (int ab = 0; ab < 4; ++ab) S->bidx[(l * 4 + t) * 4 + ab] = nb++;
  }
  S->nblk = nb;
  HIPCHK(S->blk64.alloc((size_t)nb * E));
  if (L == 1) return PT_OK;
  if (src) {
    // blocks and (when they were kept) the interface Green's functions from the file
    if (!rec_read_device(src->fp, S->blk64.p, (uint64_t)nb * E, sizeof(double2)))
      return fail(PT_EINVAL, "saved solver: trace blocks");
    S->green_off.assign((size_t)L * 4, SIZE_MAX);
    if (!src->green) return PT_OK;
    size_t need = 0;
    std::vector<size_t> offs((size_t)L * 4, SIZE_MAX);
    for (int l = 0; l < L; ++l) {
      const size_t ng = green_rows(S->lay[l]).size();
      for (size_t k = 0; k < ng; ++k) {
        offs[(size_t)l * 4 + k] = need;
        need += (size_t)NX * ((size_t)S->lay[l].n * NX);
      }
    }
    if (S->green.alloc(need) != hipSuccess) {
      S->green.release();
      return fail(PT_ENOMEM, "interface Green's functions");
    }
    g_green_total += need * sizeof(double2);
    S->green_off = offs;
    if (!rec_read_device(src->fp, S->green.p, need, sizeof(double2)))
      return fail(PT_EINVAL, "saved solver: interface Green's functions");
    return PT_OK;
  }

  int maxq = 0;
  int maxR = 0;
  for (auto& y : S->lay) {
    maxq = std::max(maxq, (y.top_ext ? 1 : 0) + (y.bot_ext ? 1 : 0));
    maxR = std::max(maxR, y.R);
  }
  DevBuf<double2> Wx, Bx, Kr;
  DevBuf<int32_t> rows;
  const size_t wel = (size_t)maxq * NX * maxR * NX;
  pt_status rc = PT_OK;
  // raw blocks K_{j,k} of one layer, j in {0, 1, n, n+1} x k in {0, 1, n, n+1}
  if (Wx.alloc(wel) != hipSuccess || Bx.alloc(wel) != hipSuccess || rows.alloc(4) != hipSuccess ||
      Kr.alloc(16 * E) != hipSuccess) {
    Wx.release();
    Bx.release();
    Kr.release();
    rows.release();
    return fail(PT_ENOMEM, "extraction workspace");
  }
  // interface Green's functions of the pre-solve (from the float64 factors,
  // which every precision form keeps)
  S->green_off.assign((size_t)L * 4, SIZE_MAX);
  if (S->opt.presolve != 0) {
    size_t need = 0;
    for (int l = 0; l < L; ++l) {
      const Layer& y = S->lay[l];
      need += green_rows(y).size() * NX * ((size_t)y.n * NX);
    }
    // auto: at most a third of the free memory, a sixteenth of the device per
    // solver and a quarter of the device over all solvers of the process, so
    // that solvers set up later still find room for their factors
    size_t freeb = 0, totalb = 0;
    const size_t bytes = need * sizeof(double2);
    const bool fits = hipMemGetInfo(&freeb, &totalb) == hipSuccess && bytes <= freeb / 3 && bytes <= totalb / 16 &&
                      g_green_total.load() + bytes <= totalb / 4;
    if (S->opt.presolve == 1 || fits) {
      if (S->green.alloc(need) != hipSuccess) {
        S->green.release();
        if (S->opt.presolve == 1) {
          Wx.release();
          Bx.release();
          rows.release();
          return fail(PT_ENOMEM, "interface Green's functions");
        }
        (void)hipGetLastError();
      } else {
        g_green_total += bytes;
        size_t off = 0;
        for (int l = 0; l < L; ++l) {
          const Layer& y = S->lay[l];
          const size_t ng = green_rows(y).size();
          for (size_t k = 0; k < ng; ++k) {
            S->green_off[(size_t)l * 4 + k] = off;
            off += (size_t)NX * ((size_t)y.n * NX);
          }
        }
      }
    }
  }
  DevBuf<double2> gax, gaz;
  if (S->green.p) {
    std::vector<double2> hax(NX);
    for (int i = 0; i < NX; ++i) hax[i] = d2(S->ax_host[i]);
    if (gax.alloc(NX) != hipSuccess || gaz.alloc(maxR) != hipSuccess ||
        hipMemcpy(gax.p, hax.data(), NX * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess) {
      gax.release();
      gaz.release();
      Wx.release();
      Bx.release();
      rows.release();
      return fail(PT_EHIP, "green scaling");
    }
  }
  const size_t saved_jobs = S->hjobs.size();
  for (int l = 0; l < L && rc == PT_OK; ++l) {
    const Layer& y = S->lay[l];
    // unit right-hand sides at rows 1 and n only: the columns at rows 0 and n+1
    // follow from them (Lemma 4 with the layer's reciprocity, below)
    std::vector<int32_t> src;
    if (y.top_ext) src.push_back(y.r1);
    if (y.bot_ext) src.push_back(y.rn);
    const int nq = (int)src.size();
    const int nrhs = nq * NX;
    const int64_t ld = (int64_t)y.R * NX;
    // per-layer local solve jobs (this layer only, rows from 0): the unit
    // right-hand sides sit in the trace rows, and the rows read back (trace
    // rows, owned rows) lie between them
    std::vector<std::vector<Job>> fw, bw;
    std::vector<int> zlo, zhi;
    rhs_window(S, zlo, zhi);
    build_local_jobs(S, {l}, {0}, fw, bw, {zlo[l]}, {zhi[l]}, {zlo[l]}, {zhi[l]});
    S->hjobs.resize(saved_jobs);
    std::vector<Launch> lf, lb;
    for (auto& v : fw) lf.push_back(push_launch(S, v, PT_CLS_LOCAL));
    for (auto& v : bw) lb.push_back(push_launch(S, v, PT_CLS_LOCAL));
    S->jobs.release();
    if (S->jobs.alloc(S->hjobs.size()) != hipSuccess) {
      rc = fail(PT_ENOMEM, "jobs");
      break;
    }
    if (hipMemcpy(S->jobs.p, S->hjobs.data(), S->hjobs.size() * sizeof(Job), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(rows.p, src.data(), nq * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
      rc = fail(PT_EHIP, "upload extraction jobs");
      break;
    }
    if (launch_zero(Bx.p, (int64_t)nrhs * ld, st) != hipSuccess ||
        launch_identity_rhs(Bx.p, rows.p, nq, NX, ld, st) != hipSuccess) {
      rc = fail(PT_EHIP, "identity rhs");
      break;
    }
    rc = run_local(S, lf, lb, nrhs, ld, Wx.p, Bx.p);
    if (rc != PT_OK) break;
    if (S->green.p) {
      // rows src[k] of this layer's inverse over its owned rows
      std::vector<double2> haz(y.R);
      const std::vector<RowZ> rz = local_rows(S, y);
      for (int r = 0; r < y.R; ++r) haz[r] = d2(rz[r].a);
      if (hipMemcpy(gaz.p, haz.data(), y.R * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess) {
        rc = fail(PT_EHIP, "green scaling");
        break;
      }
      const std::vector<int> gr = green_rows(y);
      for (size_t g = 0; g < gr.size() && rc == PT_OK; ++g) {
        int q = 0;  // the extraction solve's column block of that source row
        while (src[q] != gr[g]) ++q;
        if (launch_pack_green(Wx.p, ld, q, gr[g], y.top_ext, y.n, NX, gax.p, gaz.p,
                              S->green.p + S->green_off[(size_t)l * 4 + g], st) != hipSuccess)
          rc = fail(PT_EHIP, "pack_green");
      }
      if (rc != PT_OK) break;
    }
    // Raw blocks K_{j,k} (slot 4 j' + k' for j, k in rows {0, 1, n, n+1}).  The
    // columns at rows 1 and n come from the solve; the others from Lemma 4 read
    // column-wise through the layer's reciprocity (the extrapolators equal their
    // Dalpha-scaled transposes), with E_up = -u_0 Delta_0^-1, E_dn = -l_{n+1} Sigma_{n+1}^-1:
    //   K_{j,0} = K_{j,1} E_up (j >= 1),      K_{0,0} = E_up (K_{1,0} + I),
    //   K_{j,n+1} = K_{j,n} E_dn (j <= n),    K_{n+1,n+1} = E_dn (K_{n,n+1} + I).
    const int trow[4] = {y.r0, y.r1, y.rn, y.rn1};
    auto kslot = [&](int jj, int kk) { return Kr.p + (size_t)(jj * 4 + kk) * E; };
    auto qof = [&](int row) {
      for (int q = 0; q < nq; ++q)
        if (src[q] == row) return q;
      return -1;
    };
    for (int jj = 0; jj < 4 && rc == PT_OK; ++jj)
      for (int kk : {1, 2})
        if (trow[jj] >= 0 && qof(trow[kk]) >= 0 &&
            launch_pack_block(Wx.p, ld, qof(trow[kk]), trow[jj], NX, 1.0, 0.0, kslot(jj, kk), nullptr, st) !=
                hipSuccess)
          rc = fail(PT_EHIP, "pack_block");
    if (rc == PT_OK && y.top_ext) {
      const double2 up = d2(-S->ucoef[y.rowbase + y.r0]);
      const double2* dinv0 = S->dinv64.p + (size_t)(y.rowbase + y.r0) * E;
      for (int jj : {1, 2, 3})
        if (rc == PT_OK && trow[jj] >= 0 &&
            launch_setup_gemm(kslot(jj, 1), dinv0, kslot(jj, 0), NX, up, 0.0, st) != hipSuccess)
          rc = fail(PT_EHIP, "setup_gemm");
      if (rc == PT_OK && launch_setup_gemm(dinv0, kslot(1, 0), kslot(0, 0), NX, up, 1.0, st) != hipSuccess)
        rc = fail(PT_EHIP, "setup_gemm");
    }
    if (rc == PT_OK && y.bot_ext) {
      const double2 lo = d2(-S->lcoef[y.rowbase + y.rn1]);
      const double2* dinv1 = S->dinv64.p + (size_t)(y.rowbase + y.rn1) * E;
      for (int jj : {0, 1, 2})
        if (rc == PT_OK && trow[jj] >= 0 &&
            launch_setup_gemm(kslot(jj, 2), dinv1, kslot(jj, 3), NX, lo, 0.0, st) != hipSuccess)
          rc = fail(PT_EHIP, "setup_gemm");
      if (rc == PT_OK && launch_setup_gemm(dinv1, kslot(2, 3), kslot(3, 3), NX, lo, 1.0, st) != hipSuccess)
        rc = fail(PT_EHIP, "setup_gemm");
    }
    // pack the signed blocks
    auto slot_of = [&](int row) {
      for (int jj = 0; jj < 4; ++jj)
        if (trow[jj] == row) return jj;
      return -1;
    };
    struct P {
      int type, a, b, trow, srow;
      double sign, shift;
    };
    std::vector<P> packs;
    if (y.top_ext && y.bot_ext) {
      // T_dn = [[K_{n,1}, -K_{n,0}], [K_{n+1,1}, -K_{n+1,0}]]
      packs.push_back({T_DN, 0, 0, y.rn, y.r1, 1, 0});
      packs.push_back({T_DN, 0, 1, y.rn, y.r0, -1, 0});
      packs.push_back({T_DN, 1, 0, y.rn1, y.r1, 1, 0});
      packs.push_back({T_DN, 1, 1, y.rn1, y.r0, -1, 0});
      // T_up = [[-K_{0,n+1}, K_{0,n}], [-K_{1,n+1}, K_{1,n}]]
      packs.push_back({T_UP, 0, 0, y.r0, y.rn1, -1, 0});
      packs.push_back({T_UP, 0, 1, y.r0, y.rn, 1, 0});
      packs.push_back({T_UP, 1, 0, y.r1, y.rn1, -1, 0});
      packs.push_back({T_UP, 1, 1, y.r1, y.rn, 1, 0});
    }
    if (y.bot_ext) {
      // B_up - J0 = [[-K_{n,n+1} - I, K_{n,n}], [-K_{n+1,n+1}, K_{n+1,n}]]
      packs.push_back({B_UP, 0, 0, y.rn, y.rn1, -1, -1});
      packs.push_back({B_UP, 0, 1, y.rn, y.rn, 1, 0});
      packs.push_back({B_UP, 1, 0, y.rn1, y.rn1, -1, 0});
      packs.push_back({B_UP, 1, 1, y.rn1, y.rn, 1, 0});
    }
    if (y.top_ext) {
      // B_dn - J1 = [[K_{0,1}, -K_{0,0}], [K_{1,1}, -K_{1,0} - I]]
      packs.push_back({B_DN, 0, 0, y.r0, y.r1, 1, 0});
      packs.push_back({B_DN, 0, 1, y.r0, y.r0, -1, 0});
      packs.push_back({B_DN, 1, 0, y.r1, y.r1, 1, 0});
      packs.push_back({B_DN, 1, 1, y.r1, y.r0, -1, -1});
    }
    for (const P& pk : packs) {
      if (rc != PT_OK) break;
      const int id = S->bidx[((l * 4 + pk.type) * 2 + pk.a) * 2 + pk.b];
      if (launch_sign_copy(kslot(slot_of(pk.trow), slot_of(pk.srow)), S->blk64.p + (size_t)id * E, NX, pk.sign,
                           pk.shift, st) != hipSuccess)
        rc = fail(PT_EHIP, "pack_block");
    }
    if (hipStreamSynchronize(st) != hipSuccess && rc == PT_OK) rc = fail(PT_EHIP, "extraction sync");
  }
  S->hjobs.resize(saved_jobs);
  Wx.release();
  Bx.release();
  Kr.release();
  rows.release();
  gax.release();
  gaz.release();
  return rc;
}

// Reconstruction jobs that address the volume fields in place (no copies in
// or out of a layer-local field): the owned rows of layer l are rows
// own_start.. of the output u (base 1) and of the sources f (base 2, taken
// with the scale h^2), all with the column stride NZ NX of those fields.  The
// only other rows a reconstruction touches are the extension rows 0 and n+1
// (solution rows 2l and 2l + 1 of a scratch field, base 0) and the forced
// right-hand-side rows 0, 1, n, n+1 (rows 2L + e of the same scratch field,
// one per forcing entry e, written by launch_rec_rhs).  Not built when the
// scratch rows do not fit NZ rows.
void build_direct_reconstruction(pt_solver* S, const std::vector<int>& lo, const std::vector<int>& hi,
                                 const std::vector<int>& zlo, const std::vector<int>& zhi) {
  const int L = S->L, NX = S->NX;
  S->fwd_rec.clear();
  S->bwd_rec2.clear();
  S->rec_direct = false;
  // forcing entries (interface k, segment t_a, layer, local row, sign): as the trace map's
  std::vector<int32_t> hdst, hsrc, hseg;
  std::vector<double> hsg;
  std::map<std::pair<int, int>, int> trow;  // (layer, local row) -> scratch row of its right-hand side
  auto add = [&](int k, int a, int l, int r, double sg) {
    const Layer& y = S->lay[l];
    const int e = (int)hdst.size();
    trow[{l, r}] = 2 * L + e;
    hdst.push_back(2 * L + e);
    const bool owned = r >= y.top_ext && r < y.top_ext + y.n;
    hsrc.push_back(owned ? y.own_start + r - y.top_ext : -1);
    hseg.push_back(k * 2 + a);
    hsg.push_back(sg);
  };
  for (int k = 0; k + 1 < L; ++k) {
    const Layer& up = S->lay[k];
    const Layer& dn = S->lay[k + 1];
    add(k, 0, k, up.rn1, -1.0);  // layer k, bottom interface: - e_{n+1} t_0 + e_n t_1
    add(k, 1, k, up.rn, 1.0);
    add(k, 0, k + 1, dn.r1, 1.0);  // layer k+1, top interface: + e_1 t_0 - e_0 t_1
    add(k, 1, k + 1, dn.r0, -1.0);
  }
  if (2 * L + (int)hdst.size() > S->NZ) return;
  bool bad = false;
  const double h2 = S->h * S->h;
  LocalAddr ad;
  ad.w = [&](size_t q, int r) -> VecRef {
    const Layer& y = S->lay[q];
    if (r >= y.top_ext && r < y.top_ext + y.n) return vr(1, (int64_t)(y.own_start + r - y.top_ext) * NX);
    if (r == y.r0) return vr(0, (int64_t)(2 * q) * NX);
    if (r == y.rn1) return vr(0, (int64_t)(2 * q + 1) * NX);
    bad = true;
    return none();
  };
  ad.b = [&](size_t q, int r) -> VecRef {
    const auto it = trow.find({(int)q, r});
    if (it != trow.end()) return vr(0, (int64_t)it->second * NX);
    const Layer& y = S->lay[q];
    if (r >= y.top_ext && r < y.top_ext + y.n) return vr(2, (int64_t)(y.own_start + r - y.top_ext) * NX);
    bad = true;
    return none();
  };
  ad.s = [&](size_t q, int r) { return trow.count({(int)q, r}) ? 1.0 : h2; };
  std::vector<int> ls(L), rb(L, 0);
  for (int l = 0; l < L; ++l) ls[l] = l;
  std::vector<std::vector<Job>> fw, bw;
  build_local_jobs(S, ls, rb, fw, bw, lo, hi, zlo, zhi, &ad);
  if (bad) return;
  if (!hdst.empty() && (S->rr_dst.alloc(hdst.size()) != hipSuccess || S->rr_src.alloc(hsrc.size()) != hipSuccess ||
                        S->rr_seg.alloc(hseg.size()) != hipSuccess || S->rr_sign.alloc(hsg.size()) != hipSuccess ||
                        hipMemcpy(S->rr_dst.p, hdst.data(), hdst.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
                        hipMemcpy(S->rr_src.p, hsrc.data(), hsrc.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
                        hipMemcpy(S->rr_seg.p, hseg.data(), hseg.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
                        hipMemcpy(S->rr_sign.p, hsg.data(), hsg.size() * 8, hipMemcpyHostToDevice) != hipSuccess))
    return;
  for (auto& v : fw)
    if (!v.empty()) S->fwd_rec.push_back(push_launch(S, v, PT_CLS_LOCAL));
  for (auto& v : bw)
    if (!v.empty()) S->bwd_rec2.push_back(push_launch(S, v, PT_CLS_LOCAL));
  S->n_rec_rhs = (int)hdst.size();
  S->rec_direct = true;
}

// The system closed by extrapolation relations (Section 3.4, Def.
// polarized_out_going), unknowns as in the jump system.  Per interface k the
// rows at row n of layer k and row 1 of layer k+1 are the jump system's (the
// regularised integral equations); the other row of each pair is an
// extrapolation relation with the one-sided extrapolators of Def. extrapolator,
// E_down = -l Sigma_{n+1}^-1 (layer k) and E_up = -u Delta_0^-1 (layer k+1),
// the layers' one-row Schur complements (l, u the couplings of those rows):
//   y_dn(k, n+1) = d_k(n+1) - E_down d_k(n),   y_up(k, 0) = a_k(0) - E_up a_k(1).
// D (eq. splitting_out_going) keeps the couplings within a polarization and R
// the rest, so R's extrapolation rows vanish and its other rows are the jump
// system's R rows.  Since E_down K_{n,j} = K_{n+1,j} for the sources above row n
// (Lemma extrapolator_def), D^-1 = D_jump^-1 T with T the one-step
// extrapolation r_dn(n+1) += E_down r_dn(n), r_up(0) += E_up r_up(1).
// Launches: opX + opX2 (bases 0 = x, 2 = y: the integral rows, the
// extrapolation rows), opRX (y = R x
// on the two rows it has), gsRX (cur = v - R prev: bases 0 = v, 1 = prev,
// 2 = cur; the split planes in the mixed form), tX (T in place on base 2).
void build_extrap_jobs(pt_solver* S) {
  const int L = S->L;
  const double2 one = make_double2(1.0, 0.0);
  std::vector<Job> jx, jx2, jr, jg, jt;
  for (int k = 0; k <= L - 2; ++k) {
    const Layer& ya = S->lay[k];
    const Layer& yb = S->lay[k + 1];
    const cd l = S->lcoef[ya.rowbase + ya.rn1];
    const cd uc = S->ucoef[yb.rowbase + yb.r0];
    const void* Sg = S->dinv(k, ya.rn1);      // Sigma_{n+1}^-1 of layer k
    const void* Dl = S->dinv(k + 1, yb.r0);   // Delta_0^-1 of layer k+1
    // A, row n of the down pair: d_k(n) + a_k(n) - T_dn(k)(d + a)_{k-1} - (B_up(k) - J0) a_k
    {
      Job j = empty_job();
      j.Y = vr(2, S->seg(0, k, 0));
      j.P = vr(0, S->seg(0, k, 0));
      j.alpha = make_double2(-1.0, 0.0);
      if (k >= 1)
        for (int b = 0; b < 2; ++b)
          add_term(j, S->blk_term(k, T_DN, 0, b), vr(0, S->seg(0, k - 1, b)), vr(0, S->seg(1, k - 1, b)), one);
      for (int b = 0; b < 2; ++b) add_term(j, S->blk_term(k, B_UP, 0, b), vr(0, S->seg(1, k, b)));
      jx.push_back(j);
    }
    // A, row 1 of the up pair: a_k(1) + d_k(1) - T_up(k+1)(a + d)_{k+1} - (B_dn(k+1) - J1) d_k
    {
      Job u = empty_job();
      u.Y = vr(2, S->seg(1, k, 1));
      u.P = vr(0, S->seg(1, k, 1));
      u.alpha = make_double2(-1.0, 0.0);
      if (k + 1 <= L - 2)
        for (int b = 0; b < 2; ++b)
          add_term(u, S->blk_term(k + 1, T_UP, 1, b), vr(0, S->seg(1, k + 1, b)), vr(0, S->seg(0, k + 1, b)), one);
      for (int b = 0; b < 2; ++b) add_term(u, S->blk_term(k + 1, B_DN, 1, b), vr(0, S->seg(0, k, b)));
      jx.push_back(u);
    }
    // A, extrapolation rows: d_k(n+1) + l Sigma^-1 d_k(n), a_k(0) + u Delta^-1 a_k(1)
    {
      Job j = empty_job();
      j.Y = vr(2, S->seg(0, k, 1));
      j.P = vr(0, S->seg(0, k, 1));
      j.alpha = d2(l);
      add_term(j, Sg, vr(0, S->seg(0, k, 0)));
      jx2.push_back(j);
      Job u = empty_job();
      u.Y = vr(2, S->seg(1, k, 0));
      u.P = vr(0, S->seg(1, k, 0));
      u.alpha = d2(uc);
      add_term(u, Dl, vr(0, S->seg(1, k, 1)));
      jx2.push_back(u);
    }
    // R rows (0, k, n) and (1, k, 1): -(T_dn(k) a_{k-1} + (B_up(k) - J0) a_k), likewise up
    for (int gs = 0; gs < 2; ++gs) {
      // gs = 0: y = R x (bases 0 = x, 2 = y); gs = 1: cur = v - R prev (0 = v, 1 = prev, 2 = cur)
      const int xin = gs ? 1 : 0;
      auto term = [&](int l_, int type, int a, int b) { return gs ? S->blk_pre(l_, type, a, b) : S->blk_term(l_, type, a, b); };
      // R's rows are -(T a + (B - J) a): y = R x takes alpha -1, cur = v - R prev alpha +1
      const double2 al = make_double2(gs ? 1.0 : -1.0, 0.0);
      Job j = empty_job();
      j.Y = vr(2, S->seg(0, k, 0));
      j.P = gs ? vr(0, S->seg(0, k, 0)) : none();
      j.alpha = al;
      if (k >= 1)
        for (int b = 0; b < 2; ++b) add_term(j, term(k, T_DN, 0, b), vr(xin, S->seg(1, k - 1, b)));
      for (int b = 0; b < 2; ++b) add_term(j, term(k, B_UP, 0, b), vr(xin, S->seg(1, k, b)));
      Job u = empty_job();
      u.Y = vr(2, S->seg(1, k, 1));
      u.P = gs ? vr(0, S->seg(1, k, 1)) : none();
      u.alpha = al;
      if (k + 1 <= L - 2)
        for (int b = 0; b < 2; ++b) add_term(u, term(k + 1, T_UP, 1, b), vr(xin, S->seg(0, k + 1, b)));
      for (int b = 0; b < 2; ++b) add_term(u, term(k + 1, B_DN, 1, b), vr(xin, S->seg(0, k, b)));
      (gs ? jg : jr).push_back(j);
      (gs ? jg : jr).push_back(u);
    }
    // T in place: c_dn(n+1) -= l Sigma^-1 c_dn(n), c_up(0) -= u Delta^-1 c_up(1)
    // (a preconditioner step: the split-bfloat16 planes of the two factors in the mixed form)
    {
      const size_t E = split_block_elems(S->NX);
      const void* Tsg = S->split ? (const void*)(S->xbf.p + (size_t)(2 * k) * E) : Sg;
      const void* Tdl = S->split ? (const void*)(S->xbf.p + (size_t)(2 * k + 1) * E) : Dl;
      Job j = empty_job();
      j.Y = vr(2, S->seg(0, k, 1));
      j.P = j.Y;
      j.alpha = d2(-l);
      add_term(j, Tsg, vr(2, S->seg(0, k, 0)));
      jt.push_back(j);
      Job u = empty_job();
      u.Y = vr(2, S->seg(1, k, 0));
      u.P = u.Y;
      u.alpha = d2(-uc);
      add_term(u, Tdl, vr(2, S->seg(1, k, 1)));
      jt.push_back(u);
    }
  }
  // the integral rows (four blocks each) and the extrapolation rows (one) in
  // separate launches: mixed in one, the long jobs' tiles would set its length
  S->opX = push_launch(S, jx, PT_CLS_OPERATOR);
  S->opX2 = push_launch(S, jx2, PT_CLS_OPERATOR);
  S->opRX = push_launch(S, jr, PT_CLS_OPERATOR);
  S->gsRX = push_launch(S, jg, PT_CLS_REFLECT, true, true);
  S->tX = push_launch(S, jt, PT_CLS_REFLECT, false, S->split);
}

void build_online_jobs(pt_solver* S) {
  const int L = S->L, NX = S->NX;
  S->hjobs.clear();
  // local solves over all layers of the (nrhs, sumR, NX) fields
  {
    std::vector<int> ls(L), rb(L);
    for (int l = 0; l < L; ++l) {
      ls[l] = l;
      rb[l] = S->lay[l].rowbase;
    }
    std::vector<std::vector<Job>> fw, bw;
    build_local_jobs(S, ls, rb, fw, bw);
    S->fwd.clear();
    S->bwd.clear();
    for (auto& v : fw) {
      S->fwd.push_back(push_launch(S, v, PT_CLS_LOCAL));
      index_layers(S, S->fwd.back());
    }
    for (auto& v : bw) S->bwd.push_back(push_launch(S, v, PT_CLS_LOCAL));
    // backward passes that stop at the rows their caller reads: the trace
    // rows 0, 1, n, n+1 (pre-solve) and the owned rows (reconstruction)
    std::vector<int> lo_pre(L), hi_pre(L), lo_rec(L), hi_rec(L);
    for (int l = 0; l < L; ++l) {
      const Layer& y = S->lay[l];
      int lo = y.R, hi = -1;
      for (int r : {y.r0, y.r1, y.rn, y.rn1})
        if (r >= 0) {
          lo = std::min(lo, r);
          hi = std::max(hi, r);
        }
      lo_pre[l] = hi >= 0 ? lo : y.mid;
      hi_pre[l] = hi >= 0 ? hi : y.mid;
      lo_rec[l] = y.top_ext;
      hi_rec[l] = y.top_ext + y.n - 1;
    }
    // pre-solve by the interface Green's functions: w^l(row j) = sum over owned rows
    // of G^l_j h^2 f^l, one job per (layer, trace row) in layer order
    S->green_launch = Launch{};
    S->green_ext = Launch{};
    if (S->green.p) {
      std::vector<Job> js, jext;
      for (int l = 0; l < L; ++l) {
        const Layer& y = S->lay[l];
        const std::vector<int> src = green_rows(y);
        // rows 0 and n+1 from rows 1 and n: w(0) = -u Delta_0^-1 w(1), w(n+1) = -l Sigma_{n+1}^-1 w(n)
        if (y.top_ext) {
          Job j = empty_job();
          j.Y = vr(0, (int64_t)(y.rowbase + y.r0) * NX);
          j.alpha = d2(-S->ucoef[y.rowbase + y.r0]);
          add_term(j, S->dinv(l, y.r0), vr(0, (int64_t)(y.rowbase + y.r1) * NX));
          jext.push_back(j);
        }
        if (y.bot_ext) {
          Job j = empty_job();
          j.Y = vr(0, (int64_t)(y.rowbase + y.rn1) * NX);
          j.alpha = d2(-S->lcoef[y.rowbase + y.rn1]);
          add_term(j, S->dinv(l, y.rn1), vr(0, (int64_t)(y.rowbase + y.rn) * NX));
          jext.push_back(j);
        }
        for (size_t k = 0; k < src.size(); ++k) {
          Job j = empty_job();
          j.Y = vr(0, (int64_t)(y.rowbase + src[k]) * NX);
          add_term(j, S->green.p + S->green_off[(size_t)l * 4 + k], vr(1, (int64_t)(y.rowbase + y.top_ext) * NX));
          j.kw[0] = y.n * NX;
          j.ldm[0] = y.n * NX;
          js.push_back(j);
        }
      }
      S->green_launch = push_launch(S, js, PT_CLS_PRESOLVE);
      index_layers(S, S->green_launch);
      S->green_ext = push_launch(S, jext, PT_CLS_PRESOLVE);
      index_layers(S, S->green_ext);
      // K-split form for wide passes: each (layer, trace row) product split into
      // S_l ranges of owned rows, partial sums in S_l free owned rows per trace
      // row (rows te+2 .. te+2+4 S_l-1, clear of the trace rows), then summed
      std::vector<Job> jsp;
      std::vector<int32_t> hd, hs, hc;
      S->gsum_off.assign(L + 1, 0);
      bool room = true;  // every layer has 4 free owned rows between its trace rows
      for (const Layer& y : S->lay) room = room && (y.n - 3) / 4 >= 1;
      // ranges per layer: at least 8, and enough that a range spans about 256
      // chunks of kNzChunk columns (a tall layer's ranges then keep their
      // nonzero-chunk lists, and no workgroup walks a long chunk sequence),
      // within the room for the partial rows
      auto ranges = [&](const Layer& y) {
        const long chunks = ((long)y.n * NX + kNzChunk - 1) / kNzChunk;
        const int want = (int)std::max<long>(8, (chunks + 255) / 256);
        return std::max(1, std::min(want, (y.n - 3) / 4));
      };
      // one nonzero-chunk list per (layer, owned-row range), shared by the
      // layer's trace rows: the products skip the chunks where every source
      // column is zero (compact sources leave most of a layer's inputs zero)
      std::vector<int64_t> nzo;
      std::vector<int32_t> nzk;
      S->nz_off.assign(L + 1, 0);
      int stride = 1;
      for (int l = 0; l < L && room; ++l) {
        const Layer& y = S->lay[l];
        const int ns = ranges(y), per = (y.n + ns - 1) / ns;
        for (int p = 0; p < ns; ++p) {
          const int r_lo = p * per, r_hi = std::min(y.n, r_lo + per);
          if (r_lo >= r_hi) continue;
          nzo.push_back((int64_t)(y.rowbase + y.top_ext + r_lo) * NX);
          nzk.push_back((r_hi - r_lo) * NX);
          stride = std::max(stride, 1 + ((r_hi - r_lo) * NX + kNzChunk - 1) / kNzChunk);
        }
        S->nz_off[l + 1] = (int)nzo.size();
      }
      S->nz_stride = stride;
      // a list must fit the kernel's LDS copy: longer ranges keep every chunk
      const bool lists = room && stride - 1 <= kKlMax;
      if (lists && (S->nz_list.alloc(nzo.size() * (size_t)stride) != hipSuccess ||
                   S->nz_in_off.alloc(nzo.size()) != hipSuccess || S->nz_in_k.alloc(nzk.size()) != hipSuccess ||
                   hipMemcpy(S->nz_in_off.p, nzo.data(), nzo.size() * sizeof(int64_t), hipMemcpyHostToDevice) !=
                       hipSuccess ||
                   hipMemcpy(S->nz_in_k.p, nzk.data(), nzk.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
                       hipSuccess))
        room = false;  // no device memory for the lists: the unsplit form serves every width
      for (int l = 0; l < L && room; ++l) {
        const Layer& y = S->lay[l];
        const std::vector<int> src = green_rows(y);
        const int ns = ranges(y);  // rows te+2 .. te+1+2 ns stay below row n-1
        const int per = (y.n + ns - 1) / ns;
        for (size_t k = 0; k < src.size(); ++k) {
          const int prow0 = y.rowbase + y.top_ext + 2 + (int)k * ns;
          int cnt = 0;
          for (int p = 0; p < ns; ++p) {
            const int r_lo = p * per, r_hi = std::min(y.n, r_lo + per);
            if (r_lo >= r_hi) continue;
            Job j = empty_job();
            j.Y = vr(0, (int64_t)(prow0 + cnt) * NX);
            add_term(j, S->green.p + S->green_off[(size_t)l * 4 + k] + (size_t)r_lo * NX,
                     vr(1, (int64_t)(y.rowbase + y.top_ext + r_lo) * NX));
            j.kw[0] = (r_hi - r_lo) * NX;
            j.ldm[0] = y.n * NX;
            if (S->nz_list.p) j.kl = S->nz_list.p + (size_t)(S->nz_off[l] + cnt) * stride;
            jsp.push_back(j);
            ++cnt;
          }
          hd.push_back(y.rowbase + src[k]);
          hs.push_back(prow0);
          hc.push_back(cnt);
        }
        S->gsum_off[l + 1] = (int)hd.size();
      }
      if (room) {
        S->green_split = push_launch(S, jsp, PT_CLS_PRESOLVE);
        S->green_split.klist = S->nz_list.p != nullptr;
        index_layers(S, S->green_split);
      }
      if (!room) {
        S->green_split = Launch{};
      } else if (S->gsum_dst.alloc(hd.size()) != hipSuccess || S->gsum_src.alloc(hd.size()) != hipSuccess ||
          S->gsum_cnt.alloc(hd.size()) != hipSuccess ||
          hipMemcpy(S->gsum_dst.p, hd.data(), hd.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(S->gsum_src.p, hs.data(), hs.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(S->gsum_cnt.p, hc.data(), hc.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
        S->green_split = Launch{};  // the unsplit form then serves every width
      }
    }
    S->bwd_pre.clear();
    S->bwd_rec.clear();
    S->fwd_win.clear();
    std::vector<int> zlo, zhi;
    rhs_window(S, zlo, zhi);
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<std::vector<Job>> f2, b2;
      build_local_jobs(S, ls, rb, f2, b2, pass == 0 ? lo_pre : lo_rec, pass == 0 ? hi_pre : hi_rec, zlo, zhi);
      if (pass == 0)
        for (auto& v : f2) {
          S->fwd_win.push_back(push_launch(S, v, PT_CLS_LOCAL));
          index_layers(S, S->fwd_win.back());
        }
      auto& dst = pass == 0 ? S->bwd_pre : S->bwd_rec;
      for (auto& v : b2)
        if (!v.empty()) {
          dst.push_back(push_launch(S, v, PT_CLS_LOCAL));
          index_layers(S, dst.back());
        }
    }
    build_direct_reconstruction(S, lo_rec, hi_rec, zlo, zhi);
  }
  if (L < 2) return;
  const double2 one = make_double2(1.0, 0.0);
  // Gauss-Seidel sweep step s: bases 0 = r (unused), 1 = previous iterate, 2 = current iterate.
  //   d_k += T_dn(k) (d_{k-1} + a^prev_{k-1}),  k = s
  //   a_k += T_up(k+1) (a_{k+1} + d^prev_{k+1}), k = L-2-s
  S->sweep.clear();
  for (int s = 1; s <= L - 2; ++s) {
    std::vector<Job> js;
    const int kd = s, ku = L - 2 - s;
    for (int a = 0; a < 2; ++a) {
      Job j = empty_job();
      j.Y = vr(2, S->seg(0, kd, a));
      j.P = j.Y;
      for (int b = 0; b < 2; ++b)
        add_term(j, S->blk_pre(kd, T_DN, a, b), vr(2, S->seg(0, kd - 1, b)), vr(1, S->seg(1, kd - 1, b)), one);
      js.push_back(j);
    }
    for (int a = 0; a < 2; ++a) {
      Job j = empty_job();
      j.Y = vr(2, S->seg(1, ku, a));
      j.P = j.Y;
      for (int b = 0; b < 2; ++b)
        add_term(j, S->blk_pre(ku + 1, T_UP, a, b), vr(2, S->seg(1, ku + 1, b)), vr(1, S->seg(0, ku + 1, b)), one);
      js.push_back(j);
    }
    S->sweep.push_back(push_launch(S, js, PT_CLS_SWEEP, true, true));
  }
  // reflection terms of a Gauss-Seidel pass: cur = r + (B_up - J0) a^prev, r + (B_dn - J1) d^prev
  {
    std::vector<Job> js;
    for (int k = 0; k <= L - 2; ++k)
      for (int a = 0; a < 2; ++a) {
        Job j = empty_job();
        j.Y = vr(2, S->seg(0, k, a));
        j.P = vr(0, S->seg(0, k, a));
        for (int b = 0; b < 2; ++b) add_term(j, S->blk_pre(k, B_UP, a, b), vr(1, S->seg(1, k, b)));
        js.push_back(j);
        Job u = empty_job();
        u.Y = vr(2, S->seg(1, k, a));
        u.P = vr(0, S->seg(1, k, a));
        for (int b = 0; b < 2; ++b) add_term(u, S->blk_pre(k + 1, B_DN, a, b), vr(1, S->seg(0, k, b)));
        js.push_back(u);
      }
    S->bterm = push_launch(S, js, PT_CLS_REFLECT, true, true);
  }
  // polarized operator y = A x (bases 0 = x, 2 = y) and y = R x.  With dense
  // float64 blocks A is applied in the extrapolated form (Lemma 4): the first
  // launch forms the rows n of the down traces and the rows 1 of the up traces
  // with their four blocks each; the second gets each pair's other row from it
  // through the layer's one-row Schur complement (a stored factor),
  //   y_dn(k, n+1) = d_k(n+1) + l Sigma_{n+1}^-1 [(d_k(n) - y_dn(k, n)) + ((1 + l) / l) a_k(n)]
  //   y_up(k, 0)   = a_k(0)   + u Delta_0^-1   [(a_k(1) - y_up(k, 1)) + ((1 + u) / u) d_k(n+1)]
  // (l, u: the couplings of those rows; -1 in the paper's A scaling, where the
  // second terms vanish): 10 block reads per interface instead of 16.
  const bool extrap = !S->use_plr;
  S->opA2 = Launch{};
  for (int which = 0; which < 2; ++which) {
    std::vector<Job> js, js2;
    const bool isA = which == 0;
    for (int k = 0; k <= L - 2; ++k)
      for (int a = 0; a < 2; ++a) {
        const bool second_dn = isA && extrap && a == 1;  // row n+1 of the down pair
        const bool second_up = isA && extrap && a == 0;  // row 0 of the up pair
        if (second_dn) {
          const Layer& y = S->lay[k];
          const cd l = S->lcoef[y.rowbase + y.rn1];
          Job j = empty_job();
          j.Y = vr(2, S->seg(0, k, 1));
          j.P = vr(0, S->seg(0, k, 1));
          j.alpha = d2(l);
          add_term(j, S->dinv(k, y.rn1), vr(0, S->seg(0, k, 0)), vr(2, S->seg(0, k, 0)), make_double2(-1.0, 0.0));
          const cd one_l = cmk(1.0 + l.re, l.im);
          if (one_l.re != 0.0 || one_l.im != 0.0)
            add_term(j, S->dinv(k, y.rn1), none(), vr(0, S->seg(1, k, 0)), cdiv_h(one_l, l));
          js2.push_back(j);
        }
        if (second_up) {
          const Layer& y = S->lay[k + 1];
          const cd uc = S->ucoef[y.rowbase + y.r0];
          Job u = empty_job();
          u.Y = vr(2, S->seg(1, k, 0));
          u.P = vr(0, S->seg(1, k, 0));
          u.alpha = d2(uc);
          add_term(u, S->dinv(k + 1, y.r0), vr(0, S->seg(1, k, 1)), vr(2, S->seg(1, k, 1)), make_double2(-1.0, 0.0));
          const cd one_u = cmk(1.0 + uc.re, uc.im);
          if (one_u.re != 0.0 || one_u.im != 0.0)
            add_term(u, S->dinv(k + 1, y.r0), none(), vr(0, S->seg(0, k, 1)), cdiv_h(one_u, uc));
          js2.push_back(u);
        }
        if (!second_dn) {
        // down rows: d_k - T_dn(k)(d_{k-1} + a_{k-1}) - (B_up(k) - J0) a_k
        Job j = empty_job();
        j.Y = vr(2, S->seg(0, k, a));
        j.P = isA ? vr(0, S->seg(0, k, a)) : none();
        j.alpha = make_double2(-1.0, 0.0);
        if (k >= 1)
          for (int b = 0; b < 2; ++b)
            add_term(j, S->blk_term(k, T_DN, a, b), isA ? vr(0, S->seg(0, k - 1, b)) : vr(0, S->seg(1, k - 1, b)),
                     isA ? vr(0, S->seg(1, k - 1, b)) : none(), one);
        for (int b = 0; b < 2; ++b) add_term(j, S->blk_term(k, B_UP, a, b), vr(0, S->seg(1, k, b)));
        js.push_back(j);
        }
        if (second_up) continue;
        // up rows: a_k - T_up(k+1)(a_{k+1} + d_{k+1}) - (B_dn(k+1) - J1) d_k
        Job u = empty_job();
        u.Y = vr(2, S->seg(1, k, a));
        u.P = isA ? vr(0, S->seg(1, k, a)) : none();
        u.alpha = make_double2(-1.0, 0.0);
        if (k + 1 <= L - 2)
          for (int b = 0; b < 2; ++b)
            add_term(u, S->blk_term(k + 1, T_UP, a, b), isA ? vr(0, S->seg(1, k + 1, b)) : vr(0, S->seg(0, k + 1, b)),
                     isA ? vr(0, S->seg(0, k + 1, b)) : none(), one);
        for (int b = 0; b < 2; ++b) add_term(u, S->blk_term(k + 1, B_DN, a, b), vr(0, S->seg(0, k, b)));
        js.push_back(u);
      }
    if (isA) {
      S->opA = push_launch(S, js, PT_CLS_OPERATOR, true);
      if (!js2.empty()) S->opA2 = push_launch(S, js2, PT_CLS_OPERATOR);
    } else {
      S->opR = push_launch(S, js, PT_CLS_OPERATOR, true);
    }
  }
  if (S->opt.closure == 1) build_extrap_jobs(S);
  (void)NX;
}

pt_status alloc_online(pt_solver* S) {
  const int nr = S->opt.max_nrhs;
  const int m = S->opt.maxit;
  const size_t loc = (size_t)nr * S->sumR * S->NX;
  const size_t vol = (size_t)nr * S->NZ * S->NX;
  const size_t tr = (size_t)nr * std::max<int64_t>(S->Nt, 1);
  HIPCHK(S->W.alloc(loc));
  HIPCHK(S->Bw.alloc(loc));
  HIPCHK(S->fio.alloc(vol));
  HIPCHK(S->uio.alloc(vol));
  HIPCHK(S->nrm.alloc(nr));  // per-source norms (also the finiteness check of the one-layer solve)
  if (S->L >= 2) {
    HIPCHK(S->s.alloc(tr));
    HIPCHK(S->V.alloc(tr * (m + 1)));
    HIPCHK(S->Z.alloc(tr * m));
    HIPCHK(S->U1.alloc(tr));
    HIPCHK(S->U2.alloc(tr));
    HIPCHK(S->tmp.alloc(tr));
    HIPCHK(S->zeros.alloc(tr));
    HIPCHK(S->x.alloc(tr));
    HIPCHK(hipMemset(S->zeros.p, 0, tr * sizeof(double2)));
    HIPCHK(S->hbuf.alloc((size_t)(m + 1) * nr));
    HIPCHK(S->hacc.alloc((size_t)(m + 1) * nr));
    HIPCHK(S->Hc.alloc((size_t)nr * (m + 1) * m));
    HIPCHK(S->sn.alloc((size_t)nr * m));
    HIPCHK(S->g.alloc((size_t)nr * (m + 1)));
    HIPCHK(S->y.alloc((size_t)nr * m));
    HIPCHK(S->cs.alloc((size_t)nr * m));
    HIPCHK(S->est.alloc(nr));
    HIPCHK(S->beta.alloc(nr));
    HIPCHK(S->iters.alloc(nr));
    HIPCHK(S->done.alloc(nr));
    HIPCHK(hipHostMalloc((void**)&S->h_done, (size_t)nr * sizeof(int32_t), hipHostMallocDefault));
    // k-slice partial tiles of the split-bfloat16 launches (sized for the largest)
    if (S->split) {
      // the slice count depends on nrhs: size for the worst right-hand-side count
      size_t need = 0;
      std::vector<const Launch*> ls{&S->bterm};
      for (const Launch& Lc : S->sweep) ls.push_back(&Lc);
      for (const Launch* Lc : ls)
        for (int r = 1; r <= nr; ++r) {
          const int ks = split_kslices(Lc->njobs, S->NX, r);
          if (ks > 1) need = std::max(need, (size_t)ks * Lc->njobs * r * S->NX);
        }
      HIPCHK(S->part.alloc(need));
    }
    if (S->use_plr) HIPCHK(S->plr_part.alloc(kPlrPartEntries));
    // k-slices over workgroups of the MFMA block applies (more than 4 sources, dense blocks): up
    // to kMfmaSlicesMax partial tiles per output entry of the launch the tuner times for each
    // class (sweep steps, reflection terms, operator A; the local solves' passes too, which the
    // tuner does not slice but a loaded tuning cache may); split launches have their own workspace
    if (!S->use_plr && nr > 4) {
      int nj = 0;
      if (!S->fwd.empty()) nj = S->fwd[S->fwd.size() / 2].njobs;
      if (!S->sweep.empty() && !S->sweep[S->sweep.size() / 2].split)
        nj = std::max(nj, S->sweep[S->sweep.size() / 2].njobs);
      if (!S->bterm.split) nj = std::max(nj, S->bterm.njobs);
      nj = std::max(nj, S->opA.njobs);
      if (nj > 0) HIPCHK(S->mpart.alloc((size_t)kMfmaSlicesMax * nj * nr * S->NX));
    }
    // source-to-layer activity tables
    const int L = S->L;
    std::vector<int32_t> rl(S->sumR), os(L), no(L);
    for (int l = 0; l < L; ++l) {
      for (int r = 0; r < S->lay[l].R; ++r) rl[S->lay[l].rowbase + r] = l;
      os[l] = S->lay[l].own_start;
      no[l] = S->lay[l].n;
    }
    HIPCHK(S->row_layer.alloc(S->sumR));
    HIPCHK(S->lay_own_start.alloc(L));
    HIPCHK(S->lay_n_own.alloc(L));
    HIPCHK(hipMemcpy(S->row_layer.p, rl.data(), rl.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S->lay_own_start.p, os.data(), L * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S->lay_n_own.p, no.data(), L * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(S->act.alloc((size_t)L * nr));
    HIPCHK(S->slot_rhs.alloc((size_t)L * nr));
    HIPCHK(S->rhs_slot.alloc((size_t)L * nr));
    HIPCHK(hipHostMalloc((void**)&S->h_act, (size_t)L * nr * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&S->h_slot, (size_t)2 * L * nr * sizeof(int32_t), hipHostMallocDefault));
  }
  return PT_OK;
}

// ---------------------------------------------------------------------------
// online stages
// ---------------------------------------------------------------------------
// Gauss-Seidel preconditioner (Alg. 4): z = u^{n_it}, u^0 = 0,
// u^{i+1} = D^-1 (v - R u^i), each pass fused into one reflection launch and
// L-2 sweep launches.
pt_status precondition(pt_solver* S, const double2* v, double2* z, int nrhs) {
  const int nit = S->opt.gs_iters;
  const int64_t n = (int64_t)nrhs * S->Nt;
  const int64_t ld = S->Nt;
  if (nit == 0) {
    GPU(S, launch_copy(z, v, n, st_));
    return PT_OK;
  }
  double2* prev = S->zeros.p;
  for (int p = 1; p <= nit; ++p) {
    double2* cur = (p == nit) ? z : ((p % 2) ? S->U1.p : S->U2.p);
    Bases b{{const_cast<double2*>(v), prev, cur, nullptr}};
    if (p == 1) {
      GPU(S, launch_copy(cur, v, n, st_));
    } else {
      PTCHK(run_apply(S, S->bterm, nrhs, ld, b));
    }
    for (const Launch& Lc : S->sweep) PTCHK(run_apply(S, Lc, nrhs, ld, b));
    prev = cur;
  }
  return PT_OK;
}

// D^-1 of the extrapolation closure: the one-step extrapolation T, then the
// jump system's sweeps (no previous iterate: base 1 = zeros)
pt_status dinv_extrap_inplace(pt_solver* S, double2* c, int nrhs) {
  Bases b{{nullptr, S->zeros.p, c, nullptr}};
  PTCHK(run_apply(S, S->tX, nrhs, S->Nt, b));
  for (const Launch& Lc : S->sweep) PTCHK(run_apply(S, Lc, nrhs, S->Nt, b));
  return PT_OK;
}

// Gauss-Seidel on the extrapolation splitting (Alg. 4): u^{p} = D^-1 (v - R u^{p-1}), u^0 = 0
pt_status precondition_extrap(pt_solver* S, const double2* v, double2* z, int nrhs) {
  const int nit = S->opt.gs_iters;
  const int64_t n = (int64_t)nrhs * S->Nt;
  if (nit == 0) {
    GPU(S, launch_copy(z, v, n, st_));
    return PT_OK;
  }
  const double2* prev = nullptr;
  for (int p = 1; p <= nit; ++p) {
    double2* cur = (p == nit) ? z : ((p % 2) ? S->U1.p : S->U2.p);
    GPU(S, launch_copy(cur, v, n, st_));  // rows R does not touch keep v
    if (prev) {
      Bases b{{const_cast<double2*>(v), const_cast<double2*>(prev), cur, nullptr}};
      PTCHK(run_apply(S, S->gsRX, nrhs, S->Nt, b));
    }
    PTCHK(dinv_extrap_inplace(S, cur, nrhs));
    prev = cur;
  }
  return PT_OK;
}

pt_status system_A(pt_solver* S, const double2* x, double2* y, int nrhs) {
  if (S->opt.closure == 1) return apply_op(S, S->opX, x, y, nrhs);
  return apply_op(S, S->opA, x, y, nrhs);
}

pt_status system_M(pt_solver* S, const double2* v, double2* z, int nrhs) {
  return S->opt.closure == 1 ? precondition_extrap(S, v, z, nrhs) : precondition(S, v, z, nrhs);
}

pt_status apply_dinv(pt_solver* S, const double2* v, double2* z, int nrhs) {
  GPU(S, launch_copy(z, v, (int64_t)nrhs * S->Nt, st_));
  Bases b{{const_cast<double2*>(v), S->zeros.p, z, nullptr}};
  for (const Launch& Lc : S->sweep) PTCHK(run_apply(S, Lc, nrhs, S->Nt, b));
  return PT_OK;
}

pt_status apply_op(pt_solver* S, const Launch& op, const double2* x, double2* y, int nrhs) {
  Bases b{{const_cast<double2*>(x), nullptr, y, nullptr}};
  PTCHK(run_apply(S, op, nrhs, S->Nt, b));
  // A in the extrapolated form: the second rows of each pair from the first
  if (&op == &S->opA && S->opA2.njobs > 0) PTCHK(run_apply(S, S->opA2, nrhs, S->Nt, b));
  if (&op == &S->opX) PTCHK(run_apply(S, S->opX2, nrhs, S->Nt, b));
  return PT_OK;
}

// Newton potentials w^l = (A^l)^-1 h^2 f^l of every layer into S->W
// Green's-function pre-solve for a pass of `cols` columns: forced on, or (auto)
// while the streaming kernel takes it (<= 4 columns: one HBM pass over the
// Green's functions beats ~R dependent launches; with more columns the MFMA
// form re-reads them per k chunk and the line-by-line solve is as fast)
bool use_green(const pt_solver* S, int cols) {
  return S->green.p && (S->opt.presolve == 1 || cols <= 4 || S->green_split.njobs > 0);
}

// w^l at the trace rows of layers la..lb from the Green's functions: K-split
// products (each kept row's product over up to 8 ranges of owned rows, so
// both the streaming and the MFMA form get enough workgroups to stream the
// Green's functions), a row sum, then rows 0 and n+1 by extrapolation; one
// launch of whole row blocks when a layer has no room for the partial rows
pt_status green_presolve(pt_solver* S, int la, int lb, int cols, int64_t ld) {
  Bases b{{S->W.p, S->Bw.p, nullptr, nullptr}};
  const Launch ext = layer_range(S, S->green_ext, la, lb);
  if (S->green_split.njobs == 0) {
    const Launch sub = layer_range(S, S->green_launch, la, lb);
    if (sub.njobs > 0) PTCHK(run_apply(S, sub, cols, ld, b));
    if (ext.njobs > 0) PTCHK(run_apply(S, ext, cols, ld, b));
    return PT_OK;
  }
  // the MFMA form (> 4 columns) walks fresh nonzero-chunk lists; the streaming
  // form reads every chunk (the skipped ones would add zeros) and no list is made
  const bool lists = cols > 4 && S->green_split.klist;
  const Launch sub = layer_range(S, S->green_split, la, lb);
  const int n0 = S->nz_off[la], n1 = S->nz_off[lb + 1];
  if (lists)
    GPU(S, launch_nonzero_chunks(S->Bw.p, ld, cols, S->nz_in_off.p + n0, S->nz_in_k.p + n0, n1 - n0,
                                 S->nz_list.p + (size_t)n0 * S->nz_stride, S->nz_stride, st_));
  if (sub.njobs > 0) PTCHK(run_apply(S, sub, cols, ld, b));
  if (S->prof && !S->rec && lists && sub.njobs > 0 && !S->pend.empty()) {
    // count what the launch streamed: the chunks its lists kept
    std::vector<int32_t> h((size_t)(n1 - n0) * S->nz_stride);
    HIPCHK(hipMemcpyAsync(h.data(), S->nz_list.p + (size_t)n0 * S->nz_stride, h.size() * sizeof(int32_t),
                          hipMemcpyDeviceToHost, S->st));
    HIPCHK(hipStreamSynchronize(S->st));
    double mat = 0, vec = 0;
    const double n = S->NX;
    for (int i = 0; i < sub.njobs; ++i) {
      const Job& j = S->hjobs[sub.job0 + i];
      const int64_t e = (j.kl - S->nz_list.p) / S->nz_stride - n0;
      const double k = std::min((double)j.kw[0], (double)h[(size_t)e * S->nz_stride] * kNzChunk);
      mat += n * k;
      vec += k + n;  // inputs of the kept chunks, output rows
    }
    ProfPending& pp = S->pend.back();
    pp.bytes = mat * 16.0 + vec * cols * 16.0;
    pp.flops = 8.0 * mat * cols;
  }
  const int e0 = S->gsum_off[la], e1 = S->gsum_off[lb + 1];
  GPU(S, launch_sum_rows(S->W.p, ld, S->NX, S->gsum_dst.p + e0, S->gsum_src.p + e0, S->gsum_cnt.p + e0, e1 - e0,
                         cols, st_));
  if (ext.njobs > 0) PTCHK(run_apply(S, ext, cols, ld, b));
  return PT_OK;
}

pt_status newton(pt_solver* S, const double2* f, int nrhs) {
  GPU(S, launch_scatter_source(f, S->Bw.p, S->rowmap.p, S->sumR, S->NZ, S->NX, nrhs, S->h * S->h, st_));
  if (use_green(S, nrhs)) return green_presolve(S, 0, S->L - 1, nrhs, (int64_t)S->sumR * S->NX);
  return run_local(S, S->fwd_win, S->bwd_pre, nrhs, (int64_t)S->sumR * S->NX, S->W.p, S->Bw.p);
}

// all sources vanish: s = 0
pt_status fail_zero(pt_solver* S, double2* s, int nrhs) {
  GPU(S, launch_zero(s, (int64_t)nrhs * S->Nt, st_));
  return PT_OK;
}

// Pre-solve (Alg. 2) restricted to the layers each source touches: f^l = 0
// gives w^l = 0, so the sources active in layer l are packed into column
// slots 0..m-1 of that layer (m = the largest count over layers) and the
// local solves run on m columns instead of nrhs.  The trace right-hand side
// takes slot values back, zero for layers a source does not touch.  A source
// touches a layer where its largest magnitude exceeds 2^-80 of its largest
// magnitude anywhere: what is skipped is at most 2^-80 sqrt(R NX) of ||f||,
// far below float64 rounding of the result (smooth sources such as Gaussians
// stay nonzero in float64 tens of widths from their centre).
constexpr double kTouchRel2 = 0x1p-160;  // (2^-80)^2, on squared magnitudes

// First half: the largest source magnitude of every (source, layer) to the
// host (S->h_act); the second half reads it once the stream has got there.
pt_status trace_rhs_begin(pt_solver* S, const double2* f, int nrhs) {
  const int L = S->L;
  GPU(S, launch_source_activity(f, S->act.p, S->lay_own_start.p, S->lay_n_own.p, L, S->NZ, S->NX, nrhs, st_));
  GPU(S, hipMemcpyAsync(S->h_act, S->act.p, (size_t)nrhs * L * sizeof(double), hipMemcpyDeviceToHost, st_));
  return PT_OK;
}

// Second half: slot tables from S->h_act, the pre-solve and the gather.  The
// slot tables are uploaded from pinned memory the next call rewrites
// (*uploads set): the caller lets the stream pass the uploads before that.
pt_status trace_rhs_end(pt_solver* S, const double2* f, double2* s, int nrhs, bool* uploads) {
  const int L = S->L;
  *uploads = false;
  int32_t* slot_rhs = S->h_slot;                       // [l][j]
  int32_t* rhs_slot = S->h_slot + (size_t)L * nrhs;    // [r][l]
  std::vector<int> cnt(L, 0);
  for (int r = 0; r < nrhs; ++r) {
    const double* a = S->h_act + (size_t)r * L;
    double mx = 0.0;
    bool finite = true;
    for (int l = 0; l < L; ++l) {
      finite = finite && std::isfinite(a[l]);
      mx = std::max(mx, a[l]);
    }
    for (int l = 0; l < L; ++l) {
      // NaN or Inf anywhere in a source: every layer, so the solve sees and reports it
      const bool touch = !finite || (mx > 0.0 && a[l] > kTouchRel2 * mx);
      rhs_slot[(size_t)r * L + l] = touch ? cnt[l]++ : -1;
    }
  }
  const int m = *std::max_element(cnt.begin(), cnt.end());
  // the contiguous layer range holding every touched layer: local solves run there only
  int la = L, lb = -1;
  for (int l = 0; l < L; ++l)
    if (cnt[l] > 0) {
      la = std::min(la, l);
      lb = std::max(lb, l);
    }
  if (m >= nrhs && la == 0 && lb == L - 1) {  // every layer sees every source: the dense pre-solve
    S->last_slots = nrhs;
    PTCHK(newton(S, f, nrhs));
    GPU(S, launch_trace_map(S->W.p, s, nullptr, S->g_seg.p, S->g_row.p, nullptr, S->n_gather, 0, S->sumR, S->NX,
                            S->Nt, nrhs, 0, st_));
    return PT_OK;
  }
  S->last_slots = m;
  if (m == 0) return fail_zero(S, s, nrhs);
  for (size_t e = 0; e < (size_t)L * m; ++e) slot_rhs[e] = -1;
  for (int r = 0; r < nrhs; ++r)
    for (int l = 0; l < L; ++l) {
      const int j = rhs_slot[(size_t)r * L + l];
      if (j >= 0) slot_rhs[(size_t)l * m + j] = r;
    }
  *uploads = true;
  GPU(S, hipMemcpyAsync(S->slot_rhs.p, slot_rhs, (size_t)L * m * sizeof(int32_t), hipMemcpyHostToDevice, st_));
  GPU(S, hipMemcpyAsync(S->rhs_slot.p, rhs_slot, (size_t)nrhs * L * sizeof(int32_t), hipMemcpyHostToDevice, st_));
  const int64_t ld = (int64_t)S->sumR * S->NX;
  GPU(S, launch_scatter_slots(f, S->Bw.p, S->rowmap.p, S->row_layer.p, S->slot_rhs.p, m, S->sumR, S->NZ, S->NX,
                              S->h * S->h, st_));
  if (use_green(S, m)) {
    PTCHK(green_presolve(S, la, lb, m, ld));
  } else {
    PTCHK(run_local_layers(S, S->fwd_win, S->bwd_pre, la, lb, m, ld, S->W.p, S->Bw.p));
  }
  GPU(S, launch_gather_slots(S->W.p, s, S->g_seg.p, S->g_row.p, S->row_layer.p, S->rhs_slot.p, S->n_gather, L,
                             S->sumR, S->NX, S->Nt, nrhs, st_));
  return PT_OK;
}

pt_status trace_rhs(pt_solver* S, const double2* f, double2* s, int nrhs) {
  PTCHK(trace_rhs_begin(S, f, nrhs));
  HIPCHK(hipStreamSynchronize(S->st));
  bool uploads = false;
  PTCHK(trace_rhs_end(S, f, s, nrhs, &uploads));
  // the pinned slot tables are rewritten by the next call: finish their uploads first
  if (uploads) HIPCHK(hipStreamSynchronize(S->st));
  return PT_OK;
}

pt_status reconstruct(pt_solver* S, const double2* f, const double2* x, double2* u, int nrhs) {
  const uintptr_t nb = (uintptr_t)nrhs * S->NZ * S->NX * sizeof(double2);
  const uintptr_t fa = reinterpret_cast<uintptr_t>(f), ua = reinterpret_cast<uintptr_t>(u);
  const bool overlap = fa < ua + nb && ua < fa + nb;  // u written in place while f is read: keep them apart
  if (S->rec_direct && !overlap && (x || S->n_rec_rhs == 0)) {
    const int64_t ld = (int64_t)S->NZ * S->NX;
    if (S->n_rec_rhs > 0)
      GPU(S, launch_rec_rhs(S->W.p, f, x, S->rr_dst.p, S->rr_src.p, S->rr_seg.p, S->rr_sign.p, S->n_rec_rhs, S->NX, ld,
                            S->Nt, (int64_t)2 * (S->L - 1) * S->NX, S->h * S->h, nrhs, st_));
    Bases b{{S->W.p, u, const_cast<double2*>(f), nullptr}};
    for (const Launch& Lc : S->fwd_rec) PTCHK(run_apply(S, Lc, nrhs, ld, b));
    for (const Launch& Lc : S->bwd_rec2) PTCHK(run_apply(S, Lc, nrhs, ld, b));
    return PT_OK;
  }
  GPU(S, launch_scatter_source(f, S->Bw.p, S->rowmap.p, S->sumR, S->NZ, S->NX, nrhs, S->h * S->h, st_));
  if (S->L >= 2)
    GPU(S, launch_trace_map(S->Bw.p, nullptr, x, S->f_seg.p, S->f_row.p, S->f_sign.p, S->n_force, 1, S->sumR, S->NX,
                            S->Nt, nrhs, (int64_t)2 * (S->L - 1) * S->NX, st_));
  PTCHK(run_local(S, S->fwd_win, S->bwd_rec, nrhs, (int64_t)S->sumR * S->NX, S->W.p, S->Bw.p));
  GPU(S, launch_gather_owned(S->W.p, u, S->rowmap.p, S->sumR, S->NZ, S->NX, nrhs, st_));
  return PT_OK;
}

// Launch iteration j of a GMRES solve with nrhs sources from its captured
// graph, capturing it on first use.  Capture failure switches the solver to
// plain launches for good (the iteration is then run directly).
template <typename F>
pt_status run_graph(pt_solver* S, int nrhs, int j, double tol, F&& iteration) {
  const auto key = std::make_pair(nrhs, j);
  auto it = S->graphs.find(key);
  if (it == S->graphs.end()) {
    (void)tol;
    if (hipStreamBeginCapture(S->st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      S->graph_failed = true;
      return iteration(j);
    }
    const pt_status rc = iteration(j);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(S->st, &g);
    if (rc != PT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    hipGraphExec_t ex = nullptr;
    if (ec != hipSuccess || !g || hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      S->graph_failed = true;
      return iteration(j);
    }
    (void)hipGraphDestroy(g);
    it = S->graphs.emplace(key, ex).first;
  }
  HIPCHK(hipGraphLaunch(it->second, S->st));
  return PT_OK;
}

void drop_graphs(pt_solver* S) {
  for (auto& kv : S->graphs) (void)hipGraphExecDestroy(kv.second);
  S->graphs.clear();
}

// Flexible GMRES (right preconditioning, classical Gram-Schmidt applied twice,
// x0 = 0, no restart) on A x = s for nrhs independent right-hand sides, in
// three parts: the start (v_0 = s / ||s||), iteration j (which leaves the
// per-source convergence flags in S->h_done once the stream has got there)
// and the end (x from the least-squares solutions).
pt_status fgmres_begin(pt_solver* S, int nrhs, bool learned) {
  const int64_t N = S->Nt;
  const int m = S->opt.maxit;
  GPU(S, launch_knorm(S->s.p, S->beta.p, nrhs, N, st_));
  GPU(S, launch_kscale(S->V.p, S->s.p, S->beta.p, nrhs, N, st_));
  GPU(S, launch_kinit(S->g.p, S->beta.p, S->done.p, S->iters.p, S->est.p, m, nrhs, st_));
  if (learned) PTCHK(learned_begin(S, nrhs));
  return PT_OK;
}

// Iteration j in two halves: the preconditioner and operator applies
// (z_j = M^-1 v_j, w = A z_j), then the Arnoldi step on w (classical
// Gram-Schmidt twice, the new basis vector, the Givens update, the
// convergence flags to S->h_done).
pt_status fgmres_iter_apply(pt_solver* S, int nrhs, int j, bool learned) {
  const size_t vs = (size_t)nrhs * S->Nt;
  double2* vj = S->V.p + (size_t)j * vs;
  double2* zj = S->Z.p + (size_t)j * vs;
  const bool augment = learned && S->learned_mode == PT_LEARN_AUGMENT;
  if (augment && (j & 1)) {
    PTCHK(learned_direction(S, zj, nrhs));
  } else {
    PTCHK(system_M(S, vj, zj, nrhs));
  }
  if (learned && !augment) {
    PTCHK(learned_step(S, vj, zj, S->tmp.p, nrhs));
  } else {
    PTCHK(system_A(S, zj, S->tmp.p, nrhs));
    if (augment && !(j & 1)) PTCHK(learned_residual(S, vj, S->tmp.p, nrhs));
  }
  return PT_OK;
}

pt_status fgmres_iter_arnoldi(pt_solver* S, int nrhs, int j, double tol) {
  const int64_t N = S->Nt;
  const int m = S->opt.maxit;
  const size_t vs = (size_t)nrhs * N;
  GPU(S, launch_zero(S->hacc.p, (int64_t)(j + 1) * nrhs, st_));
  for (int pass = 0; pass < 2; ++pass) {
    GPU(S, launch_kdot(S->V.p, S->tmp.p, S->hbuf.p, j + 1, nrhs, N, st_));
    GPU(S, launch_kupdate(S->V.p, S->tmp.p, S->hbuf.p, S->hacc.p, j + 1, nrhs, N, st_));
  }
  GPU(S, launch_knorm(S->tmp.p, S->nrm.p, nrhs, N, st_));
  GPU(S, launch_kscale(S->V.p + (size_t)(j + 1) * vs, S->tmp.p, S->nrm.p, nrhs, N, st_));
  GPU(S, launch_givens(S->Hc.p, S->hacc.p, S->nrm.p, S->cs.p, S->sn.p, S->g.p, S->est.p, S->beta.p, S->iters.p,
                       S->done.p, tol, j, m, nrhs, st_));
  GPU(S, hipMemcpyAsync(S->h_done, S->done.p, nrhs * sizeof(int32_t), hipMemcpyDeviceToHost, st_));
  return PT_OK;
}

pt_status fgmres_iter(pt_solver* S, int nrhs, int j, double tol, bool learned) {
  PTCHK(fgmres_iter_apply(S, nrhs, j, learned));
  return fgmres_iter_arnoldi(S, nrhs, j, tol);
}

pt_status fgmres_end(pt_solver* S, int nrhs) {
  const int m = S->opt.maxit;
  GPU(S, launch_ksolve(S->Hc.p, S->g.p, S->y.p, S->iters.p, m, nrhs, st_));
  GPU(S, launch_kcombine(S->Z.p, S->y.p, S->iters.p, S->x.p, m, nrhs, S->Nt, st_));
  return PT_OK;
}

pt_status fgmres(pt_solver* S, int nrhs, bool& all_conv, double tol, bool learned) {
  hipStream_t st = S->st;
  const int m = S->opt.maxit;
  PTCHK(fgmres_begin(S, nrhs, learned));
  all_conv = false;
  // the launch sequence of iteration j (captured into a graph when enabled)
  auto iteration = [&](int j) -> pt_status { return fgmres_iter(S, nrhs, j, tol, learned); };
  // (the tolerance is a kernel argument baked into a graph: graphs only for the solver's own tol)
  const bool graphs = S->opt.use_graph && !learned && !S->prof && st != nullptr && !S->graph_failed &&
                      tol == S->opt.tol;
  for (int j = 0; j < m; ++j) {
    if (graphs) {
      PTCHK(run_graph(S, nrhs, j, tol, iteration));
    } else {
      PTCHK(iteration(j));
    }
    HIPCHK(hipStreamSynchronize(st));
    bool all = true;
    for (int r = 0; r < nrhs; ++r) all = all && S->h_done[r];
    if (all) {
      all_conv = true;
      break;
    }
  }
  return fgmres_end(S, nrhs);
}

pt_status check_nrhs(const pt_solver* S, int nrhs) {
  if (!S) return fail(PT_EINVAL, "null solver");
  if (nrhs < 1 || nrhs > S->opt.max_nrhs) return fail(PT_EINVAL, "nrhs must be in 1..max_nrhs");
  return PT_OK;
}

}  // namespace polar_impl

// ---------------------------------------------------------------------------
// Fixed device scratch of pt_apply_noalloc: the Gauss-Seidel iterates, the
// staged input and the k-slice partial tiles live here instead of in the
// solver's buffers.  In host code `scratch` names a host-side stand-in; its
// device address comes from hipGetSymbolAddress, once per device, at the first
// pt_setup on that device (with the device current).
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

namespace polar_impl {
pt_status scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(PT_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return PT_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return fail(PT_EHIP, std::string("scratch address: ") + hipGetErrorString(e));
  g_scratch_ptr[device] = (unsigned char*)ptr;
  return PT_OK;
}
}  // namespace polar_impl

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

const char* pt_status_str(pt_status st) {
  switch (st) {
    case PT_OK: return "ok";
    case PT_EINVAL: return "invalid argument";
    case PT_ENOMEM: return "out of device memory";
    case PT_EHIP: return "HIP runtime error";
    case PT_ESINGULAR: return "singular local factor";
    case PT_ENOCONV: return "GMRES did not converge";
  }
  return "unknown status";
}

const char* pt_last_error(void) { return g_err.c_str(); }

void pt_free(pt_solver* S) {
  if (!S) return;
  (void)hipStreamSynchronize(S->st);
  for (auto* b : {&S->dinv64, &S->blk64, &S->W, &S->Bw, &S->fio, &S->uio, &S->s, &S->V, &S->Z, &S->U1,
                  &S->U2, &S->tmp, &S->zeros, &S->x, &S->hbuf, &S->hacc, &S->Hc, &S->sn, &S->g, &S->y})
    b->release();
  S->blk32.release();
  S->blkbf.release();
  S->part.release();
  S->plr_part.release();
  S->mpart.release();
  release_green(S);
  S->gsum_dst.release();
  S->gsum_src.release();
  S->gsum_cnt.release();
  S->nz_list.release();
  S->xbf.release();
  S->rr_dst.release();
  S->rr_src.release();
  S->rr_seg.release();
  S->rr_sign.release();
  S->nz_in_k.release();
  S->nz_in_off.release();
  for (auto* b : {&S->nrm, &S->cs, &S->est, &S->beta, &S->f_sign, &S->g_sign}) b->release();
  for (auto* b : {&S->rowmap, &S->g_seg, &S->g_row, &S->f_seg, &S->f_row, &S->iters, &S->done, &S->flag,
                  &S->row_layer, &S->lay_own_start, &S->lay_n_own, &S->slot_rhs, &S->rhs_slot})
    b->release();
  S->act.release();
  if (S->h_act) (void)hipHostFree(S->h_act);
  if (S->h_slot) (void)hipHostFree(S->h_slot);
  S->jobs.release();
  S->plr.release();
  if (S->h_done) (void)hipHostFree(S->h_done);
  for (hipEvent_t e : S->ev) (void)hipEventDestroy(e);
  drop_graphs(S);
  delete S;
}

pt_status pt_profile(pt_solver* S, int32_t enable) {
  if (!S) return fail(PT_EINVAL, "null solver");
  if (enable) {
    if (S->ev.empty()) {
      S->ev.resize(2 * kEventSlots);
      for (auto& e : S->ev) HIPCHK(hipEventCreate(&e));
    }
    PTCHK(prof_harvest(S));
    S->stats = pt_kernel_stats{};
    for (auto& k : S->cstats) k = pt_kernel_stats{};
    S->prof = true;
  } else {
    PTCHK(prof_harvest(S));
    S->prof = false;
  }
  return PT_OK;
}

pt_status pt_gauss_seidel(pt_solver* S, int32_t nrhs, const double* f, double* u, int32_t on_device, double tol,
                          int32_t maxit, int32_t* iters, double* relupd) {
  PTCHK(check_nrhs(S, nrhs));
  if (!f || !u) return fail(PT_EINVAL, "null field");
  if (S->L < 2) return fail(PT_EINVAL, "no interfaces (L = 1)");
  if (maxit < 1 || !(tol >= 0)) return fail(PT_EINVAL, "maxit must be >= 1 and tol >= 0");
  hipStream_t st = S->st;
  const size_t nv = (size_t)nrhs * S->NZ * S->NX;
  const int64_t n = (int64_t)nrhs * S->Nt;
  const double2* fd = (const double2*)f;
  double2* ud = (double2*)u;
  if (!on_device) {
    HIPCHK(hipMemcpyAsync(S->fio.p, f, nv * sizeof(double2), hipMemcpyHostToDevice, st));
    fd = S->fio.p;
    ud = S->uio.p;
  }
  PTCHK(trace_rhs(S, fd, S->s.p, nrhs));
  // float16 split planes: iterate on s scaled to unit norm per source (the inputs' range), scale back at the end
  if (S->split_f16) {
    HIPCHK(launch_knorm(S->s.p, S->est.p, nrhs, S->Nt, st));
    HIPCHK(launch_kscale(S->s.p, S->s.p, S->est.p, nrhs, S->Nt, st));
  }
  // u^{i+1} = D^-1 (s - R u^i): one fused reflection launch (none for u^0 = 0) and the sweeps
  double2* prev = S->zeros.p;
  std::vector<double> num(nrhs), den(nrhs);
  int it = 0;
  double worst = 0.0;
  bool conv = false;
  for (it = 1; it <= maxit; ++it) {
    double2* cur = (it % 2) ? S->U1.p : S->U2.p;
    Bases b{{S->s.p, prev, cur, nullptr}};
    if (it == 1) {
      HIPCHK(launch_copy(cur, S->s.p, n, st));
    } else {
      PTCHK(run_apply(S, S->bterm, nrhs, S->Nt, b));
    }
    for (const Launch& Lc : S->sweep) PTCHK(run_apply(S, Lc, nrhs, S->Nt, b));
    HIPCHK(launch_add(S->tmp.p, cur, prev, -1.0, n, st));
    HIPCHK(launch_knorm(S->tmp.p, S->nrm.p, nrhs, S->Nt, st));
    HIPCHK(launch_knorm(cur, S->beta.p, nrhs, S->Nt, st));
    HIPCHK(hipMemcpyAsync(num.data(), S->nrm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(den.data(), S->beta.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    worst = 0.0;
    for (int r = 0; r < nrhs; ++r) {
      const double ru = den[r] > 0 ? num[r] / den[r] : (num[r] > 0 ? INFINITY : 0.0);
      if (relupd) relupd[r] = ru;
      worst = std::max(worst, std::isnan(ru) ? INFINITY : ru);
    }
    prev = cur;
    if (worst < tol) {
      conv = true;
      break;
    }
  }
  if (iters) *iters = std::min(it, maxit);
  if (S->split_f16) HIPCHK(launch_kmulnorm(const_cast<double2*>(prev), S->est.p, nrhs, S->Nt, st));
  PTCHK(reconstruct(S, fd, prev, ud, nrhs));
  if (!on_device) HIPCHK(hipMemcpyAsync(u, ud, nv * sizeof(double2), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return conv ? PT_OK : fail(PT_ENOCONV, "Gauss-Seidel reached maxit before tol");
}

// ---------------------------------------------------------------------------
// several problems in one launch sequence
// ---------------------------------------------------------------------------
// Block applies of different problems share a launch when they use the same
// kernel family: same block storage (float64, float32 or split planes of one
// element type) and the same side of the form's right-hand-side threshold.
// Compressed blocks are launched alone.
int merge_key(const pt_solver* S, const Rec& r) {
  if (r.Lc.plr) return -1;
  if (r.Lc.split) return 1 + (S->split_f16 ? 2 : 0) + (r.nrhs > 16 ? 1 : 0);
  return 5 + (r.Lc.f32 ? 2 : 0) + (r.nrhs > 4 ? 1 : 0);
}

// One block apply for each problem of `grp` (its next recorded operation), in
// one launch (several problems) or with the problem's own tuned shape (one).
pt_status issue_applies(pt_solver* const* s, const std::vector<std::vector<Rec>>& recs,
                        const std::vector<size_t>& cur, const std::vector<int>& grp, hipStream_t st) {
  if (grp.size() == 1) {
    const int p = grp[0];
    const Rec& r = recs[p][cur[p]];
    return run_apply(s[p], r.Lc, r.nrhs, r.ld, r.b);
  }
  ApplySeg segs[kMaxSeg];
  int maxterms = 0;
  bool wide = false;
  for (size_t i = 0; i < grp.size(); ++i) {
    const pt_solver* S = s[grp[i]];
    const Rec& r = recs[grp[i]][cur[grp[i]]];
    segs[i] = ApplySeg{S->jobs.p + r.Lc.job0, r.Lc.njobs, S->NX, r.nrhs, r.ld, r.b, S->part.p, S->part.n};
    maxterms = std::max(maxterms, r.Lc.maxterms);
    wide = wide || r.Lc.wide;
  }
  pt_solver* S0 = s[grp[0]];
  const Rec& r0 = recs[grp[0]][cur[grp[0]]];
  const int n = (int)grp.size();
  // live timing: the merged launch is counted once, by the group's first
  // solver, in the class of its first problem, with every segment's bytes and flops
  int slot = -1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (S0->prof) {
    if (S0->ev_next >= kEventSlots) PTCHK(prof_harvest(S0));
    slot = S0->ev_next++;
    e0 = S0->ev[2 * slot];
    e1 = S0->ev[2 * slot + 1];
  }
  if (r0.Lc.split) {
    HIPCHK(launch_block_apply_split_segs(segs, n, S0->split_f16 ? 1 : 0, st, e0, e1));
  } else {
    HIPCHK(launch_block_apply_segs(segs, n, maxterms, wide, r0.Lc.f32, st, e0, e1));
  }
  if (S0->prof) {
    double bytes = 0, flops = 0;
    for (int p : grp) {
      const Rec& r = recs[p][cur[p]];
      const double es = r.Lc.split ? 8.0 : r.Lc.f32 ? 8.0 : 16.0;
      bytes += r.Lc.mat_elems * es + r.Lc.vec_elems_rhs * r.nrhs * 16.0;
      flops += 8.0 * r.Lc.mat_elems * r.nrhs;
    }
    S0->pend.push_back(ProfPending{slot, r0.Lc.cls, bytes, flops});
  }
  return PT_OK;
}

// Issue the recorded operations of every problem on stream st, each
// problem's in its order: rounds take the next operation of every problem;
// any other stream operation is issued first, block applies wait for a round
// where every problem still recording has one, and then share launches.
pt_status run_recorded(pt_solver* const* s, std::vector<std::vector<Rec>>& recs, hipStream_t st,
                       const std::vector<hipStream_t>* lanes = nullptr) {
  const int P = (int)recs.size();
  std::vector<size_t> cur(P, 0);
  if (lanes) {
    // every problem on its own stream, its operations issued in turns
    for (bool more = true; more;) {
      more = false;
      for (int p = 0; p < P; ++p) {
        if (cur[p] >= recs[p].size()) continue;
        more = true;
        const Rec& r = recs[p][cur[p]++];
        if (r.fn) {
          const hipError_t e = r.fn((*lanes)[p]);
          if (e != hipSuccess) return fail(PT_EHIP, std::string("problem ") + std::to_string(p) + ": " +
                                                        hipGetErrorString(e));
        } else {
          const hipStream_t keep = s[p]->st;
          s[p]->st = (*lanes)[p];
          const pt_status rc = run_apply(s[p], r.Lc, r.nrhs, r.ld, r.b);
          s[p]->st = keep;
          PTCHK(rc);
        }
      }
    }
    for (auto& v : recs) v.clear();
    return PT_OK;
  }
  std::vector<int> pend, grp;
  std::vector<char> taken(P);
  for (;;) {
    bool any = false, other = false;
    for (int p = 0; p < P; ++p) {
      if (cur[p] >= recs[p].size()) continue;
      any = true;
      Rec& r = recs[p][cur[p]];
      if (!r.fn) continue;
      const hipError_t e = r.fn(st);
      if (e != hipSuccess) return fail(PT_EHIP, std::string("problem ") + std::to_string(p) + ": " +
                                                    hipGetErrorString(e));
      ++cur[p];
      other = true;
    }
    if (!any) break;
    if (other) continue;
    pend.clear();
    for (int p = 0; p < P; ++p)
      if (cur[p] < recs[p].size()) pend.push_back(p);
    std::fill(taken.begin(), taken.end(), 0);
    for (size_t i = 0; i < pend.size(); ++i) {
      const int p = pend[i];
      if (taken[p]) continue;
      const int key = merge_key(s[p], recs[p][cur[p]]);
      grp.assign(1, p);
      taken[p] = 1;
      for (size_t k = i + 1; k < pend.size() && key >= 0 && (int)grp.size() < kMaxSeg; ++k) {
        const int q = pend[k];
        if (!taken[q] && merge_key(s[q], recs[q][cur[q]]) == key) {
          grp.push_back(q);
          taken[q] = 1;
        }
      }
      PTCHK(issue_applies(s, recs, cur, grp, st));
    }
    for (int p : pend) ++cur[p];
  }
  for (auto& v : recs) v.clear();
  return PT_OK;
}

// pt_solve for several problems in lockstep on one stream (the first
// solver's): each stage (inputs and source activity; pre-solve, trace
// right-hand side and GMRES start; one GMRES iteration of every problem not
// yet converged; solution and reconstruction; convergence data) is recorded
// for every problem, then issued with the block applies of different problems
// sharing launches.  The host synchronises once per stage for all problems.
// Every problem's arithmetic is that of pt_solve, up to the launch shapes of
// the merged launches (the rules' shapes for the merged size).
pt_status solve_merged(int P, pt_solver* const* s, const int32_t* nrhs, const double* const* f, double* const* u,
                       int32_t on_device, pt_rhs_info* const* info) {
  hipStream_t st = s[0]->st;
  for (int p = 0; p < P; ++p) HIPCHK(hipStreamSynchronize(s[p]->st));  // earlier work on every stream
  struct Prob {
    const double2* fd;
    double2* ud;
    hipStream_t own;
    int j = 0;
    bool live = false;
    std::vector<double> nr, be, es;
    std::vector<int32_t> it, dn;
  };
  std::vector<Prob> q(P);
  for (int p = 0; p < P; ++p) {
    q[p].own = s[p]->st;
    s[p]->st = st;
  }
  std::vector<std::vector<Rec>> recs(P);
  // The long dependent chains of the pre-solve and the reconstruction run on
  // the problems' own streams when they are distinct ("lanes"), so one
  // problem's chain overlaps another's; the GMRES iterations share launches.
  std::vector<hipStream_t> lanes(P);
  bool use_lanes = true;
  for (int p = 0; p < P; ++p) {
    lanes[p] = q[p].own;
    for (int k = 0; k < p; ++k) use_lanes = use_lanes && lanes[k] != lanes[p];
  }
  std::vector<hipEvent_t> evs(P + 1, nullptr);
  // every exit drains the problems' streams (an early one may leave copies into
  // this call's host vectors, or waits on its events, in flight), gives the
  // solvers back their streams, stops recording and frees the events
  struct Restore {
    pt_solver* const* s;
    std::vector<Prob>& q;
    std::vector<hipEvent_t>& evs;
    ~Restore() {
      for (size_t p = 0; p < q.size(); ++p) (void)hipStreamSynchronize(q[p].own);
      for (size_t p = 0; p < q.size(); ++p) {
        s[p]->st = q[p].own;
        s[p]->rec = nullptr;
      }
      for (hipEvent_t e : evs)
        if (e) (void)hipEventDestroy(e);
    }
  } restore{s, q, evs};
  if (use_lanes)
    for (auto& e : evs) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  auto record = [&](int p) { s[p]->rec = &recs[p]; };
  auto issue = [&]() -> pt_status {
    for (int p = 0; p < P; ++p) s[p]->rec = nullptr;
    return run_recorded(s, recs, st);
  };
  // a stage on the lanes: they start after the work issued on st and st waits for them
  auto issue_lanes = [&]() -> pt_status {
    if (!use_lanes) return issue();
    for (int p = 0; p < P; ++p) s[p]->rec = nullptr;
    HIPCHK(hipEventRecord(evs[P], st));
    for (int p = 0; p < P; ++p)
      if (lanes[p] != st) HIPCHK(hipStreamWaitEvent(lanes[p], evs[P], 0));
    PTCHK(run_recorded(s, recs, st, &lanes));
    for (int p = 0; p < P; ++p)
      if (lanes[p] != st) {
        HIPCHK(hipEventRecord(evs[p], lanes[p]));
        HIPCHK(hipStreamWaitEvent(st, evs[p], 0));
      }
    return PT_OK;
  };
  // inputs on the device and the sources' activity per layer
  for (int p = 0; p < P; ++p) {
    pt_solver* S = s[p];
    const size_t nv = (size_t)nrhs[p] * S->NZ * S->NX;
    q[p].fd = (const double2*)f[p];
    q[p].ud = (double2*)u[p];
    record(p);
    if (!on_device) {
      const double* fh = f[p];
      GPU(S, hipMemcpyAsync(S->fio.p, fh, nv * sizeof(double2), hipMemcpyHostToDevice, st_));
      q[p].fd = S->fio.p;
      q[p].ud = S->uio.p;
    }
    if (S->L >= 2) PTCHK(trace_rhs_begin(S, q[p].fd, nrhs[p]));
  }
  PTCHK(issue_lanes());
  HIPCHK(hipStreamSynchronize(st));
  // pre-solves, trace right-hand sides, GMRES starts
  for (int p = 0; p < P; ++p) {
    pt_solver* S = s[p];
    if (S->L < 2) continue;
    record(p);
    bool uploads = false;
    PTCHK(trace_rhs_end(S, q[p].fd, S->s.p, nrhs[p], &uploads));
    if (S->opt.closure == 1)  // extrapolation rows: zero right-hand side
      GPU(S, launch_zero_extrap_rows(S->s.p, S->L, S->NX, S->Nt, nrhs[p], st_));
    PTCHK(fgmres_begin(S, nrhs[p], false));
    q[p].live = S->opt.maxit > 0;
  }
  PTCHK(issue_lanes());
  // GMRES iterations in lockstep; a problem leaves when all its sources
  // converged.  The preconditioner and operator applies share launches; the
  // Arnoldi steps (small reductions, a handful of launches per problem) run on
  // the lanes, concurrently
  for (;;) {
    bool any = false;
    for (int p = 0; p < P; ++p) {
      if (!q[p].live) continue;
      any = true;
      record(p);
      PTCHK(fgmres_iter_apply(s[p], nrhs[p], q[p].j, false));
    }
    if (!any) break;
    PTCHK(issue());
    for (int p = 0; p < P; ++p) {
      if (!q[p].live) continue;
      record(p);
      PTCHK(fgmres_iter_arnoldi(s[p], nrhs[p], q[p].j, s[p]->opt.tol));
    }
    PTCHK(issue_lanes());
    HIPCHK(hipStreamSynchronize(st));
    for (int p = 0; p < P; ++p) {
      if (!q[p].live) continue;
      bool all = true;
      for (int r = 0; r < nrhs[p]; ++r) all = all && s[p]->h_done[r];
      if (all || ++q[p].j >= s[p]->opt.maxit) q[p].live = false;
    }
  }
  // solutions and fields
  for (int p = 0; p < P; ++p) {
    pt_solver* S = s[p];
    const size_t nv = (size_t)nrhs[p] * S->NZ * S->NX;
    record(p);
    if (S->L >= 2) PTCHK(fgmres_end(S, nrhs[p]));
    PTCHK(reconstruct(S, q[p].fd, S->L >= 2 ? S->x.p : nullptr, q[p].ud, nrhs[p]));
    if (!on_device) {
      double* uh = u[p];
      const double2* ud = q[p].ud;
      GPU(S, hipMemcpyAsync(uh, ud, nv * sizeof(double2), hipMemcpyDeviceToHost, st_));
    }
  }
  PTCHK(issue_lanes());
  // convergence data, as pt_solve decides it
  for (int p = 0; p < P; ++p) {
    pt_solver* S = s[p];
    const int n = nrhs[p];
    Prob& w = q[p];
    w.nr.assign(n, 0.0);
    w.be.assign(n, 0.0);
    w.es.assign(n, 0.0);
    w.it.assign(n, 0);
    w.dn.assign(n, 0);
    double* nr = w.nr.data();
    double* be = w.be.data();
    double* es = w.es.data();
    int32_t* it = w.it.data();
    int32_t* dn = w.dn.data();
    record(p);
    if (S->L == 1) {
      const double2* ud = w.ud;
      GPU(S, launch_knorm(ud, S->nrm.p, n, (int64_t)S->NZ * S->NX, st_));
      GPU(S, hipMemcpyAsync(nr, S->nrm.p, n * 8, hipMemcpyDeviceToHost, st_));
      continue;
    }
    if (info && info[p]) {  // true residual ||s - A x|| / ||s|| in float64
      PTCHK(system_A(S, S->x.p, S->tmp.p, n));
      GPU(S, launch_add(S->tmp.p, S->s.p, S->tmp.p, -1.0, (int64_t)n * S->Nt, st_));
      GPU(S, launch_knorm(S->tmp.p, S->nrm.p, n, S->Nt, st_));
      GPU(S, hipMemcpyAsync(nr, S->nrm.p, n * 8, hipMemcpyDeviceToHost, st_));
      GPU(S, hipMemcpyAsync(it, S->iters.p, n * 4, hipMemcpyDeviceToHost, st_));
    }
    GPU(S, hipMemcpyAsync(be, S->beta.p, n * 8, hipMemcpyDeviceToHost, st_));
    GPU(S, hipMemcpyAsync(es, S->est.p, n * 8, hipMemcpyDeviceToHost, st_));
    GPU(S, hipMemcpyAsync(dn, S->done.p, n * 4, hipMemcpyDeviceToHost, st_));
  }
  PTCHK(issue());
  HIPCHK(hipStreamSynchronize(st));
  int bad = -1;
  for (int p = 0; p < P; ++p) {
    const Prob& w = q[p];
    pt_rhs_info* inf = info ? info[p] : nullptr;
    bool conv = true;
    for (int r = 0; r < nrhs[p]; ++r) {
      if (s[p]->L == 1) {
        // one local solve, no iteration: the field is finite or the source was not
        const bool ok = std::isfinite(w.nr[r]);
        conv = conv && ok;
        if (inf) inf[r] = pt_rhs_info{0, ok ? 1 : 0, ok ? 0.0 : std::nan(""), ok ? 0.0 : std::nan(""), 0, 0};
        continue;
      }
      // a source that is not finite stops at once and is reported not converged
      const double rr = w.be[r] > 0 ? w.nr[r] / w.be[r] : (w.be[r] == 0.0 ? 0.0 : std::nan(""));
      const bool ok = w.dn[r] && std::isfinite(w.es[r]) && std::isfinite(w.be[r]) && (!inf || std::isfinite(rr));
      conv = conv && ok;
      if (inf) inf[r] = pt_rhs_info{w.it[r], ok ? 1 : 0, w.es[r], rr, 0, 0};
    }
    if (!conv && bad < 0) bad = p;
  }
  if (bad >= 0)
    return fail(PT_ENOCONV, "problem " + std::to_string(bad) +
                                ": GMRES did not converge for every source (maxit, or a source not finite)");
  return PT_OK;
}

pt_status pt_solve_batch(int32_t nprob, pt_solver* const* s, const int32_t* nrhs, const double* const* f,
                         double* const* u, int32_t on_device, pt_rhs_info* const* info) {
  if (nprob < 0 || (nprob > 0 && (!s || !nrhs || !f || !u))) return fail(PT_EINVAL, "null argument");
  for (int i = 0; i < nprob; ++i) {
    if (!s[i]) return fail(PT_EINVAL, "null solver");
    for (int j = 0; j < i; ++j)
      if (s[j] == s[i]) return fail(PT_EINVAL, "a solver appears twice in the batch");
  }
  std::vector<pt_status> st(nprob, PT_OK);
  std::vector<std::string> msg(nprob);
  std::vector<std::thread> th;
  th.reserve(nprob);
  for (int i = 0; i < nprob; ++i)
    th.emplace_back([&, i]() {
      (void)hipSetDevice(s[i]->device);  // a new thread starts on device 0
      st[i] = pt_solve(s[i], nrhs[i], f[i], u[i], on_device, info ? info[i] : nullptr);
      if (st[i] != PT_OK) msg[i] = g_err;  // the message is per thread
    });
  for (auto& t : th) t.join();
  for (int i = 0; i < nprob; ++i)
    if (st[i] != PT_OK) return fail(st[i], "problem " + std::to_string(i) + ": " + msg[i]);
  return PT_OK;
}

pt_status pt_solve_batch_merged(int32_t nprob, pt_solver* const* s, const int32_t* nrhs, const double* const* f,
                                double* const* u, int32_t on_device, pt_rhs_info* const* info) {
  if (nprob < 0 || (nprob > 0 && (!s || !nrhs || !f || !u))) return fail(PT_EINVAL, "null argument");
  for (int i = 0; i < nprob; ++i) {
    if (!s[i]) return fail(PT_EINVAL, "null solver");
    for (int j = 0; j < i; ++j)
      if (s[j] == s[i]) return fail(PT_EINVAL, "a solver appears twice in the batch");
    if (s[i]->device != s[0]->device) return fail(PT_EINVAL, "the solvers of a merged batch share one device");
    if (s[i]->learned) return fail(PT_EINVAL, "problem " + std::to_string(i) + ": a learned stage is solved alone");
    if (check_nrhs(s[i], nrhs[i]) != PT_OK) return fail(PT_EINVAL, "problem " + std::to_string(i) + ": " + g_err);
    if (!f[i] || !u[i]) return fail(PT_EINVAL, "problem " + std::to_string(i) + ": null field");
  }
  if (nprob == 0) return PT_OK;
  HIPCHK(hipSetDevice(s[0]->device));
  return solve_merged(nprob, s, nrhs, f, u, on_device, info);
}

pt_status pt_setup_batch(int32_t nprob, const pt_problem* probs, const pt_options* opts, void* const* hip_streams,
                         pt_solver** out) {
  if (nprob < 0 || (nprob > 0 && (!probs || !opts || !out))) return fail(PT_EINVAL, "null argument");
  for (int i = 0; i < nprob; ++i) out[i] = nullptr;
  if (nprob == 0) return PT_OK;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::vector<pt_status> st(nprob, PT_OK);
  std::vector<std::string> msg(nprob);
  std::vector<std::thread> th;
  th.reserve(nprob);
  for (int i = 0; i < nprob; ++i)
    th.emplace_back([&, i]() {
      (void)hipSetDevice(dev);  // the caller's device, not a new thread's default
      st[i] = setup_impl(&probs[i], &opts[i], hip_streams ? hip_streams[i] : nullptr, &out[i], nullptr);
      if (st[i] != PT_OK) msg[i] = g_err;  // the message is per thread
    });
  for (auto& t : th) t.join();
  for (int i = 0; i < nprob; ++i)
    if (st[i] != PT_OK) {
      for (int j = 0; j < nprob; ++j) {
        pt_free(out[j]);
        out[j] = nullptr;
      }
      return fail(st[i], "problem " + std::to_string(i) + ": " + msg[i]);
    }
  return PT_OK;
}

pt_status pt_profile_read(pt_solver* S, pt_kernel_stats* out) {
  if (!S || !out) return fail(PT_EINVAL, "null argument");
  PTCHK(prof_harvest(S));
  *out = S->stats;
  return PT_OK;
}

pt_status pt_profile_read_class(pt_solver* S, int32_t cls, pt_kernel_stats* out) {
  if (!S || !out) return fail(PT_EINVAL, "null argument");
  if (cls < 0 || cls >= PT_CLS_COUNT) return fail(PT_EINVAL, "unknown launch class");
  PTCHK(prof_harvest(S));
  *out = S->cstats[cls];
  return PT_OK;
}

// mean time of `reps` launches of Lc with shape tc (after one warm-up)
static pt_status time_launch(pt_solver* S, const Launch& Lc, int nrhs, int64_t ld, Bases b, const TuneCfg* tc,
                             int reps, double& us) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const bool prof = S->prof;
  S->prof = false;
  pt_status rc = run_apply_cfg(S, Lc, nrhs, ld, b, tc);
  if (rc == PT_OK && hipEventRecord(e0, S->st) != hipSuccess) rc = fail(PT_EHIP, "event");
  for (int r = 0; r < reps && rc == PT_OK; ++r) rc = run_apply_cfg(S, Lc, nrhs, ld, b, tc);
  float ms = 0.f;
  if (rc == PT_OK && (hipEventRecord(e1, S->st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                      hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = fail(PT_EHIP, "event timing");
  S->prof = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  us = 1e3 * ms / reps;
  return rc;
}

}  // extern "C"

namespace {

// Process-wide cache of tuned choices, keyed by what they depend on: the
// block size, the layer count, the form (precision, closure, compressed
// blocks), the launch class, the right-hand-side count and the launch's job
// count.  pt_tune reuses an entry instead of timing; pt_tune_cache_save /
// pt_tune_cache_load keep it across processes.
struct TuneKey {
  int NX, L, precision, closure, plr, cls, nrhs, njobs;
  bool operator<(const TuneKey& o) const {
    return std::tie(NX, L, precision, closure, plr, cls, nrhs, njobs) <
           std::tie(o.NX, o.L, o.precision, o.closure, o.plr, o.cls, o.nrhs, o.njobs);
  }
};
struct TuneVal {
  int has_cfg = 0;  // 0: the built-in rule was fastest
  TuneCfg cfg{};
  double best_us = 0, default_us = 0;
  int tried = 0;
};
constexpr int kClsPlrRank = PT_CLS_COUNT;  // pseudo-class: the leaf rank limit of compressed blocks (njobs = rank)
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune_cache;

TuneKey tune_key(const pt_solver* S, int cls, int nrhs, int njobs) {
  return TuneKey{S->NX, S->L, S->opt.precision, S->opt.closure, S->use_plr ? 1 : 0, cls, nrhs, njobs};
}

}  // namespace

namespace polar_impl {

// launches that apply the compressed blocks: refresh their streamed-entry counts (profiling bytes)
void refresh_plr_bytes(pt_solver* S) {
  auto fix = [&](Launch& Lc) {
    if (!Lc.plr) return;
    Lc.mat_elems = 0;
    for (int j = Lc.job0; j < Lc.job0 + Lc.njobs; ++j)
      for (int t = 0; t < S->hjobs[j].nterms; ++t)
        Lc.mat_elems += (double)S->plr.stored_entries(S->blk_id(S->hjobs[j].M[t]));
  };
  for (Launch& Lc : S->sweep) fix(Lc);
  for (Launch* Lc : {&S->bterm, &S->opA, &S->opA2, &S->opR, &S->opX, &S->opX2, &S->opRX, &S->gsRX, &S->tX}) fix(*Lc);
}

// Compressed blocks: the leaf rank limit r_max (Alg. 5's partition threshold) that makes the
// per-iteration applies fastest for nrhs sources, at the solver's tolerance eps.  Each candidate
// is compressed on the GPU and its sweep and operator launches timed; the fastest stays in use.
pt_status tune_plr_rank(pt_solver* S, int nrhs, double& best_cost, int& tried, bool& cached) {
  const int NX = S->NX;
  const TuneKey key = tune_key(S, kClsPlrRank, nrhs, 0);
  int best_r = 0;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      best_r = it->second.cfg.tn;
      best_cost = it->second.best_us;
      tried = 0;
      cached = true;
    }
  }
  const int root = (int)std::ceil(std::sqrt((double)NX));
  std::vector<int> cands;
  if (!cached)
    for (int r : {std::max(1, root / 2), root, 2 * root, 4 * root})
      if (std::min(r, kPlrMaxRank) == r && std::find(cands.begin(), cands.end(), r) == cands.end()) cands.push_back(r);
  Bases b{{S->s.p, S->U1.p, S->U2.p, nullptr}};
  Bases bo{{S->U1.p, nullptr, S->tmp.p, nullptr}};
  const int gs = std::max(1, S->opt.gs_iters);
  auto rebuild = [&](int r) -> pt_status {
    if (r == S->plr_rmax) return PT_OK;
    PlrSet tmp;
    const hipError_t e = tmp.build(S->blk64.p, S->nblk, NX, r, S->opt.plr_eps, S->st);
    if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? PT_ENOMEM : PT_EHIP, "PLR compression");
    HIPCHK(S->plr.adopt(tmp));
    S->plr_rmax = r;
    refresh_plr_bytes(S);
    return PT_OK;
  };
  best_cost = cached ? best_cost : 1e300;
  for (int r : cands) {
    PTCHK(rebuild(r));
    // one GMRES iteration's compressed-block launches: gs sweeps of L-2 steps, gs-1 reflection launches, A
    double t_sw = 0, t_bt = 0, t_op = 0;
    if (!S->sweep.empty()) PTCHK(time_launch(S, S->sweep[S->sweep.size() / 2], nrhs, S->Nt, b, nullptr, 3, t_sw));
    PTCHK(time_launch(S, S->bterm, nrhs, S->Nt, b, nullptr, 3, t_bt));
    PTCHK(time_launch(S, S->opA, nrhs, S->Nt, bo, nullptr, 3, t_op));
    const double cost = gs * (double)S->sweep.size() * t_sw + (gs - 1) * t_bt + t_op;
    ++tried;
    if (cost < best_cost) {
      best_cost = cost;
      best_r = r;
    }
  }
  if (best_r > 0) PTCHK(rebuild(best_r));
  if (!cached) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    TuneVal v;
    v.has_cfg = 1;
    v.cfg.tn = best_r;
    v.best_us = best_cost;
    v.tried = tried;
    g_tune_cache[key] = v;
  }
  return PT_OK;
}

}  // namespace polar_impl

extern "C" {

pt_status pt_tune(pt_solver* S, int32_t nrhs, pt_tune_entry* out) {
  PTCHK(check_nrhs(S, nrhs));
  HIPCHK(hipStreamSynchronize(S->st));
  drop_graphs(S);  // captured launches carry the old shapes
  constexpr int kReps = 3;
  constexpr double kTuneMargin = 0.98;
  // the shape the built-in rules give a launch: reported when no candidate replaces it
  auto rule_shape = [&](const Launch& Lc, int32_t& tile, int32_t& ks) {
    tile = 0;
    ks = 0;
    if (Lc.split) {
      if (nrhs > 16) {
        tile = 32;
        ks = split_kslices(Lc.njobs, S->NX, nrhs, 32);
        if ((size_t)ks * Lc.njobs * nrhs * S->NX > S->part.n) ks = 1;  // no room for the partial tiles
      } else {
        const long tasks = (long)Lc.njobs * ((S->NX + 15) / 16) * ((nrhs + 15) / 16);
        tile = 16;
        ks = tasks >= 4096 ? 1 : tasks >= 2048 ? 2 : 4;
      }
      return;
    }
    const ApplyGeom g = geom_for(S->NX, Lc.maxterms, nrhs, Lc.njobs);
    if (!Lc.plr && g.mfma) {
      tile = g.mfma;
      const long tiles = (long)Lc.njobs * g.ntiles * ((nrhs + g.mfma - 1) / g.mfma);
      ks = g.mfma == 16 ? (tiles < 256 ? 4 : tiles < 512 ? 2 : 1) : 1;
    }
  };
  const int L = S->L;
  // work buffers as inputs and outputs of the trial launches (contents overwritten)
  HIPCHK(hipMemsetAsync(S->W.p, 0, S->W.n * sizeof(double2), S->st));
  HIPCHK(hipMemsetAsync(S->Bw.p, 0, S->Bw.n * sizeof(double2), S->st));
  if (L >= 2)
    for (auto* bf : {&S->U1, &S->U2, &S->tmp, &S->s}) HIPCHK(hipMemsetAsync(bf->p, 0, bf->n * sizeof(double2), S->st));
  // compressed blocks: the leaf rank limit first (the launch shapes below are then those of its tree)
  if (S->use_plr && L >= 2) {
    double cost = 0;
    int tried = 0;
    bool cached = false;
    PTCHK(tune_plr_rank(S, nrhs, cost, tried, cached));
  }
  for (int cls = 0; cls < PT_CLS_COUNT; ++cls) {
    pt_tune_entry e{cls, 0, 0, 0, 0.0, 0.0, 0};
    const Launch* Lc = nullptr;
    Bases b{};
    int64_t ld = S->Nt;
    if (cls == PT_CLS_LOCAL && !S->fwd.empty()) {
      Lc = &S->fwd[S->fwd.size() / 2];
      b = Bases{{S->W.p, S->Bw.p, nullptr, nullptr}};
      ld = (int64_t)S->sumR * S->NX;
    } else if (cls == PT_CLS_SWEEP && L >= 3 && !S->sweep.empty()) {
      Lc = &S->sweep[S->sweep.size() / 2];
      b = Bases{{S->s.p, S->U1.p, S->U2.p, nullptr}};
    } else if (cls == PT_CLS_REFLECT && L >= 2) {
      Lc = &S->bterm;
      b = Bases{{S->s.p, S->U1.p, S->U2.p, nullptr}};
    } else if (cls == PT_CLS_OPERATOR && L >= 2) {
      Lc = &S->opA;
      b = Bases{{S->U1.p, nullptr, S->tmp.p, nullptr}};
    }
    if (Lc && Lc->njobs > 0) {
      const TuneKey key = tune_key(S, cls, nrhs, Lc->njobs);
      bool hit = false;
      {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        const auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
          hit = true;
          if (it->second.has_cfg) {
            S->tune[cls][nrhs] = it->second.cfg;
            S->tune[cls][nrhs].njobs = Lc->njobs;
            e.tile_rhs = it->second.cfg.tn ? it->second.cfg.tn : it->second.cfg.sp.tile_rhs;
            e.ksplit = it->second.cfg.tn ? std::max(it->second.cfg.ks, it->second.cfg.mks)
                                         : it->second.cfg.sp.kslices;
          } else {
            S->tune[cls].erase(nrhs);
            rule_shape(*Lc, e.tile_rhs, e.ksplit);
          }
          e.best_us = it->second.best_us;
          e.default_us = it->second.default_us;
          e.cached = 1;
        }
      }
      if (hit) {
        if (out) out[cls] = e;
        continue;
      }
      // candidate shapes of this launch
      std::vector<TuneCfg> cands;
      const ApplyGeom g = geom_for(S->NX, Lc->maxterms, nrhs, Lc->njobs);
      if (Lc->split) {
        if (nrhs > 16) {
          std::vector<int> forms{0};
          if (Lc->two_term) forms.push_back(Lc->two_term);
          for (int form : forms)
            for (int tr : {32, 64})
              for (int ks : {1, 2, 4, 8, 16})
                if ((size_t)ks * Lc->njobs * nrhs * S->NX <= S->part.n || ks == 1) {
                  TuneCfg c;
                  c.sp = SplitCfg{tr, ks, form};
                  cands.push_back(c);
                }
        } else {
          for (int ks : {1, 2, 4}) {
            TuneCfg c;
            c.sp = SplitCfg{0, ks};
            cands.push_back(c);
          }
        }
      } else if (!Lc->plr && g.mfma) {
        for (int tn : {16, 32, 64})
          for (int ks : {1, 2, 4})
            if (tn == 16 || ks == 1) {
              TuneCfg c;
              c.tn = tn;
              c.ks = ks;
              cands.push_back(c);
            }
        // k-slices over workgroups, where the workspace holds the partial tiles; not for the local
        // solves, whose passes differ in length and input window from the one timed here: two
        // slices won 2% on that pass and lost 4% over the class as a whole
        for (int tn : {16, 32, 64})
          for (int mks = 2; mks <= kMfmaSlicesMax; mks *= 2)
            if (cls != PT_CLS_LOCAL && (size_t)mks * Lc->njobs * nrhs * S->NX <= S->mpart.n) {
              TuneCfg c;
              c.tn = tn;
              c.ks = 1;
              c.mks = mks;
              cands.push_back(c);
            }
      }
      PTCHK(time_launch(S, *Lc, nrhs, ld, b, nullptr, kReps, e.default_us));
      e.best_us = e.default_us;
      e.tried = 1;
      const TuneCfg* best = nullptr;
      // a candidate replaces the rules' shape only when it is at least 2% faster, so that
      // shapes within the timing noise of each other do not change from run to run
      const double bar = kTuneMargin * e.default_us;
      for (const TuneCfg& c : cands) {
        double us = 0;
        PTCHK(time_launch(S, *Lc, nrhs, ld, b, &c, kReps, us));
        ++e.tried;
        if (us < e.best_us && us < bar) {
          e.best_us = us;
          best = &c;
        }
      }
      if (best) {
        S->tune[cls][nrhs] = *best;
        S->tune[cls][nrhs].njobs = Lc->njobs;
        e.tile_rhs = best->tn ? best->tn : best->sp.tile_rhs;
        e.ksplit = best->tn ? std::max(best->ks, best->mks) : best->sp.kslices;
      } else {
        S->tune[cls].erase(nrhs);
        rule_shape(*Lc, e.tile_rhs, e.ksplit);
      }
      TuneVal v;
      v.has_cfg = best ? 1 : 0;
      if (best) v.cfg = *best;
      v.best_us = e.best_us;
      v.default_us = e.default_us;
      v.tried = e.tried;
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune_cache[key] = v;
    }
    if (out) out[cls] = e;
  }
  HIPCHK(hipStreamSynchronize(S->st));
  return PT_OK;
}

pt_status pt_tune_cache_save(const char* path) {
  if (!path) return fail(PT_EINVAL, "null path");
  FILE* fp = std::fopen(path, "w");
  if (!fp) return fail(PT_EINVAL, std::string("cannot open ") + path + " for writing");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  bool ok = std::fprintf(fp, "# libpolar tuning cache v2: NX L precision closure plr class nrhs njobs | has_cfg tn ks "
                             "mks tile_rhs kslices stream f16 | best_us default_us tried\n") > 0;
  for (const auto& kv : g_tune_cache) {
    const TuneKey& k = kv.first;
    const TuneVal& v = kv.second;
    ok = ok && std::fprintf(fp, "%d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %.9g %.9g %d\n", k.NX, k.L,
                            k.precision, k.closure, k.plr, k.cls, k.nrhs, k.njobs, v.has_cfg, v.cfg.tn, v.cfg.ks,
                            v.cfg.mks, v.cfg.sp.tile_rhs, v.cfg.sp.kslices, v.cfg.sp.stream, v.cfg.sp.f16, v.best_us,
                            v.default_us, v.tried) > 0;
  }
  ok = std::fclose(fp) == 0 && ok;
  return ok ? PT_OK : fail(PT_EINVAL, std::string("writing ") + path + " failed");
}

pt_status pt_tune_cache_load(const char* path) {
  if (!path) return fail(PT_EINVAL, "null path");
  FILE* fp = std::fopen(path, "r");
  if (!fp) return fail(PT_EINVAL, std::string("cannot open ") + path);
  char line[512];
  std::map<TuneKey, TuneVal> add;
  bool ok = std::fgets(line, sizeof(line), fp) && std::strncmp(line, "# libpolar tuning cache v2", 26) == 0;
  while (ok && std::fgets(line, sizeof(line), fp)) {
    TuneKey k{};
    TuneVal v{};
    const int got = std::sscanf(line, "%d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %lf %lf %d", &k.NX, &k.L,
                                &k.precision, &k.closure, &k.plr, &k.cls, &k.nrhs, &k.njobs, &v.has_cfg, &v.cfg.tn,
                                &v.cfg.ks, &v.cfg.mks, &v.cfg.sp.tile_rhs, &v.cfg.sp.kslices, &v.cfg.sp.stream,
                                &v.cfg.sp.f16, &v.best_us, &v.default_us, &v.tried);
    // MFMA tiles: the kernel's widths 16, 32, 64 (0: the rules'), wave groups 1, 2, 4 (0: the rules')
    ok = got == 19 && k.cls >= 0 && k.cls <= kClsPlrRank && k.nrhs >= 1 &&
         (v.cfg.tn == 0 || v.cfg.tn == 16 || v.cfg.tn == 32 || v.cfg.tn == 64) &&
         (v.cfg.ks == 0 || v.cfg.ks == 1 || v.cfg.ks == 2 || v.cfg.ks == 4) && v.cfg.mks >= 0 &&
         v.cfg.mks <= kMfmaSlicesMax &&
         v.cfg.sp.kslices >= 0 && v.cfg.sp.kslices <= 16 &&
         (v.cfg.sp.tile_rhs == 0 || v.cfg.sp.tile_rhs == 32 || v.cfg.sp.tile_rhs == 64) && v.cfg.sp.stream >= 0 &&
         v.cfg.sp.stream <= 2;
    if (ok) add[k] = v;
  }
  std::fclose(fp);
  if (!ok) return fail(PT_EINVAL, std::string(path) + " is not a tuning cache of this library");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : add) g_tune_cache[kv.first] = kv.second;
  return PT_OK;
}

pt_status pt_setup(const pt_problem* prob, const pt_options* opt, void* hip_stream, pt_solver** out) {
  return setup_impl(prob, opt, hip_stream, out, nullptr);
}

}  // extern "C"

pt_status polar_impl::setup_impl(const pt_problem* prob, const pt_options* opt, void* hip_stream, pt_solver** out,
                                 const LoadSrc* src) {
  if (!out) return fail(PT_EINVAL, "null output pointer");
  *out = nullptr;
  PTCHK(validate(prob, opt));
  const auto t0 = std::chrono::steady_clock::now();
  pt_solver* S = new pt_solver();
  S->nx = prob->nx;
  S->nz = prob->nz;
  S->npml = prob->npml;
  S->NX = prob->nx + 2 * prob->npml;
  S->NZ = prob->nz + 2 * prob->npml;
  S->L = prob->L;
  S->h = prob->h;
  S->omega = prob->omega;
  S->C = prob->pml_C;
  S->opt = *opt;
  S->f32 = false;
  S->st = (hipStream_t)hip_stream;
  (void)hipGetDevice(&S->device);
  if (const pt_status sc = scratch_init(S->device); sc != PT_OK) {
    delete S;
    return sc;
  }
  make_layout(S);
  const int NX = S->NX, NZ = S->NZ;
  S->c_host.assign(prob->c, prob->c + (size_t)NX * NZ);
  const double delta = S->npml * S->h;
  const double h2w2 = S->h * S->h * S->omega * S->omega;

  // x-direction alphas (global profile) and the tridiagonal couplings
  std::vector<cd> ax(NX), axm(NX), axp(NX), west(NX), east(NX);
  for (int i = 0; i < NX; ++i) {
    const double p = i - S->npml + 1;
    ax[i] = pml_alpha(beyond(p, S->nx) * S->h, S->C, delta, S->omega);
    axm[i] = pml_alpha(beyond(p - 0.5, S->nx) * S->h, S->C, delta, S->omega);
    axp[i] = pml_alpha(beyond(p + 0.5, S->nx) * S->h, S->C, delta, S->omega);
    west[i] = i > 0 ? -(ax[i] * axm[i]) : cmk(0, 0);
    east[i] = i < NX - 1 ? -(ax[i] * axp[i]) : cmk(0, 0);
  }
  S->ax_host = ax;
  // per local row: diagonal of A_r and the z couplings l_r (to r-1), u_r (to r+1)
  std::vector<cd> diag((size_t)S->sumR * NX);
  S->lcoef.assign(S->sumR, cmk(0, 0));
  S->ucoef.assign(S->sumR, cmk(0, 0));
  std::vector<int32_t> rowmap(S->sumR, -1);
  for (int l = 0; l < S->L; ++l) {
    const Layer& y = S->lay[l];
    const std::vector<RowZ> rz = local_rows(S, y);
    for (int r = 0; r < y.R; ++r) {
      const int g = y.rowbase + r;
      S->lcoef[g] = -(rz[r].a * rz[r].am);
      S->ucoef[g] = -(rz[r].a * rz[r].ap);
      const cd zz = rz[r].a * (rz[r].am + rz[r].ap);
      for (int i = 0; i < NX; ++i) {
        const double c = prob->c[(size_t)rz[r].mrow * NX + i];
        const cd xx = ax[i] * (axm[i] + axp[i]);
        diag[(size_t)g * NX + i] = xx + zz + cmk(-h2w2 / (c * c), 0.0);
      }
      if (r >= y.top_ext && r < y.top_ext + y.n) rowmap[g] = y.own_start + (r - y.top_ext);
    }
  }
  (void)NZ;
  pt_status rc = PT_OK;
  auto bail = [&](pt_status s) {
    pt_free(S);
    return s;
  };
  if (S->flag.alloc(1) != hipSuccess) return bail(fail(PT_ENOMEM, "flag"));
  if (S->dinv64.alloc((size_t)S->sumR * S->block_elems()) != hipSuccess)
    return bail(fail(PT_ENOMEM, "local factors"));
  if (S->rowmap.alloc(S->sumR) != hipSuccess ||
      hipMemcpy(S->rowmap.p, rowmap.data(), S->sumR * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(PT_EHIP, "rowmap"));

  if (!src) {
    rc = factorize(S, diag, west, east);
  } else if (!rec_read_device(src->fp, S->dinv64.p, S->dinv64.n, sizeof(double2))) {
    rc = fail(PT_EINVAL, "saved solver: local factors");
  }
  if (rc != PT_OK) return bail(rc);
  rc = extract_blocks(S, src);
  if (rc != PT_OK) return bail(rc);

  // trace gather (s = W rows) and forcing (W rows += sign * t) maps
  if (S->L >= 2) {
    std::vector<int32_t> gs, gr, fs, fr;
    std::vector<double> fsg;
    for (int k = 0; k < S->L - 1; ++k) {
      const Layer& up = S->lay[k];
      const Layer& lo = S->lay[k + 1];
      const int su[2] = {up.rowbase + up.rn, up.rowbase + up.rn1};
      const int sl[2] = {lo.rowbase + lo.r0, lo.rowbase + lo.r1};
      for (int a = 0; a < 2; ++a) {
        gs.push_back((0 * (S->L - 1) + k) * 2 + a);
        gr.push_back(su[a]);
        gs.push_back((1 * (S->L - 1) + k) * 2 + a);
        gr.push_back(sl[a]);
      }
      // layer k (bottom interface k): - e_{n+1} t_0 + e_n t_1
      fs.push_back(k * 2 + 0);
      fr.push_back(su[1]);
      fsg.push_back(-1.0);
      fs.push_back(k * 2 + 1);
      fr.push_back(su[0]);
      fsg.push_back(1.0);
      // layer k+1 (top interface k): + e_1 t_0 - e_0 t_1
      fs.push_back(k * 2 + 0);
      fr.push_back(sl[1]);
      fsg.push_back(1.0);
      fs.push_back(k * 2 + 1);
      fr.push_back(sl[0]);
      fsg.push_back(-1.0);
    }
    S->n_gather = (int)gs.size();
    S->n_force = (int)fs.size();
    if (S->g_seg.alloc(gs.size()) != hipSuccess || S->g_row.alloc(gr.size()) != hipSuccess ||
        S->f_seg.alloc(fs.size()) != hipSuccess || S->f_row.alloc(fr.size()) != hipSuccess ||
        S->f_sign.alloc(fsg.size()) != hipSuccess)
      return bail(fail(PT_ENOMEM, "trace maps"));
    if (hipMemcpy(S->g_seg.p, gs.data(), gs.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(S->g_row.p, gr.data(), gr.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(S->f_seg.p, fs.data(), fs.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(S->f_row.p, fr.data(), fr.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(S->f_sign.p, fsg.data(), fsg.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(PT_EHIP, "trace maps"));
  }

  // partitioned low-rank form of the trace blocks (Alg. 5, compressed on the GPU)
  if (opt->plr && S->L >= 2) {
    int rmax = opt->plr_rmax > 0 ? opt->plr_rmax : (int)std::ceil(std::sqrt((double)NX));
    rmax = std::min(rmax, kPlrMaxRank);
    S->plr_rmax = rmax;
    const auto tp = std::chrono::steady_clock::now();
    if (src) {
      if (!src->plr || !S->plr.load(src->fp) || (int)S->plr.stored.size() != S->nblk || S->plr.n != NX)
        return bail(fail(PT_EINVAL, "saved solver: compressed blocks"));
    } else {
      const hipError_t pe = S->plr.build(S->blk64.p, S->nblk, NX, rmax, opt->plr_eps, S->st);
      if (pe != hipSuccess) return bail(fail(pe == hipErrorOutOfMemory ? PT_ENOMEM : PT_EHIP, "PLR compression"));
    }
    S->plr_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp).count();
    S->use_plr = true;
  }

  // split planes (bfloat16 or float16) of the blocks for the preconditioner of the mixed forms
  if ((opt->precision == PT_SPLIT_BF16 || opt->precision == PT_SPLIT_F16) && S->L >= 2) {
    const bool f16 = opt->precision == PT_SPLIT_F16;
    const size_t E = split_block_elems(NX);
    // the one-sided extrapolators of the extrapolation closure's D^-1 (T step) are split likewise
    std::vector<const double2*> xsrc;
    if (opt->closure == 1)
      for (int k = 0; k + 1 < S->L; ++k) {
        xsrc.push_back(S->dinv64.p + (size_t)(S->lay[k].rowbase + S->lay[k].rn1) * S->block_elems());
        xsrc.push_back(S->dinv64.p + (size_t)(S->lay[k + 1].rowbase + S->lay[k + 1].r0) * S->block_elems());
      }
    double scale = 1.0;
    if (f16) {
      // one power of two for every split matrix: the largest Frobenius norm maps to at most 2^14, so no
      // entry exceeds float16's range (65504) and entries down to 2^-17 of it keep every bit of the pair
      DevBuf<double> nb;
      const size_t cnt = (size_t)S->nblk + xsrc.size();
      std::vector<double> hn(cnt, 0.0);
      bool ok = nb.alloc(cnt) == hipSuccess &&
                launch_knorm(S->blk64.p, nb.p, S->nblk, (int64_t)NX * NX, S->st) == hipSuccess;
      for (size_t i = 0; ok && i < xsrc.size(); ++i)
        ok = launch_knorm(xsrc[i], nb.p + S->nblk + i, 1, (int64_t)NX * NX, S->st) == hipSuccess;
      ok = ok && hipMemcpyAsync(hn.data(), nb.p, cnt * sizeof(double), hipMemcpyDeviceToHost, S->st) == hipSuccess &&
           hipStreamSynchronize(S->st) == hipSuccess;
      nb.release();
      if (!ok) return bail(fail(PT_EHIP, "split-float16 scale"));
      double mx = 0.0;
      for (double v : hn) mx = std::max(mx, v);
      if (!std::isfinite(mx)) return bail(fail(PT_ESINGULAR, "trace blocks are not finite"));
      if (mx > 0.0) scale = std::ldexp(1.0, 14 - (int)std::ceil(std::log2(mx)));
    }
    S->split_f16 = f16;
    S->split_alpha = 1.0 / (scale * split_input_scale(f16 ? 1 : 0));
    if (S->blkbf.alloc((size_t)S->nblk * E) != hipSuccess) return bail(fail(PT_ENOMEM, "split blocks"));
    if (launch_split_planes(S->blk64.p, S->blkbf.p, S->nblk, NX, S->st, f16 ? 1 : 0, scale) != hipSuccess ||
        hipStreamSynchronize(S->st) != hipSuccess)
      return bail(fail(PT_EHIP, "split conversion"));
    S->split = true;
    if (!xsrc.empty()) {
      if (S->xbf.alloc(xsrc.size() * E) != hipSuccess) return bail(fail(PT_ENOMEM, "split extrapolators"));
      for (size_t i = 0; i < xsrc.size(); ++i)
        if (launch_split_planes(xsrc[i], S->xbf.p + i * E, 1, NX, S->st, f16 ? 1 : 0, scale) != hipSuccess)
          return bail(fail(PT_EHIP, "split extrapolators"));
      if (hipStreamSynchronize(S->st) != hipSuccess) return bail(fail(PT_EHIP, "split extrapolators"));
    }
  }

  // float32 form: float32 copies of the trace blocks for the Gauss-Seidel
  // preconditioner (Alg. 4); the operator, the local solves and the
  // reconstruction keep the float64 factors and blocks (also when loaded:
  // the copies are made from the float64 blocks read back)
  if (opt->precision == PT_F32) {
    if (S->blk32.alloc(S->blk64.n) != hipSuccess) return bail(fail(PT_ENOMEM, "float32 copies"));
    if ((S->blk64.n && launch_to_f32(S->blk32.p, S->blk64.p, (int64_t)S->blk64.n, S->st) != hipSuccess) ||
        hipStreamSynchronize(S->st) != hipSuccess)
      return bail(fail(PT_EHIP, "float32 conversion"));
    S->f32 = true;
  }

  build_online_jobs(S);
  if (S->split_f16) {
    // the float16 planes hold scale x the blocks and the inputs are split at 2^12 x their value:
    // the jobs of every split launch multiply their sums back (a power of two: exact)
    std::vector<const Launch*> ls{&S->bterm, &S->opA, &S->opA2, &S->opR, &S->opX, &S->opX2, &S->opRX,
                                  &S->gsRX, &S->tX};
    for (const Launch& Lc : S->sweep) ls.push_back(&Lc);
    for (const Launch* Lc : ls)
      if (Lc->split)
        for (int j = Lc->job0; j < Lc->job0 + Lc->njobs; ++j) {
          S->hjobs[j].alpha.x *= S->split_alpha;
          S->hjobs[j].alpha.y *= S->split_alpha;
        }
  }
  S->jobs.release();
  if (S->jobs.alloc(S->hjobs.size()) != hipSuccess ||
      hipMemcpy(S->jobs.p, S->hjobs.data(), S->hjobs.size() * sizeof(Job), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(PT_ENOMEM, "jobs"));
  rc = alloc_online(S);
  if (rc != PT_OK) return bail(rc);
  if (hipStreamSynchronize(S->st) != hipSuccess) return bail(fail(PT_EHIP, "setup sync"));
  S->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = S;
  return PT_OK;
}

extern "C" {

pt_status pt_get_layout(const pt_solver* S, pt_layout* o) {
  if (!S || !o) return fail(PT_EINVAL, "null argument");
  std::memset(o, 0, sizeof(*o));
  o->NX = S->NX;
  o->NZ = S->NZ;
  o->L = S->L;
  o->sumR = S->sumR;
  o->ntrace = S->Nt;
  for (int l = 0; l < std::min(S->L, 64); ++l) {
    o->R[l] = S->lay[l].R;
    o->own_start[l] = S->lay[l].own_start;
    o->n_own[l] = S->lay[l].n;
    o->top_ext[l] = S->lay[l].top_ext;
    o->bot_ext[l] = S->lay[l].bot_ext;
  }
  o->setup_ms = S->setup_ms;
  o->plr_ms = S->plr_ms;
  const size_t es = sizeof(double2);
  o->dense_block_bytes = (int64_t)S->nblk * S->block_elems() * es;
  o->block_bytes = S->use_plr ? (int64_t)(S->plr.data_entries * sizeof(double2)) : o->dense_block_bytes;
  o->plr_leaves = S->use_plr ? (int64_t)S->plr.nleaves_total : 0;
  o->green_bytes = S->green.p ? (int64_t)(S->green.n * sizeof(double2)) : 0;
  o->factor_bytes = (int64_t)S->sumR * S->block_elems() * es;
  o->max_nrhs = S->opt.max_nrhs;
  o->plr_rmax = S->use_plr ? S->plr_rmax : 0;
  o->precision = S->opt.precision;
  return PT_OK;
}

namespace {

// stored block id, sign and diagonal shift of K^l_{j,k}: block = sign * K + shift * I
// (inverse of the packing in extract_blocks)
pt_status block_of(const pt_solver* S, int32_t layer, int32_t j, int32_t k, int* id, double* sign, double* shift) {
  if (layer < 0 || layer >= S->L || j < 0 || j > 3 || k < 0 || k > 3) return fail(PT_EINVAL, "bad block index");
  static const int T[4][4] = {{B_DN, B_DN, T_UP, T_UP}, {B_DN, B_DN, T_UP, T_UP}, {T_DN, T_DN, B_UP, B_UP},
                              {T_DN, T_DN, B_UP, B_UP}};
  // (a, b, sign, shift) for each (j, k); rows: j in {0,1,n,n+1}, cols: k
  struct E {
    int a, b;
    double sign, shift;
  };
  static const E M[4][4] = {
      {{0, 1, -1, 0}, {0, 0, 1, 0}, {0, 1, 1, 0}, {0, 0, -1, 0}},
      {{1, 1, -1, -1}, {1, 0, 1, 0}, {1, 1, 1, 0}, {1, 0, -1, 0}},
      {{0, 1, -1, 0}, {0, 0, 1, 0}, {0, 1, 1, 0}, {0, 0, -1, -1}},
      {{1, 1, -1, 0}, {1, 0, 1, 0}, {1, 1, 1, 0}, {1, 0, -1, 0}},
  };
  const E e = M[j][k];
  *id = S->bidx[((layer * 4 + T[j][k]) * 2 + e.a) * 2 + e.b];
  if (*id < 0) return fail(PT_EINVAL, "layer has no such trace rows");
  *sign = e.sign;
  *shift = e.shift;
  return PT_OK;
}

void unpack_block(const std::vector<double2>& col, int NX, double sign, double shift, double* out) {
  for (int i = 0; i < NX; ++i)
    for (int c = 0; c < NX; ++c) {
      double2 v = col[(size_t)i * NX + c];  // stored row-major
      if (i == c) v.x -= shift;             // block = sign*K + shift*I  =>  K = sign*(block - shift*I)
      out[2 * ((size_t)i * NX + c)] = sign * v.x;
      out[2 * ((size_t)i * NX + c) + 1] = sign * v.y;
    }
}

}  // namespace

pt_status pt_get_block(const pt_solver* S, int32_t layer, int32_t j, int32_t k, double* out) {
  if (!S || !out) return fail(PT_EINVAL, "null argument");
  int id;
  double sign, shift;
  const pt_status st = block_of(S, layer, j, k, &id, &sign, &shift);
  if (st != PT_OK) return st;
  const size_t n = S->block_elems();
  std::vector<double2> col(n);
  HIPCHK(hipMemcpy(col.data(), S->blk64.p + (size_t)id * n, n * sizeof(double2), hipMemcpyDeviceToHost));
  unpack_block(col, S->NX, sign, shift, out);
  return PT_OK;
}

pt_status pt_get_plr_block(const pt_solver* S, int32_t layer, int32_t j, int32_t k, double* out, int32_t* nleaves,
                           int64_t* stored) {
  if (!S || !out) return fail(PT_EINVAL, "null argument");
  if (!S->use_plr) return fail(PT_EINVAL, "solver has no compressed blocks (plr = 0)");
  int id;
  double sign, shift;
  const pt_status st = block_of(S, layer, j, k, &id, &sign, &shift);
  if (st != PT_OK) return st;
  const size_t n = S->block_elems();
  double2* d = nullptr;
  HIPCHK(hipMalloc((void**)&d, n * sizeof(double2)));
  std::vector<double2> col(n);
  hipError_t e = S->plr.expand(id, d, S->st);
  if (e == hipSuccess) e = hipMemcpyAsync(col.data(), d, n * sizeof(double2), hipMemcpyDeviceToHost, S->st);
  if (e == hipSuccess) e = hipStreamSynchronize(S->st);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(PT_EHIP, hipGetErrorString(e));
  unpack_block(col, S->NX, sign, shift, out);
  if (nleaves) *nleaves = S->plr.nleaves[id];
  if (stored) *stored = (int64_t)S->plr.stored_entries(id);
  return PT_OK;
}

}  // extern "C"

namespace polar_impl {

// y = op(x) on device vectors (both pt_apply and pt_apply_noalloc).  With
// float16 split planes, the operators that run split launches (D^-1 and the
// preconditioner) see their input scaled to unit norm per source, the range
// the float16 inputs are sized for (the Krylov vectors GMRES feeds them), and
// the output is scaled back: the operators are linear.
pt_status apply_dispatch(pt_solver* S, int32_t op, const double2* xd, double2* yd, int nrhs) {
  const size_t n = (size_t)nrhs * S->Nt;
  const bool unit = S->split_f16 &&
                    (op == PT_OP_DINV || op == PT_OP_PRECOND || op == PT_OP_DINV_EXTRAP || op == PT_OP_PRECOND_EXTRAP);
  // the input staged in s (unit norm per source when `unit`)
  auto stage = [&](double2* dst) -> pt_status {
    if (unit) {
      HIPCHK(launch_knorm(xd, S->nrm.p, nrhs, S->Nt, S->st));
      HIPCHK(launch_kscale(dst, xd, S->nrm.p, nrhs, S->Nt, S->st));
    } else {
      HIPCHK(hipMemcpyAsync(dst, xd, n * sizeof(double2), hipMemcpyDeviceToDevice, S->st));
    }
    return PT_OK;
  };
  switch (op) {
    case PT_OP_A: PTCHK(apply_op(S, S->opA, xd, yd, nrhs)); break;
    case PT_OP_R: PTCHK(apply_op(S, S->opR, xd, yd, nrhs)); break;
    case PT_OP_DINV:
      if (unit) {
        PTCHK(stage(S->s.p));
        PTCHK(apply_dinv(S, S->s.p, yd, nrhs));
      } else {
        PTCHK(apply_dinv(S, xd, yd, nrhs));
      }
      break;
    case PT_OP_PRECOND:
      // the preconditioner uses U1/U2 internally: stage the input in s
      PTCHK(stage(S->s.p));
      PTCHK(precondition(S, S->s.p, yd, nrhs));
      break;
    case PT_OP_A_EXTRAP:
    case PT_OP_R_EXTRAP:
    case PT_OP_DINV_EXTRAP:
    case PT_OP_PRECOND_EXTRAP:
      if (S->opt.closure != 1) return fail(PT_EINVAL, "extrapolation operators need closure = 1");
      if (op == PT_OP_A_EXTRAP) {
        PTCHK(apply_op(S, S->opX, xd, yd, nrhs));
      } else if (op == PT_OP_R_EXTRAP) {
        HIPCHK(launch_zero(yd, (int64_t)n, S->st));  // its extrapolation rows are zero
        PTCHK(apply_op(S, S->opRX, xd, yd, nrhs));
      } else if (op == PT_OP_DINV_EXTRAP) {
        if (unit) {
          PTCHK(stage(yd));
        } else {
          HIPCHK(launch_copy(yd, xd, (int64_t)n, S->st));
        }
        PTCHK(dinv_extrap_inplace(S, yd, nrhs));
      } else {
        PTCHK(stage(S->s.p));
        PTCHK(precondition_extrap(S, S->s.p, yd, nrhs));
      }
      break;
    default: return fail(PT_EINVAL, "unknown operator");
  }
  if (unit) HIPCHK(launch_kmulnorm(yd, S->nrm.p, nrhs, S->Nt, S->st));
  return PT_OK;
}

}  // namespace polar_impl

extern "C" {

pt_status pt_apply(pt_solver* S, int32_t op, int32_t nrhs, const double* x, double* y, int32_t on_device) {
  PTCHK(check_nrhs(S, nrhs));
  if (S->L < 2) return fail(PT_EINVAL, "no interfaces (L = 1)");
  if (!x || !y) return fail(PT_EINVAL, "null vector");
  const size_t n = (size_t)nrhs * S->Nt;
  const double2* xd = (const double2*)x;
  double2* yd = (double2*)y;
  if (!on_device) {
    HIPCHK(hipMemcpyAsync(S->U2.p, x, n * sizeof(double2), hipMemcpyHostToDevice, S->st));
    xd = S->U2.p;
    yd = S->tmp.p;
  }
  PTCHK(apply_dispatch(S, op, xd, yd, nrhs));
  if (!on_device) HIPCHK(hipMemcpyAsync(y, yd, n * sizeof(double2), hipMemcpyDeviceToHost, S->st));
  HIPCHK(hipStreamSynchronize(S->st));
  return PT_OK;
}

pt_status pt_local_solve(pt_solver* S, int32_t nrhs, const double* b, double* x, int32_t on_device) {
  PTCHK(check_nrhs(S, nrhs));
  if (!b || !x) return fail(PT_EINVAL, "null field");
  const size_t n = (size_t)nrhs * S->sumR * S->NX;
  HIPCHK(hipMemcpyAsync(S->Bw.p, b, n * sizeof(double2), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        S->st));
  PTCHK(run_local(S, S->fwd, S->bwd, nrhs, (int64_t)S->sumR * S->NX, S->W.p, S->Bw.p));
  HIPCHK(hipMemcpyAsync(x, S->W.p, n * sizeof(double2), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        S->st));
  HIPCHK(hipStreamSynchronize(S->st));
  return PT_OK;
}

pt_status pt_trace_rhs(pt_solver* S, int32_t nrhs, const double* f, double* out, int32_t on_device) {
  PTCHK(check_nrhs(S, nrhs));
  if (S->L < 2) return fail(PT_EINVAL, "no interfaces (L = 1)");
  if (!f || !out) return fail(PT_EINVAL, "null field");
  const size_t nv = (size_t)nrhs * S->NZ * S->NX, nt = (size_t)nrhs * S->Nt;
  const double2* fd = (const double2*)f;
  if (!on_device) {
    HIPCHK(hipMemcpyAsync(S->fio.p, f, nv * sizeof(double2), hipMemcpyHostToDevice, S->st));
    fd = S->fio.p;
  }
  double2* sd = on_device ? (double2*)out : S->s.p;
  PTCHK(trace_rhs(S, fd, sd, nrhs));
  if (!on_device) HIPCHK(hipMemcpyAsync(out, sd, nt * sizeof(double2), hipMemcpyDeviceToHost, S->st));
  HIPCHK(hipStreamSynchronize(S->st));
  return PT_OK;
}

pt_status pt_reconstruct(pt_solver* S, int32_t nrhs, const double* f, const double* x, double* u, int32_t on_device) {
  PTCHK(check_nrhs(S, nrhs));
  if (!f || !u || (S->L >= 2 && !x)) return fail(PT_EINVAL, "null field");
  const size_t nv = (size_t)nrhs * S->NZ * S->NX, nt = (size_t)nrhs * S->Nt;
  const double2* fd = (const double2*)f;
  const double2* xd = (const double2*)x;
  double2* ud = (double2*)u;
  if (!on_device) {
    HIPCHK(hipMemcpyAsync(S->fio.p, f, nv * sizeof(double2), hipMemcpyHostToDevice, S->st));
    fd = S->fio.p;
    if (S->L >= 2) {
      HIPCHK(hipMemcpyAsync(S->x.p, x, nt * sizeof(double2), hipMemcpyHostToDevice, S->st));
      xd = S->x.p;
    }
    ud = S->uio.p;
  }
  PTCHK(reconstruct(S, fd, xd, ud, nrhs));
  if (!on_device) HIPCHK(hipMemcpyAsync(u, ud, nv * sizeof(double2), hipMemcpyDeviceToHost, S->st));
  HIPCHK(hipStreamSynchronize(S->st));
  return PT_OK;
}

pt_status pt_solve(pt_solver* S, int32_t nrhs, const double* f, double* u, int32_t on_device, pt_rhs_info* info) {
  PTCHK(check_nrhs(S, nrhs));
  if (!f || !u) return fail(PT_EINVAL, "null field");
  const size_t nv = (size_t)nrhs * S->NZ * S->NX;
  const double2* fd = (const double2*)f;
  double2* ud = (double2*)u;
  if (!on_device) {
    HIPCHK(hipMemcpyAsync(S->fio.p, f, nv * sizeof(double2), hipMemcpyHostToDevice, S->st));
    fd = S->fio.p;
    ud = S->uio.p;
  }
  bool conv = true;
  bool used_learned = false;
  std::vector<double> nr(nrhs), be(nrhs), es(nrhs);
  std::vector<int32_t> it(nrhs), dn(nrhs), kept(nrhs, 0);
  // an early exit may leave copies into these vectors in flight: drain the
  // stream before they go (a no-op after the final synchronisation)
  struct Drain {
    hipStream_t st;
    ~Drain() { (void)hipStreamSynchronize(st); }
  } drain{S->st};
  // true residual ||s - A x|| / ||s|| in float64, with the GMRES data, to the host
  auto residuals = [&]() -> pt_status {
    PTCHK(system_A(S, S->x.p, S->tmp.p, nrhs));
    HIPCHK(launch_add(S->tmp.p, S->s.p, S->tmp.p, -1.0, (int64_t)nrhs * S->Nt, S->st));
    HIPCHK(launch_knorm(S->tmp.p, S->nrm.p, nrhs, S->Nt, S->st));
    HIPCHK(hipMemcpyAsync(nr.data(), S->nrm.p, nrhs * 8, hipMemcpyDeviceToHost, S->st));
    HIPCHK(hipMemcpyAsync(be.data(), S->beta.p, nrhs * 8, hipMemcpyDeviceToHost, S->st));
    HIPCHK(hipMemcpyAsync(es.data(), S->est.p, nrhs * 8, hipMemcpyDeviceToHost, S->st));
    HIPCHK(hipMemcpyAsync(it.data(), S->iters.p, nrhs * 4, hipMemcpyDeviceToHost, S->st));
    HIPCHK(hipMemcpyAsync(dn.data(), S->done.p, nrhs * 4, hipMemcpyDeviceToHost, S->st));
    HIPCHK(hipStreamSynchronize(S->st));
    return PT_OK;
  };
  if (S->L == 1) {
    // one layer: the local solve is the global solve
    PTCHK(reconstruct(S, fd, nullptr, ud, nrhs));
  } else {
    PTCHK(trace_rhs(S, fd, S->s.p, nrhs));
    if (S->opt.closure == 1)  // extrapolation rows: zero right-hand side
      HIPCHK(launch_zero_extrap_rows(S->s.p, S->L, S->NX, S->Nt, nrhs, S->st));
    if (S->learned) {
      // learned stage first; its float64 true residual decides, the sweeps are the fallback
      PTCHK(fgmres(S, nrhs, conv, S->opt.tol, true));
      PTCHK(learned_kept(S, nrhs, kept.data()));
      PTCHK(residuals());
      bool ok = conv;
      for (int r = 0; r < nrhs; ++r) {
        const double rr = be[r] > 0 ? nr[r] / be[r] : 0.0;
        ok = ok && std::isfinite(rr) && rr <= 10.0 * S->opt.tol + 1e-300;
      }
      used_learned = ok;
    }
    if (!used_learned) PTCHK(fgmres(S, nrhs, conv, S->opt.tol, false));
    PTCHK(reconstruct(S, fd, S->x.p, ud, nrhs));
  }
  if (!on_device) HIPCHK(hipMemcpyAsync(u, ud, nv * sizeof(double2), hipMemcpyDeviceToHost, S->st));
  // Convergence is decided whether or not the caller asked for info: a source
  // that is not finite is reported PT_ENOCONV either way.
  if (S->L == 1) {
    // one local solve, no iteration: the field is finite or the source was not
    HIPCHK(launch_knorm(ud, S->nrm.p, nrhs, (int64_t)S->NZ * S->NX, S->st));
    HIPCHK(hipMemcpyAsync(nr.data(), S->nrm.p, nrhs * 8, hipMemcpyDeviceToHost, S->st));
    HIPCHK(hipStreamSynchronize(S->st));
    for (int r = 0; r < nrhs; ++r) {
      const bool ok = std::isfinite(nr[r]);
      conv = conv && ok;
      if (info) info[r] = pt_rhs_info{0, ok ? 1 : 0, ok ? 0.0 : std::nan(""), ok ? 0.0 : std::nan(""), 0, 0};
    }
  } else {
    if (info) {
      if (!used_learned) PTCHK(residuals());
    } else {
      HIPCHK(hipMemcpyAsync(be.data(), S->beta.p, nrhs * 8, hipMemcpyDeviceToHost, S->st));
      HIPCHK(hipMemcpyAsync(es.data(), S->est.p, nrhs * 8, hipMemcpyDeviceToHost, S->st));
      HIPCHK(hipMemcpyAsync(dn.data(), S->done.p, nrhs * 4, hipMemcpyDeviceToHost, S->st));
      HIPCHK(hipStreamSynchronize(S->st));
    }
    for (int r = 0; r < nrhs; ++r) {
      // a source that is not finite stops at once and is reported not converged
      const double rr = be[r] > 0 ? nr[r] / be[r] : (be[r] == 0.0 ? 0.0 : std::nan(""));
      const bool ok = dn[r] && std::isfinite(es[r]) && std::isfinite(be[r]) && (!info || std::isfinite(rr));
      conv = conv && ok;
      if (info)
        info[r] = pt_rhs_info{it[r], ok ? 1 : 0, es[r], rr, used_learned ? 1 : 0, used_learned ? kept[r] : 0};
    }
  }
  HIPCHK(hipStreamSynchronize(S->st));
  return conv ? PT_OK : fail(PT_ENOCONV, "GMRES did not converge for every source (maxit, or a source not finite)");
}


/* The variant of pt_apply that allocates nothing (see polar.h). */
pt_status pt_apply_noalloc(pt_solver* S, int32_t op, int32_t nrhs, const double* x, double* y) {
  PTCHK(check_nrhs(S, nrhs));
  if (S->L < 2) return fail(PT_EINVAL, "no interfaces (L = 1)");
  if (!x || !y) return fail(PT_EINVAL, "null vector");
  if (op < PT_OP_A || op > PT_OP_PRECOND_EXTRAP) return fail(PT_EINVAL, "unknown operator");
  unsigned char* base = (S->device >= 0 && S->device < kMaxDevices) ? g_scratch_ptr[S->device] : nullptr;
  if (!base) return fail(PT_EHIP, "no scratch address for this device");
  // scratch layout: U1 | U2 | staged input | k-slice partial tiles (each 256-byte aligned)
  const size_t vec = ((size_t)nrhs * S->Nt * sizeof(double2) + 255) & ~(size_t)255;
  size_t part = 0;  // the largest partial-tile set a launch of this call writes
  if (S->split) {
    std::vector<const Launch*> ls{&S->bterm, &S->opA, &S->opA2, &S->opR, &S->opX, &S->opX2, &S->opRX,
                                  &S->gsRX, &S->tX};
    for (const Launch& Lc : S->sweep) ls.push_back(&Lc);
    for (const Launch* Lc : ls)
      if (Lc->split && Lc->njobs > 0) {
        const size_t need = split_part_need(S, *Lc, nrhs, tuned(S, *Lc, nrhs));
        if (need <= S->part.n) part = std::max(part, need);  // the same k-slice decision as pt_apply
      }
  }
  const size_t bytes = 3 * vec + part * sizeof(float2);
  if (bytes > kScratchBytes)
    return fail(PT_EINVAL, "pt_apply_noalloc needs " + std::to_string(bytes) + " bytes of scratch for nrhs = " +
                               std::to_string(nrhs) + "; the maximum is " + std::to_string(kScratchBytes));
  // run the shared dispatch with the solver's work buffers pointed at the scratch; restored on every path
  struct Swap {
    pt_solver* S;
    double2 *u1, *u2, *s;
    float2* part;
    ~Swap() {
      S->U1.p = u1;
      S->U2.p = u2;
      S->s.p = s;
      S->part.p = part;
    }
  } keep{S, S->U1.p, S->U2.p, S->s.p, S->part.p};
  S->U1.p = (double2*)base;
  S->U2.p = (double2*)(base + vec);
  S->s.p = (double2*)(base + 2 * vec);
  S->part.p = part ? (float2*)(base + 3 * vec) : nullptr;
  PTCHK(apply_dispatch(S, op, (const double2*)x, (double2*)y, nrhs));
  HIPCHK(hipStreamSynchronize(S->st));
  return PT_OK;
}

}  // extern "C"
