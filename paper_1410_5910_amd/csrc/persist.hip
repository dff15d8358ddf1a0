// pt_save / pt_load: the offline state of a solver (Alg. 1's output, which
// Alg. 2 reuses for every right-hand side) written to and read from a file.
//
// File layout: an 8-byte magic and a version word, then records (persist.h):
// problem scalars, options, the velocity on the padded grid, flags, the
// local factors, the trace blocks, the interface Green's functions (when
// kept), the compressed blocks (PLR), and the tuned launch shapes.  The job
// lists, trace maps, split-bfloat16 planes and work buffers are rebuilt by
// the ordinary setup path from these, so a loaded solver computes exactly
// what the saved one computed.
#include <cstdio>
#include <cstring>
#include <string>

#include "persist.h"
#include "solver_internal.h"

namespace {

constexpr char kMagic[8] = {'P', 'T', 'S', 'O', 'L', 'V', 'E', 'R'};
constexpr uint32_t kVersion = 2;

struct FileCloser {
  FILE* fp;
  ~FileCloser() {
    if (fp) std::fclose(fp);
  }
};

struct TuneRec {
  int32_t cls, nrhs;
  TuneCfg cfg;
};

}  // namespace

extern "C" {

pt_status pt_save(const pt_solver* S, const char* path) {
  if (!S || !path) return fail(PT_EINVAL, "null solver or path");
  if (hipStreamSynchronize(S->st) != hipSuccess) return fail(PT_EHIP, "stream");
  FILE* fp = std::fopen(path, "wb");
  if (!fp) return fail(PT_EINVAL, std::string("cannot open ") + path + " for writing");
  FileCloser fc{fp};
  const uint32_t ver[2] = {kVersion, (uint32_t)sizeof(pt_options)};
  const int32_t pi[4] = {S->nx, S->nz, S->npml, S->L};
  const double pd[3] = {S->h, S->omega, S->C};
  const bool green = S->green.p != nullptr;
  const int32_t flags[4] = {S->f32 ? 1 : 0, green ? 1 : 0, S->use_plr ? 1 : 0, S->plr_rmax};
  const size_t E = S->block_elems();
  bool ok = std::fwrite(kMagic, sizeof(kMagic), 1, fp) == 1 && rec_write_host(fp, ver, 2, 4) &&
            rec_write_host(fp, pi, 4, 4) && rec_write_host(fp, pd, 3, 8) &&
            rec_write_host(fp, &S->opt, 1, sizeof(pt_options)) &&
            rec_write_host(fp, S->c_host.data(), S->c_host.size(), sizeof(double)) && rec_write_host(fp, flags, 4, 4);
  // in the order setup reads them back
  if (ok) ok = rec_write_device(fp, S->dinv64.p, S->dinv64.n, sizeof(double2));
  if (ok && S->L >= 2) ok = rec_write_device(fp, S->blk64.p, (uint64_t)S->nblk * E, sizeof(double2));
  if (ok && green) ok = rec_write_device(fp, S->green.p, S->green.n, sizeof(double2));
  if (ok && S->use_plr) ok = S->plr.save(fp);
  std::vector<TuneRec> tr;
  for (int c = 0; c < PT_CLS_COUNT; ++c)
    for (const auto& kv : S->tune[c]) tr.push_back(TuneRec{c, kv.first, kv.second});
  if (ok) ok = rec_write_host(fp, tr.data(), tr.size(), sizeof(TuneRec));
  if (ok) ok = std::fflush(fp) == 0;
  if (!ok) return fail(PT_EINVAL, std::string("writing ") + path + " failed");
  return PT_OK;
}

pt_status pt_load(const char* path, void* hip_stream, pt_solver** out) {
  if (!path || !out) return fail(PT_EINVAL, "null path or output pointer");
  *out = nullptr;
  FILE* fp = std::fopen(path, "rb");
  if (!fp) return fail(PT_EINVAL, std::string("cannot open ") + path);
  FileCloser fc{fp};
  char magic[8];
  uint32_t ver[2];
  int32_t pi[4], flags[4];
  double pd[3];
  pt_options opt{};
  if (std::fread(magic, sizeof(magic), 1, fp) != 1 || std::memcmp(magic, kMagic, sizeof(kMagic)) != 0)
    return fail(PT_EINVAL, std::string(path) + " is not a saved solver");
  if (!rec_read_host(fp, ver, 2, 4) || ver[0] != kVersion || ver[1] != sizeof(pt_options))
    return fail(PT_EINVAL, "saved solver: unsupported version");
  if (!rec_read_host(fp, pi, 4, 4) || !rec_read_host(fp, pd, 3, 8) || !rec_read_host(fp, &opt, 1, sizeof(opt)))
    return fail(PT_EINVAL, "saved solver: header");
  if (pi[0] < 1 || pi[1] < 1 || pi[2] < 1 || pi[0] > 1 << 20 || pi[1] > 1 << 20 || pi[2] > 1 << 16)
    return fail(PT_EINVAL, "saved solver: grid sizes");
  const size_t npad = (size_t)(pi[0] + 2 * pi[2]) * (pi[1] + 2 * pi[2]);
  std::vector<double> c(npad);
  if (!rec_read_host(fp, c.data(), npad, sizeof(double)) || !rec_read_host(fp, flags, 4, 4))
    return fail(PT_EINVAL, "saved solver: velocity");
  if ((flags[0] != 0) != (opt.precision == PT_F32) || (flags[2] != 0) != (opt.plr != 0 && pi[3] >= 2))
    return fail(PT_EINVAL, "saved solver: flags do not match the options");
  pt_problem prob{};
  prob.nx = pi[0];
  prob.nz = pi[1];
  prob.npml = pi[2];
  prob.L = pi[3];
  prob.h = pd[0];
  prob.omega = pd[1];
  prob.pml_C = pd[2];
  prob.c = c.data();
  LoadSrc src;
  src.fp = fp;
  src.green = flags[1] != 0;
  src.plr = flags[2] != 0;
  // the saved Green's functions are used as they were (no memory heuristic on load)
  if (!src.green && opt.presolve == 2) opt.presolve = 0;
  pt_solver* S = nullptr;
  PTCHK(setup_impl(&prob, &opt, hip_stream, &S, &src));
  uint64_t ntr = 0;
  uint32_t el = 0;
  const long pos = std::ftell(fp);
  if (!rec_peek(fp, ntr, el) || el != sizeof(TuneRec) || ntr > (1u << 20) || std::fseek(fp, pos, SEEK_SET) != 0) {
    pt_free(S);
    return fail(PT_EINVAL, "saved solver: tuned shapes");
  }
  std::vector<TuneRec> tr(ntr);
  if (!rec_read_host(fp, tr.data(), ntr, sizeof(TuneRec))) {
    pt_free(S);
    return fail(PT_EINVAL, "saved solver: tuned shapes");
  }
  for (const TuneRec& t : tr)
    if (t.cls >= 0 && t.cls < PT_CLS_COUNT) S->tune[t.cls][t.nrhs] = t.cfg;
  if (S->use_plr) S->plr_rmax = flags[3];  // the tree in the file may carry a tuned rank limit
  *out = S;
  return PT_OK;
}

}  // extern "C"
