// C ABI of libqx.so: handles, argument checks, the solver driver (host side of
// the conjugate-gradient engine), batches with HIP-graph replay, the force
// entry points and the launch-shape tuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/qx.h"
#include "qx_dispatch.h"
#include "qx_internal.h"
#include "qx_launch.h"

using namespace qx;

// ------------------------------------------------------------------ errors

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(QX_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define QX_HIP(call, what)                    \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

// ------------------------------------------------------------------ handles

struct qx_lattice {
  int32_t dims[4];
  uint32_t flags;
  Geo geo;
  int64_t V;
};

struct qx_gauge {
  int32_t dims[4];
  uint32_t flags;
  Geo geo;
  int prec, recon;
  const void* packed;
  std::map<int, LaunchShape> shapes;  // per nrhs
};

namespace {

Geo make_geo(const int32_t d[4], uint32_t flags) {
  Geo g;
  g.L0 = d[0];
  g.L1 = d[1];
  g.L2 = d[2];
  g.L3 = d[3];
  g.Lh = d[0] / 2;
  g.hv = (int)((int64_t)d[0] * d[1] * d[2] * d[3] / 2);
  g.s1 = g.Lh;
  g.s2 = g.Lh * d[1];
  g.s3 = g.Lh * d[1] * d[2];
  g.anti_t = (flags & QX_BC_T_ANTIPERIODIC) ? 1 : 0;
  g.stream_links = 0;
  return g;
}

bool same_lattice(const qx_gauge* a, const qx_gauge* b) {
  return !memcmp(a->dims, b->dims, sizeof a->dims) && a->flags == b->flags;
}

// ------------------------------------------------------------ tuning cache

std::mutex g_tune_mu;
std::map<std::string, LaunchShape> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const qx_gauge* g, int nrhs) {
  char buf[128];
  snprintf(buf, sizeof buf, "gfx950:%dx%dx%dx%d:p%d:r%d:n%d", g->dims[0], g->dims[1], g->dims[2],
           g->dims[3], g->prec, g->recon, nrhs);
  return buf;
}

// The cache file is a flat JSON object {"key": [nbt, lps, xcd], ...}.  Entries
// read from a file replace those of the same key; malformed entries and
// shapes that are not compiled are skipped.
bool tune_read_file_locked(const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  std::string s;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
  fclose(f);
  size_t i = 0;
  while ((i = s.find('"', i)) != std::string::npos) {
    const size_t j = s.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = s.substr(i + 1, j - i - 1);
    int nbt = 0, lps = 0, x = 0;
    // the wide shapes only for FP32 one-hop links (keys ":p1:" without ":r36:")
    const bool wide = key.find(":p1:") != std::string::npos && key.find(":r36:") == std::string::npos;
    if (sscanf(s.c_str() + j + 1, " : [ %d , %d , %d ]", &nbt, &lps, &x) == 3 &&
        nbt_lps_instantiated(nbt, lps, wide))
      g_tune[key] = LaunchShape{nbt, lps, x < 0 ? 0 : x > kMaxOrder ? kMaxOrder : x};
    i = j + 1;
  }
  return true;
}

bool tune_write_file_locked(const char* path) {
  FILE* f = fopen(path, "w");
  if (!f) return false;
  fprintf(f, "{\n");
  size_t k = 0;
  for (const auto& kv : g_tune)
    fprintf(f, "  \"%s\": [%d, %d, %d]%s\n", kv.first.c_str(), kv.second.nbt, kv.second.lps,
            kv.second.xcd, ++k < g_tune.size() ? "," : "");
  fprintf(f, "}\n");
  return fclose(f) == 0;
}

// The file named by QX_TUNE_CACHE is read once, before the first lookup.
void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = getenv("QX_TUNE_CACHE");
  if (path && *path) tune_read_file_locked(path);
}

void tune_save_locked() {
  const char* path = getenv("QX_TUNE_CACHE");
  if (path && *path) tune_write_file_locked(path);
}

LaunchShape shape_for(const qx_gauge* g, int nrhs) {
  auto it = g->shapes.find(nrhs);
  if (it != g->shapes.end()) return it->second;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto jt = g_tune.find(tune_key(g, nrhs));
  if (jt != g_tune.end()) return jt->second;
  return LaunchShape{};
}

}  // namespace

// -------------------------------------------------------------------- misc

extern "C" int qx_version(void) { return QX_VERSION; }

extern "C" const char* qx_last_error(void) { return g_err.c_str(); }

// ----------------------------------------------------------------- lattice

extern "C" int qx_lattice_create(const int32_t dims[4], uint32_t flags, qx_lattice_t** out) {
  if (!dims || !out) return fail(QX_EINVAL, "qx_lattice_create: NULL argument");
  if (flags & ~(uint32_t)QX_BC_T_ANTIPERIODIC)
    return fail(QX_EINVAL, "qx_lattice_create: unknown flags 0x%x", flags);
  int64_t V = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (dims[mu] < 2 || (dims[mu] & 1))
      return fail(QX_EINVAL, "qx_lattice_create: extent %d of direction %d must be even and >= 2",
                  dims[mu], mu);
    V *= dims[mu];
  }
  if (V >= ((int64_t)1 << 31)) return fail(QX_EINVAL, "qx_lattice_create: volume %lld too large", (long long)V);
  qx_lattice* l = new (std::nothrow) qx_lattice;
  if (!l) return fail(QX_ENOMEM, "qx_lattice_create: out of host memory");
  memcpy(l->dims, dims, sizeof l->dims);
  l->flags = flags;
  l->geo = make_geo(dims, flags);
  l->V = V;
  *out = l;
  return QX_OK;
}

extern "C" int qx_lattice_destroy(qx_lattice_t* lat) {
  delete lat;
  return QX_OK;
}

extern "C" int64_t qx_lattice_volume(const qx_lattice_t* lat) { return lat ? lat->V : -1; }

extern "C" int qx_debug_index_maps(const qx_lattice_t* lat, int32_t* lex_of_eo, int32_t* nbr_eo,
                                   hipStream_t stream) {
  if (!lat || !lex_of_eo || !nbr_eo) return fail(QX_EINVAL, "qx_debug_index_maps: NULL argument");
  QX_HIP(launch_index_maps(lat->geo, lex_of_eo, nbr_eo, stream), "qx_debug_index_maps");
  return QX_OK;
}

// ------------------------------------------------------------------- gauge

namespace {
bool prec_ok(int p) { return p == QX_PREC_F64 || p == QX_PREC_F32 || p == QX_PREC_F16; }
bool recon_ok(int r) { return r == QX_RECON_18 || r == QX_RECON_12 || r == QX_RECON_NAIK; }
// recon / 2 complex numbers per (site, direction): 6, 9, or 9 + 9 for the
// improved operator's one-hop and three-hop links
size_t gauge_bytes(const Geo& g, int prec, int recon) {
  return (size_t)8 * g.hv * (recon / 2) * link_cplx_bytes(prec);
}
size_t field_bytes(const Geo& g, int nrhs, int prec) { return (size_t)nrhs * source_bytes(g, prec); }
}  // namespace

extern "C" int qx_gauge_bytes(const qx_lattice_t* lat, int prec, int recon, size_t* bytes) {
  if (!lat || !bytes || !prec_ok(prec) || !recon_ok(recon))
    return fail(QX_EINVAL, "qx_gauge_bytes: bad argument");
  *bytes = gauge_bytes(lat->geo, prec, recon);
  return QX_OK;
}

extern "C" int qx_gauge_load(const qx_lattice_t* lat, const void* U_canon, int prec, int recon,
                             void* packed, hipStream_t stream, qx_gauge_t** out) {
  if (!lat || !U_canon || !packed || !out) return fail(QX_EINVAL, "qx_gauge_load: NULL argument");
  if (!prec_ok(prec) || !recon_ok(recon))
    return fail(QX_EINVAL, "qx_gauge_load: bad precision %d or link storage %d", prec, recon);
  unsigned long long* d_err = nullptr;
  if (recon == 12) {
    QX_HIP(hipMalloc(&d_err, sizeof *d_err), "qx_gauge_load: hipMalloc");
    hipError_t e = hipMemsetAsync(d_err, 0, sizeof *d_err, stream);
    if (e != hipSuccess) {
      hipFree(d_err);
      return hip_fail(e, "qx_gauge_load: hipMemsetAsync");
    }
  }
  hipError_t e = launch_pack_gauge(lat->geo, U_canon, prec, recon, packed, d_err, stream);
  if (e != hipSuccess) {
    if (d_err) hipFree(d_err);
    return hip_fail(e, "qx_gauge_load: pack kernel");
  }
  if (recon == 12) {
    unsigned long long bits = 0;
    e = hipMemcpyAsync(&bits, d_err, sizeof bits, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    hipFree(d_err);
    if (e != hipSuccess) return hip_fail(e, "qx_gauge_load: unitarity check");
    double err;
    memcpy(&err, &bits, sizeof err);
    if (!(err <= 1e-10))
      return fail(QX_ENOTUNITARY,
                  "qx_gauge_load: 12-real links need SU(3) links; largest deviation of rows 0-1 "
                  "from orthonormality or of row 2 from conj(row0 x row1) = %g",
                  err);
  }
  qx_gauge* g = new (std::nothrow) qx_gauge;
  if (!g) return fail(QX_ENOMEM, "qx_gauge_load: out of host memory");
  memcpy(g->dims, lat->dims, sizeof g->dims);
  g->flags = lat->flags;
  g->geo = lat->geo;
  g->prec = prec;
  g->recon = recon;
  g->packed = packed;
  *out = g;
  return QX_OK;
}

extern "C" int qx_gauge_destroy(qx_gauge_t* g) {
  delete g;
  return QX_OK;
}

// ------------------------------------------------------------------ fields

extern "C" int qx_field_bytes(const qx_lattice_t* lat, int nrhs, int prec, size_t* bytes) {
  if (!lat || !bytes || nrhs < 1 || !prec_ok(prec))
    return fail(QX_EINVAL, "qx_field_bytes: bad argument");
  *bytes = field_bytes(lat->geo, nrhs, prec);
  return QX_OK;
}

extern "C" int qx_field_pack(const qx_lattice_t* lat, int nrhs, int prec, const void* canon,
                             void* packed, hipStream_t stream) {
  if (!lat || !canon || !packed || nrhs < 1 || !prec_ok(prec))
    return fail(QX_EINVAL, "qx_field_pack: bad argument");
  QX_HIP(launch_pack_field(lat->geo, nrhs, prec, canon, packed, stream), "qx_field_pack");
  return QX_OK;
}

extern "C" int qx_field_unpack(const qx_lattice_t* lat, int nrhs, int prec, const void* packed,
                               void* canon, hipStream_t stream) {
  if (!lat || !canon || !packed || nrhs < 1 || !prec_ok(prec))
    return fail(QX_EINVAL, "qx_field_unpack: bad argument");
  QX_HIP(launch_unpack_field(lat->geo, nrhs, prec, packed, canon, stream), "qx_field_unpack");
  return QX_OK;
}

// --------------------------------------------------------------- operators

extern "C" int qx_dslash(const qx_gauge_t* g, int out_parity, int nrhs, const void* in, void* out,
                         hipStream_t stream) {
  if (!g || !in || !out || nrhs < 1 || (out_parity != 0 && out_parity != 1))
    return fail(QX_EINVAL, "qx_dslash: bad argument");
  if (in == out) return fail(QX_EINVAL, "qx_dslash: in and out must not alias");
  QX_HIP(launch_dslash(g->geo, g->prec, g->recon, g->packed, out_parity, in, out, nrhs, 0.5,
                       shape_for(g, nrhs), stream),
         "qx_dslash");
  return QX_OK;
}

extern "C" int qx_apply_A_noalloc(const qx_gauge_t* g, int nrhs, const double* masses,
                                  const void* in, void* out, hipStream_t stream) {
  if (!g || !masses || !in || !out || nrhs < 1)
    return fail(QX_EINVAL, "qx_apply_A_noalloc: bad argument");
  if (in == out) return fail(QX_EINVAL, "qx_apply_A_noalloc: buffers must not alias");
  const size_t need = (size_t)nrhs * source_bytes(g->geo, g->prec);
  if (need > kNoAllocScratchBytes)
    return fail(QX_EINVAL,
                "qx_apply_A_noalloc: %d sources need %zu bytes of scratch; the library's array "
                "holds %zu (use qx_apply_A with a workspace)",
                nrhs, need, kNoAllocScratchBytes);
  QX_HIP(launch_apply_A_noalloc(g->geo, g->prec, g->recon, g->packed, nrhs, masses, in, out,
                                shape_for(g, nrhs), stream),
         "qx_apply_A_noalloc");
  return QX_OK;
}

extern "C" int qx_apply_A(const qx_gauge_t* g, int nrhs, const double* masses, const void* in,
                          void* out, void* tmp_odd, hipStream_t stream) {
  if (!g || !masses || !in || !out || !tmp_odd || nrhs < 1)
    return fail(QX_EINVAL, "qx_apply_A: bad argument");
  if (in == out || in == tmp_odd || out == tmp_odd)
    return fail(QX_EINVAL, "qx_apply_A: buffers must not alias");
  std::vector<double> m2(nrhs);
  for (int k = 0; k < nrhs; ++k) m2[k] = masses[k] * masses[k];
  QX_HIP(launch_apply_A(g->geo, g->prec, g->recon, g->packed, nrhs, m2.data(), in, out, tmp_odd,
                        shape_for(g, nrhs), stream),
         "qx_apply_A");
  return QX_OK;
}

// ------------------------------------------------------------------ solver

namespace {

constexpr int kMaxSrcPerSys = 12;
constexpr double kStopFactor = 0.9;  // stop at an FP64 residual of 0.9 tol
constexpr int kFuseMaxBlocks = 1024;  // AUTO engine: fused sequence up to V/2 = 65536 per system
constexpr bool kAutoTwo = true;       // AUTO engine: the two-launch form of the fused sequence
constexpr int kTwoMaxPartials = 4096;
constexpr int kTwoMaxSources = 3;

struct SysSpec {
  const qx_gauge* g64;
  const qx_gauge* glo;  // == g64 for QX_CG_FP64
  int nrhs;
  std::vector<double> masses;
  const void* b;  // canonical, already offset to the first source of this system
  void* x;
};

struct Layout {
  size_t sys_off = 0, st_off = 0, gs_off = 0, total = 0;
  std::vector<size_t> partial_off, partial_x_off, partial_v_off, vlo_off, vhi_off;
};

int lo_prec(const qx_cg_params_t* p) { return p->mode == QX_CG_FP64 ? QX_PREC_F64 : QX_PREC_F32; }

// Does the batch run the two-launch fused sequence (its r' slot and extra
// partials)?  Under AUTO only for systems of at most kTwoMaxSources sources
// whose D_oe blocks each read at most kTwoMaxPartials partial sums (four per
// source and stencil block): its D_oe pass loads r, Ap and p at every
// neighbour and adds each source's sums in turn, which outweighs the launch it
// saves beyond that (mixed solves against the three-launch sequence: 16^4
// with 1 / 2 / 3 / 4 / 12 sources 0.85 / 0.96 / 0.99 / 1.09 / 1.19 of its
// time, 16^3 x 32 with 1 / 3 sources 0.96 / 1.03, 12^4 with 3 / 4 sources
// 0.98 / 1.02).
bool uses_two(const std::vector<SysSpec>& specs, int engine) {
  if (engine == QX_ENGINE_FUSED2) return true;
  if (engine != QX_ENGINE_AUTO || !kAutoTwo) return false;
  for (const auto& s : specs) {
    const int nblk = (s.g64->geo.hv + kTile - 1) / kTile;
    if (nblk > kFuseMaxBlocks || s.nrhs > kTwoMaxSources || 4 * s.nrhs * nblk > kTwoMaxPartials)
      return false;
  }
  return true;
}

Layout plan_layout(const std::vector<SysSpec>& specs, int prec_lo, int engine) {
  Layout L;
  const bool two = uses_two(specs, engine);
  size_t off = 0;
  L.sys_off = off;
  off = align_up(off + sizeof(SysDesc) * specs.size(), 256);
  L.st_off = off;
  size_t nsrc = 0;
  for (const auto& s : specs) nsrc += s.nrhs;
  off = align_up(off + 2 * sizeof(SrcState) * nsrc, 256);  // two state slots
  L.gs_off = off;
  off = align_up(off + sizeof(GridSync), 256);
  for (const auto& s : specs) {
    const Geo& g = s.g64->geo;
    const int nblk = (g.hv + kTile - 1) / kTile;
    const int vtiles = (3 * g.hv + kVTile - 1) / kVTile;
    L.partial_off.push_back(off);
    off = align_up(off + sizeof(double) * s.nrhs * nblk, 256);
    L.partial_x_off.push_back(off);
    if (two) off = align_up(off + 3 * sizeof(double) * s.nrhs * nblk, 256);
    L.partial_v_off.push_back(off);
    off = align_up(off + sizeof(double) * s.nrhs * vtiles, 256);
    L.vlo_off.push_back(off);
    off = align_up(off + (two ? 7 : 6) * field_bytes(g, s.nrhs, prec_lo), 256);
    L.vhi_off.push_back(off);
    off = align_up(off + 4 * field_bytes(g, s.nrhs, QX_PREC_F64), 256);
  }
  L.total = off;
  return L;
}

int check_params(const qx_cg_params_t* p) {
  if (!p) return fail(QX_EINVAL, "solver: NULL params");
  if (!(p->tol > 0.0) || p->max_iter < 1) return fail(QX_EINVAL, "solver: tol must be > 0 and max_iter >= 1");
  if (p->mode != QX_CG_FP64 && p->mode != QX_CG_MIXED_F32)
    return fail(QX_EINVAL, "solver: unknown mode %d", p->mode);
  if (p->mode == QX_CG_MIXED_F32 && !(p->delta > 0.0 && p->delta < 1.0))
    return fail(QX_EINVAL, "solver: delta must be in (0, 1) for the mixed mode");
  if (p->chunk < 0) return fail(QX_EINVAL, "solver: chunk must be >= 0");
  if (p->engine < QX_ENGINE_AUTO || p->engine > QX_ENGINE_FUSED2)
    return fail(QX_EINVAL, "solver: unknown engine %d", p->engine);
  return QX_OK;
}

int check_system(const qx_gauge* g64, const qx_gauge* glo, const qx_cg_params_t* p) {
  if (!g64) return fail(QX_EINVAL, "solver: NULL FP64 gauge handle");
  if (g64->prec != QX_PREC_F64) return fail(QX_EINVAL, "solver: g64 must be an FP64 gauge handle");
  if (p->mode == QX_CG_MIXED_F32) {
    if (!glo) return fail(QX_EINVAL, "solver: the mixed mode needs an FP32 or FP16 gauge handle");
    if (glo->prec != QX_PREC_F32 && glo->prec != QX_PREC_F16)
      return fail(QX_EINVAL, "solver: glo must be an FP32 or FP16 gauge handle");
    if (!same_lattice(g64, glo)) return fail(QX_EINVAL, "solver: g64 and glo are on different lattices");
    if ((glo->recon == QX_RECON_NAIK) != (g64->recon == QX_RECON_NAIK))
      return fail(QX_EINVAL, "solver: g64 and glo must both hold the improved (Naik) operator or neither");
  }
  return QX_OK;
}

// Split a caller system into pieces of at most kMaxSrcPerSys sources.
void add_specs(std::vector<SysSpec>& out, const qx_gauge* g64, const qx_gauge* glo,
               const qx_cg_params_t* p, int nrhs, const double* masses, const void* b, void* x) {
  const size_t fb = field_bytes(g64->geo, 1, QX_PREC_F64);  // canonical bytes per source
  for (int k0 = 0; k0 < nrhs; k0 += kMaxSrcPerSys) {
    SysSpec s;
    s.g64 = g64;
    s.glo = p->mode == QX_CG_FP64 ? g64 : glo;
    s.nrhs = std::min(kMaxSrcPerSys, nrhs - k0);
    s.masses.assign(masses + k0, masses + k0 + s.nrhs);
    s.b = (const char*)b + k0 * fb;
    s.x = (char*)x + k0 * fb;
    out.push_back(s);
  }
}

}  // namespace

// A planned solve: systems, their device descriptors and states inside the
// caller's workspace, a pinned host mirror of the states, and (optionally) the
// captured graph of one chunk of iterations.
struct qx_batch {
  std::vector<SysSpec> specs;
  qx_cg_params_t params;
  Layout layout;
  EngineCfg cfg;
  std::vector<SysDesc> sys;
  std::vector<SrcState> st0;
  SrcState* h_st = nullptr;  // pinned mirror of the workspace from the states to the barrier word
  SrcState* h_st0 = nullptr;  // pinned initial states (written once, at create)
  GridSync* h_gs = nullptr;  // inside h_st's buffer
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int chunk = 16, ru_every = 4;
  bool forced = false;         // launch shape set by qx_batch_tune
  LaunchShape forced_shape{};
  bool deo_forced = false;     // D_eo shape of the launch-per-pass engine set by qx_batch_tune
  LaunchShape deo_shape{};
  bool use_graph = false;
  bool persistent = false;
  int pgrid = 0;
  hipGraphExec_t graph = nullptr;
  hipStream_t graph_stream = nullptr;

  ~qx_batch() {
    if (graph) hipGraphExecDestroy(graph);
    if (h_st) hipHostFree(h_st);
    if (h_st0) hipHostFree(h_st0);
  }
};

namespace {

int build_plan(qx_batch* B, void* ws, size_t ws_bytes) {
  const qx_cg_params_t& p = B->params;
  const int prec_lo = lo_prec(&p);
  B->layout = plan_layout(B->specs, prec_lo, p.engine);
  if (!ws) return fail(QX_EINVAL, "solver: NULL workspace");
  if (ws_bytes < B->layout.total)
    return fail(QX_ENOMEM, "solver: workspace of %zu bytes, %zu needed", ws_bytes, B->layout.total);
  B->ws = (char*)ws;

  // launch shape: the tuned (or default) shape of the first system's inner links
  const SysSpec& s0 = B->specs[0];
  int nb = 1;
  for (const auto& s : B->specs) nb = std::max(nb, s.nrhs);
  LaunchShape sh = shape_for(s0.glo, nb);
  // The D_oe pass of the fused sequence loads r and p at every neighbour;
  // with all hops of one source in one wavefront that spills, so on batches
  // the fused sequence serves (AUTO) every engine splits the hops in two (the
  // engines agree bit for bit for one batch).
  int max_nblk = 0;
  for (const auto& s : B->specs) max_nblk = std::max(max_nblk, (s.g64->geo.hv + kTile - 1) / kTile);
  if (sh.nbt == 1 && sh.lps == 1 && max_nblk <= kFuseMaxBlocks) {
    LaunchShape s2 = sh;
    s2.lps = 2;
    if (shape_ok(s2, nb, cplx_bytes(prec_lo))) sh = s2;
  }
  // On batches the fused sequences serve, the solver's passes read at
  // neighbouring sites what the previous pass wrote; with each XCD on a
  // contiguous range of blocks (order 1) most of it is still in that XCD's
  // L2.  There the Dslash tuner's order 0 (dispatch order) is replaced: at
  // 16^4 the mixed solve took 3.85 ms under (1, 4, 0) and 3.60 ms under
  // (1, 4, 1).  (At 32^4 the tuned order stays: FP64 with twelve sources
  // was 8 % slower under order 1 than under the tuned order 0.)
  if (sh.xcd == 0 && max_nblk <= kFuseMaxBlocks) sh.xcd = 1;
  if (!shape_ok(sh, nb, cplx_bytes(prec_lo)) ||
      !nbt_lps_instantiated(sh.nbt, sh.lps,
                            wide_compiled(prec_lo, s0.glo->recon) && s0.glo->prec != QX_PREC_F16)) {
    // the first default that takes nb sources in one block
    const LaunchShape cands[4] = {{1, 2, 1}, {2, 2, 1}, {4, 2, 1}, {4, 1, 1}};
    sh = cands[0];
    for (const LaunchShape& c : cands)
      if (shape_ok(c, nb, cplx_bytes(prec_lo))) {
        sh = c;
        break;
      }
  }
  // Batches the launch-per-pass engine serves with several sources per
  // thread run fastest in dispatch order, whatever the Dslash tuner found
  // for the kernel alone: 32^4 with twelve sources, mixed 1.14 s under
  // (4, 2, 0) against 1.18 s under the tuned (4, 2, 1); FP64 2.19 s against
  // 2.37 s.  (One source per thread keeps the tuned order: at 32^4 the tuned
  // shapes were within 1-2 % of the best there.)
  if (max_nblk > kFuseMaxBlocks && sh.nbt > 1 && sh.xcd < 4) sh.xcd = 0;
  if (B->forced) sh = B->forced_shape;

  B->cfg = EngineCfg{};
  B->cfg.prec_lo = prec_lo;
  B->cfg.recon_lo = s0.glo->recon;
  B->cfg.recon_hi = s0.g64->recon;
  // FP16 inner links: the vectors and the arithmetic stay FP32
  B->cfg.links16 = s0.glo->prec == QX_PREC_F16;
  for (const auto& s : B->specs) {
    if (s.glo->recon != B->cfg.recon_lo || s.g64->recon != B->cfg.recon_hi ||
        s.glo->prec != s0.glo->prec)
      return fail(QX_EINVAL, "batch: all systems must use the same link storage");
  }
  B->cfg.nsrc_max = nb;
  // six or twelve sources per thread are compiled for the launch-per-pass
  // stencils of FP32 one-hop links only: other paths take at most four
  const bool fused_planned = p.engine == QX_ENGINE_FUSED || p.engine == QX_ENGINE_FUSED2 ||
                             (p.engine == QX_ENGINE_AUTO && max_nblk <= kFuseMaxBlocks);
  const bool wide_ok = wide_compiled(prec_lo, s0.glo->recon) && s0.glo->prec != QX_PREC_F16 &&
                       !fused_planned && p.engine != QX_ENGINE_PERSISTENT;
  if (!wide_ok) sh = narrow_shape(sh);
  B->cfg.shape = sh;
  B->cfg.nsys = (int)B->specs.size();
  B->cfg.d_sys = (const SysDesc*)(B->ws + B->layout.sys_off);
  B->cfg.d_st = (SrcState*)(B->ws + B->layout.st_off);
  {
    int nsrc_all = 0;
    for (const auto& s : B->specs) nsrc_all += s.nrhs;
    B->cfg.d_st1 = B->cfg.d_st + nsrc_all;
  }

  B->sys.clear();
  B->st0.clear();
  int blk = 0, vblk = 0, src = 0;
  const double stop = kStopFactor * p.tol;
  for (size_t i = 0; i < B->specs.size(); ++i) {
    const SysSpec& s = B->specs[i];
    SysDesc d{};
    d.g = s.g64->geo;
    d.g.stream_links = gauge_bytes(d.g, s.glo->prec, s.glo->recon) > kStreamLinkBytes &&
                       shape_groups(sh, nb) == 1;
    d.nsrc = s.nrhs;
    d.src0 = src;
    d.blk0 = blk;
    d.nblk = (d.g.hv + kTile - 1) / kTile;
    d.vblk0 = vblk;
    d.vtiles = (3 * d.g.hv + kVTile - 1) / kVTile;
    d.links_lo = s.glo->packed;
    d.links_hi = s.g64->packed;
    d.vlo = B->ws + B->layout.vlo_off[i];
    d.vhi = B->ws + B->layout.vhi_off[i];
    d.partials = (double*)(B->ws + B->layout.partial_off[i]);
    d.partials_x = (double*)(B->ws + B->layout.partial_x_off[i]);
    d.partials_v = (double*)(B->ws + B->layout.partial_v_off[i]);
    blk += d.nblk;
    vblk += d.nsrc * d.vtiles;
    src += d.nsrc;
    B->sys.push_back(d);
    for (int k = 0; k < s.nrhs; ++k) {
      SrcState q{};
      q.m2 = s.masses[k] * s.masses[k];
      q.delta = p.mode == QX_CG_FP64 ? 0.0 : p.delta;
      q.stop2 = stop * stop;  // multiplied by |b|^2 on the device
      q.phase = PH_RU;
      q.reason = RU_INIT;
      q.status = QX_ENOTCONVERGED;
      q.max_iter = p.max_iter;
      B->st0.push_back(q);
    }
  }
  B->cfg.nblk_total = blk;
  B->cfg.nvblk_total = vblk;
  B->cfg.nsrc_total = src;
  if (!engine_supported(B->cfg)) return fail(QX_EINVAL, "solver: unsupported configuration");
  const size_t mirror = B->layout.gs_off - B->layout.st_off + sizeof(GridSync);
  if (!B->h_st) QX_HIP(hipHostMalloc((void**)&B->h_st, mirror), "solver: hipHostMalloc");
  if (!B->h_st0)
    QX_HIP(hipHostMalloc((void**)&B->h_st0, sizeof(SrcState) * B->st0.size()),
           "solver: hipHostMalloc");
  memcpy(B->h_st0, B->st0.data(), sizeof(SrcState) * B->st0.size());
  B->h_gs = (GridSync*)((char*)B->h_st + (B->layout.gs_off - B->layout.st_off));
  // engine: launch per pass unless the persistent kernel is asked for
  B->persistent = false;
  if (p.engine == QX_ENGINE_PERSISTENT) {
    const int cap = engine_persistent_capacity(B->cfg);
    if (cap < 1)
      return fail(QX_EINVAL, "solver: the persistent engine cannot be launched on this device");
    B->persistent = true;
    // half the occupancy bound: a grid at the bound has timed out in a barrier
    // (blocks left unscheduled), the grid-stride passes take any grid size
    B->pgrid = std::max(1, std::min(cap / 2, B->cfg.nblk_total));
  }
  // the fused launch sequence finishes each reduction in every block of the
  // next vector pass: cheap while a source has few partials
  B->cfg.fused = false;
  if (!B->persistent) {
    int max_nblk = 0;
    for (const auto& d : B->sys) max_nblk = std::max(max_nblk, d.nblk);
    B->cfg.fused = p.engine == QX_ENGINE_FUSED || p.engine == QX_ENGINE_FUSED2 ||
                   (p.engine == QX_ENGINE_AUTO && max_nblk <= kFuseMaxBlocks);
  }
  B->cfg.two = B->cfg.fused && uses_two(B->specs, p.engine);
  // the launch-per-pass D_eo pass: the tuner's own choice, else the shape of
  // the other stencils
  B->cfg.deo_shape = B->cfg.shape;
  if (B->deo_forced && !B->cfg.fused && !B->persistent) {
    B->cfg.deo_shape.nbt = B->deo_shape.nbt;
    B->cfg.deo_shape.lps = B->deo_shape.lps;
  }
  if (B->persistent) {
    B->chunk = p.chunk > 0 ? p.chunk : 512;
    B->ru_every = B->chunk;
    B->use_graph = false;
  } else {
    B->chunk = p.chunk > 0 ? p.chunk : 16;
    // the fused sequence alternates two p slots: even chunks and update periods
    if (B->cfg.fused) B->chunk += B->chunk & 1;
    // An update slot costs its launches even when no source takes it.  A mixed
    // solve updates every few iterations (every 14 on the 16^4 system), so
    // it gets a slot every 4; an FP64 solve only checks its converged
    // residual, so one slot per chunk (16^4 FP64: 4.74 against 4.84 ms with
    // a slot every 4; mixed: 3.58 ms every 4, 3.78 every 16).
    B->ru_every = p.mode == QX_CG_FP64 ? B->chunk : std::min(B->chunk, 4);
  }
  return QX_OK;
}

// Upload the descriptor table and clear the grid barrier word.
int upload_plan(qx_batch* B, hipStream_t s) {
  QX_HIP(hipMemcpyAsync(B->ws + B->layout.sys_off, B->sys.data(), sizeof(SysDesc) * B->sys.size(),
                        hipMemcpyHostToDevice, s),
         "solver: descriptor upload");
  QX_HIP(hipMemsetAsync(B->ws + B->layout.gs_off, 0, sizeof(GridSync), s), "solver: barrier reset");
  QX_HIP(hipStreamSynchronize(s), "solver: upload");
  return QX_OK;
}

// The work of one chunk: `chunk` inner iterations with a reliable-update
// sequence after every `ru_every` of them and at the end, then a copy of the
// source states to the pinned host mirror.
int enqueue_chunk(qx_batch* B, hipStream_t s) {
  if (B->persistent) {
    QX_HIP(engine_persistent(B->cfg, B->chunk, (GridSync*)(B->ws + B->layout.gs_off), B->pgrid, s),
           "solver: persistent iterations");
    QX_HIP(engine_reliable_update(B->cfg, true, s), "solver: reliable update");
  } else {
    for (int i = 0; i < B->chunk; ++i) {
      QX_HIP(engine_iteration(B->cfg, i & 1, s), "solver: iteration");
      if ((i + 1) % B->ru_every == 0 || i + 1 == B->chunk)
        QX_HIP(engine_reliable_update(B->cfg, i + 1 == B->chunk, s), "solver: reliable update");
    }
  }
  const size_t n = B->persistent ? B->layout.gs_off - B->layout.st_off + sizeof(GridSync)
                                  : sizeof(SrcState) * B->cfg.nsrc_total;
  QX_HIP(hipMemcpyAsync(B->h_st, B->cfg.d_st, n, hipMemcpyDeviceToHost, s), "solver: state readback");
  return QX_OK;
}

int capture_graph(qx_batch* B, hipStream_t s) {
  if (B->graph) {
    hipGraphExecDestroy(B->graph);
    B->graph = nullptr;
  }
  if (!B->use_graph || s == nullptr) return QX_OK;
  hipGraph_t graph = nullptr;
  QX_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "batch: begin capture");
  int rc = enqueue_chunk(B, s);
  hipError_t e = hipStreamEndCapture(s, &graph);
  if (rc != QX_OK) {
    if (graph) hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "batch: end capture");
  e = hipGraphInstantiate(&B->graph, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) {
    B->graph = nullptr;
    return hip_fail(e, "batch: graph instantiate");
  }
  B->graph_stream = s;
  return QX_OK;
}

// Enqueue the start of a solve: initial states, b (and x0) packed, the
// engine's initialisation and the initial residual; the chunk graph is
// captured again if the stream differs from the one it was captured on.
int enqueue_start(qx_batch* B, hipStream_t s) {
  const qx_cg_params_t& p = B->params;
  QX_HIP(hipMemcpyAsync(B->cfg.d_st, B->h_st0, sizeof(SrcState) * B->st0.size(),
                        hipMemcpyHostToDevice, s),
         "solver: state upload");
  for (size_t i = 0; i < B->specs.size(); ++i) {
    const SysSpec& sp = B->specs[i];
    const SysDesc& d = B->sys[i];
    const size_t vs = field_bytes(d.g, d.nsrc, QX_PREC_F64);
    QX_HIP(launch_pack_field(d.g, d.nsrc, QX_PREC_F64, sp.b, (char*)d.vhi + 2 * vs, s),
           "solver: pack b");
    if (p.use_x0)
      QX_HIP(launch_pack_field(d.g, d.nsrc, QX_PREC_F64, sp.x, d.vhi, s), "solver: pack x0");
  }
  if (B->persistent)
    QX_HIP(hipMemsetAsync(B->ws + B->layout.gs_off, 0, sizeof(GridSync), s), "solver: barrier reset");
  QX_HIP(engine_init(B->cfg, p.use_x0 ? 0 : 1, s), "solver: init");
  QX_HIP(engine_reliable_update(B->cfg, true, s), "solver: initial residual");
  if (B->use_graph && B->graph && B->graph_stream != s) {
    int rc = capture_graph(B, s);
    if (rc != QX_OK) return rc;
  }
  return QX_OK;
}

int enqueue_one_chunk(qx_batch* B, hipStream_t s) {
  if (B->graph) {
    QX_HIP(hipGraphLaunch(B->graph, s), "solver: graph launch");
    return QX_OK;
  }
  return enqueue_chunk(B, s);
}

// Unpack the FP64 solutions into the callers' x buffers.
int enqueue_finish(qx_batch* B, hipStream_t s) {
  for (size_t i = 0; i < B->specs.size(); ++i) {
    const SysDesc& d = B->sys[i];
    QX_HIP(launch_unpack_field(d.g, d.nsrc, QX_PREC_F64, d.vhi, B->specs[i].x, s),
           "solver: unpack x");
  }
  return QX_OK;
}

int run_plan(qx_batch* B, qx_cg_stats_t* stats, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const qx_cg_params_t& p = B->params;
  int rc = enqueue_start(B, s);
  if (rc != QX_OK) return rc;
  const long max_chunks = (long)p.max_iter + 64;
  bool done = false;
  for (long c = 0; c < max_chunks && !done; ++c) {
    rc = enqueue_one_chunk(B, s);
    if (rc != QX_OK) return rc;
    QX_HIP(hipStreamSynchronize(s), "solver: chunk");
    if (B->persistent && B->h_gs->error)
      return fail(QX_EHIP, "solver: a grid barrier of the persistent kernel timed out");
    done = true;
    for (int k = 0; k < B->cfg.nsrc_total; ++k)
      if (B->h_st[k].phase != PH_DONE) done = false;
  }
  if (!done) return fail(QX_EHIP, "solver: the state machine did not terminate");
  rc = enqueue_finish(B, s);
  if (rc != QX_OK) return rc;
  QX_HIP(hipStreamSynchronize(s), "solver: finish");
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int k = 0; k < B->cfg.nsrc_total; ++k) {
    const SrcState& q = B->h_st[k];
    if (stats) {
      stats[k].status = q.status;
      stats[k].iters = q.iters;
      stats[k].reliable_updates = q.updates;
      stats[k].true_rel_residual = q.relres;
      stats[k].seconds = secs;
    }
    if (q.status != QX_OK && rc == QX_OK) rc = q.status;
  }
  if (rc != QX_OK)
    fail(rc, rc == QX_ENOTCONVERGED ? "solver: max_iter reached before the tolerance"
                                    : "solver: breakdown (<p,Ap> <= 0 or non-finite values)");
  return rc;
}

}  // namespace

extern "C" int qx_cg_workspace_bytes(const qx_lattice_t* lat, const qx_cg_params_t* params,
                                     int nrhs, size_t* bytes) {
  if (!lat || !bytes || nrhs < 1) return fail(QX_EINVAL, "qx_cg_workspace_bytes: bad argument");
  int rc = check_params(params);
  if (rc) return rc;
  qx_gauge tmp;
  memcpy(tmp.dims, lat->dims, sizeof tmp.dims);
  tmp.flags = lat->flags;
  tmp.geo = lat->geo;
  tmp.prec = QX_PREC_F64;
  tmp.recon = 18;
  tmp.packed = nullptr;
  std::vector<SysSpec> specs;
  std::vector<double> m(nrhs, 0.0);
  add_specs(specs, &tmp, &tmp, params, nrhs, m.data(), nullptr, nullptr);
  *bytes = plan_layout(specs, lo_prec(params), params->engine).total;
  return QX_OK;
}

extern "C" int qx_cg_solve(const qx_gauge_t* g64, const qx_gauge_t* glo,
                           const qx_cg_params_t* params, int nrhs, const double* masses,
                           const void* b, void* x, void* ws, size_t ws_bytes,
                           qx_cg_stats_t* stats, hipStream_t stream) {
  int rc = check_params(params);
  if (rc) return rc;
  rc = check_system(g64, glo, params);
  if (rc) return rc;
  if (nrhs < 1 || !masses || !b || !x) return fail(QX_EINVAL, "qx_cg_solve: bad argument");
  qx_batch B;
  B.params = *params;
  add_specs(B.specs, g64, glo, params, nrhs, masses, b, x);
  rc = build_plan(&B, ws, ws_bytes);
  if (rc) return rc;
  rc = upload_plan(&B, stream);
  if (rc) return rc;
  return run_plan(&B, stats, stream);
}

// ----------------------------------------------------------------- batches

extern "C" int qx_batch_workspace_bytes(int nsys, const qx_system_t* systems,
                                        const qx_cg_params_t* params, size_t* bytes) {
  if (nsys < 1 || !systems || !bytes) return fail(QX_EINVAL, "qx_batch_workspace_bytes: bad argument");
  int rc = check_params(params);
  if (rc) return rc;
  std::vector<SysSpec> specs;
  for (int i = 0; i < nsys; ++i) {
    const qx_system_t& s = systems[i];
    if (!s.g64 || s.nrhs < 1 || !s.masses) return fail(QX_EINVAL, "batch: bad system %d", i);
    add_specs(specs, s.g64, s.glo ? s.glo : s.g64, params, s.nrhs, s.masses, s.b, s.x);
  }
  *bytes = plan_layout(specs, lo_prec(params), params->engine).total;
  return QX_OK;
}

extern "C" int qx_batch_create(int nsys, const qx_system_t* systems, const qx_cg_params_t* params,
                               void* ws, size_t ws_bytes, hipStream_t stream, qx_batch_t** out) {
  if (nsys < 1 || !systems || !out) return fail(QX_EINVAL, "qx_batch_create: bad argument");
  int rc = check_params(params);
  if (rc) return rc;
  qx_batch* B = new (std::nothrow) qx_batch;
  if (!B) return fail(QX_ENOMEM, "qx_batch_create: out of host memory");
  B->params = *params;
  for (int i = 0; i < nsys; ++i) {
    const qx_system_t& s = systems[i];
    rc = check_system(s.g64, s.glo, params);
    if (!rc && (s.nrhs < 1 || !s.masses || !s.b || !s.x))
      rc = fail(QX_EINVAL, "qx_batch_create: bad system %d", i);
    if (rc) {
      delete B;
      return rc;
    }
    add_specs(B->specs, s.g64, s.glo, params, s.nrhs, s.masses, s.b, s.x);
  }
  if ((int)B->specs.size() > kMaxSys) {
    delete B;
    return fail(QX_EINVAL, "qx_batch_create: at most %d systems of <= 12 sources", kMaxSys);
  }
  const char* env = getenv("QX_GRAPH");
  B->use_graph = !(env && env[0] == '0');
  B->ws_bytes = ws_bytes;
  rc = build_plan(B, ws, ws_bytes);
  if (!rc) rc = upload_plan(B, stream);
  if (!rc) rc = capture_graph(B, stream);
  if (rc) {
    delete B;
    return rc;
  }
  *out = B;
  return QX_OK;
}

// Plan, upload and capture the batch under its current shape choice.
static int replan(qx_batch* B, hipStream_t s) {
  int rc = build_plan(B, B->ws, B->ws_bytes);
  if (!rc) rc = upload_plan(B, s);
  if (!rc) rc = capture_graph(B, s);
  return rc;
}

extern "C" int qx_batch_set_launch(qx_batch_t* batch, int nbt, int lps, int order,
                                   hipStream_t stream) {
  if (!batch) return fail(QX_EINVAL, "qx_batch_set_launch: NULL batch");
  qx_batch* B = batch;
  if (B->persistent) return fail(QX_EINVAL, "qx_batch_set_launch: not for the persistent engine");
  int nb = 1;
  for (const auto& sp : B->specs) nb = std::max(nb, sp.nrhs);
  const LaunchShape sh{nbt, lps, order};
  const size_t csz = cplx_bytes(lo_prec(&B->params));
  const bool wide = wide_compiled(B->cfg.prec_lo, B->cfg.recon_lo) && !B->cfg.links16;
  if (!nbt_lps_instantiated(nbt, lps, wide) || !shape_ok(sh, nb, csz))
    return fail(QX_EINVAL, "qx_batch_set_launch: shape (%d, %d, %d) not available", nbt, lps, order);
  B->forced = true;
  B->forced_shape = sh;
  B->deo_forced = false;
  return replan(B, stream);
}

extern "C" int qx_batch_set_deo_launch(qx_batch_t* batch, int deo_nbt, int deo_lps,
                                       hipStream_t stream) {
  if (!batch) return fail(QX_EINVAL, "qx_batch_set_deo_launch: NULL batch");
  qx_batch* B = batch;
  if (B->persistent || B->cfg.fused)
    return fail(QX_EINVAL, "qx_batch_set_deo_launch: only for the launch-per-pass engine");
  int nb = 1;
  for (const auto& sp : B->specs) nb = std::max(nb, sp.nrhs);
  const LaunchShape dsh{deo_nbt, deo_lps, B->cfg.shape.xcd};
  const size_t csz = cplx_bytes(lo_prec(&B->params));
  const bool wide = wide_compiled(B->cfg.prec_lo, B->cfg.recon_lo) && !B->cfg.links16;
  if (!nbt_lps_instantiated(deo_nbt, deo_lps, wide) || !shape_ok(dsh, nb, csz))
    return fail(QX_EINVAL, "qx_batch_set_deo_launch: shape (%d, %d) not available", deo_nbt,
                deo_lps);
  B->forced = true;
  B->forced_shape = B->cfg.shape;
  B->deo_forced = true;
  B->deo_shape = dsh;
  return replan(B, stream);
}

extern "C" int qx_batch_get_launch(qx_batch_t* batch, int* nbt, int* lps, int* order,
                                   int* deo_nbt, int* deo_lps) {
  if (!batch) return fail(QX_EINVAL, "qx_batch_get_launch: NULL batch");
  const EngineCfg& c = batch->cfg;
  if (nbt) *nbt = c.shape.nbt;
  if (lps) *lps = c.shape.lps;
  if (order) *order = c.shape.xcd;
  if (deo_nbt) *deo_nbt = c.deo_shape.nbt;
  if (deo_lps) *deo_lps = c.deo_shape.lps;
  return QX_OK;
}

static_assert(PASS_P == QX_PASS_P && PASS_DOE == QX_PASS_DOE && PASS_DEO == QX_PASS_DEO &&
                  PASS_XR == QX_PASS_XR && PASS_FINALIZE == QX_PASS_FINALIZE &&
                  PASS_UPDATE == QX_PASS_UPDATE && NPASS == QX_NPASS,
              "pass kinds");

extern "C" int qx_batch_profile(qx_batch_t* batch, int nchunks, qx_pass_stats_t* passes,
                                qx_cg_stats_t* stats, hipStream_t stream) {
  if (!batch || !passes || nchunks < 1 || nchunks > 64)
    return fail(QX_EINVAL, "qx_batch_profile: bad argument");
  qx_batch* B = batch;
  if (B->persistent) return fail(QX_EINVAL, "qx_batch_profile: not for the persistent engine");
  const int n = B->cfg.nsrc_total;
  // the number of sources in the given phase, read from the device states
  auto count = [&](int phase, int* out) -> int {
    QX_HIP(hipMemcpyAsync(B->h_st, B->cfg.d_st, sizeof(SrcState) * n, hipMemcpyDeviceToHost, stream),
           "qx_batch_profile: state readback");
    QX_HIP(hipStreamSynchronize(stream), "qx_batch_profile: state readback");
    int c = 0;
    for (int k = 0; k < n; ++k) c += B->h_st[k].phase == phase;
    *out = c;
    return QX_OK;
  };
  int rc = enqueue_start(B, stream);
  if (rc) return rc;
  PassProf prof;
  B->cfg.prof = &prof;
  // the launch sequence of enqueue_chunk, enqueued eagerly, the host reading
  // the states before each iteration and update to tag the launches
  for (int c = 0; c < nchunks && !rc; ++c)
    for (int i = 0; i < B->chunk && !rc; ++i) {
      rc = count(PH_RUN, &prof.nrun);
      if (rc) break;
      if (engine_iteration(B->cfg, i & 1, stream) != hipSuccess) {
        rc = fail(QX_EHIP, "qx_batch_profile: iteration");
        break;
      }
      if ((i + 1) % B->ru_every == 0 || i + 1 == B->chunk) {
        rc = count(PH_RU, &prof.nrun);
        if (!rc && engine_reliable_update(B->cfg, i + 1 == B->chunk, stream) != hipSuccess)
          rc = fail(QX_EHIP, "qx_batch_profile: reliable update");
      }
    }
  B->cfg.prof = nullptr;
  if (rc) return rc;
  if (prof.err != hipSuccess) return hip_fail(prof.err, "qx_batch_profile: events");
  QX_HIP(hipStreamSynchronize(stream), "qx_batch_profile: chunks");
  for (int k = 0; k < QX_NPASS; ++k) passes[k] = qx_pass_stats_t{};
  for (const PassProf::Rec& r : prof.recs) {
    float ms = 0.f;
    QX_HIP(hipEventElapsedTime(&ms, r.e0, r.e1), "qx_batch_profile: elapsed");
    qx_pass_stats_t& q = passes[r.kind];
    q.launches += 1;
    q.ms += ms;
    if (r.nrun > 0) {
      q.active_launches += 1;
      q.active_ms += ms;
      q.source_launches += r.nrun;
    }
  }
  QX_HIP(hipMemcpyAsync(B->h_st, B->cfg.d_st, sizeof(SrcState) * n, hipMemcpyDeviceToHost, stream),
         "qx_batch_profile: state readback");
  QX_HIP(hipStreamSynchronize(stream), "qx_batch_profile: state readback");
  if (stats)
    for (int k = 0; k < n; ++k) {
      const SrcState& q = B->h_st[k];
      stats[k].status = q.status;
      stats[k].iters = q.iters;
      stats[k].reliable_updates = q.updates;
      stats[k].true_rel_residual = q.relres;
      stats[k].seconds = 0.0;
    }
  return QX_OK;
}

extern "C" int qx_batch_tune(qx_batch_t* batch, int nchunks, int* nbt, int* lps, int* order,
                             hipStream_t stream) {
  if (!batch || nchunks < 1 || nchunks > 64)
    return fail(QX_EINVAL, "qx_batch_tune: bad argument");
  qx_batch* B = batch;
  if (B->persistent) return fail(QX_EINVAL, "qx_batch_tune: the persistent engine is not tuned");
  int nb = 1;
  for (const auto& sp : B->specs) nb = std::max(nb, sp.nrhs);
  const size_t csz = cplx_bytes(lo_prec(&B->params));
  // batches the fused sequences can serve split the hops of a site over two
  // wavefronts or more under every engine (the plan's rule, which keeps the
  // engines' bits equal): no one-wavefront shapes there
  int max_nblk = 0;
  for (const auto& d : B->sys) max_nblk = std::max(max_nblk, d.nblk);
  const bool split = max_nblk <= kFuseMaxBlocks;
  // six or twelve sources per thread only on the launch-per-pass FP32 one-hop path
  const bool wide =
      wide_compiled(B->cfg.prec_lo, B->cfg.recon_lo) && !B->cfg.links16 && !B->cfg.fused;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  QX_HIP(hipEventCreate(&e0), "qx_batch_tune: event");
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return fail(QX_EHIP, "qx_batch_tune: event");
  }
  // time one untimed and then `nchunks` timed chunks of the solve under each
  // candidate shape (the caller's x is not written: only the finish unpacks)
  B->deo_forced = false;
  auto time_shape = [&](const LaunchShape& sh, float* ms) -> int {
    B->forced = true;
    B->forced_shape = sh;
    int rc = replan(B, stream);
    if (rc) return rc;
    rc = enqueue_start(B, stream);
    if (!rc) rc = enqueue_one_chunk(B, stream);
    if (!rc) rc = enqueue_start(B, stream);
    if (rc) return rc;
    QX_HIP(hipEventRecord(e0, stream), "qx_batch_tune: event");
    for (int c = 0; c < nchunks && !rc; ++c) rc = enqueue_one_chunk(B, stream);
    if (rc) return rc;
    QX_HIP(hipEventRecord(e1, stream), "qx_batch_tune: event");
    QX_HIP(hipEventSynchronize(e1), "qx_batch_tune: chunk");
    QX_HIP(hipEventElapsedTime(ms, e0, e1), "qx_batch_tune: elapsed");
    return QX_OK;
  };
  LaunchShape best{};
  float best_ms = 1e30f;
  int rc = QX_OK;
  for (int nb_t : {1, 2, 4, 6, 12})
    for (int l : {1, 2, 4, 8})
      for (int x = 0; x <= kMaxOrder && rc != QX_EHIP; ++x) {
        const LaunchShape sh{nb_t, l, x};
        if (!nbt_lps_instantiated(nb_t, l, wide) || !shape_ok(sh, nb, csz)) continue;
        if ((nb_t > 1 && nb_t > nb) || (split && l == 1)) continue;
        float ms = 0.f;
        rc = time_shape(sh, &ms);
        if (rc == QX_OK && ms < best_ms) {
          best_ms = ms;
          best = sh;
        }
      }
  // The launch-per-pass engine's D_eo pass: other (sources per thread,
  // wavefronts per site) under the best shape for the rest, kept when the
  // chunks get faster, then the other passes' shape again beside the D_eo
  // shape found (32^4 with twelve sources, FP32: D_eo 216 us under (4, 1)
  // beside D_oe 191 us under (6, 2)).
  LaunchShape best_deo = best;
  if (rc == QX_OK && best_ms < 1e30f && !B->cfg.fused && !B->persistent) {
    for (int nb_t : {1, 2, 4, 6, 12})
      for (int l : {1, 2, 4, 8}) {
        if (rc == QX_EHIP) break;
        const LaunchShape dsh{nb_t, l, best.xcd};
        if (nb_t == best.nbt && l == best.lps) continue;
        if (!nbt_lps_instantiated(nb_t, l, wide) || !shape_ok(dsh, nb, csz)) continue;
        if ((nb_t > 1 && nb_t > nb) || (split && l == 1)) continue;
        B->deo_forced = true;
        B->deo_shape = dsh;
        float ms = 0.f;
        rc = time_shape(best, &ms);
        if (rc == QX_OK && ms < best_ms) {
          best_ms = ms;
          best_deo = dsh;
        }
      }
    // the other stencils again, beside the D_eo shape found (the two passes'
    // times add up nearly independently)
    if (rc == QX_OK) {
      B->deo_forced = true;
      B->deo_shape = best_deo;
      const LaunchShape first = best;
      for (int nb_t : {1, 2, 4, 6, 12})
        for (int l : {1, 2, 4, 8})
          for (int x = 0; x <= kMaxOrder && rc != QX_EHIP; ++x) {
            const LaunchShape sh{nb_t, l, x};
            if (sh.nbt == first.nbt && sh.lps == first.lps && sh.xcd == first.xcd) continue;
            if (!nbt_lps_instantiated(nb_t, l, wide) || !shape_ok(sh, nb, csz)) continue;
            if ((nb_t > 1 && nb_t > nb) || (split && l == 1)) continue;
            float ms = 0.f;
            rc = time_shape(sh, &ms);
            if (rc == QX_OK && ms < best_ms) {
              best_ms = ms;
              best = sh;
            }
          }
      best_deo.xcd = best.xcd;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc == QX_EHIP) {
    B->forced = false;
    B->deo_forced = false;
    return rc;
  }
  if (best_ms >= 1e30f) {
    B->forced = false;
    B->deo_forced = false;
    replan(B, stream);
    return fail(QX_EINVAL, "qx_batch_tune: no launch shape could be timed");
  }
  B->forced = true;
  B->forced_shape = best;
  B->deo_forced = best_deo.nbt != best.nbt || best_deo.lps != best.lps;
  B->deo_shape = best_deo;
  rc = replan(B, stream);
  if (rc) return rc;
  if (nbt) *nbt = best.nbt;
  if (lps) *lps = best.lps;
  if (order) *order = best.xcd;
  return QX_OK;
}

extern "C" int qx_batch_solve(qx_batch_t* batch, qx_cg_stats_t* stats, hipStream_t stream) {
  if (!batch) return fail(QX_EINVAL, "qx_batch_solve: NULL batch");
  return run_plan(batch, stats, stream);
}

extern "C" int qx_batch_solve_async(qx_batch_t* batch, int nchunks, qx_cg_stats_t* d_stats,
                                    hipStream_t stream) {
  if (!batch || !d_stats || nchunks < 1)
    return fail(QX_EINVAL, "qx_batch_solve_async: bad argument");
  qx_batch* B = batch;
  int rc = enqueue_start(B, stream);
  for (int c = 0; rc == QX_OK && c < nchunks; ++c) rc = enqueue_one_chunk(B, stream);
  if (rc == QX_OK) rc = enqueue_finish(B, stream);
  if (rc != QX_OK) return rc;
  QX_HIP(launch_batch_stats(B->cfg.d_st, B->cfg.nsrc_total,
                            B->persistent ? (const void*)(B->ws + B->layout.gs_off) : nullptr,
                            d_stats, stream),
         "qx_batch_solve_async: statistics");
  return QX_OK;
}

extern "C" int qx_batch_info(const qx_batch_t* batch, int* nsources, int* chunk) {
  if (!batch) return fail(QX_EINVAL, "qx_batch_info: NULL batch");
  if (nsources) *nsources = batch->cfg.nsrc_total;
  if (chunk) *chunk = batch->chunk;
  return QX_OK;
}

extern "C" int qx_batch_destroy(qx_batch_t* batch) {
  delete batch;
  return QX_OK;
}

// ------------------------------------------------------------------- force

extern "C" int qx_force_from_fields(const qx_gauge_t* g64, int nrhs, const void* x_packed,
                                    const void* lam_packed, void* tmp_odd, void* grad_U,
                                    hipStream_t stream) {
  if (!g64 || nrhs < 1 || !x_packed || !lam_packed || !tmp_odd || !grad_U)
    return fail(QX_EINVAL, "qx_force_from_fields: bad argument");
  if (g64->prec != QX_PREC_F64) return fail(QX_EINVAL, "qx_force_from_fields: needs FP64 links");
  if (g64->recon == QX_RECON_NAIK)
    return fail(QX_EINVAL, "qx_force_from_fields: the force is implemented for the one-hop operator");
  const Geo& g = g64->geo;
  char* y = (char*)tmp_odd;
  char* nu = y + field_bytes(g, nrhs, QX_PREC_F64);
  const LaunchShape sh = shape_for(g64, nrhs);
  QX_HIP(launch_dslash(g, QX_PREC_F64, g64->recon, g64->packed, 1, x_packed, y, nrhs, 0.5, sh,
                       stream),
         "qx_force_from_fields: D_oe x");
  const void* nup = y;
  if (lam_packed != x_packed) {
    QX_HIP(launch_dslash(g, QX_PREC_F64, g64->recon, g64->packed, 1, lam_packed, nu, nrhs, 0.5,
                         sh, stream),
           "qx_force_from_fields: D_oe lam");
    nup = nu;
  }
  QX_HIP(launch_force(g, nrhs, x_packed, lam_packed, y, nup, grad_U, stream),
         "qx_force_from_fields: outer products");
  return QX_OK;
}

namespace {
size_t force_extra_bytes(const Geo& g, int nrhs) {
  return align_up(field_bytes(g, nrhs, QX_PREC_F64), 256) + 256 * sizeof(double) + 256;
}
}  // namespace

extern "C" int qx_force_workspace_bytes(const qx_lattice_t* lat, const qx_cg_params_t* params,
                                        int nrhs, size_t* bytes) {
  if (nrhs > kMaxSrcPerSys) return fail(QX_EINVAL, "qx_force: at most %d sources", kMaxSrcPerSys);
  size_t b = 0;
  int rc = qx_cg_workspace_bytes(lat, params, nrhs, &b);
  if (rc) return rc;
  *bytes = align_up(b, 256) + force_extra_bytes(lat->geo, nrhs);
  return QX_OK;
}

extern "C" int qx_force(const qx_gauge_t* g64, const qx_gauge_t* glo, const qx_cg_params_t* params,
                        int nrhs, double mass, const void* phi, void* grad_U, double* S_out,
                        void* x_out, void* ws, size_t ws_bytes, qx_cg_stats_t* stats,
                        hipStream_t stream) {
  int rc = check_params(params);
  if (rc) return rc;
  rc = check_system(g64, glo, params);
  if (rc) return rc;
  if (g64->recon == QX_RECON_NAIK)
    return fail(QX_EINVAL, "qx_force: the force is implemented for the one-hop operator");
  if (nrhs < 1 || nrhs > kMaxSrcPerSys || !phi || !grad_U || !ws)
    return fail(QX_EINVAL, "qx_force: bad argument");
  const Geo& g = g64->geo;
  qx_batch B;
  B.params = *params;
  B.params.use_x0 = 0;
  std::vector<double> masses(nrhs, mass);
  // the solution goes to x_out when given, else it stays packed in the workspace
  void* xdst = x_out;
  std::vector<SysSpec> probe;
  add_specs(probe, g64, glo, params, nrhs, masses.data(), phi, x_out);
  const size_t solver_bytes = align_up(plan_layout(probe, lo_prec(params), params->engine).total, 256);
  if (ws_bytes < solver_bytes + force_extra_bytes(g, nrhs))
    return fail(QX_ENOMEM, "qx_force: workspace too small");
  char* extra = (char*)ws + solver_bytes;
  char* y = extra;
  double* partials = (double*)(extra + align_up(field_bytes(g, nrhs, QX_PREC_F64), 256));
  double* d_S = partials + 255;
  if (!xdst) xdst = y;  // scratch for the canonical x (same size as one packed odd field)
  add_specs(B.specs, g64, glo, params, nrhs, masses.data(), phi, xdst);
  rc = build_plan(&B, ws, solver_bytes);
  if (!rc) rc = upload_plan(&B, stream);
  if (!rc) rc = run_plan(&B, stats, stream);
  if (rc && rc != QX_ENOTCONVERGED) return rc;
  const int solve_rc = rc;
  const SysDesc& d = B.sys[0];
  const size_t vs = field_bytes(g, nrhs, QX_PREC_F64);
  const char* xhi = (const char*)d.vhi;
  const char* bhi = xhi + 2 * vs;
  // S = sum_s Re <phi_s, x_s> from the packed FP64 b and x
  QX_HIP(launch_redot(bhi, xhi, (size_t)nrhs * 3 * g.hv, partials, 255, d_S, stream),
         "qx_force: action");
  double S = 0.0;
  QX_HIP(hipMemcpyAsync(&S, d_S, sizeof S, hipMemcpyDeviceToHost, stream), "qx_force: action copy");
  // y = D_oe x in the (now free) odd slot of the FP64 vectors, then the outer products
  char* yodd = (char*)d.vhi + 3 * vs;
  const LaunchShape sh = shape_for(g64, nrhs);
  QX_HIP(launch_dslash(g, QX_PREC_F64, g64->recon, g64->packed, 1, xhi, yodd, nrhs, 0.5, sh, stream),
         "qx_force: D_oe x");
  QX_HIP(launch_force(g, nrhs, xhi, xhi, yodd, yodd, grad_U, stream), "qx_force: outer products");
  QX_HIP(hipStreamSynchronize(stream), "qx_force");
  if (S_out) *S_out = S;
  return solve_rc;
}

extern "C" int qx_action_backward(const qx_lattice_t* lat, int nrhs, double gS, const void* grad_U_S,
                                  const void* x, void* grad_U, void* grad_phi, hipStream_t stream) {
  if (!lat || nrhs < 1 || (grad_U && !grad_U_S) || (grad_phi && !x))
    return fail(QX_EINVAL, "qx_action_backward: bad argument");
  const Geo& g = lat->geo;
  if (grad_U)
    QX_HIP(launch_scale_c128(grad_U_S, gS, (size_t)4 * 2 * g.hv * 9, grad_U, stream),
           "qx_action_backward: link gradient");
  if (grad_phi)
    QX_HIP(launch_scale_c128(x, 2.0 * gS, (size_t)nrhs * g.hv * 3, grad_phi, stream),
           "qx_action_backward: source gradient");
  return QX_OK;
}

extern "C" int qx_force_su3(const qx_lattice_t* lat, const void* U_canon, const void* grad_U,
                            double* F, hipStream_t stream) {
  if (!lat || !U_canon || !grad_U || !F) return fail(QX_EINVAL, "qx_force_su3: bad argument");
  QX_HIP(launch_su3_force(lat->geo, U_canon, grad_U, F, stream), "qx_force_su3");
  return QX_OK;
}

// ------------------------------------------------------------------- probe

extern "C" int qx_probe_copy(void* dst, const void* src, size_t bytes, hipStream_t stream) {
  if (!dst || !src || bytes % 16) return fail(QX_EINVAL, "qx_probe_copy: bad argument");
  QX_HIP(launch_copy(dst, src, bytes, stream), "qx_probe_copy");
  return QX_OK;
}

extern "C" int qx_probe_read(const void* src, size_t bytes, void* scratch, hipStream_t stream) {
  if (!src || !scratch || bytes % 16) return fail(QX_EINVAL, "qx_probe_read: bad argument");
  QX_HIP(launch_read(src, bytes, (unsigned*)scratch, stream), "qx_probe_read");
  return QX_OK;
}

// ------------------------------------------------------------------ tuning

extern "C" int qx_get_launch(const qx_gauge_t* g, int nrhs, int* nbt, int* lps, int* xcd_order) {
  if (!g || nrhs < 1 || !nbt || !lps || !xcd_order)
    return fail(QX_EINVAL, "qx_get_launch: bad argument");
  const LaunchShape s = shape_for(g, nrhs);
  *nbt = s.nbt;
  *lps = s.lps;
  *xcd_order = s.xcd;
  return QX_OK;
}

extern "C" int qx_set_launch(const qx_gauge_t* g, int nrhs, int nbt, int lps, int xcd_order) {
  if (!g || nrhs < 1 || !nbt_lps_instantiated(nbt, lps, wide_compiled(g->prec, g->recon)))
    return fail(QX_EINVAL, "qx_set_launch: unsupported shape (nbt %d, lps %d)", nbt, lps);
  const LaunchShape sh{nbt, lps, xcd_order};
  // the standalone operators split the sources into passes that fit a block;
  // a solver whose sources do not fit falls back to the default shape
  if (!shape_ok(sh, 1, cplx_bytes(g->prec)))
    return fail(QX_EINVAL, "qx_set_launch: shape does not fit one block");
  const_cast<qx_gauge*>(g)->shapes[nrhs] = sh;
  return QX_OK;
}

// ------------------------------------------------------- molecular dynamics

namespace {
constexpr int kMdBlocks = 1024;  // partial sums of the action and kinetic-energy reductions
size_t md_reduce_bytes() { return align_up(sizeof(double) * (kMdBlocks + 1), 256); }

int md_sum(double* ws, double* out_host, hipStream_t s) {
  QX_HIP(hipMemcpyAsync(out_host, ws + kMdBlocks, sizeof(double), hipMemcpyDeviceToHost, s),
         "md: readback");
  QX_HIP(hipStreamSynchronize(s), "md: synchronise");
  return QX_OK;
}
}  // namespace

extern "C" int qx_gauge_action(const qx_lattice_t* lat, const void* U, double beta, void* ws,
                               size_t ws_bytes, double* S, hipStream_t stream) {
  if (!lat || !U || !ws || !S || ws_bytes < md_reduce_bytes())
    return fail(QX_EINVAL, "qx_gauge_action: bad argument");
  double* part = (double*)ws;
  QX_HIP(launch_plaquette_sum(lat->geo, U, part, kMdBlocks, part + kMdBlocks, stream),
         "qx_gauge_action");
  double sum = 0.0;
  int rc = md_sum(part, &sum, stream);
  if (rc) return rc;
  *S = beta * sum;
  return QX_OK;
}

extern "C" int qx_gauge_force(const qx_lattice_t* lat, const void* U, double beta, void* G,
                              int accumulate, hipStream_t stream) {
  if (!lat || !U || !G) return fail(QX_EINVAL, "qx_gauge_force: bad argument");
  QX_HIP(launch_gauge_grad(lat->geo, U, beta, G, accumulate ? 1 : 0, stream), "qx_gauge_force");
  return QX_OK;
}

extern "C" int qx_md_update_momenta(const qx_lattice_t* lat, const void* U, const void* G,
                                    double eps, double* p, hipStream_t stream) {
  if (!lat || !U || !G || !p) return fail(QX_EINVAL, "qx_md_update_momenta: bad argument");
  QX_HIP(launch_mom_update(lat->geo, U, G, eps, p, stream), "qx_md_update_momenta");
  return QX_OK;
}

extern "C" int qx_md_update_links(const qx_lattice_t* lat, const double* p, double eps, void* U,
                                  hipStream_t stream) {
  if (!lat || !U || !p) return fail(QX_EINVAL, "qx_md_update_links: bad argument");
  QX_HIP(launch_link_update(lat->geo, p, eps, U, stream), "qx_md_update_links");
  return QX_OK;
}

extern "C" int qx_md_kinetic(const qx_lattice_t* lat, const double* p, void* ws, size_t ws_bytes,
                             double* K, hipStream_t stream) {
  if (!lat || !p || !ws || !K || ws_bytes < md_reduce_bytes())
    return fail(QX_EINVAL, "qx_md_kinetic: bad argument");
  double* part = (double*)ws;
  QX_HIP(launch_sumsq(p, 64 * (int64_t)lat->geo.hv, part, kMdBlocks, part + kMdBlocks, stream),
         "qx_md_kinetic");
  double sum = 0.0;
  int rc = md_sum(part, &sum, stream);
  if (rc) return rc;
  *K = 0.5 * sum;
  return QX_OK;
}

extern "C" int qx_md_workspace_bytes(const qx_lattice_t* lat, const qx_md_params_t* p,
                                     size_t* bytes) {
  if (!lat || !p || !bytes) return fail(QX_EINVAL, "qx_md_workspace_bytes: bad argument");
  size_t f = 0;
  int rc = qx_force_workspace_bytes(lat, &p->cg, 1, &f);
  if (rc) return rc;
  *bytes = md_reduce_bytes() + align_up((size_t)lat->V * 4 * 9 * 16, 256) + f;
  return QX_OK;
}

extern "C" int qx_md_trajectory(qx_gauge_t* g64, qx_gauge_t* glo, const qx_md_params_t* p,
                                void* U, double* mom, const void* phi, void* ws, size_t ws_bytes,
                                double* H_start, double* H_end, int* cg_iters,
                                hipStream_t stream) {
  if (!g64 || !p || !U || !mom || !ws || !H_start || !H_end || p->nsteps < 1)
    return fail(QX_EINVAL, "qx_md_trajectory: bad argument");
  if (g64->prec != QX_PREC_F64) return fail(QX_EINVAL, "qx_md_trajectory: g64 must be FP64");
  if (g64->recon == QX_RECON_NAIK || (glo && glo->recon == QX_RECON_NAIK))
    return fail(QX_EINVAL, "qx_md_trajectory: the force is implemented for the one-hop operator");
  if (glo && !same_lattice(g64, glo))
    return fail(QX_EINVAL, "qx_md_trajectory: g64 and glo are on different lattices");
  qx_lattice lat{};
  memcpy(lat.dims, g64->dims, sizeof lat.dims);
  lat.flags = g64->flags;
  lat.geo = g64->geo;
  lat.V = 2 * (int64_t)g64->geo.hv;
  size_t need = 0;
  int rc = qx_md_workspace_bytes(&lat, p, &need);
  if (rc) return rc;
  if (ws_bytes < need) return fail(QX_ENOMEM, "qx_md_trajectory: workspace of %zu bytes, %zu needed",
                                   ws_bytes, need);
  char* w = (char*)ws;
  double* red = (double*)w;
  void* grad = w + md_reduce_bytes();
  void* fws = w + md_reduce_bytes() + align_up((size_t)lat.V * 4 * 9 * 16, 256);
  const size_t fws_bytes = need - (md_reduce_bytes() + align_up((size_t)lat.V * 4 * 9 * 16, 256));
  int iters = 0;
  // gradient of S_g + S_f at the current links into grad; S_f to *Sf
  auto force = [&](double* Sf) -> int {
    *Sf = 0.0;
    if (phi) {
      qx_cg_stats_t st{};
      int r = qx_force(g64, glo, &p->cg, 1, p->mass, phi, grad, Sf, nullptr, fws, fws_bytes, &st,
                       stream);
      iters += st.iters;
      if (r) return r;
    }
    QX_HIP(launch_gauge_grad(lat.geo, U, p->beta, grad, phi ? 1 : 0, stream), "md: gauge force");
    return QX_OK;
  };
  auto energy = [&](double Sf, double* H) -> int {
    double K = 0.0, Sg = 0.0;
    int r = qx_md_kinetic(&lat, mom, red, md_reduce_bytes(), &K, stream);
    if (!r) r = qx_gauge_action(&lat, U, p->beta, red, md_reduce_bytes(), &Sg, stream);
    *H = K + Sg + Sf;
    return r;
  };
  auto repack = [&]() -> int {
    QX_HIP(launch_pack_gauge(g64->geo, U, g64->prec, g64->recon, const_cast<void*>(g64->packed), nullptr, stream),
           "md: repack FP64 links");
    if (glo)
      QX_HIP(launch_pack_gauge(glo->geo, U, glo->prec, glo->recon, const_cast<void*>(glo->packed), nullptr, stream),
             "md: repack inner links");
    return QX_OK;
  };
  double Sf = 0.0;
  rc = repack();
  if (!rc) rc = force(&Sf);
  if (!rc) rc = energy(Sf, H_start);
  if (rc) return rc;
  QX_HIP(launch_mom_update(lat.geo, U, grad, 0.5 * p->eps, mom, stream), "md: momenta");
  for (int i = 0; i < p->nsteps; ++i) {
    QX_HIP(launch_link_update(lat.geo, mom, p->eps, U, stream), "md: links");
    rc = repack();
    if (!rc) rc = force(&Sf);
    if (rc) return rc;
    const double e = i + 1 < p->nsteps ? p->eps : 0.5 * p->eps;
    QX_HIP(launch_mom_update(lat.geo, U, grad, e, mom, stream), "md: momenta");
  }
  rc = energy(Sf, H_end);
  if (rc) return rc;
  if (cg_iters) *cg_iters = iters;
  return QX_OK;
}

// ------------------------------------------------------------------ mesons

namespace {
size_t meson_extra_bytes(const Geo& g) {
  // b and x canonical, x and y packed (three sources each), C
  return 4 * align_up(field_bytes(g, 3, QX_PREC_F64), 256) +
         align_up(sizeof(double) * 16 * (size_t)g.L3, 256);
}
}  // namespace

extern "C" int qx_meson_workspace_bytes(const qx_lattice_t* lat, const qx_cg_params_t* params,
                                        size_t* bytes) {
  if (!lat || !params || !bytes) return fail(QX_EINVAL, "qx_meson_workspace_bytes: bad argument");
  size_t b = 0;
  int rc = qx_cg_workspace_bytes(lat, params, 3, &b);
  if (rc) return rc;
  *bytes = align_up(b, 256) + meson_extra_bytes(lat->geo);
  return QX_OK;
}

extern "C" int qx_meson_correlators(const qx_gauge_t* g64, const qx_gauge_t* glo,
                                    const qx_cg_params_t* params, double mass, const int src[4],
                                    int nmask, const int* masks, double* C, void* ws,
                                    size_t ws_bytes, qx_cg_stats_t* stats, hipStream_t stream) {
  if (!g64 || !params || !src || !masks || !C || !ws || nmask < 1 || nmask > 16)
    return fail(QX_EINVAL, "qx_meson_correlators: bad argument");
  const Geo& g = g64->geo;
  const int L[4] = {g.L0, g.L1, g.L2, g.L3};
  for (int mu = 0; mu < 4; ++mu)
    if (src[mu] < 0 || src[mu] >= L[mu])
      return fail(QX_EINVAL, "qx_meson_correlators: source outside the lattice");
  if ((src[0] + src[1] + src[2] + src[3]) & 1)
    return fail(QX_EINVAL, "qx_meson_correlators: the source must be on an even site");
  for (int k = 0; k < nmask; ++k)
    if (masks[k] < 0 || masks[k] > 15) return fail(QX_EINVAL, "qx_meson_correlators: bad mask");
  qx_lattice lat{};
  memcpy(lat.dims, g64->dims, sizeof lat.dims);
  lat.flags = g64->flags;
  lat.geo = g;
  lat.V = 2 * (int64_t)g.hv;
  size_t need = 0;
  int rc = qx_meson_workspace_bytes(&lat, params, &need);
  if (rc) return rc;
  if (ws_bytes < need)
    return fail(QX_ENOMEM, "qx_meson_correlators: workspace of %zu bytes, %zu needed", ws_bytes, need);
  size_t solver = 0;
  rc = qx_cg_workspace_bytes(&lat, params, 3, &solver);
  if (rc) return rc;
  char* w = (char*)ws;
  const size_t fb = align_up(field_bytes(g, 3, QX_PREC_F64), 256);
  char* sws = w;
  char* b = w + align_up(solver, 256);
  char* x = b + fb;
  char* xp = x + fb;
  char* yp = xp + fb;
  double* Cd = (double*)(yp + fb);
  const int64_t lex = src[0] + (int64_t)L[0] * (src[1] + (int64_t)L[1] * (src[2] + (int64_t)L[2] * src[3]));
  QX_HIP(launch_point_source(g, (int)(lex >> 1), b, stream), "qx_meson_correlators: sources");
  const double ms[3] = {mass, mass, mass};
  rc = qx_cg_solve(g64, glo, params, 3, ms, b, x, sws, solver, stats, stream);
  if (rc) return rc;
  QX_HIP(launch_pack_field(g, 3, QX_PREC_F64, x, xp, stream), "qx_meson_correlators: pack");
  QX_HIP(launch_dslash(g, QX_PREC_F64, g64->recon, g64->packed, 1, xp, yp, 3, 0.5,
                       shape_for(g64, 3), stream),
         "qx_meson_correlators: D_oe");
  QX_HIP(launch_meson_contract(g, xp, yp, mass, src[3], nmask, masks, Cd, stream),
         "qx_meson_correlators: contraction");
  QX_HIP(hipMemcpyAsync(C, Cd, sizeof(double) * nmask * (size_t)g.L3, hipMemcpyDeviceToHost,
                        stream),
         "qx_meson_correlators: readback");
  QX_HIP(hipStreamSynchronize(stream), "qx_meson_correlators: synchronise");
  return QX_OK;
}

namespace {

// Average device time (ms) of one of `reps` back-to-back launches made by
// enqueue(stream, r).  The launches are captured into a HIP graph on a private
// stream, which first waits for the caller's stream, and the graph is replayed
// once untimed and once between two HIP events on that stream: the host's
// launch rate does not enter the figure, only each kernel and the dispatch gap
// between dependent kernels, as inside a solver graph.
template <typename F>
int time_launches(const char* what, hipStream_t caller, int reps, F&& enqueue, float* ms_out) {
  hipStream_t ps = nullptr;
  hipEvent_t dep = nullptr, e0 = nullptr, e1 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&ps, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&dep);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(dep, caller);
  if (e == hipSuccess) e = hipStreamWaitEvent(ps, dep, 0);
  if (e == hipSuccess) e = hipStreamBeginCapture(ps, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t el = hipSuccess;
    for (int r = 0; r < reps && el == hipSuccess; ++r) el = enqueue(ps, r);
    e = hipStreamEndCapture(ps, &graph);
    if (e == hipSuccess) e = el;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e == hipSuccess) e = hipGraphLaunch(exec, ps);
  if (e == hipSuccess) e = hipEventRecord(e0, ps);
  if (e == hipSuccess) e = hipGraphLaunch(exec, ps);
  if (e == hipSuccess) e = hipEventRecord(e1, ps);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (ps) hipStreamSynchronize(ps);
  if (exec) hipGraphExecDestroy(exec);
  if (graph) hipGraphDestroy(graph);
  if (e1) hipEventDestroy(e1);
  if (e0) hipEventDestroy(e0);
  if (dep) hipEventDestroy(dep);
  if (ps) hipStreamDestroy(ps);
  if (e != hipSuccess) return hip_fail(e, what);
  *ms_out = ms / reps;
  return QX_OK;
}

}  // namespace

extern "C" int qx_tune_cache_load(const char* path) {
  if (!path || !*path) return fail(QX_EINVAL, "qx_tune_cache_load: no path");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  if (!tune_read_file_locked(path)) return fail(QX_EINVAL, "qx_tune_cache_load: cannot read %s", path);
  return QX_OK;
}

extern "C" int qx_tune_cache_save(const char* path) {
  if (!path || !*path) return fail(QX_EINVAL, "qx_tune_cache_save: no path");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  if (!tune_write_file_locked(path)) return fail(QX_EINVAL, "qx_tune_cache_save: cannot write %s", path);
  return QX_OK;
}

extern "C" int qx_tune_dslash(const qx_gauge_t* g, int nrhs, void* scratch, hipStream_t stream) {
  if (!g || nrhs < 1 || !scratch) return fail(QX_EINVAL, "qx_tune_dslash: bad argument");
  const Geo& geo = g->geo;
  const size_t fb = field_bytes(geo, nrhs, g->prec);
  char* in = (char*)scratch;
  char* out = in + fb;
  QX_HIP(hipMemsetAsync(in, 0, fb, stream), "qx_tune_dslash: clear");
  LaunchShape best{};
  float best_ms = 1e30f;
  const int nbts[5] = {1, 2, 4, 6, 12}, lpss[4] = {1, 2, 4, 8};
  const size_t csz = cplx_bytes(g->prec);
  for (int nbt : nbts) {
    if (nbt > 1 && nbt > nrhs) continue;
    for (int lps : lpss) {
      for (int x = 0; x <= kMaxOrder; ++x) {
        const LaunchShape sh{nbt, lps, x};
        if (!nbt_lps_instantiated(nbt, lps, wide_compiled(g->prec, g->recon)) ||
            !shape_ok(sh, nrhs, csz))
          continue;
        float ms = 0.f;
        const int rc = time_launches("qx_tune_dslash: timing", stream, 20,
                                     [&](hipStream_t s, int r) {
                                       return launch_dslash(geo, g->prec, g->recon, g->packed,
                                                            r & 1, in, out, nrhs, 0.5, sh, s);
                                     },
                                     &ms);
        if (rc) return rc;
        if (ms < best_ms) {
          best_ms = ms;
          best = sh;
        }
      }
    }
  }
  const_cast<qx_gauge*>(g)->shapes[nrhs] = best;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  g_tune[tune_key(g, nrhs)] = best;
  tune_save_locked();
  return QX_OK;
}

extern "C" int qx_time_dslash(const qx_gauge_t* g, int out_parity, int nrhs, const void* in,
                              void* out, int reps, double* avg_ms, hipStream_t stream) {
  if (!g || !in || !out || !avg_ms || nrhs < 1 || reps < 1 || reps > 10000 ||
      (out_parity != 0 && out_parity != 1))
    return fail(QX_EINVAL, "qx_time_dslash: bad argument");
  if (in == out) return fail(QX_EINVAL, "qx_time_dslash: in and out must not alias");
  const LaunchShape sh = shape_for(g, nrhs);
  float ms = 0.f;
  const int rc = time_launches("qx_time_dslash", stream, reps,
                               [&](hipStream_t s, int) {
                                 return launch_dslash(g->geo, g->prec, g->recon, g->packed,
                                                      out_parity, in, out, nrhs, 0.5, sh, s);
                               },
                               &ms);
  if (rc) return rc;
  *avg_ms = ms;
  return QX_OK;
}
