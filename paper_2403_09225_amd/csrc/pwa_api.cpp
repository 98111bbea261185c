// Host side of the PWA likelihood library: argument validation, workspace
// layout, stream-ordered launches and the Newton-CG fit driver.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "pwa_analysis.h"
#include "pwa_batched.h"
#include "pwa_internal.h"

using namespace pwa;

struct pwa_ctx {
  pwa_model model;
  int32_t streams = 0;
  int32_t precision = PWA_PREC_F64;
  int K = 0, P = 0;
  ModelDev md;
  FieldSpec fs;
  int shape_L = 0, shape_T = 0, shape_R = 0;  // layout 0 = automatic
  // bound state
  bool bound = false;
  int64_t n_data = 0, n_mc = 0, stride = 0;
  int64_t mc_off = 0;   // first MC event of the stream: n_data rounded up to 64
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int* status = nullptr;
  double* tbl64 = nullptr;
  float* tbl32 = nullptr;
  int* itbl = nullptr;
  double* part = nullptr;
  double* tot = nullptr;
  double* dd = nullptr;
  double* scratch = nullptr;
  // Direction-independent totals of the last full HVP pass (in `tot`) and
  // its theta (a copy in scratch) may serve further HVPs at that theta.
  bool hvp_cache = false;
  int cache_prec = 0;
  double* planes64 = nullptr;
  float* planes32 = nullptr;
  int cu_count = 0;
  struct GridEntry {
    int prec, mode, L, T, R, blocks;
  };
  std::vector<GridEntry> grid_cache;  // resident-grid size per kernel variant
  // batched (frozen-lineshape) path
  bool frozen = false;
  int bfmt = 0, bKP = 0, bmax = 0, brows = 0, bgram_blocks = 0;
  void* bA[kSlices] = {};             // amplitude operand planes
  void* bC[kSlices] = {};             // coupling operand planes
  unsigned long long* besum = nullptr;   // sliced format: sum of the row exponents
  double* bpart = nullptr;
  double* bpart2 = nullptr;
  double* bgram_part = nullptr;
  double* bgram_xtx = nullptr;
  double* bgram = nullptr;
  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  int ev_used = 0;
  double timed_ms = 0.0;
  int64_t timed_n = 0;
  ~pwa_ctx() {
    for (auto e : ev_start) hipEventDestroy(e);
    for (auto e : ev_stop) hipEventDestroy(e);
  }
};

namespace {

// The general physics path (Flatte resonances, spin-1 parent) is built for
// up to this many resonances (wave-group shapes G x 2, G <= 8).
constexpr int kMaxGenRes = 16;

struct Layout {
  size_t status, tbl64, tbl32, itbl, part, tot, dd, scratch, planes64, planes32, total;
  int64_t stride, mc_off;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

Layout layout_of(const pwa_ctx* c, int64_t n_data, int64_t n_mc) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const int K = c->K, P = c->P;
  L.status = take(64 * sizeof(int));
  L.tbl64 = take(sizeof(double) * KPAD * TS);
  L.tbl32 = take(sizeof(float) * KPAD * TS);
  L.itbl = take(sizeof(int) * KPAD * ITS);
  L.part = take(sizeof(double) * 2 * (size_t)MAX_BLOCKS * (1 + NMOM_HVP * (size_t)K));
  L.tot = take(sizeof(double) * 4 * (1 + NMOM_HVP * (size_t)K));
  L.dd = take(sizeof(double) * 2 * (2 + 4 * (size_t)P));
  L.scratch = take(sizeof(double) * (8 * (size_t)P + 16));
  // data events from 0, MC events from mc_off: both sets start on a
  // 64-event boundary, so a 64-event batch is one aligned chunk per plane
  L.mc_off = (int64_t)align_up((size_t)n_data, 64);
  L.stride = (int64_t)align_up((size_t)(L.mc_off + n_mc), 64);
  L.planes64 = take((c->streams & PWA_STREAM_F64) ? sizeof(double) * (size_t)c->fs.n_fields * L.stride : 0);
  L.planes32 = take((c->streams & PWA_STREAM_F32) ? sizeof(float) * (size_t)c->fs.n_fields * L.stride : 0);
  L.total = off;
  return L;
}

bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

// Automatic launch shape, for every pass (NLL, NLL + grad, H v).  Layout 2
// (a block of G waves shares each batch of 64 events, wave g owns R
// resonances, the event planes staged into LDS) keeps the resonance table
// and plane pointers in scalar registers; the choice covers K with the
// fewest padded resonance slots at R <= 3 (FP64 moment accumulators: 18 R
// per lane), and 8 waves of 3 or 4 resonances (512-thread blocks, at most 2
// waves per SIMD) for 16 < K <= 32.  A 12-wave block would hold 3 waves per
// SIMD, which caps a wave at 168 VGPRs: the FP64 H v build of 12 x 2 then
// spills and runs 4x slower than 8 x 3 (2.47 against 0.59 ms at K = 20,
// 6M events).  For the NLL alone layout 2 also beats one lane per event with
// all resonances (layout 1, T = 1): 157 against 191 us at K = 12, 222 against
// 426 us at K = 30 (6M events, FP64).  Above K = 32 the passes without the
// full H v moments take 8 waves of 8 resonances (K = 40 and 64, 6M events,
// FP64: NLL 1.37 -> 0.36 ms, NLL + grad 1.42 -> 0.63 ms, direction-only H v
// 2.27 -> 0.89 ms against layout 1); the full H v pass, whose 18 moments per
// resonance do not fit 8 of them per lane, stays in layout 1 (T lanes of a
// wave share an event, 32 x 2).
void auto_shape(int K, int mode, int& L, int& T, int& R) {
  L = 2;
  if (K <= 2) { T = 1; R = 2; return; }
  if (K <= 4) { T = 1; R = 4; return; }
  if (K <= 6) { T = 2; R = 3; return; }
  if (K <= 8) { T = 4; R = 2; return; }
  if (K <= 12) { T = 4; R = 3; return; }
  if (K <= 16) { T = 8; R = 2; return; }
  if (K <= 24) { T = 8; R = 3; return; }
  if (K <= 32) { T = 8; R = 4; return; }
  if (mode != MODE_HVP) { T = 8; R = 8; return; }
  L = 1;
  T = 32; R = 2;
}

// General physics path (layout 3): G waves of 2 resonances, or 4 waves of 3
// for 8 < K <= 12 (no padded slots and half the waves repeating the
// per-event head: at K = 12, 1M + 5M events, the FP64 H v pass with a
// Flatte resonance takes 0.55 against 0.73 ms at 8 x 2, 0.75 against 0.98 ms
// for a spin-1 parent).
void auto_gen_shape(int K, int& L, int& T, int& R) {
  L = 3;
  R = 2;
  T = K <= 2 ? 1 : (K <= 4 ? 2 : (K <= 8 ? 4 : 8));
  if (K > 8 && K <= 12) {
    T = 4;
    R = 3;
  }
}

void shape_of(const pwa_ctx* c, int mode, int& L, int& T, int& R) {
  if (c->md.gen) {
    if (c->shape_L == 3) {
      L = 3;
      T = c->shape_T;
      R = c->shape_R;
    } else {
      auto_gen_shape(c->K, L, T, R);
    }
    return;
  }
  if (c->shape_L > 0) {
    L = c->shape_L;
    T = c->shape_T;
    R = c->shape_R;
  } else {
    auto_shape(c->K, mode, L, T, R);
  }
}

int grid_blocks(pwa_ctx* c, int prec, int mode, int L, int T, int R) {
  int cached = 0;
  for (const auto& g : c->grid_cache)
    if (g.prec == prec && g.mode == mode && g.L == L && g.T == T && g.R == R) cached = g.blocks;
  if (cached == 0) {
    int occ = eval_occupancy(prec, mode, L, T, R, c->fs.n_fields);
    if (occ <= 0) occ = 1;
    cached = std::max(1, std::min(MAX_BLOCKS, c->cu_count * occ));
    c->grid_cache.push_back({prec, mode, L, T, R, cached});
  }
  const int per_iter = (L >= 2) ? 64 : BLOCK / T;   // events per block per iteration
  const int64_t n = c->n_data + c->n_mc;
  const int64_t need = std::max<int64_t>(2, (n + per_iter - 1) / per_iter);
  return (int)std::min<int64_t>(cached, need);
}

void split_blocks(const pwa_ctx* c, int mode, int nb, int& nb_data, int& nb_mc) {
  if (c->n_data == 0) {
    nb_data = 0;
    nb_mc = std::max(1, nb);
    return;
  }
  const double cost = (mode == MODE_NLL) ? 1.6 : (mode == MODE_GRAD ? 1.35 : 1.2);
  const double wd = cost * (double)c->n_data, wm = (double)c->n_mc;
  nb_data = (int)llround(nb * wd / (wd + wm));
  nb_data = std::max(1, std::min(nb - 1, nb_data));
  nb_mc = std::max(1, nb - nb_data);
}

constexpr int kEventPool = 256;

// Fold the durations of all recorded event pairs into the running total.
int fold_timing(pwa_ctx* c) {
  if (c->ev_used == 0) return PWA_OK;
  if (hipEventSynchronize(c->ev_stop[c->ev_used - 1]) != hipSuccess) return PWA_E_HIP;
  for (int i = 0; i < c->ev_used; ++i) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, c->ev_start[i], c->ev_stop[i]) != hipSuccess) return PWA_E_HIP;
    c->timed_ms += ms;
    ++c->timed_n;
  }
  c->ev_used = 0;
  return PWA_OK;
}

static double* cache_theta_slot(pwa_ctx* c) { return c->scratch + 7 * c->P; }

// One evaluation: table, pass, reduction and finaliser.  With mc_only the
// grid covers the MC events alone (the data sums come out as zero).
// MODE_HVPB (an HVP at the theta of the last full HVP pass, which d_theta
// must equal) runs as a full HVP pass when no such totals are cached for
// this precision.
int run_eval(pwa_ctx* c, int mode, int out_kind, int prec, const double* d_theta,
             const double* d_v, double* d_nll, double* d_grad, double* d_hv, double* d_dd,
             hipStream_t st, bool mc_only = false) {
  int L = 2, T = 1, R = 1;
  if (mode == MODE_HVPB && !(c->hvp_cache && c->cache_prec == prec && !mc_only))
    mode = MODE_HVP;
  const bool reuse = (mode == MODE_HVPB);
  c->hvp_cache = false;   // every pass rewrites the totals; set again below
  shape_of(c, mode, L, T, R);
  const int kslots = T * R;
  hipError_t e = launch_table(d_theta, d_v, c->md, kslots, c->tbl64, c->tbl32, c->itbl, c->status, st);
  if (e != hipSuccess) return PWA_E_HIP;
  const int nb = grid_blocks(c, prec, mode, L, T, R);
  EvalArgs a;
  a.planes = prec == PWA_PREC_F32 ? (const void*)c->planes32 : (const void*)c->planes64;
  a.stride = c->stride;
  a.n_fields = c->fs.n_fields;
  a.mc_base = c->mc_off;
  a.gen = c->md.gen;
  a.nmu = c->md.parent_spin == 1 ? 2 : 1;
  a.tbl64 = c->tbl64;
  a.tbl32 = c->tbl32;
  a.itbl = c->itbl;
  a.n_data = c->n_data;
  a.n_mc = c->n_mc;
  split_blocks(c, mode, nb, a.nb_data, a.nb_mc);
  if (mc_only) {
    a.nb_data = 0;
    a.nb_mc = nb;
  }
  a.K = c->K;
  a.part = c->part;
  const bool timed = c->timing;
  if (timed) {
    if (c->ev_used == kEventPool && fold_timing(c) != PWA_OK) return PWA_E_HIP;
    if (hipEventRecord(c->ev_start[c->ev_used], st) != hipSuccess) return PWA_E_HIP;
  }
  e = launch_eval(prec, mode, L, T, R, a, a.nb_data + a.nb_mc, st);
  if (e != hipSuccess) return PWA_E_HIP;
  if (timed) {
    if (hipEventRecord(c->ev_stop[c->ev_used], st) != hipSuccess) return PWA_E_HIP;
    ++c->ev_used;
  }
  FinalArgs f;
  f.part = c->part;
  f.tot = c->tot;
  f.nb_data = a.nb_data;
  f.nb_mc = a.nb_mc;
  f.V = 1 + (mode == MODE_HVP ? NMOM_HVP : (mode == MODE_NLL ? 0 : NMOM_GRAD)) * c->K;
  f.tbl = c->tbl64;
  f.K = c->K;
  f.mode = mode;
  f.out_kind = out_kind;
  f.n_data = (double)c->n_data;
  f.n_mc = (double)c->n_mc;
  f.v = d_v;
  f.nll = d_nll;
  f.grad = d_grad;
  f.hv = d_hv;
  f.dd_out = d_dd;
  f.status = c->status;
  e = launch_final(f, st);
  if (e != hipSuccess) return PWA_E_HIP;
  if (mode == MODE_HVP && !mc_only) {
    double* ct = cache_theta_slot(c);
    if (d_theta != ct &&
        hipMemcpyAsync(ct, d_theta, sizeof(double) * c->P, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return PWA_E_HIP;
    c->hvp_cache = true;
    c->cache_prec = prec;
  } else if (reuse) {
    c->hvp_cache = true;
  }
  return PWA_OK;
}

int check_prec(const pwa_ctx* c, int prec) {
  if (prec == PWA_PREC_F64) return (c->streams & PWA_STREAM_F64) ? PWA_OK : PWA_E_INVALID;
  if (prec == PWA_PREC_F32) return (c->streams & PWA_STREAM_F32) ? PWA_OK : PWA_E_INVALID;
  return PWA_E_INVALID;
}

}  // namespace

extern "C" {

const char* pwa_status_str(int s) {
  switch (s) {
    case PWA_OK: return "ok";
    case PWA_E_INVALID: return "invalid argument";
    case PWA_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case PWA_E_HIP: return "HIP runtime error";
    case PWA_E_DOMAIN: return "NLL not finite at the start point";
    case PWA_E_NOCONV: return "fit stopped before meeting xtol";
    case PWA_E_STATE: return "context not bound to events";
    default: return "unknown status";
  }
}

int pwa_create(const pwa_model* m, int32_t streams, pwa_ctx** out) {
  if (!m || !out) return PWA_E_INVALID;
  *out = nullptr;
  if (m->n_res < 1 || m->n_res > PWA_MAX_RES) return PWA_E_INVALID;
  if (!(streams & (PWA_STREAM_F64 | PWA_STREAM_F32)) || (streams & ~3)) return PWA_E_INVALID;
  if (m->width_mode != PWA_WIDTH_MASS_DEPENDENT && m->width_mode != PWA_WIDTH_CONSTANT)
    return PWA_E_INVALID;
  if (!finite_pos(m->parent_mass) || !finite_pos(m->r)) return PWA_E_INVALID;
  for (int i = 0; i < 3; ++i)
    if (!finite_pos(m->masses[i])) return PWA_E_INVALID;
  if (!(m->parent_mass > m->masses[0] + m->masses[1] + m->masses[2])) return PWA_E_INVALID;
  if (m->parent_spin != 0 && m->parent_spin != 1) return PWA_E_INVALID;
  bool flatte = false;
  for (int k = 0; k < m->n_res; ++k) {
    if (m->channel[k] < 0 || m->channel[k] > 2) return PWA_E_INVALID;
    if (m->spin[k] < 0 || m->spin[k] > 2) return PWA_E_INVALID;
    if (m->lineshape[k] != PWA_LINESHAPE_BREIT_WIGNER && m->lineshape[k] != PWA_LINESHAPE_FLATTE)
      return PWA_E_INVALID;
    if (m->lineshape[k] == PWA_LINESHAPE_FLATTE) {
      if (m->spin[k] != 0) return PWA_E_INVALID;   // the Flatte form is for scalars
      flatte = true;
    }
  }
  if (flatte && (!finite_pos(m->flatte_masses[0]) || !finite_pos(m->flatte_masses[1]) ||
                 !(m->flatte_ratio >= 0.0) || !isfinite(m->flatte_ratio)))
    return PWA_E_INVALID;
  const bool gen = flatte || m->parent_spin == 1;
  if (gen && m->n_res > kMaxGenRes) return PWA_E_INVALID;
  pwa_ctx* c = new (std::nothrow) pwa_ctx();
  if (!c) return PWA_E_INVALID;
  c->model = *m;
  c->streams = streams;
  c->precision = (streams & PWA_STREAM_F64) ? PWA_PREC_F64 : PWA_PREC_F32;
  c->K = m->n_res;
  c->P = 4 * m->n_res;
  // field layout: s per channel, g per (channel, J), u per (channel, J >= 1)
  // of Breit-Wigner resonances; the general path adds the Flatte width
  // factor per channel, a spin-1 parent's u^mu per (channel, J), and a zero
  // plane for the factors a resonance lacks
  FieldSpec& fs = c->fs;
  for (int ch = 0; ch < 3; ++ch) {
    fs.s_field[ch] = fs.fg_field[ch] = fs.fh_field[ch] = -1;
    for (int J = 0; J < 3; ++J) {
      fs.u_field[ch][J] = fs.g_field[ch][J] = -1;
      for (int q = 0; q < 4; ++q) fs.uc_field[ch][J][q] = -1;
    }
  }
  int nf = 0;
  for (int k = 0; k < c->K; ++k) {
    const int ch = m->channel[k], J = m->spin[k];
    if (fs.s_field[ch] < 0) fs.s_field[ch] = nf++;
    if (m->lineshape[k] == PWA_LINESHAPE_FLATTE) {
      if (fs.fg_field[ch] < 0) {
        fs.fg_field[ch] = nf++;
        fs.fh_field[ch] = nf++;
      }
    } else if (fs.g_field[ch][J] < 0) {
      fs.g_field[ch][J] = nf++;
      if (J >= 1 && m->parent_spin == 0) fs.u_field[ch][J] = nf++;
    }
    if (m->parent_spin == 1 && fs.uc_field[ch][J][0] < 0) {
      for (int q = 0; q < 4; ++q) fs.uc_field[ch][J][q] = nf++;
      // the precompute writes u^mu beside the (channel, J) width factor
      if (fs.g_field[ch][J] < 0) fs.g_field[ch][J] = nf++;
    }
  }
  fs.zero_field = gen ? nf++ : -1;
  fs.n_fields = nf;
  if (nf > (gen ? MAX_GEN_FIELDS : MAX_FIELDS)) {   // bounded by the layout above
    delete c;
    return PWA_E_INVALID;
  }
  ModelDev& md = c->md;
  memset(&md, 0, sizeof(md));
  md.M2 = m->parent_mass * m->parent_mass;
  for (int i = 0; i < 3; ++i) {
    md.m[i] = m->masses[i];
    md.msq[i] = m->masses[i] * m->masses[i];
  }
  md.r2 = m->r * m->r;
  md.K = c->K;
  md.width_mode = m->width_mode;
  md.parent_spin = m->parent_spin;
  md.gen = gen ? 1 : 0;
  md.fl_msq[0] = m->flatte_masses[0] * m->flatte_masses[0];
  md.fl_msq[1] = m->flatte_masses[1] * m->flatte_masses[1];
  md.fl_ratio = m->flatte_ratio;
  for (int k = 0; k < c->K; ++k) {
    const int ch = m->channel[k], J = m->spin[k];
    const bool fl = m->lineshape[k] == PWA_LINESHAPE_FLATTE;
    md.ch[k] = ch;
    md.spin[k] = J;
    md.lineshape[k] = m->lineshape[k];
    int* f = md.fidx[k];
    const int zero = gen ? fs.zero_field : fs.s_field[ch];
    f[IT_S] = fs.s_field[ch];
    f[IT_J] = J;
    f[IT_G] = fl ? fs.fg_field[ch] : fs.g_field[ch][J];
    f[IT_H] = fl ? fs.fh_field[ch] : zero;
    if (m->parent_spin == 1) {
      f[IT_U] = fs.uc_field[ch][J][0];
      f[IT_UI] = fs.uc_field[ch][J][1];
      f[IT_U1R] = fs.uc_field[ch][J][2];
      f[IT_U1I] = fs.uc_field[ch][J][3];
    } else {
      f[IT_U] = J >= 1 ? fs.u_field[ch][J] : fs.s_field[ch];   // J = 0: u = 1 (UMUL = 0)
      f[IT_UI] = f[IT_U1R] = f[IT_U1I] = zero;
    }
  }
  *out = c;
  return PWA_OK;
}

void pwa_destroy(pwa_ctx* c) { delete c; }

int32_t pwa_n_par(const pwa_ctx* c) { return c ? c->P : -1; }

int32_t pwa_stream_fields(const pwa_ctx* c) { return c ? c->fs.n_fields : -1; }

// Events per context: every plane of the event stream is addressed with a
// 32-bit byte offset, so its padded length is limited to 2^32 bytes in FP64.
// Events per context: plane offsets of the stream fit 32 bits, and so do the
// per-lane offsets of the staged loads (up to PPI - 1 planes beyond the
// group's first: one FP64 plane, three FP32 planes).
constexpr int64_t kMaxEvents = ((int64_t)1 << 29) - 256;
constexpr int64_t kMaxEventsF32 = 357000000;

size_t pwa_workspace_bytes(const pwa_ctx* c, int64_t n_data, int64_t n_mc) {
  if (!c || n_data < 0 || n_mc < 1) return 0;
  if (n_data + n_mc > ((c->streams & PWA_STREAM_F32) ? kMaxEventsF32 : kMaxEvents)) return 0;
  return layout_of(c, n_data, n_mc).total;
}

namespace {

// Bind both event sets; the orientation arrays (d_cosb, d_gam and their MC
// counterparts) are read for a spin-1 parent only.
int bind_events(pwa_ctx* c, const double* d_s12, const double* d_s13, const double* d_cosb,
                const double* d_gam, int64_t n_data, const double* d_mc_s12,
                const double* d_mc_s13, const double* d_mc_cosb, const double* d_mc_gam,
                int64_t n_mc, void* d_ws, size_t ws_bytes, hipStream_t st) {
  if (!c || n_data < 0 || n_mc < 1) return PWA_E_INVALID;
  if (n_data > 0 && (!d_s12 || !d_s13)) return PWA_E_INVALID;
  if (!d_mc_s12 || !d_mc_s13) return PWA_E_INVALID;
  if (c->md.parent_spin == 1 && ((n_data > 0 && (!d_cosb || !d_gam)) || !d_mc_cosb || !d_mc_gam))
    return PWA_E_INVALID;
  const int64_t max_ev = (c->streams & PWA_STREAM_F32) ? kMaxEventsF32 : kMaxEvents;
  if (n_data > max_ev || n_mc > max_ev || n_data + n_mc > max_ev) return PWA_E_INVALID;
  if (!d_ws || ((uintptr_t)d_ws % 256) != 0) return PWA_E_WORKSPACE;
  const Layout L = layout_of(c, n_data, n_mc);
  if (ws_bytes < L.total) return PWA_E_WORKSPACE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PWA_E_HIP;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return PWA_E_HIP;
  c->cu_count = cus;
  c->bound = false;
  c->n_data = n_data;
  c->n_mc = n_mc;
  c->stride = L.stride;
  c->mc_off = L.mc_off;
  c->ws = (char*)d_ws;
  c->ws_bytes = ws_bytes;
  c->status = (int*)(c->ws + L.status);
  c->tbl64 = (double*)(c->ws + L.tbl64);
  c->tbl32 = (float*)(c->ws + L.tbl32);
  c->itbl = (int*)(c->ws + L.itbl);
  c->part = (double*)(c->ws + L.part);
  c->tot = (double*)(c->ws + L.tot);
  c->dd = (double*)(c->ws + L.dd);
  c->scratch = (double*)(c->ws + L.scratch);
  c->planes64 = (c->streams & PWA_STREAM_F64) ? (double*)(c->ws + L.planes64) : nullptr;
  c->planes32 = (c->streams & PWA_STREAM_F32) ? (float*)(c->ws + L.planes32) : nullptr;
  c->grid_cache.clear();
  if (hipMemsetAsync(c->status, 0, 64 * sizeof(int), st) != hipSuccess) return PWA_E_HIP;
  for (int f32 = 0; f32 < 2; ++f32) {
    void* planes = f32 ? (void*)c->planes32 : (void*)c->planes64;
    if (!planes) continue;
    if (launch_precompute(d_s12, d_s13, d_cosb, d_gam, n_data, 0, planes, L.stride, f32, c->md,
                          c->fs, st) != hipSuccess)
      return PWA_E_HIP;
    if (launch_precompute(d_mc_s12, d_mc_s13, d_mc_cosb, d_mc_gam, n_mc, L.mc_off, planes, L.stride,
                          f32, c->md, c->fs, st) != hipSuccess)
      return PWA_E_HIP;
  }
  c->bound = true;
  c->hvp_cache = false;
  return PWA_OK;
}

}  // namespace

int pwa_bind(pwa_ctx* c, const double* d_s12, const double* d_s13, int64_t n_data,
             const double* d_mc_s12, const double* d_mc_s13, int64_t n_mc, void* d_ws,
             size_t ws_bytes, hipStream_t st) {
  if (c && c->md.parent_spin != 0) return PWA_E_INVALID;
  return bind_events(c, d_s12, d_s13, nullptr, nullptr, n_data, d_mc_s12, d_mc_s13, nullptr,
                     nullptr, n_mc, d_ws, ws_bytes, st);
}

int pwa_bind_oriented(pwa_ctx* c, const double* d_s12, const double* d_s13, const double* d_cosb,
                      const double* d_gam, int64_t n_data, const double* d_mc_s12,
                      const double* d_mc_s13, const double* d_mc_cosb, const double* d_mc_gam,
                      int64_t n_mc, void* d_ws, size_t ws_bytes, hipStream_t st) {
  if (!c || c->md.parent_spin != 1) return PWA_E_INVALID;
  return bind_events(c, d_s12, d_s13, d_cosb, d_gam, n_data, d_mc_s12, d_mc_s13, d_mc_cosb,
                     d_mc_gam, n_mc, d_ws, ws_bytes, st);
}

int pwa_set_precision(pwa_ctx* c, int32_t prec) {
  if (!c) return PWA_E_INVALID;
  if (check_prec(c, prec) != PWA_OK) return PWA_E_INVALID;
  c->precision = prec;
  return PWA_OK;
}

int pwa_set_launch_shape(pwa_ctx* c, int32_t layout, int32_t T, int32_t R) {
  if (!c) return PWA_E_INVALID;
  if (layout == 0) {
    c->shape_L = c->shape_T = c->shape_R = 0;
    return PWA_OK;
  }
  // layouts 1, 2 serve Breit-Wigner models of a spin-0 parent, layout 3 the
  // general physics path
  if ((layout == 3) != (c->md.gen != 0)) return PWA_E_INVALID;
  const bool built = (layout == 1) ? shape_built(T, R)
                     : (layout == 2 ? wg_shape_built(T, R) : (layout == 3 ? gen_shape_built(T, R) : false));
  if (!built || T * R < c->K || T * R > KPAD) return PWA_E_INVALID;
  c->shape_L = layout;
  c->shape_T = T;
  c->shape_R = R;
  return PWA_OK;
}

int32_t pwa_grid_blocks(const pwa_ctx* c) {
  if (!c || !c->bound) return -1;
  int L, T, R;
  shape_of(c, MODE_HVP, L, T, R);
  return grid_blocks(const_cast<pwa_ctx*>(c), c->precision, MODE_HVP, L, T, R);
}

int pwa_set_kernel_timing(pwa_ctx* c, int32_t enable) {
  if (!c) return PWA_E_INVALID;
  if (enable && c->ev_start.empty()) {
    c->ev_start.resize(kEventPool);
    c->ev_stop.resize(kEventPool);
    for (int i = 0; i < kEventPool; ++i)
      if (hipEventCreate(&c->ev_start[i]) != hipSuccess || hipEventCreate(&c->ev_stop[i]) != hipSuccess)
        return PWA_E_HIP;
  }
  c->timing = enable != 0;
  return PWA_OK;
}

int pwa_kernel_time(pwa_ctx* c, double* total_ms, int64_t* n) {
  if (!c || !total_ms || !n) return PWA_E_INVALID;
  const int s = fold_timing(c);
  if (s != PWA_OK) return s;
  *total_ms = c->timed_ms;
  *n = c->timed_n;
  c->timed_ms = 0.0;
  c->timed_n = 0;
  return PWA_OK;
}

int pwa_nll(pwa_ctx* c, const double* d_theta, double* d_nll, hipStream_t st) {
  if (!c || !d_theta || !d_nll) return PWA_E_INVALID;
  if (!c->bound) return PWA_E_STATE;
  return run_eval(c, MODE_NLL, OUT_COMBINED, c->precision, d_theta, nullptr, d_nll, nullptr,
                  nullptr, nullptr, st);
}

int pwa_grad(pwa_ctx* c, const double* d_theta, double* d_nll, double* d_grad, hipStream_t st) {
  if (!c || !d_theta || !d_grad) return PWA_E_INVALID;
  if (!c->bound) return PWA_E_STATE;
  return run_eval(c, MODE_GRAD, OUT_COMBINED, c->precision, d_theta, nullptr, d_nll, d_grad,
                  nullptr, nullptr, st);
}

int pwa_hvp(pwa_ctx* c, const double* d_theta, const double* d_v, double* d_hv, double* d_nll,
            double* d_grad, hipStream_t st) {
  if (!c || !d_theta || !d_v || !d_hv) return PWA_E_INVALID;
  if (!c->bound) return PWA_E_STATE;
  return run_eval(c, MODE_HVP, OUT_COMBINED, c->precision, d_theta, d_v, d_nll, d_grad, d_hv,
                  nullptr, st);
}

int pwa_hvp_reuse(pwa_ctx* c, const double* d_v, double* d_hv, double* d_nll, double* d_grad,
                  hipStream_t st) {
  if (!c || !d_v || !d_hv) return PWA_E_INVALID;
  if (!c->bound) return PWA_E_STATE;
  if (!c->hvp_cache) return PWA_E_STATE;
  return run_eval(c, MODE_HVPB, OUT_COMBINED, c->precision, cache_theta_slot(c), d_v, d_nll,
                  d_grad, d_hv, nullptr, st);
}

int pwa_partials_reuse(pwa_ctx* c, const double* d_v, double* d_part, hipStream_t st) {
  if (!c || !d_v || !d_part) return PWA_E_INVALID;
  if (!c->bound) return PWA_E_STATE;
  if (!c->hvp_cache) return PWA_E_STATE;
  return run_eval(c, MODE_HVPB, OUT_PARTIALS, c->precision, cache_theta_slot(c), d_v, nullptr,
                  nullptr, nullptr, d_part, st);
}

int pwa_intensity(pwa_ctx* c, const double* d_theta, int32_t which, double* d_out,
                  hipStream_t st) {
  if (!c || !d_theta || !d_out || (which != 0 && which != 1)) return PWA_E_INVALID;
  if (!c->bound) return PWA_E_STATE;
  const int64_t n = which ? c->n_mc : c->n_data;
  const int64_t base = which ? c->mc_off : 0;
  if (launch_table(d_theta, nullptr, c->md, c->K, c->tbl64, c->tbl32, c->itbl, c->status, st) !=
      hipSuccess)
    return PWA_E_HIP;
  const bool f32 = c->precision == PWA_PREC_F32;
  return launch_intensity(f32, f32 ? (const void*)c->planes32 : (const void*)c->planes64, c->stride,
                          base, n, c->tbl64, c->itbl, c->K, c->md.gen,
                          c->md.parent_spin == 1 ? 2 : 1, d_out, st) == hipSuccess
             ? PWA_OK
             : PWA_E_HIP;
}

int pwa_partials(pwa_ctx* c, const double* d_theta, const double* d_v, double* d_part,
                 hipStream_t st) {
  if (!c || !d_theta || !d_part) return PWA_E_INVALID;
  if (!c->bound) return PWA_E_STATE;
  return run_eval(c, d_v ? MODE_HVP : MODE_GRAD, OUT_PARTIALS, c->precision, d_theta, d_v,
                  nullptr, nullptr, nullptr, d_part, st);
}

int pwa_combine(int32_t n_par, int32_t n_shards, const double* d_parts, int64_t n_data_total,
                int64_t n_mc_total, const double* d_v, double* d_nll, double* d_grad,
                double* d_hv, hipStream_t st) {
  if (n_par < 4 || n_par > 4 * PWA_MAX_RES || (n_par % 4) != 0) return PWA_E_INVALID;
  if (n_shards < 1 || !d_parts || !d_nll) return PWA_E_INVALID;
  if (n_data_total < 0 || n_mc_total < 1) return PWA_E_INVALID;
  if (d_hv && (!d_v || !d_grad)) return PWA_E_INVALID;
  return launch_combine(n_par, n_shards, d_parts, (double)n_data_total, (double)n_mc_total, d_v,
                        d_nll, d_grad, d_hv, nullptr, st) == hipSuccess
             ? PWA_OK
             : PWA_E_HIP;
}

int pwa_device_status(pwa_ctx* c, hipStream_t st) {
  if (!c) return PWA_E_INVALID;
  if (!c->bound) return PWA_E_STATE;
  int h = 0;
  if (hipMemcpyAsync(&h, c->status + 1, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
    return PWA_E_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return PWA_E_HIP;
  if (hipMemsetAsync(c->status + 1, 0, sizeof(int), st) != hipSuccess) return PWA_E_HIP;
  return h;
}

// ---------------------------------------------------------------------------
// Newton-CG fit.
// ---------------------------------------------------------------------------
namespace {

struct Fitter {
  pwa_ctx* c;
  hipStream_t st;
  int P;
  std::vector<unsigned char> free_;
  double* d_x;   // device scratch
  double* d_v;
  double* d_out; // [nll, grad(P), hv(P)]
  int prec_hvp;
  int prec_main;
  int n_nll = 0, n_grad = 0, n_hvp = 0;
  int err = PWA_OK;

  void mask(std::vector<double>& g) const {
    for (int i = 0; i < P; ++i)
      if (!free_[i]) g[i] = 0.0;
  }
  bool up(const std::vector<double>& x, double* d) {
    if (hipMemcpyAsync(d, x.data(), sizeof(double) * P, hipMemcpyHostToDevice, st) != hipSuccess) {
      err = PWA_E_HIP;
      return false;
    }
    return true;
  }
  bool down(double* h, const double* d, int n) {
    if (hipMemcpyAsync(h, d, sizeof(double) * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      err = PWA_E_HIP;
      return false;
    }
    return true;
  }
  // f and gradient at x (FP64 unless only FP32 exists)
  bool fg(const std::vector<double>& x, double& f, std::vector<double>& g) {
    if (!up(x, d_x)) return false;
    if (run_eval(c, MODE_GRAD, OUT_COMBINED, prec_main, d_x, nullptr, d_out, d_out + 1, nullptr,
                 nullptr, st) != PWA_OK) {
      err = PWA_E_HIP;
      return false;
    }
    std::vector<double> buf(1 + P);
    if (!down(buf.data(), d_out, 1 + P)) return false;
    ++n_grad;
    f = buf[0];
    g.assign(buf.begin() + 1, buf.end());
    mask(g);
    return true;
  }
  bool hvp(const std::vector<double>& x_on_device_dummy, const std::vector<double>& p,
           std::vector<double>& hp) {
    (void)x_on_device_dummy;
    if (!up(p, d_v)) return false;
    // d_x holds the Newton iterate for the whole CG solve: after the first
    // (full) pass, the direction-only pass reuses its theta-only totals
    if (run_eval(c, MODE_HVPB, OUT_COMBINED, prec_hvp, d_x, d_v, nullptr, nullptr,
                 d_out + 1 + P, nullptr, st) != PWA_OK) {
      err = PWA_E_HIP;
      return false;
    }
    hp.resize(P);
    if (!down(hp.data(), d_out + 1 + P, P)) return false;
    ++n_hvp;
    mask(hp);
    return true;
  }
};

double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

double sum_abs(const std::vector<double>& a) {
  double s = 0.0;
  for (double x : a) s += fabs(x);
  return s;
}

// Minimiser of the cubic interpolating (a, fa, ga), (b, fb, gb); NaN if none.
double cubic_min(double a, double fa, double ga, double b, double fb, double gb) {
  const double d1 = ga + gb - 3.0 * (fa - fb) / (a - b);
  const double disc = d1 * d1 - ga * gb;
  if (!(disc >= 0.0)) return NAN;
  const double d2 = copysign(sqrt(disc), b - a);
  return b - (b - a) * (gb + d2 - d1) / (gb - ga + 2.0 * d2);
}

// Strong-Wolfe line search (Nocedal & Wright, Alg. 3.5 with the zoom of
// Alg. 3.6 and cubic interpolation), c1 = 1e-4, c2 = 0.9, first step 1.
// Evaluates f and its gradient at every trial point (one fused pass each).
bool wolfe(Fitter& F, const std::vector<double>& x, double f0, const std::vector<double>& g0,
           const std::vector<double>& p, double& alpha, double& f1, std::vector<double>& g1,
           std::vector<double>& x1) {
  const double c1 = 1e-4, c2 = 0.9;
  const double d0 = dot(g0, p);
  if (!(d0 < 0.0)) return false;
  auto eval = [&](double a, double& fa, double& da, std::vector<double>& ga) {
    x1.resize(x.size());
    for (size_t i = 0; i < x.size(); ++i) x1[i] = x[i] + a * p[i];
    if (!F.fg(x1, fa, ga)) return false;
    if (!isfinite(fa)) {
      fa = INFINITY;
      da = NAN;
    } else {
      da = dot(ga, p);
    }
    return true;
  };
  double a_prev = 0.0, f_prev = f0, d_prev = d0;
  double a = 1.0;
  std::vector<double> ga;
  double lo = 0, hi = 0, flo = 0, fhi = 0, dlo = 0, dhi = 0;
  bool zoom = false;
  for (int i = 0; i < 30; ++i) {
    double fa, da;
    if (!eval(a, fa, da, ga)) return false;
    if (!isfinite(fa) || fa > f0 + c1 * a * d0 || (i > 0 && fa >= f_prev)) {
      lo = a_prev; flo = f_prev; dlo = d_prev;
      hi = a; fhi = fa; dhi = da;
      zoom = true;
      break;
    }
    if (fabs(da) <= -c2 * d0) {
      alpha = a; f1 = fa; g1 = ga;
      return true;
    }
    if (da >= 0.0) {
      lo = a; flo = fa; dlo = da;
      hi = a_prev; fhi = f_prev; dhi = d_prev;
      zoom = true;
      break;
    }
    a_prev = a; f_prev = fa; d_prev = da;
    a *= 2.0;
  }
  if (!zoom) return false;
  for (int i = 0; i < 40; ++i) {
    double at = NAN;
    if (isfinite(fhi) && isfinite(dhi)) at = cubic_min(lo, flo, dlo, hi, fhi, dhi);
    const double lo_b = std::min(lo, hi), hi_b = std::max(lo, hi), w = hi_b - lo_b;
    if (!(at > lo_b + 0.1 * w && at < hi_b - 0.1 * w)) at = 0.5 * (lo + hi);
    double fa, da;
    if (!eval(at, fa, da, ga)) return false;
    if (!isfinite(fa) || fa > f0 + c1 * at * d0 || fa >= flo) {
      hi = at; fhi = fa; dhi = da;
    } else {
      if (fabs(da) <= -c2 * d0) {
        alpha = at; f1 = fa; g1 = ga;
        return true;
      }
      if (da * (hi - lo) >= 0.0) {
        hi = lo; fhi = flo; dhi = dlo;
      }
      lo = at; flo = fa; dlo = da;
    }
    if (fabs(hi - lo) < 1e-16 * std::max(1.0, fabs(lo))) break;
  }
  // accept the best point with sufficient decrease, if any
  if (lo > 0.0 && flo < f0) {
    double fa, da;
    if (!eval(lo, fa, da, ga)) return false;
    alpha = lo; f1 = fa; g1 = ga;
    return true;
  }
  return false;
}

}  // namespace

// Forcing term below which a mixed-precision fit takes its HVPs in FP64.
constexpr double kMixedEtaSwitch = 1e-3;

// Eigen-decomposition of a symmetric n x n matrix A (row-major, destroyed)
// by cyclic Jacobi rotations: A = V diag(w) V^T, V row-major with the
// eigenvectors as columns.
void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += A[(size_t)i * n + i] * A[(size_t)i * n + i];
      for (int j = i + 1; j < n; ++j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    }
    if (off <= 1e-30 * diag || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {   // columns p, q
          const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = cs * akp - sn * akq;
          A[(size_t)k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = cs * apk - sn * aqk;
          A[(size_t)q * n + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = cs * vkp - sn * vkq;
          V[(size_t)k * n + q] = sn * vkp + cs * vkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
}

// CG preconditioner from the Hessian at the current iterate: the inverse of
// its absolute-value form V |diag(w)| V^T on the free parameters, with
// eigenvalues below 1e-6 of the largest raised to that floor (the coupling
// phase and scale directions are null directions of H).  P HVPs along the
// unit vectors of the free parameters.
bool build_preconditioner(Fitter& F, const std::vector<double>& x, std::vector<int>& fidx,
                          std::vector<double>& Minv) {
  const int P = F.P;
  fidx.clear();
  for (int i = 0; i < P; ++i)
    if (F.free_[i]) fidx.push_back(i);
  const int n = (int)fidx.size();
  std::vector<double> H((size_t)n * n), e(P, 0.0), col;
  for (int j = 0; j < n; ++j) {
    e[fidx[j]] = 1.0;
    if (!F.hvp(x, e, col)) return false;
    e[fidx[j]] = 0.0;
    for (int i = 0; i < n; ++i) H[(size_t)i * n + j] = col[fidx[i]];
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double m = 0.5 * (H[(size_t)i * n + j] + H[(size_t)j * n + i]);
      H[(size_t)i * n + j] = H[(size_t)j * n + i] = m;
    }
  std::vector<double> w, V;
  jacobi_eigen(n, H, w, V);
  double wmax = 0.0;
  for (double v : w) wmax = std::max(wmax, fabs(v));
  if (!(wmax > 0.0) || !isfinite(wmax)) return false;
  const double floor_ = 1e-6 * wmax;
  Minv.assign((size_t)n * n, 0.0);
  for (int k = 0; k < n; ++k) {
    const double s = 1.0 / std::max(fabs(w[k]), floor_);
    for (int i = 0; i < n; ++i) {
      const double vik = V[(size_t)i * n + k] * s;
      for (int j = 0; j < n; ++j) Minv[(size_t)i * n + j] += vik * V[(size_t)j * n + k];
    }
  }
  return true;
}

// z = Minv r on the free parameters (zero elsewhere); identity without a
// preconditioner.
void apply_preconditioner(const std::vector<int>& fidx, const std::vector<double>& Minv,
                          const std::vector<double>& r, std::vector<double>& z) {
  z.assign(r.size(), 0.0);
  if (Minv.empty()) {
    z = r;
    return;
  }
  const int n = (int)fidx.size();
  for (int i = 0; i < n; ++i) {
    double a = 0.0;
    for (int j = 0; j < n; ++j) a += Minv[(size_t)i * n + j] * r[fidx[j]];
    z[fidx[i]] = a;
  }
}

int pwa_fit(pwa_ctx* c, double* d_theta, const pwa_fit_opts* o, pwa_fit_report* rep,
            hipStream_t st) {
  if (!c || !d_theta || !o) return PWA_E_INVALID;
  if (!c->bound) return PWA_E_STATE;
  if (!(o->xtol > 0.0) || !isfinite(o->xtol)) return PWA_E_INVALID;
  if (o->forcing != 0 && o->forcing != 1) return PWA_E_INVALID;
  if (o->precondition != 0 && o->precondition != 1) return PWA_E_INVALID;
  if (o->reconjugate != 0 && o->reconjugate != 1) return PWA_E_INVALID;
  const int hp = o->hvp_precision;
  if (check_prec(c, hp) != PWA_OK) return PWA_E_INVALID;
  const auto t0 = std::chrono::steady_clock::now();
  auto elapsed = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  const int P = c->P;
  Fitter F;
  F.c = c;
  F.st = st;
  F.P = P;
  F.free_.assign(P, 1);
  if (o->free_mask_set)
    for (int i = 0; i < P; ++i) F.free_[i] = o->free_mask[i] ? 1 : 0;
  F.d_x = c->scratch;
  F.d_v = c->scratch + P;
  F.d_out = c->scratch + 2 * P;
  F.prec_hvp = hp;
  F.prec_main = (c->streams & PWA_STREAM_F64) ? PWA_PREC_F64 : PWA_PREC_F32;
  const int maxiter = o->maxiter > 0 ? o->maxiter : 200;
  const int cg_max = o->cg_maxiter > 0 ? o->cg_maxiter : 20 * P;

  std::vector<double> x(P), g, best_x;
  if (hipMemcpyAsync(x.data(), d_theta, sizeof(double) * P, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return PWA_E_HIP;
  double f, maggrad0 = 1.0;
  int status = PWA_OK, converged = 0, it = 0;
  if (!F.fg(x, f, g)) return F.err;
  if (!isfinite(f)) status = PWA_E_DOMAIN;
  best_x = x;
  double best_f = f;
  std::vector<double> r(P), pcg(P), xs(P), zc(P), Ap, x1, g1;
  // preconditioner state: free indices, inverse, CG steps of the last solve
  std::vector<int> fidx;
  std::vector<double> Minv;
  int last_cg = 0;
  while (status == PWA_OK) {
    if (it >= maxiter) { status = PWA_E_NOCONV; break; }
    if (o->time_cap_s > 0 && elapsed() > o->time_cap_s) { status = PWA_E_NOCONV; break; }
    // truncated CG on H p = -g (scipy's forcing term and curvature tests)
    const double maggrad = sum_abs(g);
    if (it == 0) maggrad0 = maggrad > 0.0 ? maggrad : 1.0;
    const double eta = std::min(0.5, sqrt(o->forcing == 1 ? maggrad / maggrad0 : maggrad));
    const double termcond = eta * maggrad;
    // Mixed precision: FP32 Hessian-vector products carry a relative error
    // of order 1e-5, so CG cannot meet a tolerance much below that with
    // them; Newton steps whose forcing term asks for more use FP64 HVPs.
    F.prec_hvp = (hp == PWA_PREC_F32 && eta < kMixedEtaSwitch) ? PWA_PREC_F64 : hp;
    std::fill(xs.begin(), xs.end(), 0.0);
    // the HVPs are taken at x: upload x once
    if (!F.up(x, F.d_x)) return F.err;
    // Optional preconditioner: the Hessian at the first iterate, rebuilt
    // when the previous solve needed many CG steps (it has gone stale).
    if (o->precondition == 1 && (Minv.empty() || last_cg > std::max(8, P / 4))) {
      if (!build_preconditioner(F, x, fidx, Minv)) {
        if (F.err != PWA_OK) return F.err;
        Minv.clear();
      }
    }
    r = g;
    apply_preconditioner(fidx, Minv, r, zc);
    for (int i = 0; i < P; ++i) pcg[i] = -zc[i];
    double dri0 = dot(r, zc);
    int i = 0;
    // earlier directions of this solve, their H p and p.Hp (reconjugate)
    std::vector<std::vector<double>> dirs, hdirs;
    std::vector<double> dcurv;
    for (int k = 0; k < cg_max; ++k) {
      if (sum_abs(r) <= termcond) break;
      if (o->reconjugate == 1) {
        for (size_t j = 0; j < dirs.size(); ++j) {
          const double cj = dot(pcg, hdirs[j]) / dcurv[j];
          for (int q = 0; q < P; ++q) pcg[q] -= cj * dirs[j][q];
        }
      }
      if (!F.hvp(x, pcg, Ap)) return F.err;
      const double curv = dot(pcg, Ap);
      if (0.0 <= curv && curv <= 3.0 * 2.220446049250313e-16) break;
      if (curv < 0.0) {
        if (i > 0) break;
        // first direction: step along the (preconditioned) steepest descent
        for (int j = 0; j < P; ++j) xs[j] = dri0 / (-curv) * pcg[j];
        break;
      }
      // step to the minimum along pcg: (r.z) / (p.Hp) for the recurrence's
      // direction, -(r.p) / (p.Hp) in general
      const double al = o->reconjugate == 1 ? -dot(r, pcg) / curv : dri0 / curv;
      if (o->reconjugate == 1) {
        dirs.push_back(pcg);
        hdirs.push_back(Ap);
        dcurv.push_back(curv);
      }
      for (int j = 0; j < P; ++j) {
        xs[j] += al * pcg[j];
        r[j] += al * Ap[j];
      }
      apply_preconditioner(fidx, Minv, r, zc);
      const double dri1 = dot(r, zc);
      const double be = dri1 / dri0;
      for (int j = 0; j < P; ++j) pcg[j] = -zc[j] + be * pcg[j];
      ++i;
      dri0 = dri1;
    }
    last_cg = i;
    // A Newton step already within the tolerance ends the fit here: at the
    // minimum the NLL is flat to rounding, and a line search along such a
    // step can find no decrease.
    if (sum_abs(xs) <= P * o->xtol) {
      converged = 1;
      break;
    }
    double alpha, f1;
    if (!wolfe(F, x, f, g, xs, alpha, f1, g1, x1)) {
      if (F.err != PWA_OK) return F.err;
      status = PWA_E_NOCONV;
      break;
    }
    double upd = 0.0;
    for (int j = 0; j < P; ++j) upd += fabs(alpha * xs[j]);
    x = x1;
    f = f1;
    g = g1;
    ++it;
    if (f < best_f) { best_f = f; best_x = x; }
    if (upd <= P * o->xtol) { converged = 1; break; }
  }
  if (status == PWA_E_DOMAIN) best_x = x;
  if (hipMemcpyAsync(d_theta, best_x.data(), sizeof(double) * P, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return PWA_E_HIP;
  if (rep) {
    double gm = 0.0;
    std::vector<double> gb;
    double fb = best_f;
    if (status != PWA_E_DOMAIN && F.fg(best_x, fb, gb))
      for (int j = 0; j < P; ++j) gm = std::max(gm, fabs(gb[j]));
    rep->nll = fb;
    rep->grad_max = gm;
    rep->seconds = elapsed();
    rep->iterations = it;
    rep->n_nll = F.n_nll;
    rep->n_grad = F.n_grad;
    rep->n_hvp = F.n_hvp;
    rep->status = converged ? PWA_OK : status;
    rep->converged = converged;
  }
  if (converged) return PWA_OK;
  return status;
}

// Gradient-only quasi-Newton comparator: BFGS on the inverse Hessian
// approximation (Nocedal & Wright, Alg. 6.1), first inverse scaled by
// y's/y'y after the first step (their eq. (6.20)), the same strong-Wolfe
// search as pwa_fit, FP64 NLL and gradient only.  It stops when the full
// quasi-Newton step, or a step of at least half of it, is within the
// tolerance (mean |p| <= xtol).  The paper compares Newton-CG with gradient-only
// Migrad (Sec. 3); this is that arm of the comparison in the same driver.
int pwa_fit_bfgs(pwa_ctx* c, double* d_theta, const pwa_fit_opts* o, pwa_fit_report* rep,
                 hipStream_t st) {
  if (!c || !d_theta || !o) return PWA_E_INVALID;
  if (!c->bound) return PWA_E_STATE;
  if (!(o->xtol > 0.0) || !isfinite(o->xtol)) return PWA_E_INVALID;
  const auto t0 = std::chrono::steady_clock::now();
  auto elapsed = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  const int P = c->P;
  Fitter F;
  F.c = c;
  F.st = st;
  F.P = P;
  F.free_.assign(P, 1);
  if (o->free_mask_set)
    for (int i = 0; i < P; ++i) F.free_[i] = o->free_mask[i] ? 1 : 0;
  F.d_x = c->scratch;
  F.d_v = c->scratch + P;
  F.d_out = c->scratch + 2 * P;
  F.prec_hvp = PWA_PREC_F64;
  F.prec_main = (c->streams & PWA_STREAM_F64) ? PWA_PREC_F64 : PWA_PREC_F32;
  const int maxiter = o->maxiter > 0 ? o->maxiter : 200;

  std::vector<double> x(P), g;
  if (hipMemcpyAsync(x.data(), d_theta, sizeof(double) * P, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return PWA_E_HIP;
  double f;
  int status = PWA_OK, converged = 0, it = 0;
  if (!F.fg(x, f, g)) return F.err;
  if (!isfinite(f)) status = PWA_E_DOMAIN;
  std::vector<double> best_x = x;
  double best_f = f;
  // inverse Hessian approximation (row-major P x P), identity until the
  // first curvature pair scales it
  std::vector<double> Hi((size_t)P * P, 0.0), p(P), x1, g1, s(P), y(P), Hy(P);
  for (int i = 0; i < P; ++i) Hi[(size_t)i * P + i] = 1.0;
  bool scaled = false;
  while (status == PWA_OK) {
    if (it >= maxiter) { status = PWA_E_NOCONV; break; }
    if (o->time_cap_s > 0 && elapsed() > o->time_cap_s) { status = PWA_E_NOCONV; break; }
    double gmax = 0.0;
    for (int i = 0; i < P; ++i) gmax = std::max(gmax, fabs(g[i]));
    if (gmax == 0.0) { converged = 1; break; }
    for (int i = 0; i < P; ++i) {
      double a = 0.0;
      for (int j = 0; j < P; ++j) a += Hi[(size_t)i * P + j] * g[j];
      p[i] = -a;
    }
    // before any curvature is known the step is the gradient scaled to unit
    // 2-norm (scipy's BFGS takes the same first trial length)
    if (!scaled) {
      const double gn = sqrt(dot(g, g));
      for (int i = 0; i < P; ++i) p[i] *= std::min(1.0, 1.01 / gn);
    } else if (sum_abs(p) <= P * o->xtol) {
      // a full quasi-Newton step within the tolerance ends the fit, as a
      // Newton step does in pwa_fit (no decrease is measurable below it)
      converged = 1;
      break;
    }
    double alpha, f1;
    if (!wolfe(F, x, f, g, p, alpha, f1, g1, x1)) {
      if (F.err != PWA_OK) return F.err;
      status = PWA_E_NOCONV;
      break;
    }
    double upd = 0.0;
    for (int i = 0; i < P; ++i) {
      s[i] = x1[i] - x[i];
      y[i] = g1[i] - g[i];
      upd += fabs(s[i]);
    }
    x = x1;
    f = f1;
    g = g1;
    ++it;
    if (f < best_f) { best_f = f; best_x = x; }
    // the step taken ends the fit only when it was (nearly) the full
    // quasi-Newton step: a short line-search step far from the minimum says
    // nothing about convergence
    if (alpha >= 0.5 && upd <= P * o->xtol) { converged = 1; break; }
    const double ys = dot(y, s);
    if (!(ys > 0.0)) continue;   // no curvature information: keep Hi
    if (!scaled) {
      const double sc = ys / dot(y, y);
      for (int i = 0; i < P; ++i) Hi[(size_t)i * P + i] = F.free_[i] ? sc : 1.0;
      scaled = true;
    }
    // Hi <- (I - rho s y') Hi (I - rho y s') + rho s s'
    //     = Hi - rho (s (Hi y)' + (Hi y) s') + rho (1 + rho y' Hi y) s s'
    const double rho = 1.0 / ys;
    for (int i = 0; i < P; ++i) {
      double a = 0.0;
      for (int j = 0; j < P; ++j) a += Hi[(size_t)i * P + j] * y[j];
      Hy[i] = a;
    }
    const double yHy = dot(y, Hy);
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j)
        Hi[(size_t)i * P + j] += -rho * (s[i] * Hy[j] + Hy[i] * s[j]) + rho * (1.0 + rho * yHy) * s[i] * s[j];
  }
  if (status == PWA_E_DOMAIN) best_x = x;
  if (hipMemcpyAsync(d_theta, best_x.data(), sizeof(double) * P, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return PWA_E_HIP;
  if (rep) {
    double gm = 0.0;
    std::vector<double> gb;
    double fb = best_f;
    if (status != PWA_E_DOMAIN && F.fg(best_x, fb, gb))
      for (int j = 0; j < P; ++j) gm = std::max(gm, fabs(gb[j]));
    rep->nll = fb;
    rep->grad_max = gm;
    rep->seconds = elapsed();
    rep->iterations = it;
    rep->n_nll = F.n_nll;
    rep->n_grad = F.n_grad;
    rep->n_hvp = 0;
    rep->status = converged ? PWA_OK : status;
    rep->converged = converged;
  }
  if (converged) return PWA_OK;
  return status;
}

// ---------------------------------------------------------------------------
// Batched path.
// ---------------------------------------------------------------------------
namespace {
constexpr int kBatchRowBlocks = 2048;
constexpr int kGramBlocks = 1024;   // 4 blocks per CU (37 KB of LDS each)
constexpr int kGP = 48;

struct BLayout {
  size_t A, C, esum, part, part2, gpart, xtx, gram, total;
  size_t a_plane, c_plane;   // bytes per operand plane
  int KP;
};

BLayout blayout(const pwa_ctx* c, int64_t n_data, int fmt, int max_batch) {
  BLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  L.KP = batched_kp(fmt, c->K);
  const size_t eb = batched_elem_bytes(fmt);
  // planes of one operand are contiguous (the sliced kernels index them so)
  L.a_plane = (size_t)n_data * L.KP * eb;
  L.c_plane = (size_t)L.KP * 2 * max_batch * eb;
  L.A = take(std::max<size_t>(L.a_plane * batched_a_planes(fmt), 1));
  L.C = take(L.c_plane * batched_c_planes(fmt));
  L.esum = take(sizeof(unsigned long long));
  L.part = take(sizeof(double) * 2 * (size_t)kBatchRowBlocks * max_batch);
  L.part2 = take(sizeof(double) * 2 * (size_t)kBatchChunks * max_batch);
  L.gpart = take(sizeof(double) * 2 * (size_t)kGramBlocks * kGP * kGP);
  L.xtx = take(sizeof(double) * (size_t)kGP * kGP);
  L.gram = take(sizeof(double) * 2 * (size_t)c->K * c->K);
  L.total = off;
  return L;
}
}  // namespace

size_t pwa_batched_workspace_bytes(const pwa_ctx* c, int64_t n_data, int32_t fmt,
                                   int32_t max_batch) {
  if (!c || n_data < 0 || fmt < PWA_OP_F64 || fmt > PWA_OP_F16S) return 0;
  if (max_batch < 1 || max_batch > 65536 || 2 * c->K > kGP) return 0;
  return blayout(c, n_data, fmt, max_batch).total;
}

int pwa_freeze(pwa_ctx* c, const double* d_theta, int32_t fmt, int32_t max_batch, void* d_bws,
               size_t bws_bytes, hipStream_t st) {
  if (!c || !d_theta) return PWA_E_INVALID;
  if (fmt < PWA_OP_F64 || fmt > PWA_OP_F16S || max_batch < 1 || max_batch > 65536) return PWA_E_INVALID;
  if (2 * c->K > kGP) return PWA_E_INVALID;
  // one amplitude row per event: a spin-1 parent's two helicity amplitudes
  // are not laid out on this path
  if (c->md.parent_spin != 0) return PWA_E_INVALID;
  if (!c->bound) return PWA_E_STATE;
  if (!(c->streams & PWA_STREAM_F64)) return PWA_E_INVALID;
  if (!d_bws || ((uintptr_t)d_bws % 256) != 0) return PWA_E_WORKSPACE;
  const BLayout L = blayout(c, c->n_data, fmt, max_batch);
  if (bws_bytes < L.total) return PWA_E_WORKSPACE;
  char* w = (char*)d_bws;
  c->frozen = false;
  c->bfmt = fmt;
  c->bKP = L.KP;
  c->bmax = max_batch;
  for (int s = 0; s < kSlices; ++s) {
    c->bA[s] = s < batched_a_planes(fmt) ? (void*)(w + L.A + s * L.a_plane) : nullptr;
    c->bC[s] = s < batched_c_planes(fmt) ? (void*)(w + L.C + s * L.c_plane) : nullptr;
  }
  c->besum = (unsigned long long*)(w + L.esum);
  c->bpart = (double*)(w + L.part);
  c->bpart2 = (double*)(w + L.part2);
  c->bgram_part = (double*)(w + L.gpart);
  c->bgram_xtx = (double*)(w + L.xtx);
  c->bgram = (double*)(w + L.gram);
  // a multiple of 8: the sliced kernel places the chunk blocks of one row
  // block on one XCD
  c->brows = (int)std::min<int64_t>(kBatchRowBlocks, std::max<int64_t>(8, ((c->n_data + 63) / 64 + 7) / 8 * 8));
  c->bgram_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kGramBlocks, (c->n_mc + 255) / 256));
  // resonance table at theta (v = 0): frozen M, Gamma
  if (launch_table(d_theta, nullptr, c->md, c->K, c->tbl64, c->tbl32, c->itbl, c->status, st) != hipSuccess)
    return PWA_E_HIP;
  if (launch_freeze(fmt, c->planes64, c->stride, c->n_data, c->tbl64, c->itbl, c->K, L.KP,
                    c->md.gen, c->bA, c->besum, st) != hipSuccess)
    return PWA_E_HIP;
  if (launch_gram(c->planes64, c->stride, c->mc_off, c->n_mc, c->tbl64, c->itbl, c->K, c->md.gen,
                  c->bgram_blocks, c->bgram_part, c->bgram_xtx, c->bgram, st) != hipSuccess)
    return PWA_E_HIP;
  c->frozen = true;
  return PWA_OK;
}

int pwa_nll_batched(pwa_ctx* c, const double* d_C, int32_t B, double* d_nll, hipStream_t st) {
  if (!c || !d_C || !d_nll) return PWA_E_INVALID;
  if (!c->frozen) return PWA_E_STATE;
  if (B < 1 || B > c->bmax) return PWA_E_INVALID;
  BatchArgs a;
  for (int s = 0; s < kSlices; ++s) {
    a.A[s] = c->bA[s];
    a.C[s] = c->bC[s];
  }
  a.esum = c->besum;
  a.KP = c->bKP;
  a.B = B;
  a.n = c->n_data;
  a.part = c->bpart;
  a.part2 = c->bpart2;
  return launch_batched(c->bfmt, a, c->brows, d_C, c->bgram, c->K, (double)c->n_data,
                        (double)c->n_mc, d_nll, st) == hipSuccess
             ? PWA_OK
             : PWA_E_HIP;
}

int pwa_gram(pwa_ctx* c, double* d_gram, hipStream_t st) {
  if (!c || !d_gram) return PWA_E_INVALID;
  if (!c->frozen) return PWA_E_STATE;
  return hipMemcpyAsync(d_gram, c->bgram, sizeof(double) * 2 * c->K * c->K,
                        hipMemcpyDeviceToDevice, st) == hipSuccess
             ? PWA_OK
             : PWA_E_HIP;
}

// ---------------------------------------------------------------------------
// At the minimum: Hessian, covariance, fit fractions, error propagation.
// ---------------------------------------------------------------------------

// Scratch slots (the fit driver uses [0, 4P + 1)).
static double* unit_slot(pwa_ctx* c) { return c->scratch + 5 * c->P; }
static double* mask_slot(pwa_ctx* c) { return c->scratch + 6 * c->P; }

int pwa_hessian(pwa_ctx* c, const double* d_theta, double* d_H, hipStream_t st) {
  if (!c || !d_theta || !d_H) return PWA_E_INVALID;
  if (!c->bound) return PWA_E_STATE;
  const int P = c->P;
  double* d_e = unit_slot(c);
  c->hvp_cache = false;   // the first column is a full pass at d_theta
  for (int j = 0; j < P; ++j) {
    if (launch_unit(d_e, P, j, st) != hipSuccess) return PWA_E_HIP;
    const int r = run_eval(c, MODE_HVPB, OUT_COMBINED, c->precision, d_theta, d_e, nullptr,
                           nullptr, d_H + (size_t)j * P, nullptr, st);
    if (r != PWA_OK) return r;
  }
  c->hvp_cache = false;   // as documented: only pwa_hvp starts a reuse
  return launch_symmetrise(d_H, P, st) == hipSuccess ? PWA_OK : PWA_E_HIP;
}

int pwa_fit_fractions(pwa_ctx* c, const double* d_theta, double* d_ff, double* d_dff,
                      hipStream_t st) {
  if (!c || !d_theta || !d_ff) return PWA_E_INVALID;
  if (!c->bound) return PWA_E_STATE;
  const int K = c->K, P = c->P;
  double* d_m = mask_slot(c);
  for (int k = 0; k < K; ++k) {
    if (launch_mask(d_theta, d_m, K, k, st) != hipSuccess) return PWA_E_HIP;
    const int r = run_eval(c, MODE_GRAD, OUT_PARTIALS, c->precision, d_m, nullptr, nullptr,
                           nullptr, nullptr, c->dd, st, true);
    if (r != PWA_OK) return r;
    if (launch_ff_take(c->dd, P, k, d_ff, d_dff, st) != hipSuccess) return PWA_E_HIP;
  }
  const int r = run_eval(c, MODE_GRAD, OUT_PARTIALS, c->precision, d_theta, nullptr, nullptr,
                         nullptr, nullptr, c->dd, st, true);
  if (r != PWA_OK) return r;
  return launch_ff_finish(c->dd, K, P, d_ff, d_dff, st) == hipSuccess ? PWA_OK : PWA_E_HIP;
}

// Fraction matrix: MC Gram matrix at theta's masses and widths (the batched
// path's FP64 matrix-core Gram kernel), then the coupling contraction.
constexpr int kPhiGramBlocks = 1024;
constexpr int kPhiGP = 48;   // padded 2K of the Gram kernel (K <= 24)

size_t pwa_fraction_matrix_workspace_bytes(const pwa_ctx* c) {
  // the MC Gram matrix holds one amplitude row per event: spin-0 parent only
  if (!c || c->K > 24 || !(c->streams & PWA_STREAM_F64) || c->md.parent_spin != 0) return 0;
  return align_up(sizeof(double) * 2 * (size_t)kPhiGramBlocks * kPhiGP * kPhiGP, 256) +
         align_up(sizeof(double) * 2 * (size_t)c->K * c->K, 256) +
         align_up(sizeof(double) * (size_t)kPhiGP * kPhiGP, 256);
}

int pwa_fraction_matrix(pwa_ctx* c, const double* d_theta, void* d_ws, size_t ws_bytes,
                        double* d_phi, hipStream_t st) {
  if (!c || !d_theta || !d_phi) return PWA_E_INVALID;
  const size_t need = pwa_fraction_matrix_workspace_bytes(c);
  if (need == 0) return PWA_E_INVALID;
  if (!c->bound) return PWA_E_STATE;
  if (!d_ws || ((uintptr_t)d_ws % 256) != 0 || ws_bytes < need) return PWA_E_WORKSPACE;
  c->hvp_cache = false;
  double* part = (double*)d_ws;
  double* gram = (double*)((char*)d_ws +
                           align_up(sizeof(double) * 2 * (size_t)kPhiGramBlocks * kPhiGP * kPhiGP, 256));
  double* xtx = (double*)((char*)gram + align_up(sizeof(double) * 2 * (size_t)c->K * c->K, 256));
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kPhiGramBlocks, (c->n_mc + 255) / 256));
  if (launch_table(d_theta, nullptr, c->md, c->K, c->tbl64, c->tbl32, c->itbl, c->status, st) != hipSuccess)
    return PWA_E_HIP;
  if (launch_gram(c->planes64, c->stride, c->mc_off, c->n_mc, c->tbl64, c->itbl, c->K, c->md.gen,
                  blocks, part, xtx, gram, st) != hipSuccess)
    return PWA_E_HIP;
  return launch_phi(gram, d_theta, c->K, d_phi, st) == hipSuccess ? PWA_OK : PWA_E_HIP;
}

int pwa_covariance(int32_t P, const double* H, const uint8_t* free_mask, double* cov) {
  if (P < 1 || P > 4 * PWA_MAX_RES || !H || !cov) return PWA_E_INVALID;
  std::vector<int> idx;
  for (int i = 0; i < P; ++i)
    if (!free_mask || free_mask[i]) idx.push_back(i);
  for (int i = 0; i < P * P; ++i)
    if (!isfinite(H[i])) return PWA_E_INVALID;
  const int n = (int)idx.size();
  for (int i = 0; i < P * P; ++i) cov[i] = 0.0;
  if (n == 0) return PWA_OK;
  // Cholesky factor of the free block, A = L L^T (lower triangle of L).
  std::vector<double> L((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    const double hjj = H[(size_t)idx[j] * P + idx[j]];
    double d = hjj;
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    // A pivot at or below 1e-12 n H_jj is a direction that an FP64 Hessian
    // built from event sums does not resolve (its entries carry rounding far
    // above n eps), e.g. the coupling phase or scale left free: its inverse
    // would be rounding noise, so the block counts as singular.
    if (!(d > 1e-12 * n * fabs(hjj))) return PWA_E_DOMAIN;
    const double ljj = sqrt(d);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double a = 0.5 * (H[(size_t)idx[i] * P + idx[j]] + H[(size_t)idx[j] * P + idx[i]]);
      for (int k = 0; k < j; ++k) a -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = a / ljj;
    }
  }
  // A^{-1} column by column: solve L y = e_j, then L^T x = y.
  std::vector<double> y(n), x(n);
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) {
      double a = (i == j) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) a -= L[(size_t)i * n + k] * y[k];
      y[i] = a / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double a = y[i];
      for (int k = i + 1; k < n; ++k) a -= L[(size_t)k * n + i] * x[k];
      x[i] = a / L[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) cov[(size_t)idx[i] * P + idx[j]] = x[i];
  }
  // exact symmetry (the two triangular solves round differently)
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const size_t a = (size_t)idx[i] * P + idx[j], b = (size_t)idx[j] * P + idx[i];
      const double m = 0.5 * (cov[a] + cov[b]);
      cov[a] = cov[b] = m;
    }
  return PWA_OK;
}

int pwa_propagate(int32_t P, int32_t n, const double* J, const double* cov, double* sigma) {
  if (P < 1 || n < 0 || (n > 0 && (!J || !cov || !sigma))) return PWA_E_INVALID;
  for (int r = 0; r < n; ++r) {
    const double* g = J + (size_t)r * P;
    double q = 0.0;
    for (int i = 0; i < P; ++i) {
      double a = 0.0;
      for (int j = 0; j < P; ++j) a += cov[(size_t)i * P + j] * g[j];
      q += g[i] * a;
    }
    sigma[r] = q >= 0.0 ? sqrt(q) : NAN;
  }
  return PWA_OK;
}

}  // extern "C"
