// C-ABI of the source-to-waveform library: plan, memory binding, setup and the
// forward/adjoint entry points.  Host code only; kernels live in the *.hip files.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/s2w.h"
#include "s2w_internal.h"

using namespace s2w;

namespace {

constexpr uint64_t kAlign = 256;
constexpr int kMaxWgPerCu = 4;
constexpr int kMaxSplits = 64;

inline uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }
inline int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}
inline int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Channel splits of a direct-path product with `tiles` row tiles: the count (at most smax and
// the channel count) that fills the `slots` concurrent workgroups in the most even rounds.
int direct_splits(int64_t tiles, int nchan, int slots, int smax) {
  smax = std::max(1, std::min(smax, nchan));
  int best = 1;
  double beff = -1.0;
  for (int S = 1; S <= smax; ++S) {
    const int64_t w = tiles * S;
    const int64_t rounds = (w + slots - 1) / slots;
    const double eff = (double)w / (double)(rounds * slots);
    if (eff > beff + 1e-9) {
      beff = eff;
      best = S;
    }
  }
  return best;
}

// Offsets of the regions carved out of the bound memory.
struct Layout {
  // operator store (float32 path)
  uint64_t gh, fh;
  // operator store (half-precision path)
  uint64_t gq, sg, fq, sf;
  uint64_t op_total;
  // workspace (float32 single-rupture path)
  uint64_t sh, part, yh, rh, wp, part2, gsh;
  // workspace (batched half-precision path)
  uint64_t staging, S, sig_up, sig_down, bop, U, tau_up, tau_down, part_f, yhb;
  // operator store and workspace (batched float32 path)
  uint64_t gs, fs;
  uint64_t s32, u32, part32, yh32;
  // operator store and workspace (direct time-domain path)
  uint64_t gt, ft;
  uint64_t dpart, dv, dout;
  uint64_t ws_total;
};

// Extra geometry of the direct time-domain path.
struct DirectGeo {
  bool on = false;
  int ntp;                    // nt rounded up to 16 (zero lags at the end of every stored series)
  int s_g, s_f;               // forward channel splits: elastic (over subfaults), acoustic (over grid rows)
  int s_fa, s_ga;             // adjoint channel splits: acoustic (over observers), elastic (over grid rows)
};

// Extra geometry of the batched float32 path.
struct BatchGeo32 {
  bool on = false;
  int nsk, nok, ngk;          // subfaults padded to 8, observers to 16, grid rows to 8 (zeros)
  int bp;                     // max_batch padded to a multiple of 8
  int splits_f_max = 16;      // acoustic GEMM grid-row splits
  int splits_a_max = 8;       // transposed elastic GEMM grid-row splits
};

// Type of the activation terms for product type kt (bf16 words converted to f16 meet f16 terms).
static inline int act_type(int kt) { return kt == 3 ? 2 : kt; }

// Extra geometry of the batched half-precision path.
struct HalfGeo {
  bool on = false;
  int ht_g = 1, ht_f = 1;     // stored words: 1 = bf16, 2 = f16
  int kt_g = 1, kt_f = 1;     // products: 1 = bf16, 2 = f16, 3 = bf16 words converted to f16
  int hterms_g = 2, hterms_f = 2;
  int nsq, noq, ngq, nks;     // padded subfaults (x16), observers (16 * 2^k), grid rows (x16); K steps
  int bp;                     // max_batch padded to a multiple of 8
  int splits_max;
  int rs;                     // setup rows per staging pass
};

}  // namespace

struct s2w_plan {
  s2w_desc desc;
  int device;
  int ncu;
  Geometry geo;
  HalfGeo hg;
  BatchGeo32 fb;
  DirectGeo dg;
  Layout lay;
  s2w_tuning tune;
  char* op = nullptr;
  char* ws = nullptr;
  uint64_t op_bytes = 0, ws_bytes = 0;
  std::vector<uint8_t> row_set;  // one flag per grid row set since the last bind
  bool pad_zeroed = false;       // half path: padding columns of the acoustic store cleared
  int64_t rows_missing = 0;
  std::string err;
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
};

namespace {

s2w_status fail(s2w_plan* p, s2w_status st, const char* fmt, ...) {
  if (p) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    p->err = buf;
  }
  return st;
}

s2w_status hip_fail(s2w_plan* p, hipError_t e, const char* what) {
  return fail(p, S2W_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void* ptr) { return ((uintptr_t)ptr % kAlign) == 0; }

std::mutex g_tw_mutex;
std::vector<int> g_tw_done;

hipError_t ensure_twiddles(int device) {
  std::lock_guard<std::mutex> lk(g_tw_mutex);
  if ((int)g_tw_done.size() <= device) g_tw_done.resize(device + 1, 0);
  if (g_tw_done[device]) return hipSuccess;
  hipError_t e = upload_twiddles(device);
  if (e == hipSuccess) g_tw_done[device] = 1;
  return e;
}

// Fixed device scratch of s2w_forward_noalloc, for callers that cannot allocate.  Each GPU
// the library runs on holds its own copy until the process ends.  In host code the array's
// name is only a stand-in: its device address, per device, comes from hipGetSymbolAddress
// at plan creation and is the only handle host code passes on.
static __device__ __align__(256) unsigned char scratch[S2W_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mutex;
std::vector<void*> g_scratch_ptr;       // per device; nullptr until looked up
std::vector<hipError_t> g_scratch_err;  // per device: result of the lookup

// With `device` current: look up this device's copy of the scratch array (once).
void ensure_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  if ((int)g_scratch_ptr.size() <= device) {
    g_scratch_ptr.resize(device + 1, nullptr);
    g_scratch_err.resize(device + 1, hipErrorNotReady);
  }
  if (g_scratch_ptr[device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_scratch_err[device] = e;
  if (e == hipSuccess && ptr && ((uintptr_t)ptr % kAlign) == 0) g_scratch_ptr[device] = ptr;
}

// This device's scratch address, or nullptr with the lookup's error in *err.
void* scratch_ptr(int device, hipError_t* err) {
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  if (device < 0 || device >= (int)g_scratch_ptr.size()) {
    *err = hipErrorNotReady;
    return nullptr;
  }
  *err = g_scratch_err[device];
  return g_scratch_ptr[device];
}

// Scoped switch to the plan's device.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

Layout make_layout(const s2w_desc& d, const Geometry& g, const HalfGeo& h, const BatchGeo32& f,
                   const DirectGeo& dg, int ncu) {
  Layout L{};
  const uint64_t c8 = sizeof(float2);
  uint64_t off = 0;
  if (dg.on) {
    const uint64_t ntp = (uint64_t)dg.ntp, f4 = 4;
    L.gt = off;
    off = round_up(off + (uint64_t)g.ngrid * g.nsub * ntp * f4, kAlign);
    L.ft = off;
    off = round_up(off + (uint64_t)g.ngrid * g.nobs * ntp * f4, kAlign);
    L.op_total = off;
    off = 0;
    L.dpart = off;  // grid-row partials of the first product (either direction)
    off = round_up(off + (uint64_t)std::max(dg.s_g, dg.s_fa) * g.ngrid * ntp * f4, kAlign);
    L.dv = off;     // the differenced seafloor field between the products
    off = round_up(off + (uint64_t)g.ngrid * ntp * f4, kAlign);
    L.dout = off;   // partials of the second product
    off = round_up(off + (uint64_t)std::max((uint64_t)dg.s_f * g.nobs, (uint64_t)dg.s_ga * g.nsub) * ntp * f4,
                   kAlign);
    L.ws_total = off;
    return L;
  }
  if (f.on) {
    const uint64_t bp = (uint64_t)f.bp;
    L.gs = off;
    off = round_up(off + (uint64_t)g.ngrid * g.M * f.nsk * c8, kAlign);
    L.fs = off;
    off = round_up(off + (uint64_t)g.M * f.nok * f.ngk * c8, kAlign);
    L.op_total = off;
    off = 0;
    L.s32 = off;
    off = round_up(off + (uint64_t)g.M * std::max(f.nsk, f.nok) * bp * c8, kAlign);
    L.u32 = off;
    off = round_up(off + (uint64_t)g.ngrid * g.M * bp * c8, kAlign);
    L.part32 = off;
    const uint64_t prow = std::max((uint64_t)f.splits_f_max * f.nok, (uint64_t)f.splits_a_max * f.nsk);
    off = round_up(off + prow * g.M * 2 * bp * 4, kAlign);
    L.yh32 = off;
    off = round_up(off + bp * std::max(g.nobs, g.nsub) * g.M * c8, kAlign);
    L.ws_total = off;
    return L;
  }
  if (!h.on) {
    L.gh = off;
    off = round_up(off + (uint64_t)g.ngrid * g.M * g.nsp * c8, kAlign);
    L.fh = off;
    off = round_up(off + (uint64_t)g.ngrid * g.M * g.nop * c8, kAlign);
  } else {
    L.gq = off;  // row-block-major, grid rows padded to a multiple of 16
    off = round_up(off + (uint64_t)h.ngq * g.M * h.nsq * 4, kAlign);
    L.sg = off;
    off = round_up(off + (uint64_t)g.ngrid * g.M * 4, kAlign);
    L.fq = off;
    off = round_up(off + (uint64_t)g.M * h.noq * h.ngq * 4, kAlign);
    L.sf = off;
    off = round_up(off + (uint64_t)g.ngrid * g.M * 4, kAlign);
  }
  L.op_total = off;

  off = 0;
  if (!h.on) {
    const int nwg_max = ncu * kMaxWgPerCu;
    L.sh = off;
    off = round_up(off + (uint64_t)g.M * g.nsp * c8, kAlign);
    L.part = off;
    const uint64_t part_fwd = (uint64_t)nwg_max * g.M * g.nop * c8;  // [nwg][nop][M]
    const uint64_t part_split = (uint64_t)kMaxSplits * g.M * std::max(g.nsp, g.nop) * c8;
    off = round_up(off + std::max(part_fwd, part_split), kAlign);
    L.yh = off;
    off = round_up(off + (uint64_t)std::max(g.nop, g.nsp) * g.M * c8, kAlign);
    L.rh = off;
    off = round_up(off + (uint64_t)g.M * g.nop * c8, kAlign);
    L.wp = off;
    off = round_up(off + (uint64_t)g.ngrid * g.M * c8, kAlign);
    L.part2 = L.part;  // the adjoint reuses the partial region
    L.gsh = L.yh;
  } else {
    const uint64_t bp = (uint64_t)h.bp;
    const uint64_t ncb = bp / 8;
    L.staging = off;
    off = round_up(off + (uint64_t)h.rs * g.M * std::max(h.nsq, h.noq) * c8, kAlign);
    L.S = off;
    off = round_up(off + (uint64_t)g.M * h.nsq * bp * c8, kAlign);
    L.sig_up = off;
    off = round_up(off + (uint64_t)g.M * bp * 4, kAlign);
    L.sig_down = off;
    off = round_up(off + (uint64_t)g.M * bp * 4, kAlign);
    L.bop = off;
    off = round_up(off + (uint64_t)g.M * h.nks * ncb * h.hterms_g * 1024, kAlign);
    L.U = off;
    off = round_up(off + (uint64_t)g.M * g.ngrid * bp * c8, kAlign);
    L.tau_up = off;
    off = round_up(off + (uint64_t)g.M * bp * 4, kAlign);
    L.tau_down = off;
    off = round_up(off + (uint64_t)g.M * bp * 4, kAlign);
    L.part_f = off;  // acoustic partials; the adjoint's residual spectra and elastic partials
    off = round_up(off + (uint64_t)std::max(h.splits_max * h.noq, h.nsq) * g.M * 2 * bp * 4, kAlign);
    L.yhb = off;
    off = round_up(off + bp * g.nobs * g.M * c8, kAlign);
  }
  L.ws_total = off;
  (void)d;
  return L;
}

}  // namespace

extern "C" {

int32_t s2w_abi_version(void) { return S2W_ABI_VERSION; }

const char* s2w_status_string(s2w_status st) {
  switch (st) {
    case S2W_OK: return "ok";
    case S2W_EINVAL: return "invalid argument";
    case S2W_ENOMEM: return "bound memory too small";
    case S2W_ESTATE: return "call out of order";
    case S2W_EUNSUPPORTED: return "unsupported";
    case S2W_EHIP: return "HIP error";
  }
  return "unknown status";
}

const char* s2w_last_error(const s2w_plan* plan) { return plan ? plan->err.c_str() : ""; }

s2w_status s2w_plan_create(const s2w_desc* desc, int32_t device, s2w_plan** out) {
  if (!out) return S2W_EINVAL;
  *out = nullptr;
  if (!desc) return S2W_EINVAL;
  const s2w_desc& d = *desc;
  if (d.nsub < 1 || d.nsub > 1024 || d.nobs < 1 || d.nobs > 256 || d.nt < 1 || d.nt > 512 || d.ngrid < 1 ||
      d.max_batch < 0 || d.max_batch > 1024 || !(d.dt > 0.0) || (d.diff != S2W_DIFF_NONE && d.diff != S2W_DIFF_BACKWARD))
    return S2W_EINVAL;
  if (d.g_dtype < S2W_F32 || d.g_dtype > S2W_F16 || d.f_dtype < S2W_F32 || d.f_dtype > S2W_F16) return S2W_EINVAL;
  const bool half = d.g_dtype != S2W_F32 || d.f_dtype != S2W_F32;
  if (half && (d.g_dtype == S2W_F32 || d.f_dtype == S2W_F32)) return S2W_EUNSUPPORTED;
  if (d.layout < S2W_LAYOUT_AUTO || d.layout > S2W_LAYOUT_DIRECT) return S2W_EINVAL;
  if (d.products < S2W_PRODUCTS_AUTO || d.products > S2W_PRODUCTS_F16 || (!half && d.products != S2W_PRODUCTS_AUTO))
    return S2W_EINVAL;
  if (half && (d.layout == S2W_LAYOUT_SINGLE || d.layout == S2W_LAYOUT_DIRECT)) return S2W_EUNSUPPORTED;
  const bool batched32 =
      !half && (d.layout == S2W_LAYOUT_BATCHED || (d.layout == S2W_LAYOUT_AUTO && d.max_batch >= 8));
  const bool direct = d.layout == S2W_LAYOUT_DIRECT;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return S2W_EINVAL;

  s2w_plan* p = new (std::nothrow) s2w_plan();
  if (!p) return S2W_ENOMEM;
  p->desc = d;
  p->device = device;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || ncu <= 0) ncu = 256;
  p->ncu = ncu;
  Geometry& g = p->geo;
  g.nsub = d.nsub;
  g.ngrid = d.ngrid;
  g.nobs = d.nobs;
  g.nt = d.nt;
  g.L = std::max(32, next_pow2(2 * d.nt - 1));
  g.M = g.L / 2;
  g.logM = ilog2(g.M);
  g.nsp = (d.nsub + 1) / 2 * 2;
  g.nop = (d.nobs + 1) / 2 * 2;
  g.nsp4 = g.nsp / 2;
  g.nop4 = g.nop / 2;
  g.diff = d.diff;
  g.dt = (float)d.dt;
  HalfGeo& h = p->hg;
  if (half) {
    h.on = true;
    h.ht_g = d.g_dtype == S2W_BF16 ? 1 : 2;
    h.ht_f = d.f_dtype == S2W_BF16 ? 1 : 2;
    // products: bfloat16 words either meet bfloat16 activations split into a high and a low
    // term (two products each), or are converted to float16 in registers and meet one scaled
    // f16 term, as float16 words always do (its rounding is then of the operator's own order)
    const bool f16_products = d.products != S2W_PRODUCTS_BF16;
    h.kt_g = h.ht_g == 2 ? 2 : (f16_products ? 3 : 1);
    h.kt_f = h.ht_f == 2 ? 2 : (f16_products ? 3 : 1);
    h.hterms_g = h.kt_g == 1 ? 2 : 1;
    h.hterms_f = h.kt_f == 1 ? 2 : 1;
    h.nsq = (d.nsub + 15) / 16 * 16;
    h.noq = 16 * next_pow2((d.nobs + 15) / 16);
    h.ngq = (d.ngrid + 15) / 16 * 16;
    h.nks = h.nsq / 16;
    h.bp = (std::max(d.max_batch, 1) + 7) / 8 * 8;
    h.splits_max = 16;
    h.rs = 16;
  }
  if (batched32) {
    BatchGeo32& f = p->fb;
    f.on = true;
    f.nsk = (d.nsub + 7) / 8 * 8;
    f.nok = (d.nobs + 15) / 16 * 16;
    f.ngk = (d.ngrid + 7) / 8 * 8;
    f.bp = (std::max(d.max_batch, 1) + 7) / 8 * 8;
  }
  if (direct) {
    DirectGeo& dd = p->dg;
    dd.on = true;
    dd.ntp = (d.nt + 15) / 16 * 16;
    const int nranges = (dd.ntp / 16 + 15) / 16;
    const int slots = 2 * ncu;  // two workgroups of four waves per compute unit
    auto tiles = [&](int rows, int rw) { return (int64_t)((rows + 64 * rw - 1) / (64 * rw)) * nranges; };
    dd.s_g = direct_splits(tiles(d.ngrid, 2), d.nsub, slots, 16);
    dd.s_f = direct_splits(tiles(d.nobs, 1), d.ngrid, slots, 1024);
    dd.s_fa = direct_splits(tiles(d.ngrid, 2), d.nobs, slots, 16);
    dd.s_ga = direct_splits(tiles(d.nsub, 2), d.ngrid, slots, 1024);
  }
  p->lay = make_layout(d, g, h, p->fb, p->dg, ncu);
  p->tune.fused_wg_per_cu = 1;
  p->tune.fused_rows = 8;
  p->tune.adj_cols = 16;
  p->tune.adj_splits = 16;
  p->tune.batch_path_min_b = 0;
  p->tune.gemm_cfg = -1;
  p->tune.fgemm_splits = 0;
  p->tune.fgemm_lds = 1;
  p->tune.gemm32_cfg = -1;
  p->tune.gemm32_cfg_k = -1;
  p->tune.gemm32_splits = 0;
  p->tune.adj32_splits = 0;
  p->tune.hadj_tile_f = -1;
  p->tune.hadj_tile_g = -1;
  p->tune.mid_rupts = 16;
  p->tune.adj32_cfg = -1;
  p->row_set.assign((size_t)d.ngrid, 0);
  p->rows_missing = d.ngrid;
  {
    DeviceGuard dg(device);
    if (!dg.ok) {
      delete p;
      return S2W_EHIP;
    }
    if (ensure_twiddles(device) != hipSuccess) {
      delete p;
      return S2W_EHIP;
    }
    ensure_scratch(device);  // a failed lookup only disables s2w_forward_noalloc, which reports it
  }
  *out = p;
  return S2W_OK;
}

s2w_status s2w_plan_destroy(s2w_plan* plan) {
  delete plan;
  return S2W_OK;
}

s2w_status s2w_query_sizes(const s2w_plan* p, uint64_t* operator_bytes, uint64_t* workspace_bytes) {
  if (!p) return S2W_EINVAL;
  if (operator_bytes) *operator_bytes = p->lay.op_total;
  if (workspace_bytes) *workspace_bytes = p->lay.ws_total;
  return S2W_OK;
}

s2w_status s2w_plan_layout(const s2w_plan* p, int32_t* layout) {
  if (!p || !layout) return S2W_EINVAL;
  *layout = p->dg.on ? S2W_LAYOUT_DIRECT : (p->hg.on || p->fb.on) ? S2W_LAYOUT_BATCHED : S2W_LAYOUT_SINGLE;
  return S2W_OK;
}

s2w_status s2w_transform_length(const s2w_plan* p, int32_t* L) {
  if (!p || !L) return S2W_EINVAL;
  *L = p->geo.L;
  return S2W_OK;
}

s2w_status s2w_bind_memory(s2w_plan* p, void* operator_store, uint64_t operator_bytes, void* workspace,
                           uint64_t workspace_bytes) {
  if (!p) return S2W_EINVAL;
  if (!operator_store || !workspace) return fail(p, S2W_EINVAL, "bind: null pointer");
  if (!aligned(operator_store) || !aligned(workspace)) return fail(p, S2W_EINVAL, "bind: pointers must be 256-byte aligned");
  if (operator_bytes < p->lay.op_total)
    return fail(p, S2W_ENOMEM, "bind: operator store %llu bytes < required %llu", (unsigned long long)operator_bytes,
                (unsigned long long)p->lay.op_total);
  if (workspace_bytes < p->lay.ws_total)
    return fail(p, S2W_ENOMEM, "bind: workspace %llu bytes < required %llu", (unsigned long long)workspace_bytes,
                (unsigned long long)p->lay.ws_total);
  p->op = (char*)operator_store;
  p->ws = (char*)workspace;
  p->op_bytes = operator_bytes;
  p->ws_bytes = workspace_bytes;
  std::fill(p->row_set.begin(), p->row_set.end(), 0);
  p->rows_missing = p->desc.ngrid;
  p->pad_zeroed = false;
  return S2W_OK;
}

s2w_status s2w_set_profile_events(s2w_plan* p, void* begin, void* end) {
  if (!p) return S2W_EINVAL;
  if ((begin == nullptr) != (end == nullptr)) return fail(p, S2W_EINVAL, "profile events: pass both or neither");
  p->ev_begin = (hipEvent_t)begin;
  p->ev_end = (hipEvent_t)end;
  return S2W_OK;
}

static hipError_t mark(hipEvent_t ev, hipStream_t st) { return ev ? hipEventRecord(ev, st) : hipSuccess; }

s2w_status s2w_set_tuning(s2w_plan* p, const s2w_tuning* t) {
  if (!p || !t) return S2W_EINVAL;
  s2w_tuning n = p->tune;
  if (t->fused_wg_per_cu) {
    if (t->fused_wg_per_cu < 1 || t->fused_wg_per_cu > kMaxWgPerCu) return fail(p, S2W_EINVAL, "tuning: fused_wg_per_cu");
    n.fused_wg_per_cu = t->fused_wg_per_cu;
  }
  if (t->fused_rows) {
    if (t->fused_rows != 4 && t->fused_rows != 8) return fail(p, S2W_EINVAL, "tuning: fused_rows must be 4 or 8");
    n.fused_rows = t->fused_rows;
  }
  if (t->adj_cols) {
    if (t->adj_cols != 8 && t->adj_cols != 16) return fail(p, S2W_EINVAL, "tuning: adj_cols must be 8 or 16");
    n.adj_cols = t->adj_cols;
  }
  if (t->adj_splits) {
    if (t->adj_splits < 1 || t->adj_splits > kMaxSplits) return fail(p, S2W_EINVAL, "tuning: adj_splits");
    n.adj_splits = t->adj_splits;
  }
  if (t->gemm_cfg) {
    const int c = t->gemm_cfg;
    if (!(c == -1 || c == 4 || c == 10 || c == 12 || (c >= 16 && c <= 18) || c == 24))
      return fail(p, S2W_EINVAL, "tuning: gemm_cfg must be -1, 4, 10, 12, 16, 17, 18 or 24");
    n.gemm_cfg = t->gemm_cfg == 4 ? 0 : t->gemm_cfg;
  }
  if (t->fgemm_lds) {
    if (t->fgemm_lds < 1 || t->fgemm_lds > 4) return fail(p, S2W_EINVAL, "tuning: fgemm_lds must be 1..4");
    n.fgemm_lds = t->fgemm_lds;
  }
  if (t->gemm32_cfg) {
    if (t->gemm32_cfg < -1 || t->gemm32_cfg > 4) return fail(p, S2W_EINVAL, "tuning: gemm32_cfg");
    n.gemm32_cfg = t->gemm32_cfg < 0 ? -1 : t->gemm32_cfg - 1;
  }
  if (t->gemm32_cfg_k) {
    if (t->gemm32_cfg_k < -1 || t->gemm32_cfg_k > 4) return fail(p, S2W_EINVAL, "tuning: gemm32_cfg_k");
    n.gemm32_cfg_k = t->gemm32_cfg_k < 0 ? -1 : t->gemm32_cfg_k - 1;
  }
  if (t->gemm32_splits) {
    if (t->gemm32_splits < 0 || t->gemm32_splits > 16) return fail(p, S2W_EINVAL, "tuning: gemm32_splits");
    n.gemm32_splits = t->gemm32_splits;
  }
  if (t->adj32_splits) {
    if (t->adj32_splits < 0 || t->adj32_splits > 8) return fail(p, S2W_EINVAL, "tuning: adj32_splits");
    n.adj32_splits = t->adj32_splits;
  }
  if (t->fgemm_splits) {
    if (t->fgemm_splits < 0 || t->fgemm_splits > 16) return fail(p, S2W_EINVAL, "tuning: fgemm_splits");
    n.fgemm_splits = t->fgemm_splits;
  }
  if (t->hadj_tile_f) {
    const int c = t->hadj_tile_f;
    if (!(c == -1 || c == 3 || c == 4 || (c >= 6 && c <= 8)))
      return fail(p, S2W_EINVAL, "tuning: hadj_tile_f must be -1, 3, 4, 6, 7 or 8");
    n.hadj_tile_f = t->hadj_tile_f < 0 ? -1 : t->hadj_tile_f - 1;
  }
  if (t->adj32_cfg) {
    if (t->adj32_cfg < -1 || t->adj32_cfg > 4) return fail(p, S2W_EINVAL, "tuning: adj32_cfg");
    n.adj32_cfg = t->adj32_cfg < 0 ? -1 : t->adj32_cfg - 1;
  }
  if (t->mid_rupts) {
    if (t->mid_rupts != 16 && t->mid_rupts != 32) return fail(p, S2W_EINVAL, "tuning: mid_rupts must be 16 or 32");
    n.mid_rupts = t->mid_rupts;
  }
  if (t->hadj_tile_g) {
    const int c = t->hadj_tile_g;
    if (!(c == -1 || c == 3 || c == 4 || (c >= 6 && c <= 8)))
      return fail(p, S2W_EINVAL, "tuning: hadj_tile_g must be -1, 3, 4, 6, 7 or 8");
    n.hadj_tile_g = t->hadj_tile_g < 0 ? -1 : t->hadj_tile_g - 1;
  }
  p->tune = n;
  return S2W_OK;
}

s2w_status s2w_get_tuning(const s2w_plan* p, s2w_tuning* t) {
  if (!p || !t) return S2W_EINVAL;
  *t = p->tune;
  // internal codes back to the public ones, so that get -> set round-trips
  t->gemm_cfg = p->tune.gemm_cfg == 0 ? 4 : p->tune.gemm_cfg;
  t->batch_path_min_b = 0;
  t->gemm32_cfg = p->tune.gemm32_cfg < 0 ? -1 : p->tune.gemm32_cfg + 1;
  t->gemm32_cfg_k = p->tune.gemm32_cfg_k < 0 ? -1 : p->tune.gemm32_cfg_k + 1;
  t->adj32_cfg = p->tune.adj32_cfg < 0 ? -1 : p->tune.adj32_cfg + 1;
  t->hadj_tile_f = p->tune.hadj_tile_f < 0 ? -1 : p->tune.hadj_tile_f + 1;
  t->hadj_tile_g = p->tune.hadj_tile_g < 0 ? -1 : p->tune.hadj_tile_g + 1;
  return S2W_OK;
}

// Half-precision setup: per staging pass of rs rows, transform to float32 spectra in the
// workspace, then quantize with one power-of-two scale per (grid row, bin).
static s2w_status set_operators_half(s2w_plan* p, const float* G_chunk, const float* F_chunk, int64_t row0,
                                     int64_t nrows, hipStream_t st) {
  const Geometry& g = p->geo;
  const HalfGeo& h = p->hg;
  float2* stg = (float2*)(p->ws + p->lay.staging);
  uint32_t* Gq = (uint32_t*)(p->op + p->lay.gq);
  uint32_t* Fq = (uint32_t*)(p->op + p->lay.fq);
  float* sG = (float*)(p->op + p->lay.sg);
  float* sF = (float*)(p->op + p->lay.sf);
  hipError_t e = hipSuccess;
  if (!p->pad_zeroed) {
    e = launch_zero_strided(Fq + g.ngrid, (int64_t)g.M * h.noq, h.ngq, h.ngq - g.ngrid, st);
    if (e != hipSuccess) return hip_fail(p, e, "set_operators: clear padding");
    p->pad_zeroed = true;
  }
  for (int64_t r = 0; r < nrows; r += h.rs) {
    const int64_t n = std::min<int64_t>(h.rs, nrows - r);
    e = launch_rfft_rows(G_chunk + r * g.nsub * g.nt, n, g.nsub, h.nsq, stg, (int64_t)g.M * h.nsq, 1, h.nsq, g, 1.0f,
                         st);
    if (e == hipSuccess)
      e = launch_quant_rows(h.ht_g, stg, n, g.M, g.nsub, h.nsq, Gq, row0 + r, 0, 0, 0, sG, h.ngq / 16, st);
    if (e != hipSuccess) return hip_fail(p, e, "set_operators: elastic transform/quantize");
    e = launch_rfft_rows(F_chunk + r * g.nobs * g.nt, n, g.nobs, h.noq, stg, (int64_t)g.M * h.noq, 1, h.noq, g, 1.0f,
                         st);
    if (e == hipSuccess)
      e = launch_quant_rows(h.ht_f, stg, n, g.M, g.nobs, h.noq, Fq, row0 + r, 1, (int64_t)h.noq * h.ngq, h.ngq, sF,
                            0, st);
    if (e != hipSuccess) return hip_fail(p, e, "set_operators: acoustic transform/quantize");
  }
  return S2W_OK;
}

// Batched float32 setup: the row transforms write the GEMM layouts directly,
// Gs[g][l][j] (padded subfaults zero) and Fs[l][o][g] (padded observers zero).
static s2w_status set_operators_b32(s2w_plan* p, const float* G_chunk, const float* F_chunk, int64_t row0,
                                    int64_t nrows, hipStream_t st) {
  const Geometry& g = p->geo;
  const BatchGeo32& f = p->fb;
  float2* Gs = (float2*)(p->op + p->lay.gs);
  float2* Fs = (float2*)(p->op + p->lay.fs);
  hipError_t e = hipSuccess;
  if (!p->pad_zeroed) {
    // grid-row padding columns of the acoustic store, as 32-bit words
    e = launch_zero_strided((uint32_t*)(Fs + g.ngrid), (int64_t)g.M * f.nok, 2 * (int64_t)f.ngk,
                            2 * (f.ngk - g.ngrid), st);
    if (e != hipSuccess) return hip_fail(p, e, "set_operators: clear padding");
    p->pad_zeroed = true;
  }
  e = launch_rfft_rows(G_chunk, nrows, g.nsub, f.nsk, Gs + row0 * g.M * f.nsk, (int64_t)g.M * f.nsk, 1, f.nsk, g,
                       1.0f, st);
  if (e != hipSuccess) return hip_fail(p, e, "set_operators: elastic transform");
  e = launch_rfft_rows(F_chunk, nrows, g.nobs, f.nok, Fs + row0, 1, f.ngk, (int64_t)f.nok * f.ngk, g, 1.0f, st);
  if (e != hipSuccess) return hip_fail(p, e, "set_operators: acoustic transform");
  return S2W_OK;
}

// Direct setup: the time-domain blocks are kept as given, each series padded with zero lags
// to a multiple of 16: Gt[g][j][k], Ft[g][o][k].
static s2w_status set_operators_direct(s2w_plan* p, const float* G_chunk, const float* F_chunk, int64_t row0,
                                       int64_t nrows, hipStream_t st) {
  const Geometry& g = p->geo;
  const int ntp = p->dg.ntp;
  float* Gt = (float*)(p->op + p->lay.gt) + row0 * g.nsub * ntp;
  float* Ft = (float*)(p->op + p->lay.ft) + row0 * g.nobs * ntp;
  hipError_t e = launch_pad_series(G_chunk, nrows * g.nsub, g.nt, ntp, Gt, st);
  if (e == hipSuccess) e = launch_pad_series(F_chunk, nrows * g.nobs, g.nt, ntp, Ft, st);
  if (e != hipSuccess) return hip_fail(p, e, "set_operators: time-domain store");
  return S2W_OK;
}

s2w_status s2w_set_operators(s2w_plan* p, const float* G_chunk, const float* F_chunk, int64_t row0, int64_t nrows,
                             void* stream) {
  if (!p) return S2W_EINVAL;
  if (!p->op) return fail(p, S2W_ESTATE, "set_operators: memory not bound");
  if (!G_chunk || !F_chunk) return fail(p, S2W_EINVAL, "set_operators: null chunk pointer");
  if (!aligned(G_chunk) || !aligned(F_chunk)) return fail(p, S2W_EINVAL, "set_operators: chunk pointers must be 256-byte aligned");
  if (row0 < 0 || nrows < 0 || row0 + nrows > p->desc.ngrid)
    return fail(p, S2W_EINVAL, "set_operators: rows [%lld, %lld) outside [0, %d)", (long long)row0,
                (long long)(row0 + nrows), p->desc.ngrid);
  if (nrows == 0) return S2W_OK;
  const Geometry& g = p->geo;
  DeviceGuard dg(p->device);
  if (!dg.ok) return fail(p, S2W_EHIP, "set_operators: cannot select device %d", p->device);
  hipStream_t st = (hipStream_t)stream;
  if (p->fb.on || p->hg.on || p->dg.on) {
    s2w_status hs = p->dg.on   ? set_operators_direct(p, G_chunk, F_chunk, row0, nrows, st)
                    : p->fb.on ? set_operators_b32(p, G_chunk, F_chunk, row0, nrows, st)
                               : set_operators_half(p, G_chunk, F_chunk, row0, nrows, st);
    if (hs != S2W_OK) return hs;
    for (int64_t r = row0; r < row0 + nrows; ++r) {
      if (!p->row_set[(size_t)r]) {
        p->row_set[(size_t)r] = 1;
        --p->rows_missing;
      }
    }
    return S2W_OK;
  }
  float2* Gh = (float2*)(p->op + p->lay.gh);
  float2* Fh = (float2*)(p->op + p->lay.fh);
  // spectra of row (g, column c) land at [g][c][0..M)
  hipError_t e = launch_rfft_rows(G_chunk, nrows, g.nsub, g.nsp, Gh + row0 * g.M * g.nsp, (int64_t)g.M * g.nsp, g.M,
                                  1, g, 1.0f, st);
  if (e != hipSuccess) return hip_fail(p, e, "set_operators: elastic transform");
  e = launch_rfft_rows(F_chunk, nrows, g.nobs, g.nop, Fh + row0 * g.M * g.nop, (int64_t)g.M * g.nop, g.M, 1, g,
                       1.0f, st);
  if (e != hipSuccess) return hip_fail(p, e, "set_operators: acoustic transform");
  for (int64_t r = row0; r < row0 + nrows; ++r) {
    if (!p->row_set[(size_t)r]) {
      p->row_set[(size_t)r] = 1;
      --p->rows_missing;
    }
  }
  return S2W_OK;
}

static s2w_status check_call(s2w_plan* p, const void* in, int32_t B, const void* out, const char* who) {
  if (!p) return S2W_EINVAL;
  if (B < 0 || B > p->desc.max_batch) return fail(p, S2W_EINVAL, "%s: B=%d outside [0, %d]", who, B, p->desc.max_batch);
  if (B == 0) return S2W_OK;
  if (!in || !out) return fail(p, S2W_EINVAL, "%s: null pointer", who);
  if (!aligned(in) || !aligned(out)) return fail(p, S2W_EINVAL, "%s: pointers must be 256-byte aligned", who);
  if (in == out) return fail(p, S2W_EINVAL, "%s: input and output must be distinct", who);
  if (!p->op) return fail(p, S2W_ESTATE, "%s: memory not bound", who);
  if (p->rows_missing > 0)
    return fail(p, S2W_ESTATE, "%s: %lld grid rows have no operators yet", who, (long long)p->rows_missing);
  return S2W_OK;
}

// Floats of the half path's partial region (acoustic partials; scratch of the column scales).
static int64_t part_floats(const s2w_plan* p) {
  return (int64_t)std::max(p->hg.splits_max * p->hg.noq, p->hg.nsq) * p->geo.M * 2 * p->hg.bp;
}

// Zero-padded forward transform of time rows in[b][j][n] (j < nrows) into the spectra of the
// batched products, out[l][j][b] with rows padded to nrows_pad: the register kernel for M = 256,
// else the row transform.
static hipError_t rfft_batch(const float* in, int B, int nrows, int nrows_pad, float2* out, int bp, const Geometry& g,
                             hipStream_t st) {
  const int64_t slot = (int64_t)nrows_pad * bp;
  if (g.M == 256) return launch_rfft_batch256(in, B, nrows, nrows_pad, out, bp, slot, g.nt, 1.0f, st);
  return launch_rfft_rows(in, B, nrows, nrows_pad, out, 1, bp, slot, g, 1.0f, st);
}

// Sum of the split partials part[s][l][o][2 bp] of a batched product (times tau[l][b] when given)
// and the inverse real FFT into out[b][o][n]: one fused kernel for M = 256, else the sum into
// the spectra rows yh[b][o][l] and a row transform.
static hipError_t sum_and_irfft(const float* part, int splits, int noq, int nrows, int B, int bp, const float* tau,
                                float2* yh, float* out, const Geometry& g, hipStream_t st) {
  const float scale = 1.0f / (float)g.L;
  if (g.M == 256) return launch_sum_irfft256(part, splits, noq, nrows, B, bp, tau, out, g.nt, scale, st);
  hipError_t e = launch_sum_f(part, splits, g.M, noq, nrows, B, bp, tau, yh, st);
  if (e == hipSuccess) e = launch_irfft_rows(yh, (int64_t)B * nrows, g.M, 1, out, g.nt, g, scale, st);
  return e;
}

// Batched forward on the matrix cores (half-precision stores).
static s2w_status forward_half(s2w_plan* p, const float* s, int32_t B, float* y, hipStream_t st,
                               const DispOut* disp) {
  const Geometry& g = p->geo;
  const HalfGeo& h = p->hg;
  const Layout& L = p->lay;
  float2* S = (float2*)(p->ws + L.S);
  float* sig_up = (float*)(p->ws + L.sig_up);
  float* sig_down = (float*)(p->ws + L.sig_down);
  uint4* Bop = (uint4*)(p->ws + L.bop);
  float2* U = (float2*)(p->ws + L.U);
  float* tau_up = (float*)(p->ws + L.tau_up);
  float* tau_down = (float*)(p->ws + L.tau_down);
  float* part = (float*)(p->ws + L.part_f);
  float2* yh = (float2*)(p->ws + L.yhb);
  const uint4* Gq = (const uint4*)(p->op + L.gq);
  const float* sG = (const float*)(p->op + L.sg);
  const uint4* Fq = (const uint4*)(p->op + L.fq);
  const float* sF = (const float*)(p->op + L.sf);
  const int bp = h.bp;
  const int ncb = (2 * B + 15) / 16;
  int cfg = p->tune.gemm_cfg;
  // default tiles from sweeps on the Cascadia-sized share: with converted bfloat16 words the
  // real-column tiles lose their edge (the conversions already load the vector ALUs)
  if (cfg < 0) cfg = h.kt_g == 3 ? (B <= 64 ? 16 : 24) : (B <= 64 ? 12 : 18);
  // acoustic GEMM: fgemm_lds 2 takes the eight-wave kernel on full activation fragments, 3 the
  // eight-wave kernel on real-column fragments (with either the mid-chain leaves complex64),
  // 4 the LDS-staged kernel for packed bfloat16 activations where its tile fits (else, and for
  // float16, as 3), and 1 chooses: the LDS-staged kernel for bfloat16 batches of at most 64
  // where it fits, the real-column eight-wave kernel otherwise (Cascadia-sized share, bf16:
  // 26.9 against 30.4 ms per call at B = 128, 51.3 against 52.5 ms at B = 256)
  const int fl = p->tune.fgemm_lds;
  const bool bf16_act = h.kt_f == 1;
  const bool fstaged = bf16_act && gemm_f2_supported(h.noq, B) && (fl == 4 || (fl == 1 && B <= 64));
  const bool wide_re = fl != 2;
  const int zt = fstaged ? gemm_f2_col_tiles(B) : ((g.nobs + 63) / 64) * gemm_fw_col_tiles(h.hterms_f, B, wide_re);
  int splits = p->tune.fgemm_splits;
  if (splits <= 0) splits = std::max(1, std::min(h.splits_max, 2048 / std::max(1, g.M * zt)));
  splits = std::min(splits, h.splits_max);
  hipError_t e = rfft_batch(s, B, g.nsub, h.nsq, S, bp, g, st);
  if (e == hipSuccess) {
    if (cfg == 17 || cfg == 18)
      e = launch_prep_act_re(act_type(h.kt_g), h.hterms_g, S, sig_up, sig_down, g.M, g.nsub, h.nsq, B, bp, h.nks,
                             (B + 15) / 16, Bop, st);
    else
      e = launch_prep_act(act_type(h.kt_g), h.hterms_g, S, sig_up, sig_down, g.M, g.nsub, h.nsq, B, bp, h.nks, ncb,
                          Bop, st);
  }
  if (e != hipSuccess) return hip_fail(p, e, "forward: source transform");
  e = mark(p->ev_begin, st);
  if (e == hipSuccess) {
    const int nwg = p->ncu * p->tune.fused_wg_per_cu;
    e = launch_gemm_g(h.kt_g, h.hterms_g, cfg, Gq, sG, Bop, sig_down, (float*)U, nwg, g.ngrid, g.M, h.nks, ncb, B, bp,
                      st);
  }
  if (e == hipSuccess) e = mark(p->ev_end, st);
  if (e != hipSuccess) return hip_fail(p, e, "forward: elastic matrix-core stage");
  const bool fscale = h.kt_f != 1;
  // float16 acoustic operands: the column scales come from maxima the mid-chain keeps as it
  // writes (M = 256), else from a pass over U
  int groups = 0;
  e = launch_mid_batch(U, sF, B, bp, false, fstaged, g, st, p->tune.mid_rupts, fscale ? part : nullptr,
                       part_floats(p), &groups, disp);
  if (e != hipSuccess) return hip_fail(p, e, "forward: mid-chain");
  if (fscale) {
    e = groups > 0 ? launch_col_scale_final(part, groups, g.M, B, bp, tau_up, tau_down, st)
                   : launch_col_scale(U, g.ngrid, g.M, B, bp, tau_up, tau_down, part, part_floats(p), st);
    if (e != hipSuccess) return hip_fail(p, e, "forward: activation scale");
  }
  if (fstaged) {
    e = launch_gemm_f2(Fq, (const uint2*)U, part, g.ngrid, h.ngq, g.M, h.noq, B, bp, splits, st);
  } else {
    splits = std::min(splits, h.ngq / 16);
    e = launch_gemm_fw(h.kt_f, h.hterms_f, (const uint32_t*)Fq, U, fscale ? tau_up : nullptr, part, g.ngrid, h.ngq,
                       g.M, h.noq, g.nobs, B, bp, splits, wide_re, st);
  }
  if (e != hipSuccess) return hip_fail(p, e, "forward: acoustic matrix-core stage");
  e = sum_and_irfft(part, splits, h.noq, g.nobs, B, bp, fscale ? tau_down : nullptr, yh, y, g, st);
  if (e != hipSuccess) return hip_fail(p, e, "forward: output transform");
  return S2W_OK;
}

// Default tile of the batched float32 GEMMs for a batch of B (rows x ruptures: 0 = 64 x 128,
// 1 = 128 x 32, 2 = 256 x 8, 3 = 64 x 64), from a sweep on the Cascadia-sized share: the
// products over all grid rows favour tall tiles, the grid-row reductions (few output rows)
// wide ones once the batch fills them.
static int b32_cfg(const s2w_plan* p, int B, bool few_rows) {
  if (few_rows) {
    if (p->tune.gemm32_cfg_k >= 0) return p->tune.gemm32_cfg_k;
    return B <= 8 ? 2 : (B <= 64 ? 3 : 0);
  }
  if (p->tune.gemm32_cfg >= 0) return p->tune.gemm32_cfg;
  return B <= 8 ? 2 : 1;
}

static int b32_splits(int tuned, int maxs, int M, int nrows, int B, int cfg) {
  if (tuned > 0) return std::min(tuned, maxs);
  const int64_t tiles = (int64_t)M * ((nrows + cgemm32_rows(cfg) - 1) / cgemm32_rows(cfg)) *
                        ((B + cgemm32_ruptures(cfg) - 1) / cgemm32_ruptures(cfg));
  return (int)std::max<int64_t>(1, std::min<int64_t>(maxs, 2048 / std::max<int64_t>(1, tiles)));
}

// Batched forward on the matrix cores (float32 stores).
static s2w_status forward_b32(s2w_plan* p, const float* s, int32_t B, float* y, hipStream_t st,
                              const DispOut* disp) {
  const Geometry& g = p->geo;
  const BatchGeo32& f = p->fb;
  const Layout& L = p->lay;
  const float2* Gs = (const float2*)(p->op + L.gs);
  const float2* Fs = (const float2*)(p->op + L.fs);
  float2* S = (float2*)(p->ws + L.s32);
  float2* U = (float2*)(p->ws + L.u32);
  float* part = (float*)(p->ws + L.part32);
  float2* yh = (float2*)(p->ws + L.yh32);
  const int bp = f.bp;
  // S[l][j][b]
  hipError_t e = rfft_batch(s, B, g.nsub, f.nsk, S, bp, g, st);
  if (e != hipSuccess) return hip_fail(p, e, "forward: source transform");
  // U[g][l][b] = sum_j Gs[g][l][j] S[l][j][b]
  const int cg = b32_cfg(p, B, false);
  e = mark(p->ev_begin, st);
  if (e == hipSuccess)
    e = launch_cgemm32(cg, false, false, Gs, (int64_t)g.M * f.nsk, 1, f.nsk, g.ngrid, g.ngrid, f.nsk, f.nsk, S, bp,
                       (int64_t)f.nsk * bp, f.nsk, B, bp, (float*)U, 2 * (int64_t)g.M * bp, 2 * (int64_t)bp, 0, g.M, 1,
                       st);
  if (e == hipSuccess) e = mark(p->ev_end, st);
  if (e != hipSuccess) return hip_fail(p, e, "forward: elastic matrix-core stage");
  e = launch_mid_batch(U, nullptr, B, bp, false, false, g, st, p->tune.mid_rupts, nullptr, 0, nullptr, disp);
  if (e != hipSuccess) return hip_fail(p, e, "forward: mid-chain");
  // part[split][l][o][n] = sum_{g in split} Fs[l][o][g] V[g][l][b]
  const int cf = b32_cfg(p, B, true);
  const int sf = b32_splits(p->tune.gemm32_splits, f.splits_f_max, g.M, g.nobs, B, cf);
  const int64_t prow = 2 * (int64_t)bp;
  e = launch_cgemm32(cf, false, false, Fs, f.ngk, 1, (int64_t)f.nok * f.ngk, g.nobs, f.nok, f.ngk, f.ngk, U,
                     (int64_t)g.M * bp, bp, g.ngrid, B, bp, part, prow, (int64_t)f.nok * prow,
                     (int64_t)g.M * f.nok * prow, g.M, sf, st);
  if (e != hipSuccess) return hip_fail(p, e, "forward: acoustic matrix-core stage");
  e = sum_and_irfft(part, sf, f.nok, g.nobs, B, bp, nullptr, yh, y, g, st);
  if (e != hipSuccess) return hip_fail(p, e, "forward: output transform");
  return S2W_OK;
}

// Batched adjoint on the matrix cores (float32 stores): the conjugate transposes of the two
// per-bin products around the transposed mid-chain.
static s2w_status adjoint_b32(s2w_plan* p, const float* r, int32_t B, float* gs, hipStream_t st) {
  const Geometry& g = p->geo;
  const BatchGeo32& f = p->fb;
  const Layout& L = p->lay;
  const float2* Gs = (const float2*)(p->op + L.gs);
  const float2* Fs = (const float2*)(p->op + L.fs);
  float2* R = (float2*)(p->ws + L.s32);
  float2* W = (float2*)(p->ws + L.u32);
  float* part = (float*)(p->ws + L.part32);
  float2* gh = (float2*)(p->ws + L.yh32);
  const int bp = f.bp;
  // R[l][o][b]
  hipError_t e = rfft_batch(r, B, g.nobs, f.nok, R, bp, g, st);
  if (e != hipSuccess) return hip_fail(p, e, "adjoint: residual transform");
  // W[g][l][b] = sum_o conj(Fs[l][o][g]) R[l][o][b]
  const int c1 = b32_cfg(p, B, false);
  e = launch_cgemm32(c1, true, true, Fs, 1, f.ngk, (int64_t)f.nok * f.ngk, g.ngrid, f.ngk, f.nok, f.nok, R, bp,
                     (int64_t)f.nok * bp, f.nok, B, bp, (float*)W, 2 * (int64_t)g.M * bp, 2 * (int64_t)bp, 0, g.M, 1,
                     st);
  if (e != hipSuccess) return hip_fail(p, e, "adjoint: acoustic matrix-core stage");
  e = launch_mid_batch(W, nullptr, B, bp, true, false, g, st, p->tune.mid_rupts);
  if (e != hipSuccess) return hip_fail(p, e, "adjoint: mid-chain");
  // part[split][l][j][n] = sum_{g in split} conj(Gs[g][l][j]) W'[g][l][b]
  // its own tile: by default 128 x 32 tiles from B = 9 to 64 (the subfault rows are many more
  // than the forward reduction's observer rows)
  const int c3 = p->tune.adj32_cfg >= 0 ? p->tune.adj32_cfg : (B <= 8 ? 2 : (B <= 64 ? 1 : 0));
  const int sa = b32_splits(p->tune.adj32_splits, f.splits_a_max, g.M, g.nsub, B, c3);
  const int64_t prow = 2 * (int64_t)bp;
  e = mark(p->ev_begin, st);
  if (e == hipSuccess)
    e = launch_cgemm32(c3, true, true, Gs, 1, (int64_t)g.M * f.nsk, f.nsk, g.nsub, f.nsk, g.ngrid,
                       (g.ngrid + 7) / 8 * 8, W, (int64_t)g.M * bp, bp, g.ngrid, B, bp, part, prow,
                       (int64_t)f.nsk * prow, (int64_t)g.M * f.nsk * prow, g.M, sa, st);
  if (e == hipSuccess) e = mark(p->ev_end, st);
  if (e != hipSuccess) return hip_fail(p, e, "adjoint: elastic matrix-core stage");
  e = sum_and_irfft(part, sa, f.nsk, g.nsub, B, bp, nullptr, gh, gs, g, st);
  if (e != hipSuccess) return hip_fail(p, e, "adjoint: output transform");
  return S2W_OK;
}

// Batched adjoint on the matrix cores (half-precision stores): the conjugate transposes of the
// two per-bin products around the transposed mid-chain.  The acoustic scale sF multiplies the
// first product's rows; the elastic scale sG rides on the mid-chain's output, ahead of the
// grid-row reduction.
static s2w_status adjoint_half(s2w_plan* p, const float* r, int32_t B, float* gs, hipStream_t st) {
  const Geometry& g = p->geo;
  const HalfGeo& h = p->hg;
  const Layout& L = p->lay;
  float* part = (float*)(p->ws + L.part_f);
  float2* R = (float2*)part;                     // residual spectra R[l][o][b]
  float2* W = (float2*)(p->ws + L.U);            // W[g][l][b]
  float2* gh = (float2*)(p->ws + L.S);           // rows gh[b][j][l]
  float* sig_up = (float*)(p->ws + L.sig_up);
  float* sig_down = (float*)(p->ws + L.sig_down);
  float* tau_up = (float*)(p->ws + L.tau_up);
  float* tau_down = (float*)(p->ws + L.tau_down);
  const uint32_t* Gq = (const uint32_t*)(p->op + L.gq);
  const float* sG = (const float*)(p->op + L.sg);
  const uint32_t* Fq = (const uint32_t*)(p->op + L.fq);
  const float* sF = (const float*)(p->op + L.sf);
  const int bp = h.bp;
  const bool sf16 = h.kt_f != 1, sg16 = h.kt_g != 1;  // f16 activation terms with column scales
  hipError_t e = rfft_batch(r, B, g.nobs, g.nobs, R, bp, g, st);
  if (e == hipSuccess && sf16) e = launch_act_scale(R, g.M, g.nobs, g.nobs, B, bp, sig_up, sig_down, st);
  if (e != hipSuccess) return hip_fail(p, e, "adjoint: residual transform");
  // W[g][l][b] = sF[g][l] * sum_o conj(Fq[l][o][g]) R[l][o][b]
  // default tiles (sweep on the Cascadia-sized share): eight waves on real-column activation
  // fragments, 256 rows x 256 columns above B = 128, 256 x 128 down to B = 33, 256 x 64 below
  const int shape1 = p->tune.hadj_tile_f >= 0 ? p->tune.hadj_tile_f : (B <= 32 ? 5 : (B > 128 ? 7 : 6));
  e = launch_gemm_t(h.kt_f, h.hterms_f, shape1, Fq, (int64_t)h.noq * h.ngq, 16 * (int64_t)h.ngq, h.ngq, 16, g.ngrid,
                    h.ngq, g.nobs, h.noq, R,
                    (int64_t)g.nobs * bp, bp, g.nobs, sf16 ? sig_up : nullptr, sf16 ? sig_down : nullptr, sF, g.M, 1,
                    (float*)W, 0, 2 * (int64_t)bp, 2 * (int64_t)g.M * bp, B, bp, g.M, 1, st);
  if (e != hipSuccess) return hip_fail(p, e, "adjoint: acoustic matrix-core stage");
  int groups = 0;
  e = launch_mid_batch(W, sG, B, bp, true, false, g, st, p->tune.mid_rupts, sg16 ? part : nullptr, part_floats(p),
                       &groups);
  if (e == hipSuccess && sg16)
    e = groups > 0 ? launch_col_scale_final(part, groups, g.M, B, bp, tau_up, tau_down, st)
                   : launch_col_scale(W, g.ngrid, g.M, B, bp, tau_up, tau_down, part, part_floats(p), st);
  if (e != hipSuccess) return hip_fail(p, e, "adjoint: mid-chain");
  // part[split][l][j][n] = sum_{g in split} conj(G[g][l][j]) W'[g][l][b] (row-block-major store)
  const int64_t prow = 2 * (int64_t)bp;
  // the float16 store (one term) takes 256 x 256 tiles for large batches
  const int shape3 =
      p->tune.hadj_tile_g >= 0 ? p->tune.hadj_tile_g : (B <= 32 ? 5 : (sg16 && B > 128) ? 7 : 6);
  const int sh3 = shape3 >= 5 ? shape3 - 3 : shape3;
  const int cols3 = sh3 == 2 ? 64 : (sh3 == 3 ? 128 : 256);
  const int rows3 = 256;
  const int tiles = g.M * ((g.nsub + rows3 - 1) / rows3) * ((2 * B + cols3 - 1) / cols3);
  const int fit = std::max(1, std::max(h.splits_max * h.noq, h.nsq) / h.nsq);
  int sa = p->tune.adj32_splits > 0 ? p->tune.adj32_splits : std::max(1, 2048 / std::max(1, tiles));
  sa = std::min(std::min(std::min(sa, fit), 8), (g.ngrid + 15) / 16);
  e = mark(p->ev_begin, st);
  if (e == hipSuccess)
    e = launch_gemm_t(h.kt_g, h.hterms_g, shape3, Gq, (int64_t)(h.ngq / 16) * h.nks * 256, (int64_t)h.nks * 256, 16,
                      256, g.nsub, h.nsq, g.ngrid,
                      (g.ngrid + 15) / 16 * 16, W, bp, (int64_t)g.M * bp, g.ngrid, sg16 ? tau_up : nullptr,
                      sg16 ? tau_down : nullptr, nullptr, 0, 0, part, (int64_t)g.M * h.nsq * prow,
                      (int64_t)h.nsq * prow, prow, B, bp, g.M, sa, st);
  if (e == hipSuccess) e = mark(p->ev_end, st);
  if (e != hipSuccess) return hip_fail(p, e, "adjoint: elastic matrix-core stage");
  e = sum_and_irfft(part, sa, h.nsq, g.nsub, B, bp, nullptr, gh, gs, g, st);
  if (e != hipSuccess) return hip_fail(p, e, "adjoint: output transform");
  return S2W_OK;
}

// Direct forward (eq. 4 form of eqs. 1 and 2, no FFT), one rupture at a time: the elastic
// product over subfaults into grid-row partials, their sum and D_t, the acoustic product over
// grid rows into observer partials, their sum.
static s2w_status forward_direct(s2w_plan* p, const float* s, int32_t B, float* y, hipStream_t st,
                                 const DispOut* disp) {
  const Geometry& g = p->geo;
  const DirectGeo& dd = p->dg;
  const int64_t ntp = dd.ntp;
  const float* Gt = (const float*)(p->op + p->lay.gt);
  const float* Ft = (const float*)(p->op + p->lay.ft);
  float* mpart = (float*)(p->ws + p->lay.dpart);
  float* v = (float*)(p->ws + p->lay.dv);
  float* ypart = (float*)(p->ws + p->lay.dout);
  const float dscale = g.diff ? 1.0f / g.dt : 1.0f;
  for (int b = 0; b < B; ++b) {
    const float* sb = s + (int64_t)b * g.nsub * g.nt;
    float* yb = y + (int64_t)b * g.nobs * g.nt;
    hipError_t e = mark(p->ev_begin, st);
    if (e == hipSuccess)
      e = launch_direct(2, Gt, ntp, (int64_t)g.nsub * ntp, g.ngrid, g.nsub, sb, g.nt, false, mpart,
                        (int64_t)g.ngrid * ntp, ntp, g.nt, dd.s_g, st);
    if (e == hipSuccess) e = mark(p->ev_end, st);
    if (e != hipSuccess) return hip_fail(p, e, "forward: direct elastic product");
    DispOut db{};
    if (disp) {
      db = *disp;
      db.base = disp->base + (int64_t)b * disp->row_stride;  // rupture b; rows are grid rows
      db.row_stride = disp->grid_stride;
      db.rows = g.ngrid;
      db.scale = 1.0f;
    }
    e = launch_direct_reduce(mpart, dd.s_g, (int64_t)g.ngrid * ntp, ntp, g.ngrid, g.nt, false, g.diff != 0, dscale, v,
                             ntp, st, disp ? &db : nullptr);
    if (e != hipSuccess) return hip_fail(p, e, "forward: direct seafloor sum and difference");
    e = launch_direct(1, Ft, (int64_t)g.nobs * ntp, ntp, g.nobs, g.ngrid, v, ntp, false, ypart,
                      (int64_t)g.nobs * ntp, ntp, g.nt, dd.s_f, st);
    if (e != hipSuccess) return hip_fail(p, e, "forward: direct acoustic product");
    e = launch_direct_reduce(ypart, dd.s_f, (int64_t)g.nobs * ntp, ntp, g.nobs, g.nt, false, false, 1.0f, yb, g.nt,
                             st);
    if (e != hipSuccess) return hip_fail(p, e, "forward: direct waveform sum");
  }
  return S2W_OK;
}

// Direct adjoint: the two correlations of the transpose as causal products on the time-reversed
// axis (w_rev = F^T r_rev per grid row, D_t^T as the backward difference of w_rev, then
// gs_rev = G^T w'_rev), reversed back in the final sum.
static s2w_status adjoint_direct(s2w_plan* p, const float* r, int32_t B, float* gs, hipStream_t st) {
  const Geometry& g = p->geo;
  const DirectGeo& dd = p->dg;
  const int64_t ntp = dd.ntp;
  const float* Gt = (const float*)(p->op + p->lay.gt);
  const float* Ft = (const float*)(p->op + p->lay.ft);
  float* wpart = (float*)(p->ws + p->lay.dpart);
  float* w = (float*)(p->ws + p->lay.dv);
  float* gpart = (float*)(p->ws + p->lay.dout);
  const float dscale = g.diff ? 1.0f / g.dt : 1.0f;
  for (int b = 0; b < B; ++b) {
    const float* rb = r + (int64_t)b * g.nobs * g.nt;
    float* gb = gs + (int64_t)b * g.nsub * g.nt;
    hipError_t e = launch_direct(2, Ft, ntp, (int64_t)g.nobs * ntp, g.ngrid, g.nobs, rb, g.nt, true, wpart,
                                 (int64_t)g.ngrid * ntp, ntp, g.nt, dd.s_fa, st);
    if (e != hipSuccess) return hip_fail(p, e, "adjoint: direct acoustic correlation");
    e = launch_direct_reduce(wpart, dd.s_fa, (int64_t)g.ngrid * ntp, ntp, g.ngrid, g.nt, false, g.diff != 0, dscale,
                             w, ntp, st);
    if (e != hipSuccess) return hip_fail(p, e, "adjoint: direct seafloor sum and difference");
    e = mark(p->ev_begin, st);
    if (e == hipSuccess)
      e = launch_direct(2, Gt, (int64_t)g.nsub * ntp, ntp, g.nsub, g.ngrid, w, ntp, false, gpart,
                        (int64_t)g.nsub * ntp, ntp, g.nt, dd.s_ga, st);
    if (e == hipSuccess) e = mark(p->ev_end, st);
    if (e != hipSuccess) return hip_fail(p, e, "adjoint: direct elastic correlation");
    e = launch_direct_reduce(gpart, dd.s_ga, (int64_t)g.nsub * ntp, ntp, g.nsub, g.nt, true, false, 1.0f, gb, g.nt,
                             st);
    if (e != hipSuccess) return hip_fail(p, e, "adjoint: direct slip-rate sum");
  }
  return S2W_OK;
}

static s2w_status forward_single(s2w_plan* p, const float* s, int32_t B, float* y, hipStream_t st, float2* Sh,
                                 float2* part, float2* yh, float2* Vh, const DispOut* disp);

s2w_status s2w_forward(s2w_plan* p, const float* s, int32_t B, float* y, void* stream) {
  s2w_status cs = check_call(p, s, B, y, "forward");
  if (cs != S2W_OK || B == 0) return cs;
  DeviceGuard dg(p->device);
  if (!dg.ok) return fail(p, S2W_EHIP, "forward: cannot select device %d", p->device);
  hipStream_t st = (hipStream_t)stream;
  if (p->hg.on) return forward_half(p, s, B, y, st, nullptr);
  if (p->fb.on) return forward_b32(p, s, B, y, st, nullptr);
  if (p->dg.on) return forward_direct(p, s, B, y, st, nullptr);
  return forward_single(p, s, B, y, st, (float2*)(p->ws + p->lay.sh), (float2*)(p->ws + p->lay.part),
                        (float2*)(p->ws + p->lay.yh), (float2*)(p->ws + p->lay.wp), nullptr);
}

s2w_status s2w_forward_displacement(s2w_plan* p, const float* s, int32_t B, float* y, float* m,
                                    const int32_t* times, int32_t ntimes, void* stream) {
  s2w_status cs = check_call(p, s, B, y, "forward_displacement");
  if (cs != S2W_OK) return cs;
  const Geometry& g = p->geo;
  DispOut d{};
  if (times == nullptr) {
    if (ntimes != g.nt)
      return fail(p, S2W_EINVAL, "forward_displacement: without a time list ntimes must be nt = %d", g.nt);
    d.all = 1;
  } else {
    if (ntimes < 1 || ntimes > g.nt)
      return fail(p, S2W_EINVAL, "forward_displacement: ntimes=%d outside [1, %d]", ntimes, g.nt);
    for (int i = 0; i < ntimes; ++i) {
      const int t = times[i];
      if (t < 0 || t >= g.nt) return fail(p, S2W_EINVAL, "forward_displacement: times[%d]=%d outside [0, %d)", i, t, g.nt);
      if (i > 0 && t <= times[i - 1])
        return fail(p, S2W_EINVAL, "forward_displacement: times must increase strictly (times[%d]=%d)", i, t);
      d.bits[t >> 5] |= 1u << (t & 31);
    }
    d.all = ntimes == g.nt;
  }
  if (B == 0) return S2W_OK;
  if (!m) return fail(p, S2W_EINVAL, "forward_displacement: null displacement pointer");
  if (!aligned(m)) return fail(p, S2W_EINVAL, "forward_displacement: displacement pointer must be 256-byte aligned");
  if ((const void*)m == (const void*)s || m == y)
    return fail(p, S2W_EINVAL, "forward_displacement: displacement output must be distinct from s and y");
  DeviceGuard dg(p->device);
  if (!dg.ok) return fail(p, S2W_EHIP, "forward_displacement: cannot select device %d", p->device);
  hipStream_t st = (hipStream_t)stream;
  d.base = m;
  d.scale = 1.0f / (float)g.L;
  d.rows = 1 << 30;
  if (p->hg.on || p->fb.on) {
    // transform rows are the ruptures of one grid row
    d.row_stride = (int64_t)g.ngrid * ntimes;
    d.grid_stride = ntimes;
    return p->hg.on ? forward_half(p, s, B, y, st, &d) : forward_b32(p, s, B, y, st, &d);
  }
  if (p->dg.on) {
    d.row_stride = (int64_t)g.ngrid * ntimes;  // per rupture; the direct path re-strides by grid row
    d.grid_stride = ntimes;
    return forward_direct(p, s, B, y, st, &d);
  }
  // transform rows are grid rows; forward_single offsets the base per rupture
  d.row_stride = ntimes;
  d.grid_stride = (int64_t)g.ngrid * ntimes;
  return forward_single(p, s, B, y, st, (float2*)(p->ws + p->lay.sh), (float2*)(p->ws + p->lay.part),
                        (float2*)(p->ws + p->lay.yh), (float2*)(p->ws + p->lay.wp), &d);
}

// Bytes of scratch the single-layout forward needs for its source spectrum, the fused
// kernel's per-workgroup partial spectra and their sum (the fused kernel only).
static uint64_t single_fused_scratch(const s2w_plan* p, uint64_t* o_part, uint64_t* o_yh) {
  const Geometry& g = p->geo;
  const uint64_t c8 = sizeof(float2);
  const uint64_t nwg = (uint64_t)p->ncu * p->tune.fused_wg_per_cu;
  uint64_t off = round_up((uint64_t)g.M * g.nsp * c8, kAlign);
  *o_part = off;
  off = round_up(off + nwg * g.M * g.nop * c8, kAlign);
  *o_yh = off;
  return round_up(off + (uint64_t)g.nop * g.M * c8, kAlign);
}

s2w_status s2w_forward_noalloc(s2w_plan* p, const float* s, int32_t B, float* y, void* stream) {
  s2w_status cs = check_call(p, s, B, y, "forward_noalloc");
  if (cs != S2W_OK || B == 0) return cs;
  if (p->hg.on || p->fb.on || p->dg.on)
    return fail(p, S2W_EUNSUPPORTED, "forward_noalloc: only plans with the single (float32) layout");
  if (fused_forward_opt(p->geo) > 32)
    return fail(p, S2W_EUNSUPPORTED, "forward_noalloc: %d observers at L = %d need the unfused path", p->geo.nobs,
                p->geo.L);
  uint64_t o_part = 0, o_yh = 0;
  const uint64_t need = single_fused_scratch(p, &o_part, &o_yh);
  if (need > (uint64_t)S2W_NOALLOC_SCRATCH_BYTES)
    return fail(p, S2W_EUNSUPPORTED,
                "forward_noalloc: needs %llu bytes of scratch (%d workgroups x %d observers x %d slots), the fixed "
                "array holds %llu",
                (unsigned long long)need, p->ncu * p->tune.fused_wg_per_cu, p->geo.nop, p->geo.M,
                (unsigned long long)S2W_NOALLOC_SCRATCH_BYTES);
  DeviceGuard dg(p->device);
  if (!dg.ok) return fail(p, S2W_EHIP, "forward_noalloc: cannot select device %d", p->device);
  hipError_t se = hipSuccess;
  char* base = (char*)scratch_ptr(p->device, &se);
  if (!base) return hip_fail(p, se == hipSuccess ? hipErrorInvalidSymbol : se, "forward_noalloc: scratch lookup");
  return forward_single(p, s, B, y, (hipStream_t)stream, (float2*)base, (float2*)(base + o_part),
                        (float2*)(base + o_yh), nullptr, nullptr);
}

// Single-layout forward: B passes of the fused (or, for many observers, the unfused) kernel,
// with the source spectrum in Sh, the partial spectra in part and their sum in yh; Vh holds
// the unfused path's seafloor spectra.
static s2w_status forward_single(s2w_plan* p, const float* s, int32_t B, float* y, hipStream_t st, float2* Sh,
                                 float2* part, float2* yh, float2* Vh, const DispOut* disp) {
  const Geometry& g = p->geo;
  const float2* Gh = (const float2*)(p->op + p->lay.gh);
  const float2* Fh = (const float2*)(p->op + p->lay.fh);
  const bool fused = fused_forward_opt(g) <= 32;
  if (!fused && !Vh) return fail(p, S2W_EUNSUPPORTED, "forward: the unfused path needs the bound workspace");
  const int nwg = p->ncu * p->tune.fused_wg_per_cu;
  const float inv_l = 1.0f / (float)g.L;
  for (int b = 0; b < B; ++b) {
    const float* sb = s + (int64_t)b * g.nsub * g.nt;
    float* yb = y + (int64_t)b * g.nobs * g.nt;
    hipError_t e = launch_rfft_rows(sb, 1, g.nsub, g.nsp, Sh, 0, g.M, 1, g, 1.0f, st);
    if (e != hipSuccess) return hip_fail(p, e, "forward: source transform");
    int nparts;
    DispOut db{};
    if (disp) {
      db = *disp;
      db.base = disp->base + (int64_t)b * disp->grid_stride;  // rupture b; rows are grid rows
    }
    e = mark(p->ev_begin, st);
    if (fused) {
      if (e == hipSuccess) e = launch_fused_forward(Gh, Fh, Sh, part, nwg, p->tune.fused_rows, g, st, db);
      if (e == hipSuccess) e = mark(p->ev_end, st);
      nparts = nwg;
    } else {
      if (e == hipSuccess) e = launch_forward_rows(Gh, Sh, Vh, nwg, g, st, db);
      if (e == hipSuccess) e = mark(p->ev_end, st);
      if (e == hipSuccess) e = launch_rows_acoustic(Fh, Vh, part, p->tune.adj_cols, p->tune.adj_splits, g, st);
      nparts = p->tune.adj_splits;
    }
    if (e != hipSuccess) return hip_fail(p, e, "forward: contraction");
    e = launch_sum_parts(part, nparts, (int64_t)g.nop * g.M, yh, st);
    if (e != hipSuccess) return hip_fail(p, e, "forward: partial sum");
    e = launch_irfft_rows(yh, g.nobs, g.M, 1, yb, g.nt, g, inv_l, st);
    if (e != hipSuccess) return hip_fail(p, e, "forward: output transform");
  }
  return S2W_OK;
}

s2w_status s2w_adjoint(s2w_plan* p, const float* r, int32_t B, float* gs, void* stream) {
  s2w_status cs = check_call(p, r, B, gs, "adjoint");
  if (cs != S2W_OK || B == 0) return cs;
  const Geometry& g = p->geo;
  DeviceGuard dg(p->device);
  if (!dg.ok) return fail(p, S2W_EHIP, "adjoint: cannot select device %d", p->device);
  hipStream_t st = (hipStream_t)stream;
  if (p->hg.on) return adjoint_half(p, r, B, gs, st);
  if (p->fb.on) return adjoint_b32(p, r, B, gs, st);
  if (p->dg.on) return adjoint_direct(p, r, B, gs, st);
  const float2* Gh = (const float2*)(p->op + p->lay.gh);
  const float2* Fh = (const float2*)(p->op + p->lay.fh);
  float2* Rh = (float2*)(p->ws + p->lay.rh);
  float2* Wp = (float2*)(p->ws + p->lay.wp);
  float2* part = (float2*)(p->ws + p->lay.part2);
  float2* gsh = (float2*)(p->ws + p->lay.gsh);
  const int nwg = p->ncu * p->tune.fused_wg_per_cu;
  const float inv_l = 1.0f / (float)g.L;
  for (int b = 0; b < B; ++b) {
    const float* rb = r + (int64_t)b * g.nobs * g.nt;
    float* gb = gs + (int64_t)b * g.nsub * g.nt;
    hipError_t e = launch_rfft_rows(rb, 1, g.nobs, g.nop, Rh, 0, g.M, 1, g, 1.0f, st);
    if (e != hipSuccess) return hip_fail(p, e, "adjoint: residual transform");
    e = launch_adjoint_rows(Fh, Rh, Wp, nwg, p->tune.fused_rows, g, st);
    if (e != hipSuccess) return hip_fail(p, e, "adjoint: acoustic stage");
    e = mark(p->ev_begin, st);
    if (e == hipSuccess) e = launch_adjoint_elastic(Gh, Wp, part, p->tune.adj_cols, p->tune.adj_splits, g, st);
    if (e == hipSuccess) e = mark(p->ev_end, st);
    if (e != hipSuccess) return hip_fail(p, e, "adjoint: elastic stage");
    e = launch_sum_parts(part, p->tune.adj_splits, (int64_t)g.nsp * g.M, gsh, st);
    if (e != hipSuccess) return hip_fail(p, e, "adjoint: partial sum");
    e = launch_irfft_rows(gsh, g.nsub, g.M, 1, gb, g.nt, g, inv_l, st);
    if (e != hipSuccess) return hip_fail(p, e, "adjoint: output transform");
  }
  return S2W_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// One BLTT operator on its own (Alg. 2): the batched float32 machinery with a single product.

struct s2w_bltt {
  s2w_bltt_desc desc;
  int device = 0;
  Geometry geo;           // nt, L, M (nsub/ngrid/nobs unused)
  int ncol_k = 0;         // columns padded to 8 (zeros): K of the forward product
  int nrow_k = 0;         // rows padded to 8 (zeros in the transformed adjoint input)
  int bp = 8;             // max_batch padded to 8
  int splits_f = 1, splits_a = 1;
  int ncu = 256;
  uint64_t op_total = 0, ws_total = 0;
  uint64_t o_fs = 0, o_s = 0, o_part = 0, o_yh = 0;
  char* op = nullptr;
  char* ws = nullptr;
  std::vector<uint8_t> row_set;
  int64_t rows_missing = 0;
  std::string err;
};

namespace {

s2w_status bfail(s2w_bltt* p, s2w_status st, const char* fmt, ...) {
  if (p) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    p->err = buf;
  }
  return st;
}

s2w_status bhip(s2w_bltt* p, hipError_t e, const char* what) {
  return bfail(p, S2W_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// grid-row splits of a product with `rows` output rows: enough workgroups to fill the chip
int bltt_splits(int M, int rows) {
  const int64_t tiles = (int64_t)M * ((rows + 63) / 64);
  return (int)std::max<int64_t>(1, std::min<int64_t>(8, 2048 / std::max<int64_t>(1, tiles)));
}

int bltt_cfg(int B, bool few_rows) {
  if (few_rows) return B <= 8 ? 2 : (B <= 64 ? 3 : 0);
  return B <= 64 ? 2 : 1;
}

}  // namespace

extern "C" {

s2w_status s2w_bltt_create(const s2w_bltt_desc* desc, int32_t device, s2w_bltt** out) {
  if (!out) return S2W_EINVAL;
  *out = nullptr;
  if (!desc) return S2W_EINVAL;
  const s2w_bltt_desc& d = *desc;
  if (d.nrow < 1 || d.ncol < 1 || d.nrow > (1 << 24) || d.ncol > (1 << 24) || d.nt < 1 || d.nt > 512 ||
      d.max_batch < 0 || d.max_batch > 1024)
    return S2W_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return S2W_EINVAL;
  s2w_bltt* p = new (std::nothrow) s2w_bltt();
  if (!p) return S2W_ENOMEM;
  p->desc = d;
  p->device = device;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
    p->ncu = ncu;
  Geometry& g = p->geo;
  g = Geometry{};
  g.nsub = d.ncol;
  g.ngrid = d.nrow;
  g.nobs = d.nrow;
  g.nt = d.nt;
  g.L = std::max(32, next_pow2(2 * d.nt - 1));
  g.M = g.L / 2;
  g.logM = ilog2(g.M);
  g.diff = S2W_DIFF_NONE;
  g.dt = 1.0f;
  p->ncol_k = (d.ncol + 7) / 8 * 8;
  p->nrow_k = (d.nrow + 7) / 8 * 8;
  p->bp = (std::max(d.max_batch, 1) + 7) / 8 * 8;
  p->splits_f = bltt_splits(g.M, d.nrow);
  p->splits_a = bltt_splits(g.M, d.ncol);
  const uint64_t c8 = sizeof(float2), M = (uint64_t)g.M, bp = (uint64_t)p->bp;
  p->o_fs = 0;
  p->op_total = round_up((uint64_t)d.nrow * M * p->ncol_k * c8, kAlign);
  uint64_t off = 0;
  p->o_s = off;
  off = round_up(off + M * std::max(p->ncol_k, p->nrow_k) * bp * c8, kAlign);
  p->o_part = off;
  const uint64_t prow = std::max((uint64_t)p->splits_f * p->nrow_k, (uint64_t)p->splits_a * p->ncol_k);
  off = round_up(off + prow * M * 2 * bp * 4, kAlign);
  p->o_yh = off;
  off = round_up(off + bp * std::max(d.nrow, d.ncol) * M * c8, kAlign);
  p->ws_total = off;
  p->row_set.assign((size_t)d.nrow, 0);
  p->rows_missing = d.nrow;
  {
    DeviceGuard dg(device);
    if (!dg.ok || ensure_twiddles(device) != hipSuccess) {
      delete p;
      return S2W_EHIP;
    }
  }
  *out = p;
  return S2W_OK;
}

s2w_status s2w_bltt_destroy(s2w_bltt* op) {
  delete op;
  return S2W_OK;
}

const char* s2w_bltt_last_error(const s2w_bltt* op) { return op ? op->err.c_str() : ""; }

s2w_status s2w_bltt_query_sizes(const s2w_bltt* p, uint64_t* operator_bytes, uint64_t* workspace_bytes) {
  if (!p) return S2W_EINVAL;
  if (operator_bytes) *operator_bytes = p->op_total;
  if (workspace_bytes) *workspace_bytes = p->ws_total;
  return S2W_OK;
}

s2w_status s2w_bltt_bind_memory(s2w_bltt* p, void* operator_store, uint64_t operator_bytes, void* workspace,
                                uint64_t workspace_bytes) {
  if (!p) return S2W_EINVAL;
  if (!operator_store || !workspace) return bfail(p, S2W_EINVAL, "bind: null pointer");
  if (!aligned(operator_store) || !aligned(workspace)) return bfail(p, S2W_EINVAL, "bind: pointers must be 256-byte aligned");
  if (operator_bytes < p->op_total || workspace_bytes < p->ws_total)
    return bfail(p, S2W_ENOMEM, "bind: need %llu + %llu bytes", (unsigned long long)p->op_total,
                 (unsigned long long)p->ws_total);
  p->op = (char*)operator_store;
  p->ws = (char*)workspace;
  std::fill(p->row_set.begin(), p->row_set.end(), 0);
  p->rows_missing = p->desc.nrow;
  return S2W_OK;
}

s2w_status s2w_bltt_set_blocks(s2w_bltt* p, const float* F_chunk, int64_t row0, int64_t nrows, void* stream) {
  if (!p) return S2W_EINVAL;
  if (!p->op) return bfail(p, S2W_ESTATE, "set_blocks: memory not bound");
  if (!F_chunk) return bfail(p, S2W_EINVAL, "set_blocks: null chunk pointer");
  if (!aligned(F_chunk)) return bfail(p, S2W_EINVAL, "set_blocks: chunk pointer must be 256-byte aligned");
  if (row0 < 0 || nrows < 0 || row0 + nrows > p->desc.nrow)
    return bfail(p, S2W_EINVAL, "set_blocks: rows [%lld, %lld) outside [0, %d)", (long long)row0,
                 (long long)(row0 + nrows), p->desc.nrow);
  if (nrows == 0) return S2W_OK;
  DeviceGuard dg(p->device);
  if (!dg.ok) return bfail(p, S2W_EHIP, "set_blocks: cannot select device %d", p->device);
  const Geometry& g = p->geo;
  float2* Fs = (float2*)(p->op + p->o_fs);
  // Fs[row][l][c]: the GEMM layout of the forward product (c padded with zeros)
  hipError_t e = launch_rfft_rows(F_chunk, nrows, p->desc.ncol, p->ncol_k, Fs + row0 * g.M * p->ncol_k,
                                  (int64_t)g.M * p->ncol_k, 1, p->ncol_k, g, 1.0f, (hipStream_t)stream);
  if (e != hipSuccess) return bhip(p, e, "set_blocks: transform");
  for (int64_t r = row0; r < row0 + nrows; ++r)
    if (!p->row_set[(size_t)r]) {
      p->row_set[(size_t)r] = 1;
      --p->rows_missing;
    }
  return S2W_OK;
}

static s2w_status bltt_check(s2w_bltt* p, const void* in, int32_t B, const void* out, const char* who) {
  if (!p) return S2W_EINVAL;
  if (B < 0 || B > p->desc.max_batch) return bfail(p, S2W_EINVAL, "%s: B=%d outside [0, %d]", who, B, p->desc.max_batch);
  if (B == 0) return S2W_OK;
  if (!in || !out) return bfail(p, S2W_EINVAL, "%s: null pointer", who);
  if (!aligned(in) || !aligned(out)) return bfail(p, S2W_EINVAL, "%s: pointers must be 256-byte aligned", who);
  if (in == out) return bfail(p, S2W_EINVAL, "%s: input and output must be distinct", who);
  if (!p->op) return bfail(p, S2W_ESTATE, "%s: memory not bound", who);
  if (p->rows_missing > 0) return bfail(p, S2W_ESTATE, "%s: %lld rows have no blocks yet", who, (long long)p->rows_missing);
  return S2W_OK;
}

s2w_status s2w_bltt_apply(s2w_bltt* p, const float* x, int32_t B, float* y, void* stream) {
  s2w_status cs = bltt_check(p, x, B, y, "apply");
  if (cs != S2W_OK || B == 0) return cs;
  DeviceGuard dg(p->device);
  if (!dg.ok) return bfail(p, S2W_EHIP, "apply: cannot select device %d", p->device);
  hipStream_t st = (hipStream_t)stream;
  const Geometry& g = p->geo;
  const int nrow = p->desc.nrow, ncol = p->desc.ncol, bp = p->bp;
  const float2* Fs = (const float2*)(p->op + p->o_fs);
  float2* S = (float2*)(p->ws + p->o_s);
  float* part = (float*)(p->ws + p->o_part);
  float2* yh = (float2*)(p->ws + p->o_yh);
  if (B <= 4) {
    // few inputs: per-bin matrix-vector products streaming the store once (HBM-bound);
    // inputs transformed as S[b][l][c]
    hipError_t e = launch_rfft_rows(x, B, ncol, p->ncol_k, S, (int64_t)g.M * p->ncol_k, 1, p->ncol_k, g, 1.0f, st);
    if (e != hipSuccess) return bhip(p, e, "apply: input transform");
    e = launch_bltt_gemv(Fs, S, yh, nrow, g.M, p->ncol_k, B, p->ncu, st);
    if (e != hipSuccess) return bhip(p, e, "apply: per-bin products");
    e = launch_irfft_rows(yh, (int64_t)B * nrow, g.M, 1, y, g.nt, g, 1.0f / (float)g.L, st);
    if (e != hipSuccess) return bhip(p, e, "apply: output transform");
    return S2W_OK;
  }
  // S[l][c][b]
  hipError_t e = rfft_batch(x, B, ncol, p->ncol_k, S, bp, g, st);
  if (e != hipSuccess) return bhip(p, e, "apply: input transform");
  // part[split][l][r][n] = sum_{c in split} Fs[r][l][c] S[l][c][b]
  const int splits = p->splits_f;
  const int cfg = bltt_cfg(B, splits > 1);
  const int64_t prow = 2 * (int64_t)bp;
  e = launch_cgemm32(cfg, false, false, Fs, (int64_t)g.M * p->ncol_k, 1, p->ncol_k, nrow, nrow, p->ncol_k, p->ncol_k,
                     S, bp, (int64_t)p->ncol_k * bp, p->ncol_k, B, bp, part, prow, (int64_t)p->nrow_k * prow,
                     (int64_t)g.M * p->nrow_k * prow, g.M, splits, st);
  if (e != hipSuccess) return bhip(p, e, "apply: matrix-core product");
  e = sum_and_irfft(part, splits, p->nrow_k, nrow, B, bp, nullptr, yh, y, g, st);
  if (e != hipSuccess) return bhip(p, e, "apply: output transform");
  return S2W_OK;
}

s2w_status s2w_bltt_adjoint(s2w_bltt* p, const float* y, int32_t B, float* x, void* stream) {
  s2w_status cs = bltt_check(p, y, B, x, "adjoint");
  if (cs != S2W_OK || B == 0) return cs;
  DeviceGuard dg(p->device);
  if (!dg.ok) return bfail(p, S2W_EHIP, "adjoint: cannot select device %d", p->device);
  hipStream_t st = (hipStream_t)stream;
  const Geometry& g = p->geo;
  const int nrow = p->desc.nrow, ncol = p->desc.ncol, bp = p->bp;
  const float2* Fs = (const float2*)(p->op + p->o_fs);
  float2* R = (float2*)(p->ws + p->o_s);
  float* part = (float*)(p->ws + p->o_part);
  float2* xh = (float2*)(p->ws + p->o_yh);
  // R[l][r][b] (rows padded with zeros)
  hipError_t e = rfft_batch(y, B, nrow, p->nrow_k, R, bp, g, st);
  if (e != hipSuccess) return bhip(p, e, "adjoint: input transform");
  // part[split][l][c][n] = sum_{r in split} conj(Fs[r][l][c]) R[l][r][b]
  const int splits = p->splits_a;
  const int cfg = bltt_cfg(B, splits > 1);
  const int64_t prow = 2 * (int64_t)bp;
  e = launch_cgemm32(cfg, true, true, Fs, 1, (int64_t)g.M * p->ncol_k, p->ncol_k, ncol, p->ncol_k, nrow, p->nrow_k, R,
                     bp, (int64_t)p->nrow_k * bp, p->nrow_k, B, bp, part, prow, (int64_t)p->ncol_k * prow,
                     (int64_t)g.M * p->ncol_k * prow, g.M, splits, st);
  if (e != hipSuccess) return bhip(p, e, "adjoint: matrix-core product");
  e = sum_and_irfft(part, splits, p->ncol_k, ncol, B, bp, nullptr, xh, x, g, st);
  if (e != hipSuccess) return bhip(p, e, "adjoint: output transform");
  return S2W_OK;
}

}  // extern "C"
