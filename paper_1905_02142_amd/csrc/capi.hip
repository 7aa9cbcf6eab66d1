// C ABI of the library: contexts, argument checking, workspace and launches.
// The arithmetic lives in the kernels; this file only validates, sizes buffers
// and enqueues work on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/soap.h"
#include "gap.h"
#include "neighbors.h"
#include "pair_kernels.h"
#include "soap_device.h"

extern "C" int soap_host_basis_table(int n_max, double r_cut, double sigma0_r, double* W, double* Wlo, double* eig);
extern "C" int soap_host_radial_consts(int n_max, double r_cut, double* invN_hi, double* invN_lo, double* rc4);

namespace {

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

}  // namespace

// Scratch of soap_descriptor_noalloc (pair rows, c, the central-atom factors and
// |p|), for callers that cannot allocate.  Every device the library runs on
// holds one copy for the life of the process.  In host code the name is not a
// device address: host code uses only the address that hipGetSymbolAddress
// returns for the current device (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[SOAP_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_dev;  // the device address of `scratch`, per device

// The address of `scratch` on `device`, which must be current: looked up once per
// device, then kept.
hipError_t noalloc_scratch(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize(device + 1, nullptr);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = p;
  }
  *out = g_scratch_dev[device];
  return hipSuccess;
}

}  // namespace

struct soap_ctx {
  soap_params prm{};
  soap::DevParams dp{};
  soap::DevTables ht{};
  soap::DevTables* dt = nullptr;
  int device = 0;
  void* scratch = nullptr;  // this device's copy of the no-allocation scratch array
  hipError_t scratch_err = hipSuccess;  // why `scratch` could not be looked up
  std::string err;
  long long ws_bytes = 0;
  long long ws_gen = 0;  // bumped whenever a workspace buffer is reallocated
  int* pinned = nullptr;  // host-pinned staging for structure-geometry uploads
  hipEvent_t pinned_ev = nullptr;  // completes when the last upload from the staging has been read
  int* report = nullptr;  // host-pinned pair count and error bits, written by a kernel
  int* report_dev = nullptr;  // the same memory as the device addresses it
  std::vector<char> meta_host;  // the structure geometry last uploaded, and where
  void* meta_dev = nullptr;
  soap_tuning tune{0, 0, 256, 2, 0};
  std::string tune_cache;  // attached tuning-cache file ("" = none)
  long long tune_cache_hits = 0;
  double skin = 0.0;  // neighbour lists are built to r_cut + skin
  int built_atoms = -1, built_structures = 0;  // the geometry of the last build (meta on the device)
  Buf tune_out;  // scratch outputs of the autotuner
  size_t pinned_bytes = 0;
  // neighbour build
  Buf meta, so, atom_bin, atom_wrap, bin_count, bin_start, bin_cursor, bin_unsorted, bin_cand, counts, opre,
      scan_part, errflag;
  // descriptor / adjoint
  Buf rows, bc, c, q, pnorm, qbar, gx, gapw, e_tmp;  // gx: the pair gradients, (x, y, z, 0) per pair
  // stage timing
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  unsigned prof_mask = 0;  // stages whose events are recorded
  std::vector<Rec> prof;
  std::vector<hipEvent_t> ev_pool;
};

namespace {

soap_status fail(soap_ctx* ctx, soap_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

soap_status hip_fail(soap_ctx* ctx, hipError_t e, const char* where) {
  return fail(ctx, SOAP_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define SOAP_HIP(ctx, call)                                  \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call);   \
  } while (0)

// grow-only device buffer.  Growth frees the old allocation, which a HIP graph
// captured earlier may still name, so it bumps ctx->ws_gen (callers that replay
// graphs compare it), and it is refused while `st` is being captured (the
// allocation would not be part of the graph).  0: ok, 1: allocation failed,
// 2: growth needed under capture.
int ensure(soap_ctx* ctx, Buf& b, size_t bytes, hipStream_t st) {
  if (bytes == 0) bytes = 8;
  if (b.cap >= bytes) return 0;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return 2;
  ++ctx->ws_gen;
  if (b.p) {
    hipFree(b.p);
    ctx->ws_bytes -= (long long)b.cap;
    b.p = nullptr;
    b.cap = 0;
  }
  size_t want = bytes + bytes / 4;
  if (hipMalloc(&b.p, want) != hipSuccess) {
    b.p = nullptr;
    return 1;
  }
  b.cap = want;
  ctx->ws_bytes += (long long)want;
  return 0;
}

bool ensure_pinned(soap_ctx* ctx, size_t bytes) {
  if (ctx->pinned_bytes >= bytes) return true;
  if (ctx->pinned_ev && hipEventSynchronize(ctx->pinned_ev) != hipSuccess) return false;
  if (ctx->pinned) hipHostFree(ctx->pinned);
  ctx->pinned = nullptr;
  ctx->pinned_bytes = 0;
  if (hipHostMalloc((void**)&ctx->pinned, bytes, hipHostMallocDefault) != hipSuccess) return false;
  ctx->pinned_bytes = bytes;
  return true;
}

// (expects the caller's stream as `st` in scope)
#define SOAP_ENSURE(ctx, buf, bytes)                                                                     \
  do {                                                                                                   \
    const int e_ = ensure(ctx, buf, bytes, st);                                                          \
    if (e_ == 1) return fail(ctx, SOAP_ENOMEM, "device allocation failed");                              \
    if (e_ == 2)                                                                                         \
      return fail(ctx, SOAP_ENOTSUP, "workspace must grow during stream capture (run once outside it)"); \
  } while (0)

// the operand precision of the GAP contractions (the kernels' 0..3): the
// matrix-core power-spectrum mode contracts in BF16
int gap_precision(const soap_ctx* ctx) {
  return ctx->prm.precision == SOAP_MIXED_BF16_PS ? (int)SOAP_MIXED_BF16 : (int)ctx->prm.precision;
}

soap_status check_params(const soap_params* p, std::string& why) {
  if (!p) return why = "null parameters", SOAP_EINVAL;
  if (p->n_max < 2 || p->n_max > soap::kMaxN) return why = "n_max must be in 2..12", SOAP_EINVAL;
  if (p->l_max < 0 || p->l_max > soap::kMaxL) return why = "l_max must be in 0..12", SOAP_EINVAL;
  if (p->n_species < 1) return why = "n_species must be >= 1", SOAP_EINVAL;
  if (!(p->r_cut > 0) || !std::isfinite(p->r_cut)) return why = "r_cut must be positive", SOAP_EINVAL;
  if (!(p->r_soft > 0) || p->r_soft > p->r_cut) return why = "r_soft must be in (0, r_cut]", SOAP_EINVAL;
  if (p->r_soft < p->r_cut && !(p->n_f > 0)) return why = "n_f must be positive", SOAP_EINVAL;
  if (!(p->sigma0_r > 0) || !(p->sigma0_perp > 0)) return why = "sigma0_r and sigma0_perp must be positive", SOAP_EINVAL;
  if (!(p->alpha_r >= 0) || !(p->alpha_perp >= 0) || !(p->a >= 0))
    return why = "alpha_r, alpha_perp and a must be >= 0", SOAP_EINVAL;
  if (!std::isfinite(p->central_weight)) return why = "central_weight must be finite", SOAP_EINVAL;
  if (p->l_weight != 0 && p->l_weight != 1) return why = "l_weight must be 0 or 1", SOAP_EINVAL;
  if (p->precision < SOAP_FP64 || p->precision > SOAP_MIXED_BF16_PS) return why = "unknown precision", SOAP_EINVAL;
  if (p->precision == SOAP_MIXED_BF16_PS && p->n_species * p->n_max > 48)
    return why = "the matrix-core power spectrum takes at most 48 channels (n_species * n_max)", SOAP_ENOTSUP;
  if (p->radial_precision < SOAP_RADIAL_AUTO || p->radial_precision > SOAP_RADIAL_DD)
    return why = "unknown radial precision", SOAP_EINVAL;
  return SOAP_OK;
}

// Pairs the kernels may touch: the count, or the capacity while the count is
// still on the device (then every kernel cuts its pair ranges there).
long long pair_bound(const soap_nlist* nl) { return nl->n_pairs >= 0 ? nl->n_pairs : nl->capacity; }
const int* pair_count(const soap_nlist* nl) {
  return nl->n_pairs == SOAP_PAIRS_DEFERRED ? nl->offsets + nl->n_atoms : nullptr;
}

soap_status check_nlist(soap_ctx* ctx, const soap_nlist* nl) {
  if (!nl) return fail(ctx, SOAP_EINVAL, "null neighbour list");
  if (nl->n_atoms < 0 || nl->capacity < 0 || (nl->n_pairs < 0 && nl->n_pairs != SOAP_PAIRS_DEFERRED))
    return fail(ctx, SOAP_EINVAL, "negative sizes in neighbour list");
  if (nl->n_pairs > nl->capacity) return fail(ctx, SOAP_EINVAL, "neighbour list holds more pairs than its capacity");
  if (pair_bound(nl) > 2147483647LL) return fail(ctx, SOAP_ENOTSUP, "more than 2^31-1 pairs");
  if (!nl->offsets && (nl->n_atoms > 0 || nl->n_pairs == SOAP_PAIRS_DEFERRED))
    return fail(ctx, SOAP_EINVAL, "null offsets");
  if (pair_bound(nl) > 0 && (!nl->j || !nl->dx || !nl->dy || !nl->dz || !nl->rev))
    return fail(ctx, SOAP_EINVAL, "null per-pair arrays");
  return SOAP_OK;
}

soap_status check_lds(soap_ctx* ctx) {
  const size_t lim = 64 * 1024;  // per-workgroup LDS without opting in to more
  if (soap::descriptor_lds_bytes(ctx->dp) > lim || soap::adjoint_lds_bytes(ctx->dp) > lim)
    return fail(ctx, SOAP_ENOTSUP, "descriptor too large for one workgroup's LDS (reduce n_species, n_max or l_max)");
  return SOAP_OK;
}

hipEvent_t take_event(soap_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// records hipEvents around one kernel group while profiling is on
struct StageTimer {
  soap_ctx* ctx;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  StageTimer(soap_ctx* c, int s, hipStream_t stream) : ctx(c), stage(s), st(stream) {
    if ((ctx->prof_mask >> stage) & 1u) {
      a = take_event(ctx);
      if (a && hipEventRecord(a, st) != hipSuccess) {
        ctx->ev_pool.push_back(a);
        a = nullptr;
      }
    }
  }
  ~StageTimer() { stop(); }
  void stop() {
    if (!a) return;
    hipEvent_t b = take_event(ctx);
    if (b && hipEventRecord(b, st) == hipSuccess) ctx->prof.push_back({stage, a, b});
    else {
      ctx->ev_pool.push_back(a);
      if (b) ctx->ev_pool.push_back(b);
    }
    a = nullptr;
  }
};

// forward descriptor into the context's buffers (c, q, |p|)
// (qc: optional bf16 copy of q for the GAP contraction, row pitch qc_pitch)
// the same into caller-provided buffers: pair rows (pair_rows_bytes), c
// (c_doubles_per_atom per atom) and the central-atom factors (kMaxN doubles);
// with `timed`, the stages record their events while profiling is on
soap_status forward_into(soap_ctx* ctx, const soap_nlist* nl, const int32_t* species, double* q, double* pnorm,
                         bool deriv, hipStream_t st, void* rows, bool rows_f32, void* c, double* bc, void* qc,
                         int qc_pitch, bool timed) {
  const soap::DevParams& P = ctx->dp;
  const size_t NP = (size_t)pair_bound(nl);
  const unsigned mask = ctx->prof_mask;
  if (!timed) ctx->prof_mask = 0;
  soap_status s = SOAP_OK;
  for (int part = 1; part <= 2 && s == SOAP_OK; ++part) {
    StageTimer tm(ctx, part == 1 ? SOAP_STAGE_PAIR_PREP : SOAP_STAGE_PAIR_ANGULAR, st);
    const hipError_t e = soap::launch_pair_prep(P, ctx->dt, (long long)NP, pair_count(nl), nl->dx, nl->dy, nl->dz,
                                                rows, rows_f32, deriv, bc, ctx->tune.prep_block, part, st);
    if (e != hipSuccess) s = hip_fail(ctx, e, "launch_pair_prep");
  }
  if (s == SOAP_OK) {
    StageTimer tm(ctx, SOAP_STAGE_DESCRIPTOR, st);
    const hipError_t e = soap::launch_descriptor(P, ctx->dt, nl->n_atoms, nl->offsets, (int)NP, nl->j, species, rows,
                                                 rows_f32, bc, c, q, P.K, pnorm, qc, qc_pitch, st);
    if (e != hipSuccess) s = hip_fail(ctx, e, "launch_descriptor");
  }
  ctx->prof_mask = mask;
  return s;
}

// store_f32: the pair fields and c stored in FP32 (the mixed modes' energy and
// force path with the FP64 radial stage; the arithmetic stays FP64)
soap_status forward(soap_ctx* ctx, const soap_nlist* nl, const int32_t* species, double* q, double* pnorm,
                    bool deriv, hipStream_t st, void* qc = nullptr, int qc_pitch = 0, bool store_f32 = false) {
  const soap::DevParams& P = ctx->dp;
  const size_t N = (size_t)nl->n_atoms, NP = (size_t)pair_bound(nl);
  SOAP_ENSURE(ctx, ctx->c, (store_f32 ? sizeof(float) : sizeof(double)) * N * soap::c_doubles_per_atom(P));
  SOAP_ENSURE(ctx, ctx->rows, soap::pair_rows_bytes(P, (long long)NP, store_f32));
  SOAP_ENSURE(ctx, ctx->bc, sizeof(double) * soap::kMaxN);
  return forward_into(ctx, nl, species, q, pnorm, deriv, st, ctx->rows.p, store_f32, ctx->c.p, (double*)ctx->bc.p, qc,
                      qc_pitch, true);
}

}  // namespace

extern "C" {

const char* soap_status_string(soap_status s) {
  switch (s) {
    case SOAP_OK: return "ok";
    case SOAP_EINVAL: return "invalid argument";
    case SOAP_ENOMEM: return "out of device memory";
    case SOAP_EOVERFLOW: return "neighbour list capacity exceeded";
    case SOAP_EHIP: return "HIP runtime error";
    case SOAP_ENOTSUP: return "not supported";
  }
  return "unknown status";
}

const char* soap_last_error(const soap_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

long long soap_workspace_bytes(const soap_ctx* ctx) { return ctx ? ctx->ws_bytes : 0; }

long long soap_workspace_generation(const soap_ctx* ctx) { return ctx ? ctx->ws_gen : -1; }

int soap_descriptor_dim(const soap_ctx* ctx) { return ctx ? ctx->dp.K : 0; }

soap_status soap_create(const soap_params* p, soap_ctx** out) {
  if (!out) return SOAP_EINVAL;
  *out = nullptr;
  std::string why;
  soap_status s = check_params(p, why);
  if (s != SOAP_OK) return s;
  soap_ctx* ctx = new soap_ctx();
  ctx->prm = *p;
  soap::DevParams& d = ctx->dp;
  d.n = p->n_max;
  d.l = p->l_max;
  d.ns = p->n_species;
  d.nch = d.ns * d.n;
  d.LL = (d.l + 1) * (d.l + 1);
  d.K = d.nch * (d.nch + 1) / 2 * (d.l + 1);
  d.buffer = p->r_soft < p->r_cut ? 1 : 0;
  d.l_weight = p->l_weight;
  d.ps_mfma = p->precision == SOAP_MIXED_BF16_PS ? 1 : 0;
  d.radial_dd = p->radial_precision == SOAP_RADIAL_DD ||
                (p->radial_precision == SOAP_RADIAL_AUTO && p->precision == SOAP_FP64 && p->n_max >= 8);
  d.rc = p->r_cut;
  d.rs = p->r_soft;
  d.nf = p->n_f;
  d.inv_rc = 1.0 / p->r_cut;
  d.s0r = p->sigma0_r;
  d.s0p = p->sigma0_perp;
  d.ar = p->alpha_r;
  d.ap = p->alpha_perp;
  d.a = p->a;
  d.cw = p->central_weight;
  for (int g = 0; g < 3; ++g) {
    // degree l has l + 1 records (l, m >= 0): longest first, each to the lane with
    // the fewest so far (the lowest such lane on a tie)
    const int R = 2 << g;
    int load[8] = {};
    for (int u = 0; u < 8; ++u) d.tail_deg[g][u] = 0;
    for (int l = d.l; l >= 0; --l) {
      int b = 0;
      for (int u = 1; u < R; ++u)
        if (load[u] < load[b]) b = u;
      d.tail_deg[g][b] |= (unsigned short)(1u << l);
      load[b] += l + 1;
    }
  }
  soap::DevTables& t = ctx->ht;
  double W[16 * 16], Wl[16 * 16];
  if (soap_host_basis_table(d.n, d.rc, d.s0r, W, Wl, nullptr) != 0 ||
      soap_host_radial_consts(d.n, d.rc, t.invN, t.invNl, t.rcinv) != 0) {
    delete ctx;
    return SOAP_EINVAL;
  }
  for (int k = 0; k < d.n; ++k)
    for (int al = 0; al < d.n; ++al) {
      t.W[k * soap::kMaxN + al] = W[k * d.n + al];
      t.Wl[k * soap::kMaxN + al] = Wl[k * d.n + al];
    }
  for (int l = 0; l <= soap::kMaxL + 1; ++l) t.lw[l] = p->l_weight ? 1.0 : 2.0 * l + 1.0;
  soap::build_angular_tables(d, t);
  if (hipGetDevice(&ctx->device) != hipSuccess || hipMalloc((void**)&ctx->dt, sizeof(soap::DevTables)) != hipSuccess) {
    delete ctx;
    return SOAP_EHIP;
  }
  if (hipMemcpy(ctx->dt, &t, sizeof(soap::DevTables), hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(ctx->dt);
    delete ctx;
    return SOAP_EHIP;
  }
  // set-up of soap_descriptor_noalloc: the address of this device's scratch array
  // (a failure disables that entry point only, which reports it)
  ctx->scratch_err = noalloc_scratch(ctx->device, &ctx->scratch);
  if (ctx->scratch_err != hipSuccess) ctx->scratch = nullptr;
  *out = ctx;
  return SOAP_OK;
}

void soap_destroy(soap_ctx* ctx) {
  if (!ctx) return;
  Buf* bufs[] = {&ctx->meta, &ctx->so, &ctx->atom_bin, &ctx->atom_wrap, &ctx->bin_count, &ctx->bin_start,
                 &ctx->bin_cursor, &ctx->bin_unsorted, &ctx->bin_cand, &ctx->counts, &ctx->opre, &ctx->scan_part, &ctx->errflag, &ctx->rows, &ctx->bc, &ctx->c,
                 &ctx->q, &ctx->pnorm, &ctx->qbar, &ctx->gx, &ctx->gapw, &ctx->e_tmp, &ctx->tune_out};
  for (Buf* b : bufs)
    if (b->p) hipFree(b->p);
  for (auto& r : ctx->prof) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  for (hipEvent_t e : ctx->ev_pool) hipEventDestroy(e);
  if (ctx->dt) hipFree(ctx->dt);
  if (ctx->pinned_ev) {
    hipEventSynchronize(ctx->pinned_ev);
    hipEventDestroy(ctx->pinned_ev);
  }
  if (ctx->pinned) hipHostFree(ctx->pinned);
  if (ctx->report) hipHostFree(ctx->report);
  delete ctx;
}

}  // extern "C"

namespace {

// Everything of a neighbour build up to the filled list, enqueued on st with no
// host synchronisation.  The pair count stays on the device (offsets[n_atoms]);
// the fill writes only below the capacity, so a list that
// overflows is detected afterwards, from the count, without any access beyond it.
soap_status enqueue_build(soap_ctx* ctx, int n_atoms, const double* pos, const double* cells, const int32_t* pbc,
                          const int32_t* struct_offsets, int n_structures, soap_nlist* nl, hipStream_t st) {
  if (!nl || !cells || !pbc || n_atoms < 0 || n_structures < 1)
    return fail(ctx, SOAP_EINVAL, "null argument or non-positive structure count");
  if (n_atoms > 0 && !pos) return fail(ctx, SOAP_EINVAL, "null positions");
  if (!nl->offsets) return fail(ctx, SOAP_EINVAL, "null offsets array");
  if (nl->capacity < 0) return fail(ctx, SOAP_EINVAL, "negative capacity");
  if (nl->capacity > 2147483647LL) return fail(ctx, SOAP_ENOTSUP, "capacity above 2^31-1 pairs");
  if (nl->capacity > 0 && (!nl->j || !nl->img || !nl->rev || !nl->center || !nl->dx || !nl->dy || !nl->dz))
    return fail(ctx, SOAP_EINVAL, "null per-pair arrays");
  const double rc = ctx->dp.rc + ctx->skin;  // the list's cutoff
  // per-structure cell-list geometry
  std::vector<soap::StructMeta> meta(n_structures);
  std::vector<int> so(n_structures + 1);
  int n_bins = 0;
  long long n_opre = 0;  // per-(centre, slab offset) hit prefixes of the count pass
  for (int s = 0; s <= n_structures; ++s) {
    so[s] = struct_offsets ? struct_offsets[s] : (s == 0 ? 0 : n_atoms);
    if (s > 0 && so[s] < so[s - 1]) return fail(ctx, SOAP_EINVAL, "structure offsets must be non-decreasing");
  }
  if (so[0] != 0 || so[n_structures] != n_atoms) return fail(ctx, SOAP_EINVAL, "structure offsets must span 0..n_atoms");
  for (int s = 0; s < n_structures; ++s) {
    soap::StructMeta& M = meta[s];
    const double* c = cells + 9 * s;
    for (int k = 0; k < 9; ++k) {
      if (!std::isfinite(c[k])) return fail(ctx, SOAP_EINVAL, "non-finite cell");
      M.cell[k] = c[k];
    }
    const double det = c[0] * (c[4] * c[8] - c[5] * c[7]) - c[1] * (c[3] * c[8] - c[5] * c[6]) +
                       c[2] * (c[3] * c[7] - c[4] * c[6]);
    if (!(std::fabs(det) > 1e-12)) return fail(ctx, SOAP_EINVAL, "singular cell");
    // inverse (cell rows are lattice vectors: fractional = position * inv)
    M.inv[0] = (c[4] * c[8] - c[5] * c[7]) / det;
    M.inv[1] = (c[2] * c[7] - c[1] * c[8]) / det;
    M.inv[2] = (c[1] * c[5] - c[2] * c[4]) / det;
    M.inv[3] = (c[5] * c[6] - c[3] * c[8]) / det;
    M.inv[4] = (c[0] * c[8] - c[2] * c[6]) / det;
    M.inv[5] = (c[2] * c[3] - c[0] * c[5]) / det;
    M.inv[6] = (c[3] * c[7] - c[4] * c[6]) / det;
    M.inv[7] = (c[1] * c[6] - c[0] * c[7]) / det;
    M.inv[8] = (c[0] * c[4] - c[1] * c[3]) / det;
    int nb_total = 1;
    for (int a = 0; a < 3; ++a) {
      const double* u = c + 3 * ((a + 1) % 3);
      const double* v = c + 3 * ((a + 2) % 3);
      const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
      const double w = std::fabs(det) / std::sqrt(cx * cx + cy * cy + cz * cz);
      M.pbc[a] = pbc[3 * s + a] ? 1 : 0;
      if (M.pbc[a]) {
        // bins of width >= r_cut / cell_split: a centre scans (2 cell_split + 1)^3 of them
        int nb = (int)std::floor(w * ctx->tune.cell_split / (rc * (1.0 + 2e-9)));
        if (nb < 1) nb = 1;
        if (nb > 256) nb = 256;
        M.nbin[a] = nb;
        M.R[a] = (int)std::ceil(rc * nb / w * (1.0 + 1e-9));
        if (M.R[a] > soap::kWrapMax / 2) return fail(ctx, SOAP_ENOTSUP, "cell far thinner than the cutoff");
      } else {
        M.nbin[a] = 1;
        M.R[a] = 0;
      }
      nb_total *= M.nbin[a];
    }
    M.bin0 = n_bins;
    M.atom0 = so[s];
    M.atom1 = so[s + 1];
    M.n_off = (2 * M.R[0] + 1) * (2 * M.R[1] + 1) * (2 * M.R[2] + 1);
    M.pad_ = 0;
    M.obase = n_opre;
    n_opre += (long long)M.n_off * (so[s + 1] - so[s]);
    if (nb_total > (1 << 30) - n_bins) return fail(ctx, SOAP_ENOTSUP, "too many cell-list bins");
    n_bins += nb_total;
  }
  const size_t up = sizeof(soap::StructMeta) * n_structures + sizeof(int) * (n_structures + 1);
  std::vector<char> img(up);
  std::memcpy(img.data(), meta.data(), sizeof(soap::StructMeta) * n_structures);
  std::memcpy(img.data() + sizeof(soap::StructMeta) * n_structures, so.data(), sizeof(int) * (n_structures + 1));
  const size_t meta_cap0 = ctx->meta.cap;
  SOAP_ENSURE(ctx, ctx->meta, up);
  if (ctx->meta.cap != meta_cap0) ctx->meta_dev = nullptr;  // a new allocation holds nothing yet
  SOAP_ENSURE(ctx, ctx->atom_bin, sizeof(int) * n_atoms);
  SOAP_ENSURE(ctx, ctx->atom_wrap, sizeof(int) * n_atoms);
  SOAP_ENSURE(ctx, ctx->bin_count, sizeof(int) * n_bins);
  SOAP_ENSURE(ctx, ctx->bin_start, sizeof(int) * (n_bins + 1));
  SOAP_ENSURE(ctx, ctx->bin_cursor, sizeof(int) * n_bins);
  SOAP_ENSURE(ctx, ctx->bin_cand, sizeof(soap::Cand) * n_atoms);
  SOAP_ENSURE(ctx, ctx->opre, sizeof(int) * (size_t)std::max(n_opre, 1LL));
  SOAP_ENSURE(ctx, ctx->bin_unsorted, sizeof(int) * n_atoms);
  SOAP_ENSURE(ctx, ctx->counts, sizeof(int) * n_atoms);
  SOAP_ENSURE(ctx, ctx->scan_part,
              sizeof(int) * (size_t)std::max(soap::scan_partials_needed(n_atoms), soap::scan_partials_needed(n_bins)));
  SOAP_ENSURE(ctx, ctx->errflag, sizeof(int) * 4);
  // the structure geometry is uploaded only when it differs from what the device holds
  if (ctx->meta.p != ctx->meta_dev || ctx->meta_host != img) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return fail(ctx, SOAP_ENOTSUP, "new structure geometry during stream capture (build once outside it first)");
    if (!ensure_pinned(ctx, std::max<size_t>(up, 64))) return fail(ctx, SOAP_ENOMEM, "pinned allocation failed");
    // the staging may still be read by the previous upload
    if (ctx->pinned_ev) SOAP_HIP(ctx, hipEventSynchronize(ctx->pinned_ev));
    else SOAP_HIP(ctx, hipEventCreateWithFlags(&ctx->pinned_ev, hipEventDisableTiming));
    std::memcpy(ctx->pinned, img.data(), up);
    SOAP_HIP(ctx, hipMemcpyAsync(ctx->meta.p, ctx->pinned, up, hipMemcpyHostToDevice, st));
    SOAP_HIP(ctx, hipEventRecord(ctx->pinned_ev, st));
    ctx->meta_host.swap(img);
    ctx->meta_dev = ctx->meta.p;
  }
  int* err = (int*)ctx->errflag.p;
  StageTimer tm(ctx, SOAP_STAGE_NEIGHBORS, st);
  const soap::StructMeta* dmeta = (const soap::StructMeta*)ctx->meta.p;
  const int* dso = (const int*)((const char*)ctx->meta.p + sizeof(soap::StructMeta) * n_structures);
  if (soap::bin_small_fits(n_atoms, n_bins)) {
    // the cell list of a small system in one launch
    SOAP_HIP(ctx, soap::launch_bin_small(n_atoms, pos, dmeta, dso, n_structures, n_bins, (int*)ctx->atom_bin.p,
                                         (int*)ctx->atom_wrap.p, (int*)ctx->bin_start.p, (soap::Cand*)ctx->bin_cand.p,
                                         err, st));
  } else {
    SOAP_HIP(ctx, soap::launch_init_build(n_bins, (int*)ctx->bin_count.p, (int*)ctx->bin_cursor.p, err, st));
    if (n_atoms > 0) {
      SOAP_HIP(ctx, soap::launch_bin_atoms(n_atoms, pos, dmeta, dso, n_structures, (int*)ctx->atom_bin.p,
                                           (int*)ctx->atom_wrap.p, (int*)ctx->bin_count.p, err, st));
    }
    SOAP_HIP(ctx, soap::scan_exclusive((const int*)ctx->bin_count.p, n_bins, (int*)ctx->bin_start.p,
                                       (int*)ctx->scan_part.p, st));
    if (n_atoms > 0) {
      SOAP_HIP(ctx, soap::launch_fill_bins(n_atoms, pos, (const int*)ctx->atom_bin.p, (const int*)ctx->atom_wrap.p,
                                           (const int*)ctx->bin_start.p, (int*)ctx->bin_cursor.p,
                                           (int*)ctx->bin_unsorted.p, (soap::Cand*)ctx->bin_cand.p, st));
    }
  }
  if (n_atoms > 0) {
    SOAP_HIP(ctx, soap::launch_pairs(false, n_atoms, pos, dmeta, dso, n_structures, rc, (const int*)ctx->atom_bin.p,
                                     (const int*)ctx->atom_wrap.p, (const int*)ctx->bin_start.p,
                                     (const soap::Cand*)ctx->bin_cand.p, (int*)ctx->counts.p, (int*)ctx->opre.p,
                                     nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, err,
                                     st));
  }
  SOAP_HIP(ctx, soap::scan_exclusive((const int*)ctx->counts.p, n_atoms, nl->offsets, (int*)ctx->scan_part.p, st));
  if (n_atoms > 0 && nl->capacity > 0) {
    SOAP_HIP(ctx, soap::launch_pairs(true, n_atoms, pos, dmeta, dso, n_structures, rc, (const int*)ctx->atom_bin.p,
                                     (const int*)ctx->atom_wrap.p, (const int*)ctx->bin_start.p,
                                     (const soap::Cand*)ctx->bin_cand.p, nullptr, (int*)ctx->opre.p, nl->offsets,
                                     nl->capacity, nl->j, nl->img, nl->center, nl->dx, nl->dy, nl->dz, nl->rev, err,
                                     st));
  }
  nl->n_atoms = n_atoms;
  nl->n_structures = n_structures;
  nl->n_pairs = SOAP_PAIRS_DEFERRED;
  ctx->built_atoms = n_atoms;
  ctx->built_structures = n_structures;
  return SOAP_OK;
}

// Waits for the last build on st and reads its pair count and error bits (one
// kernel writes both into pinned host memory).  Input errors come first, then
// capacity overflow (required_pairs holds the count needed).
soap_status read_report(soap_ctx* ctx, const soap_nlist* nl, long long* total_out, hipStream_t st) {
  if (!ctx->report) {
    if (hipHostMalloc((void**)&ctx->report, 64, hipHostMallocDefault) != hipSuccess) {
      ctx->report = nullptr;
      return fail(ctx, SOAP_ENOMEM, "pinned allocation failed");
    }
    if (hipHostGetDevicePointer((void**)&ctx->report_dev, ctx->report, 0) != hipSuccess) {
      hipHostFree(ctx->report);
      ctx->report = nullptr;
      return fail(ctx, SOAP_EHIP, "pinned report buffer has no device address");
    }
  }
  if (!ctx->errflag.p) return fail(ctx, SOAP_EINVAL, "no neighbour build on this context");
  SOAP_HIP(ctx, soap::launch_report(nl->offsets + nl->n_atoms, (const int*)ctx->errflag.p, ctx->report_dev, st));
  SOAP_HIP(ctx, hipStreamSynchronize(st));
  const long long total = ((volatile int*)ctx->report)[0];
  const int eb = ((volatile int*)ctx->report)[1];
  if (total_out) *total_out = total;
  if (eb & soap::kErrNonFinite) return fail(ctx, SOAP_EINVAL, "non-finite atomic position");
  if (eb & soap::kErrCoincident) return fail(ctx, SOAP_EINVAL, "coincident atoms (distance below 1e-8)");
  if (eb & soap::kErrFarOutside) return fail(ctx, SOAP_EINVAL, "atom more than 500 cells outside its cell");
  if (total < 0) return fail(ctx, SOAP_ENOTSUP, "pair count overflows 32-bit offsets");
  if (total > nl->capacity) return fail(ctx, SOAP_EOVERFLOW, "neighbour list capacity too small");
  return SOAP_OK;
}

}  // namespace

extern "C" {

soap_status soap_build_neighbors(soap_ctx* ctx, int n_atoms, const double* pos, const double* cells,
                                 const int32_t* pbc, const int32_t* struct_offsets, int n_structures,
                                 soap_nlist* nl, long long* required_pairs, hipStream_t st) {
  if (!ctx) return SOAP_EINVAL;
  soap_status s = enqueue_build(ctx, n_atoms, pos, cells, pbc, struct_offsets, n_structures, nl, st);
  if (s != SOAP_OK) return s;
  long long total = 0;
  s = read_report(ctx, nl, &total, st);
  if (required_pairs) *required_pairs = total;
  nl->n_pairs = s == SOAP_OK ? total : 0;
  return s;
}

soap_status soap_build_neighbors_async(soap_ctx* ctx, int n_atoms, const double* pos, const double* cells,
                                       const int32_t* pbc, const int32_t* struct_offsets, int n_structures,
                                       soap_nlist* nl, hipStream_t st) {
  if (!ctx) return SOAP_EINVAL;
  return enqueue_build(ctx, n_atoms, pos, cells, pbc, struct_offsets, n_structures, nl, st);
}

soap_status soap_neighbors_check(soap_ctx* ctx, const soap_nlist* nl, long long* n_pairs, hipStream_t st) {
  if (!ctx) return SOAP_EINVAL;
  if (!nl || !nl->offsets || nl->n_atoms < 0) return fail(ctx, SOAP_EINVAL, "null or empty neighbour list");
  return read_report(ctx, nl, n_pairs, st);
}

soap_status soap_descriptor(soap_ctx* ctx, const soap_nlist* nl, const int32_t* species, double* q, double* p_norm,
                            hipStream_t st) {
  if (!ctx) return SOAP_EINVAL;
  soap_status s = check_nlist(ctx, nl);
  if (s != SOAP_OK) return s;
  if ((s = check_lds(ctx)) != SOAP_OK) return s;
  if (nl->n_atoms > 0 && (!species || !q)) return fail(ctx, SOAP_EINVAL, "null species or output");
  double* pn = p_norm;
  if (!pn) {
    SOAP_ENSURE(ctx, ctx->pnorm, sizeof(double) * (size_t)nl->n_atoms);
    pn = (double*)ctx->pnorm.p;
  }
  return forward(ctx, nl, species, q, pn, false, st);
}

soap_status soap_descriptor_noalloc(soap_ctx* ctx, const soap_nlist* nl, const int32_t* species, double* q,
                                    double* p_norm, hipStream_t st) {
  if (!ctx) return SOAP_EINVAL;
  soap_status s = check_nlist(ctx, nl);
  if (s != SOAP_OK) return s;
  if ((s = check_lds(ctx)) != SOAP_OK) return s;
  if (nl->n_atoms > 0 && (!species || !q)) return fail(ctx, SOAP_EINVAL, "null species or output");
  const soap::DevParams& P = ctx->dp;
  const size_t N = (size_t)nl->n_atoms, NP = (size_t)pair_bound(nl);
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t b_rows = up(soap::pair_rows_bytes(P, (long long)NP));
  const size_t b_c = up(sizeof(double) * N * soap::c_doubles_per_atom(P));
  const size_t b_bc = up(sizeof(double) * soap::kMaxN);
  const size_t b_pn = p_norm ? 0 : up(sizeof(double) * N);
  const size_t need = b_rows + b_c + b_bc + b_pn;
  if (need > (size_t)SOAP_NOALLOC_SCRATCH_BYTES)
    return fail(ctx, SOAP_ENOTSUP,
                "soap_descriptor_noalloc needs " + std::to_string(need) + " bytes of scratch for " +
                    std::to_string(N) + " atoms and " + std::to_string(NP) + " pairs; it has " +
                    std::to_string((size_t)SOAP_NOALLOC_SCRATCH_BYTES));
  if (!ctx->scratch) return hip_fail(ctx, ctx->scratch_err, "soap_descriptor_noalloc scratch address");
  int cur = -1;
  SOAP_HIP(ctx, hipGetDevice(&cur));
  if (cur != ctx->device) return fail(ctx, SOAP_EINVAL, "the current device is not the context's");
  char* base = static_cast<char*>(ctx->scratch);
  double* rows = reinterpret_cast<double*>(base);
  double* c = reinterpret_cast<double*>(base + b_rows);
  double* bc = reinterpret_cast<double*>(base + b_rows + b_c);
  double* pn = p_norm ? p_norm : reinterpret_cast<double*>(base + b_rows + b_c + b_bc);
  return forward_into(ctx, nl, species, q, pn, false, st, rows, false, c, bc, nullptr, 0, false);
}

soap_status soap_descriptor_grad(soap_ctx* ctx, const soap_nlist* nl, const int32_t* species, const double* q_bar,
                                 double* pos_grad, hipStream_t st) {
  if (!ctx) return SOAP_EINVAL;
  soap_status s = check_nlist(ctx, nl);
  if (s != SOAP_OK) return s;
  if ((s = check_lds(ctx)) != SOAP_OK) return s;
  if (nl->n_atoms == 0) return SOAP_OK;
  if (!species || !q_bar || !pos_grad) return fail(ctx, SOAP_EINVAL, "null species, q_bar or pos_grad");
  const soap::DevParams& P = ctx->dp;
  const size_t N = (size_t)nl->n_atoms, NP = (size_t)pair_bound(nl);
  SOAP_ENSURE(ctx, ctx->q, sizeof(double) * N * P.K);
  SOAP_ENSURE(ctx, ctx->pnorm, sizeof(double) * N);
  SOAP_ENSURE(ctx, ctx->gx, 4 * sizeof(double) * NP);  // (x, y, z, 0) per pair
  if ((s = forward(ctx, nl, species, (double*)ctx->q.p, (double*)ctx->pnorm.p, true, st)) != SOAP_OK) return s;
  {
    StageTimer tm(ctx, SOAP_STAGE_PAIR_ADJOINT, st);
    SOAP_HIP(ctx, soap::launch_pair_adjoint(P, ctx->dt, nl->n_atoms, nl->offsets, (int)NP, nl->j, species,
                                            ctx->rows.p, false, ctx->c.p,
                                            (const double*)ctx->q.p, P.K, (const double*)ctx->pnorm.p, q_bar, nullptr,
                                            P.K, (double*)ctx->gx.p, nullptr, nullptr, 4, st));
  }
  StageTimer tm(ctx, SOAP_STAGE_FORCE_GATHER, st);
  SOAP_HIP(ctx, soap::launch_force_gather(nl->n_atoms, nl->offsets, (int)NP, nl->rev, (const double*)ctx->gx.p,
                                          pos_grad, true, st));
  return SOAP_OK;
}

soap_status soap_descriptor_jacobian(soap_ctx* ctx, const soap_nlist* nl, const int32_t* species, int k0, int k1,
                                     double* jac, hipStream_t st) {
  if (!ctx) return SOAP_EINVAL;
  soap_status s = check_nlist(ctx, nl);
  if (s != SOAP_OK) return s;
  if ((s = check_lds(ctx)) != SOAP_OK) return s;
  const soap::DevParams& P = ctx->dp;
  if (k0 < 0 || k1 > P.K || k0 >= k1) return fail(ctx, SOAP_EINVAL, "need 0 <= k0 < k1 <= K");
  if (nl->n_atoms == 0) return SOAP_OK;
  if (!species || !jac) return fail(ctx, SOAP_EINVAL, "null species or Jacobian");
  const size_t N = (size_t)nl->n_atoms, NP = (size_t)pair_bound(nl);
  SOAP_ENSURE(ctx, ctx->q, sizeof(double) * N * P.K);
  SOAP_ENSURE(ctx, ctx->pnorm, sizeof(double) * N);
  SOAP_ENSURE(ctx, ctx->qbar, sizeof(double) * N * P.K);
  if ((s = forward(ctx, nl, species, (double*)ctx->q.p, (double*)ctx->pnorm.p, true, st)) != SOAP_OK) return s;
  // column k of every atom's Jacobian: the pair adjoint with qbar = e_k on every
  // row (each q_i depends on the pairs of centre i only)
  double* qb = (double*)ctx->qbar.p;
  for (int k = k0; k < k1; ++k) {
    SOAP_HIP(ctx, soap::launch_unit_rows((int)N, P.K, k, k == k0 ? -1 : k - 1, qb, st));
    double* tile = jac + (size_t)(k - k0) * 3 * NP;
    StageTimer tm(ctx, SOAP_STAGE_PAIR_ADJOINT, st);
    SOAP_HIP(ctx, soap::launch_pair_adjoint(P, ctx->dt, nl->n_atoms, nl->offsets, (int)NP, nl->j, species,
                                            ctx->rows.p, false, ctx->c.p,
                                            (const double*)ctx->q.p, P.K, (const double*)ctx->pnorm.p, qb, nullptr, P.K,
                                            tile, tile + NP, tile + 2 * NP, 1, st));
  }
  return SOAP_OK;
}

soap_status gap_energy_forces(soap_ctx* ctx, const soap_nlist* nl, const int32_t* species, const double* q_sparse,
                              const double* alpha, int M, int zeta, double* e_atom, double* forces,
                              double* alpha_grad, hipStream_t st) {
  if (!ctx) return SOAP_EINVAL;
  soap_status s = check_nlist(ctx, nl);
  if (s != SOAP_OK) return s;
  if ((s = check_lds(ctx)) != SOAP_OK) return s;
  if (M < 1 || zeta < 1) return fail(ctx, SOAP_EINVAL, "M and zeta must be >= 1");
  if (!q_sparse || !alpha) return fail(ctx, SOAP_EINVAL, "null sparse set or weights");
  if (nl->n_atoms > 0 && (!species || !e_atom)) return fail(ctx, SOAP_EINVAL, "null species or energies");
  const soap::DevParams& P = ctx->dp;
  const size_t N = (size_t)nl->n_atoms, NP = (size_t)pair_bound(nl);
  if (N == 0) {
    if (alpha_grad) SOAP_HIP(ctx, soap::launch_fill(alpha_grad, M, 0.0, st));  // a kernel, capturable
    return SOAP_OK;
  }
  SOAP_ENSURE(ctx, ctx->q, sizeof(double) * N * P.K);
  SOAP_ENSURE(ctx, ctx->pnorm, sizeof(double) * N);
  const int prec = gap_precision(ctx);
  const bool fused = forces && ctx->tune.gap_fused && soap::gap_fused_supported(P.K, prec);
  // unfused BF16: the descriptor kernel also writes the bf16 operand copy of q
  // into the GAP workspace, and the scores pass converts only the sparse set
  void* qc = nullptr;
  if (!fused) {
    SOAP_ENSURE(ctx, ctx->gapw, soap::gap_workspace_bytes((int)N, M, P.K, prec));
    qc = soap::gap_q_operand(prec, (int)N, M, P.K, ctx->gapw.p);
  }
  // the mixed modes store the pair fields, c and Qbar in FP32 (their rounding,
  // about 6e-8 relative, is far below that of the GAP operands; Qbar is an FP32
  // accumulator there anyway); the arithmetic stays FP64
  const bool store_f32 = prec != 0 && !P.radial_dd;
  const size_t es = store_f32 ? sizeof(float) : sizeof(double);
  if ((s = forward(ctx, nl, species, (double*)ctx->q.p, (double*)ctx->pnorm.p, forces != nullptr, st, qc,
                   soap::gap_q_pitch(P.K), store_f32)) != SOAP_OK)
    return s;
  // the unfused Qbar pass splits its contraction over the sparse points into
  // parts that the adjoint adds
  const int slices = fused ? 1 : soap::gap_qbar_slices((int)N, M, P.K, prec, ctx->tune.gap_tile);
  void* qbar = nullptr;
  if (forces) {
    SOAP_ENSURE(ctx, ctx->qbar, es * slices * N * P.K);
    qbar = ctx->qbar.p;
  }
  if (fused) {
    const int target = ctx->tune.gap_slices > 0 ? ctx->tune.gap_slices : 512;
    SOAP_ENSURE(ctx, ctx->gapw, soap::gap_fused_workspace_bytes((int)N, M, P.K, prec, target));
    StageTimer tm(ctx, SOAP_STAGE_GAP_FUSED, st);
    SOAP_HIP(ctx, soap::launch_gap_fused(prec, (int)N, M, P.K, (const double*)ctx->q.p, q_sparse, alpha, zeta, e_atom,
                                         alpha_grad, qbar, store_f32, ctx->gapw.p, target, st));
  } else {
    {
      StageTimer tm(ctx, SOAP_STAGE_GAP_SCORES, st);
      // with forces the Qbar pass also finishes the energy and dE/dalpha sums
      SOAP_HIP(ctx, soap::launch_gap_scores(prec, (int)N, M, P.K, (const double*)ctx->q.p, q_sparse, alpha, zeta,
                                            e_atom, alpha_grad, qbar == nullptr, qc != nullptr, ctx->gapw.p,
                                            ctx->tune.gap_tile, st));
    }
    if (qbar) {
      StageTimer tm(ctx, SOAP_STAGE_GAP_QBAR, st);
      SOAP_HIP(ctx, soap::launch_gap_qbar(prec, (int)N, M, P.K, qbar, store_f32, e_atom, alpha_grad, ctx->gapw.p,
                                          slices, ctx->tune.gap_tile, st));
    }
  }
  if (forces) {
    SOAP_ENSURE(ctx, ctx->gx, 4 * sizeof(double) * NP);  // (x, y, z, 0) per pair
    {
      StageTimer tm(ctx, SOAP_STAGE_PAIR_ADJOINT, st);
      SOAP_HIP(ctx, soap::launch_pair_adjoint(P, ctx->dt, nl->n_atoms, nl->offsets, (int)NP, nl->j, species,
                                              ctx->rows.p, store_f32, ctx->c.p, (const double*)ctx->q.p, P.K,
                                              (const double*)ctx->pnorm.p, qbar,
                                              slices == 2 ? (char*)qbar + es * N * P.K : nullptr, P.K,
                                              (double*)ctx->gx.p, nullptr, nullptr, 4, st));
    }
    StageTimer tm(ctx, SOAP_STAGE_FORCE_GATHER, st);
    SOAP_HIP(ctx, soap::launch_force_gather(nl->n_atoms, nl->offsets, (int)NP, nl->rev, (const double*)ctx->gx.p,
                                            forces, false, st));
  }
  return SOAP_OK;
}

soap_status soap_update_pair_vectors(soap_ctx* ctx, const soap_nlist* nl, const double* pos, hipStream_t st) {
  if (!ctx) return SOAP_EINVAL;
  soap_status s = check_nlist(ctx, nl);
  if (s != SOAP_OK) return s;
  if (nl->n_atoms != ctx->built_atoms || nl->n_structures != ctx->built_structures || !ctx->meta.p)
    return fail(ctx, SOAP_EINVAL, "the list does not match the last build on this context");
  if (nl->n_atoms > 0 && !pos) return fail(ctx, SOAP_EINVAL, "null positions");
  const int ns = nl->n_structures;
  const soap::StructMeta* dmeta = (const soap::StructMeta*)ctx->meta.p;
  const int* dso = (const int*)((const char*)ctx->meta.p + sizeof(soap::StructMeta) * ns);
  SOAP_HIP(ctx, soap::launch_pair_vectors(pair_bound(nl), pair_count(nl), pos, dmeta, dso, ns, nl->center, nl->j,
                                          nl->img, nl->dx, nl->dy, nl->dz, st));
  return SOAP_OK;
}

soap_status soap_set_neighbor_skin(soap_ctx* ctx, double skin) {
  if (!ctx) return SOAP_EINVAL;
  if (!(skin >= 0.0) || !(skin <= ctx->dp.rc)) return fail(ctx, SOAP_EINVAL, "skin must be in [0, r_cut]");
  ctx->skin = skin;
  return SOAP_OK;
}

soap_status soap_get_tuning(const soap_ctx* ctx, soap_tuning* out) {
  if (!ctx || !out) return SOAP_EINVAL;
  *out = ctx->tune;
  return SOAP_OK;
}

soap_status soap_set_tuning(soap_ctx* ctx, const soap_tuning* t) {
  if (!ctx || !t) return SOAP_EINVAL;
  if ((t->gap_fused != 0 && t->gap_fused != 1) || t->gap_slices < 0 || t->gap_slices > (1 << 20) ||
      (t->prep_block != 64 && t->prep_block != 128 && t->prep_block != 256) || t->cell_split < 1 ||
      t->cell_split > 3 || (t->gap_tile != 0 && t->gap_tile != 1))
    return fail(ctx, SOAP_EINVAL, "tuning field out of range");
  ctx->tune = *t;
  return SOAP_OK;
}

soap_status soap_autotune(soap_ctx* ctx, const soap_nlist* nl, const int32_t* species, const double* q_sparse,
                          const double* alpha, int M, int zeta, int repeats, soap_tuning* chosen, hipStream_t st) {
  if (!ctx) return SOAP_EINVAL;
  if (!nl || repeats < 1) return fail(ctx, SOAP_EINVAL, "null neighbour list or repeats < 1");
  soap_tuning_key key{};
  const bool cached = !ctx->tune_cache.empty();
  if (cached) {
    soap_status ks = soap_tuning_key_for(ctx, nl->n_atoms, M, &key);
    if (ks != SOAP_OK) return fail(ctx, ks, "tuning key: device query failed");
    soap_tuning hit{};
    int found = 0;
    if (soap_tuning_cache_lookup(ctx->tune_cache.c_str(), &key, &hit, &found) == SOAP_OK && found &&
        soap_set_tuning(ctx, &hit) == SOAP_OK) {
      ++ctx->tune_cache_hits;
      if (chosen) *chosen = hit;
      return SOAP_OK;
    }
  }
  const size_t N = (size_t)std::max(0, nl->n_atoms);
  SOAP_ENSURE(ctx, ctx->tune_out, sizeof(double) * (4 * N + (size_t)std::max(M, 0) + 1));
  double* e = (double*)ctx->tune_out.p;
  double* F = e + N;
  double* ab = F + 3 * N;
  const unsigned prof = ctx->prof_mask;
  ctx->prof_mask = 0;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    ctx->prof_mask = prof;
    return fail(ctx, SOAP_EHIP, "event creation failed");
  }
  auto time_it = [&](float& ms) -> soap_status {
    soap_status s = gap_energy_forces(ctx, nl, species, q_sparse, alpha, M, zeta, e, F, ab, st);  // warm-up
    if (s != SOAP_OK) return s;
    if (hipEventRecord(a, st) != hipSuccess) return fail(ctx, SOAP_EHIP, "event record failed");
    for (int r = 0; r < repeats; ++r)
      if ((s = gap_energy_forces(ctx, nl, species, q_sparse, alpha, M, zeta, e, F, ab, st)) != SOAP_OK) return s;
    if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&ms, a, b) != hipSuccess)
      return fail(ctx, SOAP_EHIP, "event timing failed");
    return SOAP_OK;
  };
  soap_tuning best = ctx->tune;
  float best_ms = 0.0f;
  soap_status s = time_it(best_ms);
  const bool fusable = soap::gap_fused_supported(ctx->dp.K, gap_precision(ctx));
  const bool tiles = gap_precision(ctx) == SOAP_MIXED_BF16;  // two BF16 tile shapes
  struct Axis {
    int soap_tuning::*field;
    std::vector<int> cand;
  };
  const std::vector<Axis> axes = {
      {&soap_tuning::prep_block, {64, 128, 256}},
      {&soap_tuning::gap_fused, fusable ? std::vector<int>{0, 1} : std::vector<int>{0}},
      {&soap_tuning::gap_slices, fusable ? std::vector<int>{256, 512, 1024, 2048} : std::vector<int>{}},
      {&soap_tuning::gap_tile, tiles ? std::vector<int>{0, 1} : std::vector<int>{}},
  };
  for (const Axis& ax : axes) {
    if (s != SOAP_OK) break;
    if (ax.field == &soap_tuning::gap_slices && !best.gap_fused) continue;
    if (ax.field == &soap_tuning::gap_tile && best.gap_fused) continue;
    for (int v : ax.cand) {
      if (v == best.*ax.field) continue;
      ctx->tune = best;
      ctx->tune.*ax.field = v;
      float ms = 0.0f;
      if ((s = time_it(ms)) != SOAP_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best = ctx->tune;
      }
    }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  ctx->tune = best;
  ctx->prof_mask = prof;
  if (s != SOAP_OK) return s;
  if (chosen) *chosen = best;
  if (cached && soap_tuning_cache_store(ctx->tune_cache.c_str(), &key, &best) != SOAP_OK)
    return fail(ctx, SOAP_ENOMEM, "tuning cache: cannot write " + ctx->tune_cache);
  return SOAP_OK;
}

soap_status soap_autotune_neighbors(soap_ctx* ctx, int n_atoms, const double* pos, const double* cells,
                                    const int32_t* pbc, const int32_t* struct_offsets, int n_structures,
                                    soap_nlist* nl, int repeats, soap_tuning* chosen, hipStream_t st) {
  if (!ctx) return SOAP_EINVAL;
  if (!nl || repeats < 1) return fail(ctx, SOAP_EINVAL, "null neighbour list or repeats < 1");
  const soap_tuning start = ctx->tune;
  const unsigned prof = ctx->prof_mask;
  ctx->prof_mask = 0;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    ctx->prof_mask = prof;
    return fail(ctx, SOAP_EHIP, "event creation failed");
  }
  soap_status s = SOAP_OK;
  soap_tuning best = start;
  float best_ms = 0.0f;
  for (int split = 1; split <= 3 && s == SOAP_OK; ++split) {
    ctx->tune = start;
    ctx->tune.cell_split = split;
    // warm-up build, checked: every setting lists the same pairs, so an
    // overflow here is an overflow for all of them
    s = soap_build_neighbors_async(ctx, n_atoms, pos, cells, pbc, struct_offsets, n_structures, nl, st);
    if (s == SOAP_OK) s = soap_neighbors_check(ctx, nl, nullptr, st);
    if (s != SOAP_OK) break;
    if (hipEventRecord(a, st) != hipSuccess) {
      s = fail(ctx, SOAP_EHIP, "event record failed");
      break;
    }
    for (int r = 0; r < repeats && s == SOAP_OK; ++r)
      s = soap_build_neighbors_async(ctx, n_atoms, pos, cells, pbc, struct_offsets, n_structures, nl, st);
    float ms = 0.0f;
    if (s == SOAP_OK && (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                         hipEventElapsedTime(&ms, a, b) != hipSuccess))
      s = fail(ctx, SOAP_EHIP, "event timing failed");
    if (s == SOAP_OK && (split == 1 || ms < best_ms)) {
      best_ms = ms;
      best = ctx->tune;
    }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  ctx->prof_mask = prof;
  ctx->tune = s == SOAP_OK ? best : start;
  if (s != SOAP_OK) return s;
  // the list of the chosen setting, with the host-side count
  long long required = 0;
  if ((s = soap_build_neighbors(ctx, n_atoms, pos, cells, pbc, struct_offsets, n_structures, nl, &required, st)) !=
      SOAP_OK)
    return s;
  if (chosen) *chosen = best;
  return SOAP_OK;
}

// ------------------------------------------------------------ tuning cache
namespace {

bool key_text(const soap_tuning_key* k, std::string& out) {
  const size_t n = strnlen(k->arch, sizeof(k->arch));
  if (n == 0 || n == sizeof(k->arch)) return false;
  for (size_t t = 0; t < n; ++t)
    if (k->arch[t] <= ' ' || k->arch[t] > '~') return false;  // one printable token
  std::ostringstream o;
  o << "soap-tuning " << k->version << ' ' << std::string(k->arch, n) << ' ' << k->n_channels << ' ' << k->l_max
    << ' ' << k->K << ' ' << k->M << ' ' << k->precision << ' ' << k->radial_dd << ' ' << k->size_class;
  out = o.str();
  return true;
}

// the setting of a line "<key text> = a b c d e" whose key text equals `key`
bool parse_entry(const std::string& line, const std::string& key, soap_tuning& t) {
  const size_t eq = line.find(" = ");
  if (eq == std::string::npos || line.compare(0, eq, key) != 0 || eq != key.size()) return false;
  std::istringstream v(line.substr(eq + 3));
  soap_tuning r{};
  if (!(v >> r.gap_fused >> r.gap_slices >> r.prep_block >> r.cell_split >> r.gap_tile)) return false;
  std::string rest;
  if (v >> rest) return false;
  t = r;
  return true;
}

}  // namespace

soap_status soap_tuning_key_for(const soap_ctx* ctx, int n_atoms, int M, soap_tuning_key* out) {
  if (!ctx || !out || n_atoms < 0 || M < 0) return SOAP_EINVAL;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) return SOAP_EHIP;
  soap_tuning_key k{};
  k.version = SOAP_TUNING_CACHE_VERSION;
  k.n_channels = ctx->dp.nch;
  k.l_max = ctx->prm.l_max;
  k.K = ctx->dp.K;
  k.M = M;
  k.precision = (int)ctx->prm.precision;
  k.radial_dd = ctx->dp.radial_dd;
  int c = 0;
  for (long long v = n_atoms; v > 0; v >>= 1) ++c;
  k.size_class = c;
  size_t t = 0;
  for (; t + 1 < sizeof(k.arch) && prop.gcnArchName[t] && prop.gcnArchName[t] != ':'; ++t)
    k.arch[t] = prop.gcnArchName[t];
  k.arch[t] = '\0';
  *out = k;
  return SOAP_OK;
}

soap_status soap_tuning_cache_lookup(const char* path, const soap_tuning_key* key, soap_tuning* out, int* found) {
  if (!path || !key || !out || !found) return SOAP_EINVAL;
  *found = 0;
  std::string kt;
  if (!key_text(key, kt)) return SOAP_EINVAL;
  std::ifstream f(path);
  if (!f) return SOAP_OK;  // no file: an empty cache
  std::string line;
  while (std::getline(f, line)) {
    soap_tuning t{};
    if (parse_entry(line, kt, t)) {  // the last matching entry wins
      *out = t;
      *found = 1;
    }
  }
  return SOAP_OK;
}

soap_status soap_tuning_cache_store(const char* path, const soap_tuning_key* key, const soap_tuning* t) {
  if (!path || !key || !t) return SOAP_EINVAL;
  std::string kt;
  if (!key_text(key, kt)) return SOAP_EINVAL;
  std::vector<std::string> lines;
  {
    std::ifstream f(path);
    std::string line;
    soap_tuning dummy{};
    while (f && std::getline(f, line))
      if (!parse_entry(line, kt, dummy)) lines.push_back(line);
  }
  std::ostringstream e;
  e << kt << " = " << t->gap_fused << ' ' << t->gap_slices << ' ' << t->prep_block << ' ' << t->cell_split << ' '
    << t->gap_tile;
  lines.push_back(e.str());
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream o(tmp, std::ios::trunc);
    for (const std::string& l : lines) o << l << '\n';
    o.flush();
    if (!o) {
      std::remove(tmp.c_str());
      return SOAP_ENOMEM;
    }
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return SOAP_ENOMEM;
  }
  return SOAP_OK;
}

soap_status soap_set_tuning_cache(soap_ctx* ctx, const char* path) {
  if (!ctx) return SOAP_EINVAL;
  ctx->tune_cache = path ? path : "";
  return SOAP_OK;
}

long long soap_tuning_cache_hits(const soap_ctx* ctx) { return ctx ? ctx->tune_cache_hits : -1; }

soap_status soap_profile(soap_ctx* ctx, int enable) {
  if (!ctx) return SOAP_EINVAL;
  ctx->prof_mask = enable ? ~0u : 0u;
  return SOAP_OK;
}

soap_status soap_profile_stages(soap_ctx* ctx, unsigned mask) {
  if (!ctx) return SOAP_EINVAL;
  ctx->prof_mask = mask;
  return SOAP_OK;
}

soap_status soap_profile_read(soap_ctx* ctx, double* ms, long long* launches) {
  if (!ctx || !ms || !launches) return SOAP_EINVAL;
  for (int k = 0; k < SOAP_STAGE_COUNT; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  soap_status res = SOAP_OK;
  for (auto& r : ctx->prof) {
    float t = 0.0f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
      res = fail(ctx, SOAP_EHIP, "event timing failed");
    } else {
      ms[r.stage] += t;
      launches[r.stage] += 1;
    }
    ctx->ev_pool.push_back(r.a);
    ctx->ev_pool.push_back(r.b);
  }
  ctx->prof.clear();
  return res;
}

const char* soap_stage_name(int stage) {
  static const char* names[SOAP_STAGE_COUNT] = {"neighbors",    "descriptor", "gap_scores", "gap_qbar",
                                                "pair_adjoint", "force_gather", "gap_fused", "pair_prep",
                                                "cbar",         "pair_angular"};
  return (stage >= 0 && stage < SOAP_STAGE_COUNT) ? names[stage] : "unknown";
}

soap_status soap_radial_basis_table(int n_max, double r_cut, double sigma0_r, double* W, double* lambda) {
  if (n_max < 2 || n_max > soap::kMaxN || !(r_cut > 0) || !(sigma0_r > 0) || !W) return SOAP_EINVAL;
  return soap_host_basis_table(n_max, r_cut, sigma0_r, W, nullptr, lambda) == 0 ? SOAP_OK : SOAP_EINVAL;
}

}  // extern "C"
