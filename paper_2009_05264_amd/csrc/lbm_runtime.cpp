// Host runtime of the C ABI declared in include/lbmflow.h: parameter
// validation, device memory layout, wall maps, initial state, stepping,
// read-out, diagnostics, checkpoints and the Maxwell helper.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbmflow.h"
#include "lbm_internal.h"
#include "lbm_runtime.h"

using namespace lbm;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

int lbm_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHECK(expr)                                                                     \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return lbm_fail(LBM_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

extern "C" const char* lbm_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ physics helpers (host, FP64)
namespace {

double crit_T(const lbm_params& p) { return 0.0778 * p.a / (0.45724 * p.b * p.R); }
double kappa_of(const lbm_params& p) {
  return 0.37464 + 1.54226 * p.omega - 0.26992 * p.omega * p.omega;
}
// Peng-Robinson pressure (Eq. 12).
double pr_p(const lbm_params& P, double rho, double T) {
  const double s = std::sqrt(T / crit_T(P));
  const double sa = 1.0 + kappa_of(P) * (1.0 - s);
  return rho * P.R * T / (1.0 - P.b * rho) -
         P.a * sa * sa * rho * rho / (1.0 + 2.0 * P.b * rho - P.b * P.b * rho * rho);
}
// Pseudopotential (Eq. 11) at (rho, T), 0 where p - rho/3 has the wrong sign.
double pr_psi(const lbm_params& P, double rho, double T) {
  const double q = 2.0 * (pr_p(P, rho, T) - rho / 3.0) / (P.c0 * P.g);
  return q > 0.0 ? std::sqrt(q) : 0.0;
}

unsigned long long splitmix64_host(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int rates(const lbm_params& p, double* s_nu, double* s_e, double* s_eps, double* s_q) {
  *s_nu = 1.0 / p.tau_f;
  *s_e = p.s_e > 0 ? p.s_e : *s_nu;
  *s_eps = p.s_eps > 0 ? p.s_eps : *s_nu;
  *s_q = p.s_q > 0 ? p.s_q : 8.0 * (2.0 - *s_nu) / (8.0 - *s_nu);
  return 0;
}

int validate(const lbm_params* p) {
  if (!p) return lbm_fail(LBM_E_INVALID, "params is NULL");
  if (p->nx < 3 || p->ny < 3 || p->nx > 32767 || p->ny > 32767)
    return lbm_fail(LBM_E_INVALID, "nx, ny must lie in [3, 32767] (got %d x %d)", p->nx, p->ny);
  if (p->storage < LBM_STORE_F32 || p->storage > LBM_STORE_BF16_DEV)
    return lbm_fail(LBM_E_INVALID, "unknown storage %d", p->storage);
  if ((p->bc_x != LBM_BCX_PERIODIC && p->bc_x != LBM_BCX_CHANNEL && p->bc_x != LBM_BCX_CHANNEL_P) ||
      (p->bc_y != LBM_BCY_PERIODIC && p->bc_y != LBM_BCY_WALLS))
    return lbm_fail(LBM_E_INVALID, "unknown boundary kind");
  if (!(p->tau_f > 0.5) || !(p->tau_g > 0.5))
    return lbm_fail(LBM_E_INVALID, "tau_f and tau_g must exceed 1/2");
  double sn, se, sp, sq;
  rates(*p, &sn, &se, &sp, &sq);
  if (!(se > 0 && se < 2) || !(sp > 0 && sp < 2) || !(sq > 0 && sq < 2))
    return lbm_fail(LBM_E_INVALID, "MRT rates must lie in (0, 2)");
  if (!(p->c_v > 0)) return lbm_fail(LBM_E_INVALID, "c_v must be positive");
  if (!(std::fabs(p->u_in) < 0.1)) return lbm_fail(LBM_E_INVALID, "|u_in| must be < 0.1");
  if (!(p->T_in > 0) || !(p->T_iso > 0))
    return lbm_fail(LBM_E_INVALID, "temperatures must be positive");
  if (!(p->a > 0) || !(p->b > 0) || !(p->R > 0) || !(p->c0 > 0) || p->g == 0)
    return lbm_fail(LBM_E_INVALID, "EOS constants out of range");
  if (!std::isfinite(p->G_wet) || !std::isfinite(p->beta))
    return lbm_fail(LBM_E_INVALID, "G_wet and beta must be finite");
  if (p->bc_x != LBM_BCX_PERIODIC && p->nx < 3)
    return lbm_fail(LBM_E_INVALID, "a channel needs nx >= 3");
  if (p->bc_x == LBM_BCX_CHANNEL_P && !(p->rho_out > 0))
    return lbm_fail(LBM_E_INVALID, "a constant-pressure outlet needs rho_out > 0");
  {
    // The kernels address a state buffer with 32-bit byte offsets: its ny
    // rows of 9 direction planes, plus the base shift of the boundary pull
    // (a row, a column and two planes), must stay below 2 GB (checked with
    // two planes of margin per row).
    const bool half = p->storage == LBM_STORE_F16_DEV || p->storage == LBM_STORE_BF16_DEV;
    const double e2 = (half ? 2.0 : 4.0) * (p->isothermal ? 1.0 : 2.0);
    const double pitch = (double)lbm_pitch(p->nx);
    if (11.0 * pitch * (p->ny + 2.0) * e2 > 2147483648.0 - 16777216.0)
      return lbm_fail(LBM_E_INVALID, "domain %d x %d too large for one state buffer (32-bit offsets)", p->nx,
                      p->ny);
  }
  return LBM_OK;
}

}  // namespace

// ------------------------------------------------------------------ layout
namespace {

struct Layout {
  size_t state, fold, psiw, Tw, heater, partials, rpart, l1, macc, mhist, rbar, nff, ring, stepc, out, desc, self,
      tiles, total;
  size_t state_bytes, fold_bytes;
};

int elem_bytes(int storage) { return storage == LBM_STORE_F16_DEV || storage == LBM_STORE_BF16_DEV ? 2 : 4; }
int max_tiles(const lbm_params& p) {
  // column-edge strips (at most two) may be cut into single rows
  const int strips = (p.nx + kStripInterior - 1) / kStripInterior;
  const int t = std::min(strips, 2) * p.ny + strips * ((p.ny + kMinTileRows - 1) / kMinTileRows + 2);
  return (t + 63) / 64 * 64;  // also the stride of the SoA partial sums
}

Layout layout_of(const lbm_params& p) {
  Layout L{};
  // ny rows of 9 direction planes of pitch (f, g) pairs (f alone when isothermal)
  const size_t per_node = p.isothermal ? 9 : 18;
  const size_t nodes = (size_t)lbm_pitch(p.nx) * p.ny;
  L.state_bytes = align_up(per_node * nodes * elem_bytes(p.storage), 256);
  L.fold_bytes = align_up(3 * (size_t)p.ny * sizeof(float), 256);
  const size_t mt = max_tiles(p);
  size_t o = 0;
  L.state = o; o += 2 * L.state_bytes;
  L.fold = o; o += 2 * L.fold_bytes;
  L.psiw = o; o += 2 * align_up(p.nx * sizeof(float), 256);
  L.Tw = o; o += 2 * align_up(p.nx * sizeof(float), 256);
  L.heater = o; o += align_up(p.nx * sizeof(int), 256);
  L.partials = o; o += 2 * align_up(mt * kPartials * sizeof(double), 256);
  L.rpart = o; o += align_up(mt * kPartials * sizeof(double), 256);
  L.l1 = o; o += 2 * align_up(kFin * kPartials * sizeof(double), 256);
  L.macc = o; o += 2 * align_up(kAccSlots * kAccStride * sizeof(unsigned long long), 256);
  L.mhist = o; o += 2 * align_up(mt * sizeof(unsigned long long), 256);
  L.rbar = o; o += 256;
  L.nff = o; o += 256;
  L.ring = o; o += align_up(kRing * sizeof(DiagRec), 256);
  L.stepc = o; o += 256;
  L.out = o; o += 4 * align_up((size_t)p.nx * p.ny * sizeof(float), 256);
  L.desc = o; o += align_up(sizeof(DevDomain), 256);
  L.self = o; o += align_up(kFin * sizeof(FinEntry), 256);
  L.tiles = o; o += align_up(mt * sizeof(Tile), 256);
  L.total = o;
  return L;
}

}  // namespace

// ------------------------------------------------------------------ API
extern "C" double lbm_neutral_G_wet(const lbm_params* p) {
  // A flat wall removes the solid neighbours from both sums of Eq. 9, whose
  // missing pull is (1 + beta)/2 sum_solid G_i psi^2 c_i; with G_i = 18 g w_i
  // (Eq. 10 on D2Q9) Eq. 15 returns it exactly when G_wet = 9 g (1 + beta).
  return p ? 9.0 * p->g * (1.0 + p->beta) : 0.0;
}

extern "C" int lbm_params_default(lbm_params* p) {
  if (!p) return lbm_fail(LBM_E_INVALID, "params is NULL");
  memset(p, 0, sizeof(*p));
  p->nx = 200;
  p->ny = 50;
  p->storage = LBM_STORE_F32;
  p->bc_x = LBM_BCX_CHANNEL;
  p->bc_y = LBM_BCY_WALLS;
  p->a = 2.0 / 49.0;
  p->b = 2.0 / 21.0;
  p->R = 1.0;
  p->omega = 0.344;
  p->beta = 1.16;
  p->c0 = 6.0;
  p->g = -1.0;
  p->tau_f = 1.0;
  p->s_e = p->s_eps = p->s_q = 0.0;
  p->tau_g = 0.6;
  p->c_v = 6.0;
  p->ga_x = 0.0;
  p->ga_y = -5e-5;
  const double Tc = crit_T(*p);
  const double Ts = 0.86 * Tc;
  p->u_in = 0.005;
  p->T_in = 0.95 * Ts;
  p->U_out = -1.0;
  p->T_iso = Ts;
  // saturated densities at 0.86 Tc (Maxwell construction of these constants)
  p->rho_mid = 0.5 * (6.4989457632878835 + 0.3796789993997205);
  p->rho_out = 6.4989457632878835;
  p->rho_ref = 0.0;
  p->T_ref = 0.0;
  p->G_wet = lbm_neutral_G_wet(p);
  return LBM_OK;
}

extern "C" int lbm_required_bytes(const lbm_params* p, size_t* bytes) {
  int rc = validate(p);
  if (rc) return rc;
  if (!bytes) return lbm_fail(LBM_E_INVALID, "bytes is NULL");
  *bytes = layout_of(*p).total;
  return LBM_OK;
}

namespace {

void fill_desc(lbm_domain* d) {
  const lbm_params& p = d->P;
  DevDomain& D = d->host;
  const double Tc = crit_T(p);
  double s_nu, s_e, s_eps, s_q;
  rates(p, &s_nu, &s_e, &s_eps, &s_q);
  D.nx = p.nx;
  D.ny = p.ny;
  D.pitch = lbm_pitch(p.nx);
  D.storage = p.storage;
  D.bc_x = p.bc_x;
  D.bc_y = p.bc_y;
  D.isothermal = p.isothermal;
  D.single_phase = p.single_phase;
  D.a = (float)p.a;
  D.b = (float)p.b;
  D.R = (float)p.R;
  D.kappa = (float)kappa_of(p);
  D.Tc = (float)Tc;
  D.beta = (float)p.beta;
  // Eq. 15 with G_i = 18 g w_i (Eq. 10 on D2Q9): G_wet w_i = (G_wet / 18 g) G_i
  D.kw = (float)(p.G_wet / (18.0 * p.g));
  D.c0g2 = (float)(2.0 / (p.c0 * p.g));
  D.G1 = (float)(2.0 * p.g);
  D.G2 = (float)(0.5 * p.g);
  D.half_1mb = (float)(0.5 * (1.0 - p.beta));
  D.s_e = (float)s_e;
  D.s_eps = (float)s_eps;
  D.s_q = (float)s_q;
  D.s_nu = (float)s_nu;
  D.omega_g = (float)(1.0 / p.tau_g);
  D.inv_cv = (float)(1.0 / p.c_v);
  D.ga_x = (float)p.ga_x;
  D.ga_y = (float)p.ga_y;
  D.fb_x = (float)p.fb_x;
  D.fb_y = (float)p.fb_y;
  D.u_in = (float)p.u_in;
  D.T_in = (float)p.T_in;
  const double U = p.U_out >= 0 ? p.U_out : p.u_in;
  D.U_out = (float)U;
  D.inv_1pU = (float)(1.0 / (1.0 + U));
  D.in_geq = (float)(p.T_in * (1.0 + 3.0 * p.u_in * p.u_in));
  D.inv_1mu = (float)(1.0 / (1.0 - p.u_in));
  D.rho_ref = (float)p.rho_ref;
  D.T_ref = (float)p.T_ref;
  D.T_iso = (float)p.T_iso;
  D.rho_mid = (float)p.rho_mid;
  D.dro = (float)(p.rho_ref - p.rho_out);
}

}  // namespace

extern "C" int lbm_create(const lbm_params* p, void* hip_stream, void* dev_mem, size_t dev_bytes,
                          lbm_domain** out) {
  int rc = validate(p);
  if (rc) return rc;
  if (!out) return lbm_fail(LBM_E_INVALID, "out is NULL");
  *out = nullptr;
  const Layout L = layout_of(*p);
  if (dev_mem && dev_bytes < L.total)
    return lbm_fail(LBM_E_INVALID, "caller buffer of %zu bytes is smaller than the %zu required",
                    dev_bytes, L.total);
  if (dev_mem && ((uintptr_t)dev_mem & 255))
    return lbm_fail(LBM_E_INVALID, "caller buffer must be 256-byte aligned");
  lbm_domain* d = new (std::nothrow) lbm_domain();
  if (!d) return lbm_fail(LBM_E_NOMEM, "host allocation failed");
  d->P = *p;
  d->rows = 0;  // automatic
  d->state_ab = 2 * L.state_bytes;
  d->write_through = d->state_ab <= kWriteThroughMaxBytes;
  {
    // SIMDs of the current device (four per compute unit), for the tile shape
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      d->simds = 4 * cus;
  }
  (void)hipGetDevice(&d->device);
  if (hip_stream) {
    d->stream = (hipStream_t)hip_stream;
    d->own_stream = false;
  } else {
    if (hipStreamCreateWithFlags(&d->stream, hipStreamNonBlocking) != hipSuccess) {
      delete d;
      return lbm_fail(LBM_E_DEVICE, "hipStreamCreate failed");
    }
    d->own_stream = true;
  }
  if (dev_mem) {
    d->mem = (char*)dev_mem;
    d->own_mem = false;
  } else {
    void* m = nullptr;
    if (hipMalloc(&m, L.total) != hipSuccess) {
      if (d->own_stream) (void)hipStreamDestroy(d->stream);
      delete d;
      return lbm_fail(LBM_E_NOMEM, "hipMalloc of %zu bytes failed", L.total);
    }
    d->mem = (char*)m;
    d->own_mem = true;
  }
  d->bytes = L.total;
  char* m = d->mem;
  fill_desc(d);
  DevDomain& D = d->host;
  D.buf[0] = m + L.state;
  D.buf[1] = m + L.state + L.state_bytes;
  D.fold[0] = (float*)(m + L.fold);
  D.fold[1] = (float*)(m + L.fold + L.fold_bytes);
  const size_t mb = align_up(p->nx * sizeof(float), 256);
  d->psiw_d[0] = (float*)(m + L.psiw);
  d->psiw_d[1] = (float*)(m + L.psiw + mb);
  d->Tw_d[0] = (float*)(m + L.Tw);
  d->Tw_d[1] = (float*)(m + L.Tw + mb);
  D.psiw[0] = d->psiw_d[0];
  D.psiw[1] = d->psiw_d[1];
  D.Tw[0] = d->Tw_d[0];
  D.Tw[1] = d->Tw_d[1];
  d->heater_d = (int*)(m + L.heater);
  D.heater = d->heater_d;
  const size_t pb = align_up(max_tiles(*p) * kPartials * sizeof(double), 256);
  D.partials[0] = (double*)(m + L.partials);
  D.partials[1] = (double*)(m + L.partials + pb);
  D.readout_partials = (double*)(m + L.rpart);
  D.pstride = max_tiles(*p);
  const size_t l1b = align_up(kFin * kPartials * sizeof(double), 256);
  D.l1[0] = (double*)(m + L.l1);
  D.l1[1] = (double*)(m + L.l1 + l1b);
  const size_t ab = align_up(kAccSlots * kAccStride * sizeof(unsigned long long), 256);
  D.macc[0] = (unsigned long long*)(m + L.macc);
  D.macc[1] = (unsigned long long*)(m + L.macc + ab);
  const size_t hb = align_up(max_tiles(*p) * sizeof(unsigned long long), 256);
  D.mhist[0] = (unsigned long long*)(m + L.mhist);
  D.mhist[1] = (unsigned long long*)(m + L.mhist + hb);
  D.rbar = (double*)(m + L.rbar);
  D.nf_flag = (int*)(m + L.nff);
  D.ring = (DiagRec*)(m + L.ring);
  D.step_dev = (long long*)(m + L.stepc);
  const size_t ob = align_up((size_t)p->nx * p->ny * sizeof(float), 256);
  for (int k = 0; k < 4; ++k) D.out[k] = (float*)(m + L.out + k * ob);
  D.parity = 0;
  d->dev = (DevDomain*)(m + L.desc);
  d->fins_d = (FinEntry*)(m + L.self);
  d->tiles_d = (Tile*)(m + L.tiles);
  std::vector<FinEntry> fe(kFin);
  for (int f = 0; f < kFin; ++f) {
    fe[f].d = d->dev;
    fe[f].f = f;
    fe[f].pad = 0;
  }
  if (hipMemcpy(d->fins_d, fe.data(), kFin * sizeof(FinEntry), hipMemcpyHostToDevice) != hipSuccess) {
    lbm_destroy(d);
    return lbm_fail(LBM_E_DEVICE, "descriptor upload failed");
  }
  // default walls: inlet temperature, neutral wall (rho_w = rho of the initial
  // uniform state is not known here -> zero pseudopotential until set)
  std::vector<float> z(p->nx, 0.f), tw(p->nx, (float)p->T_in);
  std::vector<int> hz(p->nx, 0);
  for (int s = 0; s < 2; ++s) {
    if (hipMemcpy(d->psiw_d[s], z.data(), p->nx * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d->Tw_d[s], tw.data(), p->nx * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
      lbm_destroy(d);
      return lbm_fail(LBM_E_DEVICE, "map upload failed");
    }
  }
  d->heater_h.assign(p->nx, 0);
  d->Tw_h[0].assign(p->nx, p->T_in);
  d->Tw_h[1].assign(p->nx, p->T_in);
  if (hipMemcpy(d->heater_d, hz.data(), p->nx * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    lbm_destroy(d);
    return lbm_fail(LBM_E_DEVICE, "map upload failed");
  }
  rc = lbm_build_tiles(d);
  if (rc) {
    lbm_destroy(d);
    return rc;
  }
  *out = d;
  return LBM_OK;
}

// A batched domain is stepped on its batch's stream: wait for that stream
// before the domain's own stream reads or writes its state.
static hipError_t wait_batch(lbm_domain* d) {
  return d->batch_stream && d->batch_stream != d->stream ? hipStreamSynchronize(d->batch_stream)
                                                         : hipSuccess;
}

extern "C" int lbm_destroy(lbm_domain* d) {
  if (!d) return LBM_OK;
  if (d->in_batch) return lbm_fail(LBM_E_STATE, "domain is part of a batch; destroy the batch first");
  if (d->stream) (void)hipStreamSynchronize(d->stream);
  lbm_drop_graphs(d);
  if (d->own_mem && d->mem) (void)hipFree(d->mem);
  if (d->own_stream && d->stream) (void)hipStreamDestroy(d->stream);
  delete d;
  return LBM_OK;
}

extern "C" int lbm_set_wall_maps(lbm_domain* d, int side, const double* T_wall, const double* rho_w,
                                 const int32_t* heater) {
  if (!d) return lbm_fail(LBM_E_INVALID, "domain is NULL");
  if (side != LBM_SIDE_S && side != LBM_SIDE_N) return lbm_fail(LBM_E_INVALID, "bad side %d", side);
  if (!T_wall || !rho_w) return lbm_fail(LBM_E_INVALID, "T_wall and rho_w are required");
  const int nx = d->P.nx;
  std::vector<float> ps(nx), tw(nx);
  for (int x = 0; x < nx; ++x) {
    if (!(rho_w[x] >= 0) || !(T_wall[x] > 0))
      return lbm_fail(LBM_E_INVALID, "rho_w >= 0 and T_wall > 0 required (x = %d)", x);
    ps[x] = (float)pr_psi(d->P, rho_w[x], T_wall[x]);
    tw[x] = (float)T_wall[x];
    d->Tw_h[side][x] = T_wall[x];
  }
  HIPCHECK(wait_batch(d));  // the new maps apply from the next step on
  HIPCHECK(hipMemcpyAsync(d->psiw_d[side], ps.data(), nx * sizeof(float), hipMemcpyHostToDevice, d->stream));
  HIPCHECK(hipMemcpyAsync(d->Tw_d[side], tw.data(), nx * sizeof(float), hipMemcpyHostToDevice, d->stream));
  if (side == LBM_SIDE_S) {
    std::vector<int> h(nx, 0);
    if (heater)
      for (int x = 0; x < nx; ++x) h[x] = heater[x] ? 1 : 0;
    d->heater_h = h;
    HIPCHECK(hipMemcpyAsync(d->heater_d, h.data(), nx * sizeof(int), hipMemcpyHostToDevice, d->stream));
  }
  HIPCHECK(hipStreamSynchronize(d->stream));
  return LBM_OK;
}

// Every tile's last reading of the running mass totals, per parity (all
// tiles hold the same value; set after a retiling or a load).
hipError_t fill_mhist(lbm_domain* d, unsigned long long h0, unsigned long long h1) {
  const size_t n = (size_t)d->host.pstride;
  std::vector<unsigned long long> v(n, h0);
  hipError_t e = hipMemcpyAsync(d->host.mhist[0], v.data(), n * sizeof(v[0]), hipMemcpyHostToDevice, d->stream);
  if (e != hipSuccess) return e;
  std::fill(v.begin(), v.end(), h1);
  e = hipMemcpyAsync(d->host.mhist[1], v.data(), n * sizeof(v[0]), hipMemcpyHostToDevice, d->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(d->stream);
}

namespace {

// Checks of lbm_init_fields and the FP64 mass of the initial density (fixed
// order), which the first state's buoyancy uses as its mean.
int init_args(lbm_domain* d, const double* rho0, const double* T0, double rho_u, double T_u, double noise,
              uint64_t seed, double* sum) {
  if (!d) return lbm_fail(LBM_E_INVALID, "domain is NULL");
  if (d->in_batch) return lbm_fail(LBM_E_STATE, "domain is part of a batch");
  if (!rho0 && !(rho_u > 0)) return lbm_fail(LBM_E_INVALID, "rho_uniform must be positive");
  if (!T0 && !(T_u > 0)) return lbm_fail(LBM_E_INVALID, "T_uniform must be positive");
  const int nx = d->P.nx, ny = d->P.ny;
  const size_t n = (size_t)nx * ny;
  double s = 0.0;
  if (rho0) {
    for (size_t i = 0; i < n; ++i) s += rho0[i];
  } else {
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const unsigned long long z = splitmix64_host(seed ^ (unsigned long long)((long long)y * nx + x));
        const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
        s += rho_u * (1.0 + noise * (2.0 * u - 1.0));
      }
  }
  *sum = s;
  return LBM_OK;
}

// The initial state from device copies of the optional arrays (staged by
// the caller of this function), then the reduction state; waits for it.
int init_on_device(lbm_domain* d, const double* rd, const double* td, double rho_u, double T_u, double noise,
                   uint64_t seed, double sum) {
  d->host.parity = 0;
  HIPCHECK(hipMemcpyAsync(d->dev, &d->host, sizeof(DevDomain), hipMemcpyHostToDevice, d->stream));
  HIPCHECK(lbm_launch_init(d->P.storage, d->dev, d->host, rd, td, rho_u, T_u, noise, seed, 0, d->stream));
  HIPCHECK(lbm_launch_init_aux(d->dev, sum, d->stream));
  HIPCHECK(hipStreamSynchronize(d->stream));
  d->step = 0;
  d->inited = true;
  return LBM_OK;
}

}  // namespace

extern "C" int lbm_init_fields(lbm_domain* d, const double* rho0, const double* T0, double rho_u,
                               double T_u, double noise, uint64_t seed) {
  double sum = 0.0;
  int rc = init_args(d, rho0, T0, rho_u, T_u, noise, seed, &sum);
  if (rc) return rc;
  const size_t bytes = (size_t)d->P.nx * d->P.ny * sizeof(double);
  // device staging of the host arrays, freed before returning
  double* stage[2] = {nullptr, nullptr};
  const double* src[2] = {rho0, T0};
  for (int k = 0; k < 2 && !rc; ++k) {
    if (!src[k]) continue;
    if (hipMalloc(&stage[k], bytes) != hipSuccess) {
      stage[k] = nullptr;
      rc = lbm_fail(LBM_E_NOMEM, "hipMalloc of %zu staging bytes failed", bytes);
    } else if (hipMemcpy(stage[k], src[k], bytes, hipMemcpyHostToDevice) != hipSuccess) {
      rc = lbm_fail(LBM_E_DEVICE, "upload of the initial fields failed");
    }
  }
  if (!rc) rc = init_on_device(d, stage[0], stage[1], rho_u, T_u, noise, seed, sum);
  for (double* p : stage)
    if (p) (void)hipFree(p);
  return rc;
}

// ------------------------------------------------------------------ init without allocation
// lbm_init_fields_noalloc stages the host arrays in this fixed device array
// instead of hipMalloc'd memory: two planes (density, temperature) of at
// most LBM_NOALLOC_MAX_NODES doubles, held by every device the library runs
// on until the process ends.  In host code `scratch` only names the symbol;
// its device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[2 * LBM_NOALLOC_MAX_NODES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (looked up on the first call on
// that device, with it current).
int scratch_on(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return lbm_fail(LBM_E_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    HIPCHECK(hipGetDevice(&cur));
    if (cur != dev) HIPCHECK(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) HIPCHECK(hipSetDevice(cur));
    if (e != hipSuccess || !p)
      return lbm_fail(LBM_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}
}  // namespace

extern "C" int lbm_init_fields_noalloc(lbm_domain* d, const double* rho0, const double* T0, double rho_u,
                                       double T_u, double noise, uint64_t seed) {
  double sum = 0.0;
  int rc = init_args(d, rho0, T0, rho_u, T_u, noise, seed, &sum);
  if (rc) return rc;
  const size_t n = (size_t)d->P.nx * d->P.ny;
  if ((rho0 || T0) && n > (size_t)LBM_NOALLOC_MAX_NODES)
    return lbm_fail(LBM_E_INVALID, "%d x %d = %zu nodes exceed the %d of the fixed staging array; use lbm_init_fields",
                    d->P.nx, d->P.ny, n, LBM_NOALLOC_MAX_NODES);
  double* base = nullptr;
  rc = scratch_on(d->device, &base);
  if (rc) return rc;
  double* stage[2] = {nullptr, nullptr};
  const double* src[2] = {rho0, T0};
  for (int k = 0; k < 2; ++k) {
    if (!src[k]) continue;
    stage[k] = base + (size_t)k * LBM_NOALLOC_MAX_NODES;
    HIPCHECK(hipMemcpyAsync(stage[k], src[k], n * sizeof(double), hipMemcpyHostToDevice, d->stream));
  }
  return init_on_device(d, stage[0], stage[1], rho_u, T_u, noise, seed, sum);
}

int lbm_enqueue_steps(lbm_domain* d, int64_t nsteps) {
  for (int64_t k = 0; k < nsteps; ++k) {
    // the domain's own tile table has parity 0 (stepping is refused in a batch)
    const int phase = (int)((d->step + k) & 1);
    HIPCHECK(lbm_launch_step(d->P.storage, d->tiles_d, d->ntiles, d->fins_d, kFin, d->grid, phase,
                             d->write_through, d->stream));
  }
  d->step += nsteps;
  return LBM_OK;
}

extern "C" int lbm_step(lbm_domain* d, int64_t nsteps) {
  if (!d) return lbm_fail(LBM_E_INVALID, "domain is NULL");
  if (!d->inited) return lbm_fail(LBM_E_STATE, "lbm_init_fields has not been called");
  if (nsteps < 0) return lbm_fail(LBM_E_INVALID, "nsteps must be >= 0");
  return lbm_run_steps(d, nsteps);
}

extern "C" int lbm_sync(lbm_domain* d) {
  if (!d) return lbm_fail(LBM_E_INVALID, "domain is NULL");
  HIPCHECK(wait_batch(d));
  HIPCHECK(hipStreamSynchronize(d->stream));
  return LBM_OK;
}

extern "C" int64_t lbm_step_count(const lbm_domain* d) { return d ? d->step : -1; }

static int readout(lbm_domain* d) {
  if (!d->inited) return lbm_fail(LBM_E_STATE, "lbm_init_fields has not been called");
  HIPCHECK(wait_batch(d));
  // the domain's own tile table (parity 0), also while it is in a batch: the
  // phase is the parity of the step whose state is read
  HIPCHECK(lbm_launch_readout(d->P.storage, d->tiles_d, d->ntiles, (int)(d->step & 1), d->stream));
  return LBM_OK;
}

extern "C" int lbm_read_fields_device(lbm_domain* d, float* rho, float* ux, float* uy, float* T) {
  if (!d) return lbm_fail(LBM_E_INVALID, "domain is NULL");
  int rc = readout(d);
  if (rc) return rc;
  const size_t n = (size_t)d->P.nx * d->P.ny;
  float* dsts[4] = {rho, ux, uy, T};
  for (int k = 0; k < 4; ++k)
    if (dsts[k])
      HIPCHECK(hipMemcpyAsync(dsts[k], d->host.out[k], n * sizeof(float), hipMemcpyDeviceToDevice, d->stream));
  HIPCHECK(hipStreamSynchronize(d->stream));
  return LBM_OK;
}

extern "C" int lbm_read_fields(lbm_domain* d, double* rho, double* ux, double* uy, double* T) {
  if (!d) return lbm_fail(LBM_E_INVALID, "domain is NULL");
  int rc = readout(d);
  if (rc) return rc;
  const size_t n = (size_t)d->P.nx * d->P.ny;
  std::vector<float> tmp(n);
  double* dsts[4] = {rho, ux, uy, T};
  for (int k = 0; k < 4; ++k) {
    if (!dsts[k]) continue;
    HIPCHECK(hipMemcpyAsync(tmp.data(), d->host.out[k], n * sizeof(float), hipMemcpyDeviceToHost, d->stream));
    HIPCHECK(hipStreamSynchronize(d->stream));
    for (size_t i = 0; i < n; ++i) dsts[k][i] = tmp[i];
  }
  return LBM_OK;
}

// Heater cells of the current wall map and ny / (T_h - T_in) / cells, T_h
// their mean wall temperature (0 without heater cells).
static double nusselt_factor(const lbm_domain* d) {
  int nh = 0;
  double th = 0.0;
  if (d->P.bc_y == LBM_BCY_WALLS)
    for (int x = 0; x < d->P.nx; ++x)
      if (d->heater_h[x]) {
        ++nh;
        th += d->Tw_h[0][x];
      }
  const double dT = nh > 0 ? th / nh - d->P.T_in : 0.0;
  return nh > 0 && dT != 0.0 ? (double)d->P.ny / dT / nh : 0.0;
}

// One diagnostics record from the reduced sums v[kPartials], with the two
// derived numbers: the heater Nusselt number Nu_h = ny / (T_h - T_in) x the
// mean over the heater cells of (T_h - T(x, 0)) / (1/2) = nu_factor x the
// heater flux sum, and the centreline pressure drop p_in - p_out.
static void fill_diag(double nu_factor, int64_t step, const double* v, lbm_diag* out) {
  out->step = step;
  out->mass = v[P_MASS];
  out->energy = v[P_ENERGY];
  out->heater_q = v[P_HEATQ];
  out->vapor_cells = v[P_VAPOR];
  out->psi_clamped = v[P_CLAMP];
  out->nonfinite = v[P_NONFINITE];
  out->p_in = v[P_PIN];
  out->p_out = v[P_POUT];
  out->nu_heater = nu_factor * v[P_HEATQ];
  out->dp = v[P_PIN] - v[P_POUT];
}

extern "C" int lbm_read_diag(lbm_domain* d, lbm_diag* out) {
  if (!d || !out) return lbm_fail(LBM_E_INVALID, "NULL argument");
  int rc = readout(d);
  if (rc) return rc;
  double* res = (double*)(d->host.rbar) + 16;  // scratch inside the 256-byte rbar block
  HIPCHECK(lbm_launch_finalize(d->host.readout_partials, d->host.pstride, d->ntiles, res, d->stream));
  double h[kPartials];
  HIPCHECK(hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, d->stream));
  HIPCHECK(hipStreamSynchronize(d->stream));
  fill_diag(nusselt_factor(d), d->step, h, out);
  return LBM_OK;
}

extern "C" int lbm_diag_history(lbm_domain* d, lbm_diag* out, int max, int* n) {
  if (!d || !out || !n) return lbm_fail(LBM_E_INVALID, "NULL argument");
  std::vector<DiagRec> ring(kRing);
  HIPCHECK(wait_batch(d));
  HIPCHECK(hipStreamSynchronize(d->stream));
  HIPCHECK(hipMemcpy(ring.data(), d->host.ring, kRing * sizeof(DiagRec), hipMemcpyDeviceToHost));
  std::vector<DiagRec> valid;
  for (auto& r : ring)
    if (r.step >= 0) valid.push_back(r);
  std::sort(valid.begin(), valid.end(), [](const DiagRec& a, const DiagRec& b) { return a.step < b.step; });
  const int k = std::min<int>(max, (int)valid.size());
  const int off = (int)valid.size() - k;
  const double nu_factor = nusselt_factor(d);
  for (int i = 0; i < k; ++i) {
    const DiagRec& r = valid[off + i];
    fill_diag(nu_factor, r.step, r.v, &out[i]);
  }
  *n = k;
  return LBM_OK;
}

// ------------------------------------------------------------------ checkpoints
namespace {
// A checkpoint holds the state the next step reads, independent of the
// tiling: state buffer, outlet memory, the pending diagnostics reductions
// (per-tile partials summed into totals), the level-1 slices, the device
// step counter, the running mass totals and the tiles' common last reading.
struct CkptHeader {
  char magic[8];
  int32_t nx, ny, storage, isothermal;
  int64_t step;
  uint64_t state_bytes, fold_bytes;
};
struct CkptTail {
  double part_tot[kPartials];
  double l1[2][kFin * kPartials];
  long long step_dev;
  unsigned long long macc[2][kAccSlots * kAccStride];
  unsigned long long mhist[2];
};

// Totals of the pending per-tile partial sums (parity q), host side.
int partial_totals(lbm_domain* d, int q, double tot[kPartials]) {
  const size_t stride = d->host.pstride;
  std::vector<double> part(stride * kPartials);
  HIPCHECK(hipMemcpy(part.data(), d->host.partials[q], part.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (int k = 0; k < kPartials; ++k) {
    tot[k] = 0.0;
    for (int t = 0; t < d->ntiles; ++t) tot[k] += part[(size_t)k * stride + t];
  }
  return LBM_OK;
}

// Pending partial sums of parity q replaced by their totals in tile 0.
int put_partial_totals(lbm_domain* d, int q, const double tot[kPartials]) {
  const size_t stride = d->host.pstride;
  std::vector<double> part(stride * kPartials, 0.0);
  for (int k = 0; k < kPartials; ++k) part[(size_t)k * stride] = tot[k];
  HIPCHECK(hipMemcpy(d->host.partials[q], part.data(), part.size() * sizeof(double), hipMemcpyHostToDevice));
  return LBM_OK;
}
}  // namespace

extern "C" int lbm_save(lbm_domain* d, const char* path) {
  if (!d || !path) return lbm_fail(LBM_E_INVALID, "NULL argument");
  if (!d->inited) return lbm_fail(LBM_E_STATE, "nothing to save");
  const Layout L = layout_of(d->P);
  HIPCHECK(wait_batch(d));
  HIPCHECK(hipStreamSynchronize(d->stream));
  // the state of step s lives in buffer s & 1 (alone or in a batch)
  const int ph = (int)(d->step & 1);
  std::vector<char> st(L.state_bytes), fo(L.fold_bytes);
  CkptTail t{};
  HIPCHECK(hipMemcpy(st.data(), d->host.buf[ph], L.state_bytes, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(fo.data(), d->host.fold[ph], L.fold_bytes, hipMemcpyDeviceToHost));
  int rc = partial_totals(d, ph ^ 1, t.part_tot);
  if (rc) return rc;
  // stored in the order of the step parity (index 0: the next step's own)
  for (int k = 0; k < 2; ++k) {
    const int q = ph ^ k;
    HIPCHECK(hipMemcpy(t.l1[k], d->host.l1[q], sizeof(t.l1[k]), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(t.macc[k], d->host.macc[q], sizeof(t.macc[k]), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(&t.mhist[k], d->host.mhist[q], sizeof(t.mhist[k]), hipMemcpyDeviceToHost));
  }
  HIPCHECK(hipMemcpy(&t.step_dev, d->host.step_dev, sizeof(t.step_dev), hipMemcpyDeviceToHost));
  FILE* f = fopen(path, "wb");
  if (!f) return lbm_fail(LBM_E_INVALID, "cannot open %s for writing", path);
  CkptHeader h{};
  memcpy(h.magic, "LBMCKPT4", 8);
  h.nx = d->P.nx;
  h.ny = d->P.ny;
  h.storage = d->P.storage;
  h.isothermal = d->P.isothermal;
  h.step = d->step;
  h.state_bytes = L.state_bytes;
  h.fold_bytes = L.fold_bytes;
  bool ok = fwrite(&h, sizeof(h), 1, f) == 1 && fwrite(st.data(), 1, st.size(), f) == st.size() &&
            fwrite(fo.data(), 1, fo.size(), f) == fo.size() && fwrite(&t, sizeof(t), 1, f) == 1;
  ok = (fclose(f) == 0) && ok;
  return ok ? LBM_OK : lbm_fail(LBM_E_INVALID, "write to %s failed", path);
}

extern "C" int lbm_load(lbm_domain* d, const char* path) {
  if (!d || !path) return lbm_fail(LBM_E_INVALID, "NULL argument");
  if (d->in_batch) return lbm_fail(LBM_E_STATE, "domain is part of a batch");
  FILE* f = fopen(path, "rb");
  if (!f) return lbm_fail(LBM_E_INVALID, "cannot open %s", path);
  CkptHeader h{};
  const Layout L = layout_of(d->P);
  if (fread(&h, sizeof(h), 1, f) != 1 || memcmp(h.magic, "LBMCKPT4", 8) != 0 || h.nx != d->P.nx ||
      h.ny != d->P.ny || h.storage != d->P.storage || h.isothermal != d->P.isothermal ||
      h.state_bytes != L.state_bytes || h.fold_bytes != L.fold_bytes) {
    fclose(f);
    return lbm_fail(LBM_E_INVALID, "%s does not match this domain (geometry or storage)", path);
  }
  std::vector<char> st(L.state_bytes), fo(L.fold_bytes);
  CkptTail t{};
  bool ok = fread(st.data(), 1, st.size(), f) == st.size() && fread(fo.data(), 1, fo.size(), f) == fo.size() &&
            fread(&t, sizeof(t), 1, f) == 1;
  fclose(f);
  if (!ok) return lbm_fail(LBM_E_INVALID, "%s is truncated", path);
  HIPCHECK(hipStreamSynchronize(d->stream));
  d->step = h.step;
  d->host.parity = 0;
  HIPCHECK(hipMemcpy(d->dev, &d->host, sizeof(DevDomain), hipMemcpyHostToDevice));
  const int ph = (int)(d->step & 1);
  HIPCHECK(hipMemcpy(d->host.buf[ph], st.data(), L.state_bytes, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(d->host.fold[ph], fo.data(), L.fold_bytes, hipMemcpyHostToDevice));
  int rc = put_partial_totals(d, ph ^ 1, t.part_tot);
  if (rc) return rc;
  for (int k = 0; k < 2; ++k) {
    const int q = ph ^ k;
    HIPCHECK(hipMemcpy(d->host.l1[q], t.l1[k], sizeof(t.l1[k]), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(d->host.macc[q], t.macc[k], sizeof(t.macc[k]), hipMemcpyHostToDevice));
  }
  HIPCHECK(fill_mhist(d, t.mhist[ph], t.mhist[ph ^ 1]));
  HIPCHECK(hipMemcpy(d->host.step_dev, &t.step_dev, sizeof(t.step_dev), hipMemcpyHostToDevice));
  HIPCHECK(hipMemset(d->host.nf_flag, 0, sizeof(int)));
  // the per-step records restart from the loaded state (the ring is not saved)
  HIPCHECK(hipMemset(d->host.ring, 0xFF, kRing * sizeof(DiagRec)));
  d->inited = true;
  return LBM_OK;
}

// Whether a step since the last initialisation or load met a non-finite
// density or temperature (waits for the domain's stream).
int lbm_nonfinite_seen(lbm_domain* d, int* seen) {
  HIPCHECK(wait_batch(d));
  int v = 0;
  HIPCHECK(hipMemcpyAsync(&v, d->host.nf_flag, sizeof(int), hipMemcpyDeviceToHost, d->stream));
  HIPCHECK(hipStreamSynchronize(d->stream));
  *seen = v != 0;
  return LBM_OK;
}

// ------------------------------------------------------------------ Maxwell construction
extern "C" int lbm_maxwell(const lbm_params* p, double T, double* rho_l, double* rho_v, double* p_sat) {
  if (!p || !rho_l || !rho_v || !p_sat) return lbm_fail(LBM_E_INVALID, "NULL argument");
  const double Tc = crit_T(*p);
  if (!(T > 0 && T < Tc)) return lbm_fail(LBM_E_INVALID, "T must lie in (0, Tc = %g)", Tc);
  const double b = p->b, a = p->a, R = p->R;
  const double s = std::sqrt(T / Tc);
  const double sa = 1.0 + kappa_of(*p) * (1.0 - s);
  const double aa = a * sa * sa;
  auto P = [&](double v) { return R * T / (v - b) - aa / (v * v + 2 * b * v - b * b); };
  auto dP = [&](double v) {
    const double q = v * v + 2 * b * v - b * b;
    return -R * T / ((v - b) * (v - b)) + aa * (2 * v + 2 * b) / (q * q);
  };
  // primitive of P dv
  const double r2 = std::sqrt(2.0);
  auto I = [&](double v) {
    return R * T * std::log(v - b) - aa / (2 * r2 * b) * std::log((v + b - r2 * b) / (v + b + r2 * b));
  };
  auto bisect = [](auto f, double lo, double hi) {
    double flo = f(lo);
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      const double fm = f(mid);
      if ((fm > 0) == (flo > 0)) {
        lo = mid;
        flo = fm;
      } else {
        hi = mid;
      }
    }
    return 0.5 * (lo + hi);
  };
  // spinodals: sign changes of dP on a geometric grid of v
  double vmin = 0, vmax = 0;
  int found = 0;
  double vprev = b * 1.0001, dprev = dP(vprev);
  for (int k = 1; k <= 200000 && found < 2; ++k) {
    const double v = b * 1.0001 * std::pow(1e4 / 1.0001, k / 200000.0);
    const double dv = dP(v);
    if ((dv > 0) != (dprev > 0)) {
      const double root = bisect(dP, vprev, v);
      if (found == 0) vmin = root; else vmax = root;
      ++found;
    }
    vprev = v;
    dprev = dv;
  }
  if (found < 2) return lbm_fail(LBM_E_INVALID, "no van der Waals loop at T = %g", T);
  const double plo = std::max(P(vmin), 1e-9 * P(vmax)), phi = P(vmax);
  auto roots = [&](double ps, double* vl, double* vg) {
    *vl = bisect([&](double v) { return P(v) - ps; }, b * (1 + 1e-12), vmin);
    double hi = 2 * vmax;
    while (P(hi) >= ps) hi *= 2;
    *vg = bisect([&](double v) { return P(v) - ps; }, vmax, hi);
  };
  auto area = [&](double ps) {
    double vl, vg;
    roots(ps, &vl, &vg);
    return (I(vg) - I(vl)) - ps * (vg - vl);
  };
  const double eps = 1e-12 * (phi - plo);
  const double ps = bisect(area, plo + eps, phi - eps);
  double vl, vg;
  roots(ps, &vl, &vg);
  *rho_l = 1.0 / vl;
  *rho_v = 1.0 / vg;
  *p_sat = ps;
  return LBM_OK;
}

extern "C" int lbm_set_tile_rows(lbm_domain* d, int rows) {
  if (!d) return lbm_fail(LBM_E_INVALID, "domain is NULL");
  if (rows < 0) return lbm_fail(LBM_E_INVALID, "rows must be >= 0");
  // the batch holds copies of the domain's tiles
  if (d->in_batch) return lbm_fail(LBM_E_STATE, "domain is part of a batch");
  // State kept per tile moves to the new tiling: the pending partial sums of
  // the last launch go to tile 0 as totals (the finalizers' slices of the
  // new tiling then sum to the same values), and every new tile gets the
  // common last reading of the running mass totals.
  const int ph = (int)(d->step & 1);
  double tot[kPartials] = {0};
  unsigned long long hist[2] = {0ull, 0ull};
  if (d->inited) {
    HIPCHECK(hipStreamSynchronize(d->stream));
    int rc = partial_totals(d, ph ^ 1, tot);
    if (rc) return rc;
    HIPCHECK(hipMemcpy(&hist[0], d->host.mhist[0], sizeof(hist[0]), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(&hist[1], d->host.mhist[1], sizeof(hist[1]), hipMemcpyDeviceToHost));
  }
  d->rows = rows == 0 ? 0 : std::max(rows, kMinTileRows);
  int rc = lbm_build_tiles(d);
  if (rc) return rc;
  if (d->inited) {
    rc = put_partial_totals(d, ph ^ 1, tot);
    if (rc) return rc;
    HIPCHECK(fill_mhist(d, hist[0], hist[1]));
  }
  return LBM_OK;
}

extern "C" int lbm_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (!dst || !src) return lbm_fail(LBM_E_INVALID, "NULL buffer");
  if (((uintptr_t)dst & 15) || ((uintptr_t)src & 15) || (bytes & 15))
    return lbm_fail(LBM_E_INVALID, "buffers and size must be 16-byte aligned");
  HIPCHECK(lbm_launch_copy(dst, src, bytes, (hipStream_t)hip_stream));
  return LBM_OK;
}
