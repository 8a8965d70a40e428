// gfx950 kernels of the coupled pseudopotential / thermal D2Q9 time step
// (arXiv:2009.05264, Sec. 2).
//
// Work decomposition: one 64-lane wavefront owns a tile = a strip of 64
// consecutive columns (60 interior columns plus a 2-column halo on each
// side) and marches up a segment of rows.  At march position r it
//   stage 1: pulls and applies the boundary rules for row r, takes moments,
//            evaluates the EOS and the pseudopotential (Eqs. 4, 6, 11, 12, 17);
//   stage 2: forms the interaction force of row r-1 from the pseudopotential
//            of rows r-2..r (Eqs. 8-10, 14, 15) and its actual velocity (Eq. 7);
//   stage 3: forms div u of row r-2 from the actual velocities of rows
//            r-3..r-1, the phase-change source (Eq. 19) and collides both
//            distributions (Eqs. 2, 3, 5, 16, 18), storing the post-collision
//            values of its own node.
// Three rotating row slots live in registers; x neighbours come from
// cross-lane shuffles.  No LDS, no barrier.  All arithmetic is FP32 on the
// deviations f_i - w_i rho_ref, g_i - w_i T_ref; the HBM storage is FP32,
// FP16 or BF16 (template parameter).
//
// Reductions for the diagnostics and for the mean density of the buoyancy
// force are fixed-order FP64: each tile writes its partial sums; the first
// tile of each domain sums the previous launch's partials at the start of the
// next launch (kernel boundaries order the two).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbmflow.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

// D2Q9 velocities: rest, +x, +y, -x, -y, (+,+), (-,+), (-,-), (+,-)
__device__ constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
__device__ constexpr float WF[9] = {4.f / 9, 1.f / 9, 1.f / 9, 1.f / 9, 1.f / 9,
                                    1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};

// ---------------------------------------------------------------- storage
template <int S>
struct Codec;
template <>
struct Codec<LBM_STORE_F32> {
  using T = float;
  static __device__ __forceinline__ float ld(const T* p, long long i) { return p[i]; }
  static __device__ __forceinline__ void st(T* p, long long i, float v) { p[i] = v; }
};
template <>
struct Codec<LBM_STORE_F32_DEV> : Codec<LBM_STORE_F32> {};
template <>
struct Codec<LBM_STORE_F16_DEV> {
  using T = _Float16;
  static __device__ __forceinline__ float ld(const T* p, long long i) { return (float)p[i]; }
  static __device__ __forceinline__ void st(T* p, long long i, float v) {
    v = fminf(fmaxf(v, -65504.f), 65504.f);  // saturate, round to nearest even
    p[i] = (_Float16)v;
  }
};
template <>
struct Codec<LBM_STORE_BF16_DEV> {
  using T = uint16_t;
  static __device__ __forceinline__ float ld(const T* p, long long i) {
    return __uint_as_float(((uint32_t)p[i]) << 16);
  }
  static __device__ __forceinline__ void st(T* p, long long i, float v) {
    v = fminf(fmaxf(v, -3.3895313892515355e38f), 3.3895313892515355e38f);
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    p[i] = (uint16_t)(u >> 16);
  }
};

__device__ __forceinline__ int wrap(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// Per-lane data of one lattice row of the tile.
struct Row {
  float h[9], k[9];      // pulled distributions (deviation form)
  float rho, drho, ux, uy, T, dT, inv_rho;
  float psi, A, B, dpdT; // A = beta psi, B = psi^2 (wall rows: psi_w)
  float Fx, Fy, uax, uay;
};

// Peng-Robinson EOS (Eq. 12), pseudopotential (Eq. 11), (dp/dT)_rho.
__device__ __forceinline__ void eos(const DevDomain& D, float rho, float T, float& p, float& psi,
                                    float& dpdT, int& clamped) {
  const float s = sqrtf(T * D.inv_Tc);
  const float sa = 1.f + D.kappa * (1.f - s);
  const float alpha = sa * sa;
  const float br = D.b * rho;
  const float r1 = 1.f / (1.f - br);
  const float r2 = 1.f / (1.f + br * (2.f - br));
  const float ar2 = D.a * rho * rho * r2;
  p = rho * D.R * T * r1 - alpha * ar2;
  float q = (p - rho * (1.f / 3.f)) * D.c0g2;
  clamped = !(q >= 0.f);
  q = clamped ? 0.f : q;
  psi = sqrtf(q);
  dpdT = rho * D.R * r1 + ar2 * D.kappa * sa / (s * D.Tc);
}

// Pull of node (xc, y) from the post-collision buffer with the boundary
// rules (bounce-back / anti-bounce-back at wall rows, Zou-He inlet,
// convective outlet).  xc in [0, nx), y in [0, ny).
template <int S>
__device__ __forceinline__ void pull(const DevDomain& D, const typename Codec<S>::T* src,
                                     const float* fold, int xc, int y, bool thermal, float h[9],
                                     float k[9]) {
  using C = Codec<S>;
  const int nx = D.nx, ny = D.ny;
  const long long pl = D.plane;
  const long long own = (long long)y * D.pitch + xc;
  const bool walls = D.bc_y == LBM_BCY_WALLS;
  const bool chan = D.bc_x == LBM_BCX_CHANNEL;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    int xs = xc - CX[i];
    int ys = y - CY[i];
    if (walls && (ys < 0 || ys >= ny)) {
      const int o = OPP[i];
      const int xm = chan ? clampi(xs, 0, nx - 1) : (xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs));
      h[i] = C::ld(src, o * pl + own);
      if (thermal) {
        const float Tw = (ys < 0 ? D.Tw[0] : D.Tw[1])[xm];
        k[i] = -C::ld(src, (9 + o) * pl + own) + 2.f * WF[i] * (Tw - D.T_ref);
      }
    } else {
      ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
      if (!chan) xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
      if (xs >= 0 && xs < nx) {
        const long long idx = (long long)ys * D.pitch + xs;
        h[i] = C::ld(src, i * pl + idx);
        if (thermal) k[i] = C::ld(src, (9 + i) * pl + idx);
      } else {
        h[i] = 0.f;  // ghost source: set by the inlet / outlet rule below
        k[i] = 0.f;
      }
    }
  }
  if (!chan) return;
  if (xc == 0) {
    // Zou-He velocity inlet; unknowns are 1, 5, 8 unless a wall row is the source.
    const float u = D.u_in;
    const float rin = (D.rho_ref + h[0] + h[2] + h[4] + 2.f * (h[3] + h[6] + h[7])) / (1.f - u);
    const bool unk5 = !(walls && y - 1 < 0);
    const bool unk8 = !(walls && y + 1 >= ny);
    const float d24 = 0.5f * (h[2] - h[4]);
    h[1] = h[3] + (2.f / 3.f) * rin * u;
    if (unk5) h[5] = h[7] - d24 + rin * u * (1.f / 6.f);
    if (unk8) h[8] = h[6] + d24 + rin * u * (1.f / 6.f);
    if (thermal) {
      const float gin = D.in_geq - D.T_ref;
      k[1] = -C::ld(src, (9 + 3) * pl + own) + 2.f * WF[1] * gin;
      if (unk5) k[5] = -C::ld(src, (9 + 7) * pl + own) + 2.f * WF[5] * gin;
      if (unk8) k[8] = -C::ld(src, (9 + 6) * pl + own) + 2.f * WF[8] * gin;
    }
  }
  if (xc == nx - 1) {
    // Convective outlet for 3, 6, 7 from the values just pulled at nx-2.
    const int xn = nx - 2;
    const long long own2 = (long long)y * D.pitch + xn;
    const int dirs[3] = {3, 6, 7};
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int i = dirs[m];
      const int ys = y - CY[i];
      if (walls && (ys < 0 || ys >= ny)) continue;  // wall rule already applied
      const int ysw = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
      // pull of direction i at (nx-2, y): source (nx-1, y - cy)
      const long long sidx = (long long)ysw * D.pitch + (nx - 1);
      float hn, kn = 0.f;
      hn = C::ld(src, i * pl + sidx);
      if (thermal) kn = C::ld(src, (9 + i) * pl + sidx);
      (void)own2;
      h[i] = (fold[m * ny + y] + D.U_out * hn) * D.inv_1pU;
      if (thermal) k[i] = kn;
    }
  }
}

template <int S>
__device__ __forceinline__ void store_node(const DevDomain& D, typename Codec<S>::T* dst, int x,
                                           int y, bool thermal, const float hs[9],
                                           const float ks[9]) {
  using C = Codec<S>;
  const long long idx = (long long)y * D.pitch + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) C::st(dst, i * D.plane + idx, hs[i]);
  if (thermal) {
#pragma unroll
    for (int i = 0; i < 9; ++i) C::st(dst, (9 + i) * D.plane + idx, ks[i]);
  }
}

// MRT collision with exact-difference forcing, in deviation form.  b_k =
// S_k m_k(f - f^eq) - m_k(Delta F) for the moments (rho, e, eps, jx, qx, jy,
// qy, pxx, pxy) of the Lallemand-Luo basis, f* = f - M^-1 b.
__device__ __forceinline__ void collide_f(const DevDomain& D, const Row& R, float hs[9]) {
  const float* h = R.h;
  const float A13 = h[1] + h[3], A24 = h[2] + h[4];
  const float Dg = h[5] + h[6] + h[7] + h[8];
  const float d13 = h[1] - h[3], d24 = h[2] - h[4];
  const float d57 = h[5] - h[7], d86 = h[8] - h[6];
  const float jx = d13 + d57 + d86;
  const float jy = d24 + d57 - d86;
  const float me = -4.f * h[0] - (A13 + A24) + 2.f * Dg;
  const float meps = 4.f * h[0] - 2.f * (A13 + A24) + Dg;
  const float mqx = -2.f * d13 + d57 + d86;
  const float mqy = -2.f * d24 + d57 - d86;
  const float mxx = A13 - A24;
  const float mxy = (h[5] + h[7]) - (h[6] + h[8]);
  const float ux = R.ux, uy = R.uy;
  const float rho = R.rho;
  const float ru2 = jx * ux + jy * uy;  // rho u^2
  // non-equilibrium parts
  const float ne = me + 2.f * R.drho - 3.f * ru2;
  const float neps = meps - R.drho + 3.f * ru2;
  const float nqx = mqx + jx;
  const float nqy = mqy + jy;
  const float nxx = mxx - (jx * ux - jy * uy);
  const float nxy = mxy - jx * uy;
  // forcing: Delta u = F/rho, s = 2u + Delta u
  const float Fx = R.Fx, Fy = R.Fy;
  const float sx = 2.f * ux + Fx * R.inv_rho, sy = 2.f * uy + Fy * R.inv_rho;
  const float Fs = Fx * sx + Fy * sy;
  (void)rho;
  const float ae = (D.s_e * ne - 3.f * Fs) * (1.f / 36.f);
  const float aeps = (D.s_eps * neps + 3.f * Fs) * (1.f / 36.f);
  const float aqx = (D.s_q * nqx + Fx) * (1.f / 12.f);
  const float aqy = (D.s_q * nqy + Fy) * (1.f / 12.f);
  const float axx = (D.s_nu * nxx - (Fx * sx - Fy * sy)) * 0.25f;
  const float axy = (D.s_nu * nxy - 0.5f * (Fx * sy + Fy * sx)) * 0.25f;
  const float ajx = -Fx * (1.f / 6.f), ajy = -Fy * (1.f / 6.f);
  const float E1 = -ae - 2.f * aeps, E2 = 2.f * ae + aeps;
  const float X = ajx - 2.f * aqx, Y = ajy - 2.f * aqy;
  const float X2 = ajx + aqx, Y2 = ajy + aqy;
  hs[0] = h[0] - (-4.f * ae + 4.f * aeps);
  hs[1] = h[1] - (E1 + X + axx);
  hs[2] = h[2] - (E1 + Y - axx);
  hs[3] = h[3] - (E1 - X + axx);
  hs[4] = h[4] - (E1 - Y - axx);
  hs[5] = h[5] - (E2 + X2 + Y2 + axy);
  hs[6] = h[6] - (E2 - X2 + Y2 - axy);
  hs[7] = h[7] - (E2 - X2 - Y2 + axy);
  hs[8] = h[8] - (E2 + X2 - Y2 - axy);
}

// BGK relaxation of g towards g^eq(T, u_act) plus the source w_i phi.
__device__ __forceinline__ void collide_g(const DevDomain& D, const Row& R, float phi, float ks[9]) {
  const float om = D.omega_g;
  const float tT = om * R.T;
  const float u2 = R.uax * R.uax + R.uay * R.uay;
  const float base = om * R.dT + phi - 1.5f * tT * u2;
  const float keep = 1.f - om;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float cu = (float)CX[i] * R.uax + (float)CY[i] * R.uay;
    ks[i] = keep * R.k[i] + WF[i] * (base + tT * cu * (3.f + 4.5f * cu));
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

// Fixed-order sum of ntiles partial records by one wave; lane 0 gets it.
__device__ __forceinline__ void sum_partials(const double* parts, int ntiles, double out[kPartials]) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int q = 0; q < kPartials; ++q) out[q] = 0.0;
  for (int t = lane; t < ntiles; t += kWave) {
#pragma unroll
    for (int q = 0; q < kPartials; ++q) out[q] += parts[(long long)t * kPartials + q];
  }
#pragma unroll
  for (int q = 0; q < kPartials; ++q) out[q] = wave_sum(out[q]);
}

template <int S, int MODE>
__device__ void run_tile(const Tile& tl, int gphase) {
  using C = Codec<S>;
  const DevDomain& D = *tl.d;
  const int lane = threadIdx.x & (kWave - 1);
  const int phase = gphase ^ D.parity;
  const int nx = D.nx, ny = D.ny;
  const bool chan = D.bc_x == LBM_BCX_CHANNEL;
  const bool walls = D.bc_y == LBM_BCY_WALLS;
  const bool thermal = !D.isothermal;
  const typename C::T* src = (const typename C::T*)D.buf[phase];
  typename C::T* dst = (typename C::T*)D.buf[phase ^ 1];
  const float* fold = D.fold[phase];
  float* fold_dst = D.fold[phase ^ 1];

  if (MODE == MODE_STEP && tl.local == 0) {
    // Finalize the previous launch's reductions of this domain.
    double sums[kPartials];
    sum_partials(D.partials[phase ^ 1], D.ntiles, sums);
    if (lane == 0) {
      const long long st = *D.step_dev;
      D.rbar[phase ^ 1] = sums[P_MASS] / ((double)nx * (double)ny);
      DiagRec& rec = D.ring[(st + kRing) % kRing];
      rec.step = st - 1;
#pragma unroll
      for (int q = 0; q < kPartials; ++q) rec.v[q] = sums[q];
      *D.step_dev = st + 1;
    }
  }

  const int x = tl.x0 - 2 + lane;
  const int xc = chan ? clampi(x, 0, nx - 1) : wrap(x, nx);
  const int xw = xc;  // wall-map column of this lane's solid cells
  const bool interior = lane >= 2 && lane < kWave - 2 && x < nx;
  const float gbar = (float)((double)D.rho_ref - D.rbar[phase]);  // rho_ref - rho_bar

  double acc_mass = 0.0, acc_energy = 0.0, acc_q = 0.0;
  int acc_vap = 0, acc_clamp = 0, acc_nf = 0;
  double acc_pin = 0.0, acc_pout = 0.0;

  Row R0, R1, R2;
  bool s0 = false, s1 = false, s2 = false;  // solid flags of the three slots
  float uy_prev = 0.f;                      // u_act,y of the row below the collided one
  bool sprev = false;

  const int r_end = MODE == MODE_STEP ? tl.y1 + 1 : tl.y1;
  for (int r = tl.y0 - 2; r <= r_end; ++r) {
    // ---- stage 1: row r into R0
    const bool solid = walls && (r < 0 || r >= ny);
    if (solid) {
      const float pw = (r < 0 ? D.psiw[0] : D.psiw[1])[xw];
      R0.psi = pw;
      R0.A = D.beta * pw;
      R0.B = pw * pw;
    } else {
      const int ry = walls ? r : wrap(r, ny);
      pull<S>(D, src, fold, xc, ry, thermal, R0.h, R0.k);
      float drho = 0.f, dT = 0.f;
#pragma unroll
      for (int i = 0; i < 9; ++i) drho += R0.h[i];
      if (thermal) {
#pragma unroll
        for (int i = 0; i < 9; ++i) dT += R0.k[i];
      } else {
        dT = D.T_iso - D.T_ref;
      }
      const float rho = D.rho_ref + drho;
      const float T = D.T_ref + dT;
      const float jx = (R0.h[1] - R0.h[3]) + (R0.h[5] - R0.h[7]) + (R0.h[8] - R0.h[6]);
      const float jy = (R0.h[2] - R0.h[4]) + (R0.h[5] - R0.h[7]) + (R0.h[6] - R0.h[8]);
      const float inv_rho = 1.f / rho;
      R0.rho = rho;
      R0.drho = drho;
      R0.T = T;
      R0.dT = dT;
      R0.inv_rho = inv_rho;
      R0.ux = jx * inv_rho;
      R0.uy = jy * inv_rho;
      float p, psi, dpdT;
      int clamped;
      eos(D, rho, T, p, psi, dpdT, clamped);
      R0.psi = psi;
      R0.A = D.beta * psi;
      R0.B = psi * psi;
      R0.dpdT = dpdT;
      if (interior && r >= tl.y0 && r < tl.y1) {
        acc_mass += (double)rho;
        acc_energy += (double)T;
        acc_vap += rho < D.rho_mid;
        acc_clamp += clamped;
        acc_nf += !(isfinite(rho) && isfinite(T));
        if (walls && ry == 0 && D.heater[x]) acc_q += 2.0 * (double)(D.Tw[0][x] - T);
        if (ry == ny / 2) {
          if (x == 0) acc_pin = (double)p;
          if (x == nx - 1) acc_pout = (double)p;
        }
        if (MODE == MODE_STEP && chan && x == nx - 1) {
          fold_dst[0 * ny + ry] = R0.h[3];
          fold_dst[1 * ny + ry] = R0.h[6];
          fold_dst[2 * ny + ry] = R0.h[7];
        }
      }
    }
    s0 = solid;

    // ---- stage 2: force and actual velocity of row q = r - 1 (slot R1)
    if (r >= tl.y0) {
      if (s1) {
        R1.uax = 0.f;
        R1.uay = 0.f;
      } else {
        float Fx = 0.f, Fy = 0.f;
        if (!D.single_phase) {
          const float VA = D.G1 * R1.A + D.G2 * (R0.A + R2.A);
          const float VB = D.G1 * R1.B + D.G2 * (R0.B + R2.B);
          const float DA = R0.A - R2.A;
          const float DB = R0.B - R2.B;
          const float VAr = __shfl_down(VA, 1, kWave), VAl = __shfl_up(VA, 1, kWave);
          const float VBr = __shfl_down(VB, 1, kWave), VBl = __shfl_up(VB, 1, kWave);
          const float DAr = __shfl_down(DA, 1, kWave), DAl = __shfl_up(DA, 1, kWave);
          const float DBr = __shfl_down(DB, 1, kWave), DBl = __shfl_up(DB, 1, kWave);
          const float SAx = VAr - VAl, SBx = VBr - VBl;
          const float SAy = D.G1 * DA + D.G2 * (DAr + DAl);
          const float SBy = D.G1 * DB + D.G2 * (DBr + DBl);
          Fx = -R1.psi * SAx - D.half_1mb * SBx;
          Fy = -R1.psi * SAy - D.half_1mb * SBy;
        }
        const float dr = R1.drho + gbar;  // rho - rho_bar
        Fx += dr * D.ga_x + D.fb_x;
        Fy += dr * D.ga_y + D.fb_y;
        R1.Fx = Fx;
        R1.Fy = Fy;
        R1.uax = R1.ux + 0.5f * Fx * R1.inv_rho;
        R1.uay = R1.uy + 0.5f * Fy * R1.inv_rho;
        if (MODE == MODE_READOUT && interior && r - 1 >= tl.y0 && r - 1 < tl.y1) {
          const long long o = (long long)(r - 1) * nx + x;
          D.out[0][o] = R1.rho;
          D.out[1][o] = R1.uax;
          D.out[2][o] = R1.uay;
          D.out[3][o] = R1.T;
        }
      }
    }

    // ---- stage 3: source and collisions of row c = r - 2 (slot R2)
    if (MODE == MODE_STEP && r >= tl.y0 + 2) {
      const int c = r - 2;
      float uxl = __shfl_up(R2.uax, 1, kWave);
      float uxr = __shfl_down(R2.uax, 1, kWave);
      if (chan) {
        if (x == 0) uxl = R2.uax;
        if (x == nx - 1) uxr = R2.uax;
      }
      const float dux = 0.5f * (uxr - uxl);
      const float un_c = s1 ? R2.uay : R1.uay, un_m = s1 ? -R2.uay : R1.uay;
      const float us_c = sprev ? R2.uay : uy_prev, us_m = sprev ? -R2.uay : uy_prev;
      const float div_adv = dux + 0.5f * (un_c - us_c);
      const float div_mass = dux + 0.5f * (un_m - us_m);
      const float phi = R2.T * (div_adv - R2.dpdT * R2.inv_rho * D.inv_cv * div_mass);
      float hs[9], ks[9];
      collide_f(D, R2, hs);
      if (thermal) collide_g(D, R2, phi, ks);
      if (interior) store_node<S>(D, dst, x, walls ? c : wrap(c, ny), thermal, hs, ks);
      uy_prev = R2.uay;
      sprev = s2;
    } else if (MODE == MODE_STEP && r == tl.y0 + 1) {
      // row y0 - 1 becomes the "row below" of the first collided row
      uy_prev = R2.uay;
      sprev = s2;
    }

    // rotate slots: R2 <- R1 <- R0
    R2 = R1;
    R1 = R0;
    s2 = s1;
    s1 = s0;
  }

  // ---- tile partial sums (fixed order: lane tree)
  double v[kPartials] = {acc_mass, acc_energy, acc_q, (double)acc_vap, (double)acc_clamp,
                         (double)acc_nf, acc_pin, acc_pout};
#pragma unroll
  for (int q = 0; q < kPartials; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0) {
    double* out = (MODE == MODE_STEP ? D.partials[phase] : D.readout_partials) +
                  (long long)tl.local * kPartials;
#pragma unroll
    for (int q = 0; q < kPartials; ++q) out[q] = v[q];
  }
}

// Bijection from launch order to tile index that hands each XCD (blocks are
// dispatched round-robin over the 8 XCDs) a contiguous run of tiles, so the
// halos that neighbouring tiles share stay in one L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int q = n >> 3, rem = n & 7;
  const int k = b & 7, i = b >> 3;
  return k * q + min(k, rem) + i;
}

template <int S, int MODE>
__global__ __launch_bounds__(kWave) void step_kernel(const Tile* __restrict__ tiles, int ntiles,
                                                     int gphase) {
  for (int b = blockIdx.x; b < ntiles; b += gridDim.x) {
    const int t = xcd_tile(b, ntiles);
    const Tile tl = tiles[t];
    run_tile<S, MODE>(tl, gphase);
  }
}

__global__ __launch_bounds__(kWave) void finalize_kernel(const double* __restrict__ parts,
                                                         int ntiles, double* out) {
  double sums[kPartials];
  sum_partials(parts, ntiles, sums);
  if ((threadIdx.x & (kWave - 1)) == 0)
    for (int q = 0; q < kPartials; ++q) out[q] = sums[q];
}

// SplitMix64 output function (Steele, Lea & Flood 2014) of state z.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

template <int S>
__global__ void init_kernel(DevDomain D, const double* rho0, const double* T0, double rho_u,
                            double T_u, double noise, unsigned long long seed, int b) {
  using C = Codec<S>;
  const long long n = (long long)D.nx * D.ny;
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < n;
       id += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(id % D.nx), y = (int)(id / D.nx);
    double r;
    if (rho0) {
      r = rho0[id];
    } else {
      const unsigned long long z = splitmix64(seed ^ (unsigned long long)((long long)y * D.nx + x));
      const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
      r = rho_u * (1.0 + noise * (2.0 * u - 1.0));
    }
    const double t = T0 ? T0[id] : T_u;
    typename C::T* buf = (typename C::T*)D.buf[b];
    const long long idx = (long long)y * D.pitch + x;
    const double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                         1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    for (int i = 0; i < 9; ++i) C::st(buf, i * D.plane + idx, (float)(W[i] * (r - (double)D.rho_ref)));
    if (!D.isothermal)
      for (int i = 0; i < 9; ++i)
        C::st(buf, (9 + i) * D.plane + idx, (float)(W[i] * (t - (double)D.T_ref)));
    if (D.bc_x == LBM_BCX_CHANNEL && x == D.nx - 1) {
      D.fold[b][0 * D.ny + y] = (float)(W[3] * (r - (double)D.rho_ref));
      D.fold[b][1 * D.ny + y] = (float)(W[6] * (r - (double)D.rho_ref));
      D.fold[b][2 * D.ny + y] = (float)(W[7] * (r - (double)D.rho_ref));
    }
  }
}

__global__ void copy_kernel(float4* __restrict__ dst, const float4* __restrict__ src, long long n4) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n4;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

// ------------------------------------------------------------------ launchers
#define DISPATCH_STORE(storage, F) \
  switch (storage) {               \
    case LBM_STORE_F32: F(LBM_STORE_F32); break;          \
    case LBM_STORE_F32_DEV: F(LBM_STORE_F32_DEV); break;  \
    case LBM_STORE_F16_DEV: F(LBM_STORE_F16_DEV); break;  \
    case LBM_STORE_BF16_DEV: F(LBM_STORE_BF16_DEV); break; \
    default: return hipErrorInvalidValue;                 \
  }

hipError_t lbm_launch_step(int storage, const Tile* tiles, int ntiles, int grid, int phase,
                           hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (grid <= 0 || grid > ntiles) grid = ntiles;
#define L(SS) hipLaunchKernelGGL((step_kernel<SS, MODE_STEP>), dim3(grid), dim3(kWave), 0, s, tiles, ntiles, phase)
  DISPATCH_STORE(storage, L)
#undef L
  return hipGetLastError();
}

hipError_t lbm_launch_readout(int storage, const Tile* tiles, int ntiles, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
#define L(SS) hipLaunchKernelGGL((step_kernel<SS, MODE_READOUT>), dim3(ntiles), dim3(kWave), 0, s, tiles, ntiles, phase)
  DISPATCH_STORE(storage, L)
#undef L
  return hipGetLastError();
}

hipError_t lbm_launch_finalize(DevDomain*, const double* partials, int ntiles, double* out8,
                               hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kWave), 0, s, partials, ntiles, out8);
  return hipGetLastError();
}

hipError_t lbm_launch_init(int storage, DevDomain*, const DevDomain& dh, const double* rho0,
                           const double* T0, double rho_u, double T_u, double noise,
                           unsigned long long seed, int b, hipStream_t s) {
  const long long n = (long long)dh.nx * dh.ny;
  const int block = 256;
  const int grid = (int)std::min<long long>((n + block - 1) / block, 65536);
#define L(SS) hipLaunchKernelGGL((init_kernel<SS>), dim3(grid), dim3(block), 0, s, dh, rho0, T0, rho_u, T_u, noise, seed, b)
  DISPATCH_STORE(storage, L)
#undef L
  return hipGetLastError();
}

hipError_t lbm_launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const long long n4 = (long long)(bytes / 16);
  const int block = 256;
  const int grid = (int)std::min<long long>((n4 + block - 1) / block, 256 * 64);
  if (n4 > 0)
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(block), 0, s, (float4*)dst, (const float4*)src, n4);
  return hipGetLastError();
}
