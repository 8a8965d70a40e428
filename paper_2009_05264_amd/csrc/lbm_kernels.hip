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
// force are fixed-order FP64: each tile writes its partial sums; in the next
// launch kFin finalizer waves per domain reduce slices of them, and the
// launch after that sums the slices (kernel boundaries order every step).
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
// Distributions are addressed as (wave-uniform base, 32-bit per-lane byte
// offset) in the global address space, which maps every load and store to
// one saddr+voffset instruction.
#define AS1 __attribute__((address_space(1)))
#define AS4 __attribute__((address_space(4)))
typedef const char AS1* gptr;
typedef char AS1* gptr_w;

__device__ __forceinline__ gptr_w as_global(const void* p) { return (gptr_w)(uintptr_t)p; }

template <int S>
struct Codec;
template <>
struct Codec<LBM_STORE_F32> {
  static constexpr int E = 4;  // bytes per value
  static __device__ __forceinline__ float ld(gptr b, uint32_t off) { return *(const float AS1*)(b + off); }
  static __device__ __forceinline__ void st(gptr_w b, uint32_t off, float v) { *(float AS1*)(b + off) = v; }
};
template <>
struct Codec<LBM_STORE_F32_DEV> : Codec<LBM_STORE_F32> {};
template <>
struct Codec<LBM_STORE_F16_DEV> {
  static constexpr int E = 2;
  static __device__ __forceinline__ float ld(gptr b, uint32_t off) {
    return (float)*(const _Float16 AS1*)(b + off);
  }
  static __device__ __forceinline__ void st(gptr_w b, uint32_t off, float v) {
    v = fminf(fmaxf(v, -65504.f), 65504.f);  // saturate, round to nearest even
    *(_Float16 AS1*)(b + off) = (_Float16)v;
  }
};
template <>
struct Codec<LBM_STORE_BF16_DEV> {
  static constexpr int E = 2;
  static __device__ __forceinline__ float ld(gptr b, uint32_t off) {
    return __uint_as_float(((uint32_t) * (const uint16_t AS1*)(b + off)) << 16);
  }
  static __device__ __forceinline__ void st(gptr_w b, uint32_t off, float v) {
    v = fminf(fmaxf(v, -3.3895313892515355e38f), 3.3895313892515355e38f);
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    *(uint16_t AS1*)(b + off) = (uint16_t)(u >> 16);
  }
};

typedef const DevDomain AS4& DRef;

// Raw buffer access for the interior path: one resource per buffer, a
// wave-uniform byte offset per distribution plane (SGPR) and one per-lane
// byte offset per row (VGPR).
typedef __amdgpu_buffer_rsrc_t Rsrc;
// Byte offsets at or above kRange are outside the resource: stores there are
// dropped and loads return 0 (raw-buffer bounds check), which lets lanes
// without a node of their own issue the same store instruction unmasked.
constexpr int kRange = 0x7FFFFF00;
constexpr int kDrop = 0x7FFFFF00;
__device__ __forceinline__ Rsrc make_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, kRange, 0x00020000);
}
template <int S>
struct BufIO;
template <>
struct BufIO<LBM_STORE_F32> {
  template <int IMM>
  static __device__ __forceinline__ float ld(Rsrc r, int voff, int soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff + IMM * 4, soff, 0));
  }
  static __device__ __forceinline__ void st(Rsrc r, int voff, int soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
  }
};
template <>
struct BufIO<LBM_STORE_F32_DEV> : BufIO<LBM_STORE_F32> {};
template <>
struct BufIO<LBM_STORE_F16_DEV> {
  template <int IMM>
  static __device__ __forceinline__ float ld(Rsrc r, int voff, int soff) {
    const unsigned short u = __builtin_amdgcn_raw_buffer_load_b16(r, voff + IMM * 2, soff, 0);
    return (float)__builtin_bit_cast(_Float16, u);
  }
  static __device__ __forceinline__ void st(Rsrc r, int voff, int soff, float v) {
    v = fminf(fmaxf(v, -65504.f), 65504.f);  // saturate, round to nearest even
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)v), r, voff, soff, 0);
  }
};
template <>
struct BufIO<LBM_STORE_BF16_DEV> {
  template <int IMM>
  static __device__ __forceinline__ float ld(Rsrc r, int voff, int soff) {
    const unsigned short u = __builtin_amdgcn_raw_buffer_load_b16(r, voff + IMM * 2, soff, 0);
    return __uint_as_float(((uint32_t)u) << 16);
  }
  static __device__ __forceinline__ void st(Rsrc r, int voff, int soff, float v) {
    v = fminf(fmaxf(v, -3.3895313892515355e38f), 3.3895313892515355e38f);
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)(u >> 16), r, voff, soff, 0);
  }
};

// Hardware reciprocal and square root (1 ulp); the path needs no correctly
// rounded division.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

__device__ __forceinline__ int wrap(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }
// Periodic wrap of v in [-n, 2n).
__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Peng-Robinson EOS (Eq. 12), pseudopotential (Eq. 11), (dp/dT)_rho.
__device__ __forceinline__ void eos(DRef D, float rho, float T, float& p, float& psi,
                                    float& dpdT, int& clamped) {
  const float s = fsqrt(T * D.inv_Tc);
  const float sa = 1.f + D.kappa * (1.f - s);
  const float alpha = sa * sa;
  const float br = D.b * rho;
  const float r1 = rcp(1.f - br);
  const float r2 = rcp(1.f + br * (2.f - br));
  const float ar2 = D.a * rho * rho * r2;
  p = rho * D.R * T * r1 - alpha * ar2;
  float q = (p - rho * (1.f / 3.f)) * D.c0g2;
  clamped = !(q >= 0.f);
  q = clamped ? 0.f : q;
  psi = fsqrt(q);
  dpdT = rho * D.R * r1 + ar2 * D.kappa * sa * rcp(s * D.Tc);
}

// Raw-buffer pull.  The resource base sits one row and one column before
// the buffer, so the source of direction i is: plane offset (SGPR) + the
// row-and-column offset of its source row at the lane's column (VGPR) +
// (1 - cx_i) elements (immediate).  vf[i] / vg[i] are the per-lane offsets of
// the f / g source of direction i, so[i] the plane offsets (0-8 f, 9-17 g).
template <int S, int I>
__device__ __forceinline__ float ld_dir(Rsrc rs, int voff, int soff) {
  constexpr int imm = 1 - CX[I];
  return BufIO<S>::template ld<imm>(rs, voff, soff);
}

template <int S, bool TH>
__device__ __forceinline__ void pull_dirs(Rsrc rs, const int (&vf)[9], const int (&vg)[9],
                                          const int (&so)[18], float (&h)[9], float (&k)[9]) {
  h[0] = ld_dir<S, 0>(rs, vf[0], so[0]);
  h[1] = ld_dir<S, 1>(rs, vf[1], so[1]);
  h[2] = ld_dir<S, 2>(rs, vf[2], so[2]);
  h[3] = ld_dir<S, 3>(rs, vf[3], so[3]);
  h[4] = ld_dir<S, 4>(rs, vf[4], so[4]);
  h[5] = ld_dir<S, 5>(rs, vf[5], so[5]);
  h[6] = ld_dir<S, 6>(rs, vf[6], so[6]);
  h[7] = ld_dir<S, 7>(rs, vf[7], so[7]);
  h[8] = ld_dir<S, 8>(rs, vf[8], so[8]);
  if (TH) {
    k[0] = ld_dir<S, 0>(rs, vg[0], so[9]);
    k[1] = ld_dir<S, 1>(rs, vg[1], so[10]);
    k[2] = ld_dir<S, 2>(rs, vg[2], so[11]);
    k[3] = ld_dir<S, 3>(rs, vg[3], so[12]);
    k[4] = ld_dir<S, 4>(rs, vg[4], so[13]);
    k[5] = ld_dir<S, 5>(rs, vg[5], so[14]);
    k[6] = ld_dir<S, 6>(rs, vg[6], so[15]);
    k[7] = ld_dir<S, 7>(rs, vg[7], so[16]);
    k[8] = ld_dir<S, 8>(rs, vg[8], so[17]);
  }
}

// MRT collision with exact-difference forcing, in deviation form.  b_k =
// S_k m_k(f - f^eq) - m_k(Delta F) for the moments (rho, e, eps, jx, qx, jy,
// qy, pxx, pxy) of the Lallemand-Luo basis, f* = f - M^-1 b.
__device__ __forceinline__ void collide_f(DRef D, const float h[9], float drho, float jx,
                                          float jy, float ux, float uy, float Fx, float Fy,
                                          float irho, float hs[9]) {
  const float A13 = h[1] + h[3], A24 = h[2] + h[4];
  const float Dg = h[5] + h[6] + h[7] + h[8];
  const float d13 = h[1] - h[3], d24 = h[2] - h[4];
  const float d57 = h[5] - h[7], d86 = h[8] - h[6];
  const float me = -4.f * h[0] - (A13 + A24) + 2.f * Dg;
  const float meps = 4.f * h[0] - 2.f * (A13 + A24) + Dg;
  const float mqx = -2.f * d13 + d57 + d86;
  const float mqy = -2.f * d24 + d57 - d86;
  const float mxx = A13 - A24;
  const float mxy = (h[5] + h[7]) - (h[6] + h[8]);
  const float ru2 = jx * ux + jy * uy;  // rho u^2
  // non-equilibrium parts
  const float ne = me + 2.f * drho - 3.f * ru2;
  const float neps = meps - drho + 3.f * ru2;
  const float nqx = mqx + jx;
  const float nqy = mqy + jy;
  const float nxx = mxx - (jx * ux - jy * uy);
  const float nxy = mxy - jx * uy;
  // forcing: Delta u = F/rho, s = 2u + Delta u
  const float sx = 2.f * ux + Fx * irho, sy = 2.f * uy + Fy * irho;
  const float Fs = Fx * sx + Fy * sy;
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
__device__ __forceinline__ void collide_g(DRef D, const float k[9], float dT, float T,
                                          float uax, float uay, float phi, float ks[9]) {
  const float om = D.omega_g;
  const float tT = om * T;
  const float u2 = uax * uax + uay * uay;
  const float base = om * dT + phi - 1.5f * tT * u2;
  const float keep = 1.f - om;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float cu = (float)CX[i] * uax + (float)CY[i] * uay;
    ks[i] = keep * k[i] + WF[i] * (base + tT * cu * (3.f + 4.5f * cu));
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

// Fixed-order sum of tiles [t0, t1) of SoA partial sums by one wave; every
// lane gets the result.  Loads are issued four tiles at a time per lane.
__device__ __forceinline__ void sum_partials(const double* parts, int stride, int t0, int t1,
                                             double out[kPartials]) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int q = 0; q < kPartials; ++q) {
    const double* a = parts + (long long)q * stride;
    double acc = 0.0;
    int t = t0 + lane;
    for (; t + 3 * kWave < t1; t += 4 * kWave) {
      const double v0 = a[t], v1 = a[t + kWave], v2 = a[t + 2 * kWave], v3 = a[t + 3 * kWave];
      acc += v0;
      acc += v1;
      acc += v2;
      acc += v3;
    }
    for (; t < t1; t += kWave) acc += a[t];
    out[q] = wave_sum(acc);
  }
}

// One wavefront's march over a tile.  Rolling per-lane state: row r just
// pulled (a), row r-1 (b: force, u_act, f collision), row r-2 (c: source and
// g collision), and u_act,y of row r-3 (d).  The loop body is instantiated
// with compile-time stage flags so that the steady-state iteration is one
// straight path with a fixed number of loads and stores.
//
// KIND 0 (interior): every source of the tile lies inside the domain.
// KIND 1 (row edge) and 2 (column edge): the same raw-buffer pull with the
// boundary rules folded into the addresses -- periodic rows wrap in the row
// offsets; a wall row reads the opposite direction at the node itself
// (bounce-back) through its plane offsets; with KIND 2, lanes of the first /
// last column also correct their x-sources (periodic wrap, or the inlet /
// outlet sources).  The value-level parts of the rules (anti-bounce-back
// temperatures, Zou-He, convective blend) are applied when the row is
// consumed.
template <int S, int MODE, int KIND, bool TH>
struct TileRun {
  static constexpr bool EDGE = KIND != 0;  // rows near a wall or the periodic seam
  static constexpr bool XE = KIND == 2;    // the tile reaches column 0 or nx - 1
  using C = Codec<S>;
  DRef D;
  const Tile AS4& tl;
  int lane, phase, nx, ny, x, xc;
  bool chan, walls, interior, xlo, xhi, has_out;
  const float* fold;
  float* fold_dst;
  Rsrc rs, rd;
  int pitch, sst[18];
  float gbar;
  int r_end;
  // boundary tiles: -1 in lanes whose column is 0 (mL) / nx-1 (mR)
  int mL = 0, mR = 0;
  // wall constants, south (S) and north (N): psi of the false wall density
  // at xc and the wall temperature at xc, m(xc-1), m(xc+1)
  float psiS = 0.f, twS0 = 0.f, twS1 = 0.f, twS2 = 0.f;
  float psiN = 0.f, twN0 = 0.f, twN1 = 0.f, twN2 = 0.f;
  bool heat = false;
  Rsrc rfo, rfd;  // outlet memory, this launch's source and destination
  // reductions
  double acc_mass = 0.0, acc_energy = 0.0, acc_q = 0.0, acc_pin = 0.0, acc_pout = 0.0;
  int acc_vap = 0, acc_clamp = 0, acc_nf = 0;
  // prefetched rows, double-buffered: a loaded register is first touched one
  // iteration after its load was issued; pfo: outlet memory of that row
  float ph[2][9], pk[2][9], pfo[2][3];
  // row a (r)
  float a_drho = 0.f, a_jx = 0.f, a_jy = 0.f, a_dT = 0.f, a_psi = 0.f, a_A = 0.f, a_B = 0.f, a_dpdT = 0.f;
  bool sa = false;
  // row b (r-1)
  float bh[9], bk[9];
  float b_drho = 0.f, b_jx = 0.f, b_jy = 0.f, b_dT = 0.f, b_psi = 0.f, b_A = 0.f, b_B = 0.f, b_dpdT = 0.f;
  bool sb = false;
  // row c (r-2)
  float ck[9];
  float c_A = 0.f, c_B = 0.f, c_dT = 0.f, c_dpdT = 0.f, c_irho = 0.f, c_uax = 0.f, c_uay = 0.f;
  bool sc = false;
  // row d (r-3)
  float d_uay = 0.f;
  bool sd = false;

  __device__ __forceinline__ TileRun(const Tile AS4& t, int gphase)
      : D(*(const DevDomain AS4*)t.d), tl(t) {
    lane = threadIdx.x & (kWave - 1);
    phase = gphase ^ D.parity;
    nx = D.nx;
    ny = D.ny;
    chan = XE && D.bc_x == LBM_BCX_CHANNEL;
    walls = EDGE && D.bc_y == LBM_BCY_WALLS;
    fold = D.fold[phase];
    fold_dst = D.fold[phase ^ 1];
    x = tl.x0 - 2 + lane;
    xc = !XE ? x : (chan ? clampi(x, 0, nx - 1) : wrap(x, nx));
    interior = lane >= 2 && lane < kWave - 2 && x < nx;
    xlo = chan && x == 0;
    xhi = chan && x == nx - 1;
    has_out = chan && tl.x0 + kWave - 3 >= nx - 1;
    mL = XE && xc == 0 ? -1 : 0;
    mR = XE && xc == nx - 1 ? -1 : 0;
    pitch = D.pitch;
    constexpr int E = C::E;
    const int plane = (int)D.plane;
    rs = make_rsrc((const char*)D.buf[phase] - (pitch + 1) * E);
    rd = make_rsrc(D.buf[phase ^ 1]);
#pragma unroll
    for (int i = 0; i < 18; ++i) sst[i] = i * plane * E;
    // mean density two states back: sum of the level-1 slices written by the
    // previous launch's finalizers
    double mass = lane < kFin ? D.l1[phase][lane * kPartials + P_MASS] : 0.0;
    mass = wave_sum(mass);
    gbar = (float)((double)D.rho_ref - mass / ((double)nx * (double)ny));
    r_end = MODE == MODE_STEP ? tl.y1 + 1 : tl.y1;
#pragma unroll
    for (int i = 0; i < 9; ++i) ph[0][i] = pk[0][i] = ph[1][i] = pk[1][i] = bh[i] = bk[i] = ck[i] = 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i) pfo[0][i] = pfo[1][i] = 0.f;
    if (EDGE) {
      // Every load and store of a boundary tile is issued unconditionally
      // (offset kDrop where it has nothing to move), so that the march keeps
      // a fixed count of memory operations per row.
      if (XE) {
        rfo = make_rsrc(fold);
        rfd = make_rsrc(fold_dst);
      }
      const bool needS = walls && tl.y0 - 2 <= 0, needN = walls && r_end >= ny - 1;
      const int xm = chan ? max(xc - 1, 0) : (xc == 0 ? nx - 1 : xc - 1);
      const int xp = chan ? min(xc + 1, nx - 1) : (xc == nx - 1 ? 0 : xc + 1);
      const int oS = needS ? xc * 4 : kDrop, oN = needN ? xc * 4 : kDrop;
      const int mS = needS ? xm * 4 : kDrop, mN = needN ? xm * 4 : kDrop;
      const int pS = needS ? xp * 4 : kDrop, pN = needN ? xp * 4 : kDrop;
      const Rsrc rT0 = make_rsrc(D.Tw[0]), rT1 = make_rsrc(D.Tw[1]);
      const Rsrc rP0 = make_rsrc(D.psiw[0]), rP1 = make_rsrc(D.psiw[1]);
      psiS = ld32(rP0, oS);
      twS0 = ld32(rT0, oS);
      twS1 = ld32(rT0, mS);
      twS2 = ld32(rT0, pS);
      psiN = ld32(rP1, oN);
      twN0 = ld32(rT1, oN);
      twN1 = ld32(rT1, mN);
      twN2 = ld32(rT1, pN);
      const int oH = walls && tl.y0 == 0 ? xc * 4 : kDrop;
      heat = __builtin_amdgcn_raw_buffer_load_b32(make_rsrc(D.heater), oH, 0, 0) != 0u;
    }
  }

  static __device__ __forceinline__ float ld32(Rsrc r, int voff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
  }

  template <int B>
  __device__ __forceinline__ void fetch(int rr) {
    constexpr int E = C::E;
    int vf[9], vg[9], so[18];
#pragma unroll
    for (int i = 0; i < 18; ++i) so[i] = sst[i];
    if (!EDGE) {
      const int v0 = (rr * pitch + xc) * E;
      const int vr[3] = {v0, v0 + pitch * E, v0 + 2 * pitch * E};
#pragma unroll
      for (int i = 0; i < 9; ++i) vf[i] = vg[i] = vr[1 - CY[i]];
    } else {
      // a solid row (beyond a wall) moves nothing: every offset is kDrop
      const bool solid = walls && (rr < 0 || rr >= ny);
      const int ro = walls ? clampi(rr, 0, ny - 1) : wrap1(rr, ny);
      const bool wS = walls && ro == 0, wN = walls && ro == ny - 1;
      const int rsr = wS ? ro : (ro == 0 ? ny - 1 : ro - 1);
      const int rnr = wN ? ro : (ro == ny - 1 ? 0 : ro + 1);
      const int PE = pitch * E;
      const int R0 = (rsr + 1) * PE, R1 = (ro + 1) * PE, R2 = (rnr + 1) * PE;
      const int xe = xc * E;
      const int vr[3] = {solid ? kDrop : xe + R0, solid ? kDrop : xe + R1, solid ? kDrop : xe + R2};
#pragma unroll
      for (int i = 0; i < 9; ++i) vf[i] = vg[i] = vr[1 - CY[i]];
      // bounce-back sources: the opposite direction at the node itself
      if (wS) {
        so[2] = sst[4];
        so[5] = sst[7] + E;
        so[6] = sst[8] - E;
        so[11] = sst[13];
        so[14] = sst[16] + E;
        so[15] = sst[17] - E;
      }
      if (wN) {
        so[4] = sst[2];
        so[7] = sst[5] - E;
        so[8] = sst[6] + E;
        so[13] = sst[11];
        so[16] = sst[14] - E;
        so[17] = sst[15] + E;
      }
      if (XE) {
        const int mLr = solid ? 0 : mL, mRr = solid ? 0 : mR;
        const int P = sst[1];
        int cL1, cL5, cL8, gL1, gL5, gL8, cR3, cR6, cR7;
        if (chan) {
          // inlet column: the f slots of 1, 5, 8 (replaced by Zou-He) carry g
          // of 3, 7, 6 at the node itself for the anti-bounce-back rule; the g
          // slots keep their in-buffer ghost source.  Outlet column: the
          // sources of 3, 6, 7 move from column nx to column nx-1.
          cL1 = TH ? 11 * P + E : 0;
          cL5 = (TH && !wS) ? 11 * P + E + (R1 - R0) : 0;
          cL8 = (TH && !wN) ? 7 * P + E + (R1 - R2) : 0;
          gL1 = gL5 = gL8 = 0;
          cR3 = -E;
          cR6 = wS ? 0 : -E;
          cR7 = wN ? 0 : -E;
        } else {
          const int W = nx * E;
          cL1 = W;
          cL5 = wS ? 0 : W;
          cL8 = wN ? 0 : W;
          gL1 = cL1;
          gL5 = cL5;
          gL8 = cL8;
          cR3 = -W;
          cR6 = wS ? 0 : -W;
          cR7 = wN ? 0 : -W;
        }
        vf[1] += mLr & cL1;
        vf[5] += mLr & cL5;
        vf[8] += mLr & cL8;
        vg[1] += mLr & gL1;
        vg[5] += mLr & gL5;
        vg[8] += mLr & gL8;
        vf[3] += mRr & cR3;
        vf[6] += mRr & cR6;
        vf[7] += mRr & cR7;
        vg[3] += mRr & cR3;
        vg[6] += mRr & cR6;
        vg[7] += mRr & cR7;
        const int vo = has_out && !solid ? ro * 4 : kDrop;
        pfo[B][0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rfo, vo, 0, 0));
        pfo[B][1] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rfo, vo, ny * 4, 0));
        pfo[B][2] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rfo, vo, 2 * ny * 4, 0));
      }
    }
    pull_dirs<S, TH>(rs, vf, vg, so, ph[B], pk[B]);
  }

  // Value-level boundary rules of row r (own row ro) on the pulled values.
  __device__ __forceinline__ void fix_row(int ro, float* h, float* k, const float* fo) {
    const bool wS = walls && ro == 0, wN = walls && ro == ny - 1;
    if (TH && wS) {
      const float dT0 = twS0 - D.T_ref, dTm = twS1 - D.T_ref, dTp = twS2 - D.T_ref;
      k[2] = -k[2] + 2.f * WF[2] * dT0;
      k[5] = -k[5] + 2.f * WF[5] * dTm;
      k[6] = -k[6] + 2.f * WF[6] * dTp;
    }
    if (TH && wN) {
      const float dT0 = twN0 - D.T_ref, dTm = twN1 - D.T_ref, dTp = twN2 - D.T_ref;
      k[4] = -k[4] + 2.f * WF[4] * dT0;
      k[7] = -k[7] + 2.f * WF[7] * dTp;
      k[8] = -k[8] + 2.f * WF[8] * dTm;
    }
    if (chan && mL) {
      // Zou-He velocity inlet; anti-bounce-back inlet temperature
      const float u = D.u_in;
      if (TH) {
        const float gin = D.in_geq - D.T_ref;
        k[1] = -h[1] + 2.f * WF[1] * gin;
        if (!wS) k[5] = -h[5] + 2.f * WF[5] * gin;
        if (!wN) k[8] = -h[8] + 2.f * WF[8] * gin;
      }
      const float rin = (D.rho_ref + h[0] + h[2] + h[4] + 2.f * (h[3] + h[6] + h[7])) * D.inv_1mu;
      const float d24 = 0.5f * (h[2] - h[4]);
      h[1] = h[3] + (2.f / 3.f) * rin * u;
      if (!wS) h[5] = h[7] - d24 + rin * u * (1.f / 6.f);
      if (!wN) h[8] = h[6] + d24 + rin * u * (1.f / 6.f);
    }
    if (chan && mR) {
      // convective outlet: blend with the previous step's value
      h[3] = (fo[0] + D.U_out * h[3]) * D.inv_1pU;
      if (!wS) h[6] = (fo[1] + D.U_out * h[6]) * D.inv_1pU;
      if (!wN) h[7] = (fo[2] + D.U_out * h[7]) * D.inv_1pU;
    }
  }

  // ST2: form force and u_act of row r-1; OUT2: also collide f of row r-1
  // and store it (step) or write the read-out fields (read-out);
  // ST3: source and g collision of row r-2; PF: prefetch row r+1.
  // B: prefetch buffer holding row r (row r + 1 goes to the other one).
  template <bool ST2, bool OUT2, bool ST3, bool PF, int B>
  __device__ __forceinline__ void iter(int r) {
    constexpr int E = C::E;
    float* ah = ph[B];
    float* ak = pk[B];
    // ---------------- stage 1: row r
    sa = walls && (r < 0 || r >= ny);
    if (PF) fetch<B ^ 1>(min(r + 1, r_end));
    int fo_off = kDrop;  // outlet memory store of this row
    if (sa) {
      const float psiW = r < 0 ? psiS : psiN;
      a_psi = psiW;
      a_A = D.beta * psiW;
      a_B = psiW * psiW;
    } else {
      const int ry = (!EDGE || walls) ? r : wrap1(r, ny);
      if (EDGE) fix_row(ry, ah, ak, pfo[B]);
      float drho = 0.f, dT = 0.f;
#pragma unroll
      for (int i = 0; i < 9; ++i) drho += ah[i];
      if (TH) {
#pragma unroll
        for (int i = 0; i < 9; ++i) dT += ak[i];
      } else {
        dT = D.T_iso - D.T_ref;
      }
      const float rho = D.rho_ref + drho;
      const float T = D.T_ref + dT;
      a_drho = drho;
      a_dT = dT;
      a_jx = (ah[1] - ah[3]) + (ah[5] - ah[7]) + (ah[8] - ah[6]);
      a_jy = (ah[2] - ah[4]) + (ah[5] - ah[7]) + (ah[6] - ah[8]);
      float p, psi, dpdT;
      int clamped;
      eos(D, rho, T, p, psi, dpdT, clamped);
      a_psi = psi;
      a_A = D.beta * psi;
      a_B = psi * psi;
      a_dpdT = dpdT;
      if (r >= tl.y0 && r < tl.y1) {
        if (interior) {
          acc_mass += (double)rho;
          acc_energy += (double)T;
          acc_vap += rho < D.rho_mid;
          acc_clamp += clamped;
          acc_nf += !(isfinite(rho) && isfinite(T));
        }
        if (EDGE && interior) {
          if (walls && ry == 0 && heat) acc_q += 2.0 * (double)(twS0 - T);
          if (ry == ny / 2) {
            if (x == 0) acc_pin = (double)p;
            if (x == nx - 1) acc_pout = (double)p;
          }
          if (chan && x == nx - 1) fo_off = ry * 4;
        }
      }
    }
    if (XE && MODE == MODE_STEP) {
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(ah[3]), rfd, fo_off, 0, 0);
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(ah[6]), rfd, fo_off, ny * 4, 0);
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(ah[7]), rfd, fo_off, 2 * ny * 4, 0);
    }

    // ---------------- stage 2: row q = r - 1 (b): force, u_act, f collision
    float b_uax = 0.f, b_uay = 0.f, b_irho = 0.f;
    if (ST2 && !sb) {
      float Fx = 0.f, Fy = 0.f;
      if (!D.single_phase) {
        const float VA = D.G1 * b_A + D.G2 * (a_A + c_A);
        const float VB = D.G1 * b_B + D.G2 * (a_B + c_B);
        const float DA = a_A - c_A;
        const float DB = a_B - c_B;
        const float VAr = __shfl_down(VA, 1, kWave), VAl = __shfl_up(VA, 1, kWave);
        const float VBr = __shfl_down(VB, 1, kWave), VBl = __shfl_up(VB, 1, kWave);
        const float DAr = __shfl_down(DA, 1, kWave), DAl = __shfl_up(DA, 1, kWave);
        const float DBr = __shfl_down(DB, 1, kWave), DBl = __shfl_up(DB, 1, kWave);
        const float SAx = VAr - VAl, SBx = VBr - VBl;
        const float SAy = D.G1 * DA + D.G2 * (DAr + DAl);
        const float SBy = D.G1 * DB + D.G2 * (DBr + DBl);
        Fx = -b_psi * SAx - D.half_1mb * SBx;
        Fy = -b_psi * SAy - D.half_1mb * SBy;
      }
      const float dr = b_drho + gbar;  // rho - rho_bar
      Fx += dr * D.ga_x + D.fb_x;
      Fy += dr * D.ga_y + D.fb_y;
      const float rho = D.rho_ref + b_drho;
      b_irho = rcp(rho);
      const float ux = b_jx * b_irho, uy = b_jy * b_irho;
      b_uax = ux + 0.5f * Fx * b_irho;
      b_uay = uy + 0.5f * Fy * b_irho;
      if (OUT2) {
        const int q = r - 1;
        if (MODE == MODE_READOUT) {
          if (interior) {
            const long long o = (long long)q * nx + x;
            D.out[0][o] = rho;
            D.out[1][o] = b_uax;
            D.out[2][o] = b_uay;
            D.out[3][o] = D.T_ref + b_dT;
          }
        } else {
          float hs[9];
          collide_f(D, bh, b_drho, b_jx, b_jy, ux, uy, Fx, Fy, b_irho, hs);
          const int voff = interior ? (q * pitch + x) * E : kDrop;
#pragma unroll
          for (int i = 0; i < 9; ++i) BufIO<S>::st(rd, voff, sst[i], hs[i]);
        }
      }
    }

    // ---------------- stage 3: row c = r - 2: source and g collision
    if (MODE == MODE_STEP && TH && ST3) {
      const int cr = r - 2;
      float uxl = __shfl_up(c_uax, 1, kWave);
      float uxr = __shfl_down(c_uax, 1, kWave);
      if (xlo) uxl = c_uax;
      if (xhi) uxr = c_uax;
      const float dux = 0.5f * (uxr - uxl);
      const float un_c = sb ? c_uay : b_uay, un_m = sb ? -c_uay : b_uay;
      const float us_c = sd ? c_uay : d_uay, us_m = sd ? -c_uay : d_uay;
      const float div_adv = dux + 0.5f * (un_c - us_c);
      const float div_mass = dux + 0.5f * (un_m - us_m);
      const float T = D.T_ref + c_dT;
      const float phi = T * (div_adv - c_dpdT * c_irho * D.inv_cv * div_mass);
      float ks[9];
      collide_g(D, ck, c_dT, T, c_uax, c_uay, phi, ks);
      const int voff = interior ? (cr * pitch + x) * E : kDrop;
#pragma unroll
      for (int i = 0; i < 9; ++i) BufIO<S>::st(rd, voff, sst[9 + i], ks[i]);
    }

    // ---------------- rotate: d <- c <- b <- a
    d_uay = c_uay;
    sd = sc;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      ck[i] = bk[i];
      bk[i] = ak[i];
      bh[i] = ah[i];
    }
    c_A = b_A;
    c_B = b_B;
    c_dT = b_dT;
    c_dpdT = b_dpdT;
    c_irho = b_irho;
    c_uax = b_uax;
    c_uay = b_uay;
    sc = sb;
    b_drho = a_drho;
    b_jx = a_jx;
    b_jy = a_jy;
    b_dT = a_dT;
    b_psi = a_psi;
    b_A = a_A;
    b_B = a_B;
    b_dpdT = a_dpdT;
    sb = sa;
  }

  __device__ __forceinline__ void run() {
    const int y0 = tl.y0, y1 = tl.y1;
    fetch<0>(y0 - 2);
    iter<false, false, false, true, 0>(y0 - 2);
    iter<false, false, false, true, 1>(y0 - 1);
    if (MODE == MODE_STEP) {
      iter<true, false, false, true, 0>(y0);
      iter<true, true, false, true, 1>(y0 + 1);
      // steady state: rows y0+2 .. y1, two per trip (buffers 0, 1)
      int r = y0 + 2;
      for (; r + 1 <= y1; r += 2) {
        iter<true, true, true, true, 0>(r);
        iter<true, true, true, true, 1>(r + 1);
      }
      if (r <= y1) {
        iter<true, true, true, true, 0>(r);
        iter<true, false, true, false, 1>(y1 + 1);
      } else {
        iter<true, false, true, false, 0>(y1 + 1);
      }
    } else {
      iter<true, false, false, true, 0>(y0);
      int r = y0 + 1;
      for (; r + 1 < y1; r += 2) {
        iter<true, true, false, true, 1>(r);
        iter<true, true, false, true, 0>(r + 1);
      }
      if (r < y1) {
        iter<true, true, false, true, 1>(r);
        iter<true, true, false, false, 0>(y1);
      } else {
        iter<true, true, false, false, 1>(y1);
      }
    }
    // tile partial sums (fixed order: lane tree)
    double v[kPartials] = {acc_mass, acc_energy, acc_q, (double)acc_vap, (double)acc_clamp,
                           (double)acc_nf, acc_pin, acc_pout};
#pragma unroll
    for (int q = 0; q < kPartials; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0) {
      double* out = (MODE == MODE_STEP ? D.partials[phase] : D.readout_partials) + tl.local;
#pragma unroll
      for (int q = 0; q < kPartials; ++q) out[(long long)q * D.pstride] = v[q];
    }
  }
};

// Finalizer wave f of a domain: sums slice f of the previous launch's
// per-tile partials into level-1 slot f.  Wave 0 also records the
// diagnostics of the state two launches back (whose level-1 slices the
// previous launch produced) and advances the device step counter.
__device__ void finalize_slice(const FinEntry AS4& fe, int gphase) {
  DRef D = *(const DevDomain AS4*)fe.d;
  const int lane = threadIdx.x & (kWave - 1);
  const int phase = gphase ^ D.parity;
  const int f = fe.f;
  const int T = D.ntiles;
  const int t0 = (int)((long long)T * f / kFin), t1 = (int)((long long)T * (f + 1) / kFin);
  double sums[kPartials];
  sum_partials(D.partials[phase ^ 1], D.pstride, t0, t1, sums);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < kPartials; ++q) D.l1[phase ^ 1][f * kPartials + q] = sums[q];
  }
  if (f == 0) {
    double rec[kPartials];
#pragma unroll
    for (int q = 0; q < kPartials; ++q)
      rec[q] = wave_sum(lane < kFin ? D.l1[phase][lane * kPartials + q] : 0.0);
    if (lane == 0) {
      const long long st = *D.step_dev;
      if (st >= 2) {
        DiagRec& r = D.ring[(st - 2) % kRing];
        r.step = st - 2;
#pragma unroll
        for (int q = 0; q < kPartials; ++q) r.v[q] = rec[q];
      }
      *D.step_dev = st + 1;
    }
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
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2))) void step_kernel(
    const Tile* __restrict__ tiles, int ntiles, const FinEntry* __restrict__ fins, int nfin,
    int gphase) {
  // Blocks [0, nfin_pad) are finalizer waves (nfin_pad: nfin rounded up to
  // the 8 XCDs so tile blocks keep the XCD of their index).
  const int nfin_pad = (nfin + 7) & ~7;
  if (MODE == MODE_STEP && (int)blockIdx.x < nfin_pad) {
    if ((int)blockIdx.x < nfin) finalize_slice(((const FinEntry AS4*)fins)[blockIdx.x], gphase);
    return;
  }
  const int skip = MODE == MODE_STEP ? nfin_pad : 0;
  const int nb = gridDim.x - skip;
  for (int b = blockIdx.x - skip; b < ntiles; b += nb) {
    const int t = xcd_tile(b, ntiles);
    const Tile AS4& tl = ((const Tile AS4*)tiles)[t];
    DRef D = *(const DevDomain AS4*)tl.d;
    const int r_end = MODE == MODE_STEP ? tl.y1 + 1 : tl.y1;
    const bool xin = tl.x0 >= 3 && tl.x0 + kWave - 2 < D.nx;
    const bool yin = tl.y0 - 2 >= 1 && r_end <= D.ny - 2;
    if (D.isothermal) {
      if (!xin) TileRun<S, MODE, 2, false>(tl, gphase).run();
      else if (!yin) TileRun<S, MODE, 1, false>(tl, gphase).run();
      else TileRun<S, MODE, 0, false>(tl, gphase).run();
    } else {
      if (!xin) TileRun<S, MODE, 2, true>(tl, gphase).run();
      else if (!yin) TileRun<S, MODE, 1, true>(tl, gphase).run();
      else TileRun<S, MODE, 0, true>(tl, gphase).run();
    }
  }
}

__global__ __launch_bounds__(kWave) void finalize_kernel(const double* __restrict__ parts,
                                                         int stride, int ntiles, double* out) {
  double sums[kPartials];
  sum_partials(parts, stride, 0, ntiles, sums);
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
  gptr_w buf = as_global(D.buf[b]);
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
    const uint32_t idx = (uint32_t)(y * D.pitch + x);
    const double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                         1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    for (int i = 0; i < 9; ++i)
      C::st(buf, (uint32_t)(i * (uint32_t)D.plane + idx) * C::E, (float)(W[i] * (r - (double)D.rho_ref)));
    if (!D.isothermal)
      for (int i = 0; i < 9; ++i)
        C::st(buf, (uint32_t)((9 + i) * (uint32_t)D.plane + idx) * C::E,
              (float)(W[i] * (t - (double)D.T_ref)));
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

hipError_t lbm_launch_step(int storage, const Tile* tiles, int ntiles, const FinEntry* fins,
                           int nfin, int grid, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (grid <= 0 || grid > ntiles) grid = ntiles;
  grid += (nfin + 7) & ~7;
#define L(SS) hipLaunchKernelGGL((step_kernel<SS, MODE_STEP>), dim3(grid), dim3(kWave), 0, s, tiles, ntiles, fins, nfin, phase)
  DISPATCH_STORE(storage, L)
#undef L
  return hipGetLastError();
}

hipError_t lbm_launch_readout(int storage, const Tile* tiles, int ntiles, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
#define L(SS) hipLaunchKernelGGL((step_kernel<SS, MODE_READOUT>), dim3(ntiles), dim3(kWave), 0, s, tiles, ntiles, (const FinEntry*)nullptr, 0, phase)
  DISPATCH_STORE(storage, L)
#undef L
  return hipGetLastError();
}

hipError_t lbm_launch_finalize(const double* partials, int stride, int ntiles, double* out8,
                               hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kWave), 0, s, partials, stride, ntiles, out8);
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
