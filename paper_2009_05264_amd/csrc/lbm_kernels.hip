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
__device__ __forceinline__ Rsrc make_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, 0x7FFFFFFF, 0x00020000);
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

// Byte offset of distribution plane i (0-8 f, 9-17 g) at element idx.
template <int S>
__device__ __forceinline__ uint32_t boff(DRef D, int i, uint32_t idx) {
  return (uint32_t)(i * (uint32_t)D.plane + idx) * (uint32_t)Codec<S>::E;
}

// Convective outlet for direction I (memory slot M) at node (nx-1, y): the
// value pulled this step at (nx-2, y), i.e. the post-collision value of
// direction I at (nx-1, y - cy_I), blended with the previous step's value.
template <int S, int I, int M>
__device__ __forceinline__ void outlet_dir(DRef D, gptr src, const float* fold, int y, bool thermal,
                                           float h[9], float k[9]) {
  using C = Codec<S>;
  const int ny = D.ny;
  const int ys = y - CY[I];
  if (D.bc_y == LBM_BCY_WALLS && (ys < 0 || ys >= ny)) return;  // wall rule already applied
  const int ysw = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
  const uint32_t sidx = (uint32_t)(ysw * D.pitch + (D.nx - 1));
  const float hn = C::ld(src, boff<S>(D, I, sidx));
  h[I] = (fold[M * ny + y] + D.U_out * hn) * D.inv_1pU;
  if (thermal) k[I] = C::ld(src, boff<S>(D, 9 + I, sidx));
}

// Pull of an interior node (every source inside the domain).  The resource
// base sits one row and one column before the buffer, so the source of
// direction i is  plane offset (SGPR) + row offset of y - cy_i (one of three
// VGPRs) + (1 - cx_i) elements (immediate).
template <int S, int I>
__device__ __forceinline__ float ld_dir(Rsrc rs, const int vrow[3], int soff) {
  constexpr int m = 1 - CY[I];
  constexpr int imm = 1 - CX[I];
  return BufIO<S>::template ld<imm>(rs, vrow[m], soff);
}

template <int S>
__device__ __forceinline__ void pull_fast(Rsrc rs, const int sp[18], const int vrow[3], bool thermal,
                                          float h[9], float k[9]) {
  h[0] = ld_dir<S, 0>(rs, vrow, sp[0]);
  h[1] = ld_dir<S, 1>(rs, vrow, sp[1]);
  h[2] = ld_dir<S, 2>(rs, vrow, sp[2]);
  h[3] = ld_dir<S, 3>(rs, vrow, sp[3]);
  h[4] = ld_dir<S, 4>(rs, vrow, sp[4]);
  h[5] = ld_dir<S, 5>(rs, vrow, sp[5]);
  h[6] = ld_dir<S, 6>(rs, vrow, sp[6]);
  h[7] = ld_dir<S, 7>(rs, vrow, sp[7]);
  h[8] = ld_dir<S, 8>(rs, vrow, sp[8]);
  if (thermal) {
    k[0] = ld_dir<S, 0>(rs, vrow, sp[9]);
    k[1] = ld_dir<S, 1>(rs, vrow, sp[10]);
    k[2] = ld_dir<S, 2>(rs, vrow, sp[11]);
    k[3] = ld_dir<S, 3>(rs, vrow, sp[12]);
    k[4] = ld_dir<S, 4>(rs, vrow, sp[13]);
    k[5] = ld_dir<S, 5>(rs, vrow, sp[14]);
    k[6] = ld_dir<S, 6>(rs, vrow, sp[15]);
    k[7] = ld_dir<S, 7>(rs, vrow, sp[16]);
    k[8] = ld_dir<S, 8>(rs, vrow, sp[17]);
  }
}

// Pull of node (xc, y) from the post-collision buffer with the boundary
// rules (bounce-back / anti-bounce-back at wall rows, Zou-He inlet,
// convective outlet).  xc in [0, nx), y in [0, ny).
template <int S>
__device__ __forceinline__ void pull(DRef D, gptr src, const float* fold, int xc, int y,
                                     bool thermal, float h[9], float k[9]) {
  using C = Codec<S>;
  const int nx = D.nx, ny = D.ny;
  const uint32_t own = (uint32_t)(y * D.pitch + xc);
  const bool walls = D.bc_y == LBM_BCY_WALLS;
  const bool chan = D.bc_x == LBM_BCX_CHANNEL;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    int xs = xc - CX[i];
    int ys = y - CY[i];
    if (walls && (ys < 0 || ys >= ny)) {
      const int o = OPP[i];
      const int xm = chan ? clampi(xs, 0, nx - 1) : (xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs));
      h[i] = C::ld(src, boff<S>(D, o, own));
      if (thermal) {
        const float Tw = (ys < 0 ? D.Tw[0] : D.Tw[1])[xm];
        k[i] = -C::ld(src, boff<S>(D, 9 + o, own)) + 2.f * WF[i] * (Tw - D.T_ref);
      }
    } else {
      ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
      if (!chan) xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
      if (xs >= 0 && xs < nx) {
        const uint32_t idx = (uint32_t)(ys * D.pitch + xs);
        h[i] = C::ld(src, boff<S>(D, i, idx));
        if (thermal) k[i] = C::ld(src, boff<S>(D, 9 + i, idx));
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
    const float rin = (D.rho_ref + h[0] + h[2] + h[4] + 2.f * (h[3] + h[6] + h[7])) * D.inv_1mu;
    const bool unk5 = !(walls && y - 1 < 0);
    const bool unk8 = !(walls && y + 1 >= ny);
    const float d24 = 0.5f * (h[2] - h[4]);
    h[1] = h[3] + (2.f / 3.f) * rin * u;
    if (unk5) h[5] = h[7] - d24 + rin * u * (1.f / 6.f);
    if (unk8) h[8] = h[6] + d24 + rin * u * (1.f / 6.f);
    if (thermal) {
      const float gin = D.in_geq - D.T_ref;
      k[1] = -C::ld(src, boff<S>(D, 9 + 3, own)) + 2.f * WF[1] * gin;
      if (unk5) k[5] = -C::ld(src, boff<S>(D, 9 + 7, own)) + 2.f * WF[5] * gin;
      if (unk8) k[8] = -C::ld(src, boff<S>(D, 9 + 6, own)) + 2.f * WF[8] * gin;
    }
  }
  if (xc == nx - 1) {
    // Convective outlet for 3, 6, 7 from the values just pulled at nx-2.
    outlet_dir<S, 3, 0>(D, src, fold, y, thermal, h, k);
    outlet_dir<S, 6, 1>(D, src, fold, y, thermal, h, k);
    outlet_dir<S, 7, 2>(D, src, fold, y, thermal, h, k);
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

// Per-lane data of the row whose force is being formed (stage 2) and of the
// row below it (stage 3).
struct RowA {  // row r: just pulled
  float h[9], k[9];
  float drho, jx, jy, dT, psi, A, B, dpdT;
};

template <int S, int MODE>
__device__ void run_tile(const Tile AS4& tl, int gphase) {
  using C = Codec<S>;
  DRef D = *(const DevDomain AS4*)tl.d;
  const int lane = threadIdx.x & (kWave - 1);
  const int phase = gphase ^ D.parity;
  const int nx = D.nx, ny = D.ny;
  const bool chan = D.bc_x == LBM_BCX_CHANNEL;
  const bool walls = D.bc_y == LBM_BCY_WALLS;
  const bool thermal = !D.isothermal;
  gptr src = as_global(D.buf[phase]);
  gptr_w dst = as_global(D.buf[phase ^ 1]);
  const float* fold = D.fold[phase];
  float* fold_dst = D.fold[phase ^ 1];

  const int x = tl.x0 - 2 + lane;
  const int xc = chan ? clampi(x, 0, nx - 1) : wrap(x, nx);
  const bool interior = lane >= 2 && lane < kWave - 2 && x < nx;
  const float gbar = (float)((double)D.rho_ref - D.rbar[phase]);  // rho_ref - rho_bar
  const bool xlo = chan && x == 0, xhi = chan && x == nx - 1;

  double acc_mass = 0.0, acc_energy = 0.0, acc_q = 0.0;
  int acc_vap = 0, acc_clamp = 0, acc_nf = 0;
  double acc_pin = 0.0, acc_pout = 0.0;

  // row r (a), row r-1 (b), row r-2 (c); s* = wall row flags
  RowA a;
  bool sa = false;
  float bh[9], bk[9];
  float b_drho = 0.f, b_jx = 0.f, b_jy = 0.f, b_dT = 0.f, b_psi = 0.f, b_A = 0.f, b_B = 0.f, b_dpdT = 0.f;
  bool sb = false;
  float ck[9];
  float c_A = 0.f, c_B = 0.f, c_dT = 0.f, c_dpdT = 0.f, c_irho = 0.f, c_uax = 0.f, c_uay = 0.f;
  bool sc = false;
  float d_uay = 0.f;  // u_act,y of row r-3
  bool sd = false;
#pragma unroll
  for (int i = 0; i < 9; ++i) bh[i] = bk[i] = ck[i] = 0.f;

  const int r_end = MODE == MODE_STEP ? tl.y1 + 1 : tl.y1;
  // The pull of row r + 1 is issued before row r is processed, so its memory
  // latency overlaps the arithmetic of the current iteration.
  float nh[9], nk[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) nh[i] = nk[i] = 0.f;
  // A tile whose 64 columns and their x-neighbours lie inside the domain
  // pulls interior rows with no boundary logic, through buffer resources.
  const bool xfast = tl.x0 >= 3 && tl.x0 + kWave - 2 < nx;
  constexpr int E = C::E;
  const int pitch = D.pitch;
  const int plane = (int)D.plane;
  const Rsrc rs = make_rsrc((const char*)D.buf[phase] - (pitch + 1) * E);
  const Rsrc rd = make_rsrc(D.buf[phase ^ 1]);
  int sst[18];  // byte offset of each distribution plane
#pragma unroll
  for (int i = 0; i < 18; ++i) sst[i] = i * plane * E;
  auto fetch = [&](int rr) {
    if (xfast && rr >= 1 && rr <= ny - 2) {
      const int v0 = (rr * pitch + xc) * E;
      const int vrow[3] = {v0, v0 + pitch * E, v0 + 2 * pitch * E};
      pull_fast<S>(rs, sst, vrow, thermal, nh, nk);
    }
    else if (!(walls && (rr < 0 || rr >= ny))) {
      pull<S>(D, src, fold, xc, walls ? rr : wrap(rr, ny), thermal, nh, nk);
    }
  };
  fetch(tl.y0 - 2);
  for (int r = tl.y0 - 2; r <= r_end; ++r) {
    // ---------------- stage 1: row r
    sa = walls && (r < 0 || r >= ny);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      a.h[i] = nh[i];
      a.k[i] = nk[i];
    }
    if (r < r_end) fetch(r + 1);
    if (sa) {
      const float pw = (r < 0 ? D.psiw[0] : D.psiw[1])[xc];
      a.psi = pw;
      a.A = D.beta * pw;
      a.B = pw * pw;
    } else {
      const int ry = walls ? r : wrap(r, ny);
      float drho = 0.f, dT = 0.f;
#pragma unroll
      for (int i = 0; i < 9; ++i) drho += a.h[i];
      if (thermal) {
#pragma unroll
        for (int i = 0; i < 9; ++i) dT += a.k[i];
      } else {
        dT = D.T_iso - D.T_ref;
      }
      const float rho = D.rho_ref + drho;
      const float T = D.T_ref + dT;
      a.drho = drho;
      a.dT = dT;
      a.jx = (a.h[1] - a.h[3]) + (a.h[5] - a.h[7]) + (a.h[8] - a.h[6]);
      a.jy = (a.h[2] - a.h[4]) + (a.h[5] - a.h[7]) + (a.h[6] - a.h[8]);
      float p, psi, dpdT;
      int clamped;
      eos(D, rho, T, p, psi, dpdT, clamped);
      a.psi = psi;
      a.A = D.beta * psi;
      a.B = psi * psi;
      a.dpdT = dpdT;
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
          fold_dst[0 * ny + ry] = a.h[3];
          fold_dst[1 * ny + ry] = a.h[6];
          fold_dst[2 * ny + ry] = a.h[7];
        }
      }
    }

    // ---------------- stage 2: row q = r - 1 (b): force, u_act, f collision
    float b_uax = 0.f, b_uay = 0.f, b_irho = 0.f;
    if (r >= tl.y0 && !sb) {
      float Fx = 0.f, Fy = 0.f;
      if (!D.single_phase) {
        const float VA = D.G1 * b_A + D.G2 * (a.A + c_A);
        const float VB = D.G1 * b_B + D.G2 * (a.B + c_B);
        const float DA = a.A - c_A;
        const float DB = a.B - c_B;
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
      const int q = r - 1;
      if (MODE == MODE_READOUT) {
        if (interior && q >= tl.y0 && q < tl.y1) {
          const long long o = (long long)q * nx + x;
          D.out[0][o] = rho;
          D.out[1][o] = b_uax;
          D.out[2][o] = b_uay;
          D.out[3][o] = D.T_ref + b_dT;
        }
      } else if (q >= tl.y0 && q < tl.y1) {
        float hs[9];
        collide_f(D, bh, b_drho, b_jx, b_jy, ux, uy, Fx, Fy, b_irho, hs);
        if (interior) {
          const int voff = (q * pitch + x) * E;
#pragma unroll
          for (int i = 0; i < 9; ++i) BufIO<S>::st(rd, voff, sst[i], hs[i]);
        }
      }
    }

    // ---------------- stage 3: row c = r - 2: source and g collision
    if (MODE == MODE_STEP && thermal && r >= tl.y0 + 2) {
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
      if (interior) {
        const int voff = (cr * pitch + x) * E;
#pragma unroll
        for (int i = 0; i < 9; ++i) BufIO<S>::st(rd, voff, sst[9 + i], ks[i]);
      }
    }

    // ---------------- rotate: d <- c <- b <- a
    d_uay = c_uay;
    sd = sc;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      ck[i] = bk[i];
      bk[i] = a.k[i];
      bh[i] = a.h[i];
    }
    c_A = b_A;
    c_B = b_B;
    c_dT = b_dT;
    c_dpdT = b_dpdT;
    c_irho = b_irho;
    c_uax = b_uax;
    c_uay = b_uay;
    sc = sb;
    b_drho = a.drho;
    b_jx = a.jx;
    b_jy = a.jy;
    b_dT = a.dT;
    b_psi = a.psi;
    b_A = a.A;
    b_B = a.B;
    b_dpdT = a.dpdT;
    sb = sa;
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

// Sum of the previous launch's per-tile partials of one domain: lagged mean
// density for the buoyancy force, the diagnostics record, the step counter.
__device__ void finalize_domain(DRef D, int gphase) {
  const int lane = threadIdx.x & (kWave - 1);
  const int phase = gphase ^ D.parity;
  double sums[kPartials];
  sum_partials(D.partials[phase ^ 1], D.ntiles, sums);
  if (lane == 0) {
    const long long st = *D.step_dev;
    D.rbar[phase ^ 1] = sums[P_MASS] / ((double)D.nx * (double)D.ny);
    DiagRec& rec = D.ring[(st + kRing) % kRing];
    rec.step = st - 1;
#pragma unroll
    for (int q = 0; q < kPartials; ++q) rec.v[q] = sums[q];
    *D.step_dev = st + 1;
  }
}

// Blocks [0, kFinalizers) finalize the domains' reductions while the other
// blocks process tiles; tile blocks keep the XCD of their index (kFinalizers
// is a multiple of the 8 XCDs).
constexpr int kFinalizers = 8;

template <int S, int MODE>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(3))) void step_kernel(
    const Tile* __restrict__ tiles, int ntiles, DevDomain* const* __restrict__ doms, int ndoms,
    int gphase) {
  if (MODE == MODE_STEP && blockIdx.x < kFinalizers) {
    for (int i = blockIdx.x; i < ndoms; i += kFinalizers)
      finalize_domain(*(const DevDomain AS4*)((DevDomain* const AS4*)doms)[i], gphase);
    return;
  }
  const int nb = gridDim.x - (MODE == MODE_STEP ? kFinalizers : 0);
  for (int b = blockIdx.x - (MODE == MODE_STEP ? kFinalizers : 0); b < ntiles; b += nb) {
    const int t = xcd_tile(b, ntiles);
    run_tile<S, MODE>(((const Tile AS4*)tiles)[t], gphase);
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

hipError_t lbm_launch_step(int storage, const Tile* tiles, int ntiles, DevDomain* const* doms,
                           int ndoms, int grid, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (grid <= 0 || grid > ntiles) grid = ntiles;
  grid += kFinalizers;
#define L(SS) hipLaunchKernelGGL((step_kernel<SS, MODE_STEP>), dim3(grid), dim3(kWave), 0, s, tiles, ntiles, doms, ndoms, phase)
  DISPATCH_STORE(storage, L)
#undef L
  return hipGetLastError();
}

hipError_t lbm_launch_readout(int storage, const Tile* tiles, int ntiles, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
#define L(SS) hipLaunchKernelGGL((step_kernel<SS, MODE_READOUT>), dim3(ntiles), dim3(kWave), 0, s, tiles, ntiles, (DevDomain* const*)nullptr, 0, phase)
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
