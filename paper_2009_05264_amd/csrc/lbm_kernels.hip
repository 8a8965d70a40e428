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
// FP16 or BF16 (template parameter), one plane per direction holding the
// (f_i, g_i) pair of every node (f_i alone for isothermal domains); the
// nine direction planes of a row are stored one after the other, so that
// the rows a wave pulls and stores lie together in memory.
//
// Reductions for the diagnostics are fixed-order FP64: each tile writes its
// partial sums; in the next launch kFin finalizer waves per domain reduce
// slices of them, and the launch after that sums the slices (kernel
// boundaries order every step).  The mean density of the buoyancy force
// (Eq. 14) is that of the previous state: every tile adds the exact
// fixed-point mass of its nodes into running totals with integer atomics
// (order-free, so bitwise reproducible), and the next launch's tiles read
// the totals and subtract their own previous reading.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

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
  static __device__ __forceinline__ void st(gptr_w b, uint32_t off, float v) { *(float AS1*)(b + off) = v; }
};
template <>
struct Codec<LBM_STORE_F32_DEV> : Codec<LBM_STORE_F32> {};
template <>
struct Codec<LBM_STORE_F16_DEV> {
  static constexpr int E = 2;
  static __device__ __forceinline__ void st(gptr_w b, uint32_t off, float v) {
    v = fminf(fmaxf(v, -65504.f), 65504.f);  // saturate, round to nearest even
    *(_Float16 AS1*)(b + off) = (_Float16)v;
  }
};
template <>
struct Codec<LBM_STORE_BF16_DEV> {
  static constexpr int E = 2;
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
// two-element vectors for the packed 16-bit conversions of the stores
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
// Cache-policy operand of the state stores: 0 (default, write-back in the L2)
// or kWriteThrough (SC1: agent-scope stores, which the L2 writes through);
// the host picks one per launch from the size of the state it touches.
constexpr int kWriteThrough = 16;
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
  static constexpr bool kRaw = false;  // as PairIO
  static __device__ __forceinline__ float unpack(float w) { return w; }
  template <int IMM>
  static __device__ __forceinline__ float ld(Rsrc r, int voff, int soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff + IMM * 4, soff, 0));
  }
  template <int CP>
  static __device__ __forceinline__ void st(Rsrc r, int voff, int soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, CP);
  }
};
template <>
struct BufIO<LBM_STORE_F32_DEV> : BufIO<LBM_STORE_F32> {};

// Thermal domains store f_i and g_i of a node side by side (one 8-byte or
// 4-byte pair), so one load or store moves both distributions of a
// direction.  IMM is an offset in pairs.
//
// kRaw: the 16-bit formats load the packed bits into the prefetch registers
// (f holds the word, g is left alone) and unpack() converts them when the
// row is consumed.  Converting at load time would make the loop wait, before
// its back-edge, for the row it has just prefetched.
template <int S>
struct PairIO;
template <>
struct PairIO<LBM_STORE_F32> {
  static constexpr int E2 = 8;
  static constexpr bool kRaw = false;
  static __device__ __forceinline__ void unpack(float, float&, float&) {}
  template <int IMM>
  static __device__ __forceinline__ void ld(Rsrc r, int voff, int soff, float& f, float& g) {
    const unsigned long long w =
        __builtin_bit_cast(unsigned long long, __builtin_amdgcn_raw_buffer_load_b64(r, voff + IMM * E2, soff, 0));
    f = __uint_as_float((uint32_t)w);
    g = __uint_as_float((uint32_t)(w >> 32));
  }
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  template <int CP>
  static __device__ __forceinline__ void st(Rsrc r, int voff, int soff, float f, float g) {
    // Empty register constraint: keeps the pair operands as register values,
    // so that the packing below is not rewritten into a widened memory load
    // of the source arrays (which would pin them in private memory).
    asm("" : "+v"(f), "+v"(g));
    const unsigned long long w = (unsigned long long)__float_as_uint(f) |
                                 ((unsigned long long)__float_as_uint(g) << 32);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, w), r, voff, soff, CP);
  }
};
template <>
struct PairIO<LBM_STORE_F32_DEV> : PairIO<LBM_STORE_F32> {};
template <>
struct PairIO<LBM_STORE_F16_DEV> {
  static constexpr int E2 = 4;
  static constexpr bool kRaw = true;
  template <int IMM>
  static __device__ __forceinline__ void ld(Rsrc r, int voff, int soff, float& f, float& g) {
    f = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff + IMM * E2, soff, 0));
  }
  static __device__ __forceinline__ void unpack(float w, float& f, float& g) {
    const uint32_t u = __float_as_uint(w);
    f = (float)__builtin_bit_cast(_Float16, (unsigned short)(u & 0xFFFFu));
    g = (float)__builtin_bit_cast(_Float16, (unsigned short)(u >> 16));
  }
  // saturate, then round both to nearest even in one packed conversion
  // (f in the low half)
  template <int CP>
  static __device__ __forceinline__ void st(Rsrc r, int voff, int soff, float f, float g) {
    const f32x2 v = {fminf(fmaxf(f, -65504.f), 65504.f), fminf(fmaxf(g, -65504.f), 65504.f)};
    const uint32_t w = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
    __builtin_amdgcn_raw_buffer_store_b32(w, r, voff, soff, CP);
  }
};
template <>
struct PairIO<LBM_STORE_BF16_DEV> {
  static constexpr int E2 = 4;
  static constexpr bool kRaw = true;
  template <int IMM>
  static __device__ __forceinline__ void ld(Rsrc r, int voff, int soff, float& f, float& g) {
    f = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff + IMM * E2, soff, 0));
  }
  static __device__ __forceinline__ void unpack(float w, float& f, float& g) {
    const uint32_t u = __float_as_uint(w);
    f = __uint_as_float(u << 16);
    g = __uint_as_float(u & 0xFFFF0000u);
  }
  // saturate to the largest finite value, then round both to nearest even
  // in one packed conversion (f in the low half)
  template <int CP>
  static __device__ __forceinline__ void st(Rsrc r, int voff, int soff, float f, float g) {
    constexpr float kMax = 3.3895313892515355e38f;
    const f32x2 v = {fminf(fmaxf(f, -kMax), kMax), fminf(fmaxf(g, -kMax), kMax)};
    const uint32_t w = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
    __builtin_amdgcn_raw_buffer_store_b32(w, r, voff, soff, CP);
  }
};
template <>
struct BufIO<LBM_STORE_F16_DEV> {
  static constexpr bool kRaw = true;
  template <int IMM>
  static __device__ __forceinline__ float ld(Rsrc r, int voff, int soff) {
    return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, voff + IMM * 2, soff, 0));
  }
  static __device__ __forceinline__ float unpack(float w) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)__float_as_uint(w));
  }
  template <int CP>
  static __device__ __forceinline__ void st(Rsrc r, int voff, int soff, float v) {
    v = fminf(fmaxf(v, -65504.f), 65504.f);  // saturate, round to nearest even
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)v), r, voff, soff, CP);
  }
};
template <>
struct BufIO<LBM_STORE_BF16_DEV> {
  static constexpr bool kRaw = true;
  template <int IMM>
  static __device__ __forceinline__ float ld(Rsrc r, int voff, int soff) {
    return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, voff + IMM * 2, soff, 0));
  }
  static __device__ __forceinline__ float unpack(float w) { return __uint_as_float(__float_as_uint(w) << 16); }
  template <int CP>
  static __device__ __forceinline__ void st(Rsrc r, int voff, int soff, float v) {
    v = fminf(fmaxf(v, -3.3895313892515355e38f), 3.3895313892515355e38f);
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)(u >> 16), r, voff, soff, CP);
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
// One reciprocal square root gives both sqrt(T/Tc) = T / sqrt(T Tc) and the
// 1 / sqrt(T Tc) of d alpha / dT; one reciprocal of the product of the two
// denominators gives both of their reciprocals.
__device__ __forceinline__ void eos(DRef D, float rho, float T, float& p, float& psi,
                                    float& dpdT, int& clamped) {
  const float rs = __builtin_amdgcn_rsqf(T * D.Tc);  // 1 / sqrt(T Tc)
  const float s = T * rs;                             // sqrt(T / Tc)
  const float sa = 1.f + D.kappa * (1.f - s);
  const float alpha = sa * sa;
  const float br = D.b * rho;
  const float d1 = 1.f - br;
  const float d2 = 1.f + br * (2.f - br);
  const float rp = rcp(d1 * d2);
  const float r1 = d2 * rp;  // 1 / (1 - b rho)
  const float r2 = d1 * rp;  // 1 / (1 + 2 b rho - b^2 rho^2)
  const float ar2 = D.a * rho * rho * r2;
  p = rho * D.R * T * r1 - alpha * ar2;
  float q = (p - rho * (1.f / 3.f)) * D.c0g2;
  clamped = !(q >= 0.f);
  q = clamped ? 0.f : q;
  psi = fsqrt(q);
  dpdT = rho * D.R * r1 + ar2 * D.kappa * sa * rs;
}

// Raw-buffer pull.  The resource base sits one row and one column before
// the buffer (and, for column-edge tiles, a further offset below it, see
// TileRun), so the source of direction i is: plane offset so[i] (SGPR) +
// the row-and-column offset vf[i] of its source row at the lane's column
// (VGPR) + (1 - cx_i) elements (immediate).  Thermal domains load the
// (f_i, g_i) pair of the source in one access; isothermal ones f_i alone.
template <int S, bool TH, int I>
__device__ __forceinline__ void ld_dir(Rsrc rs, int voff, int soff, float& f, float& g) {
  constexpr int imm = 1 - CX[I];
  if (TH)
    PairIO<S>::template ld<imm>(rs, voff, soff, f, g);
  else
    f = BufIO<S>::template ld<imm>(rs, voff, soff);
}

template <int S, bool TH>
__device__ __forceinline__ void pull_dirs(Rsrc rs, const int (&vf)[9], const int (&so)[9], float (&h)[9],
                                          float (&k)[9]) {
  ld_dir<S, TH, 0>(rs, vf[0], so[0], h[0], k[0]);
  ld_dir<S, TH, 1>(rs, vf[1], so[1], h[1], k[1]);
  ld_dir<S, TH, 2>(rs, vf[2], so[2], h[2], k[2]);
  ld_dir<S, TH, 3>(rs, vf[3], so[3], h[3], k[3]);
  ld_dir<S, TH, 4>(rs, vf[4], so[4], h[4], k[4]);
  ld_dir<S, TH, 5>(rs, vf[5], so[5], h[5], k[5]);
  ld_dir<S, TH, 6>(rs, vf[6], so[6], h[6], k[6]);
  ld_dir<S, TH, 7>(rs, vf[7], so[7], h[7], k[7]);
  ld_dir<S, TH, 8>(rs, vf[8], so[8], h[8], k[8]);
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
  // c_i . u_act, written out (no multiplications by zero components)
  const float cu[9] = {0.f, uax, uay, -uax, -uay, uax + uay, uay - uax, -uax - uay, uax - uay};
  ks[0] = keep * k[0] + WF[0] * base;
#pragma unroll
  for (int i = 1; i < 9; ++i) ks[i] = keep * k[i] + WF[i] * (base + tT * cu[i] * (3.f + 4.5f * cu[i]));
}

// Neighbour exchange across the wavefront by DPP wave shifts: shfl_dn1
// gives lane i the value of lane i + 1, shfl_up1 that of lane i - 1; the
// end lane without a source (63, resp. 0) reads 0.  Those are outer halo
// lanes: what they form reaches only the other halo lane's stage 3, and
// neither stores nor adds to the tile sums.  (A move with no previous
// value to keep needs no copy of its source into the destination.)
__device__ __forceinline__ float shfl_dn1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xF, 0xF, true));  // wave_shl:1
}
__device__ __forceinline__ float shfl_up1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xF, 0xF, true));  // wave_shr:1
}

// One DPP move of a 32-bit value; lanes of rows outside ROWS get 0 (a
// move of all rows keeps no previous value, so it needs no copy).
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i32(int v) {
  if constexpr (ROWS == 0xF)
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
  else
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, false);
}

// The same move of a double (both halves).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = dpp_i32<CTRL, ROWS>((int)(unsigned)u);
  const int hi = dpp_i32<CTRL, ROWS>((int)(unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the wavefront in a fixed order by DPP moves: two quad
// permutations and the two mirrors leave every lane of a 16-lane row with
// the row's sum; two row broadcasts then accumulate rows 0-3 into lane 63,
// whose value every lane gets.  Called with every lane active.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_f64<0x140, 0xF>(v);  // row_mirror
  v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum of v over lanes 0-15 (an inclusive scan along the first DPP row,
// whose last lane then holds the total), returned to every lane.
__device__ __forceinline__ unsigned long long row0_sum_u64(unsigned long long v) {
  // lanes without a source (the first of each row) read 0
  auto shr = [](unsigned long long x, auto ctrl) {
    const int lo = dpp_i32<decltype(ctrl)::value, 0xF>((int)(unsigned)x);
    const int hi = dpp_i32<decltype(ctrl)::value, 0xF>((int)(unsigned)(x >> 32));
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
  };
  v += shr(v, std::integral_constant<int, 0x111>{});  // row_shr:1
  v += shr(v, std::integral_constant<int, 0x112>{});  // row_shr:2
  v += shr(v, std::integral_constant<int, 0x114>{});  // row_shr:4
  v += shr(v, std::integral_constant<int, 0x118>{});  // row_shr:8
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 15);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 15);
  return ((unsigned long long)hi << 32) | lo;
}

// Fixed-point form (2^32 units) of a tile's mass sum; non-finite or absurd
// sums (a diverged run, flagged by the non-finite count) contribute zero.
__device__ __forceinline__ unsigned long long to_fixed(double m) {
  return (unsigned long long)(long long)(fabs(m) < 1e9 ? m * kMassScale : 0.0);
}

// The same tree for 32-bit integers (exact).
__device__ __forceinline__ int wave_sum_int(int v) {
  v += dpp_i32<0xB1, 0xF>(v);
  v += dpp_i32<0x4E, 0xF>(v);
  v += dpp_i32<0x141, 0xF>(v);
  v += dpp_i32<0x140, 0xF>(v);
  v += dpp_i32<0x142, 0xA>(v);
  v += dpp_i32<0x143, 0xC>(v);
  return __builtin_amdgcn_readlane(v, 63);
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
template <int S, int MODE, int KIND, bool TH, int NB, bool WT>
struct TileRun {
  static constexpr bool EDGE = KIND != 0;  // rows near a wall or the periodic seam
  static constexpr int CP = WT ? kWriteThrough : 0;  // cache policy of the state stores
  static constexpr bool XE = KIND == 2;    // the tile reaches column 0 or nx - 1
  static_assert(NB >= 2 && NB <= 4, "prefetch depth");
  using C = Codec<S>;
  // bytes per plane element: an (f, g) pair, or f alone when isothermal
  static constexpr int E2 = TH ? PairIO<S>::E2 : C::E;
  DRef D;
  const Tile AS4& tl;
  int lane, phase, nx, ny, x, xc;
  bool chan, walls, interior, xlo, xhi, has_out;
  const float* fold;
  float* fold_dst;
  Rsrc rs, rd;
  int pitch;    // elements from a row to the next in one direction plane
  int sst[9];   // byte offsets of the direction planes within a row
  int kb;             // extra base offset of the pull resource (column-edge tiles)
  float gbar;     // rho_ref - mean density (formed in run(), first used by stage 2)
  unsigned long long mtot, mprev;  // running mass totals: one slot per lane; this tile's previous reading
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
  double mass_tile = 0.0;  // wave total of acc_mass once the tile's rows are in (stepping)
  int acc_vap = 0, acc_clamp = 0, acc_nf = 0;
  // prefetched rows in NB rotating buffers: the loads of row r + NB - 1 are
  // issued while row r is consumed, so a loaded register is first touched
  // NB - 1 iterations after its load was issued; pfo: outlet memory of the row
  float ph[NB][9], pk[NB][9], pfo[NB][3];
  // row a (r)
  float a_drho = 0.f, a_jx = 0.f, a_jy = 0.f, a_dT = 0.f, a_psi = 0.f, a_A = 0.f, a_B = 0.f, a_dpdT = 0.f;
  bool sa = false;
  // row b (r-1)
  float bh[9], bk[9];
  float b_drho = 0.f, b_jx = 0.f, b_jy = 0.f, b_dT = 0.f, b_psi = 0.f, b_A = 0.f, b_B = 0.f, b_dpdT = 0.f;
  bool sb = false;
  // row c (r-2); fc: post-collision f of row c, stored with its g
  float ck[9], fc[9];
  float c_A = 0.f, c_B = 0.f, c_dT = 0.f, c_dpdT = 0.f, c_irho = 0.f, c_uax = 0.f, c_uay = 0.f;
  bool sc = false;
  // row d (r-3)
  float d_uay = 0.f;
  bool sd = false;

  __device__ __forceinline__ TileRun(const Tile AS4& t, int gphase)
      : D(*(const DevDomain AS4*)t.d), tl(t) {
    lane = threadIdx.x & (kWave - 1);
    // The first row loads need only the tile record: buffers, sizes and
    // strides come from it, not from the descriptor it points to.
    phase = gphase ^ tl.parity;
    nx = tl.nx;
    ny = tl.ny;
    chan = XE && D.bc_x != LBM_BCX_PERIODIC;
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
    pitch = tl.ystride;
    const int plane = tl.istride;
#pragma unroll
    for (int i = 0; i < 9; ++i) sst[i] = i * plane * E2;
    // Column-edge tiles of thermal domains redirect some inlet sources to a
    // lower plane (a negative per-lane offset): their resource base sits two
    // planes lower still, so every per-lane offset stays non-negative.
    kb = XE && TH ? 2 * sst[1] : 0;
    // both pointers at fixed offsets of the record, then selected
    void* const b0 = tl.buf[0];
    void* const b1 = tl.buf[1];
    rs = make_rsrc((const char*)(phase ? b1 : b0) - kb - (pitch + 1) * E2);
    rd = make_rsrc(phase ? b0 : b1);
    r_end = MODE == MODE_STEP ? tl.y1 + 1 : tl.y1;
#pragma unroll
    for (int i = 0; i < 9; ++i) bh[i] = bk[i] = ck[i] = fc[i] = 0.f;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int i = 0; i < 9; ++i) ph[b][i] = pk[b][i] = 0.f;
#pragma unroll
      for (int i = 0; i < 3; ++i) pfo[b][i] = 0.f;
    }
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

  // this state's mass for the next launch's buoyancy: each lane's FP64 sum
  // of FP32 densities is exact, and so is the tile's FP64 total (at most 64
  // x ~2^14 with a 2^-32 grain for densities above 2^-9), so the fixed-point
  // total is exact and tiling-independent
  __device__ __forceinline__ void flush_mass() {
    mass_tile = wave_sum(acc_mass);
    const unsigned long long m = to_fixed(mass_tile);
    if (lane == 0)
      __hip_atomic_fetch_add(&D.macc[phase][(tl.local & (kAccSlots - 1)) * kAccStride], m, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }

  static __device__ __forceinline__ float ld32(Rsrc r, int voff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
  }

  // Pull row rr into buffer B.  A row past the tile's last one (the
  // look-ahead of the final iterations) is issued with offset kDrop, which
  // moves nothing, so every iteration has the same memory operations.
  template <int B>
  __device__ __forceinline__ void fetch(int rr) {
    const bool past = rr > r_end;
    int vf[9], so[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) so[i] = sst[i];
    if (!EDGE) {
      const int v0 = (rr * pitch + xc) * E2;
      const int vr[3] = {past ? kDrop : v0, past ? kDrop : v0 + pitch * E2, past ? kDrop : v0 + 2 * pitch * E2};
#pragma unroll
      for (int i = 0; i < 9; ++i) vf[i] = vr[1 - CY[i]];
    } else {
      // a solid row (beyond a wall) moves nothing: every offset is kDrop
      const bool solid = past || (walls && (rr < 0 || rr >= ny));
      const int ro = walls ? clampi(rr, 0, ny - 1) : wrap1(rr, ny);
      const bool wS = walls && ro == 0, wN = walls && ro == ny - 1;
      const int rsr = wS ? ro : (ro == 0 ? ny - 1 : ro - 1);
      const int rnr = wN ? ro : (ro == ny - 1 ? 0 : ro + 1);
      const int PE = pitch * E2;
      const int R0 = (rsr + 1) * PE, R1 = (ro + 1) * PE, R2 = (rnr + 1) * PE;
      const int xe = xc * E2 + kb;
      const int vr[3] = {solid ? kDrop : xe + R0, solid ? kDrop : xe + R1, solid ? kDrop : xe + R2};
#pragma unroll
      for (int i = 0; i < 9; ++i) vf[i] = vr[1 - CY[i]];
      // bounce-back sources: the opposite direction at the node itself
      if (wS) {
        so[2] = sst[4];
        so[5] = sst[7] + E2;
        so[6] = sst[8] - E2;
      }
      if (wN) {
        so[4] = sst[2];
        so[7] = sst[5] - E2;
        so[8] = sst[6] + E2;
      }
      if (XE) {
        const int mLr = solid ? 0 : mL, mRr = solid ? 0 : mR;
        const int P = sst[1];
        int cL1, cL5, cL8, cR3, cR6, cR7;
        if (chan) {
          // Inlet column: the sources of 1, 5, 8 (ghosts; f is set by Zou-He)
          // move to the pairs of 3, 7, 6 at the node itself, whose g the
          // anti-bounce-back rule needs.  Outlet column: the sources of 3,
          // 6, 7 move from column nx to column nx-1.
          cL1 = TH ? 2 * P + E2 : 0;
          cL5 = (TH && !wS) ? 2 * P + E2 + (R1 - R0) : 0;
          cL8 = (TH && !wN) ? -2 * P + E2 + (R1 - R2) : 0;
          cR3 = -E2;
          cR6 = wS ? 0 : -E2;
          cR7 = wN ? 0 : -E2;
        } else {
          const int W = nx * E2;
          cL1 = W;
          cL5 = wS ? 0 : W;
          cL8 = wN ? 0 : W;
          cR3 = -W;
          cR6 = wS ? 0 : -W;
          cR7 = wN ? 0 : -W;
        }
        vf[1] += mLr & cL1;
        vf[5] += mLr & cL5;
        vf[8] += mLr & cL8;
        vf[3] += mRr & cR3;
        vf[6] += mRr & cR6;
        vf[7] += mRr & cR7;
        const int vo = has_out && !solid ? ro * 4 : kDrop;
        pfo[B][0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rfo, vo, 0, 0));
        pfo[B][1] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rfo, vo, ny * 4, 0));
        pfo[B][2] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rfo, vo, 2 * ny * 4, 0));
      }
    }
    pull_dirs<S, TH>(rs, vf, so, ph[B], pk[B]);
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
        // the pairs pulled for 1, 5, 8 are those of 3, 7, 6 at this node
        k[1] = -k[1] + 2.f * WF[1] * gin;
        if (!wS) k[5] = -k[5] + 2.f * WF[5] * gin;
        if (!wN) k[8] = -k[8] + 2.f * WF[8] * gin;
      }
      const float rin = (D.rho_ref + h[0] + h[2] + h[4] + 2.f * (h[3] + h[6] + h[7])) * D.inv_1mu;
      const float d24 = 0.5f * (h[2] - h[4]);
      h[1] = h[3] + (2.f / 3.f) * rin * u;
      if (!wS) h[5] = h[7] - d24 + rin * u * (1.f / 6.f);
      if (!wN) h[8] = h[6] + d24 + rin * u * (1.f / 6.f);
    }
    if (chan && mR) {
      if (D.bc_x == LBM_BCX_CHANNEL_P) {
        // Constant-pressure outlet: non-equilibrium bounce-back at density
        // rho_out.  The known populations give rho_out (1 + u) = f_0 + f_2 +
        // f_4 + 2 (f_1 + f_5 + f_8); as w_0 + w_2 + w_4 + 2 (w_1 + w_5 +
        // w_8) = 1, in deviation form rho_out u = (rho_ref - rho_out) + the
        // same sum of h, with no cancellation when rho_out = rho_ref.  Next
        // to a wall the redirected pulls already hold the populations of
        // x = nx-2 (zero gradient), which is the corner rule.
        if (!wS && !wN) {
          const float ru = D.dro + h[0] + h[2] + h[4] + 2.f * (h[1] + h[5] + h[8]);
          const float d24 = 0.5f * (h[2] - h[4]);
          h[3] = h[1] - (2.f / 3.f) * ru;
          h[6] = h[8] - d24 - ru * (1.f / 6.f);
          h[7] = h[5] + d24 - ru * (1.f / 6.f);
        }
      } else {
        // convective outlet: blend with the previous step's value
        h[3] = (fo[0] + D.U_out * h[3]) * D.inv_1pU;
        if (!wS) h[6] = (fo[1] + D.U_out * h[6]) * D.inv_1pU;
        if (!wN) h[7] = (fo[2] + D.U_out * h[7]) * D.inv_1pU;
      }
    }
  }

  // ST2: form force and u_act of row r-1; OUT2: also collide f of row r-1
  // and store it (step) or write the read-out fields (read-out);
  // ST3: source and g collision of row r-2; PF: prefetch row r+1.
  // B: prefetch buffer holding row r (row r + 1 goes to the other one).
  template <bool ST2, bool OUT2, bool ST3, bool PF, int B>
  __device__ __forceinline__ void iter(int r) {
    float* ah = ph[B];
    float* ak = pk[B];
    // ---------------- stage 1: row r
    sa = walls && (r < 0 || r >= ny);
    if (PF) fetch<(B + NB - 1) % NB>(r + NB - 1);
    // 16-bit storage: convert the row's packed words now (see PairIO)
    float uh[9], uk[9];
    if constexpr (TH ? PairIO<S>::kRaw : BufIO<S>::kRaw) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        if constexpr (TH)
          PairIO<S>::unpack(ph[B][i], uh[i], uk[i]);
        else
          uh[i] = BufIO<S>::unpack(ph[B][i]);
      }
      ah = uh;
      if constexpr (TH) ak = uk;
    }
    int fo_off = kDrop;  // outlet memory store of this row
    if (sa) {
      // a solid cell enters only the adhesion sum of Eq. 15:
      // -G_wet psi(x) w_i psi_w c_i = -psi(x) (kw G_i) psi_w c_i
      const float psiW = r < 0 ? psiS : psiN;
      a_psi = psiW;
      a_A = D.kw * psiW;
      a_B = 0.f;
    } else {
      const int ry = (!EDGE || walls) ? r : wrap1(r, ny);
      if (EDGE) fix_row(ry, ah, ak, pfo[B]);
      float drho = ah[0], dT;
#pragma unroll
      for (int i = 1; i < 9; ++i) drho += ah[i];
      if (TH) {
        dT = ak[0];
#pragma unroll
        for (int i = 1; i < 9; ++i) dT += ak[i];
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
    float fnew[9];  // post-collision f of row q
#pragma unroll
    for (int i = 0; i < 9; ++i) fnew[i] = 0.f;
    if (ST2 && !sb) {
      float Fx = 0.f, Fy = 0.f;
      if (!D.single_phase) {
        const float VA = D.G1 * b_A + D.G2 * (a_A + c_A);
        const float VB = D.G1 * b_B + D.G2 * (a_B + c_B);
        const float DA = a_A - c_A;
        const float DB = a_B - c_B;
        const float VAr = shfl_dn1(VA), VAl = shfl_up1(VA);
        const float VBr = shfl_dn1(VB), VBl = shfl_up1(VB);
        const float DAr = shfl_dn1(DA), DAl = shfl_up1(DA);
        const float DBr = shfl_dn1(DB), DBl = shfl_up1(DB);
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
          collide_f(D, bh, b_drho, b_jx, b_jy, ux, uy, Fx, Fy, b_irho, fnew);
        }
      }
    }
    // Isothermal: f alone is stored here.  Every step iteration issues the
    // same nine stores (offset kDrop when there is nothing to store), so the
    // count of memory operations between a row's loads and their use is the
    // same on every path into the loop and the waits stay partial.
    if (MODE == MODE_STEP && !TH) {
      const int voff = OUT2 && !sb && interior ? ((r - 1) * pitch + x) * E2 : kDrop;
#pragma unroll
      for (int i = 0; i < 9; ++i) BufIO<S>::template st<CP>(rd, voff, sst[i], fnew[i]);
    }

    // ---------------- stage 3: row c = r - 2: source and g collision
    if (MODE == MODE_STEP && TH && !ST3) {
#pragma unroll
      for (int i = 0; i < 9; ++i) PairIO<S>::template st<CP>(rd, kDrop, sst[i], 0.f, 0.f);  // same count, see above
    }
    if (MODE == MODE_STEP && TH && ST3) {
      const int cr = r - 2;
      float uxl = shfl_up1(c_uax);
      float uxr = shfl_dn1(c_uax);
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
      const int voff = interior ? (cr * pitch + x) * E2 : kDrop;
#pragma unroll
      for (int i = 0; i < 9; ++i) PairIO<S>::template st<CP>(rd, voff, sst[i], fc[i], ks[i]);
    }

    // ---------------- rotate: d <- c <- b <- a
    d_uay = c_uay;
    sd = sc;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      ck[i] = bk[i];
      bk[i] = ak[i];
      bh[i] = ah[i];
      if (MODE == MODE_STEP && TH) fc[i] = fnew[i];
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

  // K consecutive iterations with stage-2 output, the first on buffer B.
  template <int B, int K>
  __device__ __forceinline__ void trip(int r) {
    if constexpr (K > 0) {
      iter<true, true, MODE == MODE_STEP, true, B % NB>(r);
      trip<B + 1, K - 1>(r + 1);
    }
  }

  // The last rem (< NB) iterations with output from row r, then, when
  // stepping, the final iteration.
  template <int B0, int K>
  __device__ __forceinline__ void tail(int r, int rem) {
    if constexpr (K < NB) {
      if (rem == K) {
        trip<B0, K>(r);
        if (MODE == MODE_STEP) iter<true, false, true, true, (B0 + K) % NB>(r + K);
      } else {
        tail<B0, K + 1>(r, rem);
      }
    }
  }

  // Iterations from row r (buffer B0 holds row r) to r_end, NB per trip.
  // When stepping, the final iteration (r_end = y1 + 1) only finishes stage
  // 3 of row y1 - 1: its stage-2 row y1 belongs to the next tile.
  template <int B0>
  __device__ __forceinline__ void steady(int r) {
    const int r_out = MODE == MODE_STEP ? r_end - 1 : r_end;  // last row-r with stage-2 output
    for (; r + NB - 1 <= r_out; r += NB) trip<B0, NB>(r);
    // rows before r (y1 - 1, the tile's last own row, among them) have their
    // moments: hand the mass to the next launch now, so the atomic's round
    // trip overlaps the remaining iterations
    if (MODE == MODE_STEP) flush_mass();
    tail<B0, 0>(r, r_out - r + 1);
  }

  __device__ __forceinline__ void run() {
    // Rows y0-2 .. r_end are pulled (r_end = y1 + 1 when stepping: stage 3
    // of the last row needs u_act of the row above it).  Stage 2 starts at
    // the third row, its collision output at the fourth, stage 3 at the
    // fifth.
    const int y0 = tl.y0;
    fetch<0>(y0 - 2);
    // Mean density of the previous state: the running mass totals the
    // previous launch added to (one slot per lane) and this tile's reading
    // of them two launches back, combined below once the first rows are in
    // flight.  Issued after the first row's loads, which need the tile
    // record alone, and by every lane (no branch ahead of them).  Plain
    // loads: both were last written in earlier launches, whose writes the
    // kernel boundary makes visible.
    {
      const unsigned long long w = D.macc[phase ^ 1][min(lane, kAccSlots - 1) * kAccStride];
      mtot = lane < kAccSlots ? w : 0ull;
      mprev = D.mhist[phase ^ 1][tl.local];
    }
    if constexpr (NB >= 3) fetch<1>(y0 - 1);
    if constexpr (NB >= 4) fetch<2>(y0);
    iter<false, false, false, true, 0>(y0 - 2);
    iter<false, false, false, true, 1 % NB>(y0 - 1);
    {
      static_assert(kAccSlots == 16, "the slots are summed along one DPP row");
      const unsigned long long tot = row0_sum_u64(mtot);
      if (MODE == MODE_STEP && lane == 0) D.mhist[phase ^ 1][tl.local] = tot;  // read back two launches on
      const double mass = (double)(long long)(tot - mprev) * (1.0 / kMassScale);
      gbar = (float)((double)D.rho_ref - mass / ((double)nx * (double)ny));
    }
    iter<true, false, false, true, 2 % NB>(y0);
    iter<true, true, false, true, 3 % NB>(y0 + 1);
    steady<4 % NB>(y0 + 2);
    // tile partial sums: FP64 in a fixed order (DPP lane tree), the counts as
    // exact 32-bit integers; heater and pressure sums are zero off the edge
    // tiles (fewer cross-lane rounds at the end of every tile)
    double v[kPartials];
    v[P_MASS] = MODE == MODE_STEP ? mass_tile : wave_sum(acc_mass);
    v[P_ENERGY] = wave_sum(acc_energy);
    v[P_VAPOR] = (double)wave_sum_int(acc_vap);
    v[P_CLAMP] = (double)wave_sum_int(acc_clamp);
    v[P_NONFINITE] = (double)wave_sum_int(acc_nf);
    v[P_HEATQ] = EDGE ? wave_sum(acc_q) : 0.0;
    v[P_PIN] = EDGE ? wave_sum(acc_pin) : 0.0;
    v[P_POUT] = EDGE ? wave_sum(acc_pout) : 0.0;
    if (lane == 0) {
      double* out = (MODE == MODE_STEP ? D.partials[phase] : D.readout_partials) + tl.local;
#pragma unroll
      for (int q = 0; q < kPartials; ++q) out[(long long)q * D.pstride] = v[q];
    }
    if (MODE == MODE_STEP && lane == 0 && v[P_NONFINITE] > 0.0) *D.nf_flag = 1;  // sticky, for the server
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

// Row buffers of interior tiles (look-ahead kDepthInterior - 1 rows).  Two,
// as on boundary tiles: deeper look-ahead (3 or 4 buffers) measured slower
// on both the cache-resident and the HBM-resident channel.
constexpr int kDepthInterior = 2;

template <int S, int MODE, bool WT>
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
    // the path comes with the tile record: no descriptor load before the branch
    const int kind = tl.kind;
    const int k = MODE == MODE_STEP ? (kind & 3) : ((kind >> 2) & 3);
    if (kind & kTileIsothermal) {
      if (k == kTileColumnEdge) TileRun<S, MODE, 2, false, 2, WT>(tl, gphase).run();
      else if (k == kTileRowEdge) TileRun<S, MODE, 1, false, 2, WT>(tl, gphase).run();
      else TileRun<S, MODE, 0, false, kDepthInterior, WT>(tl, gphase).run();
    } else {
      if (k == kTileColumnEdge) TileRun<S, MODE, 2, true, 2, WT>(tl, gphase).run();
      else if (k == kTileRowEdge) TileRun<S, MODE, 1, true, 2, WT>(tl, gphase).run();
      else TileRun<S, MODE, 0, true, kDepthInterior, WT>(tl, gphase).run();
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
    const double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                         1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    // plane i holds f_i (isothermal) or the (f_i, g_i) pair of each node;
    // the planes of row y follow each other from element 9 pitch y
    const uint32_t E2 = D.isothermal ? C::E : 2 * C::E;
    for (int i = 0; i < 9; ++i) {
      const uint32_t o = ((uint32_t)(9 * y + i) * (uint32_t)D.pitch + (uint32_t)x) * E2;
      C::st(buf, o, (float)(W[i] * (r - (double)D.rho_ref)));
      if (!D.isothermal) C::st(buf, o + C::E, (float)(W[i] * (t - (double)D.T_ref)));
    }
    if (D.bc_x != LBM_BCX_PERIODIC && x == D.nx - 1) {
      D.fold[b][0 * D.ny + y] = (float)(W[3] * (r - (double)D.rho_ref));
      D.fold[b][1 * D.ny + y] = (float)(W[6] * (r - (double)D.rho_ref));
      D.fold[b][2 * D.ny + y] = (float)(W[7] * (r - (double)D.rho_ref));
    }
  }
}

// Reduction state of a freshly initialised domain (one block): the running
// mass totals give the first state's buoyancy the mean initial density
// (mass0 / nodes; the first launch, parity 0, reads parity 1), every tile's
// last reading is zero, the pending diagnostics sums of the "previous"
// launches hold the initial mass, the step counter and the non-finite flag
// are zero and the per-step records are empty (step -1).
__global__ __launch_bounds__(256) void init_aux_kernel(DevDomain* D, double mass0) {
  const int t = threadIdx.x, nt = blockDim.x;
  const unsigned long long m0 = (unsigned long long)(long long)llrint(mass0 * kMassScale);
  for (int k = t; k < kAccSlots * kAccStride; k += nt) {
    D->macc[0][k] = 0ull;
    D->macc[1][k] = k == 0 ? m0 : 0ull;
  }
  for (int k = t; k < D->pstride; k += nt) {
    D->mhist[0][k] = 0ull;
    D->mhist[1][k] = 0ull;
  }
  for (int k = t; k < kPartials * D->pstride; k += nt) D->partials[1][k] = k == P_MASS * D->pstride ? mass0 : 0.0;
  for (int k = t; k < kFin * kPartials; k += nt) {
    D->l1[0][k] = k == P_MASS ? mass0 : 0.0;
    D->l1[1][k] = k == P_MASS ? mass0 : 0.0;
  }
  for (int k = t; k < kRing; k += nt) {
    D->ring[k].step = -1;
#pragma unroll
    for (int q = 0; q < kPartials; ++q) D->ring[k].v[q] = __builtin_nan("");
  }
  if (t == 0) {
    *D->step_dev = 0;
    *D->nf_flag = 0;
  }
}

// Streaming copy: each block moves one contiguous chunk of chunk 16-byte
// elements, four loads in flight per thread before their stores.  Whole
// chunks per block keep each DRAM page's traffic together, which measured
// faster than a grid-stride loop on arrays larger than the last-level cache.
typedef float vf4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void copy_kernel(vf4* __restrict__ dst, const vf4* __restrict__ src,
                                                   long long n4, long long chunk) {
  const long long b0 = blockIdx.x * chunk;
  const long long b1 = b0 + chunk < n4 ? b0 + chunk : n4;
  for (long long i = b0 + threadIdx.x; i < b1; i += 4 * 256) {
    vf4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long j = i + u * 256;
      v[u] = j < b1 ? src[j] : vf4(0.f);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long j = i + u * 256;
      if (j < b1) dst[j] = v[u];
    }
  }
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
                           int nfin, int grid, int phase, bool write_through, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (grid <= 0 || grid > ntiles) grid = ntiles;
  grid += (nfin + 7) & ~7;
#define L(SS)                                                                                              \
  if (write_through)                                                                                      \
    hipLaunchKernelGGL((step_kernel<SS, MODE_STEP, true>), dim3(grid), dim3(kWave), 0, s, tiles, ntiles, fins, \
                       nfin, phase);                                                                      \
  else                                                                                                    \
    hipLaunchKernelGGL((step_kernel<SS, MODE_STEP, false>), dim3(grid), dim3(kWave), 0, s, tiles, ntiles, fins, \
                       nfin, phase);
  DISPATCH_STORE(storage, L)
#undef L
  return hipGetLastError();
}

hipError_t lbm_launch_readout(int storage, const Tile* tiles, int ntiles, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
#define L(SS) hipLaunchKernelGGL((step_kernel<SS, MODE_READOUT, false>), dim3(ntiles), dim3(kWave), 0, s, tiles, ntiles, (const FinEntry*)nullptr, 0, phase)
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

hipError_t lbm_launch_init_aux(DevDomain* dev, double mass0, hipStream_t s) {
  hipLaunchKernelGGL(init_aux_kernel, dim3(1), dim3(256), 0, s, dev, mass0);
  return hipGetLastError();
}

hipError_t lbm_launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const long long n4 = (long long)(bytes / 16);
  if (n4 <= 0) return hipSuccess;
  // chunks of at least 4096 elements (64 KiB), at most 32768 blocks
  const long long chunk = std::max<long long>(4096, (n4 + 32767) / 32768);
  const int grid = (int)((n4 + chunk - 1) / chunk);
  hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, s, (vf4*)dst, (const vf4*)src, n4, chunk);
  return hipGetLastError();
}
