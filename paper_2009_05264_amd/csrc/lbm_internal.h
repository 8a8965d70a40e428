// Internal layout shared by the host runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kStripInterior = 60;  // interior columns per wave (64 - 2 - 2 halo)
constexpr int kPartials = 8;        // doubles per tile partial
constexpr int kRing = 4096;         // per-step diagnostics records kept on device
constexpr int kFin = 16;            // finalizer waves per domain (level-1 slices)
constexpr int kAccSlots = 16;       // fixed-point mass accumulators per domain and parity
constexpr int kAccStride = 16;      // 64-bit words between slots: one 128-byte line each
// fixed-point scale of the mass accumulators: 2^32 units per unit density
constexpr double kMassScale = 4294967296.0;
// Launches whose A/B state (all domains of the launch) is at most this size
// store the new state write-through (agent-scope stores, which the L2 passes
// on at once); larger ones keep the default write-back stores.  An A/B state
// that fits the 256 MB Infinity Cache is re-read from it by the next launch,
// and write-back stores left up to the whole L2 dirty at the end of every
// launch, written back before the next launch started: on MI355X the
// write-through stores measured 4-10 % faster per step from 6 MB to 207 MB
// of state (1600x200 FP32: 13.5 -> 12.2 us), and 3-18 % slower from 302 MB
// up, where the state streams from HBM.
constexpr size_t kWriteThroughMaxBytes = 224ull << 20;

// Elements per row of one direction plane: nx rounded up to 32, plus 32 when
// that is a multiple of 1024.  The nine planes of a row then never sit at
// strides of a multiple of 32 KB (FP32 pairs), which map onto the same
// memory channels: 8192x1024 FP32 263 -> 256 us per step, FP16 145 -> 144
// us; other widths measured unchanged or slower with the extra columns.
inline int lbm_pitch(int nx) {
  const int p = (nx + 31) / 32 * 32;
  return p % 1024 == 0 ? p + 32 : p;
}

// Partial sums of one tile, in this order.
enum { P_MASS = 0, P_ENERGY, P_HEATQ, P_VAPOR, P_CLAMP, P_NONFINITE, P_PIN, P_POUT };

// One diagnostics record (same layout as lbm_diag).
struct DiagRec {
  long long step;
  double v[kPartials];
};

// Device-resident descriptor of one domain.  All physics constants are
// pre-converted to float on the host.
struct DevDomain {
  int nx, ny, pitch, storage;  // pitch: elements per row of one direction plane (lbm_pitch)
  int bc_x, bc_y, isothermal, single_phase;
  int ntiles, pad0;
  // EOS / force constants
  float a, b, R, kappa;
  float kw, Tc, beta, c0g2;       // c0g2 = 2 / (c0 g); kw = G_wet / (18 g): Eq. 15 as G_wet w_i = kw G_i
  float G1, G2, half_1mb, pad1;    // half_1mb = (1 - beta) / 2
  // collision
  float s_e, s_eps, s_q, s_nu;
  float omega_g, inv_cv, pad2, pad3;
  float ga_x, ga_y, fb_x, fb_y;
  float u_in, T_in, U_out, inv_1pU;  // inv_1pU = 1 / (1 + U_out)
  float in_geq;                      // T_in (1 + 3 u_in^2): inlet anti-bounce-back state
  float inv_1mu;                     // 1 / (1 - u_in)
  float rho_ref, T_ref, T_iso, rho_mid;
  float dro;      // rho_ref - rho_out of the constant-pressure outlet
  float pad4;
  // buffers
  void* buf[2];         // state A/B: [ny][9][pitch] (row, direction plane, column) of (f_i, g_i)
                        // pairs (f_i alone when isothermal)
  float* fold[2];       // convective-outlet memory [3][ny] (deviation form), A/B; unused by the
                        // constant-pressure outlet
  const float* psiw[2]; // pseudopotential of the false wall density, S and N, [nx]
  const float* Tw[2];   // wall temperature, S and N, [nx]
  const int* heater;    // bottom heater flags [nx]
  double* partials[2];  // [kPartials][pstride] per launch parity (SoA over tiles)
  double* l1[2];        // [kFin][kPartials] slice sums of the partials, per parity
  // Mean density of the previous state for the buoyancy force (Eq. 14):
  // each launch adds its exact fixed-point mass into macc[parity] (running
  // totals, kAccSlots slots); a tile reads the totals of the other parity
  // and keeps them in mhist[parity][tile], so the difference from its
  // previous reading is the mass of the state one launch back.
  unsigned long long* macc[2];   // [kAccSlots * kAccStride] per parity (slot k at k * kAccStride)
  unsigned long long* mhist[2];  // [pstride] per parity
  int* nf_flag;         // set to 1 by a step that meets a non-finite density or temperature
  double* rbar;         // scratch for read-out reductions
  DiagRec* ring;        // [kRing]
  long long* step_dev;  // device step counter (written only by the first tile)
  double* readout_partials;  // [kPartials][pstride]
  int pstride;          // tile capacity of the partial-sum arrays
  int pad6;
  float* out[4];        // read-out fields rho, ux, uy, T [ny][nx]
  int parity;           // storage buffer parity offset
  int pad5;
};

// One finalizer wave: slice f of domain d's per-tile partial sums.
struct FinEntry {
  DevDomain* d;
  int f, pad;
};

// One tile of the step kernel: a 64-lane strip starting two columns left of
// x0, covering rows [y0, y1).  The record repeats the descriptor fields that
// the first row loads need (state buffers, sizes, strides) and carries the
// table's launch parity, so that a wave issues its first loads
// one memory round trip after it starts (the tile record) instead of two
// (the record, then the descriptor it points to).  One 64-byte line per
// tile.
struct alignas(64) Tile {
  DevDomain* d;
  void* buf[2];  // the descriptor's state buffers A/B
  int x0, y0, y1;
  int local;  // tile index within its domain (partials slot); 0 = first tile
  // code path, chosen on the host so that a wave branches on its tile record
  // alone: bits 0-1 when stepping, bits 2-3 for read-out (kTileInterior,
  // kTileRowEdge, kTileColumnEdge); kTileIsothermal when the domain is
  // isothermal
  int kind;
  // added to the launch phase: 0 in a domain's own table, the domain's
  // descriptor parity in a batch's table (the buffer of the state being read
  // is buf[launch phase ^ parity])
  int parity;
  int nx, ny;   // the descriptor's sizes
  int ystride;  // elements from a row of a direction plane to the next (9 pitch)
  int istride;  // elements from a direction plane to the next within a row (pitch)
};
static_assert(sizeof(Tile) == 64, "one tile record per 64-byte line");

enum TileKind { kTileInterior = 0, kTileRowEdge = 1, kTileColumnEdge = 2, kTileIsothermal = 16 };

enum StepMode { MODE_STEP = 0, MODE_READOUT = 1 };

}  // namespace lbm

// Launch wrappers (lbm_kernels.hip).
// write_through: store the new state with the write-through cache policy
// (see kWriteThroughMaxBytes).
hipError_t lbm_launch_step(int storage, const lbm::Tile* tiles, int ntiles,
                           const lbm::FinEntry* fins, int nfins, int grid, int phase, bool write_through,
                           hipStream_t s);
hipError_t lbm_launch_readout(int storage, const lbm::Tile* tiles, int ntiles, int phase,
                              hipStream_t s);
hipError_t lbm_launch_finalize(const double* partials, int pstride, int ntiles, double* out8,
                               hipStream_t s);
hipError_t lbm_launch_init(int storage, lbm::DevDomain* dhost_copy_dev, const lbm::DevDomain& dh,
                           const double* rho0, const double* T0, double rho_u, double T_u,
                           double noise, unsigned long long seed, int buf_index, hipStream_t s);
hipError_t lbm_launch_init_aux(lbm::DevDomain* dev, double mass0, hipStream_t s);
hipError_t lbm_launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
