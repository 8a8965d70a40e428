/*
 * lbmflow.h -- C ABI of the MI355X (gfx950) implementation of one coupled
 * time step of the pseudopotential / thermal D2Q9 lattice-Boltzmann method
 * for flow boiling (Mukherjee, Basu & Mondal, arXiv:2009.05264).
 *
 * The operation behind every entry point is the per-time-step update of
 * Sec. 2 of the paper:
 *   - pull streaming with the boundary rules of Sec. 2C: halfway bounce-back
 *     at no-slip walls, non-equilibrium (Zou-He) bounce-back at the velocity
 *     inlet, anti-bounce-back for temperature, a convective outlet with zero
 *     temperature gradient;
 *   - moments (Eqs. 4, 6, 17), the Peng-Robinson EOS (Eq. 12) and the
 *     pseudopotential (Eq. 11);
 *   - the beta-weighted Shan-Chen force (Eqs. 8-10) over the fluid
 *     neighbours, adhesion -G_wet psi(x) sum_solid w_i psi(rho_w) c_i through
 *     the false wall density (Eq. 15), buoyancy (rho - rho_avg) g_a (Eq. 14)
 *     with rho_avg the mean density of the previous state;
 *   - exact-difference forcing (Eqs. 5, 7) in a multiple-relaxation-time
 *     collision that reduces to the BGK operator of Eq. 2 when all rates are
 *     equal;
 *   - the thermal distribution (Eqs. 16-18) with the phase-change source of
 *     the second form of Eq. 19.
 *
 * Conventions
 *   - Every call returns int: LBM_OK (0) or a negative LBM_E_* code; the
 *     message of the last failure on the calling thread is lbm_last_error().
 *     No call aborts and no C++ exception crosses the ABI.
 *   - Handles are opaque.  One handle is used by one host thread at a time.
 *   - Host arrays are caller-owned, row-major [ny][nx] (x fastest), copied
 *     in or out during the call.
 *   - Device memory is either allocated by the library (dev_mem == NULL at
 *     lbm_create, freed by lbm_destroy) or supplied by the caller (a device
 *     pointer of at least lbm_required_bytes() bytes, 256-byte aligned, owned
 *     and freed by the caller after lbm_destroy).
 *   - Streams are caller-owned hipStream_t passed as void*; NULL selects a
 *     stream created by the library.  lbm_step and lbm_batch_step only
 *     enqueue work; lbm_sync blocks until it is done.  Read calls
 *     synchronise the stream themselves.
 *   - Fields are in lattice units.  Sizes are int32 (nx, ny < 32768).
 */
#ifndef LBMFLOW_H
#define LBMFLOW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_OK = 0,
  LBM_E_INVALID = -1, /* argument outside its documented range           */
  LBM_E_NOMEM = -2,   /* device or host allocation failed                */
  LBM_E_CAP = -3,     /* request exceeds a capacity (server memory cap)  */
  LBM_E_DEVICE = -4,  /* HIP runtime error                               */
  LBM_E_NAN = -5,     /* non-finite values detected in the fields        */
  LBM_E_STATE = -6    /* call out of order (e.g. step before init)       */
};

/* Storage of the distributions in HBM.  Computation is FP32 in all cases.
 * *_DEV stores the deviation f_i - w_i rho_ref (and g_i - w_i T_ref).      */
enum { LBM_STORE_F32 = 0, LBM_STORE_F32_DEV = 1, LBM_STORE_F16_DEV = 2, LBM_STORE_BF16_DEV = 3 };
/* x boundaries: periodic; or a velocity inlet at x = -1 (non-equilibrium
 * bounce-back for f, anti-bounce-back with the inlet state for g, Sec. 2C)
 * with a convective outlet at x = nx (LBM_BCX_CHANNEL) or a constant-pressure
 * outlet (LBM_BCX_CHANNEL_P: non-equilibrium bounce-back fixing the outlet
 * density at rho_out, Sec. 2C); both outlets take zero temperature gradient. */
enum { LBM_BCX_PERIODIC = 0, LBM_BCX_CHANNEL = 1, LBM_BCX_CHANNEL_P = 2 };
/* y boundaries: periodic, or no-slip isothermal walls at y = -1 and y = ny. */
enum { LBM_BCY_PERIODIC = 0, LBM_BCY_WALLS = 1 };
enum { LBM_SIDE_S = 0, LBM_SIDE_N = 1 };

/* Model and domain parameters (lbm_params_default fills the flow-boiling
 * channel).  Rates s_e, s_eps, s_q <= 0 select the defaults s_e = s_eps =
 * 1/tau_f and s_q = 8(2 - s_nu)/(8 - s_nu) (the value that makes the
 * bounce-back wall exactly halfway for Poiseuille flow). */
typedef struct {
  int32_t nx, ny;       /* fluid nodes, >= 3 each                         */
  int32_t storage;      /* LBM_STORE_*                                    */
  int32_t bc_x, bc_y;   /* LBM_BCX_*, LBM_BCY_*                           */
  int32_t isothermal;   /* 1: temperature frozen at T_iso, g not stored   */
  int32_t single_phase; /* 1: Shan-Chen and adhesion forces off           */
  int32_t reserved;
  double a, b, R, omega;         /* Peng-Robinson constants, Eq. 12        */
  double beta, c0, g;            /* Eq. 8 weighting, Eq. 11 c0, sign of G  */
  double tau_f, s_e, s_eps, s_q; /* MRT: s_nu = 1/tau_f (Eq. 2 relation)   */
  double tau_g, c_v;             /* Eq. 16 relaxation time, Eq. 19 c_v     */
  double ga_x, ga_y;             /* buoyancy acceleration g_a, Eq. 14      */
  double fb_x, fb_y;             /* constant body-force density            */
  double u_in, T_in;             /* inlet velocity (|u_in| < 0.1) and temperature */
  double U_out;                  /* convective-outlet speed (< 0: use u_in) */
  double T_iso;                  /* temperature when isothermal            */
  double rho_mid;                /* vapour threshold for diagnostics       */
  double rho_ref, T_ref;         /* reference state of *_DEV storage       */
  double rho_out;                /* outlet density of LBM_BCX_CHANNEL_P (> 0) */
  double G_wet;                  /* adhesion strength of Eq. 15: a solid neighbour  */
                                 /* at c_i adds -G_wet psi(x) w_i psi(rho_w) c_i;   */
                                 /* default lbm_neutral_G_wet (finite)              */
} lbm_params;

typedef struct lbm_domain lbm_domain;
typedef struct lbm_batch lbm_batch;

/* Diagnostics of one state, reduced in FP64 over the fluid nodes. */
typedef struct {
  int64_t step;        /* state index (number of completed steps)          */
  double mass;         /* sum rho                                          */
  double energy;       /* sum T                                            */
  double heater_q;     /* sum over heater cells of 2 (T_wall - T(x, 0)):    */
                       /* the wall heat flux behind the Nusselt number      */
                       /* and delta T* of Sec. 3B                           */
  double vapor_cells;  /* number of nodes with rho < rho_mid               */
  double psi_clamped;  /* nodes where p - rho/3 > 0 made psi imaginary     */
  double nonfinite;    /* nodes with non-finite rho or T                   */
  double p_in, p_out;  /* EOS pressure at (0, ny/2) and (nx-1, ny/2)       */
  double nu_heater;    /* heater Nusselt number, ny / (T_h - T_in) x        */
                       /* heater_q / (heater cells), T_h the mean wall      */
                       /* temperature of the heater cells of the wall map   */
                       /* in force when read; 0 without heater cells        */
  double dp;           /* centreline pressure drop p_in - p_out            */
} lbm_diag;

const char* lbm_last_error(void);

/* Fill p with the defaults (200x50 channel, PR constants of Sec. 2A). */
int lbm_params_default(lbm_params* p);
/* The G_wet of Eq. 15 (not printed in the paper) at which a flat wall whose
 * false density equals the adjacent fluid's exerts no net force on it:
 * 9 g (1 + beta), since Eq. 10 on D2Q9 is G_i = 18 g w_i and Eq. 9 over the
 * fluid neighbours alone lacks (1 + beta)/2 sum_solid G_i psi^2 c_i.
 * Host only; 0 for NULL. */
double lbm_neutral_G_wet(const lbm_params* p);

/* Device bytes a domain with these parameters needs (state buffers, outlet
 * memory, wall maps, reductions and read-out fields). */
int lbm_required_bytes(const lbm_params* p, size_t* bytes);

/* Create a domain on the current HIP device.  Validates p (LBM_E_INVALID):
 * nx, ny >= 3; tau_f, tau_g > 1/2; 0 < s_* < 2; c_v > 0; |u_in| < 0.1;
 * temperatures > 0; the state buffer addressable with 32-bit offsets
 * (11 pitch x (ny + 2) elements under 2 GB, pitch = nx rounded up to 32: the
 * 9 direction planes of every row with a margin; about 24 M nodes with FP32
 * thermal storage, 48 M with FP16/BF16).  dev_mem/dev_bytes: see
 * Conventions. */
int lbm_create(const lbm_params* p, void* hip_stream, void* dev_mem, size_t dev_bytes,
               lbm_domain** out);
/* LBM_E_STATE (nothing freed) while the domain is in a batch. */
int lbm_destroy(lbm_domain* d);

/* Wall maps of one side (LBM_SIDE_S bottom, LBM_SIDE_N top), nx entries:
 * wall temperature (anti-bounce-back value), false wall density rho_w of
 * Eq. 15 (rho_w >= 0), heater flags (bottom side only, may be NULL) that
 * select the cells summed in lbm_diag.heater_q.  Defaults: T_in, rho_w of a
 * neutral wall is not assumed -- set both sides before lbm_init_fields when
 * bc_y == LBM_BCY_WALLS. */
int lbm_set_wall_maps(lbm_domain* d, int side, const double* T_wall, const double* rho_w,
                      const int32_t* heater);

/* Initial state (Sec. 2C starts the channel from saturated liquid at rest):
 * post-collision f = f^eq(rho0, 0), g = w_i T0 at every node,
 * with rho0 = the array, or rho_uniform (1 + noise_rel * xi(x, y)) where xi
 * in [-1, 1) is the SplitMix64 variate of seed ^ (y nx + x); T0 = the array
 * or T_uniform.  Resets the step counter and the lagged mean density.
 * LBM_E_STATE while the domain is in a batch. */
int lbm_init_fields(lbm_domain* d, const double* rho0, const double* T0, double rho_uniform,
                    double T_uniform, double noise_rel, uint64_t seed);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops that re-initialise resident domains,
 * harnesses that forbid hipMalloc): lbm_init_fields with the host arrays
 * staged in a fixed device array of the library instead of hipMalloc'd
 * memory.  Same arguments, same result (bitwise) and same synchronisation as
 * lbm_init_fields; it calls no allocating routine.  With rho0 or T0 given,
 * nx * ny must not exceed LBM_NOALLOC_MAX_NODES (LBM_E_INVALID otherwise;
 * uniform initial states have no limit).  The staging array (16 MiB,
 * 2 x LBM_NOALLOC_MAX_NODES doubles) is held by each GPU the library runs on
 * until the process ends and is shared by every call on that GPU: calls
 * that overlap on one GPU (from several host threads, or on several
 * streams) race for it and must be serialised by the caller. */
#define LBM_NOALLOC_MAX_NODES (1 << 20)
int lbm_init_fields_noalloc(lbm_domain* d, const double* rho0, const double* T0, double rho_uniform,
                            double T_uniform, double noise_rel, uint64_t seed);

/* Enqueue nsteps time steps (the update of Sec. 2 summarised at the top of
 * this file) on the domain's stream (nsteps >= 0): one kernel launch per
 * step.  A call of fewer than 64 steps launches them one by one.  A longer
 * call launches one or two singly (so that an even count remains), then
 * replays captured hipGraphs of 2 to 256 launches, one set per start phase
 * (all captured by the first call of 64 or more steps, before any is
 * launched; dropped when the tiling changes): at most one graph of each
 * shorter length, then repeats of the 256-launch graph.  nsteps == 0
 * enqueues nothing and captures the graphs that are not captured yet (so
 * that a timed call captures nothing).  Results are bitwise the same
 * however nsteps is split. */
int lbm_step(lbm_domain* d, int64_t nsteps);
/* Waits for the domain's stream (and its batch's, while it is in one). */
int lbm_sync(lbm_domain* d);
int64_t lbm_step_count(const lbm_domain* d);

/* Fields of the current state (post-streaming): rho, actual velocity u_act
 * of Eq. 7, T.  Host FP64 arrays [ny][nx]; any pointer may be NULL.  The
 * read-outs, lbm_diag_history and lbm_save of a domain in a batch first
 * wait for the batch's stream. */
int lbm_read_fields(lbm_domain* d, double* rho, double* ux, double* uy, double* T);
/* Same fields into caller device buffers of nx*ny floats (no host copy). */
int lbm_read_fields_device(lbm_domain* d, float* rho, float* ux, float* uy, float* T);

/* Diagnostics of the current state (FP64 sums of the lbm_diag fields; the
 * vapour count uses rho < rho_mid, the phase test of the departure
 * statistics of Sec. 3B). */
int lbm_read_diag(lbm_domain* d, lbm_diag* out);
/* Per-step diagnostics recorded on the device by lbm_step (ring of the last
 * capacity states, oldest first).  *n receives the number written. */
int lbm_diag_history(lbm_domain* d, lbm_diag* out, int max, int* n);

/* Checkpoint: state buffer, outlet memory, the mean density the next step
 * uses, pending diagnostics, step counter.  Independent of the tiling: a
 * checkpoint loads into a domain of the same geometry and storage whatever
 * its tile rows.  The per-step records of lbm_diag_history are not saved:
 * after lbm_load they restart with the states the loaded run produces.
 * lbm_load: LBM_E_STATE while the domain is in a batch. */
int lbm_save(lbm_domain* d, const char* path);
int lbm_load(lbm_domain* d, const char* path);

/* Maxwell equal-area coexistence of the Peng-Robinson EOS of p at T < Tc
 * (the construction of Sec. 2D, Fig. 4b): saturated liquid and vapour
 * densities and the saturation pressure (host FP64; LBM_E_INVALID outside
 * 0 < T < Tc). */
int lbm_maxwell(const lbm_params* p, double T, double* rho_l, double* rho_v, double* p_sat);

/* Rows per tile of the step kernel: 0 selects the automatic choice (the
 * shortest tiles of 4 to 7 rows whose waves all fit on the device's SIMDs at
 * once; otherwise 7 rows with FP32 storage, 8 with FP16/BF16); values below
 * 2 act as 2.  Results do not depend on it (bitwise).  Synchronises the
 * domain's stream (the pending partial sums move to the new tiling) and
 * drops its replay graphs.  LBM_E_STATE while the domain is in a batch. */
int lbm_set_tile_rows(lbm_domain* d, int rows);

/* Host only (no device call): the tiles lbm_create makes for an nx x ny
 * domain with the given storage on a device of `simds` SIMDs (0: 1024, the
 * MI355X count), at `rows` rows per tile (0: the automatic choice).  Tile t
 * covers columns [x0[t], min(x0[t] + 60, nx)) and rows [y0[t], y1[t]), in
 * launch order; the first min(max, count) tiles are written (the arrays may
 * be NULL when max is 0), *n receives the count and *rows_used (may be NULL)
 * the rows per tile.  LBM_E_INVALID for nx or ny below 3 or bad pointers. */
int lbm_tile_plan(int nx, int ny, int storage, int simds, int rows, int* rows_used, int* x0, int* y0,
                  int* y1, int max, int* n);

/* Batched execution: n domains (all created on the same device, stepped
 * together, one launch per step over the concatenated tile table, replayed
 * from captured hipGraphs as in lbm_step).  tune_cache_json: NULL = no autotuning:
 * domains on automatic rows (lbm_set_tile_rows 0) get one tile height chosen
 * for the batch's combined tiles (fewest rounds of waves on the SIMDs times
 * the row steps of a tile); "" = autotune on the batch without a cache file,
 * otherwise a text file the autotuner reads and appends to.  The autotuner
 * times each option by stepping the batch: those are real steps of every
 * domain (22 per option, 15 options: rows 4, 6, 7, 8, 12 x grids of one
 * workgroup per tile, 8 or 16 per compute unit), counted by lbm_step_count.
 * lbm_batch_destroy gives every domain its own rows setting back.  Results
 * do not depend on the tile choice (bitwise). */
int lbm_batch_create(lbm_domain* const* doms, int n, const char* tune_cache_json, lbm_batch** out);
/* As lbm_step, over all domains of the batch (nsteps == 0: capture only). */
int lbm_batch_step(lbm_batch* b, int64_t nsteps);
int lbm_batch_sync(lbm_batch* b);
/* Synchronises the batch's stream and hands its domains back for stepping
 * alone (a domain retiled for the batch gets its own rows back; a device
 * error from that is returned after the batch is freed). */
int lbm_batch_destroy(lbm_batch* b);

/* ---------------------------------------------------------------- serving
 * A server owns a queue of flow-boiling solves.  lbm_server_submit records a
 * request (parameters, wall maps and initial state are copied) with its
 * arrival time.  Each lbm_server_pump call
 *   1. admits queued requests in arrival order while their device footprint
 *      (lbm_required_bytes) fits under the cap next to the resident ones and
 *      a slot is free (a request that does not fit is passed over, not
 *      blocking smaller ones behind it), creating and initialising each
 *      domain on the server's stream;
 *   2. steps every running request together, one launch per step over all
 *      their tiles (lbm_batch_*), for min(quantum, smallest remaining
 *      budget) steps, and waits for them;
 *   3. retires the requests whose budget is reached (time to solution =
 *      completion minus arrival, host steady clock).
 * Results of a finished request stay resident (and count against the cap)
 * until lbm_server_release.  A request's result does not depend on what it
 * was batched with: each domain keeps its own tiles and reductions.
 * The server is used by one host thread at a time.                         */
typedef struct lbm_server lbm_server;

/* Boundary maps and initial state of one request (arrays of nx entries,
 * copied at submit).  Wall maps are required when bc_y == LBM_BCY_WALLS;
 * heater may be NULL. */
typedef struct {
  const double* T_wall_s;
  const double* rho_w_s;
  const int32_t* heater;
  const double* T_wall_n;
  const double* rho_w_n;
  double rho_init, T_init, noise; /* lbm_init_fields(rho_uniform, T_uniform, noise_rel) */
  uint64_t seed;
} lbm_request;

enum { LBM_REQ_QUEUED = 0, LBM_REQ_RUNNING = 1, LBM_REQ_DONE = 2, LBM_REQ_CANCELLED = 3,
       LBM_REQ_FAILED = 4 };

typedef struct {
  int64_t queued, running, done;
  size_t resident_bytes, peak_resident_bytes;
  double lups;          /* lattice updates completed by the server        */
  double busy_seconds;  /* device time of the quanta (events around each) */
  int64_t failed;       /* requests in LBM_REQ_FAILED                     */
} lbm_server_info;

/* hbm_cap_bytes > 0: bound on the summed footprint of resident requests;
 * max_slots > 0: bound on running requests; quantum_steps > 0: steps between
 * admission points.  hip_stream as for lbm_create. */
int lbm_server_create(size_t hbm_cap_bytes, int max_slots, int64_t quantum_steps, void* hip_stream,
                      lbm_server** out);
/* LBM_E_CAP if the request alone exceeds the cap (it is not queued). */
int lbm_server_submit(lbm_server* s, const lbm_params* p, const lbm_request* r, int64_t step_budget,
                      uint64_t* req_id);
/* One admission + quantum + retirement round, waiting for the quantum (a
 * quantum left on the device by lbm_server_pump_async is waited for and
 * retired first); *running (may be NULL) receives the number of requests
 * still running. */
int lbm_server_pump(lbm_server* s, int* running);
/* The same round without waiting: if a quantum is on the device and has not
 * completed (an event recorded after it is queried), returns at once with
 * *in_flight = 1; otherwise retires it (step 3), admits (step 1) and
 * launches the next quantum (step 2) without waiting for it.  Requests
 * submitted while a quantum runs are admitted when it has been retired, so
 * a host loop that calls this between submissions records arrival times as
 * they happen.  Completion times are taken when the retiring call sees the
 * event complete.  *running and *in_flight may be NULL. */
int lbm_server_pump_async(lbm_server* s, int* running, int* in_flight);
/* *state = LBM_REQ_*; *time_to_solution_s (may be NULL) = completion minus
 * arrival in seconds once done, else -1.  LBM_REQ_FAILED: the request could
 * not be started (its lbm_create/lbm_init_fields error), or its density or
 * temperature turned non-finite (LBM_E_NAN; checked on every request at the
 * end of each quantum, the request is retired and its memory freed while
 * the others keep running); lbm_last_error() then names the reason. */
int lbm_server_poll(lbm_server* s, uint64_t req_id, int* state, double* time_to_solution_s);
/* Fields / diagnostics of a finished request (as lbm_read_fields/_diag). */
int lbm_server_read_fields(lbm_server* s, uint64_t req_id, double* rho, double* ux, double* uy,
                           double* T);
int lbm_server_read_diag(lbm_server* s, uint64_t req_id, lbm_diag* out);
/* Free the device state of a finished request. */
int lbm_server_release(lbm_server* s, uint64_t req_id);
/* Drop a queued or running request (its device state is freed). */
int lbm_server_cancel(lbm_server* s, uint64_t req_id);
int lbm_server_stats(lbm_server* s, lbm_server_info* out);
int lbm_server_destroy(lbm_server* s);

/* The server's admission rule on its own (host only): scan footprints[0..n)
 * in order, admitting each that fits in cap - used while free_slots remain;
 * admit[0..*n_admit) receives the admitted indices. */
int lbm_admission_plan(const size_t* footprints, int n, size_t cap, size_t used, int free_slots,
                       int* admit, int* n_admit);

/* Plain device copy of bytes (HBM copy ceiling and counter calibration):
 * dst, src device pointers, 16-byte aligned, bytes a multiple of 16
 * (LBM_E_INVALID otherwise); enqueued on hip_stream. */
int lbm_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* LBMFLOW_H */
