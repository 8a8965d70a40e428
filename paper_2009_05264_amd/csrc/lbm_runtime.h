// Host-side objects behind the opaque handles of include/lbmflow.h.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/lbmflow.h"
#include "lbm_internal.h"

constexpr int kMinTileRows = 2;
constexpr int kDefaultTileRows = 8;

struct GraphEntry {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct lbm_domain {
  lbm_params P{};
  lbm::DevDomain host{};          // host copy of the device descriptor
  lbm::DevDomain* dev = nullptr;  // device descriptor
  lbm::FinEntry* fins_d = nullptr;  // this domain's finalizer waves (kFin entries)
  hipStream_t stream = nullptr;
  bool own_stream = false;
  char* mem = nullptr;
  bool own_mem = false;
  size_t bytes = 0;
  std::vector<lbm::Tile> tiles_h;
  lbm::Tile* tiles_d = nullptr;
  int ntiles = 0;
  int rows = kDefaultTileRows;
  int grid = 0;  // 0: one workgroup per tile
  int simds = 1024;  // SIMDs of the device (automatic tile rows)
  int device = 0;    // HIP device the domain was created on
  int batch_rows = 0;  // automatic rows chosen for the batch the domain is in (0: its own choice)
  size_t state_ab = 0;  // bytes of the A/B state
  bool write_through = false;  // state_ab <= kWriteThroughMaxBytes
  float* psiw_d[2] = {nullptr, nullptr};
  float* Tw_d[2] = {nullptr, nullptr};
  int* heater_d = nullptr;
  std::vector<int> heater_h;
  std::vector<double> Tw_h[2];
  int64_t step = 0;
  bool inited = false;
  bool in_batch = false;
  hipStream_t batch_stream = nullptr;  // stream the domain's batch runs on (while in one)
  std::vector<GraphEntry> graphs;  // replay graphs of this domain, by start phase and length (lbm_batch.cpp)
};

int lbm_fail(int code, const char* fmt, ...);
int lbm_build_tiles(lbm_domain* d);
long long lbm_tile_count(int nx, int ny, int rows);  // tiles lbm_build_tiles makes at that height
int lbm_enqueue_steps(lbm_domain* d, int64_t n);
int lbm_run_steps(lbm_domain* d, int64_t n);
void lbm_drop_graphs(lbm_domain* d);
int lbm_nonfinite_seen(lbm_domain* d, int* seen);
// Every step of the batch a single launch, with no replay graphs to capture
// (the serving loop rebuilds its batch whenever the running set changes).
void lbm_batch_plain_launches(lbm_batch* b);
// lbm_batch_destroy, optionally leaving the domains at the batch's tile
// heights (lbm_batch.cpp).
int lbm_batch_release(lbm_batch* b, bool keep_tiles);
