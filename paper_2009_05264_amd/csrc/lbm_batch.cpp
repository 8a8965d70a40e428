// Graph replay of single-domain stepping, batched execution of many domains
// in one launch per step, and the tile autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/lbmflow.h"
#include "lbm_internal.h"
#include "lbm_runtime.h"

using namespace lbm;

#define HIPCHECK(expr)                                                                     \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return lbm_fail(LBM_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

void lbm_drop_graphs(lbm_domain* d) {
  for (auto& g : d->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  d->graphs.clear();
}

// Launch pairs (phase p then phase p ^ 1) captured once and replayed: the
// kernels take everything that changes from step to step from device memory.
static int capture_pairs(hipStream_t s, GraphEntry* g, int pairs, int p, int (*enqueue)(void*, int),
                         void* ctx) {
  HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int rc = 0;
  for (int q = 0; q < pairs && !rc; ++q) {
    rc = enqueue(ctx, p);
    if (!rc) rc = enqueue(ctx, p ^ 1);
  }
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(s, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return lbm_fail(LBM_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return lbm_fail(LBM_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  g->graph = graph;
  g->exec = exec;
  return LBM_OK;
}

static int capture_pair(hipStream_t s, GraphEntry* g, int (*enqueue)(void*, int), void* ctx) {
  return capture_pairs(s, g, 1, 0, enqueue, ctx);
}

// Replay graphs of 2^k launch pairs, k < kGraphLevels, one set per start
// phase (entry p * kGraphLevels + k).  Whatever is queued behind a graph
// starts ~8 us after the graph's last kernel ends (kernel traces of the
// 1600x200 channel; consecutive launches inside a graph, or plain launches,
// start without a gap), so graphs are long: up to 256 launches, that start
// paid once per 256 steps.  Any even step count is replayed as at most one
// graph of each shorter length (the binary digits of its pairs) plus repeats
// of the longest graph, so a call of n steps launches at most n / 256 + 7
// graphs.
constexpr int kGraphLevels = 8;

// Calls shorter than this are launched one kernel at a time: the host
// submits a launch faster than a step runs (measured with steps down to 7.6
// us, a 200x50 channel), so plain launches leave no gaps, and a short call
// would pay the start behind each of its graphs (20 steps of the 1600x200
// channel from an idle device: 11.68 us per step with graphs, 11.13 with
// plain launches).  Longer calls replay graphs, which keep the device fed
// whatever the host does meanwhile.
constexpr int64_t kGraphMinSteps = 64;

// Captures every replay graph not captured yet, before any of them is
// launched: a capture never lands between launches of a call.
static int ensure_graphs(hipStream_t s, std::vector<GraphEntry>& g, int (*enqueue)(void*, int), void* ctx) {
  if ((int)g.size() < 2 * kGraphLevels) g.resize(2 * kGraphLevels);
  for (int q = 0; q < 2; ++q)
    for (int k = 0; k < kGraphLevels; ++k) {
      GraphEntry& e = g[q * kGraphLevels + k];
      if (e.exec) continue;
      int rc = capture_pairs(s, &e, 1 << k, q, enqueue, ctx);
      if (rc) return rc;
    }
  return LBM_OK;
}

// Replays the even part of n steps, the first of launch phase p; *done
// counts the steps enqueued (the at most one step left over is the
// caller's).
static int replay_steps(hipStream_t s, std::vector<GraphEntry>& g, int64_t n, int p,
                        int (*enqueue)(void*, int), void* ctx, int64_t* done) {
  *done = 0;
  const int64_t pairs = n / 2;
  if (pairs == 0) return LBM_OK;
  int rc = ensure_graphs(s, g, enqueue, ctx);
  if (rc) return rc;
  const int top = kGraphLevels - 1;
  GraphEntry* set = &g[p * kGraphLevels];
  // shorter graphs first: the device starts on them while the host still
  // submits the longer ones
  for (int k = 0; k < top; ++k)
    if ((pairs >> k) & 1) HIPCHECK(hipGraphLaunch(set[k].exec, s));
  for (int64_t k = 0; k < (pairs >> top); ++k) HIPCHECK(hipGraphLaunch(set[top].exec, s));
  *done = 2 * pairs;
  return LBM_OK;
}

// Single launches that open a call of n >= kGraphMinSteps steps: one when n
// is odd, so that the replay graphs cover an even number of steps and end
// the call (nothing of the call waits behind a graph), and a first pair, so
// that the device starts on it before the first graph is submitted.
static int64_t head_launches(int64_t n) { return 2 + (n & 1); }

static int enqueue_domain_phase(void* ctx, int phase) {
  lbm_domain* d = (lbm_domain*)ctx;
  HIPCHECK(lbm_launch_step(d->P.storage, d->tiles_d, d->ntiles, d->fins_d, kFin, d->grid, phase,
                           d->write_through, d->stream));
  return LBM_OK;
}

int lbm_run_steps(lbm_domain* d, int64_t n) {
  if (d->in_batch) return lbm_fail(LBM_E_STATE, "domain is part of a batch; step the batch");
  if (n == 0) return ensure_graphs(d->stream, d->graphs, enqueue_domain_phase, d);
  if (n < kGraphMinSteps) return lbm_enqueue_steps(d, n);
  const int64_t head = head_launches(n);
  int rc = lbm_enqueue_steps(d, head);
  if (rc) return rc;
  n -= head;
  int64_t done = 0;
  rc = replay_steps(d->stream, d->graphs, n, (int)(d->step & 1), enqueue_domain_phase, d, &done);
  d->step += done;
  return rc;
}

// ------------------------------------------------------------------ batches
struct lbm_batch {
  std::vector<lbm_domain*> doms;
  hipStream_t stream = nullptr;
  // one tile table per storage kind present in the batch
  struct Group {
    int storage;
    Tile* tiles_d = nullptr;
    int ntiles = 0;
    int grid = 0;
    FinEntry* fins_d = nullptr;  // finalizer waves of the group's domains
    int nfins = 0;
    bool write_through = false;  // the group's A/B state is at most kWriteThroughMaxBytes
  };
  std::vector<Group> groups;
  std::vector<GraphEntry> graphs;  // [p * kGraphLevels + k]: 2^k launch pairs from phase p
  GraphEntry probe;                // the autotuner's timing graph (one launch pair)
  bool plain = false;              // every step a single launch (lbm_batch_plain_launches)
  int64_t k = 0;  // steps done by the batch
  int rows = kDefaultTileRows;
  std::vector<int> saved_rows;  // each domain's own rows setting, restored by lbm_batch_destroy
};

// Tiles of each domain in its own layout, concatenated in the order of the
// domains, grouped by storage kind.
static int build_groups(lbm_batch* b) {
  for (auto& g : b->groups) {
    if (g.tiles_d) (void)hipFree(g.tiles_d);
    if (g.fins_d) (void)hipFree(g.fins_d);
  }
  b->groups.clear();
  std::map<int, std::vector<Tile>> by;
  std::map<int, std::vector<FinEntry>> fby;
  std::map<int, size_t> state_by;
  for (lbm_domain* d : b->doms) {
    state_by[d->P.storage] += d->state_ab;
    auto& v = by[d->P.storage];
    const size_t at = v.size();
    v.insert(v.end(), d->tiles_h.begin(), d->tiles_h.end());
    // the batch's launch phase is offset by the domain's parity
    for (size_t i = at; i < v.size(); ++i) v[i].parity = d->host.parity;
    for (int f = 0; f < kFin; ++f) fby[d->P.storage].push_back(FinEntry{d->dev, f, 0});
  }
  for (auto& kv : by) {
    lbm_batch::Group g;
    g.storage = kv.first;
    g.ntiles = (int)kv.second.size();
    const auto& fl = fby[kv.first];
    g.nfins = (int)fl.size();
    g.write_through = state_by[kv.first] <= kWriteThroughMaxBytes;
    HIPCHECK(hipMalloc(&g.tiles_d, g.ntiles * sizeof(Tile)));
    HIPCHECK(hipMemcpy(g.tiles_d, kv.second.data(), g.ntiles * sizeof(Tile), hipMemcpyHostToDevice));
    HIPCHECK(hipMalloc(&g.fins_d, g.nfins * sizeof(FinEntry)));
    HIPCHECK(hipMemcpy(g.fins_d, fl.data(), g.nfins * sizeof(FinEntry), hipMemcpyHostToDevice));
    b->groups.push_back(g);
  }
  return LBM_OK;
}

static int enqueue_batch_phase(void* ctx, int phase) {
  lbm_batch* b = (lbm_batch*)ctx;
  for (auto& g : b->groups)
    HIPCHECK(lbm_launch_step(g.storage, g.tiles_d, g.ntiles, g.fins_d, g.nfins, g.grid, phase, g.write_through,
                             b->stream));
  return LBM_OK;
}

static void drop_graph(GraphEntry* g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  *g = GraphEntry{};
}

static void drop_batch_graph(lbm_batch* b) {
  for (auto& g : b->graphs) drop_graph(&g);
  b->graphs.clear();
  drop_graph(&b->probe);
}

// Without the autotuner, the domains on automatic rows get one tile height
// chosen for the batch as a whole.  Each domain alone picks its rows for its
// own tiles only, and the combined launch may then queue several tile
// chains on a SIMD.  A step of a batch that is not bound by memory traffic
// lasts about (rounds of waves on the SIMDs) x (row steps of a chain,
// rows + 4): the height (4 to 8 rows) that minimises this product is taken,
// ties going to the taller tiles (fewer halo rows); a batch of one domain
// leaves it at its own automatic height.  The choice is undone by
// lbm_batch_destroy (lbm_batch_release can keep it for the next batch).
static int batch_auto_rows(lbm_batch* b) {
  bool any = false;
  for (lbm_domain* d : b->doms) any = any || d->rows == 0;
  if (!any) return LBM_OK;
  int pick = 0;  // a lone domain takes its own automatic height
  if (b->doms.size() >= 2) {
    const long long simds = b->doms[0]->simds;
    long long best = -1;
    for (int r = 4; r <= 8; ++r) {
      long long waves = 0;
      for (lbm_domain* d : b->doms)
        waves += (d->rows == 0 ? lbm_tile_count(d->P.nx, d->P.ny, r) : d->ntiles) + kFin;
      const long long cost = (waves + simds - 1) / simds * (r + 4);
      if (best < 0 || cost <= best) {
        best = cost;
        pick = r;
      }
    }
  }
  bool changed = false;
  for (lbm_domain* d : b->doms) {
    // a domain a previous batch left at this height (lbm_batch_release
    // keeping the tiles) keeps its tiles
    if (d->rows != 0 || d->batch_rows == pick) continue;
    d->batch_rows = pick;
    d->in_batch = false;
    int rc = lbm_set_tile_rows(d, 0);
    d->in_batch = true;
    if (rc) return rc;
    d->host.parity = (int)((d->step - b->k) & 1);
    HIPCHECK(hipMemcpy(d->dev, &d->host, sizeof(DevDomain), hipMemcpyHostToDevice));
    changed = true;
  }
  return changed ? build_groups(b) : LBM_OK;
}

// Retile every domain (rows per tile) keeping the pending reductions.
static int retile(lbm_batch* b, int rows) {
  for (lbm_domain* d : b->doms) {
    d->in_batch = false;
    int rc = lbm_set_tile_rows(d, rows);
    d->in_batch = true;
    if (rc) return rc;
    // lbm_set_tile_rows re-uploads the descriptor with parity 0; restore it
    d->host.parity = (int)((d->step - b->k) & 1);
    HIPCHECK(hipMemcpy(d->dev, &d->host, sizeof(DevDomain), hipMemcpyHostToDevice));
  }
  b->rows = rows;
  return build_groups(b);
}

static int batch_steps_plain(lbm_batch* b, int64_t n) {
  for (int64_t i = 0; i < n; ++i) {
    int rc = enqueue_batch_phase(b, (int)((b->k + i) & 1));
    if (rc) return rc;
  }
  b->k += n;
  for (lbm_domain* d : b->doms) d->step += n;
  return LBM_OK;
}

// Mean time of one step of the batch over `reps` graph pairs (steps are real).
static int time_config(lbm_batch* b, int reps, float* ms) {
  drop_batch_graph(b);
  if (b->k & 1) {
    int rc = batch_steps_plain(b, 1);
    if (rc) return rc;
  }
  int rc = capture_pair(b->stream, &b->probe, enqueue_batch_phase, b);
  if (rc) return rc;
  HIPCHECK(hipGraphLaunch(b->probe.exec, b->stream));  // warm-up pair
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  HIPCHECK(hipEventRecord(e0, b->stream));
  for (int r = 0; r < reps; ++r) HIPCHECK(hipGraphLaunch(b->probe.exec, b->stream));
  HIPCHECK(hipEventRecord(e1, b->stream));
  HIPCHECK(hipEventSynchronize(e1));
  float t = 0;
  HIPCHECK(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const int64_t done = 2 * (reps + 1);
  b->k += done;
  for (lbm_domain* d : b->doms) d->step += done;
  *ms = t / (2.0f * reps);
  return LBM_OK;
}

static std::string batch_key(const lbm_batch* b) {
  std::ostringstream os;
  long long nodes = 0;
  for (lbm_domain* d : b->doms) nodes += (long long)d->P.nx * d->P.ny;
  os << "v2_n" << b->doms.size() << "_nodes" << nodes;
  return os.str();
}

// Autotuner: rows per tile x workgroups per launch, measured on the batch
// itself; the winner is cached per batch signature in a small text file.
static int autotune(lbm_batch* b, const char* cache) {
  const std::string key = batch_key(b);
  if (cache) {
    std::ifstream in(cache);
    std::string k;
    int rows, gridmul;
    while (in >> k >> rows >> gridmul) {
      if (k == key) {
        int rc = retile(b, rows);
        if (rc) return rc;
        for (auto& g : b->groups) g.grid = gridmul > 0 ? std::min(g.ntiles, 256 * gridmul) : 0;
        return LBM_OK;
      }
    }
  }
  const int row_opts[] = {4, 6, 7, 8, 12};
  const int grid_opts[] = {0, 8, 16};
  float best = 1e30f;
  int brow = kDefaultTileRows, bgrid = 0;
  for (int rows : row_opts) {
    int rc = retile(b, rows);
    if (rc) return rc;
    for (int gm : grid_opts) {
      for (auto& g : b->groups) g.grid = gm > 0 ? std::min(g.ntiles, 256 * gm) : 0;
      float ms = 0;
      rc = time_config(b, 10, &ms);
      if (rc) return rc;
      if (ms < best) {
        best = ms;
        brow = rows;
        bgrid = gm;
      }
    }
  }
  int rc = retile(b, brow);
  if (rc) return rc;
  for (auto& g : b->groups) g.grid = bgrid > 0 ? std::min(g.ntiles, 256 * bgrid) : 0;
  drop_batch_graph(b);
  if (cache) {
    std::ofstream out(cache, std::ios::app);
    out << key << " " << brow << " " << bgrid << "\n";
  }
  return LBM_OK;
}

extern "C" int lbm_batch_create(lbm_domain* const* doms, int n, const char* tune_cache_json,
                                lbm_batch** out) {
  if (!doms || n <= 0 || !out) return lbm_fail(LBM_E_INVALID, "bad batch arguments");
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    if (!doms[i]) return lbm_fail(LBM_E_INVALID, "domain %d is NULL", i);
    if (!doms[i]->inited) return lbm_fail(LBM_E_STATE, "domain %d is not initialised", i);
    if (doms[i]->in_batch) return lbm_fail(LBM_E_STATE, "domain %d already belongs to a batch", i);
    for (int j = 0; j < i; ++j)
      if (doms[j] == doms[i]) return lbm_fail(LBM_E_INVALID, "domain %d appears twice", i);
  }
  lbm_batch* b = new lbm_batch();
  b->stream = doms[0]->stream;
  for (int i = 0; i < n; ++i) {
    hipError_t e = hipStreamSynchronize(doms[i]->stream);
    if (e != hipSuccess) {
      delete b;
      return lbm_fail(LBM_E_DEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
    }
    b->doms.push_back(doms[i]);
    b->saved_rows.push_back(doms[i]->rows);
  }
  int rc = LBM_OK;
  for (lbm_domain* d : b->doms) {
    d->in_batch = true;
    d->batch_stream = b->stream;
    d->host.parity = (int)(d->step & 1);
    hipError_t e = hipMemcpy(d->dev, &d->host, sizeof(DevDomain), hipMemcpyHostToDevice);
    if (e != hipSuccess && !rc) rc = lbm_fail(LBM_E_DEVICE, "descriptor upload: %s", hipGetErrorString(e));
  }
  if (!rc) rc = build_groups(b);
  if (!rc && tune_cache_json) rc = autotune(b, tune_cache_json[0] ? tune_cache_json : nullptr);
  else if (!rc) rc = batch_auto_rows(b);
  if (rc) {
    const std::string msg = lbm_last_error();
    lbm_batch_destroy(b);
    return lbm_fail(rc, "%s", msg.c_str());
  }
  *out = b;
  return LBM_OK;
}

void lbm_batch_plain_launches(lbm_batch* b) {
  if (b) b->plain = true;
}

extern "C" int lbm_batch_step(lbm_batch* b, int64_t n) {
  if (!b) return lbm_fail(LBM_E_INVALID, "batch is NULL");
  if (n < 0) return lbm_fail(LBM_E_INVALID, "nsteps must be >= 0");
  if (n == 0) return b->plain ? LBM_OK : ensure_graphs(b->stream, b->graphs, enqueue_batch_phase, b);
  if (n < kGraphMinSteps || b->plain) return batch_steps_plain(b, n);
  const int64_t head = head_launches(n);
  int rc = batch_steps_plain(b, head);
  if (rc) return rc;
  n -= head;
  int64_t done = 0;
  rc = replay_steps(b->stream, b->graphs, n, (int)(b->k & 1), enqueue_batch_phase, b, &done);
  b->k += done;
  for (lbm_domain* d : b->doms) d->step += done;
  return rc;
}

extern "C" int lbm_batch_sync(lbm_batch* b) {
  if (!b) return lbm_fail(LBM_E_INVALID, "batch is NULL");
  HIPCHECK(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

// The domains leave the batch, which is freed.  Unless keep_tiles, each
// domain gets its own rows setting back (lbm_batch_destroy); with
// keep_tiles the domains stay tiled at the batch's heights, so that the next
// batch built from them at the same height retiles none of them (the
// serving loop rebuilds its batch whenever the running set changes; every
// retile waits for a few small copies per domain).
int lbm_batch_release(lbm_batch* b, bool keep_tiles) {
  if (!b) return LBM_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_batch_graph(b);
  for (auto& g : b->groups) {
    if (g.tiles_d) (void)hipFree(g.tiles_d);
    if (g.fins_d) (void)hipFree(g.fins_d);
  }
  int rc = LBM_OK;
  for (size_t i = 0; i < b->doms.size(); ++i) {
    lbm_domain* d = b->doms[i];
    d->in_batch = false;
    d->batch_stream = nullptr;
    d->host.parity = 0;
    (void)hipMemcpy(d->dev, &d->host, sizeof(DevDomain), hipMemcpyHostToDevice);
    const int own = i < b->saved_rows.size() ? b->saved_rows[i] : d->rows;
    if (!keep_tiles && (d->batch_rows || d->rows != own)) {
      // back to the domain's own rows (the batch height or the autotuner's
      // choice undone; pending sums carried over)
      d->batch_rows = 0;
      const int r = lbm_set_tile_rows(d, own);
      if (r && rc == LBM_OK) rc = r;
    }
  }
  delete b;
  return rc;
}

extern "C" int lbm_batch_destroy(lbm_batch* b) { return lbm_batch_release(b, false); }
