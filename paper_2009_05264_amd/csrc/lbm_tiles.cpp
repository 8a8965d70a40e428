// Tile shapes of a domain: the row segments of each 64-lane strip, the code
// path of each tile and the automatic rows per tile.  Kept apart from the
// rest of the runtime because the step kernel's measured traffic and
// duration depend on this code and on the kernel source alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
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

// Row segments [y0, y1) of one strip.  Tiles that run the boundary path do
// more work per row, so they get fewer rows: strips that reach column 0 or
// nx - 1 are cut in chunks of (rows + 1) / 4 rows (at least one); the other
// strips get a 3-row head and tail (the rows within two of a wall or of the
// periodic seam) and near-equal chunks of about `rows` in between.
static void strip_segments(int ny, int rows, bool column_edge, std::vector<std::pair<int, int>>& seg) {
  seg.clear();
  if (column_edge) {
    const int re = std::max(1, (rows + 1) / 4);
    for (int y = 0; y < ny; y += re) seg.push_back({y, std::min(ny, y + re)});
    return;
  }
  const int h = std::min(3, ny), t = std::min(3, ny - h);
  seg.push_back({0, h});
  const int len = ny - h - t;
  if (len > 0) {
    const int nb = (len + rows - 1) / rows;
    int y = h;
    for (int k = 0; k < nb; ++k) {
      const int n = len / nb + (k < len % nb ? 1 : 0);
      seg.push_back({y, y + n});
      y += n;
    }
  }
  if (t > 0) seg.push_back({ny - t, ny});
}

// A strip whose 64 lanes reach column 0, 1 or 2, or column nx-1 or beyond,
// takes the column-edge path (inlet, outlet or periodic seam).
static bool strip_is_column_edge(int x0, int nx) { return !(x0 >= 3 && x0 + kWave - 2 < nx); }

static bool half_storage(int storage) {
  return storage == LBM_STORE_F16_DEV || storage == LBM_STORE_BF16_DEV;
}

long long lbm_tile_count(int nx, int ny, int rows) {
  const int strips = (nx + kStripInterior - 1) / kStripInterior;
  std::vector<std::pair<int, int>> seg;
  long long n = 0;
  for (int t = 0; t < strips; ++t) {
    strip_segments(ny, rows, strip_is_column_edge(t * kStripInterior, nx), seg);
    n += (long long)seg.size();
  }
  return n;
}

// Rows per tile (automatic).  A tile's march spends four extra row steps
// filling its pipeline, and one wave runs it from start to end, so a step
// of a domain whose tiles all run at once lasts about one tile chain: take
// the shortest tiles (4 to 7 rows) whose waves, with the finalizer waves,
// fit on the SIMDs at once.  Larger domains run in several rounds, bound by
// memory traffic, where 7 rows measured best with FP32 storage (1-4 % ahead
// of 8 from 1600x400 to 8192x2048); with 16-bit storage 8 rows while the
// state fits the Infinity Cache (12 rows 10-27 % slower from 1600x400 to
// 3200x800) and 12 rows once it streams from HBM (8192x2048 304.5 -> 288.2
// us per step, 8192x1024 151.5 -> 149.4 us).
static int lbm_auto_rows(int nx, int ny, int simds, bool half, bool streaming) {
  for (int r = 4; r < 8; ++r)
    if (lbm_tile_count(nx, ny, r) + kFin <= simds) return r;
  return half ? (streaming ? 12 : 8) : 7;
}

// Whether a thermal domain's A/B state streams from HBM (the write-back
// store policy of the runtime, kWriteThroughMaxBytes).
static bool streams_from_hbm(int nx, int ny, int storage) {
  const size_t elem = half_storage(storage) ? 2 : 4;
  const size_t nodes = (size_t)lbm_pitch(nx) * (size_t)ny;
  const size_t state = (18 * nodes * elem + 255) / 256 * 256;
  return 2 * state > kWriteThroughMaxBytes;
}

// The tile list of an nx x ny domain at `rows` rows per tile, in launch
// order (local indices and the descriptor pointer left to the caller).
static void plan_tiles(int nx, int ny, int rows, bool isothermal, std::vector<Tile>& out) {
  const int strips = (nx + kStripInterior - 1) / kStripInterior;
  out.clear();
  std::vector<std::pair<int, int>> seg;
  for (int t = 0; t < strips; ++t) {
    const int x0 = t * kStripInterior;
    const bool column_edge = strip_is_column_edge(x0, nx);
    strip_segments(ny, rows, column_edge, seg);
    for (const auto& sg : seg) {
      Tile tl{};
      tl.x0 = x0;
      tl.y0 = sg.first;
      tl.y1 = sg.second;
      // Otherwise a tile whose pulled rows (y0-2 .. r_end, r_end = y1+1 when
      // stepping, y1 for read-out) reach row 0 or ny-1 takes the row-edge path.
      auto kind = [&](int r_end) {
        return column_edge ? kTileColumnEdge
               : (tl.y0 - 2 >= 1 && r_end <= ny - 2) ? kTileInterior
                                                      : kTileRowEdge;
      };
      tl.kind = kind(tl.y1 + 1) | kind(tl.y1) << 2 | (isothermal ? kTileIsothermal : 0);
      out.push_back(tl);
    }
  }
  // Row-major launch order: the tiles in flight at any time cover a few
  // full-width row bands, so every plane is streamed in long contiguous
  // runs (DRAM pages, TLB reach) rather than in narrow vertical bands.
  std::stable_sort(out.begin(), out.end(), [](const Tile& a, const Tile& b) {
    return a.y0 != b.y0 ? a.y0 < b.y0 : a.x0 < b.x0;
  });
}

extern "C" int lbm_tile_plan(int nx, int ny, int storage, int simds, int rows, int* rows_used, int* x0,
                             int* y0, int* y1, int max, int* n) {
  if (nx < 3 || ny < 3 || rows < 0 || max < 0 || !n || (max > 0 && (!x0 || !y0 || !y1)))
    return lbm_fail(LBM_E_INVALID, "bad tile-plan arguments");
  if (storage < LBM_STORE_F32 || storage > LBM_STORE_BF16_DEV)
    return lbm_fail(LBM_E_INVALID, "unknown storage %d", storage);
  const int r = rows > 0 ? std::max(kMinTileRows, rows)
                         : lbm_auto_rows(nx, ny, simds > 0 ? simds : 1024, half_storage(storage),
                                         streams_from_hbm(nx, ny, storage));
  std::vector<Tile> tiles;
  plan_tiles(nx, ny, r, false, tiles);
  for (int i = 0; i < max && i < (int)tiles.size(); ++i) {
    x0[i] = tiles[i].x0;
    y0[i] = tiles[i].y0;
    y1[i] = tiles[i].y1;
  }
  if (rows_used) *rows_used = r;
  *n = (int)tiles.size();
  return LBM_OK;
}

int lbm_build_tiles(lbm_domain* d) {
  lbm_drop_graphs(d);
  const int nx = d->P.nx, ny = d->P.ny;
  const int rows = d->rows > 0         ? std::max(kMinTileRows, d->rows)
                   : d->batch_rows > 0 ? d->batch_rows
                                       : lbm_auto_rows(nx, ny, d->simds, half_storage(d->P.storage),
                                                       !d->write_through);
  plan_tiles(nx, ny, rows, d->P.isothermal != 0, d->tiles_h);
  for (size_t i = 0; i < d->tiles_h.size(); ++i) {
    Tile& tl = d->tiles_h[i];
    tl.d = d->dev;
    tl.local = (int)i;
    tl.buf[0] = d->host.buf[0];
    tl.buf[1] = d->host.buf[1];
    tl.nx = d->host.nx;
    tl.ny = d->host.ny;
    tl.ystride = 9 * d->host.pitch;  // a row holds its 9 direction planes
    tl.istride = d->host.pitch;
    tl.parity = 0;  // the domain's own table: launched with the step's own phase
  }
  if ((int)d->tiles_h.size() > d->host.pstride)
    return lbm_fail(LBM_E_CAP, "tile table of %zu tiles exceeds its capacity %d", d->tiles_h.size(),
                    d->host.pstride);
  d->ntiles = (int)d->tiles_h.size();
  d->host.ntiles = d->ntiles;
  HIPCHECK(hipMemcpyAsync(d->tiles_d, d->tiles_h.data(), d->ntiles * sizeof(Tile),
                          hipMemcpyHostToDevice, d->stream));
  HIPCHECK(hipMemcpyAsync(d->dev, &d->host, sizeof(DevDomain), hipMemcpyHostToDevice, d->stream));
  HIPCHECK(hipStreamSynchronize(d->stream));
  return LBM_OK;
}
