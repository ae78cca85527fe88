// Many uneven scenes in one launch sequence: walks, FP64 boundary data,
// cache means and the gather of every scene run as five kernels over the
// concatenated work of all scenes (walk ids, cache points, gather tiles).
// bvc_batch_plan uploads the scene table once; bvc_batch_launch only
// enqueues kernels (the counters are cleared by a kernel, not a memset), so a
// caller can capture it in a HIP graph and replay it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "bvc_internal.hpp"

struct bvc_batch_s {
  bvc::BatchDev dev;
  int max_depth = 0;
};

namespace bvc {
namespace {

constexpr int kGatherTilePoints = 512;  // evaluation points per gather block

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t table, counters, U, D, w1, exit, a, b, total;
};

int plan_sizes(const bvc_batch_item* items, int n, int& dim, uint64_t& walks, int64_t& cache, int64_t& tiles) {
  if (!items || n < 1) return fail(BVC_EINVAL, "batch needs at least one item");
  walks = 0;
  cache = 0;
  tiles = 0;
  dim = 0;
  int has_src = -1;
  for (int s = 0; s < n; ++s) {
    const bvc_batch_item& it = items[s];
    int rc = check_scene(it.scene);
    if (rc) return rc;
    const int d = it.scene->h.dim;
    if (dim == 0) dim = d;
    if (d != dim) return fail(BVC_EINVAL, "all scenes of a batch must have the same dimension");
    const bvc_walk_params& p = it.walk;
    if (p.dtype != BVC_F32) return fail(BVC_EUNSUPPORTED, "batched walks run in FP32");
    if (p.n_dev) return fail(BVC_EUNSUPPORTED, "batched walks take host counts");
    if (p.order) return fail(BVC_EUNSUPPORTED, "batched walks take no launch order");
    if (!(p.eps > 0) || p.max_steps < 1 || p.n_walks < 1) return fail(BVC_EINVAL, "bad walk parameters");
    rc = check_field(p.g, d, "g");
    if (rc) return rc;
    rc = check_field(p.f, d, "f");
    if (rc) return rc;
    if (p.f.kind != 0 && p.f.kind != 1 && p.f.kind != 3 && p.f.kind != 8)
      return fail(BVC_EUNSUPPORTED, "walk source terms are constants, Gaussian sums or exponential planes");
    if (p.sigma != 0.0) return fail(BVC_EUNSUPPORTED, "batched walks are built for sigma = 0");
    if (p.open_radius != 0.0) return fail(BVC_EUNSUPPORTED, "batched walks are built for bounded domains");
    if (p.side_read != 0) return fail(BVC_EUNSUPPORTED, "batched walks read g at the closest point (no side rule)");
    const int src = p.f.kind != 0;
    if (has_src < 0) has_src = src;
    if (src != has_src) return fail(BVC_EUNSUPPORTED, "mixing scenes with and without sources in one batch");
    if (it.n_cache < 0 || it.n_eval < 0) return fail(BVC_EINVAL, "negative size");
    if ((uint64_t)it.n_cache * (uint64_t)p.n_walks >= (1ull << 32)) return fail(BVC_EINVAL, "n_cache * W >= 2^32");
    if (it.n_cache > 0 && (!it.x || !it.nrm || !it.R0 || !it.xbar || !it.w || !it.cx || !it.cn))
      return fail(BVC_EINVAL, "null cache array");
    if (it.n_eval > 0 && (!it.eval_x || !it.u)) return fail(BVC_EINVAL, "null evaluation array");
    walks += (uint64_t)it.n_cache * (uint64_t)p.n_walks;
    cache += it.n_cache;
    tiles += (it.n_eval + kGatherTilePoints - 1) / kGatherTilePoints;
  }
  if (tiles >= (1ll << 31)) return fail(BVC_EINVAL, "too many gather tiles");
  return BVC_OK;
}

Layout layout(int n, int dim, uint64_t walks, int64_t cache) {
  Layout L;
  size_t off = 0;
  auto put = [&](size_t& o, size_t bytes) {
    o = off;
    off = al(off + std::max<size_t>(bytes, 1));
  };
  put(L.table, (size_t)n * sizeof(BatchSceneDev));
  put(L.counters, 4 * sizeof(unsigned long long));
  put(L.U, walks * 4);
  put(L.D, walks * 4);
  put(L.w1, walks * 4);
  put(L.exit, (size_t)dim * walks * 4);
  put(L.a, (size_t)cache * 4);
  put(L.b, (size_t)cache * 4);
  L.total = off;
  return L;
}

}  // namespace
}  // namespace bvc

using namespace bvc;

extern "C" {

size_t bvc_batch_workspace_bytes(const bvc_batch_item* items, int32_t n_items) {
  int dim;
  uint64_t walks;
  int64_t cache, tiles;
  if (plan_sizes(items, n_items, dim, walks, cache, tiles)) return 0;
  return layout(n_items, dim, walks, cache).total;
}

int bvc_batch_plan(const bvc_batch_item* items, int32_t n_items, void* workspace, size_t ws_bytes, void* stream,
                   bvc_batch* out) {
  if (!out) return fail(BVC_EINVAL, "out is null");
  *out = nullptr;
  int dim;
  uint64_t walks;
  int64_t cache, tiles;
  int rc = plan_sizes(items, n_items, dim, walks, cache, tiles);
  if (rc) return rc;
  const Layout L = layout(n_items, dim, walks, cache);
  if (!workspace || ws_bytes < L.total) return fail(BVC_EINVAL, "batch workspace too small");
  if (((uintptr_t)workspace & 255) != 0) return fail(BVC_EINVAL, "workspace must be 256-byte aligned");
  char* ws = (char*)workspace;
  std::vector<BatchSceneDev> table(n_items);
  uint64_t woff = 0;
  int64_t coff = 0, toff = 0;
  int max_depth = 0, has_src = 0;
  for (int s = 0; s < n_items; ++s) {
    const bvc_batch_item& it = items[s];
    BatchSceneDev& t = table[s];
    std::memset(&t, 0, sizeof(t));
    t.S = it.scene->h.view();
    t.g = to_dev(it.walk.g);
    t.f = to_dev(it.walk.f);
    t.eps = it.walk.eps;
    t.max_steps = it.walk.max_steps;
    t.W = it.walk.n_walks;
    t.seed = it.walk.seed;
    t.batch = it.walk.batch;
    t.cv = it.walk.control_variate;
    t.n_cache = it.n_cache;
    t.n_eval = it.n_eval;
    t.x = it.x;
    t.nrm = it.nrm;
    t.R0 = it.R0;
    t.xbar = it.xbar;
    t.w = it.w;
    t.cx = it.cx;
    t.cn = it.cn;
    t.ex = it.eval_x;
    t.u = it.u;
    t.walk_off = woff;
    t.cache_off = coff;
    t.tile_off = toff;
    woff += (uint64_t)it.n_cache * (uint64_t)it.walk.n_walks;
    coff += it.n_cache;
    toff += (it.n_eval + kGatherTilePoints - 1) / kGatherTilePoints;
    max_depth = std::max(max_depth, it.scene->h.depth);
    has_src |= it.walk.f.kind != 0;
  }
  hipStream_t st = (hipStream_t)stream;
  rc = check_hip(hipMemcpyAsync(ws + L.table, table.data(), table.size() * sizeof(BatchSceneDev),
                                hipMemcpyHostToDevice, st),
                 "batch table upload");
  if (rc) return rc;
  rc = check_hip(hipStreamSynchronize(st), "batch table sync");
  if (rc) return rc;
  bvc_batch b = new (std::nothrow) bvc_batch_s;
  if (!b) return fail(BVC_ENOMEM, "host allocation failed");
  BatchDev& d = b->dev;
  d.scenes = (const BatchSceneDev*)(ws + L.table);
  d.n_scenes = n_items;
  d.dim = dim;
  d.has_src = has_src;
  d.total_walks = walks;
  d.total_cache = cache;
  d.total_tiles = tiles;
  d.U = (float*)(ws + L.U);
  d.D = (float*)(ws + L.D);
  d.w1 = (float*)(ws + L.w1);
  d.exit = (float*)(ws + L.exit);
  d.a = (float*)(ws + L.a);
  d.b = (float*)(ws + L.b);
  d.counters = (unsigned long long*)(ws + L.counters);
  b->max_depth = max_depth;
  *out = b;
  return BVC_OK;
}

int bvc_batch_launch(bvc_batch b, void* stream) {
  if (!b) return fail(BVC_EINVAL, "batch is null");
  hipStream_t st = (hipStream_t)stream;
  int rc = launch_batch_walks(b->dev, b->max_depth, 0, st);
  if (rc) return rc;
  return launch_batch_gather(b->dev, st);
}

int bvc_batch_counters(bvc_batch b, uint64_t** dev_counters) {
  if (!b || !dev_counters) return fail(BVC_EINVAL, "null argument");
  *dev_counters = (uint64_t*)b->dev.counters;
  return BVC_OK;
}

int bvc_batch_results(bvc_batch b, float** U, float** D, float** a, float** bv) {
  if (!b || !U || !D || !a || !bv) return fail(BVC_EINVAL, "null argument");
  *U = b->dev.U;
  *D = b->dev.D;
  *a = b->dev.a;
  *bv = b->dev.b;
  return BVC_OK;
}

int bvc_batch_destroy(bvc_batch b) {
  delete b;
  return BVC_OK;
}

}  // extern "C"
