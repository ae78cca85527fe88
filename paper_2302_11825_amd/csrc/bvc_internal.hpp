// Internal declarations shared by the host entry points and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/bvc.h"

namespace bvc {

constexpr int kLeafMax = 4;      // primitives per BVH leaf
constexpr int kMaxDepth = 48;    // bound on the traversal stack
constexpr double kPi = 3.141592653589793238462643383279502884;

// Child link encoding: >= 0 internal node index; < 0 leaf ~(start << 3 | (count - 1)).
__host__ __device__ inline int encode_leaf(int start, int count) { return ~((start << 3) | (count - 1)); }
__host__ __device__ inline int leaf_start(int c) { return (~c) >> 3; }
__host__ __device__ inline int leaf_count(int c) { return ((~c) & 7) + 1; }

// Device view of an uploaded scene (pointers into the caller's buffer).
struct SceneDev {
  int dim;
  int np, nv, ne, n_nodes, depth;
  const double* V;      // [nv][dim] original vertices
  const int* P;         // [np][dim] original primitives
  const int* E;         // [ne][2] unique edges (3D)
  const int2* child;    // [n_nodes] child links
  const double* box64;  // [n_nodes][4*dim]: child0 lo, child0 hi, child1 lo, child1 hi
  const float* box32;   // same, rounded outward
  const double* slab64; // 3D [n_nodes][12]: per child, a unit axis n and the range [smin, smax]
                        // of n.y over the child's triangles (n0 smin0 smax0 n1 smin1 smax1 0 0)
  const float* slab32;  // same with the axis rounded to FP32 and the range widened outward
  const double* prim64; // leaf order: 2D [np][4] (a, b); 3D [np][12] (a, b, c, |b-a|^2, (b-a).(c-a), |c-a|^2)
  const float* prim32;  // same layout in FP32
  const int* prim_id;   // leaf order -> original primitive id
  const double* fn;     // 3D [np][3] unit face normals (original order)
  const double* epn;    // 3D [np][9] edge pseudonormals of edges (ab, bc, ca)
  const double* vpn;    // 3D [nv][3] angle-weighted vertex pseudonormals
  const double* cdf;    // [n_el + 1] sampling CDF for the current (l, sides)
  const double* meas;   // [n_el] element measures
  int n_el;
  int sides;
  double l;
};

struct FieldDev {
  int kind;
  int n_coef;
  const double* coef;
  double param[8];
};

inline FieldDev to_dev(const bvc_field& f) {
  FieldDev d;
  d.kind = f.kind;
  d.n_coef = f.n_coef;
  d.coef = f.coef;
  for (int i = 0; i < 8; ++i) d.param[i] = f.param[i];
  return d;
}

// Host-side scene.
struct SceneHost {
  int dim = 0;
  int64_t nv = 0, np = 0, ne = 0;
  std::vector<double> V;
  std::vector<int> P;
  std::vector<int> E;
  std::vector<int2> child;
  std::vector<double> box64;
  std::vector<float> box32;
  std::vector<double> slab64;
  std::vector<float> slab32;
  std::vector<double> prim64;
  std::vector<float> prim32;
  std::vector<int> prim_id;
  std::vector<double> fn, epn, vpn;
  std::vector<double> seg_measure;  // length (2D) / area (3D) per primitive
  std::vector<double> edge_len;     // 3D
  int depth = 0;
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  double boundary_measure = 0;
  // device placement
  size_t bytes = 0;
  size_t off_V = 0, off_P = 0, off_E = 0, off_child = 0, off_box64 = 0, off_box32 = 0, off_slab64 = 0,
         off_slab32 = 0,
         off_prim64 = 0, off_prim32 = 0, off_prim_id = 0, off_fn = 0, off_epn = 0, off_vpn = 0,
         off_cdf = 0, off_meas = 0;
  int64_t n_el_max = 0;
  char* dev = nullptr;
  // cached sampling table
  double cdf_l = -1;
  int cdf_sides = -1;
  int64_t cdf_n_el = 0;
  SceneDev view() const;
};

// One scene of a multi-scene batch (device table entry).
struct BatchSceneDev {
  SceneDev S;
  FieldDev g, f;
  double eps;
  int max_steps, W;
  uint64_t seed;
  uint32_t batch;
  int cv;
  int64_t n_cache, n_eval;
  const double* x;     // cache [dim][n_cache] FP64
  const double* nrm;
  const double* R0;
  const double* xbar;
  const double* w;
  const float* cx;     // cache [dim][n_cache] FP32
  const float* cn;
  const float* ex;     // evaluation points [dim][n_eval] FP32
  float* u;            // [n_eval]
  uint64_t walk_off;   // first walk of this scene in the batch's walk space
  int64_t cache_off;   // first cache point in the batch's concatenated arrays
  int64_t tile_off;    // first gather tile (512 evaluation points each)
};

struct BatchDev {
  const BatchSceneDev* scenes;
  int n_scenes;
  int dim;
  int has_src;
  uint64_t total_walks;
  int64_t total_cache;
  int64_t total_tiles;
  float* U;       // [total_walks]
  float* D;       // [total_walks]
  float* exit;    // [dim][total_walks]
  float* w1;      // [total_walks]
  float* a;       // [total_cache]
  float* b;       // [total_cache]
  unsigned long long* counters;  // [4]
  unsigned long long chunk;      // walk ids per queue claim (set at launch)
};

// Batch launchers (walks.hip, kernels_gather.hip).
int launch_batch_walks(const BatchDev& b, int max_depth, int blocks, hipStream_t st);
int launch_batch_gather(const BatchDev& b, hipStream_t st);

// Clamping correction launchers (kernels_clamp.hip).
int launch_ray_hits(const SceneHost& h, int64_t n, const double* x, const int* wind, double l, int sides, double c,
                    double t_max, int n_rays, int max_hits, uint64_t seed, uint32_t batch, double* slot_x,
                    double* slot_R0, double* slot_xbar, double* slot_w, int* flags, unsigned long long* counters,
                    hipStream_t st);
int launch_point_winding(const SceneHost& h, int64_t n, const double* x, int* wind, hipStream_t st);
int launch_corr_sum(const bvc_field& g, int dim, int dtype, int64_t n, int n_rays, int max_hits,
                    const double* slot_w, const void* EX, const void* U, const int64_t* out, void* u,
                    hipStream_t st);

// Error helpers (thread-local message).
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int check_hip(hipError_t e, const char* what);
int check_scene(bvc_scene s);
int check_field(const bvc_field& f, int dim, const char* name);
int num_cus();
// Zero `bytes` (a multiple of 4) of device memory with a kernel rather than a
// memset node, so the call stays correct inside a captured HIP graph.
int zero_async(void* p, size_t bytes, hipStream_t st);

}  // namespace bvc

struct bvc_scene_s {
  bvc::SceneHost h;
  // walk-on-stars tables of this scene as a Neumann part, built at its first
  // bvc_wost_walks into pinned host memory, so that every call uploads them
  // without waiting: [links | cones], wost_bytes = {links, cones} in bytes
  void* wost_tab = nullptr;
  size_t wost_bytes[2] = {0, 0};
  std::mutex wost_mu;
  bvc_scene_s() = default;
  bvc_scene_s(const bvc_scene_s&) = delete;
  bvc_scene_s& operator=(const bvc_scene_s&) = delete;
  ~bvc_scene_s();
};
