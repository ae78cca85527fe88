// Host-side scene: validation, BVH build, pseudonormals, sampling tables and
// the upload into a caller-owned device buffer.
//
// The BVH is a binary AABB hierarchy (the paper's closest-point structure,
// Section 4 "Setup") built by binned surface-area splits of the primitive
// centroids (16 bins per axis; a median split along the widest axis where no
// bin boundary separates them), stored in breadth-first order with both child boxes inside the
// parent, so one node fetch gives the two boxes a nearest-first traversal
// compares.  An FP32 copy of the boxes is rounded outward so that it stays
// conservative for the FP32 walks.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <queue>

#include "bvc_internal.hpp"

namespace bvc {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return BVC_OK;
  return fail(BVC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

struct TmpNode {
  double lo[3], hi[3];
  int left = -1, right = -1;  // tmp ids (internal)
  int start = 0, count = 0;   // leaf range
  bool leaf = false;
  int depth = 1;
};

float round_down(double v) {
  float f = (float)v;
  if ((double)f > v) f = std::nextafter(f, -INFINITY);
  return f;
}
float round_up(double v) {
  float f = (float)v;
  if ((double)f < v) f = std::nextafter(f, INFINITY);
  return f;
}

struct Builder {
  int dim;
  const std::vector<double>& plo;
  const std::vector<double>& phi;
  const std::vector<double>& cen;
  std::vector<int>& perm;
  std::vector<TmpNode> nodes;
  int leaf_max;

  // Half perimeter (2D) or half surface area (3D) of a box.
  double box_cost(const double* lo, const double* hi) const {
    double e[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) e[a] = std::max(0.0, hi[a] - lo[a]);
    return dim == 2 ? e[0] + e[1] : e[0] * e[1] + e[1] * e[2] + e[2] * e[0];
  }

  // Binned surface-area split: minimise n_L cost(L) + n_R cost(R) over 16
  // centroid bins per axis.  Returns the size of the left part after
  // partitioning perm[start, start+count), or -1 when no split separates.
  int sah_split(int start, int count, const double* clo, const double* chi) {
    constexpr int kBins = 16;
    double best = INFINITY;
    int best_axis = -1, best_bin = -1;
    for (int a = 0; a < dim; ++a) {
      const double ext = chi[a] - clo[a];
      if (!(ext > 0)) continue;
      int cnt[kBins] = {0};
      double blo[kBins][3], bhi[kBins][3];
      for (int b = 0; b < kBins; ++b)
        for (int q = 0; q < 3; ++q) {
          blo[b][q] = INFINITY;
          bhi[b][q] = -INFINITY;
        }
      for (int i = start; i < start + count; ++i) {
        const int p = perm[i];
        int b = (int)(kBins * (cen[(size_t)p * dim + a] - clo[a]) / ext);
        b = std::min(kBins - 1, std::max(0, b));
        ++cnt[b];
        for (int q = 0; q < dim; ++q) {
          blo[b][q] = std::min(blo[b][q], plo[(size_t)p * dim + q]);
          bhi[b][q] = std::max(bhi[b][q], phi[(size_t)p * dim + q]);
        }
      }
      // suffix boxes
      double rlo[kBins][3], rhi[kBins][3];
      int rcnt[kBins];
      for (int b = kBins - 1; b >= 0; --b) {
        rcnt[b] = cnt[b] + (b + 1 < kBins ? rcnt[b + 1] : 0);
        for (int q = 0; q < 3; ++q) {
          rlo[b][q] = std::min(blo[b][q], b + 1 < kBins ? rlo[b + 1][q] : INFINITY);
          rhi[b][q] = std::max(bhi[b][q], b + 1 < kBins ? rhi[b + 1][q] : -INFINITY);
        }
      }
      double llo[3] = {INFINITY, INFINITY, INFINITY}, lhi[3] = {-INFINITY, -INFINITY, -INFINITY};
      int lcnt = 0;
      for (int b = 0; b + 1 < kBins; ++b) {
        lcnt += cnt[b];
        for (int q = 0; q < 3; ++q) {
          llo[q] = std::min(llo[q], blo[b][q]);
          lhi[q] = std::max(lhi[q], bhi[b][q]);
        }
        const int rc = rcnt[b + 1];
        if (lcnt == 0 || rc == 0) continue;
        const double cost = lcnt * box_cost(llo, lhi) + rc * box_cost(rlo[b + 1], rhi[b + 1]);
        if (cost < best) {
          best = cost;
          best_axis = a;
          best_bin = b;
        }
      }
    }
    if (best_axis < 0) return -1;
    const double ext = chi[best_axis] - clo[best_axis];
    auto mid = std::stable_partition(perm.begin() + start, perm.begin() + start + count, [&](int p) {
      int b = (int)(kBins * (cen[(size_t)p * dim + best_axis] - clo[best_axis]) / ext);
      b = std::min(kBins - 1, std::max(0, b));
      return b <= best_bin;
    });
    return (int)(mid - (perm.begin() + start));
  }

  int build(int start, int count, int depth) {
    int id = (int)nodes.size();
    nodes.emplace_back();
    TmpNode nd;
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int a = 0; a < 3; ++a) {
      nd.lo[a] = a < dim ? INFINITY : 0;
      nd.hi[a] = a < dim ? -INFINITY : 0;
    }
    for (int i = start; i < start + count; ++i) {
      int p = perm[i];
      for (int a = 0; a < dim; ++a) {
        nd.lo[a] = std::min(nd.lo[a], plo[(size_t)p * dim + a]);
        nd.hi[a] = std::max(nd.hi[a], phi[(size_t)p * dim + a]);
        clo[a] = std::min(clo[a], cen[(size_t)p * dim + a]);
        chi[a] = std::max(chi[a], cen[(size_t)p * dim + a]);
      }
    }
    nd.depth = depth;
    if (count <= leaf_max) {
      nd.leaf = true;
      nd.start = start;
      nd.count = count;
      nodes[id] = nd;
      return id;
    }
    const std::vector<double>& c = cen;
    int d = dim;
    int half = -1;
    if (depth < 32) half = sah_split(start, count, clo, chi);
    if (half <= 0 || half >= count) {
      // median split along the widest centroid axis (also bounds the depth)
      int axis = 0;
      for (int a = 1; a < dim; ++a)
        if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
      half = count / 2;
      std::nth_element(perm.begin() + start, perm.begin() + start + half, perm.begin() + start + count,
                       [&](int x, int y) {
                         double cx = c[(size_t)x * d + axis], cy = c[(size_t)y * d + axis];
                         return cx < cy || (cx == cy && x < y);
                       });
    }
    nodes[id] = nd;
    int l = build(start, half, depth + 1);
    int r = build(start + half, count - half, depth + 1);
    nodes[id].left = l;
    nodes[id].right = r;
    return id;
  }
};

double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

SceneDev SceneHost::view() const {
  SceneDev s;
  s.dim = dim;
  s.np = (int)np;
  s.nv = (int)nv;
  s.ne = (int)ne;
  s.n_nodes = (int)child.size();
  s.depth = depth;
  s.V = (const double*)(dev + off_V);
  s.P = (const int*)(dev + off_P);
  s.E = (const int*)(dev + off_E);
  s.child = (const int2*)(dev + off_child);
  s.box64 = (const double*)(dev + off_box64);
  s.box32 = (const float*)(dev + off_box32);
  s.slab64 = dim == 3 ? (const double*)(dev + off_slab64) : nullptr;
  s.slab32 = dim == 3 ? (const float*)(dev + off_slab32) : nullptr;
  s.prim64 = (const double*)(dev + off_prim64);
  s.prim32 = (const float*)(dev + off_prim32);
  s.prim_id = (const int*)(dev + off_prim_id);
  s.fn = (const double*)(dev + off_fn);
  s.epn = (const double*)(dev + off_epn);
  s.vpn = (const double*)(dev + off_vpn);
  s.cdf = (const double*)(dev + off_cdf);
  s.meas = (const double*)(dev + off_meas);
  s.n_el = (int)cdf_n_el;
  s.sides = cdf_sides;
  s.l = cdf_l;
  return s;
}

static int build_scene(SceneHost& S, int dim, const double* verts, int64_t nv, const int* prims,
                       int64_t np) {
  S.dim = dim;
  S.nv = nv;
  S.np = np;
  S.V.assign(verts, verts + nv * dim);
  S.P.assign(prims, prims + np * dim);
  for (int64_t i = 0; i < nv * dim; ++i)
    if (!std::isfinite(S.V[i])) return fail(BVC_EINVAL, "vertex coordinate is not finite");
  for (int64_t i = 0; i < np * dim; ++i)
    if (S.P[i] < 0 || S.P[i] >= nv) return fail(BVC_EINVAL, "primitive index out of range");
  // measures and degeneracy checks
  S.seg_measure.resize(np);
  S.boundary_measure = 0;
  for (int64_t p = 0; p < np; ++p) {
    const double* a = &S.V[(size_t)S.P[p * dim] * dim];
    const double* b = &S.V[(size_t)S.P[p * dim + 1] * dim];
    double m;
    if (dim == 2) {
      m = std::sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]));
      if (!(m > 0)) return fail(BVC_EINVAL, "zero-length segment " + std::to_string(p));
    } else {
      const double* c = &S.V[(size_t)S.P[p * dim + 2] * dim];
      double ab[3], ac[3], x[3];
      for (int q = 0; q < 3; ++q) {
        ab[q] = b[q] - a[q];
        ac[q] = c[q] - a[q];
      }
      cross3(ab, ac, x);
      m = 0.5 * std::sqrt(dot3(x, x));
      if (!(m > 0)) return fail(BVC_EINVAL, "zero-area triangle " + std::to_string(p));
    }
    S.seg_measure[p] = m;
    S.boundary_measure += m;
  }
  for (int a = 0; a < 3; ++a) {
    S.lo[a] = a < dim ? INFINITY : 0;
    S.hi[a] = a < dim ? -INFINITY : 0;
  }
  for (int64_t v = 0; v < nv; ++v)
    for (int a = 0; a < dim; ++a) {
      S.lo[a] = std::min(S.lo[a], S.V[v * dim + a]);
      S.hi[a] = std::max(S.hi[a], S.V[v * dim + a]);
    }
  // primitive bounds and centroids
  std::vector<double> plo(np * dim), phi(np * dim), cen(np * dim);
  for (int64_t p = 0; p < np; ++p)
    for (int a = 0; a < dim; ++a) {
      double mn = INFINITY, mx = -INFINITY, s = 0;
      for (int c = 0; c < dim; ++c) {
        double v = S.V[(size_t)S.P[p * dim + c] * dim + a];
        mn = std::min(mn, v);
        mx = std::max(mx, v);
        s += v;
      }
      plo[p * dim + a] = mn;
      phi[p * dim + a] = mx;
      cen[p * dim + a] = s / dim;
    }
  std::vector<int> perm(np);
  std::iota(perm.begin(), perm.end(), 0);
  // Up to three primitives per leaf while the node indices fit (measured
  // best for the walks' closest-point queries among 1 to 8: shallower trees
  // trade node expansions for primitive tests, which the traversal takes one
  // per step); larger scenes use leaves of up to kLeafMax primitives.
  const int leaf_max = np < (1 << 17) ? 3 : kLeafMax;
  Builder B{dim, plo, phi, cen, perm, {}, leaf_max};
  B.nodes.reserve(2 * np + 2);
  int root = B.build(0, (int)np, 1);
  std::vector<TmpNode>& T = B.nodes;
  // a single-leaf scene gets an internal root with an empty sibling
  if (T[root].leaf) {
    TmpNode r = T[root];
    TmpNode leafcopy = T[root];
    leafcopy.depth = 2;
    r.leaf = false;
    TmpNode empty;
    for (int a = 0; a < 3; ++a) {
      empty.lo[a] = INFINITY;
      empty.hi[a] = -INFINITY;
    }
    empty.leaf = true;
    empty.start = 0;
    empty.count = 1;
    empty.depth = 2;
    T.push_back(empty);
    T.push_back(leafcopy);
    T[root] = r;
    T[root].left = (int)T.size() - 1;
    T[root].right = (int)T.size() - 2;
  }
  // breadth-first numbering of internal nodes
  std::vector<int> bfs_id(T.size(), -1);
  std::vector<int> order;
  std::queue<int> q;
  q.push(root);
  while (!q.empty()) {
    int t = q.front();
    q.pop();
    if (T[t].leaf) continue;
    bfs_id[t] = (int)order.size();
    order.push_back(t);
    q.push(T[t].left);
    q.push(T[t].right);
  }
  int nn = (int)order.size();
  if (nn >= (1 << 17)) return fail(BVC_EUNSUPPORTED, "scene needs more than 2^17 BVH nodes");
  int bw = 4 * dim;  // doubles per node: two children x (lo, hi)
  S.child.resize(nn);
  S.box64.assign((size_t)nn * bw, 0.0);
  S.box32.assign((size_t)nn * bw, 0.0f);
  S.depth = 0;
  for (int i = 0; i < nn; ++i) {
    const TmpNode& nd = T[order[i]];
    S.depth = std::max(S.depth, nd.depth);
    int kids[2] = {nd.left, nd.right};
    int link[2];
    for (int c = 0; c < 2; ++c) {
      const TmpNode& k = T[kids[c]];
      link[c] = k.leaf ? encode_leaf(k.start, k.count) : bfs_id[kids[c]];
      for (int a = 0; a < dim; ++a) {
        double lo = k.lo[a], hi = k.hi[a];
        S.box64[(size_t)i * bw + c * 2 * dim + a] = lo;
        S.box64[(size_t)i * bw + c * 2 * dim + dim + a] = hi;
        S.box32[(size_t)i * bw + c * 2 * dim + a] = std::isfinite(lo) ? round_down(lo) : (float)lo;
        S.box32[(size_t)i * bw + c * 2 * dim + dim + a] = std::isfinite(hi) ? round_up(hi) : (float)hi;
      }
    }
    S.child[i] = make_int2(link[0], link[1]);
  }
  if (dim == 3) {
    // A second bound per child (3D): the slab of its triangles along their
    // area-weighted mean normal n.  Every point y of those triangles has
    // smin <= n.y <= smax, so the distance from p to any of them is at least
    // the distance from n.p to [smin, smax]; a patch of a smooth surface is
    // thin along its normal, where its box is not.  The FP64 range is widened
    // by the rounding of n.p in FP64, the FP32 one by that of n.p in FP32 for
    // |p| up to four times the scene's extent (and by the FP32 axis's
    // departure from unit length), so both stay lower bounds.
    std::vector<int> rs(T.size(), 0), re(T.size(), 0);
    std::vector<int> post;
    std::vector<std::pair<int, bool>> st{{root, false}};
    while (!st.empty()) {
      auto [t, done] = st.back();
      st.pop_back();
      if (T[t].leaf) {
        rs[t] = T[t].start;
        re[t] = T[t].start + T[t].count;
      } else if (!done) {
        st.push_back({t, true});
        st.push_back({T[t].left, false});
        st.push_back({T[t].right, false});
      } else {
        rs[t] = std::min(rs[T[t].left], rs[T[t].right]);
        re[t] = std::max(re[T[t].left], re[T[t].right]);
      }
    }
    double M = 1.0;
    for (int a = 0; a < 3; ++a) M = std::max(M, 4.0 * std::max(std::fabs(S.lo[a]), std::fabs(S.hi[a])));
    S.slab64.assign((size_t)nn * 12, 0.0);
    S.slab32.assign((size_t)nn * 12, 0.0f);
    for (int i = 0; i < nn; ++i) {
      const TmpNode& nd = T[order[i]];
      int kids[2] = {nd.left, nd.right};
      for (int c = 0; c < 2; ++c) {
        const TmpNode& k = T[kids[c]];
        double* o64 = &S.slab64[(size_t)i * 12 + c * 5];
        float* o32 = &S.slab32[(size_t)i * 12 + c * 5];
        if (!std::isfinite(k.lo[0])) {  // the empty sibling of a single-leaf root
          o64[2] = o32[2] = 1;
          o64[3] = o32[3] = INFINITY;
          o64[4] = o32[4] = -INFINITY;
          continue;
        }
        double n[3] = {0, 0, 0}, area2 = 0;
        for (int j = rs[kids[c]]; j < re[kids[c]]; ++j) {
          const int t = perm[j];
          const double* A = &S.V[(size_t)S.P[3 * t] * 3];
          const double* Bv = &S.V[(size_t)S.P[3 * t + 1] * 3];
          const double* Cv = &S.V[(size_t)S.P[3 * t + 2] * 3];
          double ab[3], ac[3], x[3];
          for (int a = 0; a < 3; ++a) {
            ab[a] = Bv[a] - A[a];
            ac[a] = Cv[a] - A[a];
          }
          cross3(ab, ac, x);
          for (int a = 0; a < 3; ++a) n[a] += x[a];
          area2 += std::sqrt(dot3(x, x));
        }
        double len = std::sqrt(dot3(n, n));
        if (!(len > 1e-9 * area2)) {
          // no dominant normal (a closed or folded patch): the axis of the
          // box's thinnest side, which then adds nothing but costs nothing
          int a_min = 0;
          for (int a = 1; a < 3; ++a)
            if (k.hi[a] - k.lo[a] < k.hi[a_min] - k.lo[a_min]) a_min = a;
          n[0] = n[1] = n[2] = 0;
          n[a_min] = 1;
          len = 1;
        }
        double n64[3], n32d[3];
        float n32[3];
        for (int a = 0; a < 3; ++a) {
          n64[a] = n[a] / len;
          n32[a] = (float)n64[a];
          n32d[a] = (double)n32[a];
        }
        double lo64 = INFINITY, hi64 = -INFINITY, lo32 = INFINITY, hi32 = -INFINITY;
        for (int j = rs[kids[c]]; j < re[kids[c]]; ++j)
          for (int v = 0; v < 3; ++v) {
            const double* y = &S.V[(size_t)S.P[3 * perm[j] + v] * 3];
            const double s64 = dot3(n64, y), s32 = dot3(n32d, y);
            lo64 = std::min(lo64, s64);
            hi64 = std::max(hi64, s64);
            lo32 = std::min(lo32, s32);
            hi32 = std::max(hi32, s32);
          }
        const double l1_64 = std::fabs(n64[0]) + std::fabs(n64[1]) + std::fabs(n64[2]);
        const double l1_32 = std::fabs(n32d[0]) + std::fabs(n32d[1]) + std::fabs(n32d[2]);
        const double m64 = 16.0 * std::ldexp(1.0, -53) * M * l1_64;
        const double m32 = 16.0 * std::ldexp(1.0, -24) * M * l1_32;
        for (int a = 0; a < 3; ++a) {
          o64[a] = n64[a];
          o32[a] = n32[a];
        }
        o64[3] = lo64 - m64;
        o64[4] = hi64 + m64;
        o32[3] = round_down(lo32 - m32);
        o32[4] = round_up(hi32 + m32);
      }
    }
  }
  // leaf-ordered primitive records
  int pw = dim == 2 ? 4 : 12;
  S.prim64.assign((size_t)np * pw, 0.0);
  S.prim32.assign((size_t)np * pw, 0.0f);
  S.prim_id.resize(np);
  for (int64_t i = 0; i < np; ++i) {
    int p = perm[i];
    S.prim_id[i] = p;
    for (int c = 0; c < dim; ++c)
      for (int a = 0; a < dim; ++a) {
        double v = S.V[(size_t)S.P[(size_t)p * dim + c] * dim + a];
        S.prim64[(size_t)i * pw + c * dim + a] = v;
        S.prim32[(size_t)i * pw + c * dim + a] = (float)v;
      }
    if (dim == 3) {
      // the closest-point test's |b-a|^2, (b-a).(c-a), |c-a|^2, from the edge
      // vectors each precision's test forms itself (FP32 differences of the
      // FP32 vertices), summed in FP64
      double* r64 = &S.prim64[(size_t)i * pw];
      float* r32 = &S.prim32[(size_t)i * pw];
      double e64[2][3], e32[2][3];
      for (int e = 0; e < 2; ++e)
        for (int a = 0; a < 3; ++a) {
          e64[e][a] = r64[3 * (e + 1) + a] - r64[a];
          e32[e][a] = (double)(r32[3 * (e + 1) + a] - r32[a]);
        }
      const int pairs[3][2] = {{0, 0}, {0, 1}, {1, 1}};
      for (int k = 0; k < 3; ++k) {
        double s64 = 0.0, s32 = 0.0;
        for (int a = 0; a < 3; ++a) {
          s64 += e64[pairs[k][0]][a] * e64[pairs[k][1]][a];
          s32 += e32[pairs[k][0]][a] * e32[pairs[k][1]][a];
        }
        r64[9 + k] = s64;
        r32[9 + k] = (float)s32;
      }
    }
  }
  if (dim == 3) {
    // face normals, angle-weighted vertex pseudonormals, edge pseudonormals
    S.fn.assign(np * 3, 0.0);
    S.vpn.assign(nv * 3, 0.0);
    S.epn.assign(np * 9, 0.0);
    for (int64_t t = 0; t < np; ++t) {
      const double* A = &S.V[(size_t)S.P[3 * t] * 3];
      const double* Bv = &S.V[(size_t)S.P[3 * t + 1] * 3];
      const double* C = &S.V[(size_t)S.P[3 * t + 2] * 3];
      double ab[3], ac[3], n[3];
      for (int a = 0; a < 3; ++a) {
        ab[a] = Bv[a] - A[a];
        ac[a] = C[a] - A[a];
      }
      cross3(ab, ac, n);
      double len = std::sqrt(dot3(n, n));
      for (int a = 0; a < 3; ++a) S.fn[3 * t + a] = n[a] / len;
      const double* corner[3] = {A, Bv, C};
      for (int c = 0; c < 3; ++c) {
        double u[3], v[3];
        for (int a = 0; a < 3; ++a) {
          u[a] = corner[(c + 1) % 3][a] - corner[c][a];
          v[a] = corner[(c + 2) % 3][a] - corner[c][a];
        }
        double cs = dot3(u, v) / std::sqrt(dot3(u, u) * dot3(v, v));
        double ang = std::acos(std::max(-1.0, std::min(1.0, cs)));
        int vi = S.P[3 * t + c];
        for (int a = 0; a < 3; ++a) S.vpn[3 * vi + a] += ang * S.fn[3 * t + a];
      }
    }
    struct Rec {
      int64_t key;
      int64_t t;
      int e;
    };
    std::vector<Rec> rec;
    rec.reserve(3 * np);
    for (int64_t t = 0; t < np; ++t)
      for (int e = 0; e < 3; ++e) {
        int64_t a = S.P[3 * t + e], b = S.P[3 * t + (e + 1) % 3];
        rec.push_back({std::min(a, b) * nv + std::max(a, b), t, e});
      }
    std::stable_sort(rec.begin(), rec.end(), [](const Rec& x, const Rec& y) { return x.key < y.key; });
    S.E.clear();
    S.edge_len.clear();
    for (size_t i = 0; i < rec.size();) {
      size_t j = i;
      double sum[3] = {0, 0, 0};
      while (j < rec.size() && rec[j].key == rec[i].key) {
        for (int a = 0; a < 3; ++a) sum[a] += S.fn[3 * rec[j].t + a];
        ++j;
      }
      for (size_t k = i; k < j; ++k)
        for (int a = 0; a < 3; ++a) S.epn[9 * rec[k].t + 3 * rec[k].e + a] = sum[a];
      int a0 = (int)(rec[i].key / nv), a1 = (int)(rec[i].key % nv);
      S.E.push_back(a0);
      S.E.push_back(a1);
      const double* A = &S.V[(size_t)a0 * 3];
      const double* Bv = &S.V[(size_t)a1 * 3];
      double ab[3] = {Bv[0] - A[0], Bv[1] - A[1], Bv[2] - A[2]};
      S.edge_len.push_back(std::sqrt(dot3(ab, ab)));
      i = j;
    }
    S.ne = (int64_t)S.E.size() / 2;
  }
  // device layout
  S.n_el_max = dim == 2 ? 2 * np + nv : np + S.ne + nv;
  size_t off = 0;
  auto place = [&](size_t& o, size_t bytes) {
    o = off;
    off = align256(off + std::max<size_t>(bytes, 1));
  };
  place(S.off_V, S.V.size() * sizeof(double));
  place(S.off_P, S.P.size() * sizeof(int));
  place(S.off_E, S.E.size() * sizeof(int));
  place(S.off_child, S.child.size() * sizeof(int2));
  place(S.off_box64, S.box64.size() * sizeof(double));
  place(S.off_box32, S.box32.size() * sizeof(float));
  place(S.off_slab64, S.slab64.size() * sizeof(double));
  place(S.off_slab32, S.slab32.size() * sizeof(float));
  place(S.off_prim64, S.prim64.size() * sizeof(double));
  place(S.off_prim32, S.prim32.size() * sizeof(float));
  place(S.off_prim_id, S.prim_id.size() * sizeof(int));
  place(S.off_fn, S.fn.size() * sizeof(double));
  place(S.off_epn, S.epn.size() * sizeof(double));
  place(S.off_vpn, S.vpn.size() * sizeof(double));
  place(S.off_cdf, (size_t)(S.n_el_max + 1) * sizeof(double));
  place(S.off_meas, (size_t)S.n_el_max * sizeof(double));
  S.bytes = off;
  return BVC_OK;
}

// Sampling table of the candidate measure for (l, sides), in the element
// order: 2D segments (each side in turn) then vertex circles; 3D faces, edge
// cylinders, vertex spheres.  Prefix sums run sequentially in FP64.
int ensure_cdf(SceneHost& S, double l, int sides, hipStream_t stream) {
  if (S.cdf_l == l && S.cdf_sides == sides) return BVC_OK;
  std::vector<double> meas;
  if (S.dim == 2) {
    for (int64_t p = 0; p < S.np; ++p)
      for (int s = 0; s < sides; ++s) meas.push_back(S.seg_measure[p]);
    for (int64_t v = 0; v < S.nv; ++v) meas.push_back(2 * kPi * l);
  } else {
    for (int64_t p = 0; p < S.np; ++p) meas.push_back(S.seg_measure[p]);
    for (int64_t e = 0; e < S.ne; ++e) meas.push_back(2 * kPi * l * S.edge_len[e]);
    for (int64_t v = 0; v < S.nv; ++v) meas.push_back(4 * kPi * l * l);
  }
  std::vector<double> cdf(meas.size() + 1);
  cdf[0] = 0;
  for (size_t i = 0; i < meas.size(); ++i) cdf[i + 1] = cdf[i] + meas[i];
  int rc = check_hip(hipMemcpyAsync(S.dev + S.off_cdf, cdf.data(), cdf.size() * sizeof(double),
                                    hipMemcpyHostToDevice, stream),
                     "cdf upload");
  if (rc) return rc;
  rc = check_hip(hipMemcpyAsync(S.dev + S.off_meas, meas.data(), meas.size() * sizeof(double),
                                hipMemcpyHostToDevice, stream),
                 "measure upload");
  if (rc) return rc;
  rc = check_hip(hipStreamSynchronize(stream), "cdf upload sync");
  if (rc) return rc;
  S.cdf_l = l;
  S.cdf_sides = sides;
  S.cdf_n_el = (int64_t)meas.size();
  return BVC_OK;
}

double candidate_measure(const SceneHost& S, double l, int sides) {
  double total = 0;
  if (S.dim == 2) {
    for (int64_t p = 0; p < S.np; ++p)
      for (int s = 0; s < sides; ++s) total += S.seg_measure[p];
    for (int64_t v = 0; v < S.nv; ++v) total += 2 * kPi * l;
  } else {
    for (int64_t p = 0; p < S.np; ++p) total += S.seg_measure[p];
    for (int64_t e = 0; e < S.ne; ++e) total += 2 * kPi * l * S.edge_len[e];
    for (int64_t v = 0; v < S.nv; ++v) total += 4 * kPi * l * l;
  }
  return total;
}

}  // namespace bvc

using namespace bvc;

extern "C" {

const char* bvc_last_error(void) { return g_err.c_str(); }
const char* bvc_version(void) { return "bvc-mi355x 0.1 (gfx950)"; }

int bvc_scene_create(int32_t dim, const double* verts, int64_t n_verts, const int32_t* prims,
                     int64_t n_prims, bvc_scene* out) {
  if (!out) return fail(BVC_EINVAL, "out is null");
  *out = nullptr;
  if (dim != 2 && dim != 3) return fail(BVC_EINVAL, "dim must be 2 or 3");
  if (!verts || !prims) return fail(BVC_EINVAL, "verts/prims is null");
  if (n_verts < dim || n_prims < 1) return fail(BVC_EINVAL, "empty scene");
  if (n_prims >= (1 << 27) || n_verts >= (1 << 30)) return fail(BVC_EINVAL, "scene too large");
  bvc_scene s = new (std::nothrow) bvc_scene_s;
  if (!s) return fail(BVC_ENOMEM, "host allocation failed");
  int rc;
  try {
    rc = build_scene(s->h, dim, verts, n_verts, prims, n_prims);
  } catch (const std::bad_alloc&) {
    rc = fail(BVC_ENOMEM, "host allocation failed");
  }
  if (rc) {
    delete s;
    return rc;
  }
  *out = s;
  return BVC_OK;
}

int bvc_scene_get_info(bvc_scene s, bvc_scene_info* out) {
  if (!s || !out) return fail(BVC_EINVAL, "null argument");
  const SceneHost& h = s->h;
  out->dim = h.dim;
  out->n_verts = h.nv;
  out->n_prims = h.np;
  out->n_edges = h.ne;
  out->n_nodes = (int64_t)h.child.size();
  out->depth = h.depth;
  for (int a = 0; a < 3; ++a) {
    out->lo[a] = h.lo[a];
    out->hi[a] = h.hi[a];
  }
  double d2 = 0;
  for (int a = 0; a < h.dim; ++a) d2 += (h.hi[a] - h.lo[a]) * (h.hi[a] - h.lo[a]);
  out->diagonal = std::sqrt(d2);
  out->boundary_measure = h.boundary_measure;
  out->device_bytes = h.bytes;
  out->uploaded = h.dev != nullptr;
  return BVC_OK;
}

int bvc_scene_export_bvh(bvc_scene s, int32_t* child, double* boxes, int32_t* order) {
  if (!s) return fail(BVC_EINVAL, "null scene");
  const SceneHost& h = s->h;
  if (child)
    for (size_t i = 0; i < h.child.size(); ++i) {
      child[2 * i] = h.child[i].x;
      child[2 * i + 1] = h.child[i].y;
    }
  if (boxes) std::copy(h.box64.begin(), h.box64.end(), boxes);
  if (order) std::copy(h.prim_id.begin(), h.prim_id.end(), order);
  return BVC_OK;
}

int bvc_scene_export_slabs(bvc_scene s, double* slabs) {
  if (!s || !slabs) return fail(BVC_EINVAL, "null argument");
  const SceneHost& h = s->h;
  if (h.dim != 3) return fail(BVC_EUNSUPPORTED, "slab bounds exist for 3D scenes only");
  std::copy(h.slab64.begin(), h.slab64.end(), slabs);
  return BVC_OK;
}

int bvc_scene_upload(bvc_scene s, void* buf, size_t bytes, void* stream) {
  if (!s || !buf) return fail(BVC_EINVAL, "null argument");
  SceneHost& h = s->h;
  if (bytes < h.bytes) return fail(BVC_EINVAL, "device buffer too small");
  if (((uintptr_t)buf & 255) != 0) return fail(BVC_EINVAL, "device buffer must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  std::vector<char> staging(h.bytes, 0);
  auto put = [&](size_t off, const void* p, size_t n) {
    if (n) std::memcpy(staging.data() + off, p, n);
  };
  put(h.off_V, h.V.data(), h.V.size() * sizeof(double));
  put(h.off_P, h.P.data(), h.P.size() * sizeof(int));
  put(h.off_E, h.E.data(), h.E.size() * sizeof(int));
  put(h.off_child, h.child.data(), h.child.size() * sizeof(int2));
  put(h.off_box64, h.box64.data(), h.box64.size() * sizeof(double));
  put(h.off_box32, h.box32.data(), h.box32.size() * sizeof(float));
  put(h.off_slab64, h.slab64.data(), h.slab64.size() * sizeof(double));
  put(h.off_slab32, h.slab32.data(), h.slab32.size() * sizeof(float));
  put(h.off_prim64, h.prim64.data(), h.prim64.size() * sizeof(double));
  put(h.off_prim32, h.prim32.data(), h.prim32.size() * sizeof(float));
  put(h.off_prim_id, h.prim_id.data(), h.prim_id.size() * sizeof(int));
  put(h.off_fn, h.fn.data(), h.fn.size() * sizeof(double));
  put(h.off_epn, h.epn.data(), h.epn.size() * sizeof(double));
  put(h.off_vpn, h.vpn.data(), h.vpn.size() * sizeof(double));
  int rc = check_hip(hipMemcpyAsync(buf, staging.data(), h.bytes, hipMemcpyHostToDevice, st),
                     "scene upload");
  if (rc) return rc;
  rc = check_hip(hipStreamSynchronize(st), "scene upload sync");
  if (rc) return rc;
  h.dev = (char*)buf;
  h.cdf_l = -1;
  h.cdf_sides = -1;
  return BVC_OK;
}

bvc_scene_s::~bvc_scene_s() {
  if (wost_tab) {
    // uploads from the pinned tables may still be in flight
    (void)hipDeviceSynchronize();
    (void)hipHostFree(wost_tab);
  }
}

int bvc_scene_destroy(bvc_scene s) {
  delete s;
  return BVC_OK;
}

int bvc_cache_measure(bvc_scene s, double l, int32_t sides, double* measure) {
  if (!s || !measure) return fail(BVC_EINVAL, "null argument");
  if (!(l > 0)) return fail(BVC_EINVAL, "offset l must be positive");
  if (sides != 1 && sides != 2) return fail(BVC_EINVAL, "sides must be 1 or 2");
  if (sides == 2 && s->h.dim == 3) return fail(BVC_EUNSUPPORTED, "two-sided offsets are 2D only");
  *measure = candidate_measure(s->h, l, sides);
  return BVC_OK;
}

}  // extern "C"
