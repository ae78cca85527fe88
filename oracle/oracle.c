/*
 * Plain FP64 CPU oracle for Boundary Value Caching with walk on spheres.
 * TEST INFRASTRUCTURE ONLY (see oracle.h): loaded by the tests, the smoke
 * check and the CPU-baseline leg of the benchmark, never by the product path.
 *
 * Everything here is written for checkability, not speed: plain loops in the
 * order the paper states them, FP64 throughout, no blocking or fusion.  The
 * only acceleration is a simple median-split BVH for closest points, checked
 * against the brute-force scan it replaces.  OpenMP splits independent outer
 * loops (cache points, evaluation points); it never reorders a sum.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ======================================================================== */
/* Philox-4x32-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2,  */
/* 3", SC'11): ten rounds of two 32x32->64 multiplies with a Weyl key update. */
/* ======================================================================== */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t mul_a = 0xD2511F53u, mul_b = 0xCD9E8D57u;
  const uint32_t weyl_a = 0x9E3779B9u, weyl_b = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t prod_a = (uint64_t)mul_a * (uint64_t)x0;
    uint64_t prod_b = (uint64_t)mul_b * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(prod_b >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)prod_b;
    uint32_t y2 = (uint32_t)(prod_a >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)prod_a;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
    k0 += weyl_a;
    k1 += weyl_b;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

static double u53(uint32_t hi, uint32_t lo) {
  uint64_t bits = ((uint64_t)hi << 21) | (uint64_t)(lo >> 11);
  return (double)bits * (1.0 / 9007199254740992.0); /* 2^-53 */
}

void orc_uniform_pair(uint64_t seed, uint32_t block, uint32_t id, uint32_t batch,
                      uint32_t tag, double* ua, double* ub) {
  uint32_t ctr[4] = {block, id, batch, tag};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  *ua = u53(w[0], w[1]);
  *ub = u53(w[2], w[3]);
}

/* ======================================================================== */
/* Scene, BVH and closest points                                             */
/* ======================================================================== */

typedef struct {
  double lo[3], hi[3];
  int64_t left, right; /* children (internal) or -1 */
  int64_t start, count; /* primitive range in perm (leaf) */
} onode;

struct orc_scene {
  int dim;
  int64_t nv, np;
  double* V;
  int32_t* P;
  int64_t n_nodes;
  onode* nodes;
  int32_t* perm;
  /* 3D only */
  double* fnorm;    /* unit face normals (np x 3) */
  double* vpn;      /* angle-weighted vertex pseudonormals (nv x 3) */
  double* epn;      /* per-triangle edge pseudonormals (np x 3 edges x 3) */
  int64_t ne;
  int32_t* edges;   /* unique edges (ne x 2) */
};

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

static void prim_bounds(const orc_scene* s, int64_t p, double* lo, double* hi, double* cen) {
  int d = s->dim;
  for (int a = 0; a < d; ++a) {
    lo[a] = INFINITY;
    hi[a] = -INFINITY;
    cen[a] = 0;
  }
  for (int c = 0; c < d; ++c) {
    const double* v = s->V + (int64_t)s->P[p * d + c] * d;
    for (int a = 0; a < d; ++a) {
      if (v[a] < lo[a]) lo[a] = v[a];
      if (v[a] > hi[a]) hi[a] = v[a];
      cen[a] += v[a] / d;
    }
  }
}

typedef struct {
  const double* cen;
  int axis;
  int dim;
} sort_ctx;
static sort_ctx g_sort; /* build is single-threaded */
static int cmp_prim(const void* pa, const void* pb) {
  int32_t a = *(const int32_t*)pa, b = *(const int32_t*)pb;
  double ca = g_sort.cen[(int64_t)a * g_sort.dim + g_sort.axis];
  double cb = g_sort.cen[(int64_t)b * g_sort.dim + g_sort.axis];
  if (ca < cb) return -1;
  if (ca > cb) return 1;
  return (a < b) ? -1 : (a > b);
}

static int64_t build_node(orc_scene* s, const double* plo, const double* phi, const double* cen,
                          int64_t start, int64_t count) {
  int d = s->dim;
  int64_t id = s->n_nodes++;
  onode* nd = &s->nodes[id];
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int a = 0; a < 3; ++a) {
    nd->lo[a] = (a < d) ? INFINITY : 0;
    nd->hi[a] = (a < d) ? -INFINITY : 0;
  }
  for (int64_t i = start; i < start + count; ++i) {
    int32_t p = s->perm[i];
    for (int a = 0; a < d; ++a) {
      if (plo[(int64_t)p * d + a] < nd->lo[a]) nd->lo[a] = plo[(int64_t)p * d + a];
      if (phi[(int64_t)p * d + a] > nd->hi[a]) nd->hi[a] = phi[(int64_t)p * d + a];
      if (cen[(int64_t)p * d + a] < clo[a]) clo[a] = cen[(int64_t)p * d + a];
      if (cen[(int64_t)p * d + a] > chi[a]) chi[a] = cen[(int64_t)p * d + a];
    }
  }
  nd->start = start;
  nd->count = count;
  nd->left = nd->right = -1;
  if (count <= 4) return id;
  int axis = 0;
  for (int a = 1; a < d; ++a)
    if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
  g_sort.cen = cen;
  g_sort.axis = axis;
  g_sort.dim = d;
  qsort(s->perm + start, (size_t)count, sizeof(int32_t), cmp_prim);
  int64_t half = count / 2;
  int64_t l = build_node(s, plo, phi, cen, start, half);
  int64_t r = build_node(s, plo, phi, cen, start + half, count - half);
  s->nodes[id].left = l;
  s->nodes[id].right = r;
  s->nodes[id].count = 0;
  return id;
}

static int cmp_edge(const void* pa, const void* pb) {
  const int64_t* a = (const int64_t*)pa;
  const int64_t* b = (const int64_t*)pb;
  return (a[0] < b[0]) ? -1 : (a[0] > b[0]);
}

static void build_pseudonormals(orc_scene* s) {
  int64_t np = s->np, nv = s->nv;
  s->fnorm = (double*)calloc((size_t)np * 3, sizeof(double));
  s->vpn = (double*)calloc((size_t)nv * 3, sizeof(double));
  s->epn = (double*)calloc((size_t)np * 9, sizeof(double));
  for (int64_t t = 0; t < np; ++t) {
    const double* A = s->V + 3 * (int64_t)s->P[3 * t];
    const double* B = s->V + 3 * (int64_t)s->P[3 * t + 1];
    const double* C = s->V + 3 * (int64_t)s->P[3 * t + 2];
    double ab[3], ac[3], n[3];
    for (int a = 0; a < 3; ++a) {
      ab[a] = B[a] - A[a];
      ac[a] = C[a] - A[a];
    }
    cross3(ab, ac, n);
    double len = sqrt(dot3(n, n));
    for (int a = 0; a < 3; ++a) s->fnorm[3 * t + a] = n[a] / len;
    /* interior angle at each corner weights the vertex pseudonormal */
    const double* corner[3] = {A, B, C};
    for (int c = 0; c < 3; ++c) {
      const double* o = corner[c];
      const double* p1 = corner[(c + 1) % 3];
      const double* p2 = corner[(c + 2) % 3];
      double u[3], v[3];
      for (int a = 0; a < 3; ++a) {
        u[a] = p1[a] - o[a];
        v[a] = p2[a] - o[a];
      }
      double cang = dot3(u, v) / sqrt(dot3(u, u) * dot3(v, v));
      if (cang > 1) cang = 1;
      if (cang < -1) cang = -1;
      double ang = acos(cang);
      int64_t vi = s->P[3 * t + c];
      for (int a = 0; a < 3; ++a) s->vpn[3 * vi + a] += ang * s->fnorm[3 * t + a];
    }
  }
  /* unique edges: key = min*nv + max, with the triangle and local edge */
  int64_t m = 3 * np;
  int64_t* rec = (int64_t*)malloc((size_t)m * 3 * sizeof(int64_t));
  for (int64_t t = 0; t < np; ++t)
    for (int e = 0; e < 3; ++e) {
      int64_t a = s->P[3 * t + e], b = s->P[3 * t + (e + 1) % 3];
      int64_t lo = a < b ? a : b, hi = a < b ? b : a;
      rec[3 * (3 * t + e)] = lo * nv + hi;
      rec[3 * (3 * t + e) + 1] = t;
      rec[3 * (3 * t + e) + 2] = e;
    }
  qsort(rec, (size_t)m, 3 * sizeof(int64_t), cmp_edge);
  s->edges = (int32_t*)malloc((size_t)m * 2 * sizeof(int32_t));
  s->ne = 0;
  for (int64_t i = 0; i < m;) {
    int64_t j = i;
    double sum[3] = {0, 0, 0};
    while (j < m && rec[3 * j] == rec[3 * i]) {
      int64_t t = rec[3 * j + 1];
      for (int a = 0; a < 3; ++a) sum[a] += s->fnorm[3 * t + a];
      ++j;
    }
    for (int64_t q = i; q < j; ++q) {
      int64_t t = rec[3 * q + 1], e = rec[3 * q + 2];
      for (int a = 0; a < 3; ++a) s->epn[9 * t + 3 * e + a] = sum[a];
    }
    s->edges[2 * s->ne] = (int32_t)(rec[3 * i] / nv);
    s->edges[2 * s->ne + 1] = (int32_t)(rec[3 * i] % nv);
    s->ne++;
    i = j;
  }
  free(rec);
}

orc_scene* orc_scene_new(int dim, const double* verts, int64_t nv, const int32_t* prims,
                         int64_t np) {
  orc_scene* s = (orc_scene*)calloc(1, sizeof(orc_scene));
  s->dim = dim;
  s->nv = nv;
  s->np = np;
  s->V = (double*)malloc((size_t)nv * dim * sizeof(double));
  memcpy(s->V, verts, (size_t)nv * dim * sizeof(double));
  s->P = (int32_t*)malloc((size_t)np * dim * sizeof(int32_t));
  memcpy(s->P, prims, (size_t)np * dim * sizeof(int32_t));
  double* plo = (double*)malloc((size_t)np * dim * sizeof(double));
  double* phi = (double*)malloc((size_t)np * dim * sizeof(double));
  double* cen = (double*)malloc((size_t)np * dim * sizeof(double));
  for (int64_t p = 0; p < np; ++p) {
    double lo[3], hi[3], c[3];
    prim_bounds(s, p, lo, hi, c);
    for (int a = 0; a < dim; ++a) {
      plo[p * dim + a] = lo[a];
      phi[p * dim + a] = hi[a];
      cen[p * dim + a] = c[a];
    }
  }
  s->perm = (int32_t*)malloc((size_t)np * sizeof(int32_t));
  for (int64_t p = 0; p < np; ++p) s->perm[p] = (int32_t)p;
  s->nodes = (onode*)malloc((size_t)(2 * np + 1) * sizeof(onode));
  s->n_nodes = 0;
  build_node(s, plo, phi, cen, 0, np);
  free(plo);
  free(phi);
  free(cen);
  if (dim == 3) build_pseudonormals(s);
  return s;
}

void orc_scene_free(orc_scene* s) {
  if (!s) return;
  free(s->V);
  free(s->P);
  free(s->nodes);
  free(s->perm);
  free(s->fnorm);
  free(s->vpn);
  free(s->epn);
  free(s->edges);
  free(s);
}

/* Closest point on segment [a, b]; exact endpoints when the projection clamps. */
static double closest_segment(const double* x, const double* a, const double* b, double* c) {
  double e0 = b[0] - a[0], e1 = b[1] - a[1];
  double t = ((x[0] - a[0]) * e0 + (x[1] - a[1]) * e1) / (e0 * e0 + e1 * e1);
  if (t <= 0) {
    c[0] = a[0];
    c[1] = a[1];
  } else if (t >= 1) {
    c[0] = b[0];
    c[1] = b[1];
  } else {
    c[0] = a[0] + t * e0;
    c[1] = a[1] + t * e1;
  }
  double d0 = x[0] - c[0], d1 = x[1] - c[1];
  return d0 * d0 + d1 * d1;
}

/* Closest point on triangle (a, b, c) by Voronoi-region classification
 * (Ericson, Real-Time Collision Detection, Sec. 5.1.5).  region: 0 face,
 * 1/2/3 vertex a/b/c, 4/5/6 edge ab/bc/ca. */
static double closest_triangle(const double* p, const double* a, const double* b,
                               const double* c, double* q, int* region) {
  double ab[3], ac[3], ap[3], bp[3], cp[3];
  for (int i = 0; i < 3; ++i) {
    ab[i] = b[i] - a[i];
    ac[i] = c[i] - a[i];
    ap[i] = p[i] - a[i];
    bp[i] = p[i] - b[i];
    cp[i] = p[i] - c[i];
  }
  double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
  double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
  double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
  double vc = d1 * d4 - d3 * d2;
  double vb = d5 * d2 - d1 * d6;
  double va = d3 * d6 - d5 * d4;
  if (d1 <= 0 && d2 <= 0) {
    for (int i = 0; i < 3; ++i) q[i] = a[i];
    *region = 1;
  } else if (d3 >= 0 && d4 <= d3) {
    for (int i = 0; i < 3; ++i) q[i] = b[i];
    *region = 2;
  } else if (vc <= 0 && d1 >= 0 && d3 <= 0) {
    double v = d1 / (d1 - d3);
    for (int i = 0; i < 3; ++i) q[i] = a[i] + v * ab[i];
    *region = 4;
  } else if (d6 >= 0 && d5 <= d6) {
    for (int i = 0; i < 3; ++i) q[i] = c[i];
    *region = 3;
  } else if (vb <= 0 && d2 >= 0 && d6 <= 0) {
    double w = d2 / (d2 - d6);
    for (int i = 0; i < 3; ++i) q[i] = a[i] + w * ac[i];
    *region = 6;
  } else if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) {
    double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    for (int i = 0; i < 3; ++i) q[i] = b[i] + w * (c[i] - b[i]);
    *region = 5;
  } else {
    double den = 1.0 / (va + vb + vc);
    double v = vb * den, w = vc * den;
    for (int i = 0; i < 3; ++i) q[i] = a[i] + ab[i] * v + ac[i] * w;
    *region = 0;
  }
  double dd[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
  return dot3(dd, dd);
}

static double prim_dist2(const orc_scene* s, int64_t p, const double* x, double* c, int* region) {
  if (s->dim == 2) {
    *region = 0;
    return closest_segment(x, s->V + 2 * (int64_t)s->P[2 * p], s->V + 2 * (int64_t)s->P[2 * p + 1], c);
  }
  return closest_triangle(x, s->V + 3 * (int64_t)s->P[3 * p], s->V + 3 * (int64_t)s->P[3 * p + 1],
                          s->V + 3 * (int64_t)s->P[3 * p + 2], c, region);
}

static double box_dist2(const onode* n, const double* x, int dim) {
  double d2 = 0;
  for (int a = 0; a < dim; ++a) {
    double e = 0;
    if (x[a] < n->lo[a]) e = n->lo[a] - x[a];
    else if (x[a] > n->hi[a]) e = x[a] - n->hi[a];
    d2 += e * e;
  }
  return d2;
}

/* Update the best candidate with lexicographic (d^2, primitive id) order. */
static void consider(const orc_scene* s, int64_t p, const double* x, double* best, int64_t* bp,
                     double* bc, int* breg) {
  double c[3];
  int reg;
  double d2 = prim_dist2(s, p, x, c, &reg);
  if (d2 < *best || (d2 == *best && p < *bp)) {
    *best = d2;
    *bp = p;
    *breg = reg;
    for (int a = 0; a < s->dim; ++a) bc[a] = c[a];
  }
}

static void closest_full(const orc_scene* s, const double* x, int brute, double* d2out,
                         double* xbar, int64_t* prim, int* region) {
  double best = INFINITY;
  int64_t bp = -1;
  int breg = 0;
  double bc[3] = {0, 0, 0};
  if (brute) {
    for (int64_t p = 0; p < s->np; ++p) consider(s, p, x, &best, &bp, bc, &breg);
  } else {
    int64_t stack[128];
    double sd[128];
    int top = 0;
    stack[top] = 0;
    sd[top++] = box_dist2(&s->nodes[0], x, s->dim);
    while (top > 0) {
      --top;
      int64_t ni = stack[top];
      if (sd[top] > best) continue;
      const onode* nd = &s->nodes[ni];
      if (nd->left < 0) {
        for (int64_t i = nd->start; i < nd->start + nd->count; ++i)
          consider(s, s->perm[i], x, &best, &bp, bc, &breg);
        continue;
      }
      double dl = box_dist2(&s->nodes[nd->left], x, s->dim);
      double dr = box_dist2(&s->nodes[nd->right], x, s->dim);
      /* push the farther child first so the nearer one is visited next */
      if (dl <= dr) {
        stack[top] = nd->right;
        sd[top++] = dr;
        stack[top] = nd->left;
        sd[top++] = dl;
      } else {
        stack[top] = nd->left;
        sd[top++] = dl;
        stack[top] = nd->right;
        sd[top++] = dr;
      }
    }
  }
  *d2out = best;
  for (int a = 0; a < s->dim; ++a) xbar[a] = bc[a];
  *prim = bp;
  *region = breg;
}

void orc_closest(const orc_scene* s, const double* x, int brute, double* dist, double* xbar,
                 int32_t* prim) {
  double d2;
  int64_t p;
  int reg;
  closest_full(s, x, brute, &d2, xbar, &p, &reg);
  *dist = sqrt(d2);
  if (prim) *prim = (int32_t)p;
}

void orc_closest_batch(const orc_scene* s, int64_t n, const double* x, int brute, double* dist,
                       double* xbar, int32_t* prim) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i)
    orc_closest(s, x + i * s->dim, brute, dist + i, xbar + i * s->dim, prim ? prim + i : NULL);
}

/* Winding number of a closed polygon around x (edge-crossing rule). */
static int winding2d(const orc_scene* s, const double* x) {
  int wn = 0;
  for (int64_t p = 0; p < s->np; ++p) {
    const double* a = s->V + 2 * (int64_t)s->P[2 * p];
    const double* b = s->V + 2 * (int64_t)s->P[2 * p + 1];
    double side = (b[0] - a[0]) * (x[1] - a[1]) - (x[0] - a[0]) * (b[1] - a[1]);
    if (a[1] <= x[1]) {
      if (b[1] > x[1] && side > 0) ++wn;
    } else {
      if (b[1] <= x[1] && side < 0) --wn;
    }
  }
  return wn;
}

int orc_inside(const orc_scene* s, const double* x) {
  if (s->dim == 2) return winding2d(s, x);
  double d2, xb[3];
  int64_t p;
  int reg;
  closest_full(s, x, 0, &d2, xb, &p, &reg);
  const double* N;
  if (reg == 0) N = s->fnorm + 3 * p;
  else if (reg <= 3) N = s->vpn + 3 * (int64_t)s->P[3 * p + (reg - 1)];
  else N = s->epn + 9 * p + 3 * (reg - 4);
  double v[3] = {x[0] - xb[0], x[1] - xb[1], x[2] - xb[2]};
  return dot3(v, N) < 0 ? 1 : 0;
}

void orc_classify(const orc_scene* s, int64_t n, const double* x, double l, int32_t* cls) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    const double* xi = x + i * s->dim;
    if (orc_inside(s, xi) == 0) {
      cls[i] = 0;
      continue;
    }
    double d, xb[3];
    orc_closest(s, xi, 0, &d, xb, NULL);
    cls[i] = (d > l) ? 1 : 2;
  }
}

/* ======================================================================== */
/* Fields                                                                   */
/* ======================================================================== */
/* Ein(z) = int_0^z (1 - e^-t)/t dt.  Power series for small z; for larger z
 * Ein = E1(z) + ln z + gamma with E1 from its continued fraction evaluated by
 * the modified Lentz method (Abramowitz & Stegun 5.1.11 and 5.1.22). */
double orc_ein(double z) {
  const double euler_gamma = 0.57721566490153286061;
  if (z <= 0) return 0;
  if (z < 2.0) {
    double sum = 0, pw = 1, fact = 1;
    for (int k = 1; k < 60; ++k) {
      pw *= z;
      fact *= k;
      double term = pw / (k * fact);
      sum += (k % 2 == 1) ? term : -term;
      if (term < 1e-18 * fabs(sum)) break;
    }
    return sum;
  }
  const double tiny = 1e-300;
  double bcoef = z + 1.0;
  double cf = 1.0 / tiny;
  double df = 1.0 / bcoef;
  double h = df;
  for (int i = 1; i < 500; ++i) {
    double acoef = -(double)i * (double)i;
    bcoef += 2.0;
    df = 1.0 / (acoef * df + bcoef);
    cf = bcoef + acoef / cf;
    double delta = cf * df;
    h *= delta;
    if (fabs(delta - 1.0) < 1e-16) break;
  }
  return h * exp(-z) + log(z) + euler_gamma;
}

static double harmonic2d(double k, double alpha, double beta, const double* x) {
  int kk = (int)k;
  double re = 1, im = 0;
  for (int i = 0; i < kk; ++i) {
    double nre = re * x[0] - im * x[1];
    double nim = re * x[1] + im * x[0];
    re = nre;
    im = nim;
  }
  return alpha * re + beta * exp(x[0]) * cos(x[1]);
}

/* Orthonormal real solid harmonic r^l Y_lm (no Condon-Shortley phase), via
 * the associated Legendre recurrences in cos(theta). */
static double solid_harmonic(int l, int m, const double* x) {
  double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  int am = m < 0 ? -m : m;
  if (r == 0) return (l == 0) ? 0.5 / sqrt(ORC_PI) : 0.0;
  double ct = x[2] / r;
  double st = sqrt(fmax(0.0, 1 - ct * ct));
  double phi = atan2(x[1], x[0]);
  double pmm = 1;
  for (int i = 1; i <= am; ++i) pmm *= (2 * i - 1) * st;
  double plm = pmm, p1 = 0, p2 = 0;
  for (int ll = am; ll <= l; ++ll) {
    if (ll == am) plm = pmm;
    else if (ll == am + 1) plm = ct * (2 * am + 1) * pmm;
    else plm = (ct * (2 * ll - 1) * p1 - (ll + am - 1) * p2) / (ll - am);
    p2 = p1;
    p1 = plm;
  }
  double ratio = 1; /* (l-|m|)! / (l+|m|)! */
  for (int i = l - am + 1; i <= l + am; ++i) ratio /= i;
  double nrm = sqrt((2 * l + 1) / (4 * ORC_PI) * ratio);
  double ang = 1;
  if (m > 0) ang = sqrt(2.0) * cos(m * phi);
  if (m < 0) ang = sqrt(2.0) * sin(am * phi);
  return pow(r, l) * nrm * plm * ang;
}

static double fourier_phi(int b, double th) {
  if (b == 0) return 1.0;
  int j = (b + 1) / 2;
  return (b % 2 == 1) ? cos(j * th) : sin(j * th);
}

double orc_basis_eval(const orc_field* F, int dim, int m, const double* x) {
  switch (F->kind) {
    case ORC_FIELD_FOURIER_2D:
      return fourier_phi(m, atan2(x[1] - F->param[1], x[0] - F->param[0]));
    case ORC_FIELD_SOLID_HARMONICS_3D: {
      int l = 0;
      while ((l + 1) * (l + 1) <= m) ++l;
      return solid_harmonic(l, m - l * l - l, x);
    }
    case ORC_FIELD_GAUSS_SUM: {
      const double* c = F->coef + m * (1 + dim);
      double r2 = 0;
      for (int a = 0; a < dim; ++a) r2 += (x[a] - c[1 + a]) * (x[a] - c[1 + a]);
      return exp(-r2 / (2 * F->param[0] * F->param[0]));
    }
    default:
      return 0.0;
  }
}

double orc_field_eval(const orc_field* F, int dim, const double* x) {
  if (!F) return 0.0;
  const double* p = F->param;
  switch (F->kind) {
    case ORC_FIELD_ZERO:
      return 0.0;
    case ORC_FIELD_CONST:
      return p[0];
    case ORC_FIELD_HARMONIC_2D:
      return harmonic2d(p[0], p[1], p[2], x);
    case ORC_FIELD_GAUSS_SUM: {
      int ng = F->n_coef / (1 + dim);
      double sum = 0;
      for (int k = 0; k < ng; ++k) sum += F->coef[k * (1 + dim)] * orc_basis_eval(F, dim, k, x);
      return sum;
    }
    case ORC_FIELD_GAUSS_POTENTIAL_2D: {
      int ng = F->n_coef / 3;
      double s = p[0], sum = 0;
      for (int k = 0; k < ng; ++k) {
        const double* c = F->coef + 3 * k;
        double r2 = (x[0] - c[1]) * (x[0] - c[1]) + (x[1] - c[2]) * (x[1] - c[2]);
        sum += c[0] * s * s / 2 * orc_ein(r2 / (2 * s * s));
      }
      return sum + harmonic2d(p[1], p[2], p[3], x);
    }
    case ORC_FIELD_SOLID_HARMONICS_3D:
    case ORC_FIELD_FOURIER_2D: {
      double sum = 0;
      for (int m = 0; m < F->n_coef; ++m) sum += F->coef[m] * orc_basis_eval(F, dim, m, x);
      return sum;
    }
    case ORC_FIELD_POINT_SOURCE: {
      double r2 = 0;
      for (int a = 0; a < dim; ++a) r2 += (x[a] - p[1 + a]) * (x[a] - p[1 + a]);
      return dim == 2 ? p[0] * 0.5 * log(r2) : p[0] / sqrt(r2);
    }
    case ORC_FIELD_EXP_PLANE: {
      double e = 0;
      for (int a = 0; a < dim; ++a) e += p[1 + a] * x[a];
      return p[0] * exp(e);
    }
    case ORC_FIELD_WEDGE_2D: {
      double dx = x[0] - p[2], dy = x[1] - p[3];
      double phi = atan2(dy, dx);
      if (phi < 0) phi += 2 * ORC_PI;
      return p[0] * pow(hypot(dx, dy), p[1]) * cos(p[1] * phi);
    }
    case ORC_FIELD_QUADRATIC: {
      double r2 = 0;
      for (int a = 0; a < dim; ++a) r2 += (x[a] - p[2 + a]) * (x[a] - p[2 + a]);
      return p[0] * r2 + p[1];
    }
  }
  return 0.0;
}

void orc_field_eval_batch(const orc_field* F, int dim, int64_t n, const double* x, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = orc_field_eval(F, dim, x + i * dim);
}

/* ======================================================================== */
/* Green's functions of the Laplacian (Appendix A.1, with G_3D = -1/(4 pi r)) */
/* ======================================================================== */
void orc_greens(int dim, const double* x, const double* y, const double* ny, double* G,
                double* dGdx, double* dGdn, double* d2Gdxdn) {
  double yx[3] = {0, 0, 0}; /* y - x */
  double r2 = 0;
  for (int a = 0; a < dim; ++a) {
    yx[a] = y[a] - x[a];
    r2 += yx[a] * yx[a];
  }
  double r = sqrt(r2);
  double ndot = 0;
  if (ny)
    for (int a = 0; a < dim; ++a) ndot += ny[a] * yx[a];
  if (dim == 2) {
    double c = 1.0 / (2 * ORC_PI);
    if (G) *G = c * log(r);
    if (dGdx)
      for (int a = 0; a < 2; ++a) dGdx[a] = c * (-yx[a]) / r2;
    if (dGdn) *dGdn = c * ndot / r2;
    if (d2Gdxdn)
      for (int a = 0; a < 2; ++a) d2Gdxdn[a] = c * (2 * ndot * yx[a] / (r2 * r2) - ny[a] / r2);
  } else {
    double c = 1.0 / (4 * ORC_PI);
    double r3 = r2 * r;
    if (G) *G = -c / r;
    if (dGdx)
      for (int a = 0; a < 3; ++a) dGdx[a] = c * (-yx[a]) / r3;
    if (dGdn) *dGdn = c * ndot / r3;
    if (d2Gdxdn)
      for (int a = 0; a < 3; ++a) d2Gdxdn[a] = c * (3 * ndot * yx[a] / (r3 * r2) - ny[a] / r3);
  }
}

/* ======================================================================== */
/* Screened Poisson (Eq. 1 with sigma > 0; Appendix A.2)                     */
/* ======================================================================== */
/* I_n(x) = sum_k (x/2)^(2k+n) / (k! (k+n)!) for moderate x; beyond, the
 * integral (1/pi) int_0^pi e^(x cos t) cos(n t) dt by the trapezoid rule,
 * which is exponentially accurate for this periodic integrand. */
static double bessel_i(int n, double x) {
  x = fabs(x);
  if (x <= 20.0) {
    double h = 0.5 * x, term = n ? h : 1.0, sum = term;
    for (int k = 1; k < 200; ++k) {
      term *= h * h / ((double)k * (double)(k + n));
      sum += term;
      if (term < 1e-18 * sum) break;
    }
    return sum;
  }
  int N = (int)(2 * x + 40);
  double sum = 0;
  for (int j = 0; j <= N; ++j) {
    double t = ORC_PI * j / N;
    double f = exp(x * cos(t)) * cos(n * t);
    sum += (j == 0 || j == N) ? 0.5 * f : f;
  }
  return sum / N;
}
/* K_n(x) = int_0^inf e^(-x cosh t) cosh(n t) dt by the trapezoid rule, which
 * is exponentially accurate for this even, analytic integrand; the step
 * follows the width of its peak at t = 0 (about 1/sqrt(x) for large x). */
static double bessel_k(int n, double x) {
  double h = 0.1 / fmax(1.0, sqrt(x) / 3.0);
  double tmax = acosh(fmax(750.0 / x, 1.0)) + 1.0;
  double sum = 0.5 * exp(-x);
  for (int j = 1;; ++j) {
    double t = h * j;
    if (t > tmax) break;
    sum += exp(-x * cosh(t)) * cosh(n * t);
  }
  return h * sum;
}
double orc_bessel_i0(double x) { return bessel_i(0, x); }
double orc_bessel_i1(double x) { return bessel_i(1, x); }
double orc_bessel_k0(double x) { return bessel_k(0, x); }
double orc_bessel_k1(double x) { return bessel_k(1, x); }

void orc_greens_sigma(int dim, double sigma, const double* x, const double* y, const double* ny,
                      double* G, double* dGdx, double* dGdn, double* d2Gdxdn) {
  if (!(sigma > 0)) {
    orc_greens(dim, x, y, ny, G, dGdx, dGdn, d2Gdxdn);
    return;
  }
  /* G^s = -K0(sr)/(2pi) (2D), -e^(-sr)/(4 pi r) (3D); the derivatives are the
   * Poisson ones times Q (Appendix A.2): Q = sr K1(sr) (2D),
   * e^(-sr)(1 + sr) (3D), and dQ/dx = s^2 K0(sr)(y - x) (2D),
   * s^2 e^(-sr)(y - x) (3D). */
  double G0, g0[3], n0 = 0, d0[3];
  orc_greens(dim, x, y, ny, &G0, g0, ny ? &n0 : NULL, ny ? d0 : NULL);
  double yx[3] = {0, 0, 0}, r2 = 0;
  for (int a = 0; a < dim; ++a) {
    yx[a] = y[a] - x[a];
    r2 += yx[a] * yx[a];
  }
  double r = sqrt(r2), s = sqrt(sigma), sr = s * r;
  double Q, dq; /* dQ/dx = dq (y - x) */
  if (dim == 2) {
    double k0 = bessel_k(0, sr), k1 = bessel_k(1, sr);
    if (G) *G = -k0 / (2 * ORC_PI);
    Q = sr * k1;
    dq = sigma * k0;
  } else {
    double e = exp(-sr);
    if (G) *G = -e / (4 * ORC_PI * r);
    Q = e * (1 + sr);
    dq = sigma * e;
  }
  if (dGdx)
    for (int a = 0; a < dim; ++a) dGdx[a] = Q * g0[a];
  if (dGdn) *dGdn = Q * n0;
  if (d2Gdxdn)
    for (int a = 0; a < dim; ++a) d2Gdxdn[a] = Q * d0[a] + n0 * dq * yx[a];
}

/* i1(x) = (x cosh x - sinh x)/x^2, the modified spherical Bessel function of
 * order 1, by its series sum_k x^(2k+1) / (2^k k! (2k+3)!!) below 1. */
static double sph_i1(double x) {
  if (x < 1.0) {
    double term = x / 3.0, sum = term;
    for (int k = 1; k < 30; ++k) {
      term *= x * x / (2.0 * k * (2.0 * k + 3.0));
      sum += term;
    }
    return sum;
  }
  return (x * cosh(x) - sinh(x)) / (x * x);
}

double orc_screen_ball_weight(int dim, double sigma, double R) {
  if (!(sigma > 0)) return 1.0;
  double x = sqrt(sigma) * R;
  if (dim == 2) return 1.0 / bessel_i(0, x);
  return x < 1e-8 ? 1.0 : x / sinh(x);
}

double orc_screen_grad_weight(int dim, double sigma, double R) {
  if (!(sigma > 0)) return dim / R;
  double s = sqrt(sigma), x = s * R;
  if (dim == 2) return s / bessel_i(1, x);
  return s / sph_i1(x);
}

/* The in-ball source term of the screened equation (Eq. 1 with sigma > 0 and
 * f != 0).  Ball B(c, R), point y at r = t R from c.  The screened ball
 * Green's function (zero on the sphere, for -Lap + sigma) is
 *   2D  [K0(s r) - K0(s R) I0(s r) / I0(s R)] / (2 pi),
 *   3D  sinh(s (R - r)) / (4 pi r sinh(s R)),           s = sqrt(sigma),
 * and the walks sample y from the Laplace one, ln(R/r)/(2 pi) or
 * (1/r - 1/R)/(4 pi); this is the ratio of the two, in (0, 1].  It tends to 1
 * as sigma -> 0. */
double orc_screen_source_ratio(int dim, double sigma, double R, double t) {
  if (!(sigma > 0)) return 1.0;
  double s = sqrt(sigma), r = t * R;
  if (dim == 2) {
    double num = orc_bessel_k0(s * r) - orc_bessel_k0(s * R) * bessel_i(0, s * r) / bessel_i(0, s * R);
    return num / -log(t);
  }
  double z = s * R * (1 - t);
  double shz = z < 1e-8 ? 1.0 : sinh(z) / z; /* sinh(z)/z */
  return s * R * shz / sinh(s * R);
}

/* The same ratio for the gradient of the in-ball source term at the centre
 * (the first ball of Eq. 7): the centre gradient of the screened ball
 * Green's function points along y - c with magnitude
 *   2D  s [K1(s r) - I1(s r) K1(s R) / I1(s R)] / (2 pi),
 *   3D  [e^(-s r)(1 + s r)/r^2 - e^(-s R)(1 + s R)/R^2 i1(s r)/i1(s R)] / (4 pi)
 * (the free-space kernel's radial derivative minus the order-1 mode of the
 * part that cancels it on the sphere), against the Laplace magnitudes
 * (1/r - r/R^2)/(2 pi) and (1/r^2 - r/R^3)/(4 pi). */
double orc_screen_grad_source_ratio(int dim, double sigma, double R, double t) {
  if (!(sigma > 0)) return 1.0;
  double s = sqrt(sigma), r = t * R;
  if (dim == 2) {
    double num = s * (orc_bessel_k1(s * r) - bessel_i(1, s * r) * orc_bessel_k1(s * R) / bessel_i(1, s * R));
    return num / (1 / r - r / (R * R));
  }
  double num = exp(-s * r) * (1 + s * r) - exp(-s * R) * (1 + s * R) * t * t * sph_i1(s * r) / sph_i1(s * R);
  return num / (1 - t * t * t);
}

void orc_gather_sigma(int dim, double sigma, int64_t K, const double* ex, int64_t N, const double* cy,
                      const double* cn, const double* a, const double* b, int64_t M, const double* sy,
                      const double* sw, double* u, double* grad, double* cond) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < K; ++k) {
    const double* x = ex + k * dim;
    double uk = 0, ck = 0, gk[3] = {0, 0, 0};
    for (int64_t i = 0; i < N; ++i) {
      double G, dGdx[3], dGdn, d2[3];
      orc_greens_sigma(dim, sigma, x, cy + i * dim, cn + i * dim, &G, dGdx, &dGdn, d2);
      uk += dGdn * a[i] - G * b[i];
      ck += fabs(dGdn * a[i]) + fabs(G * b[i]);
      for (int q = 0; q < dim; ++q) gk[q] += d2[q] * a[i] - dGdx[q] * b[i];
    }
    for (int64_t j = 0; j < M; ++j) {
      double G, dGdx[3];
      orc_greens_sigma(dim, sigma, x, sy + j * dim, NULL, &G, dGdx, NULL, NULL);
      uk += G * sw[j];
      ck += fabs(G * sw[j]);
      for (int q = 0; q < dim; ++q) gk[q] += dGdx[q] * sw[j];
    }
    u[k] = uk;
    if (cond) cond[k] = ck;
    if (grad)
      for (int q = 0; q < dim; ++q) grad[k * dim + q] = gk[q];
  }
}

/* ======================================================================== */
/* Cache sampling on the offset boundary                                    */
/* ======================================================================== */
typedef struct {
  int64_t n_el;
  int32_t* kind;  /* 0 segment/face offset, 1 vertex circle/sphere, 2 edge cylinder */
  int32_t* idx;   /* primitive, vertex or edge index */
  int32_t* side;  /* +1 inward (left of a CCW segment, against the face normal), -1 outward */
  double* meas;
  double* cdf;    /* n_el + 1 */
} elem_table;

static void make_elements(const orc_scene* s, double l, int sides, elem_table* T) {
  int d = s->dim;
  int64_t n = (d == 2) ? s->np * sides + s->nv : s->np + s->ne + s->nv;
  T->n_el = n;
  T->kind = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  T->idx = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  T->side = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  T->meas = (double*)malloc((size_t)n * sizeof(double));
  T->cdf = (double*)malloc((size_t)(n + 1) * sizeof(double));
  int64_t e = 0;
  if (d == 2) {
    for (int64_t p = 0; p < s->np; ++p) {
      const double* a = s->V + 2 * (int64_t)s->P[2 * p];
      const double* b = s->V + 2 * (int64_t)s->P[2 * p + 1];
      double len = sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]));
      for (int sd = 0; sd < sides; ++sd) {
        T->kind[e] = 0;
        T->idx[e] = (int32_t)p;
        T->side[e] = sd == 0 ? 1 : -1;
        T->meas[e] = len;
        ++e;
      }
    }
    for (int64_t v = 0; v < s->nv; ++v) {
      T->kind[e] = 1;
      T->idx[e] = (int32_t)v;
      T->side[e] = 0;
      T->meas[e] = 2 * ORC_PI * l;
      ++e;
    }
  } else {
    for (int64_t p = 0; p < s->np; ++p) {
      const double* A = s->V + 3 * (int64_t)s->P[3 * p];
      const double* B = s->V + 3 * (int64_t)s->P[3 * p + 1];
      const double* C = s->V + 3 * (int64_t)s->P[3 * p + 2];
      double ab[3], ac[3], c[3];
      for (int a = 0; a < 3; ++a) {
        ab[a] = B[a] - A[a];
        ac[a] = C[a] - A[a];
      }
      cross3(ab, ac, c);
      T->kind[e] = 0;
      T->idx[e] = (int32_t)p;
      T->side[e] = 1;
      T->meas[e] = 0.5 * sqrt(dot3(c, c));
      ++e;
    }
    for (int64_t q = 0; q < s->ne; ++q) {
      const double* A = s->V + 3 * (int64_t)s->edges[2 * q];
      const double* B = s->V + 3 * (int64_t)s->edges[2 * q + 1];
      double ab[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
      T->kind[e] = 2;
      T->idx[e] = (int32_t)q;
      T->side[e] = 0;
      T->meas[e] = 2 * ORC_PI * l * sqrt(dot3(ab, ab));
      ++e;
    }
    for (int64_t v = 0; v < s->nv; ++v) {
      T->kind[e] = 1;
      T->idx[e] = (int32_t)v;
      T->side[e] = 0;
      T->meas[e] = 4 * ORC_PI * l * l;
      ++e;
    }
  }
  T->cdf[0] = 0;
  for (int64_t i = 0; i < n; ++i) T->cdf[i + 1] = T->cdf[i] + T->meas[i];
}

static void free_elements(elem_table* T) {
  free(T->kind);
  free(T->idx);
  free(T->side);
  free(T->meas);
  free(T->cdf);
}

double orc_candidate_measure(const orc_scene* s, double l, int sides) {
  elem_table T;
  make_elements(s, l, sides, &T);
  double m = T.cdf[T.n_el];
  free_elements(&T);
  return m;
}

/* Candidate point of element e at stratified residual r and second uniform v. */
static void candidate_point(const orc_scene* s, const elem_table* T, int64_t e, double r,
                            double v, double l, double* x) {
  int d = s->dim;
  int32_t k = T->kind[e], i = T->idx[e];
  if (d == 2) {
    if (k == 0) {
      const double* a = s->V + 2 * (int64_t)s->P[2 * i];
      const double* b = s->V + 2 * (int64_t)s->P[2 * i + 1];
      double t0 = b[0] - a[0], t1 = b[1] - a[1];
      double len = sqrt(t0 * t0 + t1 * t1);
      double n0 = t1 / len, n1 = -t0 / len; /* outward normal of a CCW polygon */
      double q0 = a[0] + r * t0, q1 = a[1] + r * t1;
      x[0] = q0 - T->side[e] * l * n0;
      x[1] = q1 - T->side[e] * l * n1;
    } else {
      const double* c = s->V + 2 * (int64_t)i;
      double ang = 2 * ORC_PI * r;
      x[0] = c[0] + l * cos(ang);
      x[1] = c[1] + l * sin(ang);
    }
    return;
  }
  if (k == 0) {
    const double* A = s->V + 3 * (int64_t)s->P[3 * i];
    const double* B = s->V + 3 * (int64_t)s->P[3 * i + 1];
    const double* C = s->V + 3 * (int64_t)s->P[3 * i + 2];
    double su = sqrt(r);
    double b0 = 1 - su, b1 = su * (1 - v), b2 = su * v;
    double ab[3], ac[3], nn[3];
    for (int a = 0; a < 3; ++a) {
      ab[a] = B[a] - A[a];
      ac[a] = C[a] - A[a];
    }
    cross3(ab, ac, nn);
    double len = sqrt(dot3(nn, nn));
    for (int a = 0; a < 3; ++a) x[a] = b0 * A[a] + b1 * B[a] + b2 * C[a] - l * nn[a] / len;
  } else if (k == 2) {
    const double* A = s->V + 3 * (int64_t)s->edges[2 * i];
    const double* B = s->V + 3 * (int64_t)s->edges[2 * i + 1];
    double t[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    double len = sqrt(dot3(t, t));
    for (int a = 0; a < 3; ++a) t[a] /= len;
    /* frame: helper axis with the smallest |t| component (first on ties) */
    int ax = 0;
    for (int a = 1; a < 3; ++a)
      if (fabs(t[a]) < fabs(t[ax])) ax = a;
    double h[3] = {0, 0, 0};
    h[ax] = 1;
    double e1[3], e2[3];
    cross3(t, h, e1);
    double l1 = sqrt(dot3(e1, e1));
    for (int a = 0; a < 3; ++a) e1[a] /= l1;
    cross3(t, e1, e2);
    double ang = 2 * ORC_PI * v;
    double ca = cos(ang), sa = sin(ang);
    for (int a = 0; a < 3; ++a) x[a] = A[a] + r * (B[a] - A[a]) + l * (ca * e1[a] + sa * e2[a]);
  } else {
    const double* c = s->V + 3 * (int64_t)i;
    double z = 1 - 2 * r;
    double rho = sqrt(fmax(0.0, 1 - z * z));
    double ang = 2 * ORC_PI * v;
    x[0] = c[0] + l * rho * cos(ang);
    x[1] = c[1] + l * rho * sin(ang);
    x[2] = c[2] + l * z;
  }
}

int64_t orc_sample_cache(const orc_scene* s, int64_t n, double l, int sides, uint64_t seed,
                         uint32_t batch, double* x, double* nrm, double* w, double* xbar,
                         double* R0, int32_t* accept) {
  int d = s->dim;
  elem_table T;
  make_elements(s, l, sides, &T);
  double M = T.cdf[T.n_el];
  int64_t n_acc = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : n_acc)
  for (int64_t k = 0; k < n; ++k) {
    double ua, ub;
    orc_uniform_pair(seed, 0, (uint32_t)k, batch, 3, &ua, &ub);
    double target = ((double)k + ua) / (double)n * M;
    /* largest e with cdf[e] <= target */
    int64_t lo = 0, hi = T.n_el - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi + 1) / 2;
      if (T.cdf[mid] <= target) lo = mid;
      else hi = mid - 1;
    }
    int64_t e = lo;
    double r = (target - T.cdf[e]) / T.meas[e];
    if (r < 0) r = 0;
    if (r > 1) r = 1;
    double* xk = x + k * d;
    candidate_point(s, &T, e, r, ub, l, xk);
    double dist, xb[3];
    orc_closest(s, xk, 0, &dist, xb, NULL);
    int ok = (dist >= l * (1 - 1e-9)) && (orc_inside(s, xk) != 0);
    accept[k] = ok;
    n_acc += ok;
    R0[k] = dist;
    w[k] = M / (double)n;
    for (int a = 0; a < d; ++a) {
      xbar[k * d + a] = xb[a];
      nrm[k * d + a] = (xb[a] - xk[a]) / dist;
    }
  }
  free_elements(&T);
  return n_acc;
}

/* Cache points on the boundary of a region of interest R inside the domain
 * (Section 3.2, "Boundary Specification"): uniform density 1/|dR| over the
 * primitives of the closed boundary `roi` (stratified uniforms through the
 * cumulative primitive measures, Philox tag 6), the unit outward normal of R
 * (the primitive's own: CCW segments, outward-wound triangles), weight
 * |dR|/n, and the distance and closest point on the domain boundary `dom`
 * where the walks run.  A point is accepted when it lies strictly inside the
 * domain.  Returns the number accepted. */
int64_t orc_sample_roi(const orc_scene* dom, const orc_scene* roi, int64_t n, uint64_t seed, uint32_t batch,
                       double* x, double* nrm, double* w, double* xbar, double* R0, int32_t* accept) {
  int d = roi->dim;
  int64_t np = roi->np;
  double* cdf = (double*)malloc((size_t)(np + 1) * sizeof(double));
  cdf[0] = 0;
  for (int64_t p = 0; p < np; ++p) {
    double m;
    if (d == 2) {
      const double* a = roi->V + 2 * (int64_t)roi->P[2 * p];
      const double* b = roi->V + 2 * (int64_t)roi->P[2 * p + 1];
      m = sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]));
    } else {
      const double* A = roi->V + 3 * (int64_t)roi->P[3 * p];
      const double* B = roi->V + 3 * (int64_t)roi->P[3 * p + 1];
      const double* C = roi->V + 3 * (int64_t)roi->P[3 * p + 2];
      double ab[3], ac[3], c[3];
      for (int a = 0; a < 3; ++a) {
        ab[a] = B[a] - A[a];
        ac[a] = C[a] - A[a];
      }
      cross3(ab, ac, c);
      m = 0.5 * sqrt(dot3(c, c));
    }
    cdf[p + 1] = cdf[p] + m;
  }
  double M = cdf[np];
  int64_t n_acc = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : n_acc)
  for (int64_t k = 0; k < n; ++k) {
    double ua, ub;
    orc_uniform_pair(seed, 0, (uint32_t)k, batch, 6, &ua, &ub);
    double target = ((double)k + ua) / (double)n * M;
    int64_t lo = 0, hi = np - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi + 1) / 2;
      if (cdf[mid] <= target) lo = mid;
      else hi = mid - 1;
    }
    double r = (target - cdf[lo]) / (cdf[lo + 1] - cdf[lo]);
    if (r < 0) r = 0;
    if (r > 1) r = 1;
    double* xk = x + k * d;
    double* nk = nrm + k * d;
    if (d == 2) {
      const double* a = roi->V + 2 * (int64_t)roi->P[2 * lo];
      const double* b = roi->V + 2 * (int64_t)roi->P[2 * lo + 1];
      double t0 = b[0] - a[0], t1 = b[1] - a[1];
      double len = sqrt(t0 * t0 + t1 * t1);
      xk[0] = a[0] + r * t0;
      xk[1] = a[1] + r * t1;
      nk[0] = t1 / len;
      nk[1] = -t0 / len;
    } else {
      const double* A = roi->V + 3 * (int64_t)roi->P[3 * lo];
      const double* B = roi->V + 3 * (int64_t)roi->P[3 * lo + 1];
      const double* C = roi->V + 3 * (int64_t)roi->P[3 * lo + 2];
      double su = sqrt(r);
      double b0 = 1 - su, b1 = su * (1 - ub), b2 = su * ub;
      double ab[3], ac[3], c[3];
      for (int a = 0; a < 3; ++a) {
        ab[a] = B[a] - A[a];
        ac[a] = C[a] - A[a];
        xk[a] = b0 * A[a] + b1 * B[a] + b2 * C[a];
      }
      cross3(ab, ac, c);
      double len = sqrt(dot3(c, c));
      for (int a = 0; a < 3; ++a) nk[a] = c[a] / len;
    }
    double dist, xb[3];
    orc_closest(dom, xk, 0, &dist, xb, NULL);
    int ok = dist > 0 && orc_inside(dom, xk) != 0;
    accept[k] = ok;
    n_acc += ok;
    R0[k] = dist;
    w[k] = M / (double)n;
    for (int a = 0; a < d; ++a) xbar[k * d + a] = xb[a];
  }
  free(cdf);
  return n_acc;
}

void orc_sample_sources(const orc_scene* s, const orc_field* f, int64_t m, const double* lo,
                        const double* hi, double l, uint64_t seed, uint32_t batch, double* y,
                        double* sw) {
  int d = s->dim;
  int64_t M = 1;
  double vol = 1;
  for (int a = 0; a < d; ++a) {
    M *= m;
    vol *= hi[a] - lo[a];
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t j = 0; j < M; ++j) {
    double u[4];
    orc_uniform_pair(seed, 0, (uint32_t)j, batch, 4, &u[0], &u[1]);
    orc_uniform_pair(seed, 1, (uint32_t)j, batch, 4, &u[2], &u[3]);
    int64_t rem = j;
    double* yj = y + j * d;
    for (int a = 0; a < d; ++a) {
      int64_t c = rem % m;
      rem /= m;
      yj[a] = lo[a] + ((double)c + u[a]) / (double)m * (hi[a] - lo[a]);
    }
    double dist, xb[3];
    orc_closest(s, yj, 0, &dist, xb, NULL);
    int in = orc_inside(s, yj) != 0 && dist > l;
    sw[j] = in ? vol / (double)M * orc_field_eval(f, d, yj) : 0.0;
  }
}

/* ======================================================================== */
/* Walk on spheres with the ball gradient estimator                          */
/* ======================================================================== */
/* Uniform direction from step k's block 4k. */
static void walk_direction(uint64_t seed, uint32_t k, uint32_t id, uint32_t batch, uint32_t tag,
                           int dim, double* nu) {
  double ua, ub;
  orc_uniform_pair(seed, 4 * k, id, batch, tag, &ua, &ub);
  if (dim == 2) {
    double th = 2 * ORC_PI * ua;
    nu[0] = cos(th);
    nu[1] = sin(th);
  } else {
    double z = 1 - 2 * ua;
    double rho = sqrt(fmax(0.0, 1 - z * z));
    double ph = 2 * ORC_PI * ub;
    nu[0] = rho * cos(ph);
    nu[1] = rho * sin(ph);
    nu[2] = z;
  }
}

/* Point of a ball B(c, R) drawn with density proportional to |G^B(c, .)|:
 * radius fraction sqrt(U1 U2) in 2D (density 4 s ln(1/s)), median of three
 * uniforms in 3D (density 6 s (1-s)); direction uniform.  Blocks 4k+1..4k+3. */
static double ball_source_point(uint64_t seed, uint32_t k, uint32_t id, uint32_t batch,
                                uint32_t tag, int dim, const double* c, double R, double* y) {
  double u1, u2, u3, u4, u5, u6;
  orc_uniform_pair(seed, 4 * k + 1, id, batch, tag, &u1, &u2);
  orc_uniform_pair(seed, 4 * k + 2, id, batch, tag, &u3, &u4);
  if (dim == 2) {
    double s = sqrt(u1 * u2);
    double th = 2 * ORC_PI * u3;
    y[0] = c[0] + R * s * cos(th);
    y[1] = c[1] + R * s * sin(th);
    return s;
  }
  double lo = u1 < u2 ? u1 : u2, hi = u1 < u2 ? u2 : u1;
  double s = u3 < lo ? lo : (u3 > hi ? hi : u3);
  orc_uniform_pair(seed, 4 * k + 3, id, batch, tag, &u5, &u6);
  double z = 1 - 2 * u5;
  double rho = sqrt(fmax(0.0, 1 - z * z));
  double ph = 2 * ORC_PI * u6;
  y[0] = c[0] + R * s * rho * cos(ph);
  y[1] = c[1] + R * s * rho * sin(ph);
  y[2] = c[2] + R * s * z;
  return s;
}

/* The gradient source sample of the first ball (Eq. 7 with a source): the
 * centre gradient of the in-ball source term, minus the integral of
 * grad_x G^B(c, y) f(y), is E[-m(t) R y_hat f(y)] with y = c + t R y_hat:
 *   2D  t from the density (3/2)(1 - t^2), m = 2/3 (the Laplace magnitude
 *       integrates to 2R/3 over the disk), y_hat at angle 2 pi U3;
 *   3D  t uniform, m = 1 - t^3 (the magnitude's radial density (4/3)(1 - t^3)
 *       times its integral 3R/4), y_hat uniform on the sphere.
 * Uniforms: 2D the second of block 2 and the first of block 3 (tag); 3D
 * block 0 (direction) and the first of block 1 under tag | 128.  Returns t;
 * *m receives the weight. */
static double grad_source_point(uint64_t seed, uint32_t id, uint32_t batch, uint32_t tag, int dim,
                                const double* c, double R, double* yhat, double* y, double* m) {
  if (dim == 2) {
    double u1, u2, u3, u4;
    orc_uniform_pair(seed, 2, id, batch, tag, &u1, &u2);
    orc_uniform_pair(seed, 3, id, batch, tag, &u3, &u4);
    double t = 2 * sin(asin(u2) / 3);
    double th = 2 * ORC_PI * u3;
    yhat[0] = cos(th);
    yhat[1] = sin(th);
    y[0] = c[0] + R * t * yhat[0];
    y[1] = c[1] + R * t * yhat[1];
    *m = 2.0 / 3.0;
    return t;
  }
  double a, b, t, w;
  orc_uniform_pair(seed, 0, id, batch, tag | 128u, &a, &b);
  orc_uniform_pair(seed, 1, id, batch, tag | 128u, &t, &w);
  double z = 1 - 2 * a;
  double rho = sqrt(fmax(0.0, 1 - z * z));
  double ph = 2 * ORC_PI * b;
  yhat[0] = rho * cos(ph);
  yhat[1] = rho * sin(ph);
  yhat[2] = z;
  for (int q = 0; q < 3; ++q) y[q] = c[q] + R * t * yhat[q];
  *m = 1 - t * t * t;
  return t;
}

/* Exported views of the two samplers above, for the density tests. */
void orc_sample_direction(uint64_t seed, uint32_t k, uint32_t id, uint32_t batch, uint32_t tag,
                          int dim, double* nu) {
  walk_direction(seed, k, id, batch, tag, dim, nu);
}
double orc_sample_grad_source(uint64_t seed, uint32_t id, uint32_t batch, uint32_t tag, int dim,
                              const double* c, double R, double* yhat, double* y, double* m) {
  return grad_source_point(seed, id, batch, tag, dim, c, R, yhat, y, m);
}
void orc_sample_ball_source(uint64_t seed, uint32_t k, uint32_t id, uint32_t batch, uint32_t tag,
                            int dim, const double* c, double R, double* y) {
  ball_source_point(seed, k, id, batch, tag, dim, c, R, y);
}
/* Radius fraction of the 2D gradient source sample: density (3/2)(1 - s^2). */
double orc_grad_radius(double u) { return 2 * sin(asin(u) / 3); }

/* Where a walk that stops at pos, at distance d from its closest boundary
 * point pb, reads the boundary data: at pb itself (Section 3.1), or, with
 * the side rule of double-sided data (p->side_read, Appendix B), at pb
 * approached from the walk's side by 1e-3 eps, so that data that differ on
 * the two sides of a boundary curve are read on the side the walk reached. */
static void read_point(const orc_walk_params* p, int dim, const double* pos, const double* pb, double d,
                       double* e) {
  const double t = p->side_read && d > 0 ? 1e-3 * p->eps / d : 0.0;
  for (int a = 0; a < dim; ++a) e[a] = pb[a] + t * (pos[a] - pb[a]);
}

/* The control variate c = g at the cache point's closest boundary point
 * xbar; with the side rule, at xbar moved 1e-3 of the way back to the cache
 * point x, on the point's own side of a boundary with double-sided data.
 * Any constant keeps the Eq. 7 estimate unbiased (E[nu] = 0). */
static double control_value(const orc_walk_params* p, const orc_field* g, int dim, const double* x,
                            const double* xbar) {
  if (!p->control_variate) return 0.0;
  if (!p->side_read) return orc_field_eval(g, dim, xbar);
  double e[3] = {0, 0, 0};
  for (int a = 0; a < dim; ++a) e[a] = xbar[a] + 1e-3 * (x[a] - xbar[a]);
  return orc_field_eval(g, dim, e);
}

/* Open (unbounded) 3D domains, Appendix B.  Outside a sphere B(c, Rb) that
 * encloses the whole boundary, Brownian motion from x (r = |x - c| > Rb) ever
 * reaches the sphere with probability Rb / r; otherwise it escapes to
 * infinity, where the solution vanishes.  Given that it reaches the sphere,
 * its first hit point follows the sphere's exterior harmonic measure from x,
 * normalised.  By the Kelvin transform that is the interior harmonic measure
 * from the image point x* = c + (Rb/r)^2 (x - c): the distance s from x* to
 * the hit point has density proportional to 1/s^2 on [Rb - a, Rb + a],
 * a = Rb^2 / r.  Inverting its CDF at v and writing rho = Rb / r, m = 1 - 2v,
 * the polar angle t of the hit point about the direction of x - c is
 *   cos t = (m + rho (m^2 + 3)/2 + rho^2 m + rho^3 (m^2 - 1)/2) / (1 + rho m)^2,
 * which keeps its accuracy as rho -> 0 (the hit point seen from infinity is
 * uniform: cos t = m).  The azimuth is 2 pi w about the orthonormal frame of
 * Duff et al. 2017 ("Building an orthonormal basis, revisited"). */
int orc_sphere_reentry(const double* c, double Rb, const double* x, double u, double v, double w, double* y) {
  double e[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
  double r = sqrt(dot3(e, e));
  double rho = Rb / r;
  if (u >= rho) return 1;
  for (int a = 0; a < 3; ++a) e[a] /= r;
  double m = 1 - 2 * v;
  double q = 1 + rho * m;
  double ct = (m + rho * (m * m + 3) / 2 + rho * rho * m + rho * rho * rho * (m * m - 1) / 2) / (q * q);
  if (ct > 1) ct = 1;
  if (ct < -1) ct = -1;
  double st = sqrt(1 - ct * ct);
  double sg = e[2] >= 0 ? 1.0 : -1.0;
  double ha = -1 / (sg + e[2]);
  double hb = e[0] * e[1] * ha;
  double t1[3] = {1 + sg * e[0] * e[0] * ha, sg * hb, -sg * e[0]};
  double t2[3] = {hb, sg + e[1] * e[1] * ha, -e[1]};
  double ph = 2 * ORC_PI * w;
  double cp = cos(ph), sp = sin(ph);
  for (int a = 0; a < 3; ++a) y[a] = c[a] + Rb * (ct * e[a] + st * (cp * t1[a] + sp * t2[a]));
  return 0;
}

/* A walk that has just jumped (jump index k) into an open domain's far
 * region: escape (returns 1) or move onto the enclosing sphere. */
static int open_step(const orc_walk_params* p, uint32_t k, uint32_t id, uint32_t tag, double* pos) {
  const double* c = p->open_center;
  double e[3] = {pos[0] - c[0], pos[1] - c[1], pos[2] - c[2]};
  if (!(dot3(e, e) > p->open_radius * p->open_radius)) return 0;
  double u, v, w, w2;
  orc_uniform_pair(p->seed, k, id, p->batch, tag | 8u, &u, &v);
  orc_uniform_pair(p->seed, k, id, p->batch, tag | 16u, &w, &w2);
  double y[3];
  if (orc_sphere_reentry(c, p->open_radius, pos, u, v, w, y)) return 1;
  for (int a = 0; a < 3; ++a) pos[a] = y[a];
  return 0;
}

void orc_walk(const orc_scene* s, const orc_field* g, const orc_field* f,
              const orc_walk_params* p, int mode, const double* x, const double* n, double R0,
              const double* xbar, uint32_t id, double* U, double* grad, double* exit_pt,
              double* w1, int32_t* steps, int32_t* capped) {
  int dim = s->dim;
  uint32_t tag = mode == 0 ? 1u : 2u;
  int has_f = f && f->kind != ORC_FIELD_ZERO;
  *capped = 0;
  if (mode == 1 && R0 < p->eps) {
    /* the evaluation point already lies in the epsilon shell */
    double e[3] = {0, 0, 0};
    read_point(p, dim, x, xbar, R0, e);
    *U = orc_field_eval(g, dim, e);
    for (int a = 0; a < dim; ++a) {
      grad[a] = 0;
      exit_pt[a] = e[a];
    }
    *w1 = 0;
    *steps = 0;
    return;
  }
  /* First ball B(x, R0): no termination test at x itself. */
  double nu0[3], pos[3];
  walk_direction(p->seed, 0, id, p->batch, tag, dim, nu0);
  for (int a = 0; a < dim; ++a) pos[a] = x[a] + R0 * nu0[a];
  const int open = dim == 3 && p->open_radius > 0;
  int escaped = open && open_step(p, 0, id, tag, pos);
  const int screened = p->sigma > 0;
  /* the first ball's source terms: u (weight R0^2/(2 dim) times the screened
   * ratio) and the gradient (weight m(t) R0 times its screened ratio) */
  double src_u = 0, src_g = 0, yhat_g[3] = {0, 0, 0};
  if (has_f) {
    double yu[3], yg[3], m;
    double tu = ball_source_point(p->seed, 0, id, p->batch, tag, dim, x, R0, yu);
    src_u = R0 * R0 / (2.0 * dim) * orc_screen_source_ratio(dim, p->sigma, R0, tu) * orc_field_eval(f, dim, yu);
    double tg = grad_source_point(p->seed, id, p->batch, tag, dim, x, R0, yhat_g, yg, &m);
    src_g = m * R0 * orc_screen_grad_source_ratio(dim, p->sigma, R0, tg) * orc_field_eval(f, dim, yg);
  }
  /* Walk on spheres from the first-ball point.  With screening every ball
   * the walk crosses multiplies the estimate by its mean-value factor, and a
   * ball's source term counts with the factors of the balls before it; the
   * first ball's factor is applied to U below, not to W (the estimate of u at
   * the first-ball point that the gradient uses). */
  double S = 0, W = 0, pb[3] = {0, 0, 0}, thr = 1.0;
  int32_t k;
  for (k = 1;; ++k) {
    if (escaped) {
      /* u = 0 at infinity */
      W = S;
      for (int a = 0; a < dim; ++a) pb[a] = NAN;
      break;
    }
    double d;
    orc_closest(s, pos, 0, &d, pb, NULL);
    if (d < p->eps || k >= p->max_steps) {
      *capped = !(d < p->eps);
      double e[3] = {0, 0, 0};
      read_point(p, dim, pos, pb, d, e);
      for (int a = 0; a < dim; ++a) pb[a] = e[a];
      W = thr * orc_field_eval(g, dim, pb) + S;
      break;
    }
    if (has_f) {
      double y[3];
      double t = ball_source_point(p->seed, (uint32_t)k, id, p->batch, tag, dim, pos, d, y);
      S -= thr * d * d / (2.0 * dim) * orc_screen_source_ratio(dim, p->sigma, d, t) * orc_field_eval(f, dim, y);
    }
    if (screened) thr *= orc_screen_ball_weight(dim, p->sigma, d);
    double nu[3];
    walk_direction(p->seed, (uint32_t)k, id, p->batch, tag, dim, nu);
    for (int a = 0; a < dim; ++a) pos[a] += d * nu[a];
    if (open) escaped = open_step(p, (uint32_t)k, id, tag, pos);
  }
  *steps = k;
  double gw = dim / R0;
  if (screened) {
    *U = orc_screen_ball_weight(dim, p->sigma, R0) * W - src_u;
    gw = orc_screen_grad_weight(dim, p->sigma, R0);
  } else {
    *U = W - src_u;
  }
  /* the escape rule holds for the Laplace equation without a source only */
  if (open && (screened || has_f)) *U = NAN;
  double c = control_value(p, g, dim, x, xbar);
  double wn = 0;
  for (int a = 0; a < dim; ++a) {
    grad[a] = gw * nu0[a] * (W - c) - yhat_g[a] * src_g;
    exit_pt[a] = pb[a];
    if (n) wn += nu0[a] * n[a];
  }
  *w1 = gw * wn;
}

int32_t orc_walk_queries(const orc_scene* s, const orc_walk_params* p, int mode, const double* x,
                         double R0, uint32_t id, int32_t max_q, double* q, int32_t* hint) {
  int dim = s->dim;
  uint32_t tag = mode == 0 ? 1u : 2u;
  if (mode == 1 && R0 < p->eps) return 0;
  double nu[3], pos[3], pb[3];
  walk_direction(p->seed, 0, id, p->batch, tag, dim, nu);
  for (int a = 0; a < dim; ++a) pos[a] = x[a] + R0 * nu[a];
  int32_t prev = -1, n = 0;
  for (int32_t k = 1; n < max_q; ++k) {
    for (int a = 0; a < dim; ++a) q[n * dim + a] = pos[a];
    hint[n++] = prev;
    double d;
    int32_t prim;
    orc_closest(s, pos, 0, &d, pb, &prim);
    if (d < p->eps || k >= p->max_steps) break;
    walk_direction(p->seed, (uint32_t)k, id, p->batch, tag, dim, nu);
    for (int a = 0; a < dim; ++a) pos[a] += d * nu[a];
    prev = prim;
  }
  return n;
}

void orc_bvh_visits(const orc_scene* s, int64_t n_nodes, const int32_t* child, const double* boxes,
                    const double* slabs, const int32_t* order, int64_t n_q, const double* q,
                    const int32_t* hint, double* nodes, double* prims) {
  int dim = s->dim;
  (void)n_nodes;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n_q; ++i) {
    const double* x = q + i * dim;
    double best = INFINITY, c[3];
    int reg;
    int64_t nn = 0, np = 0;
    if (hint[i] >= 0) {
      best = prim_dist2(s, hint[i], x, c, &reg);
      ++np;
    }
    int32_t stack[256];
    double bound[256];
    int top = 0;
    stack[top] = 0;
    bound[top++] = 0.0;
    while (top > 0) {
      --top;
      int32_t link = stack[top];
      if (bound[top] > best) continue;
      if (link < 0) {
        int32_t start = (~link) >> 3, cnt = ((~link) & 7) + 1;
        for (int32_t j = start; j < start + cnt; ++j) {
          double d2 = prim_dist2(s, order[j], x, c, &reg);
          ++np;
          if (d2 < best) best = d2;
        }
        continue;
      }
      ++nn;
      double db[2];
      for (int ch = 0; ch < 2; ++ch) {
        const double* lo = boxes + (int64_t)link * 4 * dim + ch * 2 * dim;
        const double* hi = lo + dim;
        double d2 = 0;
        for (int a = 0; a < dim; ++a) {
          double e = 0;
          if (x[a] < lo[a]) e = lo[a] - x[a];
          else if (x[a] > hi[a]) e = x[a] - hi[a];
          d2 += e * e;
        }
        if (slabs) {
          /* a second lower bound: the distance from n.x to the child's slab
             [smin, smax] along its axis n */
          const double* sl = slabs + (int64_t)link * 12 + ch * 5;
          double t = sl[0] * x[0] + sl[1] * x[1] + sl[2] * x[2], e = 0;
          if (t < sl[3]) e = sl[3] - t;
          else if (t > sl[4]) e = t - sl[4];
          if (e * e > d2) d2 = e * e;
        }
        db[ch] = d2;
      }
      /* the farther child goes below the nearer one */
      int near = db[1] < db[0] ? 1 : 0;
      stack[top] = child[2 * link + (1 - near)];
      bound[top++] = db[1 - near];
      stack[top] = child[2 * link + near];
      bound[top++] = db[near];
    }
    nodes[i] = (double)nn;
    prims[i] = (double)np;
  }
}

void orc_cache_walks(const orc_scene* s, const orc_field* g, const orc_field* f,
                     const orc_walk_params* p, int64_t n_cache, const double* x,
                     const double* nrm, const double* R0, const double* xbar, double* U,
                     double* D, double* exit_pt, double* w1, int32_t* steps) {
  int dim = s->dim;
  int64_t W = p->n_walks;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n_cache; ++i) {
    for (int64_t j = 0; j < W; ++j) {
      int64_t id = i * W + j;
      double u, gr[3], ex[3], ww;
      int32_t st, cap;
      orc_walk(s, g, f, p, 0, x + i * dim, nrm + i * dim, R0[i], xbar + i * dim, (uint32_t)id, &u,
               gr, ex, &ww, &st, &cap);
      double dn = 0;
      for (int a = 0; a < dim; ++a) dn += nrm[i * dim + a] * gr[a];
      U[id] = u;
      D[id] = dn;
      if (exit_pt)
        for (int a = 0; a < dim; ++a) exit_pt[id * dim + a] = ex[a];
      if (w1) w1[id] = ww;
      if (steps) steps[id] = st;
    }
  }
}

void orc_cache_walks_subset(const orc_scene* s, const orc_field* g, const orc_field* f,
                            const orc_walk_params* p, int64_t n_ids, const int64_t* ids,
                            const double* x, const double* nrm, const double* R0,
                            const double* xbar, double* U, double* D, int32_t* steps) {
  int dim = s->dim;
  int64_t W = p->n_walks;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < n_ids; ++q) {
    int64_t id = ids[q];
    int64_t i = id / W;
    double u, gr[3], ex[3], ww;
    int32_t st, cap;
    orc_walk(s, g, f, p, 0, x + i * dim, nrm + i * dim, R0[i], xbar + i * dim, (uint32_t)id, &u, gr,
             ex, &ww, &st, &cap);
    double dn = 0;
    for (int a = 0; a < dim; ++a) dn += nrm[i * dim + a] * gr[a];
    U[q] = u;
    D[q] = dn;
    if (steps) steps[q] = st;
  }
}

void orc_reduce(int64_t n_cache, int32_t W, const double* U, const double* D, double* uhat,
                double* dudn) {
  for (int64_t i = 0; i < n_cache; ++i) {
    double su = 0, sd = 0;
    for (int32_t j = 0; j < W; ++j) {
      su += U[i * W + j];
      sd += D[i * W + j];
    }
    uhat[i] = su / W;
    dudn[i] = sd / W;
  }
}

void orc_pointwise(const orc_scene* s, const orc_field* g, const orc_field* f,
                   const orc_walk_params* p, int64_t n, const double* x, double* u,
                   double* grad, int64_t* total_steps) {
  int dim = s->dim;
  int64_t W = p->n_walks;
  int64_t tot = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : tot)
  for (int64_t k = 0; k < n; ++k) {
    double R0, xb[3];
    orc_closest(s, x + k * dim, 0, &R0, xb, NULL);
    double su = 0, sg[3] = {0, 0, 0};
    for (int64_t j = 0; j < W; ++j) {
      double uu, gr[3], ex[3], ww;
      int32_t st, cap;
      orc_walk(s, g, f, p, 1, x + k * dim, NULL, R0, xb, (uint32_t)(k * W + j), &uu, gr, ex, &ww,
               &st, &cap);
      su += uu;
      for (int a = 0; a < dim; ++a) sg[a] += gr[a];
      tot += st;
    }
    u[k] = su / W;
    if (grad)
      for (int a = 0; a < dim; ++a) grad[k * dim + a] = sg[a] / W;
  }
  if (total_steps) *total_steps = tot;
}

/* ======================================================================== */
/* Gather: Monte Carlo estimators of the boundary integral equation          */
/* ======================================================================== */
void orc_gather(int dim, int64_t K, const double* ex, int64_t N, const double* cy,
                const double* cn, const double* a, const double* b, int64_t M,
                const double* sy, const double* sw, double* u, double* grad, double* cond) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < K; ++k) {
    const double* x = ex + k * dim;
    double uk = 0, ck = 0, gk[3] = {0, 0, 0};
    for (int64_t i = 0; i < N; ++i) {
      double G, dGdx[3], dGdn, d2[3];
      orc_greens(dim, x, cy + i * dim, cn + i * dim, &G, dGdx, &dGdn, d2);
      uk += dGdn * a[i] - G * b[i];
      ck += fabs(dGdn * a[i]) + fabs(G * b[i]);
      for (int q = 0; q < dim; ++q) gk[q] += d2[q] * a[i] - dGdx[q] * b[i];
    }
    for (int64_t j = 0; j < M; ++j) {
      double G, dGdx[3];
      orc_greens(dim, x, sy + j * dim, NULL, &G, dGdx, NULL, NULL);
      uk += G * sw[j];
      ck += fabs(G * sw[j]);
      for (int q = 0; q < dim; ++q) gk[q] += dGdx[q] * sw[j];
    }
    u[k] = uk;
    if (cond) cond[k] = ck;
    if (grad)
      for (int q = 0; q < dim; ++q) grad[k * dim + q] = gk[q];
  }
}

void orc_gather_backward(int dim, int64_t K, const double* ex, const double* r, int64_t N,
                         const double* cy, const double* cn, const double* a, const double* b,
                         int64_t M, const double* sy, const double* sw, double* dLda,
                         double* dLdb, double* dLds, double* dLdx) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < N; ++i) {
    double sa = 0, sb = 0;
    for (int64_t k = 0; k < K; ++k) {
      double G, dGdn;
      orc_greens(dim, ex + k * dim, cy + i * dim, cn + i * dim, &G, NULL, &dGdn, NULL);
      sa += r[k] * dGdn;
      sb -= r[k] * G;
    }
    dLda[i] = sa;
    dLdb[i] = sb;
  }
  if (dLds) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < M; ++j) {
      double ss = 0;
      for (int64_t k = 0; k < K; ++k) {
        double G;
        orc_greens(dim, ex + k * dim, sy + j * dim, NULL, &G, NULL, NULL, NULL);
        ss += r[k] * G;
      }
      dLds[j] = ss;
    }
  }
  if (dLdx) {
    double* u = (double*)malloc((size_t)K * sizeof(double));
    double* g = (double*)malloc((size_t)K * dim * sizeof(double));
    orc_gather(dim, K, ex, N, cy, cn, a, b, M, sy, sw, u, g, NULL);
    for (int64_t k = 0; k < K; ++k)
      for (int q = 0; q < dim; ++q) dLdx[k * dim + q] = r[k] * g[k * dim + q];
    free(u);
    free(g);
  }
}

void orc_basis_means(const orc_field* basis, int dim, int64_t n_cache, int32_t W,
                     const double* exit_pt, const double* w1, const double* xbar, int cv,
                     double* E, double* F) {
  int nb = basis->n_coef;
  if (basis->kind == ORC_FIELD_GAUSS_SUM) nb = basis->n_coef / (1 + dim);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n_cache; ++i) {
    for (int m = 0; m < nb; ++m) {
      double base = cv ? orc_basis_eval(basis, dim, m, xbar + i * dim) : 0.0;
      double se = 0, sf = 0;
      for (int32_t j = 0; j < W; ++j) {
        int64_t id = i * W + j;
        /* a walk that escaped an open domain (NaN exit) reads u = 0 at
         * infinity whatever the data: every basis value is 0 there */
        const double* e = exit_pt + id * dim;
        double phi = isnan(e[0]) ? 0.0 : orc_basis_eval(basis, dim, m, e);
        se += phi;
        sf += w1[id] * (phi - base);
      }
      E[i * nb + m] = se / W;
      F[i * nb + m] = sf / W;
    }
  }
}

/* ======================================================================== */
/* Walk on stars for mixed Dirichlet / Neumann boundaries (Section 3.1: the  */
/* WoSt estimator the cache relies on; 2D segments and 3D triangles, Neumann */
/* data h, no source term)                                                  */
/* ======================================================================== */
/* The Dirichlet part `dir` and the Neumann part `neu` are two element sets
 * of one boundary (2D: counter-clockwise segments; 3D: triangles with
 * outward normals by the right-hand rule).
 *
 * 2D: seen from x, a vertex of the Neumann part is a silhouette point when
 * both Neumann segments at it lie on the same side of the line through x and
 * the vertex, or when the Neumann part ends there. */
typedef struct {
  int32_t* prev;     /* per Neumann segment: start vertex of the Neumann segment ending at its start, or -1 */
  int32_t* has_next; /* 1 when a Neumann segment starts at its end vertex */
  int32_t* straight; /* 1 when the segment and the one ending at its start are collinear */
  /* 3D: per triangle and edge k (vertex k to vertex k+1 mod 3) */
  int32_t* nb;       /* the Neumann triangle across the edge, or -1 (the Neumann part ends there) */
  int32_t* flat;     /* 1 when that triangle is coplanar with this one (no fold at the edge) */
} neu_links;

static void free_links(neu_links* L) {
  free(L->prev);
  free(L->has_next);
  free(L->straight);
  free(L->nb);
  free(L->flat);
}

typedef struct {
  int32_t lo, hi, tri, k;
} edge_rec;

static int edge_cmp(const void* a, const void* b) {
  const edge_rec* x = (const edge_rec*)a;
  const edge_rec* y = (const edge_rec*)b;
  if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
  if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
  if (x->tri != y->tri) return x->tri < y->tri ? -1 : 1;
  return x->k - y->k;
}

static neu_links make_links(const orc_scene* neu) {
  neu_links L = {NULL, NULL, NULL, NULL, NULL};
  int64_t np = neu->np, nv = neu->nv;
  if (neu->dim == 3) {
    /* triangles across each edge from the sorted list of edges by vertex pair */
    L.nb = (int32_t*)malloc((size_t)np * 3 * sizeof(int32_t));
    L.flat = (int32_t*)malloc((size_t)np * 3 * sizeof(int32_t));
    edge_rec* E = (edge_rec*)malloc((size_t)np * 3 * sizeof(edge_rec));
    for (int64_t t = 0; t < np; ++t)
      for (int k = 0; k < 3; ++k) {
        int32_t a = neu->P[3 * t + k], b = neu->P[3 * t + (k + 1) % 3];
        E[3 * t + k].lo = a < b ? a : b;
        E[3 * t + k].hi = a < b ? b : a;
        E[3 * t + k].tri = (int32_t)t;
        E[3 * t + k].k = k;
        L.nb[3 * t + k] = -1;
        L.flat[3 * t + k] = 0;
      }
    qsort(E, (size_t)np * 3, sizeof(edge_rec), edge_cmp);
    for (int64_t i = 0; i + 1 < np * 3; ++i) {
      if (E[i].lo != E[i + 1].lo || E[i].hi != E[i + 1].hi) continue;
      const edge_rec *e = &E[i], *f = &E[i + 1];
      L.nb[3 * e->tri + e->k] = f->tri;
      L.nb[3 * f->tri + f->k] = e->tri;
      const double* n1 = neu->fnorm + 3 * (int64_t)e->tri;
      const double* n2 = neu->fnorm + 3 * (int64_t)f->tri;
      double c[3];
      cross3(n1, n2, c);
      int fl = sqrt(dot3(c, c)) <= 1e-12 && dot3(n1, n2) > 0;
      L.flat[3 * e->tri + e->k] = L.flat[3 * f->tri + f->k] = fl;
      ++i;
    }
    free(E);
    return L;
  }
  L.prev = (int32_t*)malloc((size_t)np * sizeof(int32_t));
  L.has_next = (int32_t*)malloc((size_t)np * sizeof(int32_t));
  L.straight = (int32_t*)malloc((size_t)np * sizeof(int32_t));
  int32_t* ends_at = (int32_t*)malloc((size_t)nv * sizeof(int32_t));
  int32_t* starts_at = (int32_t*)malloc((size_t)nv * sizeof(int32_t));
  for (int64_t v = 0; v < nv; ++v) ends_at[v] = starts_at[v] = -1;
  for (int64_t q = 0; q < np; ++q) {
    starts_at[neu->P[2 * q]] = (int32_t)q;
    ends_at[neu->P[2 * q + 1]] = (int32_t)q;
  }
  for (int64_t q = 0; q < np; ++q) {
    int32_t r = ends_at[neu->P[2 * q]];
    L.prev[q] = r >= 0 ? neu->P[2 * r] : -1;
    L.has_next[q] = starts_at[neu->P[2 * q + 1]] >= 0;
    L.straight[q] = 0;
    if (r >= 0) {
      /* no corner at the start vertex: the two segments continue one line */
      const double* u = neu->V + 2 * (int64_t)L.prev[q];
      const double* a = neu->V + 2 * (int64_t)neu->P[2 * q];
      const double* b = neu->V + 2 * (int64_t)neu->P[2 * q + 1];
      double e0 = a[0] - u[0], e1 = a[1] - u[1], f0 = b[0] - a[0], f1 = b[1] - a[1];
      L.straight[q] = fabs(e0 * f1 - e1 * f0) <= 1e-12 * hypot(e0, e1) * hypot(f0, f1) && e0 * f0 + e1 * f1 > 0;
    }
  }
  free(ends_at);
  free(starts_at);
  return L;
}

static double cross2(double ax, double ay, double bx, double by) { return ax * by - ay * bx; }

/* Side of point w relative to the line from x through v: +1, -1, or 0 when
 * within a relative 1e-9 of it (a walk standing on a Neumann segment lies on
 * that segment's line only up to rounding). */
static int line_side(const double* x, const double* v, const double* w) {
  double vx = v[0] - x[0], vy = v[1] - x[1], wx = w[0] - v[0], wy = w[1] - v[1];
  double c = cross2(vx, vy, wx, wy);
  if (fabs(c) <= 1e-9 * hypot(vx, vy) * hypot(wx, wy)) return 0;
  return c > 0 ? 1 : -1;
}

/* Side of x relative to the plane of a triangle with unit normal n through
 * the point v: +1 in front (the side the normal points to), -1 behind, 0
 * within a relative 1e-9 of the plane (a walk standing on a Neumann face lies
 * in its plane only up to rounding). */
static int plane_side(const double* x, const double* v, const double* n) {
  double d[3] = {x[0] - v[0], x[1] - v[1], x[2] - v[2]};
  double s = dot3(n, d);
  if (fabs(s) <= 1e-9 * sqrt(dot3(d, d))) return 0;
  return s > 0 ? 1 : -1;
}

static double segment_dist3(const double* x, const double* a, const double* b) {
  double e[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, r[3] = {x[0] - a[0], x[1] - a[1], x[2] - a[2]};
  double t = dot3(r, e) / dot3(e, e);
  t = t < 0 ? 0 : (t > 1 ? 1 : t);
  double d[3] = {r[0] - t * e[0], r[1] - t * e[1], r[2] - t * e[2]};
  return sqrt(dot3(d, d));
}

/* Distance from x to the closest silhouette of the Neumann part.
 * 2D: a corner vertex whose two Neumann neighbours do not lie strictly on
 * opposite sides of the line from x through it (both on one side; one on the
 * line, x looking along a segment past the corner; both on it, the fold at
 * the tip of a thin Neumann curve), and the ends of Neumann runs.  A vertex
 * where the boundary continues straight is no corner and never a silhouette.
 * 3D: an edge where the Neumann part ends, and an edge between two
 * non-coplanar Neumann triangles unless x lies strictly in front of both
 * planes or strictly behind both (one seen from the front and the other
 * from the back is a fold of the surface as seen from x; x in one of the
 * planes sees that face edge-on). */
static double silhouette_distance(const orc_scene* neu, const neu_links* L, const double* x) {
  double best = INFINITY;
  if (neu->dim == 3) {
    for (int64_t t = 0; t < neu->np; ++t)
      for (int k = 0; k < 3; ++k) {
        int32_t nb = L->nb[3 * t + k];
        if (nb >= 0 && (nb < t || L->flat[3 * t + k])) continue; /* each interior edge once; flat edges never */
        const double* a = neu->V + 3 * (int64_t)neu->P[3 * t + k];
        const double* b = neu->V + 3 * (int64_t)neu->P[3 * t + (k + 1) % 3];
        int sil = 1;
        if (nb >= 0) {
          int s1 = plane_side(x, a, neu->fnorm + 3 * t), s2 = plane_side(x, a, neu->fnorm + 3 * (int64_t)nb);
          sil = !(s1 * s2 > 0);
        }
        if (sil) best = fmin(best, segment_dist3(x, a, b));
      }
    return best;
  }
  for (int64_t q = 0; q < neu->np; ++q) {
    const double* a = neu->V + 2 * (int64_t)neu->P[2 * q];
    const double* b = neu->V + 2 * (int64_t)neu->P[2 * q + 1];
    int sil = 1;
    if (L->straight[q]) {
      sil = 0;
    } else if (L->prev[q] >= 0) {
      const double* u = neu->V + 2 * (int64_t)L->prev[q];
      int s1 = line_side(x, a, u), s2 = line_side(x, a, b);
      /* a corner hides nothing only when its neighbours lie strictly on
       * opposite sides of the line of sight; with both on it the boundary
       * folds back there (the tip of a thin Neumann curve) */
      sil = !(s1 * s2 < 0);
    }
    if (sil) best = fmin(best, hypot(a[0] - x[0], a[1] - x[1]));
    if (!L->has_next[q]) best = fmin(best, hypot(b[0] - x[0], b[1] - x[1]));
  }
  return best;
}

/* Nearest crossing of the ray x + t w, lo < t <= hi, with a Neumann element
 * the ray leaves the domain through (w . n_out > 0), so that of the two
 * faces of a double-sided Neumann sheet (Appendix B) the ray meets the one
 * facing its own side: its t (INFINITY if none), and the element in *el (-1
 * if none).  3D: the ray's parameters on the triangle by Cramer's rule on
 * x + t w = a + u (b - a) + v (c - a). */
static double neumann_hit(const orc_scene* neu, const double* x, const double* w, double lo, double hi,
                          int64_t* el) {
  double best = INFINITY;
  *el = -1;
  if (neu->dim == 3) {
    for (int64_t t3 = 0; t3 < neu->np; ++t3) {
      const double* a = neu->V + 3 * (int64_t)neu->P[3 * t3];
      const double* b = neu->V + 3 * (int64_t)neu->P[3 * t3 + 1];
      const double* c = neu->V + 3 * (int64_t)neu->P[3 * t3 + 2];
      double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
      double n[3];
      cross3(e1, e2, n);
      double den = dot3(w, n);
      if (!(den > 0)) continue;
      double r[3] = {x[0] - a[0], x[1] - a[1], x[2] - a[2]}, rw[3];
      cross3(r, w, rw);
      double t = -dot3(r, n) / den;
      double u = -dot3(rw, e2) / den;
      double v = dot3(rw, e1) / den;
      if (t > lo && t <= hi && u >= 0 && v >= 0 && u + v <= 1 && t < best) {
        best = t;
        *el = t3;
      }
    }
    return best;
  }
  for (int64_t q = 0; q < neu->np; ++q) {
    const double* a = neu->V + 2 * (int64_t)neu->P[2 * q];
    const double* b = neu->V + 2 * (int64_t)neu->P[2 * q + 1];
    double e0 = b[0] - a[0], e1 = b[1] - a[1];
    double den = cross2(w[0], w[1], e0, e1);
    if (!(den > 0)) continue;
    double r0 = a[0] - x[0], r1 = a[1] - x[1];
    double t = cross2(r0, r1, e0, e1) / den;
    double u = cross2(r0, r1, w[0], w[1]) / den;
    if (t > lo && t <= hi && u >= 0 && u <= 1 && t < best) {
      best = t;
      *el = q;
    }
  }
  return best;
}

/* The Neumann term of one star (Section 3.1; the boundary integral of the
 * Green's representation on the star St(x, R) with u's normal derivative h
 * known on the Neumann part): I = int over the Neumann part of the star's
 * boundary of G^B(x, z) h(z) dz, divided by alpha(x) = 1/2 when x stands on
 * the Neumann part (the star is then a half ball at x) and 1 inside.  With
 * R at most the silhouette distance, that part is every point of a Neumann
 * element within R of x whose element x does not lie strictly behind.  One
 * sample: the elements within R (1 + 1e-9) of x (x not strictly behind) form
 * the set C of total measure |C| (a superset of the elements that meet the
 * ball: one beyond R draws a point outside it and adds 0, so the estimate
 * stays unbiased; the margin keeps in C the elements that touch the ball
 * where R is set by a silhouette, at distance R up to rounding); one element is drawn with probability measure /
 * |C| by an exponential race (key -ln(1 - U_e) / measure_e, the smallest
 * wins; U_e from Philox block e, the element's index, tag | 32 | (k << 8)),
 * which does not depend on the order the elements are visited in; z is
 * uniform on it (block 4k + 1, tag | 64: 2D a + U1 (b - a); 3D barycentric
 * (1 - s, s (1 - U2), s U2), s = sqrt(U1)); the estimate is
 * |C| G^B(x, z) h(z) / alpha when |z - x| < R, else 0.  G^B(x, z) is
 * ln(R / r) / (2 pi) in 2D and (1 / r - 1 / R) / (4 pi) in 3D. */
static double neumann_term(const orc_scene* neu, const orc_field* h, const orc_walk_params* p, uint32_t k,
                           uint32_t id, uint32_t tag, const double* x, double R, int onb) {
  int dim = neu->dim;
  double AC = 0, key_best = INFINITY;
  int64_t pick = -1;
  for (int64_t e = 0; e < neu->np; ++e) {
    const double* a = neu->V + dim * (int64_t)neu->P[dim * e];
    double c[3];
    int reg;
    if (!(prim_dist2(neu, e, x, c, &reg) < R * R * (1 + 2e-9))) continue;
    double meas;
    if (dim == 2) {
      const double* b = neu->V + 2 * (int64_t)neu->P[2 * e + 1];
      double n_out[2] = {b[1] - a[1], -(b[0] - a[0])};
      double len = hypot(n_out[0], n_out[1]);
      double sd = (n_out[0] * (x[0] - a[0]) + n_out[1] * (x[1] - a[1])) / len;
      if (sd > 1e-9 * hypot(x[0] - a[0], x[1] - a[1])) continue; /* strictly behind */
      meas = len;
    } else {
      if (plane_side(x, a, neu->fnorm + 3 * e) > 0) continue;
      const double* b = neu->V + 3 * (int64_t)neu->P[3 * e + 1];
      const double* cc = neu->V + 3 * (int64_t)neu->P[3 * e + 2];
      double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {cc[0] - a[0], cc[1] - a[1], cc[2] - a[2]};
      double nn[3];
      cross3(e1, e2, nn);
      meas = 0.5 * sqrt(dot3(nn, nn));
    }
    AC += meas;
    double u, unused;
    orc_uniform_pair(p->seed, (uint32_t)e, id, p->batch, tag | 32u | (k << 8), &u, &unused);
    double key = -log(1.0 - u) / meas;
    if (key < key_best) {
      key_best = key;
      pick = e;
    }
  }
  if (pick < 0) return 0.0;
  double u1, u2, z[3] = {0, 0, 0};
  orc_uniform_pair(p->seed, 4 * k + 1, id, p->batch, tag | 64u, &u1, &u2);
  const double* a = neu->V + dim * (int64_t)neu->P[dim * pick];
  const double* b = neu->V + dim * (int64_t)neu->P[dim * pick + 1];
  if (dim == 2) {
    for (int q = 0; q < 2; ++q) z[q] = a[q] + u1 * (b[q] - a[q]);
  } else {
    const double* c = neu->V + 3 * (int64_t)neu->P[3 * pick + 2];
    double s = sqrt(u1);
    for (int q = 0; q < 3; ++q) z[q] = (1 - s) * a[q] + s * (1 - u2) * b[q] + s * u2 * c[q];
  }
  double r2 = 0;
  for (int q = 0; q < dim; ++q) r2 += (z[q] - x[q]) * (z[q] - x[q]);
  double r = sqrt(r2);
  if (!(r < R) || !(r > 0)) return 0.0;
  double G = dim == 2 ? log(R / r) / (2 * ORC_PI) : (1.0 / r - 1.0 / R) / (4 * ORC_PI);
  return AC * G * orc_field_eval(h, dim, z) / (onb ? 0.5 : 1.0);
}

/* One walk on stars (modes as orc_wost_walks). */
static void wost_walk(const orc_scene* dir, const orc_scene* neu, const neu_links* L, const orc_field* g,
                      const orc_field* h, const orc_walk_params* p, int mode, const double* x, const double* n,
                      double R0, const double* xbar, uint32_t id, double* U, double* D, int32_t* steps,
                      int32_t* capped) {
  int dim = dir->dim;
  uint32_t tag = mode == 0 ? 1u : 2u;
  double pos[3] = {0, 0, 0}, nin[3] = {0, 0, 0}, nu0[3] = {0, 0, 0};
  for (int q = 0; q < dim; ++q) pos[q] = x[q];
  int onb = 0;
  int32_t k = 0;
  double SN = 0.0;
  *capped = 0;
  if (mode == 0) {
    /* first ball, wholly inside the domain: the gradient estimate of Eq. 7 */
    walk_direction(p->seed, 0, id, p->batch, tag, dim, nu0);
    for (int q = 0; q < dim; ++q) pos[q] = x[q] + R0 * nu0[q];
    k = 1;
  } else if (mode == 3) {
    onb = 1;
    for (int q = 0; q < dim; ++q) nin[q] = -n[q];
  }
  double W;
  for (;; ++k) {
    double dD, qD[3];
    orc_closest(dir, pos, 0, &dD, qD, NULL);
    if (dD < p->eps || k >= p->max_steps) {
      *capped = !(dD < p->eps);
      double e[3];
      read_point(p, dim, pos, qD, dD, e);
      W = orc_field_eval(g, dim, e);
      break;
    }
    double R = fmax(fmin(dD, silhouette_distance(neu, L, pos)), p->eps);
    if (h && h->kind != 0) SN += neumann_term(neu, h, p, (uint32_t)k, id, tag, pos, R, onb);
    double w[3];
    walk_direction(p->seed, (uint32_t)k, id, p->batch, tag, dim, w);
    double wn = 0;
    for (int q = 0; q < dim; ++q) wn += w[q] * nin[q];
    if (onb && wn < 0)
      for (int q = 0; q < dim; ++q) w[q] = -w[q];
    int64_t el;
    double t = neumann_hit(neu, pos, w, 1e-9 * R, R, &el);
    if (el >= 0) {
      for (int q = 0; q < dim; ++q) pos[q] += t * w[q];
      if (dim == 2) {
        const double* a = neu->V + 2 * (int64_t)neu->P[2 * el];
        const double* b = neu->V + 2 * (int64_t)neu->P[2 * el + 1];
        double e0 = b[0] - a[0], e1 = b[1] - a[1], len = hypot(e0, e1);
        nin[0] = -e1 / len; /* inward normal of a counter-clockwise boundary */
        nin[1] = e0 / len;
      } else {
        for (int q = 0; q < 3; ++q) nin[q] = -neu->fnorm[3 * el + q];
      }
      onb = 1;
    } else {
      for (int q = 0; q < dim; ++q) pos[q] += R * w[q];
      onb = 0;
    }
  }
  *steps = k;
  *U = W + SN;
  if (D) {
    *D = 0;
    if (mode == 0) {
      double c = control_value(p, g, dim, x, xbar), dn = 0;
      for (int q = 0; q < dim; ++q) dn += nu0[q] * n[q];
      *D = (double)dim / R0 * dn * (*U - c);
    }
  }
}

void orc_silhouette_distances(const orc_scene* neu, int64_t n, const double* x, double* d) {
  neu_links L = make_links(neu);
  for (int64_t i = 0; i < n; ++i) d[i] = silhouette_distance(neu, &L, x + neu->dim * i);
  free_links(&L);
}

void orc_wost_walks(const orc_scene* dir, const orc_scene* neu, const orc_field* g, const orc_field* h,
                    const orc_walk_params* p, int mode, int64_t n, const double* x, const double* nrm,
                    const double* R0, const double* xbar, double* U, double* D, int32_t* steps) {
  neu_links L = make_links(neu);
  int64_t W = p->n_walks;
  int dim = dir->dim;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < W; ++j) {
      int64_t id = i * W + j;
      int32_t st, cap;
      double uu, dd;
      wost_walk(dir, neu, &L, g, h, p, mode, x + dim * i, nrm ? nrm + dim * i : NULL, R0 ? R0[i] : 0.0,
                xbar ? xbar + dim * i : NULL, (uint32_t)id, &uu, &dd, &st, &cap);
      U[id] = uu;
      if (D) D[id] = dd;
      if (steps) steps[id] = st;
    }
  }
  free_links(&L);
}

/* Cache candidates for a boundary with a Neumann part (Section 3.2, "Boundary
 * Specification": samples on the Neumann part and on the offset Dirichlet
 * boundary at distance l > eps).  One stratified draw (Philox tag 7) over the
 * concatenated measures of the offset Dirichlet elements (as
 * orc_sample_cache with sides 1, on the Dirichlet segments `dir`) followed
 * by the Neumann segments `neu`.  An offset candidate is kept when its
 * distance to the Dirichlet part is l (1e-9 relative), it lies inside the
 * domain `full` and (when junction_drop > 0) no closer than junction_drop * l
 * to the Neumann part; a Neumann candidate when its distance to the
 * Dirichlet part exceeds l.  Outputs: x, nrm (offset points: towards the closest Dirichlet
 * point; Neumann points: the segment's outward normal), w = total measure /
 * n, xbar = closest Dirichlet point, R0 = distance to the whole boundary,
 * type (0 offset, 1 Neumann), accept.  Returns the number accepted. */
int64_t orc_sample_mixed(const orc_scene* full, const orc_scene* dir, const orc_scene* neu, int64_t n, double l,
                         double junction_drop, uint64_t seed, uint32_t batch, double* x, double* nrm, double* w,
                         double* xbar, double* R0, int32_t* type, int32_t* accept) {
  elem_table T;
  make_elements(dir, l, 1, &T);
  double MD = T.cdf[T.n_el];
  double* cn = (double*)malloc((size_t)(neu->np + 1) * sizeof(double));
  cn[0] = 0;
  for (int64_t q = 0; q < neu->np; ++q) {
    const double* a = neu->V + 2 * (int64_t)neu->P[2 * q];
    const double* b = neu->V + 2 * (int64_t)neu->P[2 * q + 1];
    cn[q + 1] = cn[q] + hypot(b[0] - a[0], b[1] - a[1]);
  }
  double M = MD + cn[neu->np];
  int64_t n_acc = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : n_acc)
  for (int64_t k = 0; k < n; ++k) {
    double ua, ub;
    orc_uniform_pair(seed, 0, (uint32_t)k, batch, 7, &ua, &ub);
    double target = ((double)k + ua) / (double)n * M;
    double* xk = x + 2 * k;
    double* nk = nrm + 2 * k;
    double dD, xb[3];
    int ok;
    if (target < MD) {
      int64_t lo = 0, hi = T.n_el - 1;
      while (lo < hi) {
        int64_t mid = (lo + hi + 1) / 2;
        if (T.cdf[mid] <= target) lo = mid;
        else hi = mid - 1;
      }
      double r = (target - T.cdf[lo]) / T.meas[lo];
      r = r < 0 ? 0 : (r > 1 ? 1 : r);
      candidate_point(dir, &T, lo, r, ub, l, xk);
      orc_closest(dir, xk, 0, &dD, xb, NULL);
      ok = fabs(dD - l) <= 1e-9 * l && orc_inside(full, xk) != 0;
      for (int a = 0; a < 2; ++a) nk[a] = (xb[a] - xk[a]) / dD;
      type[k] = 0;
    } else {
      double t2 = target - MD;
      int64_t lo = 0, hi = neu->np - 1;
      while (lo < hi) {
        int64_t mid = (lo + hi + 1) / 2;
        if (cn[mid] <= t2) lo = mid;
        else hi = mid - 1;
      }
      const double* a = neu->V + 2 * (int64_t)neu->P[2 * lo];
      const double* b = neu->V + 2 * (int64_t)neu->P[2 * lo + 1];
      double e0 = b[0] - a[0], e1 = b[1] - a[1], len = hypot(e0, e1);
      double r = (t2 - cn[lo]) / len;
      r = r < 0 ? 0 : (r > 1 ? 1 : r);
      xk[0] = a[0] + r * e0;
      xk[1] = a[1] + r * e1;
      nk[0] = e1 / len;
      nk[1] = -e0 / len;
      orc_closest(dir, xk, 0, &dD, xb, NULL);
      ok = dD > l;
      type[k] = 1;
    }
    double dF, xf[3];
    orc_closest(full, xk, 0, &dF, xf, NULL);
    /* optional: an offset point within junction_drop * l of the Neumann part
     * is dropped (its first ball, no larger than that distance, gives the
     * Eq. 7 estimate a variance that grows like (l / R0)^2); the boundary
     * integral then loses that much length where the offset curve meets the
     * Neumann part.  0 keeps every point of the offset curve. */
    if (type[k] == 0 && dF < junction_drop * l) ok = 0;
    R0[k] = dF;
    xbar[2 * k] = xb[0];
    xbar[2 * k + 1] = xb[1];
    w[k] = M / (double)n;
    accept[k] = ok;
    n_acc += ok;
  }
  free(cn);
  free_elements(&T);
  return n_acc;
}

/* ======================================================================== */
/* Clamped double-layer kernel and its bias correction (Section 3.3,         */
/* Eqs. 8-9)                                                                 */
/* ======================================================================== */
/* |dG/dn(x, z)| = |n . (z - x)| / (|S| r^dim) <= 1 / (|S| r^(dim-1)), so no
 * boundary point farther than this radius has |dG/dn| above c. */
double orc_clamp_radius(int dim, double c) {
  if (!(c > 0)) return INFINITY;
  return dim == 2 ? 1.0 / (2 * ORC_PI * c) : sqrt(1.0 / (4 * ORC_PI * c));
}

/* Eq. 3 with dG/dn replaced by its clamp to [-c, c] (Eq. 9): the first
 * integral of Eq. 8 estimated with the cache samples, plus the single-layer
 * and source terms unchanged. */
void orc_gather_clamped(int dim, int64_t K, const double* ex, int64_t N, const double* cy,
                        const double* cn, const double* a, const double* b, int64_t M,
                        const double* sy, const double* sw, double c, double* u) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < K; ++k) {
    const double* x = ex + k * dim;
    double uk = 0;
    for (int64_t i = 0; i < N; ++i) {
      double G, dGdn;
      orc_greens(dim, x, cy + i * dim, cn + i * dim, &G, NULL, &dGdn, NULL);
      double kc = dGdn > c ? c : (dGdn < -c ? -c : dGdn);
      uk += kc * a[i] - G * b[i];
    }
    for (int64_t j = 0; j < M; ++j) {
      double G;
      orc_greens(dim, x, sy + j * dim, NULL, &G, NULL, NULL, NULL);
      uk += G * sw[j];
    }
    u[k] = uk;
  }
}

/* Intersections of a ray with the offset boundary dR = {z inside : d(z) = l},
 * the boundary of the region whose cache the gather uses (Section 3.2).  The
 * candidates are the ray's crossings with every piece of the candidate set the
 * cache sampler draws from (segment or face offsets at distance l, vertex
 * circles or spheres, edge cylinders; both segment sides when sides = 2); a
 * candidate belongs to dR when no boundary point is closer than l (up to
 * 1e-9 relative) and it lies inside, the sampler's own acceptance rule. */
typedef struct {
  double t;
  double z[3];
  double n[3];
} orc_hit;

typedef struct {
  orc_hit* h;
  int64_t n, cap;
} hit_list;

static void hit_push(hit_list* L, const double* x, const double* w, double t, const double* n, int dim) {
  if (L->n == L->cap) {
    L->cap = L->cap ? 2 * L->cap : 16;
    L->h = (orc_hit*)realloc(L->h, (size_t)L->cap * sizeof(orc_hit));
  }
  orc_hit* H = &L->h[L->n++];
  H->t = t;
  for (int a = 0; a < 3; ++a) {
    H->z[a] = a < dim ? x[a] + t * w[a] : 0.0;
    H->n[a] = a < dim ? n[a] : 0.0;
  }
}

static int hit_cmp(const void* p, const void* q) {
  double a = ((const orc_hit*)p)->t, b = ((const orc_hit*)q)->t;
  return a < b ? -1 : (a > b ? 1 : 0);
}

/* Roots of t^2 + 2 qb t + qc = 0 (a unit-speed ray against a circle or
 * sphere of radius l around c, qb = w.(x - c), qc = |x - c|^2 - l^2). */
static int unit_quadratic(double qb, double qc, double* t) {
  double disc = qb * qb - qc;
  if (disc < 0) return 0;
  double s = sqrt(disc);
  t[0] = -qb - s;
  t[1] = -qb + s;
  return 2;
}

static void round_candidates(const double* x, const double* w, const double* c, double l, double t_max, int dim,
                             hit_list* L) {
  double qb = 0, qc = -l * l, t[2];
  for (int a = 0; a < dim; ++a) {
    qb += w[a] * (x[a] - c[a]);
    qc += (x[a] - c[a]) * (x[a] - c[a]);
  }
  int nr = unit_quadratic(qb, qc, t);
  for (int r = 0; r < nr; ++r) {
    if (!(t[r] > 0 && t[r] <= t_max)) continue;
    double n[3];
    for (int a = 0; a < dim; ++a) n[a] = (c[a] - (x[a] + t[r] * w[a])) / l;
    hit_push(L, x, w, t[r], n, dim);
  }
}

int32_t orc_offset_hits(const orc_scene* s, double l, int sides, const double* x, const double* w, double t_max,
                        int32_t max_hits, double* t_out, double* z_out, double* n_out) {
  int dim = s->dim;
  hit_list C = {NULL, 0, 0};
  if (dim == 2) {
    for (int64_t p = 0; p < s->np; ++p) {
      const double* a = s->V + 2 * (int64_t)s->P[2 * p];
      const double* b = s->V + 2 * (int64_t)s->P[2 * p + 1];
      double e0 = b[0] - a[0], e1 = b[1] - a[1];
      double len = sqrt(e0 * e0 + e1 * e1);
      double n0 = e1 / len, n1 = -e0 / len; /* outward normal of a CCW polygon */
      for (int sd = 0; sd < sides; ++sd) {
        double side = sd == 0 ? 1.0 : -1.0;
        /* offset segment a' + u e, a' = a - side l n; solve x + t w = a' + u e */
        double ap0 = a[0] - side * l * n0, ap1 = a[1] - side * l * n1;
        double den = w[0] * e1 - w[1] * e0; /* cross(w, e) */
        if (den == 0) continue;
        double r0 = ap0 - x[0], r1 = ap1 - x[1];
        double t = (r0 * e1 - r1 * e0) / den;
        double u = (r0 * w[1] - r1 * w[0]) / den;
        if (!(t > 0 && t <= t_max && u >= 0 && u <= 1)) continue;
        double n[2] = {side * n0, side * n1};
        hit_push(&C, x, w, t, n, 2);
      }
    }
    for (int64_t v = 0; v < s->nv; ++v) round_candidates(x, w, s->V + 2 * v, l, t_max, 2, &C);
  } else {
    for (int64_t p = 0; p < s->np; ++p) {
      const double* A = s->V + 3 * (int64_t)s->P[3 * p];
      const double* B = s->V + 3 * (int64_t)s->P[3 * p + 1];
      const double* Cc = s->V + 3 * (int64_t)s->P[3 * p + 2];
      double ab[3], ac[3], nn[3];
      for (int a = 0; a < 3; ++a) {
        ab[a] = B[a] - A[a];
        ac[a] = Cc[a] - A[a];
      }
      cross3(ab, ac, nn);
      double len = sqrt(dot3(nn, nn));
      for (int a = 0; a < 3; ++a) nn[a] /= len;
      /* inward offset triangle A - l n + beta ab + gamma ac (Moller and
       * Trumbore's ray-triangle test, solved by Cramer's rule) */
      double Ap[3], pv[3], tv[3], qv[3];
      for (int a = 0; a < 3; ++a) Ap[a] = A[a] - l * nn[a];
      cross3(w, ac, pv);
      double det = dot3(ab, pv);
      if (det == 0) continue;
      for (int a = 0; a < 3; ++a) tv[a] = x[a] - Ap[a];
      double beta = dot3(tv, pv) / det;
      cross3(tv, ab, qv);
      double gam = dot3(w, qv) / det;
      double t = dot3(ac, qv) / det;
      if (!(beta >= 0 && gam >= 0 && beta + gam <= 1 && t > 0 && t <= t_max)) continue;
      hit_push(&C, x, w, t, nn, 3);
    }
    for (int64_t q = 0; q < s->ne; ++q) {
      const double* A = s->V + 3 * (int64_t)s->edges[2 * q];
      const double* B = s->V + 3 * (int64_t)s->edges[2 * q + 1];
      double e[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
      double L2 = dot3(e, e), L = sqrt(L2);
      double eh[3] = {e[0] / L, e[1] / L, e[2] / L};
      double w0[3] = {x[0] - A[0], x[1] - A[1], x[2] - A[2]};
      double we = dot3(w, eh), w0e = dot3(w0, eh);
      double wp[3], w0p[3];
      for (int a = 0; a < 3; ++a) {
        wp[a] = w[a] - we * eh[a];
        w0p[a] = w0[a] - w0e * eh[a];
      }
      double qa = dot3(wp, wp);
      if (qa == 0) continue;
      double qb = dot3(w0p, wp), qc = dot3(w0p, w0p) - l * l;
      double disc = qb * qb - qa * qc;
      if (disc < 0) continue;
      double sq = sqrt(disc);
      double ts[2] = {(-qb - sq) / qa, (-qb + sq) / qa};
      for (int r = 0; r < 2; ++r) {
        double t = ts[r];
        if (!(t > 0 && t <= t_max)) continue;
        double along = (w0e + t * we) / L; /* axial parameter on the edge */
        if (!(along >= 0 && along <= 1)) continue;
        double n[3];
        for (int a = 0; a < 3; ++a) n[a] = -(w0p[a] + t * wp[a]) / l;
        hit_push(&C, x, w, t, n, 3);
      }
    }
    for (int64_t v = 0; v < s->nv; ++v) round_candidates(x, w, s->V + 3 * v, l, t_max, 3, &C);
  }
  /* keep the candidates on dR, nearest first */
  hit_list H = {NULL, 0, 0};
  for (int64_t i = 0; i < C.n; ++i) {
    double d, xb[3];
    orc_closest(s, C.h[i].z, 0, &d, xb, NULL);
    if (d >= l * (1 - 1e-9) && orc_inside(s, C.h[i].z) != 0) {
      if (H.n == H.cap) {
        H.cap = H.cap ? 2 * H.cap : 16;
        H.h = (orc_hit*)realloc(H.h, (size_t)H.cap * sizeof(orc_hit));
      }
      H.h[H.n++] = C.h[i];
    }
  }
  if (H.n > 1) qsort(H.h, (size_t)H.n, sizeof(orc_hit), hit_cmp);
  for (int64_t i = 0; i < H.n && i < max_hits; ++i) {
    if (t_out) t_out[i] = H.h[i].t;
    for (int a = 0; a < dim; ++a) {
      if (z_out) z_out[i * dim + a] = H.h[i].z[a];
      if (n_out) n_out[i * dim + a] = H.h[i].n[a];
    }
  }
  int32_t count = (int32_t)H.n;
  free(C.h);
  free(H.h);
  return count;
}

/* Direction of ray j from point k: uniform on the unit circle or sphere from
 * Philox block j, id k, tag 5. */
void orc_ray_direction(uint64_t seed, uint32_t j, uint32_t k, uint32_t batch, int dim, double* w) {
  double ua, ub;
  orc_uniform_pair(seed, j, k, batch, 5, &ua, &ub);
  if (dim == 2) {
    double th = 2 * ORC_PI * ua;
    w[0] = cos(th);
    w[1] = sin(th);
  } else {
    double z = 1 - 2 * ua;
    double rho = sqrt(fmax(0.0, 1 - z * z));
    double ph = 2 * ORC_PI * ub;
    w[0] = rho * cos(ph);
    w[1] = rho * sin(ph);
    w[2] = z;
  }
}

/* Second integral of Eq. 8 at n points inside R: with dG/dn(x, z) dz the
 * signed solid angle that z subtends at x, a uniform ray direction w and the
 * ray's crossings z of dR give the estimate
 *   sum_z sign(dG/dn) max(0, 1 - c/|dG/dn(x, z)|) u(z),
 * averaged over n_rays rays.  Only crossings with |dG/dn| > c contribute;
 * they are ranked h = 0, 1, ... nearest first, a ray keeps max_hits of them,
 * and u at crossing h of ray j of point k is one pointwise walk from it
 * (mode 1, walk id (k n_rays + j) max_hits + h) or, when u_at_hits is not
 * NULL, that field's value (for checks of the ray sampling alone).  Only
 * crossings within orc_clamp_radius can contribute.  stats (optional, 3
 * entries): contributing crossings found, walks run, rays with more than
 * max_hits contributing crossings. */
void orc_clamp_correction(const orc_scene* s, const orc_field* g, const orc_field* f, const orc_walk_params* p,
                          double l, int sides, double c, int32_t n_rays, int32_t max_hits,
                          const orc_field* u_at_hits, int64_t n, const double* x, double* corr, int64_t* stats) {
  int dim = s->dim;
  double t_max = orc_clamp_radius(dim, c);
  const int32_t cap = 1024;
  int64_t found = 0, walks = 0, over = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : found, walks, over)
  for (int64_t k = 0; k < n; ++k) {
    const double* xk = x + k * dim;
    double* tz = (double*)malloc((size_t)cap * (1 + 2 * dim) * sizeof(double));
    double* zz = tz + cap;
    double* nz = zz + (size_t)cap * dim;
    double sum = 0;
    for (int32_t j = 0; j < n_rays; ++j) {
      double w[3];
      orc_ray_direction(p->seed, (uint32_t)j, (uint32_t)k, p->batch, dim, w);
      int32_t nh = orc_offset_hits(s, l, sides, xk, w, t_max, cap, tz, zz, nz);
      int32_t h = 0;
      for (int32_t i = 0; i < nh && i < cap; ++i) {
        const double* z = zz + (size_t)i * dim;
        double dGdn;
        orc_greens(dim, xk, z, nz + (size_t)i * dim, NULL, NULL, &dGdn, NULL);
        double mag = fabs(dGdn);
        if (!(mag > c)) continue;
        ++found;
        if (h >= max_hits) continue;
        double wgt = (dGdn > 0 ? 1.0 : -1.0) * (1 - c / mag);
        double val;
        if (u_at_hits) {
          val = orc_field_eval(u_at_hits, dim, z);
        } else {
          double R0, xb[3], gr[3], ex[3], w1;
          int32_t st, cp;
          orc_closest(s, z, 0, &R0, xb, NULL);
          uint32_t id = (uint32_t)(((int64_t)k * n_rays + j) * max_hits + h);
          orc_walk(s, g, f, p, 1, z, NULL, R0, xb, id, &val, gr, ex, &w1, &st, &cp);
          ++walks;
        }
        sum += wgt * val;
        ++h;
      }
      if (h >= max_hits && nh > 0) {
        /* count the ray when contributing crossings were left out */
        int32_t m = 0;
        for (int32_t i = 0; i < nh && i < cap; ++i) {
          double dGdn;
          orc_greens(dim, xk, zz + (size_t)i * dim, nz + (size_t)i * dim, NULL, NULL, &dGdn, NULL);
          if (fabs(dGdn) > c) ++m;
        }
        if (m > max_hits) ++over;
      }
    }
    corr[k] = sum / n_rays;
    free(tz);
  }
  if (stats) {
    stats[0] = found;
    stats[1] = walks;
    stats[2] = over;
  }
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
