// FP64 CPU oracle of the recursive differentiable transparent-mesh ray tracer.
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
// benchmark's CPU-baseline leg load this library.  It shares no code, header,
// table or helper with the HIP library; both sides only consume the same
// seeded input arrays.
//
// What it computes (paper, Sec. 3.3 "Differentiable Mesh Ray Tracer" and
// Sec. 3.2 "Light Interaction with Transparent Objects"):
//   * vertex normals: one third of the sum of the unit face normals (Eq. 13),
//     blended with the barycentric weights and then normalised (Eq. 12);
//   * closest-hit ray/triangle intersection ("first triangle the ray hits");
//   * recursive tracing to a depth cap: a miss returns the environment
//     radiance, a hit splits into a reflected ray (Eq. 3) and a refracted ray
//     (Eq. 4-6), blended with the Fresnel weights R and T = 1 - R (Eq. 7-8),
//     total internal reflection keeps only the reflected ray, and a hit
//     reached from inside the object is attenuated by exp(-sigma t), the
//     Beer-Lambert integral (Eq. 9-11) for a constant absorption rate, or,
//     for a spatially varying rate mu_t(x) held in a trilinear RGB grid, the
//     sum of mu_t at S midpoints of the segment times the step t / S (the
//     quadrature of Eq. 11);
//   * gradients of the rendered colours with respect to vertex positions,
//     IoR, absorption rate (or grid values) and equirect texels, by plain
//     reverse-mode automatic
//     differentiation (a Wengert tape per camera ray), with the discrete path
//     (triangle ids, TIR branches, hit/miss, env texel cell) held fixed.
//
// Readings where the paper is silent or garbled are listed in the design
// notes; in short: cos(theta_i) = -d.n, eta_r = eta_t/eta_i with ambient IoR
// 1, the blended shading normal is normalised, inside/outside is decided by the geometric
// normal of the hit, a ray hitting at the depth cap contributes 0 and its
// weight is reported as truncated, the environment is at infinity (equirect
// bilinear lookup or a frequency-encoded MLP of the direction).
//
// parity pins: see tests/test_oracle_*.py (closed forms for a glass slab,
// Fresnel textbook values, energy conservation, invisible object at eta = 1,
// brute force vs BVH, central finite differences for every gradient).
//
// Everything is FP64.  The MLP environment is a plain FP64 network: its
// weights are whatever the caller passes (the tests pass the device's bf16
// weights widened exactly), and every activation, product and sum is FP64.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// reverse-mode AD: a Wengert list of binary nodes with local partials
// ---------------------------------------------------------------------------
struct TapeNode {
  int a, b;
  double da, db;
  double v;      // the node's value (used by the rounding-error bound)
  float u;       // relative rounding error its FP32 evaluation may carry
};

struct Tape {
  std::vector<TapeNode> nodes;
  int push(int a, double da, int b, double db, double v, float u) {
    nodes.push_back({a, b, da, db, v, u});
    return (int)nodes.size() - 1;
  }
};

// Relative error charged to one FP32 operation by the rounding-error bound:
// the unit roundoff 2^-24 for correctly rounded arithmetic and square roots,
// twice that for the library functions (exp, atan2, acos, sin, cos, within
// two units in the last place) and for results the other side computes in
// several FP32 steps from exact inputs (a camera ray direction).
constexpr float kU32 = 5.9604644775390625e-08f;
constexpr float kUlp32x2 = 1.1920928955078125e-07f;

thread_local Tape* g_tape = nullptr;

struct Var {
  double v;
  int i;  // tape index, -1 = constant
  Var() : v(0.0), i(-1) {}
  Var(double x) : v(x), i(-1) {}
};

inline Var mk(double v, int a, double da, int b = -1, double db = 0.0, float u = kU32) {
  Var r;
  r.v = v;
  if (a < 0 && b < 0) {
    r.i = -1;
  } else {
    r.i = g_tape->push(a, da, b, db, v, u);
  }
  return r;
}
// An input: exact (u = 0) unless it is itself the result of FP32 arithmetic
// on the other side (a camera ray direction: u = kUlp32x2).
inline Var leaf(double v, float u = 0.0f) {
  Var r;
  r.v = v;
  r.i = g_tape->push(-1, 0.0, -1, 0.0, v, u);
  return r;
}
inline Var operator+(Var x, Var y) { return mk(x.v + y.v, x.i, 1.0, y.i, 1.0); }
inline Var operator-(Var x, Var y) { return mk(x.v - y.v, x.i, 1.0, y.i, -1.0); }
inline Var operator*(Var x, Var y) { return mk(x.v * y.v, x.i, y.v, y.i, x.v); }
inline Var operator/(Var x, Var y) {
  return mk(x.v / y.v, x.i, 1.0 / y.v, y.i, -x.v / (y.v * y.v));
}
inline Var operator-(Var x) { return mk(-x.v, x.i, -1.0); }
inline Var Sqrt(Var x) {
  double s = std::sqrt(x.v);
  return mk(s, x.i, 0.5 / s);
}
inline Var Exp(Var x) {
  double e = std::exp(x.v);
  return mk(e, x.i, e, -1, 0.0, kUlp32x2);
}
inline Var Acos(Var x) {
  double s = std::sqrt(std::max(1.0 - x.v * x.v, 0.0));
  return mk(std::acos(x.v), x.i, -1.0 / s, -1, 0.0, kUlp32x2);
}
inline Var Atan2(Var y, Var x) {
  double r2 = x.v * x.v + y.v * y.v;
  return mk(std::atan2(y.v, x.v), y.i, x.v / r2, x.i, -y.v / r2, kUlp32x2);
}
inline Var Sin(Var x) { return mk(std::sin(x.v), x.i, std::cos(x.v), -1, 0.0, kUlp32x2); }
inline Var Cos(Var x) { return mk(std::cos(x.v), x.i, -std::sin(x.v), -1, 0.0, kUlp32x2); }
inline Var Relu(Var x) { return x.v > 0.0 ? x : Var(0.0); }
inline double val(Var x) { return x.v; }

inline double Sqrt(double x) { return std::sqrt(x); }
inline double Exp(double x) { return std::exp(x); }
inline double Acos(double x) { return std::acos(x); }
inline double Atan2(double y, double x) { return std::atan2(y, x); }
inline double Sin(double x) { return std::sin(x); }
inline double Cos(double x) { return std::cos(x); }
inline double Relu(double x) { return x > 0.0 ? x : 0.0; }
inline double val(double x) { return x; }

template <class S>
struct V3 {
  S x, y, z;
};
template <class S>
inline V3<S> add(V3<S> a, V3<S> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class S>
inline V3<S> sub(V3<S> a, V3<S> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class S>
inline V3<S> scl(V3<S> a, S s) { return {a.x * s, a.y * s, a.z * s}; }
template <class S>
inline S dot(V3<S> a, V3<S> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class S>
inline V3<S> cross(V3<S> a, V3<S> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class S>
inline V3<S> normalize(V3<S> a) {
  S n = Sqrt(dot(a, a));
  return {a.x / n, a.y / n, a.z / n};
}
template <class S>
inline V3<double> vval(V3<S> a) { return {val(a.x), val(a.y), val(a.z)}; }

}  // namespace

extern "C" {

// Environment description.  kind 0 = equirect map [H][W][3], kind 1 = MLP.
typedef struct {
  int kind;
  int W, H;
  const double* tex;        // [H*W*3]
  int n_freq;               // MLP: encoding frequencies (input = 3 + 6 n_freq)
  int n_layers;             // MLP: hidden layers
  int width;                // MLP: hidden width
  int in_pad;               // MLP: padded input width
  const double* weights;    // MLP: concatenated row-major [out][in] per layer
  const double* biases;     // MLP: concatenated per layer
} or_env;

// Spatially varying absorption rate (Eq. 11 and its quadrature): an RGB grid
// of nx*ny*nz nodes, node (i, j, k) at lo + (i/(nx-1), j/(ny-1), k/(nz-1)) *
// (hi - lo), value mu[((k*ny + j)*nx + i)*3 + c]; mu_t(x) is the trilinear
// interpolant at x clamped into the box; an interior segment of length t from
// o along d is attenuated by exp(-(t/S) sum_{s<S} mu_t(o + (s + 1/2)(t/S) d)).
typedef struct {
  const double* mu;
  int nx, ny, nz;  // >= 2 each
  int samples;     // S >= 1
  double lo[3], hi[3];
} or_absorption;

typedef struct {
  const double* V;  // [nv*3]
  int nv;
  const int* F;     // [nf*3]
  int nf;
  double eta;       // IoR of the object (ambient medium 1)
  double sigma[3];  // RGB absorption rate per unit length
  const or_env* env;
  int max_depth;     // D: generations 0..D are intersected; a hit at D is truncated
  int terminal_env;  // 0: truncated hit returns 0; 1: returns A * E(d)
  double t_eps;      // minimum hit distance
  int use_bvh;       // 1: BVH, 0: brute force over all triangles
  const or_absorption* absorb;  // NULL: the constant rate sigma
  const struct or_field* field; // NULL: no volumetric environment field
  // Test instrument, not part of the method (0 = off): every ray the tracer
  // starts (camera rays and every child) has each component of its origin and
  // direction scaled by (1 + jitter xi), xi uniform in [-1, 1) from a
  // counter-based hash of (jitter_seed, ray index, node number).  A parity
  // test measures with it how much a result moves when every ray is rounded
  // the way a float32 evaluation rounds it.
  double jitter;
  uint64_t jitter_seed;
} or_scene;

// Volumetric environment field outside the object (the exterior half of the
// sampling split of Sec. 3.3, a radiance field of a coarse dense grid and
// triplanes as in Sec. 3.1 "Environment Initialization").  Inside the box
// [lo, hi] the feature of a point x is the trilinear interpolant of the grid
// (node (i, j, k) at lo + (i/(nx-1), j/(ny-1), k/(nz-1)) (hi - lo), value
// grid[((k ny + j) nx + i) 4 + ch]) plus the bilinear interpolants of three
// planes of res x res nodes over the box's faces: plane 0 over (x, y), 1 over
// (x, z), 2 over (y, z), node (i, j) of plane p (i along its first axis, j
// along its second) at planes[((p res + j) res + i) 4 + ch].  Channel 0 gives
// the density softplus(f0) = log(1 + e^f0), channels 1-3 the RGB colour.  An
// exterior segment is clipped to the box and sampled at the midpoints of S
// equal steps of length h: alpha_k = 1 - exp(-sigma_k h), transmittance
// T_k = prod_{j<k} (1 - alpha_j), emitted C = sum_k T_k alpha_k c_k, and the
// segment passes T = prod_k (1 - alpha_k) of what lies beyond it.
typedef struct or_field {
  const double* grid;    // [nz][ny][nx][4]
  int nx, ny, nz;        // >= 2 each
  const double* planes;  // [3][res][res][4]
  int res;               // >= 2
  int samples;           // S >= 1
  double lo[3], hi[3];
} or_field;

enum {
  OR_FLAG_DEGEN = 1,    // shading normal on the wrong side, geometric normal used
  OR_FLAG_LEAK = 2,     // a ray inside the object escaped without a hit
  OR_FLAG_GRAZING = 4,  // cos(theta_i) < 0.1 somewhere on the path
  OR_FLAG_TIRB = 8,     // |1 - sin^2 theta_t| < 1e-2 somewhere (TIR boundary)
  OR_FLAG_TRUNC = 16,   // some hit reached the depth cap
  OR_FLAG_KINK = 128,   // an environment lookup within 1e-5 rad of a gradient
                        // discontinuity (bilinear texel-centre line, ReLU kink)
};

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// BVH (binary, median split on the longest centroid axis, <= 4 tris / leaf)
// ---------------------------------------------------------------------------
struct BNode {
  double lo[3], hi[3];
  int left, right;   // children, or -1
  int first, count;  // leaf range into order[]
};

struct BVH {
  std::vector<BNode> nodes;
  std::vector<int> order;
};

void tri_bounds(const or_scene& sc, int f, double lo[3], double hi[3]) {
  for (int k = 0; k < 3; ++k) {
    lo[k] = 1e300;
    hi[k] = -1e300;
  }
  for (int j = 0; j < 3; ++j) {
    const double* p = sc.V + 3 * sc.F[3 * f + j];
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], p[k]);
      hi[k] = std::max(hi[k], p[k]);
    }
  }
}

int build_rec(const or_scene& sc, BVH& b, std::vector<double>& cen, int first, int count) {
  BNode n;
  for (int k = 0; k < 3; ++k) {
    n.lo[k] = 1e300;
    n.hi[k] = -1e300;
  }
  for (int i = first; i < first + count; ++i) {
    double lo[3], hi[3];
    tri_bounds(sc, b.order[i], lo, hi);
    for (int k = 0; k < 3; ++k) {
      n.lo[k] = std::min(n.lo[k], lo[k]);
      n.hi[k] = std::max(n.hi[k], hi[k]);
    }
  }
  // widen each box by a small relative margin so that pruning is conservative
  for (int k = 0; k < 3; ++k) {
    double m = 1e-9 * (std::fabs(n.lo[k]) + std::fabs(n.hi[k])) + 1e-12;
    n.lo[k] -= m;
    n.hi[k] += m;
  }
  n.left = n.right = -1;
  n.first = first;
  n.count = count;
  int idx = (int)b.nodes.size();
  b.nodes.push_back(n);
  if (count <= 4) return idx;
  double clo[3] = {1e300, 1e300, 1e300}, chi[3] = {-1e300, -1e300, -1e300};
  for (int i = first; i < first + count; ++i) {
    for (int k = 0; k < 3; ++k) {
      clo[k] = std::min(clo[k], cen[3 * b.order[i] + k]);
      chi[k] = std::max(chi[k], cen[3 * b.order[i] + k]);
    }
  }
  int ax = 0;
  for (int k = 1; k < 3; ++k)
    if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
  int mid = first + count / 2;
  std::nth_element(b.order.begin() + first, b.order.begin() + mid, b.order.begin() + first + count,
                   [&](int p, int q) {
                     double cp = cen[3 * p + ax], cq = cen[3 * q + ax];
                     return cp < cq || (cp == cq && p < q);
                   });
  int l = build_rec(sc, b, cen, first, mid - first);
  int r = build_rec(sc, b, cen, mid, first + count - mid);
  b.nodes[idx].left = l;
  b.nodes[idx].right = r;
  b.nodes[idx].count = 0;
  return idx;
}

void build_bvh(const or_scene& sc, BVH& b) {
  b.nodes.clear();
  b.order.resize(sc.nf);
  std::vector<double> cen(3 * (size_t)sc.nf);
  for (int f = 0; f < sc.nf; ++f) {
    b.order[f] = f;
    for (int k = 0; k < 3; ++k) {
      double s = 0;
      for (int j = 0; j < 3; ++j) s += sc.V[3 * sc.F[3 * f + j] + k];
      cen[3 * f + k] = s / 3.0;
    }
  }
  if (sc.nf > 0) build_rec(sc, b, cen, 0, sc.nf);
}

// Moller-Trumbore in FP64 with inclusive edges.  Returns true on a hit with
// t > t_eps; outputs t and the barycentric weights of v1 and v2.
bool mt_hit(const or_scene& sc, int f, const double o[3], const double d[3], double& t, double& b1,
            double& b2) {
  const double* v0 = sc.V + 3 * sc.F[3 * f + 0];
  const double* v1 = sc.V + 3 * sc.F[3 * f + 1];
  const double* v2 = sc.V + 3 * sc.F[3 * f + 2];
  V3<double> e1{v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
  V3<double> e2{v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
  V3<double> dd{d[0], d[1], d[2]};
  V3<double> s{o[0] - v0[0], o[1] - v0[1], o[2] - v0[2]};
  V3<double> p = cross(dd, e2);
  double det = dot(e1, p);
  if (det == 0.0) return false;
  double inv = 1.0 / det;
  double u = dot(s, p) * inv;
  if (u < 0.0 || u > 1.0) return false;
  V3<double> q = cross(s, e1);
  double v = dot(dd, q) * inv;
  if (v < 0.0 || u + v > 1.0) return false;
  double tt = dot(e2, q) * inv;
  if (!(tt > sc.t_eps)) return false;
  t = tt;
  b1 = u;
  b2 = v;
  return true;
}

struct Hit {
  int tri = -1;
  double t = 0, b1 = 0, b2 = 0;
};

inline bool better(double t, int f, const Hit& h) {
  return h.tri < 0 || t < h.t || (t == h.t && f < h.tri);
}

Hit closest_brute(const or_scene& sc, const double o[3], const double d[3], int skip) {
  Hit h;
  for (int f = 0; f < sc.nf; ++f) {
    if (f == skip) continue;
    double t, b1, b2;
    if (mt_hit(sc, f, o, d, t, b1, b2) && better(t, f, h)) {
      h.tri = f;
      h.t = t;
      h.b1 = b1;
      h.b2 = b2;
    }
  }
  return h;
}

// slab test; returns entry distance or +inf when the box is missed
double box_enter(const BNode& n, const double o[3], const double d[3], double tmax) {
  double t0 = 0.0, t1 = tmax;
  for (int k = 0; k < 3; ++k) {
    if (d[k] == 0.0) {
      if (o[k] < n.lo[k] || o[k] > n.hi[k]) return INFINITY;
      continue;
    }
    double a = (n.lo[k] - o[k]) / d[k];
    double b = (n.hi[k] - o[k]) / d[k];
    if (a > b) std::swap(a, b);
    t0 = std::max(t0, a);
    t1 = std::min(t1, b);
  }
  return t0 <= t1 ? t0 : INFINITY;
}

Hit closest_bvh(const or_scene& sc, const BVH& b, const double o[3], const double d[3], int skip) {
  Hit h;
  if (b.nodes.empty()) return h;
  int stack[128];
  int sp = 0;
  stack[sp++] = 0;
  while (sp) {
    const BNode& n = b.nodes[stack[--sp]];
    double tmax = h.tri >= 0 ? h.t * (1.0 + 1e-12) : INFINITY;
    if (box_enter(n, o, d, tmax) == INFINITY) continue;
    if (n.left < 0) {
      for (int i = n.first; i < n.first + n.count; ++i) {
        int f = b.order[i];
        if (f == skip) continue;
        double t, b1, b2;
        if (mt_hit(sc, f, o, d, t, b1, b2) && better(t, f, h)) {
          h.tri = f;
          h.t = t;
          h.b1 = b1;
          h.b2 = b2;
        }
      }
    } else {
      stack[sp++] = n.right;
      stack[sp++] = n.left;
    }
  }
  return h;
}

// ---------------------------------------------------------------------------
// per-ray evaluation context
// ---------------------------------------------------------------------------
struct Shared {
  const or_scene* sc;
  BVH bvh;
  std::vector<double> Nv;                 // vertex normals (FP64 values)
  std::vector<std::vector<int>> vfaces;   // vertex -> incident faces (ascending)
};

template <class S>
struct Ctx;

template <>
struct Ctx<double> {
  const Shared* sh;
  double eta;
  double sigma[3];
  V3<double> mu(int node) const {
    const double* m = sh->sc->absorb->mu + 3 * (size_t)node;
    return {m[0], m[1], m[2]};
  }
  V3<double> pos(int v) const {
    const double* p = sh->sc->V + 3 * v;
    return {p[0], p[1], p[2]};
  }
  // field parameter k (grid nodes first, then plane nodes), 4 channels
  void fpar(int64_t k, double* out) const {
    const or_field& f = *sh->sc->field;
    const int64_t ng = (int64_t)f.nx * f.ny * f.nz;
    const double* p = k < ng ? f.grid + 4 * k : f.planes + 4 * (k - ng);
    for (int c = 0; c < 4; ++c) out[c] = p[c];
  }
  V3<double> nrm(int v) {
    const double* p = sh->Nv.data() + 3 * v;
    return {p[0], p[1], p[2]};
  }
};

template <class S>
V3<S> vertex_normal_def(const Shared& sh, int v, Ctx<S>& cx);

template <>
struct Ctx<Var> {
  const Shared* sh;
  Var eta;
  Var sigma[3];
  std::unordered_map<int, V3<Var>> P;   // vertex -> leaf position
  std::unordered_map<int, V3<Var>> N;   // vertex -> normal on the tape
  std::unordered_map<int, V3<Var>> G;   // absorption grid node -> RGB leaf
  std::unordered_map<int64_t, std::array<Var, 4>> FP;  // field parameter -> 4 leaves
  void fpar(int64_t k, Var* out) {
    auto it = FP.find(k);
    if (it == FP.end()) {
      const or_field& f = *sh->sc->field;
      const int64_t ng = (int64_t)f.nx * f.ny * f.nz;
      const double* p = k < ng ? f.grid + 4 * k : f.planes + 4 * (k - ng);
      it = FP.emplace(k, std::array<Var, 4>{leaf(p[0]), leaf(p[1]), leaf(p[2]), leaf(p[3])}).first;
    }
    for (int c = 0; c < 4; ++c) out[c] = it->second[c];
  }
  V3<Var> mu(int node) {
    auto it = G.find(node);
    if (it != G.end()) return it->second;
    const double* m = sh->sc->absorb->mu + 3 * (size_t)node;
    V3<Var> r{leaf(m[0]), leaf(m[1]), leaf(m[2])};
    G.emplace(node, r);
    return r;
  }
  V3<Var> pos(int v) {
    auto it = P.find(v);
    if (it != P.end()) return it->second;
    const double* p = sh->sc->V + 3 * v;
    V3<Var> r{leaf(p[0]), leaf(p[1]), leaf(p[2])};
    P.emplace(v, r);
    return r;
  }
  V3<Var> nrm(int v) {
    auto it = N.find(v);
    if (it != N.end()) return it->second;
    V3<Var> r = vertex_normal_def<Var>(*sh, v, *this);
    N.emplace(v, r);
    return r;
  }
};

// Eq. 13: vertex normal = one third of the sum of the unit normals of the
// faces around the vertex, as written (not renormalised: its length grows
// with the valence and shrinks with the spread of the face normals, and so
// does its weight in the blend of Eq. 12).  Faces of zero area contribute
// nothing.
template <class S>
V3<S> vertex_normal_def(const Shared& sh, int v, Ctx<S>& cx) {
  V3<S> acc{S(0.0), S(0.0), S(0.0)};
  const int* F = sh.sc->F;
  for (int f : sh.vfaces[v]) {
    V3<S> a = cx.pos(F[3 * f]), b = cx.pos(F[3 * f + 1]), c = cx.pos(F[3 * f + 2]);
    V3<S> n = cross(sub(b, a), sub(c, a));
    double len2 = val(dot(n, n));
    if (!(len2 > 0.0)) continue;
    acc = add(acc, normalize(n));
  }
  return scl(acc, S(1.0 / 3.0));
}

// ---------------------------------------------------------------------------
// spatially varying absorption (Eq. 11 with the rate sampled along the segment)
// ---------------------------------------------------------------------------
// Trilinear interpolant of the grid at x.  Per axis the position is mapped to
// grid units u = (x - lo) (n - 1) / (hi - lo); outside [0, n - 1] it is
// clamped (a constant, so no derivative flows through that axis).  The cell is
// chosen from the value (held fixed, like every other discrete choice).
template <class S>
V3<S> grid_mu(Ctx<S>& cx, V3<S> x) {
  const or_absorption& G = *cx.sh->sc->absorb;
  const int n[3] = {G.nx, G.ny, G.nz};
  const S xs[3] = {x.x, x.y, x.z};
  int cell[3];
  S f[3];
  for (int a = 0; a < 3; ++a) {
    const double scale = (double)(n[a] - 1) / (G.hi[a] - G.lo[a]);
    const double u = (val(xs[a]) - G.lo[a]) * scale;
    if (!(u > 0.0)) {
      cell[a] = 0;
      f[a] = S(0.0);
    } else if (!(u < (double)(n[a] - 1))) {
      cell[a] = n[a] - 2;
      f[a] = S(1.0);
    } else {
      cell[a] = std::min((int)std::floor(u), n[a] - 2);
      f[a] = (xs[a] - S(G.lo[a])) * S(scale) - S((double)cell[a]);
    }
  }
  V3<S> acc{S(0.0), S(0.0), S(0.0)};
  for (int c = 0; c < 8; ++c) {
    const int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
    S w = (dx ? f[0] : S(1.0) - f[0]) * (dy ? f[1] : S(1.0) - f[1]) * (dz ? f[2] : S(1.0) - f[2]);
    const int node = ((cell[2] + dz) * G.ny + (cell[1] + dy)) * G.nx + (cell[0] + dx);
    acc = add(acc, scl(cx.mu(node), w));
  }
  return acc;
}

// Optical depth of the segment o + s d, s in [0, t], per channel: the sum of
// mu_t at the midpoints of S equal steps times the step length.
template <class S>
V3<S> grid_tau(Ctx<S>& cx, V3<S> o, V3<S> d, S t) {
  const int ns = cx.sh->sc->absorb->samples;
  const S h = t / S((double)ns);
  V3<S> acc{S(0.0), S(0.0), S(0.0)};
  for (int k = 0; k < ns; ++k) acc = add(acc, grid_mu(cx, add(o, scl(d, h * S(k + 0.5)))));
  return scl(acc, h);
}

// ---------------------------------------------------------------------------
// volumetric environment field (exterior segments)
// ---------------------------------------------------------------------------
inline double Softplus(double x) { return x > 30.0 ? x : std::log1p(std::exp(x)); }
inline Var Softplus(Var x) {
  double e = std::exp(-std::fabs(x.v));
  double v = x.v > 0 ? x.v + std::log1p(e) : std::log1p(std::exp(x.v));
  double dv = 1.0 / (1.0 + std::exp(-x.v));
  return mk(v, x.i, dv, -1, 0.0, kUlp32x2);
}

// Position along one axis in node units u = (x - lo)(n - 1)/(hi - lo), the
// cell (held fixed) and the fraction in it; margin: distance (node units) to
// the nearest cell boundary, less what float32 arithmetic can move u by (x,
// the bounds and the scale each rounded, about 2^-24 (3 |u| + 4 |x| scale)
// in node units, taken 8 times): a sample closer than that to a boundary may
// fall in the other cell in float32, where the field's gradient jumps.
template <class S>
void field_axis(S x, double lo, double hi, int n, int& cell, S& frac, double& margin) {
  const double scale = (double)(n - 1) / (hi - lo);
  const double u = (val(x) - lo) * scale;
  const double slack = 8.0 * 0x1p-24 * (3.0 * std::fabs(u) + 4.0 * std::fabs(val(x)) * scale);
  if (!(u > 0.0)) {
    cell = 0;
    frac = S(0.0);
    margin = 0.0;
  } else if (!(u < (double)(n - 1))) {
    cell = n - 2;
    frac = S(1.0);
    margin = 0.0;
  } else {
    cell = std::min((int)std::floor(u), n - 2);
    frac = (x - S(lo)) * S(scale) - S((double)cell);
    margin = std::min(u - cell, cell + 1 - u) - slack;
  }
}

// Feature (4 channels) at x inside the box; margin: the smallest distance,
// in cell units, from x to a cell boundary of the grid or a plane.
template <class S>
void field_feature(Ctx<S>& cx, V3<S> x, S out[4], double& margin) {
  const or_field& F = *cx.sh->sc->field;
  const S xs[3] = {x.x, x.y, x.z};
  int cg[3];
  S fg[3];
  double mg[3];
  const int n[3] = {F.nx, F.ny, F.nz};
  for (int a = 0; a < 3; ++a) field_axis(xs[a], F.lo[a], F.hi[a], n[a], cg[a], fg[a], mg[a]);
  int cp[3];
  S fp[3];
  double mp[3];
  for (int a = 0; a < 3; ++a) field_axis(xs[a], F.lo[a], F.hi[a], F.res, cp[a], fp[a], mp[a]);
  margin = std::min({mg[0], mg[1], mg[2], mp[0], mp[1], mp[2]});
  for (int c = 0; c < 4; ++c) out[c] = S(0.0);
  S v[4];
  for (int k = 0; k < 8; ++k) {
    const int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
    S w = (dx ? fg[0] : S(1.0) - fg[0]) * (dy ? fg[1] : S(1.0) - fg[1]) * (dz ? fg[2] : S(1.0) - fg[2]);
    const int64_t node = ((int64_t)(cg[2] + dz) * F.ny + (cg[1] + dy)) * F.nx + (cg[0] + dx);
    cx.fpar(node, v);
    for (int c = 0; c < 4; ++c) out[c] = out[c] + w * v[c];
  }
  const int64_t ng = (int64_t)F.nx * F.ny * F.nz;
  const int ax[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  for (int p = 0; p < 3; ++p) {
    const int a = ax[p][0], b = ax[p][1];
    for (int k = 0; k < 4; ++k) {
      const int di = k & 1, dj = k >> 1;
      S w = (di ? fp[a] : S(1.0) - fp[a]) * (dj ? fp[b] : S(1.0) - fp[b]);
      const int64_t node = ng + ((int64_t)p * F.res + (cp[b] + dj)) * F.res + (cp[a] + di);
      cx.fpar(node, v);
      for (int c = 0; c < 4; ++c) out[c] = out[c] + w * v[c];
    }
  }
}

// Emission C and transmittance T of the exterior segment o + s d, s in
// [0, t_end] (t_end = +inf for a ray that leaves), clipped to the field's
// box.  The clip distances depend on o and d (and t_end); which box faces
// clip is a discrete choice held fixed.  kink: set when a sample lies within
// 1e-5 cell units, beyond the float32 slack of field_axis, of a cell boundary
// (the field's gradient jumps there).
template <class S>
void field_segment(Ctx<S>& cx, V3<S> o, V3<S> d, S t_end, bool open, V3<S>& C, S& T, bool& kink) {
  const or_field& F = *cx.sh->sc->field;
  C = {S(0.0), S(0.0), S(0.0)};
  T = S(1.0);
  const S os[3] = {o.x, o.y, o.z}, ds[3] = {d.x, d.y, d.z};
  S s0 = S(0.0), s1 = t_end;
  bool have1 = !open;
  for (int a = 0; a < 3; ++a) {
    if (val(ds[a]) == 0.0) {
      if (val(os[a]) < F.lo[a] || val(os[a]) > F.hi[a]) return;
      continue;
    }
    S ta = (S(F.lo[a]) - os[a]) / ds[a], tb = (S(F.hi[a]) - os[a]) / ds[a];
    if (val(ta) > val(tb)) std::swap(ta, tb);
    if (val(ta) > val(s0)) s0 = ta;
    if (!have1 || val(tb) < val(s1)) {
      s1 = tb;
      have1 = true;
    }
  }
  if (!(val(s1) > val(s0))) return;
  const int ns = F.samples;
  const S h = (s1 - s0) / S((double)ns);
  S trans = S(1.0);
  for (int k = 0; k < ns; ++k) {
    V3<S> x = add(o, scl(d, s0 + h * S(k + 0.5)));
    S f[4];
    double margin;
    field_feature(cx, x, f, margin);
    if (margin < 1e-5) kink = true;
    S a = Exp(-(Softplus(f[0]) * h));   // 1 - alpha_k
    S w = trans * (S(1.0) - a);
    C = add(C, V3<S>{w * f[1], w * f[2], w * f[3]});
    trans = trans * a;
  }
  T = trans;
}

// ---------------------------------------------------------------------------
// environment
// ---------------------------------------------------------------------------
struct EnvOut {
  int cell_x, cell_y;  // discrete texel cell (for path signatures)
  double kink = 1e300; // angular distance (rad, first order) to the nearest
                       // direction where the lookup's gradient jumps
};

// Texel values of the equirect map.  For the gradient pass, g_texleaf (when
// set) maps a texel to its three channels as tape leaves, so the lookup is
// differentiable in the texels too.
thread_local std::unordered_map<int, V3<Var>>* g_texleaf = nullptr;
template <class S>
S tex_value(const or_env& e, int r, int c, int ch);
template <>
inline double tex_value<double>(const or_env& e, int r, int c, int ch) {
  return e.tex[((size_t)r * e.W + c) * 3 + ch];
}
template <>
inline Var tex_value<Var>(const or_env& e, int r, int c, int ch) {
  const double* p = e.tex + ((size_t)r * e.W + c) * 3;
  if (!g_texleaf) return Var(p[ch]);
  auto it = g_texleaf->find(r * e.W + c);
  if (it == g_texleaf->end())
    it = g_texleaf->emplace(r * e.W + c, V3<Var>{leaf(p[0]), leaf(p[1]), leaf(p[2])}).first;
  return ch == 0 ? it->second.x : (ch == 1 ? it->second.y : it->second.z);
}

// Equirect lookup at a direction (normalised first): phi = atan2(x, -z), theta = acos(y),
// u = phi / 2pi + 1/2, v = theta / pi, texel coords (uW - 1/2, vH - 1/2),
// bilinear, wrapping in u and clamping in v, row 0 at the zenith.
template <class S>
V3<S> env_equirect(const or_env& e, V3<S> dir, EnvOut& eo) {
  const double PI = 3.14159265358979323846;
  // the environment is a function of direction only
  V3<S> d = normalize(dir);
  S y = d.y;
  if (val(y) > 1.0) y = S(1.0);
  if (val(y) < -1.0) y = S(-1.0);
  S phi = Atan2(d.x, -d.z);
  S th = Acos(y);
  S u = phi / S(2.0 * PI) + S(0.5);
  S v = th / S(PI);
  S x = u * S((double)e.W) - S(0.5);
  S yy = v * S((double)e.H) - S(0.5);
  double x0 = std::floor(val(x)), y0 = std::floor(val(yy));
  S fx = x - S(x0), fy = yy - S(y0);
  long ix0 = (long)x0, iy0 = (long)y0;
  eo.cell_x = (int)ix0;
  eo.cell_y = (int)iy0;
  {
    // bilinear weights change slope on texel-centre lines: distance to the
    // nearest one along phi (scaled by sin theta) and along theta
    double fxv = val(x) - x0, fyv = val(yy) - y0;
    double st = std::sqrt(std::max(1.0 - val(y) * val(y), 0.0));
    double dphi = std::min(fxv, 1.0 - fxv) * 2.0 * PI / e.W * st;
    double dth = std::min(fyv, 1.0 - fyv) * PI / e.H;
    eo.kink = std::min(dphi, dth);
  }
  auto wrapx = [&](long i) { return (int)(((i % e.W) + e.W) % e.W); };
  auto clampy = [&](long i) { return (int)std::min<long>(std::max<long>(i, 0), e.H - 1); };
  int xa = wrapx(ix0), xb = wrapx(ix0 + 1);
  int ya = clampy(iy0), yb = clampy(iy0 + 1);
  auto T = [&](int r, int c, int ch) { return tex_value<S>(e, r, c, ch); };
  S w00 = (S(1.0) - fx) * (S(1.0) - fy), w01 = fx * (S(1.0) - fy);
  S w10 = (S(1.0) - fx) * fy, w11 = fx * fy;
  V3<S> out;
  S* o[3] = {&out.x, &out.y, &out.z};
  for (int ch = 0; ch < 3; ++ch)
    *o[ch] = w00 * T(ya, xa, ch) + w01 * T(ya, xb, ch) + w10 * T(yb, xa, ch) + w11 * T(yb, xb, ch);
  return out;
}

// MLP environment (env_mlp below): gamma(d) = [d, sin(2^k pi d), cos(2^k pi d)]
// for k < n_freq, zero-padded; hidden layers with ReLU; linear RGB head; plain
// FP64 throughout (the weights are whatever the caller gives).
//
// Smallest first-order angular distance to a ReLU kink: for every hidden
// pre-activation z, |z| / |dz/du| with u the unit direction (the network is
// piecewise smooth in u; its gradient jumps where a z changes sign).
double mlp_kink_margin(const or_env& e, V3<double> d) {
  const double PI = 3.14159265358979323846;
  V3<double> u = normalize(d);
  double uc[3] = {u.x, u.y, u.z};
  int in = e.in_pad;
  std::vector<double> h((size_t)in, 0.0), J((size_t)in * 3, 0.0);
  int k = 0;
  for (int c = 0; c < 3; ++c) {
    h[k] = uc[c];
    J[3 * k + c] = 1.0;
    ++k;
  }
  for (int f = 0; f < e.n_freq; ++f) {
    double w = std::ldexp(PI, f);
    for (int c = 0; c < 3; ++c) {
      h[k] = std::sin(w * uc[c]);
      J[3 * k + c] = w * std::cos(w * uc[c]);
      ++k;
    }
    for (int c = 0; c < 3; ++c) {
      h[k] = std::cos(w * uc[c]);
      J[3 * k + c] = -w * std::sin(w * uc[c]);
      ++k;
    }
  }
  double margin = 1e300;
  const double* W = e.weights;
  const double* B = e.biases;
  for (int l = 0; l < e.n_layers; ++l) {
    int out = e.width;
    std::vector<double> z((size_t)out), Jz((size_t)out * 3);
    for (int j = 0; j < out; ++j) {
      double acc = B[j], g0 = 0, g1 = 0, g2 = 0;
      for (int i = 0; i < in; ++i) {
        double w = W[(size_t)j * in + i];
        acc += w * h[i];
        g0 += w * J[3 * i];
        g1 += w * J[3 * i + 1];
        g2 += w * J[3 * i + 2];
      }
      // only the tangential part of the gradient moves z along the sphere
      double gu = g0 * u.x + g1 * u.y + g2 * u.z;
      g0 -= gu * u.x;
      g1 -= gu * u.y;
      g2 -= gu * u.z;
      double gn = std::sqrt(g0 * g0 + g1 * g1 + g2 * g2);
      if (gn > 0) margin = std::min(margin, std::fabs(acc) / gn);
      z[j] = acc;
      Jz[3 * j] = g0;
      Jz[3 * j + 1] = g1;
      Jz[3 * j + 2] = g2;
    }
    h.assign((size_t)out, 0.0);
    J.assign((size_t)out * 3, 0.0);
    for (int j = 0; j < out; ++j)
      if (z[j] > 0) {
        h[j] = z[j];
        J[3 * j] = Jz[3 * j];
        J[3 * j + 1] = Jz[3 * j + 1];
        J[3 * j + 2] = Jz[3 * j + 2];
      }
    W += (size_t)out * in;
    B += out;
    in = out;
  }
  return margin;
}

// Total number of MLP parameters (weights, then biases, in the layout of or_env).
inline size_t mlp_param_count(const or_env& e) {
  size_t nw = (size_t)e.width * e.in_pad, nb = (size_t)e.width;
  for (int l = 1; l < e.n_layers; ++l) {
    nw += (size_t)e.width * e.width;
    nb += (size_t)e.width;
  }
  nw += 3 * (size_t)e.width;
  nb += 3;
  return nw + nb;
}
inline size_t mlp_weight_count(const or_env& e) {
  size_t nw = (size_t)e.width * e.in_pad;
  for (int l = 1; l < e.n_layers; ++l) nw += (size_t)e.width * e.width;
  return nw + 3 * (size_t)e.width;
}

// For the gradient pass: when set, the network's weights and biases are tape
// leaves (created on first use for the current camera ray, weights first,
// then biases), so every lookup is differentiable in them too.
thread_local std::vector<Var>* g_mlpleaf = nullptr;
template <class S>
S mlp_param(const or_env& e, size_t k);
template <>
inline double mlp_param<double>(const or_env& e, size_t k) {
  size_t nw = mlp_weight_count(e);
  return k < nw ? e.weights[k] : e.biases[k - nw];
}
template <>
inline Var mlp_param<Var>(const or_env& e, size_t k) {
  size_t nw = mlp_weight_count(e);
  double v = k < nw ? e.weights[k] : e.biases[k - nw];
  if (!g_mlpleaf) return Var(v);
  if (g_mlpleaf->empty()) {
    size_t np = mlp_param_count(e);
    g_mlpleaf->reserve(np);
    for (size_t j = 0; j < np; ++j)
      g_mlpleaf->push_back(leaf(j < nw ? e.weights[j] : e.biases[j - nw]));
  }
  return (*g_mlpleaf)[k];
}

template <class S>
V3<S> env_mlp(const or_env& e, V3<S> dir, EnvOut& eo) {
  const double PI = 3.14159265358979323846;
  V3<S> d = normalize(dir);
  eo.cell_x = eo.cell_y = 0;
  eo.kink = mlp_kink_margin(e, vval(dir));
  std::vector<S> h((size_t)e.in_pad, S(0.0));
  S dc[3] = {d.x, d.y, d.z};
  int k = 0;
  for (int c = 0; c < 3; ++c) h[k++] = dc[c];
  for (int f = 0; f < e.n_freq; ++f) {
    double w = std::ldexp(PI, f);
    for (int c = 0; c < 3; ++c) h[k++] = Sin(S(w) * dc[c]);
    for (int c = 0; c < 3; ++c) h[k++] = Cos(S(w) * dc[c]);
  }
  // parameter k of the flat list: weights of all layers, then their biases
  const size_t nw = mlp_weight_count(e);
  size_t wo = 0, bo = nw;
  int in = e.in_pad;
  for (int l = 0; l <= e.n_layers; ++l) {
    int out = l < e.n_layers ? e.width : 3;
    std::vector<S> z((size_t)out);
    for (int j = 0; j < out; ++j) {
      S acc = mlp_param<S>(e, bo + j);
      for (int i = 0; i < in; ++i) acc = acc + mlp_param<S>(e, wo + (size_t)j * in + i) * h[i];
      if (l < e.n_layers)
        z[j] = Relu(acc);
      else
        z[j] = acc;
    }
    wo += (size_t)out * in;
    bo += out;
    h.swap(z);
    in = out;
  }
  return {h[0], h[1], h[2]};
}

template <class S>
V3<S> env_eval(const or_env& e, V3<S> d, EnvOut& eo) {
  return e.kind == 0 ? env_equirect(e, d, eo) : env_mlp(e, d, eo);
}

// ---------------------------------------------------------------------------
// recursive tracer
// ---------------------------------------------------------------------------
// SplitMix64 output function (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014), used as a 64-bit mixer.
inline uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct PathInfo {
  int flags = 0;
  uint64_t jkey = 0;  // jitter stream of this camera ray, and rays started so far
  uint64_t jn = 0;
  void start(const or_scene* sc, int64_t ray) {
    jkey = splitmix64(sc->jitter_seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(ray + 1)));
  }
  double wtrunc[3] = {0, 0, 0};
  int nseg = 0;
  // order-independent signature of the discrete path: the sum (mod 2^64) over
  // the tree's segments of a mix of (generation, triangle hit or -1, TIR)
  uint64_t sig = 0;
  void node(int g, int tri, bool tir) {
    uint64_t key = ((uint64_t)(uint32_t)g << 40) | ((uint64_t)(tir ? 1u : 0u) << 32) |
                   (uint64_t)(uint32_t)(tri + 1);
    sig += splitmix64(key);
  }
  uint64_t hash = 1469598103934665603ull;
  void mix(uint64_t x) {
    for (int i = 0; i < 8; ++i) {
      hash ^= (x >> (8 * i)) & 0xFF;
      hash *= 1099511628211ull;
    }
  }
};

struct TreeRec {
  double depth, kind, tri;   // kind 0 miss, 1 hit, 2 truncated
  double o[3], d[3], W[3];
  double R, T, A[3], t, entering, tir, cos_i;
  double E[3];
};

template <class S>
V3<S> trace(Ctx<S>& cx, V3<S> o, V3<S> d, int skip, int g, const double W[3], bool inside,
            PathInfo& pi, std::vector<TreeRec>* tree) {
  const Shared& sh = *cx.sh;
  const or_scene& sc = *sh.sc;
  pi.nseg++;
  if (sc.jitter > 0.0) {
    const uint64_t b = splitmix64(pi.jkey + 0x632BE59BD9B4E019ull * ++pi.jn);
    double xi[6];
    for (int k = 0; k < 6; ++k)
      xi[k] = 1.0 + sc.jitter * ((double)(splitmix64(b + (uint64_t)k) >> 11) * 0x1.0p-52 - 1.0);
    o = {o.x * S(xi[0]), o.y * S(xi[1]), o.z * S(xi[2])};
    d = {d.x * S(xi[3]), d.y * S(xi[4]), d.z * S(xi[5])};
  }
  double od[3] = {val(o.x), val(o.y), val(o.z)}, dd[3] = {val(d.x), val(d.y), val(d.z)};
  Hit h = sc.use_bvh ? closest_bvh(sc, sh.bvh, od, dd, skip) : closest_brute(sc, od, dd, skip);
  TreeRec rec{};
  if (tree) {
    rec.depth = g;
    rec.tri = h.tri;
    for (int k = 0; k < 3; ++k) {
      rec.o[k] = od[k];
      rec.d[k] = dd[k];
      rec.W[k] = W[k];
    }
  }
  if (h.tri < 0) {
    // Procedure step 3: no hit -> radiance from the environment.
    if (inside) pi.flags |= OR_FLAG_LEAK;
    EnvOut eo;
    V3<S> E = env_eval(*sc.env, d, eo);
    pi.mix(0xE0000000ull ^ ((uint64_t)(uint32_t)eo.cell_x << 16) ^ (uint64_t)(uint32_t)eo.cell_y);
    pi.node(g, -1, false);
    if (eo.kink < 1e-5) pi.flags |= OR_FLAG_KINK;
    if (tree) {
      rec.kind = 0;
      rec.E[0] = val(E.x);
      rec.E[1] = val(E.y);
      rec.E[2] = val(E.z);
      tree->push_back(rec);
    }
    if (sc.field && !inside) {
      // the exterior segment to the field's far side, then the environment
      V3<S> Cf;
      S Tf;
      bool kink = false;
      field_segment(cx, o, d, S(INFINITY), true, Cf, Tf, kink);
      if (kink) pi.flags |= OR_FLAG_KINK;
      return add(Cf, scl(E, Tf));
    }
    return E;
  }
  const int* F = sc.F;
  int i0 = F[3 * h.tri], i1 = F[3 * h.tri + 1], i2 = F[3 * h.tri + 2];
  V3<S> v0 = cx.pos(i0), v1 = cx.pos(i1), v2 = cx.pos(i2);
  // differentiable intersection: Moller-Trumbore on the tape, so t and the
  // barycentrics depend on the ray and the three vertices
  V3<S> e1 = sub(v1, v0), e2 = sub(v2, v0), s = sub(o, v0);
  V3<S> p = cross(d, e2);
  S det = dot(e1, p);
  S inv = S(1.0) / det;
  V3<S> q = cross(s, e1);
  S b1 = dot(s, p) * inv;
  S b2 = dot(d, q) * inv;
  S t = dot(e2, q) * inv;
  S b0 = S(1.0) - b1 - b2;
  V3<S> x = add(o, scl(d, t));
  V3<S> ng = cross(e1, e2);
  // Procedure step 2: outside / inside by the geometric normal of the hit
  bool entering = val(dot(d, ng)) < 0.0;
  // Eq. 12: shading normal = barycentric blend of the vertex normals of Eq. 13,
  // normalised for Eq. 3-6
  V3<S> m = add(add(scl(cx.nrm(i0), b0), scl(cx.nrm(i1), b1)), scl(cx.nrm(i2), b2));
  V3<S> n = normalize(m);
  if (!entering) n = scl(n, S(-1.0));
  S cos_i = -dot(d, n);
  if (!(val(cos_i) > 0.0)) {
    pi.flags |= OR_FLAG_DEGEN;
    n = normalize(ng);
    if (!entering) n = scl(n, S(-1.0));
    cos_i = -dot(d, n);
  }
  // grazing / TIR-boundary markers: either cosine below 0.1, where the Fresnel
  // and refraction derivatives (which scale like 1/cos) are ill-conditioned
  if (val(cos_i) < 0.1) pi.flags |= OR_FLAG_GRAZING;
  // eta_r = eta_t / eta_i, ambient medium 1
  S eta_i = entering ? S(1.0) : cx.eta;
  S eta_t = entering ? cx.eta : S(1.0);
  S eta_r = eta_t / eta_i;
  // Procedure step 5 / Eq. 11: attenuation over the interior segment just
  // travelled (the ray hit the surface from inside)
  V3<S> A{S(1.0), S(1.0), S(1.0)};
  // emission of the exterior segment just travelled (volumetric field)
  V3<S> Cem{S(0.0), S(0.0), S(0.0)};
  if (!entering) {
    if (sc.absorb) {
      V3<S> tau = grid_tau(cx, o, d, t);
      A = {Exp(-tau.x), Exp(-tau.y), Exp(-tau.z)};
    } else {
      A = {Exp(-cx.sigma[0] * t), Exp(-cx.sigma[1] * t), Exp(-cx.sigma[2] * t)};
    }
  } else if (sc.field) {
    // Procedure step 4: the radiance beyond the hit is mixed with the
    // environment field sampled before it
    S Tf;
    bool kink = false;
    field_segment(cx, o, d, t, false, Cem, Tf, kink);
    if (kink) pi.flags |= OR_FLAG_KINK;
    A = {Tf, Tf, Tf};
  }
  double Av[3] = {val(A.x), val(A.y), val(A.z)};
  if (tree) {
    rec.t = val(t);
    rec.entering = entering;
    rec.cos_i = val(cos_i);
    for (int k = 0; k < 3; ++k) rec.A[k] = Av[k];
  }
  // Procedure step 1: the depth cap
  if (g >= sc.max_depth) {
    pi.flags |= OR_FLAG_TRUNC;
    for (int k = 0; k < 3; ++k) pi.wtrunc[k] += W[k] * Av[k];
    pi.mix(0x70000000ull ^ (uint64_t)h.tri);
    pi.node(g, h.tri, false);
    if (tree) {
      rec.kind = 2;
      tree->push_back(rec);
    }
    if (sc.terminal_env) {
      EnvOut eo;
      V3<S> E = env_eval(*sc.env, d, eo);
      return add(Cem, V3<S>{A.x * E.x, A.y * E.y, A.z * E.z});
    }
    return Cem;
  }
  // Snell: sin^2(theta_t) = sin^2(theta_i) / eta_r^2
  S sin2t = (S(1.0) - cos_i * cos_i) / (eta_r * eta_r);
  if (std::fabs(1.0 - val(sin2t)) < 1e-2) pi.flags |= OR_FLAG_TIRB;
  // Eq. 3 with omega_i = -d
  V3<S> rdir = normalize(add(d, scl(n, S(2.0) * cos_i)));
  bool tir = val(sin2t) > 1.0;
  pi.mix(((uint64_t)h.tri << 2) ^ (tir ? 1u : 0u) ^ (entering ? 2u : 0u));
  pi.node(g, h.tri, tir);
  // the child that continues on the same side of the surface as the parent
  // stays outside/inside accordingly
  bool r_inside = !entering, t_inside = entering;
  if (tir) {
    // total internal reflection: reflection only, R = 1
    if (tree) {
      rec.kind = 1;
      rec.R = 1.0;
      rec.T = 0.0;
      rec.tir = 1;
      tree->push_back(rec);
    }
    double Wr[3] = {W[0] * Av[0], W[1] * Av[1], W[2] * Av[2]};
    V3<S> Lr = trace(cx, x, rdir, h.tri, g + 1, Wr, r_inside, pi, tree);
    return add(Cem, V3<S>{A.x * Lr.x, A.y * Lr.y, A.z * Lr.z});
  }
  S cos_t = Sqrt(S(1.0) - sin2t);
  // Eq. 7-8
  S rs = (eta_i * cos_i - eta_t * cos_t) / (eta_i * cos_i + eta_t * cos_t);
  S rp = (eta_i * cos_t - eta_t * cos_i) / (eta_i * cos_t + eta_t * cos_i);
  S R = S(0.5) * (rs * rs + rp * rp);
  S T = S(1.0) - R;
  // Eq. 4-6 with omega_i = -d: omega_t = d/eta_r + (cos_i/eta_r - cos_t) n
  V3<S> tdir = normalize(add(scl(d, S(1.0) / eta_r), scl(n, cos_i / eta_r - cos_t)));
  if (tree) {
    rec.kind = 1;
    rec.R = val(R);
    rec.T = val(T);
    rec.tir = 0;
    tree->push_back(rec);
  }
  double Wr[3], Wt[3];
  for (int k = 0; k < 3; ++k) {
    Wr[k] = W[k] * Av[k] * val(R);
    Wt[k] = W[k] * Av[k] * val(T);
  }
  // Procedure step 4: trace both children and blend with R and T
  V3<S> Lr = trace(cx, x, rdir, h.tri, g + 1, Wr, r_inside, pi, tree);
  V3<S> Lt = trace(cx, x, tdir, h.tri, g + 1, Wt, t_inside, pi, tree);
  return add(Cem, V3<S>{A.x * (R * Lr.x + T * Lt.x), A.y * (R * Lr.y + T * Lt.y),
                        A.z * (R * Lr.z + T * Lt.z)});
}

void make_shared(const or_scene* sc, Shared& sh, bool need_normals) {
  sh.sc = sc;
  if (sc->use_bvh) build_bvh(*sc, sh.bvh);
  sh.vfaces.assign(sc->nv, {});
  for (int f = 0; f < sc->nf; ++f)
    for (int j = 0; j < 3; ++j) sh.vfaces[sc->F[3 * f + j]].push_back(f);
  if (need_normals) {
    sh.Nv.assign(3 * (size_t)sc->nv, 0.0);
    Ctx<double> cx{&sh, sc->eta, {sc->sigma[0], sc->sigma[1], sc->sigma[2]}};
    for (int v = 0; v < sc->nv; ++v) {
      V3<double> n = vertex_normal_def<double>(sh, v, cx);
      sh.Nv[3 * v] = n.x;
      sh.Nv[3 * v + 1] = n.y;
      sh.Nv[3 * v + 2] = n.z;
    }
  }
}

bool valid_scene(const or_scene* sc) {
  if (!sc || !sc->V || !sc->F || !sc->env || sc->nv <= 0 || sc->nf <= 0) return false;
  if (sc->max_depth < 0 || sc->max_depth > 30) return false;
  if (!(sc->jitter >= 0.0 && sc->jitter <= 1e-3)) return false;
  if (const or_absorption* G = sc->absorb) {
    if (!G->mu || G->nx < 2 || G->ny < 2 || G->nz < 2 || G->samples < 1) return false;
    for (int a = 0; a < 3; ++a)
      if (!(G->hi[a] > G->lo[a])) return false;
  }
  if (const or_field* Fd = sc->field) {
    if (!Fd->grid || !Fd->planes || Fd->nx < 2 || Fd->ny < 2 || Fd->nz < 2 || Fd->res < 2 ||
        Fd->samples < 1)
      return false;
    for (int a = 0; a < 3; ++a)
      if (!(Fd->hi[a] > Fd->lo[a])) return false;
  }
  for (int i = 0; i < 3 * sc->nf; ++i)
    if (sc->F[i] < 0 || sc->F[i] >= sc->nv) return false;
  return true;
}

}  // namespace

extern "C" {

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Vertex normals (Eq. 12-13).  N: [nv*3].
int or_vertex_normals(const double* V, int nv, const int* F, int nf, double* N) {
  or_env dummy{};
  or_scene sc{};
  sc.V = V;
  sc.nv = nv;
  sc.F = F;
  sc.nf = nf;
  sc.env = &dummy;
  if (!valid_scene(&sc)) return 1;
  Shared sh;
  make_shared(&sc, sh, true);
  std::memcpy(N, sh.Nv.data(), sizeof(double) * 3 * (size_t)nv);
  return 0;
}

// Pinhole camera rays: eye, target, up hint, vertical FOV in degrees;
// right-handed, image row 0 at the top, rays through pixel centres.
// o, d: [W*H*3], pixel index = y*W + x.
int or_camera_rays(const double* cam, int W, int H, double* o, double* d) {
  const double PI = 3.14159265358979323846;
  V3<double> eye{cam[0], cam[1], cam[2]}, tgt{cam[3], cam[4], cam[5]}, up{cam[6], cam[7], cam[8]};
  V3<double> f = normalize(sub(tgt, eye));
  V3<double> r = normalize(cross(f, up));
  V3<double> u = cross(r, f);
  double th = std::tan(0.5 * cam[9] * PI / 180.0);
  double aspect = (double)W / (double)H;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      double px = (2.0 * (x + 0.5) / W - 1.0) * th * aspect;
      double py = (1.0 - 2.0 * (y + 0.5) / H) * th;
      V3<double> dd = normalize(add(f, add(scl(r, px), scl(u, py))));
      size_t i = (size_t)y * W + x;
      o[3 * i] = eye.x;
      o[3 * i + 1] = eye.y;
      o[3 * i + 2] = eye.z;
      d[3 * i] = dd.x;
      d[3 * i + 1] = dd.y;
      d[3 * i + 2] = dd.z;
    }
  return 0;
}

// Closest hit for n rays (skip[i] = triangle to ignore, -1 for none).
int or_intersect(const or_scene* sc, const double* o, const double* d, const int* skip, int64_t n,
                 int* tri, double* t, double* b1, double* b2) {
  if (!valid_scene(sc)) return 1;
  Shared sh;
  make_shared(sc, sh, false);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    int sk = skip ? skip[i] : -1;
    Hit h = sc->use_bvh ? closest_bvh(*sc, sh.bvh, o + 3 * i, d + 3 * i, sk)
                        : closest_brute(*sc, o + 3 * i, d + 3 * i, sk);
    tri[i] = h.tri;
    t[i] = h.t;
    b1[i] = h.b1;
    b2[i] = h.b2;
  }
  return 0;
}

// Environment radiance for n unit directions.  cell: [n*2] texel cell or NULL.
int or_env_eval(const or_env* env, const double* dirs, int64_t n, double* rgb) {
  if (!env) return 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    EnvOut eo;
    V3<double> d{dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2]};
    V3<double> e = env_eval<double>(*env, d, eo);
    rgb[3 * i] = e.x;
    rgb[3 * i + 1] = e.y;
    rgb[3 * i + 2] = e.z;
  }
  return 0;
}

// Angular distance (radians, first order) from each direction to the nearest
// direction where the environment's gradient jumps (texel-centre line of the
// bilinear map, zero of a hidden pre-activation of the MLP).
int or_env_kink_margin(const or_env* env, const double* dirs, int64_t n, double* margin) {
  if (!env) return 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    EnvOut eo;
    V3<double> d{dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2]};
    env_eval<double>(*env, d, eo);
    margin[i] = eo.kink;
  }
  return 0;
}

// Gradient of sum(grad_rgb * E(dirs)) with respect to the directions.
int or_env_eval_grad(const or_env* env, const double* dirs, int64_t n, const double* grad_rgb,
                     double* grad_dirs) {
  if (!env) return 1;
#pragma omp parallel
  {
    Tape tape;
    g_tape = &tape;
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      tape.nodes.clear();
      EnvOut eo;
      V3<Var> d{leaf(dirs[3 * i]), leaf(dirs[3 * i + 1]), leaf(dirs[3 * i + 2])};
      V3<Var> e = env_eval<Var>(*env, d, eo);
      std::vector<double> adj(tape.nodes.size(), 0.0);
      if (e.x.i >= 0) adj[e.x.i] += grad_rgb[3 * i];
      if (e.y.i >= 0) adj[e.y.i] += grad_rgb[3 * i + 1];
      if (e.z.i >= 0) adj[e.z.i] += grad_rgb[3 * i + 2];
      for (int k = (int)tape.nodes.size() - 1; k >= 0; --k) {
        double a = adj[k];
        if (a == 0.0) continue;
        const TapeNode& tn = tape.nodes[k];
        if (tn.a >= 0) adj[tn.a] += tn.da * a;
        if (tn.b >= 0) adj[tn.b] += tn.db * a;
      }
      grad_dirs[3 * i] = adj[d.x.i];
      grad_dirs[3 * i + 1] = adj[d.y.i];
      grad_dirs[3 * i + 2] = adj[d.z.i];
    }
    g_tape = nullptr;
  }
  return 0;
}

// Forward render of n camera rays (o, d unit).  Outputs per ray: rgb [n*3],
// truncated weight [n*3], flags [n], path signature hash [n], segment count [n].
// Any output pointer may be NULL.
int or_trace(const or_scene* sc, const double* o, const double* d, int64_t n, double* rgb,
             double* wtrunc, int* flags, uint64_t* hash, int* nseg, uint64_t* sig) {
  if (!valid_scene(sc)) return 1;
  Shared sh;
  make_shared(sc, sh, true);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    Ctx<double> cx{&sh, sc->eta, {sc->sigma[0], sc->sigma[1], sc->sigma[2]}};
    PathInfo pi;
    pi.start(sc, i);
    double W[3] = {1, 1, 1};
    V3<double> oo{o[3 * i], o[3 * i + 1], o[3 * i + 2]}, dd{d[3 * i], d[3 * i + 1], d[3 * i + 2]};
    V3<double> L = trace<double>(cx, oo, dd, -1, 0, W, false, pi, nullptr);
    if (rgb) {
      rgb[3 * i] = L.x;
      rgb[3 * i + 1] = L.y;
      rgb[3 * i + 2] = L.z;
    }
    if (wtrunc)
      for (int k = 0; k < 3; ++k) wtrunc[3 * i + k] = pi.wtrunc[k];
    if (flags) flags[i] = pi.flags;
    if (hash) hash[i] = pi.hash;
    if (nseg) nseg[i] = pi.nseg;
    if (sig) sig[i] = pi.sig;
  }
  return 0;
}

// Forward + reverse-mode gradient.  The scalar loss is sum_i grad_rgb[i] . C_i.
// dV [nv*3], d_eta [1], d_sigma [3] are overwritten, and with an absorption
// grid d_mu [nx*ny*nz*3] too (sigma then has no effect and d_sigma is 0), for
// an equirect environment d_tex [H*W*3], for an MLP environment d_mlp
// (every weight, then every bias, in the order of or_env), and with a
// volumetric field d_field (grid nodes, then plane nodes, 4 channels each).
// rgb, d_mu, d_tex, d_mlp and d_field may be NULL.  absolute = 1: every output is instead the sum over
// camera rays of the magnitude of each ray's contribution (the scale against
// which a sum that cancels is compared).
int or_trace_grad(const or_scene* sc, const double* o, const double* d, int64_t n,
                  const double* grad_rgb, double* rgb, double* dV, double* d_eta,
                  double* d_sigma, double* d_mu, double* d_tex, double* d_mlp, double* d_field,
                  int absolute) {
  if (!valid_scene(sc)) return 1;
  Shared sh;
  make_shared(sc, sh, true);
  int nth = 1;
#ifdef _OPENMP
  nth = omp_get_max_threads();
#endif
  std::vector<std::vector<double>> accV(nth);
  std::vector<double> accE(nth, 0.0), accS(3 * (size_t)nth, 0.0);
  const size_t nmu = sc->absorb ? 3 * (size_t)sc->absorb->nx * sc->absorb->ny * sc->absorb->nz : 0;
  std::vector<std::vector<double>> accM(nth);
  const size_t ntex = (d_tex && sc->env->kind == 0) ? 3 * (size_t)sc->env->W * sc->env->H : 0;
  std::vector<std::vector<double>> accT(nth);
  const size_t nmlp = (d_mlp && sc->env->kind == 1) ? mlp_param_count(*sc->env) : 0;
  std::vector<std::vector<double>> accW(nth);
  const size_t nfld = (d_field && sc->field)
                          ? 4 * ((size_t)sc->field->nx * sc->field->ny * sc->field->nz +
                                 3 * (size_t)sc->field->res * sc->field->res)
                          : 0;
  std::vector<std::vector<double>> accF(nth);
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    accV[tid].assign(3 * (size_t)sc->nv, 0.0);
    accM[tid].assign(nmu, 0.0);
    accT[tid].assign(ntex, 0.0);
    accW[tid].assign(nmlp, 0.0);
    accF[tid].assign(nfld, 0.0);
    Tape tape;
    g_tape = &tape;
    std::unordered_map<int, V3<Var>> texleaf;
    g_texleaf = ntex ? &texleaf : nullptr;
    std::vector<Var> mlpleaf;
    g_mlpleaf = nmlp ? &mlpleaf : nullptr;
#pragma omp for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
      const double* g = grad_rgb + 3 * i;
      tape.nodes.clear();
      texleaf.clear();
      mlpleaf.clear();
      Ctx<Var> cx;
      cx.sh = &sh;
      cx.eta = leaf(sc->eta);
      for (int k = 0; k < 3; ++k) cx.sigma[k] = leaf(sc->sigma[k]);
      PathInfo pi;
      pi.start(sc, i);
      double W[3] = {1, 1, 1};
      V3<Var> oo{Var(o[3 * i]), Var(o[3 * i + 1]), Var(o[3 * i + 2])};
      V3<Var> dd{Var(d[3 * i]), Var(d[3 * i + 1]), Var(d[3 * i + 2])};
      V3<Var> L = trace<Var>(cx, oo, dd, -1, 0, W, false, pi, nullptr);
      if (rgb) {
        rgb[3 * i] = L.x.v;
        rgb[3 * i + 1] = L.y.v;
        rgb[3 * i + 2] = L.z.v;
      }
      if (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0) continue;
      std::vector<double> adj(tape.nodes.size(), 0.0);
      if (L.x.i >= 0) adj[L.x.i] += g[0];
      if (L.y.i >= 0) adj[L.y.i] += g[1];
      if (L.z.i >= 0) adj[L.z.i] += g[2];
      for (int k = (int)tape.nodes.size() - 1; k >= 0; --k) {
        double a = adj[k];
        if (a == 0.0) continue;
        const TapeNode& tn = tape.nodes[k];
        if (tn.a >= 0) adj[tn.a] += tn.da * a;
        if (tn.b >= 0) adj[tn.b] += tn.db * a;
      }
      // absolute = 1: each camera ray's contribution enters by its magnitude
      auto A = [&](int i) { return absolute ? std::fabs(adj[i]) : adj[i]; };
      accE[tid] += A(cx.eta.i);
      for (int k = 0; k < 3; ++k) accS[3 * tid + k] += A(cx.sigma[k].i);
      for (auto& kv : cx.P) {
        double* dst = accV[tid].data() + 3 * (size_t)kv.first;
        dst[0] += A(kv.second.x.i);
        dst[1] += A(kv.second.y.i);
        dst[2] += A(kv.second.z.i);
      }
      for (auto& kv : cx.G) {
        double* dst = accM[tid].data() + 3 * (size_t)kv.first;
        dst[0] += A(kv.second.x.i);
        dst[1] += A(kv.second.y.i);
        dst[2] += A(kv.second.z.i);
      }
      for (auto& kv : texleaf) {
        double* dst = accT[tid].data() + 3 * (size_t)kv.first;
        dst[0] += A(kv.second.x.i);
        dst[1] += A(kv.second.y.i);
        dst[2] += A(kv.second.z.i);
      }
      for (size_t k = 0; k < mlpleaf.size(); ++k) accW[tid][k] += A(mlpleaf[k].i);
      if (nfld)
        for (auto& kv : cx.FP)
          for (int c = 0; c < 4; ++c) accF[tid][4 * (size_t)kv.first + c] += A(kv.second[c].i);
    }
    g_tape = nullptr;
    g_texleaf = nullptr;
    g_mlpleaf = nullptr;
  }
  std::memset(dV, 0, sizeof(double) * 3 * (size_t)sc->nv);
  if (ntex) std::memset(d_tex, 0, sizeof(double) * ntex);
  *d_eta = 0.0;
  d_sigma[0] = d_sigma[1] = d_sigma[2] = 0.0;
  if (d_mu && nmu) std::memset(d_mu, 0, sizeof(double) * nmu);
  if (nmlp) std::memset(d_mlp, 0, sizeof(double) * nmlp);
  if (nfld) std::memset(d_field, 0, sizeof(double) * nfld);
  for (int t = 0; t < nth; ++t) {
    if (accV[t].empty()) continue;
    for (size_t j = 0; j < 3 * (size_t)sc->nv; ++j) dV[j] += accV[t][j];
    *d_eta += accE[t];
    for (int k = 0; k < 3; ++k) d_sigma[k] += accS[3 * t + k];
    if (d_mu)
      for (size_t j = 0; j < nmu; ++j) d_mu[j] += accM[t][j];
    for (size_t j = 0; j < ntex; ++j) d_tex[j] += accT[t][j];
    for (size_t j = 0; j < nmlp; ++j) d_mlp[j] += accW[t][j];
    for (size_t j = 0; j < nfld; ++j) d_field[j] += accF[t][j];
  }
  return 0;
}

// First-order bound on the rounding error of an FP32 evaluation of each
// pixel's radiance (running error analysis by automatic differentiation:
// an operation z computed as z (1 + e), |e| <= u, moves the pixel by
// dC/dz z e, so |C_fp32 - C| <= sum over the computation's operations of
// |dC/dz| |z| u, to first order in u; Iri, "History of automatic
// differentiation and rounding error estimation", 1991, and Higham,
// "Accuracy and Stability of Numerical Algorithms", 2002, Sec. 3.3).  The
// sum runs over every operation of the recursion on the pixel's discrete
// path, each charged the unit roundoff 2^-24 (2^-23 for library functions);
// the mesh, IoR, absorption, environment and camera origin are exact FP32
// inputs shared by both sides, the camera direction is charged as an FP32
// result (2^-23).  bound [n*3] per channel; rgb
// [n*3] may be NULL.
int or_trace_errbound(const or_scene* sc, const double* o, const double* d, int64_t n,
                      double* rgb, double* bound) {
  if (!valid_scene(sc)) return 1;
  Shared sh;
  make_shared(sc, sh, true);
#pragma omp parallel
  {
    Tape tape;
    g_tape = &tape;
    // texels and network parameters are exact inputs: constants here
    g_texleaf = nullptr;
    g_mlpleaf = nullptr;
#pragma omp for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
      tape.nodes.clear();
      Ctx<Var> cx;
      cx.sh = &sh;
      cx.eta = leaf(sc->eta);
      for (int k = 0; k < 3; ++k) cx.sigma[k] = leaf(sc->sigma[k]);
      PathInfo pi;
      pi.start(sc, i);
      double W[3] = {1, 1, 1};
      V3<Var> oo{leaf(o[3 * i]), leaf(o[3 * i + 1]), leaf(o[3 * i + 2])};
      V3<Var> dd{leaf(d[3 * i], kUlp32x2), leaf(d[3 * i + 1], kUlp32x2), leaf(d[3 * i + 2], kUlp32x2)};
      V3<Var> L = trace<Var>(cx, oo, dd, -1, 0, W, false, pi, nullptr);
      const Var Lc[3] = {L.x, L.y, L.z};
      std::vector<double> adj(tape.nodes.size());
      for (int c = 0; c < 3; ++c) {
        if (rgb) rgb[3 * i + c] = Lc[c].v;
        double b = 0.0;
        if (Lc[c].i >= 0) {
          std::fill(adj.begin(), adj.end(), 0.0);
          adj[Lc[c].i] = 1.0;
          for (int k = (int)tape.nodes.size() - 1; k >= 0; --k) {
            double a = adj[k];
            if (a == 0.0) continue;
            const TapeNode& tn = tape.nodes[k];
            b += std::fabs(a * tn.v) * (double)tn.u;
            if (tn.a >= 0) adj[tn.a] += tn.da * a;
            if (tn.b >= 0) adj[tn.b] += tn.db * a;
          }
        }
        bound[3 * i + c] = b;
      }
    }
    g_tape = nullptr;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Silhouette (mask) term: the coverage of each pixel by the object and the
// gradient of a loss on it with respect to the vertices, through the motion
// of the object's outline (the visibility gradient the interior derivatives
// above do not carry; the paper's mask loss, Sec. 3.1 "Mask-based Geometry
// Initialization" and the appendix on the ray tracer's mesh regularization).
//
// Readings: the mask of pixel p is the fraction of its unit square in
// continuous image coordinates (pixel (x, y) = [x, x+1) x [y, y+1)) covered by
// the object's projection; its value is taken at the pixel centre (1 when the
// centre's camera ray hits the mesh), its derivative is the boundary integral
// dM_p/dtheta = int over the outline inside p of (dx/dtheta . n_out) dl, with
// n_out the image-plane normal pointing away from the covered side.  The
// outline is made of silhouette edges (one adjacent face facing the eye, the
// other not; an edge with one face counts too) at points whose camera ray
// meets no other triangle anywhere along it.  The integral is taken by a
// fixed quadrature: an edge whose projection is l pixels long gets
// n = max(1, ceil(rho l)) points at the midpoints t_k = (k + 1/2)/n of the
// segment's 3D parameter, weight |dx/dt| / n, each assigned to the pixel
// containing its projection; a point moves with its two vertices with
// weights 1 - t_k and t_k.
// ---------------------------------------------------------------------------
namespace {

struct CamBasis {
  V3<double> eye, f, r, u;
  double th, aspect;
  int W, H;
};

CamBasis cam_basis(const double* cam, int W, int H) {
  const double PI = 3.14159265358979323846;
  CamBasis c;
  c.eye = {cam[0], cam[1], cam[2]};
  V3<double> tgt{cam[3], cam[4], cam[5]}, up{cam[6], cam[7], cam[8]};
  c.f = normalize(sub(tgt, c.eye));
  c.r = normalize(cross(c.f, up));
  c.u = cross(c.r, c.f);
  c.th = std::tan(0.5 * cam[9] * PI / 180.0);
  c.aspect = (double)W / (double)H;
  c.W = W;
  c.H = H;
  return c;
}

// continuous image position of a 3D point in front of the camera (z > 0),
// and its Jacobian d(xi, yi)/dX (rows jx, jy)
bool project(const CamBasis& c, V3<double> X, double& xi, double& yi, V3<double>* jx, V3<double>* jy) {
  V3<double> w = sub(X, c.eye);
  double z = dot(w, c.f);
  if (!(z > 1e-9)) return false;
  double a = dot(w, c.r), b = dot(w, c.u);
  double sx = 0.5 * c.W / (c.th * c.aspect), sy = 0.5 * c.H / c.th;
  xi = sx * (a / z) + 0.5 * c.W;
  yi = 0.5 * c.H - sy * (b / z);
  if (jx) *jx = scl(sub(scl(c.r, 1.0 / z), scl(c.f, a / (z * z))), sx);
  if (jy) *jy = scl(sub(scl(c.u, 1.0 / z), scl(c.f, b / (z * z))), -sy);
  return true;
}

// any triangle other than f1, f2 met by the line eye + s (X - eye), s > 0
bool line_blocked(const or_scene& sc, const BVH& b, V3<double> eye, V3<double> X, int f1, int f2) {
  double o[3] = {eye.x, eye.y, eye.z};
  V3<double> dv = sub(X, eye);
  double d[3] = {dv.x, dv.y, dv.z};
  if (b.nodes.empty()) return false;
  int stack[128];
  int sp = 0;
  stack[sp++] = 0;
  while (sp) {
    const BNode& n = b.nodes[stack[--sp]];
    if (box_enter(n, o, d, INFINITY) == INFINITY) continue;
    if (n.left < 0) {
      for (int i = n.first; i < n.first + n.count; ++i) {
        int f = b.order[i];
        if (f == f1 || f == f2) continue;
        double t, b1, b2;
        if (mt_hit(sc, f, o, d, t, b1, b2)) return true;
      }
    } else {
      stack[sp++] = n.right;
      stack[sp++] = n.left;
    }
  }
  return false;
}

struct MeshEdge {
  int a, b, f1, f2;  // f2 = -1 for an edge with one face
};

std::vector<MeshEdge> mesh_edges(const or_scene& sc) {
  std::unordered_map<uint64_t, int> seen;
  std::vector<MeshEdge> E;
  for (int f = 0; f < sc.nf; ++f)
    for (int k = 0; k < 3; ++k) {
      int a = sc.F[3 * f + k], b = sc.F[3 * f + (k + 1) % 3];
      uint64_t key = ((uint64_t)(uint32_t)std::min(a, b) << 32) | (uint32_t)std::max(a, b);
      auto it = seen.find(key);
      if (it == seen.end()) {
        seen.emplace(key, (int)E.size());
        E.push_back({std::min(a, b), std::max(a, b), f, -1});
      } else {
        E[it->second].f2 = f;
      }
    }
  return E;
}

bool front_facing(const or_scene& sc, int f, V3<double> eye) {
  const double* p0 = sc.V + 3 * sc.F[3 * f];
  const double* p1 = sc.V + 3 * sc.F[3 * f + 1];
  const double* p2 = sc.V + 3 * sc.F[3 * f + 2];
  V3<double> v0{p0[0], p0[1], p0[2]}, v1{p1[0], p1[1], p1[2]}, v2{p2[0], p2[1], p2[2]};
  return dot(cross(sub(v1, v0), sub(v2, v0)), sub(v0, eye)) < 0.0;
}

}  // namespace

// Centre-sample mask of one camera: mask [W*H] = 1 where the pixel centre's
// camera ray hits the mesh (t > t_eps), else 0.
int or_mask(const or_scene* sc, const double* cam, int W, int H, double* mask) {
  if (!valid_scene(sc)) return 1;
  Shared sh;
  make_shared(sc, sh, false);
  std::vector<double> o(3 * (size_t)W * H), d(3 * (size_t)W * H);
  or_camera_rays(cam, W, H, o.data(), d.data());
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < (int64_t)W * H; ++i) {
    Hit h = sc->use_bvh ? closest_bvh(*sc, sh.bvh, o.data() + 3 * i, d.data() + 3 * i, -1)
                        : closest_brute(*sc, o.data() + 3 * i, d.data() + 3 * i, -1);
    mask[i] = h.tri >= 0 ? 1.0 : 0.0;
  }
  return 0;
}

// Gradient of sum_p grad_mask[p] M_p with respect to the vertices, by the
// outline quadrature above at density rho (points per pixel of projected
// edge length).  dV [nv*3] is overwritten.  Optional counts [2]: silhouette
// points in the image whose pixel has a nonzero grad_mask, and of those the
// ones on the outline (visible).
int or_mask_grad(const or_scene* sc, const double* cam, int W, int H, const double* grad_mask,
                 double rho, double* dV, int64_t* counts) {
  if (!valid_scene(sc) || !(rho > 0.0)) return 1;
  Shared sh;
  make_shared(sc, sh, false);
  CamBasis c = cam_basis(cam, W, H);
  std::vector<MeshEdge> E = mesh_edges(*sc);
  std::memset(dV, 0, sizeof(double) * 3 * (size_t)sc->nv);
  int64_t n_in = 0, n_vis = 0;
  auto P = [&](int v) {
    const double* p = sc->V + 3 * v;
    return V3<double>{p[0], p[1], p[2]};
  };
  for (const MeshEdge& e : E) {
    bool fa = front_facing(*sc, e.f1, c.eye);
    int front = e.f1;
    if (e.f2 >= 0) {
      bool fb = front_facing(*sc, e.f2, c.eye);
      if (fa == fb) continue;
      front = fa ? e.f1 : e.f2;
    }
    V3<double> A = P(e.a), Bv = P(e.b);
    double xa, ya, xb, yb;
    if (!project(c, A, xa, ya, nullptr, nullptr) || !project(c, Bv, xb, yb, nullptr, nullptr)) continue;
    // the front face's third vertex lies on the covered side
    int cv = sc->F[3 * front] + sc->F[3 * front + 1] + sc->F[3 * front + 2] - e.a - e.b;
    double xc, yc;
    if (!project(c, P(cv), xc, yc, nullptr, nullptr)) continue;
    double ex = xb - xa, ey = yb - ya;
    double len = std::sqrt(ex * ex + ey * ey);
    if (!(len > 0.0)) continue;
    double nx = -ey / len, ny = ex / len;
    if (nx * (xc - xa) + ny * (yc - ya) > 0.0) {
      nx = -nx;
      ny = -ny;
    }
    int ns = std::max(1, (int)std::ceil(rho * len));
    for (int k = 0; k < ns; ++k) {
      double t = (k + 0.5) / ns;
      V3<double> X = add(scl(A, 1.0 - t), scl(Bv, t));
      double xi, yi;
      V3<double> jx, jy;
      if (!project(c, X, xi, yi, &jx, &jy)) continue;
      if (!(xi >= 0.0 && xi < W && yi >= 0.0 && yi < H)) continue;
      int px = std::min((int)std::floor(xi), W - 1), py = std::min((int)std::floor(yi), H - 1);
      double g = grad_mask[(size_t)py * W + px];
      if (g == 0.0) continue;
      ++n_in;
      if (line_blocked(*sc, sh.bvh, c.eye, X, e.f1, e.f2)) continue;
      ++n_vis;
      V3<double> BA = sub(Bv, A);
      double dxt = dot(jx, BA), dyt = dot(jy, BA);
      double w = std::sqrt(dxt * dxt + dyt * dyt) / ns;
      // normal velocity per unit move of the point: n . J
      V3<double> nJ = add(scl(jx, nx), scl(jy, ny));
      V3<double> ca = scl(nJ, g * w * (1.0 - t)), cb = scl(nJ, g * w * t);
      double* da = dV + 3 * (size_t)e.a;
      double* db = dV + 3 * (size_t)e.b;
      da[0] += ca.x;
      da[1] += ca.y;
      da[2] += ca.z;
      db[0] += cb.x;
      db[1] += cb.y;
      db[2] += cb.z;
    }
  }
  if (counts) {
    counts[0] = n_in;
    counts[1] = n_vis;
  }
  return 0;
}

// Dump the path tree of one camera ray in depth-first order (parent before
// children, reflected child before refracted child).  Each record is
// or_tree_record_doubles() doubles.  Returns the number of records in the
// tree (only the first max_rec are written).
int or_trace_tree(const or_scene* sc, const double* o, const double* d, double* out, int max_rec) {
  if (!valid_scene(sc)) return -1;
  Shared sh;
  make_shared(sc, sh, true);
  Ctx<double> cx{&sh, sc->eta, {sc->sigma[0], sc->sigma[1], sc->sigma[2]}};
  PathInfo pi;
  pi.start(sc, 0);
  double W[3] = {1, 1, 1};
  std::vector<TreeRec> tree;
  trace<double>(cx, {o[0], o[1], o[2]}, {d[0], d[1], d[2]}, -1, 0, W, false, pi, &tree);
  int k = std::min<int>((int)tree.size(), max_rec);
  std::memcpy(out, tree.data(), sizeof(TreeRec) * (size_t)k);
  return (int)tree.size();
}

int or_tree_record_doubles(void) { return (int)(sizeof(TreeRec) / sizeof(double)); }

}  // extern "C"
