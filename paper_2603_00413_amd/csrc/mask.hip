// Silhouette (mask) term: each pixel's coverage by the object and the
// gradient of a loss on it with respect to the vertices through the motion of
// the object's outline (the visibility gradient that the interior derivatives
// of the tracer do not carry; the paper's mask loss, Sec. 3.1 "Mask-based
// Geometry Initialization" and the appendix on the ray tracer's mesh
// regularization).
//
// The mask of pixel p is the fraction of its unit square (pixel (x, y) covers
// [x, x+1) x [y, y+1) in continuous image coordinates) covered by the
// object's projection.  Its value is taken at the pixel centre; its
// derivative is the boundary integral of the outline's normal velocity over
// the part of the outline inside p.  The outline is made of silhouette edges
// (one adjacent face facing the eye and the other not, or an edge with one
// face) at points whose camera line meets no other triangle.  The integral is
// a fixed quadrature: an edge whose projection is l pixels long gets
// n = max(1, ceil(rho l)) points at the midpoints t_k = (k + 1/2) / n of its
// 3D parameter, weight |dx/dt| / n, each added to the pixel containing its
// projection, and a point moves with its two vertices with weights 1 - t_k
// and t_k.
//
// Kernels: k_mask_edges lists each mesh edge once (the face holding it as
// (a, b) with a < b owns it, or its only face), with its other face from the
// blob's vertex-to-face lists; k_mask_forward casts the pixel-centre rays;
// k_mask_grad takes one (camera, edge) per thread: facing test in FP64 (exact
// products of FP32 inputs, so the decision matches an FP64 evaluation),
// projection and quadrature in FP32, an any-hit walk of the binary BVH per
// point, and FP32 atomic additions into dV.
#include "dt_queue.h"

namespace {

constexpr int MT = 256;

struct MaskCams {
  CamDev c[DT_MASK_MAX_CAMERAS];
  int n;
};

__device__ __forceinline__ v3 vtx(const float* V, int i) { return load3(V + 3 * (size_t)i); }

// owner slot 3 f + k: (min, max vertex, owner face, other face or -1), or
// x = -1 when another face owns the edge
__global__ void __launch_bounds__(MT) k_mask_edges(const int32_t* F, int32_t nf, int32_t nv, BvhView bv,
                                                   int4* edges) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= 3 * (int64_t)nf) return;
  const int f = (int)(s / 3), k = (int)(s % 3);
  const int a = vclampi(F[3 * f + k], nv), b = vclampi(F[3 * f + (k + 1) % 3], nv);
  int twin = -1;
  for (int j = bv.csr_off[b]; j < bv.csr_off[b + 1]; ++j) {
    const int g = bv.csr_idx[j];
    if (g == f) continue;
    if (F[3 * g] == a || F[3 * g + 1] == a || F[3 * g + 2] == a) {
      twin = g;
      break;  // ascending lists: the smallest such face
    }
  }
  const bool own = a < b || twin < 0;
  edges[s] = own ? make_int4(a < b ? a : b, a < b ? b : a, f, twin) : make_int4(-1, -1, -1, -1);
}

// conservative slab test of a line o + s d, s > 0, against a box
__device__ __forceinline__ bool line_box(v3 o, v3 inv, v3 lo, v3 hi) {
  float tx0 = (lo.x - o.x) * inv.x, tx1 = (hi.x - o.x) * inv.x;
  float ty0 = (lo.y - o.y) * inv.y, ty1 = (hi.y - o.y) * inv.y;
  float tz0 = (lo.z - o.z) * inv.z, tz1 = (hi.z - o.z) * inv.z;
  float tmin = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.f));
  float tmax = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1));
  // slack for the rounding of the six products (a few ulps of each)
  return tmin <= tmax * (1.0f + 4.0f * 1.1920929e-07f) + 1e-30f;
}

// Does the line o + s d (s > t_eps) meet any triangle but f1 and f2?  Walks
// the binary tree with a per-thread stack; a full stack is reported as a
// hit (conservative: the point is then not counted on the outline) and
// flagged.
__device__ __forceinline__ bool line_blocked(const BvhView& bv, v3 o, v3 d, int f1, int f2, float t_eps,
                                             bool* overflow) {
  const RayPre r = ray_pre(o, d);
  const v3 inv = r.inv;
  auto leaf_hit = [&](uint32_t j) {
    const float4* L = bv.leaves + 3 * (size_t)j;
    const int f = __float_as_int(L[0].w);
    if (f == f1 || f == f2) return false;
    Hit h;
    h.tri = -1;
    h.t = INFINITY;
    h.b1 = h.b2 = 0.f;
    return tri_test(r, xyz(L[0]), xyz(L[1]), xyz(L[2]), f, t_eps, h);
  };
  if (bv.nf == 1) return leaf_hit(0u);
  uint32_t stack[64];
  int sp = 0;
  uint32_t node = 0;
  while (true) {
    const BvhNode n = bv.nodes[node];
    const v3 lo0 = mk3(n.a.x, n.a.y, n.a.z), hi0 = mk3(n.a.w, n.b.x, n.b.y);
    const v3 lo1 = mk3(n.b.z, n.b.w, n.c.x), hi1 = mk3(n.c.y, n.c.z, n.c.w);
    const uint32_t c[2] = {(uint32_t)n.d.x, (uint32_t)n.d.y};
    const bool in[2] = {line_box(o, inv, lo0, hi0), line_box(o, inv, lo1, hi1)};
    uint32_t next = DT_NO_CHILD;
    for (int k = 0; k < 2; ++k) {
      if (!in[k]) continue;
      if (c[k] & DT_LEAF_BIT) {
        if (leaf_hit(c[k] & ~DT_LEAF_BIT)) return true;
      } else if (next == DT_NO_CHILD) {
        next = c[k];
      } else {
        if (sp == 64) {
          *overflow = true;
          return true;
        }
        stack[sp++] = c[k];
      }
    }
    if (next == DT_NO_CHILD) {
      if (sp == 0) return false;
      next = stack[--sp];
    }
    node = next;
  }
}

__device__ __forceinline__ bool front_facing(const float* V, const int32_t* F, int nv, int f, const float* eye) {
  const v3 p0 = vtx(V, vclampi(F[3 * f], nv)), p1 = vtx(V, vclampi(F[3 * f + 1], nv));
  const v3 p2 = vtx(V, vclampi(F[3 * f + 2], nv));
  const double ax = (double)p1.x - p0.x, ay = (double)p1.y - p0.y, az = (double)p1.z - p0.z;
  const double bx = (double)p2.x - p0.x, by = (double)p2.y - p0.y, bz = (double)p2.z - p0.z;
  const double nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
  return nx * ((double)p0.x - eye[0]) + ny * ((double)p0.y - eye[1]) + nz * ((double)p0.z - eye[2]) < 0.0;
}

// continuous image position of X, and the rows of d(xi, yi)/dX; false if X
// is not in front of the camera
__device__ __forceinline__ bool project(const CamDev& c, v3 X, float& xi, float& yi, v3* jx, v3* jy) {
  const v3 w = X - mk3(c.eye[0], c.eye[1], c.eye[2]);
  const v3 f = mk3(c.f[0], c.f[1], c.f[2]), r = mk3(c.r[0], c.r[1], c.r[2]), u = mk3(c.u[0], c.u[1], c.u[2]);
  const float z = dot(w, f);
  if (!(z > 1e-9f)) return false;
  const float a = dot(w, r), b = dot(w, u);
  const float sx = 0.5f * (float)c.W / (c.th * c.aspect), sy = 0.5f * (float)c.H / c.th;
  const float iz = 1.0f / z;
  xi = sx * (a * iz) + 0.5f * (float)c.W;
  yi = 0.5f * (float)c.H - sy * (b * iz);
  if (jx) {
    *jx = (r * iz - f * (a * iz * iz)) * sx;
    *jy = (u * iz - f * (b * iz * iz)) * (-sy);
  }
  return true;
}

__global__ void __launch_bounds__(MT) k_mask_forward(BvhView bv, MaskCams cams, float t_eps, float* mask) {
  const int cam = blockIdx.y;
  const CamDev& c = cams.c[cam];
  const int64_t np = (int64_t)c.W * c.H;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int x = (int)(i % c.W), y = (int)(i / c.W);
  const float px = (2.0f * ((float)x + 0.5f) / (float)c.W - 1.0f) * c.th * c.aspect;
  const float py = (1.0f - 2.0f * ((float)y + 0.5f) / (float)c.H) * c.th;
  const v3 d = normalize3(mk3(c.f[0], c.f[1], c.f[2]) + mk3(c.r[0], c.r[1], c.r[2]) * px +
                          mk3(c.u[0], c.u[1], c.u[2]) * py);
  bool ovf = false;
  const bool hit = line_blocked(bv, mk3(c.eye[0], c.eye[1], c.eye[2]), d, -1, -1, t_eps, &ovf);
  mask[c.pixel_offset + i] = hit ? 1.0f : 0.0f;
}

// counts: [0] outline points in an image where the loss gradient is nonzero,
// [1] of those, points on the outline (visible), [2] stack overflows
__global__ void __launch_bounds__(MT) k_mask_grad(const float* V, const int32_t* F, int32_t nv, int32_t nf,
                                                  BvhView bv, const int4* edges, MaskCams cams,
                                                  const float* grad_mask, float rho, float* dV,
                                                  unsigned long long* counts) {
  const int cam = blockIdx.y;
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= 3 * (int64_t)nf) return;
  const int4 e = edges[s];
  if (e.x < 0) return;
  const CamDev& c = cams.c[cam];
  const bool fa = front_facing(V, F, nv, e.z, c.eye);
  int front = e.z;
  if (e.w >= 0) {
    const bool fb = front_facing(V, F, nv, e.w, c.eye);
    if (fa == fb) return;
    front = fa ? e.z : e.w;
  }
  const v3 A = vtx(V, e.x), Bv = vtx(V, e.y);
  float xa, ya, xb, yb, xc, yc;
  if (!project(c, A, xa, ya, nullptr, nullptr) || !project(c, Bv, xb, yb, nullptr, nullptr)) return;
  const int cv = vclampi(F[3 * front] + F[3 * front + 1] + F[3 * front + 2] - e.x - e.y, nv);
  if (!project(c, vtx(V, cv), xc, yc, nullptr, nullptr)) return;
  const float ex = xb - xa, ey = yb - ya;
  const float len = sqrtf(ex * ex + ey * ey);
  if (!(len > 0.f)) return;
  float nx = -ey / len, ny = ex / len;
  if (nx * (xc - xa) + ny * (yc - ya) > 0.f) {
    nx = -nx;
    ny = -ny;
  }
  const int ns = max(1, (int)ceilf(rho * len));
  const v3 eye = mk3(c.eye[0], c.eye[1], c.eye[2]);
  const v3 BA = Bv - A;
  unsigned n_in = 0, n_vis = 0, n_ovf = 0;
  for (int k = 0; k < ns; ++k) {
    const float t = ((float)k + 0.5f) / (float)ns;
    const v3 X = A * (1.0f - t) + Bv * t;
    float xi, yi;
    v3 jx, jy;
    if (!project(c, X, xi, yi, &jx, &jy)) continue;
    if (!(xi >= 0.f && xi < (float)c.W && yi >= 0.f && yi < (float)c.H)) continue;
    const int px = min((int)floorf(xi), c.W - 1), py = min((int)floorf(yi), c.H - 1);
    const float g = grad_mask[c.pixel_offset + (int64_t)py * c.W + px];
    if (g == 0.f) continue;
    ++n_in;
    bool ovf = false;
    // the line from the eye through X; X sits at parameter 1
    if (line_blocked(bv, eye, X - eye, e.z, e.w, 1e-4f, &ovf)) {
      n_ovf += ovf ? 1u : 0u;
      continue;
    }
    ++n_vis;
    const float dxt = dot(jx, BA), dyt = dot(jy, BA);
    const float w = sqrtf(dxt * dxt + dyt * dyt) / (float)ns;
    const v3 nJ = jx * nx + jy * ny;
    const v3 ca = nJ * (g * w * (1.0f - t)), cb = nJ * (g * w * t);
    atomicAdd(dV + 3 * (size_t)e.x, ca.x);
    atomicAdd(dV + 3 * (size_t)e.x + 1, ca.y);
    atomicAdd(dV + 3 * (size_t)e.x + 2, ca.z);
    atomicAdd(dV + 3 * (size_t)e.y, cb.x);
    atomicAdd(dV + 3 * (size_t)e.y + 1, cb.y);
    atomicAdd(dV + 3 * (size_t)e.y + 2, cb.z);
  }
  if (counts && n_in) {
    atomicAdd(counts, (unsigned long long)n_in);
    if (n_vis) atomicAdd(counts + 1, (unsigned long long)n_vis);
    if (n_ovf) atomicAdd(counts + 2, (unsigned long long)n_ovf);
  }
}

__global__ void k_mask_zero(float* p, int64_t n, unsigned long long* counts) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
  if (counts && blockIdx.x == 0 && threadIdx.x < 3) counts[threadIdx.x] = 0ull;
}

dt_status mask_setup(const dt_scene* sc, const dt_rays* rays, BvhView& bv, MaskCams& mc) {
  DT_REQUIRE(sc && rays, "NULL scene or rays");
  DT_REQUIRE(sc->V && sc->F && sc->bvh, "scene needs V, F and bvh");
  DT_REQUIRE(sc->nv >= 3 && sc->nf >= 1 && sc->nf <= DT_MAX_FACES && sc->nv < (1 << 30),
             "scene needs nv >= 3 and 1 <= nf <= 2^26");
  DT_REQUIRE(rays->kind == DT_RAYS_CAMERAS && rays->cameras, "the mask term takes camera rays");
  DT_REQUIRE(rays->n_cameras >= 1 && rays->n_cameras <= DT_MASK_MAX_CAMERAS,
             "the mask term takes 1..%d cameras per call", DT_MASK_MAX_CAMERAS);
  DT_REQUIRE(rays->n_pixels >= 1 && rays->n_pixels < (1ll << 31), "n_pixels must be in [1, 2^31)");
  mc.n = rays->n_cameras;
  for (int c = 0; c < mc.n; ++c) {
    const dt_camera& cam = rays->cameras[c];
    DT_REQUIRE(cam.width >= 1 && cam.height >= 1 && cam.fov_deg > 0.f && cam.fov_deg < 180.f,
               "camera %d: bad image size or field of view", c);
    DT_REQUIRE(cam.pixel_offset >= 0 && cam.pixel_offset + (int64_t)cam.width * cam.height <= rays->n_pixels,
               "camera %d: image exceeds n_pixels", c);
    if (dt_status st = make_camera(cam, c, mc.c[c])) return st;
  }
  bv = bvh_view(sc->bvh, sc->nv, sc->nf);
  return DT_OK;
}

}  // namespace

extern "C" dt_status dt_mask_bytes(int32_t nv, int32_t nf, size_t* ws_bytes) {
  DT_REQUIRE(ws_bytes, "dt_mask_bytes: NULL argument");
  DT_REQUIRE(nv >= 3 && nf >= 1 && nf <= DT_MAX_FACES, "dt_mask_bytes: need nv >= 3, 1 <= nf <= 2^26");
  *ws_bytes = dt_align(sizeof(int4) * 3 * (size_t)nf);
  return DT_OK;
}

extern "C" dt_status dt_mask_forward(const dt_scene* sc, const dt_rays* rays, float t_eps, float* mask,
                                     void* stream) {
  BvhView bv;
  MaskCams mc;
  if (dt_status st = mask_setup(sc, rays, bv, mc)) return st;
  DT_REQUIRE(mask, "dt_mask_forward: NULL mask");
  DT_REQUIRE(t_eps >= 0.f && t_eps < 1.f, "t_eps must be in [0, 1)");
  hipStream_t s = (hipStream_t)stream;
  int64_t most = 1;
  for (int c = 0; c < mc.n; ++c) most = std::max<int64_t>(most, (int64_t)mc.c[c].W * mc.c[c].H);
  hipLaunchKernelGGL(k_mask_forward, dim3(dt_blocks(most, MT), mc.n), dim3(MT), 0, s, bv, mc, t_eps, mask);
  DT_CHECK_LAUNCH();
  return DT_OK;
}

extern "C" dt_status dt_mask_backward(const dt_scene* sc, const dt_rays* rays, const float* grad_mask,
                                      float rho, float* dV, uint64_t* counts, void* ws, size_t ws_bytes,
                                      void* stream) {
  BvhView bv;
  MaskCams mc;
  if (dt_status st = mask_setup(sc, rays, bv, mc)) return st;
  DT_REQUIRE(grad_mask && dV && ws, "dt_mask_backward: NULL argument");
  DT_REQUIRE(rho > 0.f && rho <= 4096.f, "rho must be in (0, 4096]");
  const size_t need = dt_align(sizeof(int4) * 3 * (size_t)sc->nf);
  if (ws_bytes < need) {
    dt_set_error("dt_mask_backward: workspace has %zu bytes, needs %zu", ws_bytes, need);
    return DT_ERR_WORKSPACE_TOO_SMALL;
  }
  hipStream_t s = (hipStream_t)stream;
  int4* edges = (int4*)ws;
  const int64_t slots = 3 * (int64_t)sc->nf;
  hipLaunchKernelGGL(k_mask_zero, dim3(dt_blocks(3 * (int64_t)sc->nv, 256) < 4096 ? dt_blocks(3 * (int64_t)sc->nv, 256) : 4096),
                     dim3(256), 0, s, dV, 3 * (int64_t)sc->nv, (unsigned long long*)counts);
  hipLaunchKernelGGL(k_mask_edges, dim3(dt_blocks(slots, MT)), dim3(MT), 0, s, sc->F, sc->nf, sc->nv, bv, edges);
  hipLaunchKernelGGL(k_mask_grad, dim3(dt_blocks(slots, MT), mc.n), dim3(MT), 0, s, sc->V, sc->F, sc->nv, sc->nf,
                     bv, edges, mc, grad_mask, rho, dV, (unsigned long long*)counts);
  DT_CHECK_LAUNCH();
  return DT_OK;
}
