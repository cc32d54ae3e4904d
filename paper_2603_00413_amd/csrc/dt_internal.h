// Internal definitions shared by the HIP translation units of libdifftrans.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/difftrans.h"

// ---------------------------------------------------------------- errors
void dt_set_error(const char* fmt, ...);

#define DT_CHECK_HIP(expr)                                                         \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      dt_set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                   __LINE__);                                                      \
      return DT_ERR_HIP;                                                           \
    }                                                                              \
  } while (0)

#define DT_CHECK_LAUNCH() DT_CHECK_HIP(hipGetLastError())

#define DT_REQUIRE(cond, ...)         \
  do {                                \
    if (!(cond)) {                    \
      dt_set_error(__VA_ARGS__);      \
      return DT_ERR_INVALID_ARGUMENT; \
    }                                 \
  } while (0)

// ---------------------------------------------------------------- vectors
struct v3 {
  float x, y, z;
};
__host__ __device__ __forceinline__ v3 mk3(float x, float y, float z) { return {x, y, z}; }
__host__ __device__ __forceinline__ v3 operator+(v3 a, v3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__host__ __device__ __forceinline__ v3 operator-(v3 a, v3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__host__ __device__ __forceinline__ v3 operator-(v3 a) { return {-a.x, -a.y, -a.z}; }
__host__ __device__ __forceinline__ v3 operator*(v3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__host__ __device__ __forceinline__ v3 operator*(float s, v3 a) { return {a.x * s, a.y * s, a.z * s}; }
__host__ __device__ __forceinline__ v3& operator+=(v3& a, v3 b) {
  a.x += b.x;
  a.y += b.y;
  a.z += b.z;
  return a;
}
__host__ __device__ __forceinline__ float dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__host__ __device__ __forceinline__ v3 cross(v3 a, v3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ float len3(v3 a) { return sqrtf(dot(a, a)); }
__device__ __forceinline__ v3 normalize3(v3 a) {
  float r = 1.0f / sqrtf(dot(a, a));
  return a * r;
}
__device__ __forceinline__ float comp(v3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }
__device__ __forceinline__ v3 xyz(float4 a) { return {a.x, a.y, a.z}; }
__device__ __forceinline__ v3 load3(const float* p) { return {p[0], p[1], p[2]}; }

// ---------------------------------------------------------------- BVH blob
// Internal node: boxes of both children + child references + parent.
// A child reference >= 0 is an internal node; (leaf | LEAF_BIT) is a leaf,
// leaf j being the j-th triangle in Morton order.
#define DT_LEAF_BIT 0x80000000u
// largest triangle count: the wave traversal packs (leaf index << 6 | lane)
// into 32 bits
#define DT_MAX_FACES (1 << 26)

struct __align__(16) BvhNode {
  float4 a;  // lo0.x lo0.y lo0.z hi0.x
  float4 b;  // hi0.y hi0.z lo1.x lo1.y
  float4 c;  // lo1.z hi1.x hi1.y hi1.z
  int4 d;    // child0 child1 parent unused
};

// 4-wide node collapsed from the binary tree: a binary internal node at even
// depth (root = 0) becomes a 4-wide node whose children are its grandchildren
// (a leaf child stays a leaf), 2 to 4 of them.  A child reference is a 4-wide
// node index, (leaf | DT_LEAF_BIT), or DT_NO_CHILD for an unused slot.
//
// The child boxes are stored quantized (64 B per node instead of 128): per
// axis an origin p and a power of two s = 2^e, and per child and axis 8-bit
// steps, lo = p + qlo * s, hi = p + qhi * s.  The build chooses p a multiple
// of s and s large enough that every such value is exactly representable in
// FP32, rounds qlo down and qhi up, and checks the decoded bounds against the
// exact child box, so the decoded boxes contain the exact ones and the
// traversal's decisions stay conservative.
#define DT_NO_CHILD 0xFFFFFFFFu

struct __align__(16) Bvh4Node {
  float4 org;   // p.x, p.y, p.z; w: bits e_x | e_y << 8 | e_z << 16 (int8 each) | count << 24
  uint4 qlo;    // x, y, z: the four children's 8-bit lower steps on that axis (child k in byte k)
  uint4 qhi;    // x, y, z: upper steps; w unused
  uint4 child;  // child references
};

// Upper bound on the number of 4-wide nodes: with E even-depth and O odd-depth
// internal nodes, every even one but the root has an odd parent with at most
// two internal children, so E - 1 <= 2 O and E <= (2 (nf - 1) + 1) / 3.
__host__ __device__ inline int32_t bvh4_cap(int32_t nf) {
  return nf > 1 ? (int32_t)((2 * (int64_t)(nf - 1) + 1) / 3) : 1;
}

struct BvhHeader {
  int32_t nv, nf;
  int32_t depth;  // tree height (root = 1), from the build
  int32_t pad0;
  float lo[3], hi[3];  // scene bounds of face centroids
};

// Byte offsets inside the caller's blob; a pure function of (nv, nf).
struct BvhLayout {
  size_t header, nodes, nodes4, leaves, vnormals, fnormals, csr_off, csr_idx, leaf_parent, total;
};

__host__ __device__ inline size_t dt_align(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

inline BvhLayout bvh_layout(int32_t nv, int32_t nf) {
  BvhLayout L;
  size_t o = 0;
  L.header = o;
  o = dt_align(o + sizeof(BvhHeader));
  L.nodes = o;
  o = dt_align(o + sizeof(BvhNode) * (size_t)(nf > 1 ? nf - 1 : 1));
  L.nodes4 = o;
  o = dt_align(o + sizeof(Bvh4Node) * (size_t)bvh4_cap(nf));
  L.leaves = o;
  o = dt_align(o + sizeof(float4) * 3 * (size_t)nf);
  L.vnormals = o;
  o = dt_align(o + sizeof(float4) * (size_t)nv);
  L.fnormals = o;
  o = dt_align(o + sizeof(float4) * (size_t)nf);
  L.csr_off = o;
  o = dt_align(o + sizeof(int32_t) * ((size_t)nv + 1));
  L.csr_idx = o;
  o = dt_align(o + sizeof(int32_t) * 3 * (size_t)nf);
  L.leaf_parent = o;
  o = dt_align(o + sizeof(int32_t) * (size_t)nf);
  L.total = o;
  return L;
}

// View of a built blob used by the trace kernels.
struct BvhView {
  const BvhHeader* hdr;
  const BvhNode* nodes;
  const Bvh4Node* nodes4;  // traversal tree
  const float4* leaves;    // 3 per leaf: v0 (w = tri id bits), v1, v2
  const float4* vn;      // vertex normals
  const float4* fn;      // unit face normals (w = 1 if area > 0)
  const int32_t* csr_off;
  const int32_t* csr_idx;
  int32_t nf, nv;
};

inline BvhView bvh_view(const void* blob, int32_t nv, int32_t nf) {
  BvhLayout L = bvh_layout(nv, nf);
  const char* b = (const char*)blob;
  BvhView v;
  v.hdr = (const BvhHeader*)(b + L.header);
  v.nodes = (const BvhNode*)(b + L.nodes);
  v.nodes4 = (const Bvh4Node*)(b + L.nodes4);
  v.leaves = (const float4*)(b + L.leaves);
  v.vn = (const float4*)(b + L.vnormals);
  v.fn = (const float4*)(b + L.fnormals);
  v.csr_off = (const int32_t*)(b + L.csr_off);
  v.csr_idx = (const int32_t*)(b + L.csr_idx);
  v.nf = nf;
  v.nv = nv;
  return v;
}

// ---------------------------------------------------------------- workspace carving
struct Carver {
  char* base;
  size_t off, cap;
  bool overflow;
  Carver(void* p, size_t c) : base((char*)p), off(0), cap(c), overflow(false) {}
  template <class T>
  T* take(size_t count) {
    size_t o = dt_align(off);
    off = o + sizeof(T) * count;
    if (off > cap) overflow = true;
    return base ? (T*)(base + o) : nullptr;
  }
  size_t used() const { return dt_align(off); }
};

// ---------------------------------------------------------------- launch helpers
inline unsigned dt_blocks(int64_t n, int threads) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// device-wide helpers (bvh.hip)
dt_status dt_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s);
dt_status dt_scan_exclusive_i32(const int32_t* in, int32_t* out, int32_t n, int32_t* partials,
                                hipStream_t s);
size_t dt_scan_partials_count();
