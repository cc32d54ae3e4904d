// Ray-queue records shared by the wavefront kernels and the environment MLP.
#pragma once

#include "dt_device.h"

constexpr uint32_t RAY_INSIDE = 1u;  // ray flag: travelling inside the object

// 64-bit mixer: the SplitMix64 output function (Steele, Lea and Flood,
// OOPSLA 2014).  Summed over a pixel's segments it gives an order-independent
// signature of the discrete path (generation, triangle or -1, TIR).
__device__ __forceinline__ uint64_t path_mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// One generation of rays, structure of arrays.
struct Gen {
  float4 *o, *d, *w, *hit;  // origin+skip, dir+pixel, weight+flags, (t, tri, b1, b2)
  uint32_t* code;
  int2* child;
};

// Work distribution of the traversal kernel.  A generation's queue is cut into
// DT_WORK_PARTS contiguous parts of 64-ray batches, each with a cursor on a
// cache line of its own.  Every wave claims its next batch with an atomic add
// on a cursor and waits for the result, so with one cursor for the whole
// queue the thousands of resident waves queue up on a single address; spread
// over separate lines the claims proceed in parallel.  (Cursors packed into
// one line were slower still than a single one.)  Workgroup b starts on part
// b % DT_WORK_PARTS, which with the device's round-robin hand-out of
// workgroups to its 8 dies keeps each die on one region of the queue.
constexpr int DT_WORK_PARTS = 8;
struct alignas(128) WorkPart {
  uint32_t next;  // batches of the part handed out so far
  uint32_t pad[31];
};

// Next batch for the calling wave (all 64 lanes together): true with its index
// in batch, false once every part is drained.  nb: batches in the queue; p:
// the part being drained, starting at x0 = blockIdx.x % DT_WORK_PARTS.  Each
// part is visited once, so a wave returns false after at most DT_WORK_PARTS
// empty claims.
__device__ __forceinline__ bool claim_batch(WorkPart* wp, uint32_t nb, uint32_t x0, uint32_t& p,
                                            uint32_t& batch) {
  while (true) {
    const uint32_t lo = (uint32_t)(((uint64_t)nb * p) / DT_WORK_PARTS);
    const uint32_t cnt = (uint32_t)(((uint64_t)nb * (p + 1u)) / DT_WORK_PARTS) - lo;
    uint32_t k = 0;
    if ((threadIdx.x & 63u) == 0u) k = atomicAdd(&wp[p].next, 1u);
    k = (uint32_t)__builtin_amdgcn_readfirstlane((int)k);
    if (k < cnt) {
      batch = lo + k;
      return true;
    }
    p = (p + 1u) % DT_WORK_PARTS;
    if (p == x0) return false;
  }
}

// Device-side counters of a trace (also the tape header).
struct Counters {
  uint32_t count[DT_MAX_DEPTH + 2];  // rays in generation g
  uint32_t nrefl[DT_MAX_DEPTH + 2];  // reflected children emitted by g (refracted follow them)
  uint32_t hits[DT_MAX_DEPTH + 2];   // rays of g that hit the mesh
  uint32_t nmiss[DT_MAX_DEPTH + 2];  // length of the miss list of g (MLP environment)
  uint32_t dropped;
  uint32_t pad[3];
};

// Adjoint records of one generation.
struct Adj {
  float4 *L, *O, *D;  // subtree radiance, d loss / d origin, d loss / d direction
};

// Pinhole camera for one image: basis computed on the host in FP64.
struct CamDev {
  float eye[3], f[3], r[3], u[3];
  float th, aspect;
  int W, H;
  int64_t pixel_offset, base;
  int tiled;
};

// direction of the r-th ray of a camera (8x8 tiles in queue order when the
// image is a multiple of 8 in both sizes, row-major otherwise)
__device__ __forceinline__ v3 camera_ray(const CamDev& c, int64_t r, int& x, int& y) {
  if (c.tiled) {
    int64_t tile = r >> 6;
    int s = (int)(r & 63);
    int tx = (int)(tile % (c.W >> 3)), ty = (int)(tile / (c.W >> 3));
    x = tx * 8 + (s & 7);
    y = ty * 8 + (s >> 3);
  } else {
    x = (int)(r % c.W);
    y = (int)(r / c.W);
  }
  float px = (2.0f * ((float)x + 0.5f) / (float)c.W - 1.0f) * c.th * c.aspect;
  float py = (1.0f - 2.0f * ((float)y + 0.5f) / (float)c.H) * c.th;
  v3 f = mk3(c.f[0], c.f[1], c.f[2]), rt = mk3(c.r[0], c.r[1], c.r[2]), up = mk3(c.u[0], c.u[1], c.u[2]);
  return normalize3(f + rt * px + up * py);
}

// host: environment descriptor check + device view (trace.hip)
dt_status make_env(const dt_env* env, EnvDev& e);

// host: camera basis (right-handed, y up hint given by the camera, vertical FOV)
dt_status make_camera(const dt_camera& cam, int index, CamDev& cd);

// chunked compaction scan shared by the tracer and the server (trace.hip)
constexpr int DT_CHUNK = 2048;
dt_status chunk_scan(Counters* ctr, int g, unsigned long long* part, unsigned long long* other,
                     int64_t other_n, int64_t cap_next, hipStream_t s);

// environment MLP launchers (env_mlp.hip)
bool mlp_supported(const EnvDev& e);
dt_status mlp_query(const EnvDev& e, const float* dirs, int64_t n, float* rgb, hipStream_t s);
dt_status mlp_query_backward(const EnvDev& e, const float* dirs, int64_t n, const float* g,
                             float* gd, hipStream_t s);
// forward: E for the rays on the miss list of generation g, rgb[pixel] += W * E
dt_status mlp_trace_forward(const EnvDev& e, Gen q, const uint32_t* list, const Counters* ctr,
                            int g, int64_t cap, float* rgb, hipStream_t s);
// adjoint: for the rays on the list, L = E(d), D = (dE/dd)^T (dLoss/dC * W), O = 0
dt_status mlp_trace_backward(const EnvDev& e, Gen q, const uint32_t* list, const Counters* ctr,
                             int g, int64_t cap, const float* grad_rgb, Adj cur, hipStream_t s);
// the same adjoint, also adding each block's share of dLoss/d(weights, biases)
// into its row of part (rows of mlp_wgrad_params(e) floats, zeroed by the
// caller before the first generation); 64-wide networks
dt_status mlp_trace_backward_wgrad(const EnvDev& e, Gen q, const uint32_t* list, const Counters* ctr,
                                   int g, const float* grad_rgb, Adj cur, float* part, hipStream_t s);
// e.d_w / e.d_b = the rows of part summed in order
dt_status mlp_wgrad_reduce(const EnvDev& e, const float* part, hipStream_t s);
// parameters of a network (0 when the weight gradient is not supported), and
// the scratch bytes the partial sums of the largest supported one need
int64_t mlp_wgrad_params(const EnvDev& e);
size_t mlp_wgrad_scratch_bytes();
