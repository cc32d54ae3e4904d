// Wavefront recursive tracer (forward and adjoint) on the device.
//
// Rays are processed one generation at a time (generation g = rays created by
// g surface interactions; camera rays are generation 0).  Per generation:
//   k_trace : closest hit + shading decisions for every ray of the queue;
//             misses add W * E(d) to their pixel; counts of the children
//             each chunk of the queue will emit are accumulated.
//   k_scan  : exclusive scan of the per-chunk child counts.
//   k_emit  : every ray writes its reflected / refracted child into the next
//             queue at its scanned position (stable: the order of generation
//             g+1 is a pure function of generation g, so a recomputation
//             reproduces it bit for bit).
// The adjoint walks the generations backwards, each node gathering the
// subtree radiance and ray adjoints of its (at most two) children.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "dt_queue.h"

namespace {

constexpr int TB = 64;                // threads per block of the traversal kernel (one wave)
constexpr int CHUNK = DT_CHUNK;       // rays per compaction chunk
constexpr int EB = 256;               // threads per block of the emit kernel
constexpr int AB = 256;               // threads per block of the adjoint kernel
constexpr int ADJ_MAX_BLOCKS = 4096;  // grid cap of the adjoint kernel
constexpr int TRACE_MAX_BLOCKS = 256 * 4 * 7;  // grid cap of the traversal kernel: 7 resident waves per SIMD
constexpr size_t GG_SCRATCH = (size_t)32 << 20;  // workspace bytes for copies of the absorption-grid gradient
constexpr size_t FG_SCRATCH = (size_t)32 << 20;  // workspace bytes for copies of the field gradient's cell records
// Vertex adjoints of one hit, stored per node and summed per face afterwards:
// d/d p0, p1, p2 and the shading-normal adjoint mbar with the barycentrics
// (vertex normal k receives mbar b_k; mbar = 0 on flat-shaded hits).
struct FaceRec {
  float4 a;  // p0bar, b1
  float4 b;  // p1bar, b2
  float4 c;  // p2bar, -
  float4 m;  // mbar, -
};

// ------------------------------------------------------------------ plan
struct Plan {
  int D, k;
  int64_t N, npix;
  int64_t cap[DT_MAX_DEPTH + 2];
  int64_t maxcap, maxchunks;
  bool store_all;
  // tape
  size_t tape_hdr;
  size_t t_o[DT_MAX_DEPTH + 1], t_d[DT_MAX_DEPTH + 1], t_w[DT_MAX_DEPTH + 1];
  size_t t_hit[DT_MAX_DEPTH + 1], t_code[DT_MAX_DEPTH + 1], t_child[DT_MAX_DEPTH + 1];
  size_t tape_bytes;
  // workspace
  size_t w_ctr, w_parts, w_part0, w_part1;
  size_t w_ro[2], w_rd[2], w_rw[2], w_hit, w_code;
  size_t w_adj[2][3];
  size_t w_dN, w_sbar, w_red, w_miss, w_ovf, w_gscr, w_mlpg, w_fscr, w_fseg;
  size_t w_frec, w_fkey, w_fidx, w_fcnt, w_foff, w_fscan, w_fg;  // per-face gathering of vertex adjoints
  size_t w_seg_o, w_seg_d, w_seg_w, w_seg_hit, w_seg_code, w_seg_child;  // k generations each
  size_t ws_bytes;
};

bool make_plan(const dt_trace_params* p, int64_t n_rays, int64_t npix, int32_t nv, int32_t nf,
               Plan& P) {
  P.D = p->max_depth;
  P.k = p->checkpoint_stride < 1 ? 1 : p->checkpoint_stride;
  if (P.k > P.D + 1) P.k = P.D + 1;
  P.store_all = P.k == 1;
  P.N = n_rays;
  P.npix = npix;
  int64_t capu = p->queue_capacity;
  P.maxcap = 1;
  for (int g = 0; g <= DT_MAX_DEPTH + 1; ++g) {
    int64_t worst = g <= 40 ? (n_rays << (g > 30 ? 30 : g)) : INT64_MAX;
    int64_t c = g == 0 ? n_rays : (capu > 0 && capu < worst ? capu : worst);
    if (c > (int64_t)0x7fffffff) c = 0x7fffffff;
    if (c < 1) c = 1;
    P.cap[g] = c;
    if (g <= P.D && c > P.maxcap) P.maxcap = c;
  }
  P.maxchunks = (P.maxcap + CHUNK - 1) / CHUNK;
  // tape
  size_t o = 0;
  P.tape_hdr = o;
  o = dt_align(o + sizeof(Counters));
  for (int g = 0; g <= DT_MAX_DEPTH; ++g) {
    P.t_o[g] = P.t_d[g] = P.t_w[g] = P.t_hit[g] = P.t_code[g] = P.t_child[g] = (size_t)-1;
  }
  for (int g = 0; g <= P.D; ++g) {
    bool stored = P.store_all || (g % P.k) == 0;
    if (!stored) continue;
    size_t c = (size_t)P.cap[g];
    P.t_o[g] = o;
    o = dt_align(o + 16 * c);
    P.t_d[g] = o;
    o = dt_align(o + 16 * c);
    P.t_w[g] = o;
    o = dt_align(o + 16 * c);
    if (P.store_all) {
      P.t_hit[g] = o;
      o = dt_align(o + 16 * c);
      P.t_code[g] = o;
      o = dt_align(o + 4 * c);
      P.t_child[g] = o;
      o = dt_align(o + 8 * c);
    }
  }
  P.tape_bytes = o;
  // workspace
  size_t mc = (size_t)P.maxcap;
  o = 0;
  P.w_ctr = o;
  o = dt_align(o + sizeof(Counters));
  P.w_parts = o;  // traversal work cursors, per generation and part
  o = dt_align(o + sizeof(WorkPart) * DT_WORK_PARTS * (DT_MAX_DEPTH + 2));
  P.w_part0 = o;
  o = dt_align(o + 8 * ((size_t)P.maxchunks + 1));
  P.w_part1 = o;
  o = dt_align(o + 8 * ((size_t)P.maxchunks + 1));
  for (int b = 0; b < 2; ++b) {
    P.w_ro[b] = o;
    o = dt_align(o + 16 * mc);
    P.w_rd[b] = o;
    o = dt_align(o + 16 * mc);
    P.w_rw[b] = o;
    o = dt_align(o + 16 * mc);
  }
  P.w_hit = o;
  o = dt_align(o + 16 * mc);
  P.w_code = o;
  o = dt_align(o + 4 * mc);
  for (int b = 0; b < 2; ++b)
    for (int j = 0; j < 3; ++j) {
      P.w_adj[b][j] = o;
      o = dt_align(o + 16 * mc);
    }
  P.w_dN = o;
  o = dt_align(o + 12 * (size_t)nv);
  P.w_sbar = o;
  o = dt_align(o + 16 * (size_t)nv);
  P.w_red = o;  // per-(generation, block) partial sums of dIoR and dsigma
  o = dt_align(o + 16 * (size_t)(DT_MAX_DEPTH + 1) * ADJ_MAX_BLOCKS);
  P.w_miss = o;  // miss list of the current generation (MLP environment)
  o = dt_align(o + 4 * mc);
  P.w_gscr = o;  // copies of the absorption grid's gradient, summed at the end
  o = dt_align(o + GG_SCRATCH);
  P.w_fscr = o;  // copies of the volumetric field's per-cell gradient records
  o = dt_align(o + FG_SCRATCH);
  P.w_fseg = o;  // per node of the current generation: its exterior field segment for k_field_grad
  o = dt_align(o + 32 * mc);
  P.w_mlpg = o;  // per-block partial sums of the environment MLP's weight gradient
  o = dt_align(o + mlp_wgrad_scratch_bytes());
  P.w_ovf = o;   // per-lane traversal stack overflow of the traversal grid
  o = dt_align(o + 8 * (size_t)TRACE_MAX_BLOCKS * TB * (DT_STACK - DT_STACK_LDS));
  P.w_frec = o;  // vertex-adjoint record of each node of the current generation
  o = dt_align(o + sizeof(FaceRec) * mc);
  P.w_fkey = o;  // (face, rank among the face's records) per node
  o = dt_align(o + 8 * mc);
  P.w_fidx = o;  // nodes sorted by face
  o = dt_align(o + 4 * mc);
  P.w_fcnt = o;  // records per face
  o = dt_align(o + 4 * ((size_t)nf + 1));
  P.w_foff = o;  // exclusive scan of the counts
  o = dt_align(o + 4 * ((size_t)nf + 1));
  P.w_fscan = o;  // partial sums of the scan
  o = dt_align(o + 4 * dt_scan_partials_count());
  P.w_fg = o;     // per-face running totals of the vertex adjoints
  o = dt_align(o + 4 * 18 * (size_t)nf);
  size_t kk = P.store_all ? 0 : (size_t)P.k;
  P.w_seg_o = o;
  o = dt_align(o + 16 * mc * kk);
  P.w_seg_d = o;
  o = dt_align(o + 16 * mc * kk);
  P.w_seg_w = o;
  o = dt_align(o + 16 * mc * kk);
  P.w_seg_hit = o;
  o = dt_align(o + 16 * mc * kk);
  P.w_seg_code = o;
  o = dt_align(o + 4 * mc * kk);
  P.w_seg_child = o;
  o = dt_align(o + 8 * mc * kk);
  P.ws_bytes = o;
  return true;
}

// ------------------------------------------------------------------ small kernels
__global__ void k_zero_f32(float* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}
__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

__global__ void k_init_counters(Counters* c, uint32_t n0, WorkPart* wp) {
  for (int i = threadIdx.x; i < (DT_MAX_DEPTH + 2) * DT_WORK_PARTS; i += blockDim.x) wp[i].next = 0;
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    for (int g = 0; g < DT_MAX_DEPTH + 2; ++g) {
      c->count[g] = 0;
      c->nrefl[g] = 0;
      c->hits[g] = 0;
      c->nmiss[g] = 0;
    }
    c->count[0] = n0;
    c->dropped = 0;
  }
}

__global__ void k_load_counters(Counters* c, const Counters* src) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *c = *src;
    for (int g = 0; g < DT_MAX_DEPTH + 2; ++g) c->nmiss[g] = 0;
  }
}

__global__ void k_save_counters(Counters* dst, const Counters* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *c;
}

// cursors of generations g and later, before they are traced again
__global__ void k_reset_work(int g, WorkPart* wp) {
  for (int i = g * DT_WORK_PARTS + threadIdx.x; i < (DT_MAX_DEPTH + 2) * DT_WORK_PARTS; i += blockDim.x)
    wp[i].next = 0;
}

__global__ void k_stats(const Counters* c, int D, const BvhHeader* hdr, int64_t* stats) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int64_t tot = 0, gens = 0, hits = 0;
    for (int i = 0; i < DT_STATS_LEN; ++i) stats[i] = 0;
    for (int g = 0; g <= D; ++g) {
      stats[g] = c->count[g];
      stats[DT_STAT_HITS + g] = c->hits[g];
      tot += c->count[g];
      hits += c->hits[g];
      if (c->count[g]) gens = g + 1;
    }
    stats[DT_STAT_TOTAL] = tot;
    stats[DT_STAT_DROPPED] = c->dropped;
    stats[DT_STAT_GENERATIONS] = gens;
    stats[DT_STAT_BVH_DEPTH] = hdr->depth;
    stats[DT_STAT_TOTAL_HITS] = hits;
  }
}

// ------------------------------------------------------------------ ray generation (a3)
// Pinhole camera rays through pixel centres; 8x8 pixel tiles are laid out
// consecutively in the queue so that a wave starts on a coherent patch.
// up to CAM_BATCH cameras per launch, in queue order: thread r of the launch
// writes ray r of the batch (camera k starts at cam[k].base - cam[0].base)
constexpr int CAM_BATCH = 8;
struct CamBatch {
  CamDev cam[CAM_BATCH];
  int n;
};

__global__ void k_raygen(Gen q, CamBatch cb, int64_t total) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= total) return;
  const int64_t b0 = cb.cam[0].base;
  int k = 0;
  while (k + 1 < cb.n && r >= cb.cam[k + 1].base - b0) ++k;
  const CamDev& c = cb.cam[k];
  int x, y;
  v3 d = camera_ray(c, r - (c.base - b0), x, y);
  int64_t i = b0 + r;
  int pix = (int)(c.pixel_offset + (int64_t)y * c.W + x);
  q.o[i] = make_float4(c.eye[0], c.eye[1], c.eye[2], __int_as_float(-1));
  q.d[i] = make_float4(d.x, d.y, d.z, __int_as_float(pix));
  q.w[i] = make_float4(1.f, 1.f, 1.f, __int_as_float(0));
}

__global__ void k_rays_explicit(Gen q, const float* o, const float* d, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  q.o[i] = make_float4(o[3 * i], o[3 * i + 1], o[3 * i + 2], __int_as_float(-1));
  q.d[i] = make_float4(d[3 * i], d[3 * i + 1], d[3 * i + 2], __int_as_float((int)i));
  q.w[i] = make_float4(1.f, 1.f, 1.f, __int_as_float(0));
}

__device__ __forceinline__ void add_rgb(float* rgb, int pix, v3 v) {
  atomicAdd(rgb + 3 * pix, v.x);
  atomicAdd(rgb + 3 * pix + 1, v.y);
  atomicAdd(rgb + 3 * pix + 2, v.z);
}

__device__ __forceinline__ v3 mul3(v3 a, v3 b) { return mk3(a.x * b.x, a.y * b.y, a.z * b.z); }


// ------------------------------------------------------------------ k_trace (a4 + a5 decisions + a6)
template <bool GRID, bool FIELD>
__global__ void __launch_bounds__(TB, FIELD ? 4 : 7) k_trace(SceneDev sc, Gen q, int g, Counters* ctr,
                                              unsigned long long* part, float* rgb, float* wtrunc,
                                              int32_t* flags, unsigned long long* sig,
                                              int accumulate, uint2* ovf, WorkPart* wp, float4* att) {
  __shared__ uint2 stk[DT_STACK_LDS * TB];
  __shared__ LeafQueue lq;
  uint2* gstk = ovf + (size_t)(blockIdx.x * TB + threadIdx.x) * (DT_STACK - DT_STACK_LDS);
  const uint32_t n = ctr->count[g];
  const int lane = threadIdx.x & 63;
  const uint32_t nb = (n + 63u) / 64u;
  const uint32_t x0 = blockIdx.x % (unsigned)DT_WORK_PARTS;
  uint32_t p = x0, batch = 0;
  wp += (size_t)g * DT_WORK_PARTS;
  while (claim_batch(wp, nb, x0, p, batch)) {
    const uint32_t base = batch * 64u;
    uint32_t i = base + lane;
    bool active = i < n;
    bool has_r = false, has_t = false, hit = false;
    float4 o4 = make_float4(0.f, 0.f, 0.f, __int_as_float(-1)), d4 = make_float4(0.f, 0.f, 1.f, 0.f);
    if (active) {
      o4 = q.o[i];
      d4 = q.d[i];
    }
    bool ovf = false;
    const Hit h = closest_hit_wave<DT_STACK_LDS, true, false>(sc.bvh, active, xyz(o4), xyz(d4),
                                                              __float_as_int(o4.w), sc.t_eps,
                                                              stk + threadIdx.x, TB, gstk,
                                                              DT_STACK - DT_STACK_LDS, lq, &ovf);
    if (active) {
      // reloaded rather than kept in registers through the traversal
      o4 = q.o[i];
      d4 = q.d[i];
      const float4 w4 = q.w[i];
      v3 o = xyz(o4), d = xyz(d4), W = xyz(w4);
      int pix = __float_as_int(d4.w);
      uint32_t rfl = (uint32_t)__float_as_int(w4.w);
      q.hit[i] = make_float4(h.t, __int_as_float(h.tri), h.b1, h.b2);
      uint32_t code = 0;
      int pf = ovf ? DT_FLAG_STACK : 0;
      if (h.tri < 0) {
        if (rfl & RAY_INSIDE) pf |= DT_FLAG_LEAK;
        // equirect lookups here; MLP lookups are listed afterwards and run in
        // batches on the matrix cores
        if (accumulate && sc.env.kind == DT_ENV_EQUIRECT) {
          v3 E = env_equirect(sc.env, d);
          if constexpr (FIELD) {
            if (!(rfl & RAY_INSIDE)) {
              // the field along the ray to the far side of its box, then the
              // environment beyond
              v3 C;
              float T;
              field_segment(sc.fd, o, d, 0.f, true, C, T);
              E = C + E * T;
            }
          }
          add_rgb(rgb, pix, mul3(W, E));
        }
      } else {
        hit = true;
        HitGeo geo = load_geo(sc, h.tri);
        Shade s = shade<GRID, FIELD>(sc, geo, o, d, h.t, h.b1, h.b2, 0u);
        if constexpr (FIELD) {
          if (accumulate && (s.code & C_ENTER)) add_rgb(rgb, pix, mul3(W, s.Cem));
        }
        // the segment's attenuation (a sum over samples of the grid or the
        // field) handed to k_emit
        if constexpr (GRID || FIELD) {
          if (att) att[i] = make_float4(s.A.x, s.A.y, s.A.z, 0.f);
        }
        code = s.code;
        if (code & C_DEGEN) pf |= DT_FLAG_DEGEN;
        if (code & C_GRAZE) pf |= DT_FLAG_GRAZING;
        if (code & C_TIRB) pf |= DT_FLAG_TIRB;
        if (g >= sc.max_depth) {
          code |= C_TRUNC;
          pf |= DT_FLAG_TRUNC;
          if (accumulate) {
            v3 wa = mul3(W, s.A);
            if (wtrunc) add_rgb(wtrunc, pix, wa);
            if (sc.terminal_env) add_rgb(rgb, pix, mul3(wa, env_equirect(sc.env, d)));
          }
        } else {
          code |= C_HAS_R;
          has_r = true;
          if (!(code & C_TIR)) {
            code |= C_HAS_T;
            has_t = true;
          }
        }
      }
      q.code[i] = code;
      if (accumulate && flags && pf) atomicOr(flags + pix, pf);
      if (accumulate && sig) {
        bool tir = (code & C_TIR) && !(code & C_TRUNC);
        uint64_t key = ((uint64_t)(uint32_t)g << 40) | ((uint64_t)(tir ? 1u : 0u) << 32) |
                       (uint64_t)(uint32_t)(h.tri + 1);
        atomicAdd(sig + pix, (unsigned long long)path_mix64(key));
      }
    }
    uint64_t br = __ballot(has_r), bt = __ballot(has_t), bh = __ballot(hit);
    if (lane == 0 && (br | bt))
      atomicAdd(part + base / CHUNK,
                (unsigned long long)__popcll(br) | ((unsigned long long)__popcll(bt) << 32));
    if (lane == 0 && bh && accumulate) atomicAdd(&ctr->hits[g], (uint32_t)__popcll(bh));
  }
}

// ------------------------------------------------------------------ k_scan (compaction offsets)
// Single block: exclusive scan of the per-chunk (reflect | refract << 32)
// counts of generation g, next-generation count and reset of the other
// partial array.
__global__ void k_scan(Counters* ctr, int g, unsigned long long* part, unsigned long long* other,
                       int64_t other_n, int64_t cap_next) {
  __shared__ unsigned long long sh[1024];
  const uint32_t n = ctr->count[g];
  const int64_t nch = ((int64_t)n + CHUNK - 1) / CHUNK;
  unsigned long long carry = 0;
  for (int64_t base = 0; base < nch; base += blockDim.x) {
    int64_t i = base + threadIdx.x;
    unsigned long long v = i < nch ? part[i] : 0ull;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
      unsigned long long x = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0ull;
      __syncthreads();
      sh[threadIdx.x] += x;
      __syncthreads();
    }
    unsigned long long inc = sh[threadIdx.x];
    unsigned long long tot = sh[blockDim.x - 1];
    if (i < nch) part[i] = carry + inc - v;
    carry += tot;
    __syncthreads();
  }
  for (int64_t i = threadIdx.x; i < other_n; i += blockDim.x) other[i] = 0ull;
  if (threadIdx.x == 0) {
    uint32_t nr = (uint32_t)(carry & 0xffffffffull), nt = (uint32_t)(carry >> 32);
    uint64_t tot = (uint64_t)nr + nt;
    ctr->nrefl[g] = nr;
    ctr->count[g + 1] = (uint32_t)(tot < (uint64_t)cap_next ? tot : (uint64_t)cap_next);
  }
}

// ------------------------------------------------------------------ k_emit (a5 children)
// Block b re-walks chunk b in order and writes each ray's children at its
// scanned position: reflected children fill [0, n_r) of the next queue,
// refracted children [n_r, n_r + n_t).  write_rays = 0 computes indices only.
template <bool GRID, bool FIELD>
__global__ void __launch_bounds__(EB) k_emit(SceneDev sc, Gen q, Gen nx, int g, Counters* ctr,
                                             const unsigned long long* part, int64_t cap_next,
                                             int write_rays, int32_t* flags, const float4* att) {
  __shared__ uint32_t wr[EB / 64], wt[EB / 64];
  const uint32_t n = ctr->count[g];
  const int64_t base = (int64_t)blockIdx.x * CHUNK;
  if (base >= n) return;
  const uint32_t nr_tot = ctr->nrefl[g];
  unsigned long long c = part[blockIdx.x];
  uint32_t carry_r = (uint32_t)(c & 0xffffffffull), carry_t = (uint32_t)(c >> 32);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  for (int s = 0; s < CHUNK / EB; ++s) {
    int64_t i = base + (int64_t)s * EB + threadIdx.x;
    bool active = i < n;
    uint32_t code = active ? q.code[i] : 0u;
    bool hr = (code & C_HAS_R) != 0u, ht = (code & C_HAS_T) != 0u;
    uint64_t br = __ballot(hr), bt = __ballot(ht);
    if (lane == 0) {
      wr[wv] = (uint32_t)__popcll(br);
      wt[wv] = (uint32_t)__popcll(bt);
    }
    __syncthreads();
    uint32_t or_ = 0, ot = 0, tr = 0, tt = 0;
    for (int k = 0; k < EB / 64; ++k) {
      if (k < wv) {
        or_ += wr[k];
        ot += wt[k];
      }
      tr += wr[k];
      tt += wt[k];
    }
    uint32_t ir = carry_r + or_ + (uint32_t)__popcll(br & lt);
    uint32_t it = nr_tot + carry_t + ot + (uint32_t)__popcll(bt & lt);
    if (active) {
      int cr = -1, ctd = -1;
      if (hr || ht) {
        float4 o4 = q.o[i], d4 = q.d[i], w4 = q.w[i], h4 = q.hit[i];
        v3 o = xyz(o4), d = xyz(d4), W = xyz(w4);
        int pix = __float_as_int(d4.w);
        int tri = __float_as_int(h4.y);
        HitGeo geo = load_geo(sc, tri);
        Shade sh;
        if constexpr (GRID || FIELD) {
          if (att) {
            // the decisions from the code and the attenuation k_trace computed
            // (bit for bit what shade<GRID, FIELD> gives here)
            sh = shade<false, false>(sc, geo, o, d, h4.x, h4.z, h4.w, code);
            sh.A = xyz(att[i]);
          } else {
            sh = shade<GRID, FIELD>(sc, geo, o, d, h4.x, h4.z, h4.w, code);
          }
        } else {
          sh = shade<false, false>(sc, geo, o, d, h4.x, h4.z, h4.w, code);
        }
        v3 wa = mul3(W, sh.A);
        bool entering = (code & C_ENTER) != 0u;
        if (hr) {
          if ((int64_t)ir < cap_next) {
            cr = (int)ir;
            if (write_rays) {
              nx.o[ir] = make_float4(sh.x.x, sh.x.y, sh.x.z, __int_as_float(tri));
              nx.d[ir] = make_float4(sh.dr.x, sh.dr.y, sh.dr.z, __int_as_float(pix));
              v3 wr3 = wa * sh.R;
              nx.w[ir] = make_float4(wr3.x, wr3.y, wr3.z, __int_as_float(entering ? 0 : (int)RAY_INSIDE));
            }
          } else if (write_rays) {
            atomicAdd(&ctr->dropped, 1u);
            if (flags) atomicOr(flags + pix, DT_FLAG_OVERFLOW);
          }
        }
        if (ht) {
          if ((int64_t)it < cap_next) {
            ctd = (int)it;
            if (write_rays) {
              nx.o[it] = make_float4(sh.x.x, sh.x.y, sh.x.z, __int_as_float(tri));
              nx.d[it] = make_float4(sh.dt.x, sh.dt.y, sh.dt.z, __int_as_float(pix));
              v3 wt3 = wa * sh.T;
              nx.w[it] = make_float4(wt3.x, wt3.y, wt3.z, __int_as_float(entering ? (int)RAY_INSIDE : 0));
            }
          } else if (write_rays) {
            atomicAdd(&ctr->dropped, 1u);
            if (flags) atomicOr(flags + pix, DT_FLAG_OVERFLOW);
          }
        }
      }
      if (q.child) q.child[i] = make_int2(cr, ctd);
    }
    carry_r += tr;
    carry_t += tt;
    __syncthreads();
  }
}

// ------------------------------------------------------------------ adjoint (a7)
__device__ __forceinline__ v3 norm_bwd(v3 u, v3 uhat, v3 gbar) {
  float il = 1.0f / len3(u);
  return (gbar - uhat * dot(uhat, gbar)) * il;
}

__device__ __forceinline__ void atomic_add3(float* p, int idx, v3 v) {
  atomicAdd(p + 3 * idx, v.x);
  atomicAdd(p + 3 * idx + 1, v.y);
  atomicAdd(p + 3 * idx + 2, v.z);
}

// Vertex contributions of one hit node: dLoss/dp_k for its three vertices and
// dLoss/dN_k for their normals (absent where the geometric normal was used).
// Adjoint of tau = absorb_tau(G, o, d, t), in one pass over the interior
// segment's samples that also gives tau itself (the same operations as
// absorb_tau, so the same bits).  Sample k sits at x_k = o + a_k d with
// a_k = (k + 1/2) t / S, and tau = (t / S) sum_k mu(x_k), so for the
// per-channel taubar the adjoint adds h taubar . grad mu(x_k) to obar,
// a_k times that to dbar and, through h and a_k, (k + 1/2)/S of its dot with
// d plus taubar . mu(x_k) / S to tbar.  Being linear in taubar (not known
// until the attenuation A = exp(-tau) has been used), it is kept per channel
// c: G_c = sum_k h grad mu_c(x_k), D_c = sum_k a_k h grad mu_c(x_k) and
// T_c = sum_k (k + 1/2)/S h grad mu_c(x_k) . d + sum_k mu_c(x_k) / S, then
// obar += sum_c taubar_c G_c, dbar += sum_c taubar_c D_c and
// tbar += sum_c taubar_c T_c.  The gradient of the trilinear interpolant is
// read off the differences along x, then y, then z; the grid values' own
// terms are scattered by k_grid_grad.
struct TauSums {
  v3 tau;
  v3 G[3], D[3];
  float T[3];
};

__device__ __forceinline__ void absorb_tau_sums(const AbsorbDev& G, v3 o, v3 d, float t, TauSums& r) {
  const float S = (float)G.samples, h = t / S;
  const size_t sy = 3 * (size_t)G.nx, sz = sy * (size_t)G.ny;
  v3 acc = mk3(0.f, 0.f, 0.f);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    r.G[c] = mk3(0.f, 0.f, 0.f);
    r.D[c] = r.G[c];
    r.T[c] = 0.f;
  }
  for (int k = 0; k < G.samples; ++k) {
    const float a = h * ((float)k + 0.5f);
    const v3 x = o + d * a;
    acc = acc + grid_mu(G, x);
    const GridAxis ax = grid_axis(x.x, G.lo[0], G.scale[0], G.nx);
    const GridAxis ay = grid_axis(x.y, G.lo[1], G.scale[1], G.ny);
    const GridAxis az = grid_axis(x.z, G.lo[2], G.scale[2], G.nz);
    const size_t b = (size_t)az.i * sz + (size_t)ay.i * sy + 3 * (size_t)ax.i;
    const float wk = ((float)k + 0.5f) / S;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float u[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) u[q] = G.mu[b + (q >> 2) * sz + ((q >> 1) & 1) * sy + 3 * (q & 1) + c];
      // x differences on the 4 (y, z) edges, values along x; then y, then z
      float ex[4], lx[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        ex[e] = u[2 * e + 1] - u[2 * e];
        lx[e] = u[2 * e] + ax.f * ex[e];
      }
      const float ey0 = lx[1] - lx[0], ey1 = lx[3] - lx[2];
      const float ez = (lx[2] + ay.f * ey1) - (lx[0] + ay.f * ey0);
      const float gx0 = ex[0] + ay.f * (ex[1] - ex[0]), gx1 = ex[2] + ay.f * (ex[3] - ex[2]);
      const float gx = gx0 + az.f * (gx1 - gx0);
      const float gy = ey0 + az.f * (ey1 - ey0);
      const v3 q = mk3(ax.in ? gx * G.scale[0] * h : 0.f, ay.in ? gy * G.scale[1] * h : 0.f,
                       az.in ? ez * G.scale[2] * h : 0.f);
      r.G[c] += q;
      r.D[c] += q * a;
      r.T[c] += dot(q, d) * wk;
    }
  }
  r.tau = acc * h;
  const float Ms[3] = {acc.x, acc.y, acc.z};
#pragma unroll
  for (int c = 0; c < 3; ++c) r.T[c] += Ms[c] / S;
}

struct VtxAdj {
  int f;  // hit face, < 0: no contributions
  v3 p0, p1, p2, m;
  float b1, b2;
};

// Adjoint of node i of generation g: writes its record (subtree radiance,
// d/d origin, d/d direction) to cur, adds its dIoR / dsigma terms to acc and
// returns its vertex contributions.
template <bool GRID, bool FIELD>
__device__ __forceinline__ void adjoint_node(const SceneDev& sc, const Gen& q, int64_t i,
                                             const float* grad_rgb, const Adj& nxt, const Adj& cur,
                                             float4& acc, VtxAdj& out, float4* fseg) {
  float4 o4 = q.o[i], d4 = q.d[i], w4 = q.w[i], h4 = q.hit[i];
  uint32_t code = q.code[i];
  v3 o = xyz(o4), d = xyz(d4), W = xyz(w4);
  int pix = __float_as_int(d4.w);
  v3 gp = load3(grad_rgb + 3 * pix);
  v3 gW = mul3(gp, W);
  // With fseg, the field parameters' gradient is left to k_field_grad: this
  // node's exterior segment (radiance beyond it, its upstream gradient, end
  // and kind) goes to fseg and the backward here takes the ray's terms only.
  FieldDev fdv = sc.fd;
  if constexpr (FIELD) {
    if (fseg) {
      fdv.d_grid = nullptr;
      fdv.d_planes = nullptr;
      fseg[2 * i + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  if (!(code & C_HIT)) {
    if (sc.env.kind != DT_ENV_EQUIRECT) return;  // written by the MLP kernel
    v3 dd;
    if constexpr (FIELD) {
      if (!(__float_as_uint(w4.w) & RAY_INSIDE)) {
        // L = C + T E along the exterior ray
        v3 C;
        float T;
        field_segment(sc.fd, o, d, 0.f, true, C, T);
        v3 E = env_equirect_grad(sc.env, d, gW * T, &dd);
        v3 ob = mk3(0.f, 0.f, 0.f);
        float tb = 0.f;
        const v3 L = C + E * T;
        field_segment_bwd(fdv, o, d, 0.f, true, L, gW, ob, dd, tb);
        if (fseg) {
          fseg[2 * i] = make_float4(L.x, L.y, L.z, 0.f);
          fseg[2 * i + 1] = make_float4(gW.x, gW.y, gW.z, 2.f);  // open segment
        }
        cur.L[i] = make_float4(L.x, L.y, L.z, 0.f);
        cur.O[i] = make_float4(ob.x, ob.y, ob.z, 0.f);
        cur.D[i] = make_float4(dd.x, dd.y, dd.z, 0.f);
        return;
      }
    }
    v3 E = env_equirect_grad(sc.env, d, gW, &dd);
    cur.L[i] = make_float4(E.x, E.y, E.z, 0.f);
    cur.O[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    cur.D[i] = make_float4(dd.x, dd.y, dd.z, 0.f);
    return;
  }
  bool trunc = (code & C_TRUNC) != 0u;
  // with a field, a truncated hit reached from outside still emits its segment
  const bool field_seg = FIELD && (code & C_ENTER) != 0u;
  if (trunc && !sc.terminal_env && !field_seg) {
    cur.L[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    cur.O[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    cur.D[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  float t = h4.x, b1 = h4.z, b2 = h4.w;
  int tri = __float_as_int(h4.y);
  HitGeo geo = load_geo(sc, tri);
  // with the grid, the interior segment's attenuation and its adjoint sums
  // come from one pass over its samples (shade<false> leaves A to it)
  Shade s = shade<false, FIELD>(sc, geo, o, d, t, b1, b2, code);
  const bool entering = (code & C_ENTER) != 0u, tir = (code & C_TIR) != 0u;
  TauSums ts;
  if constexpr (GRID) {
    if (!entering) {
      absorb_tau_sums(sc.ab, o, d, t, ts);
      s.A = mk3(expf(-ts.tau.x), expf(-ts.tau.y), expf(-ts.tau.z));
    }
  }
  const bool degen = (code & C_DEGEN) != 0u;
  v3 L, Abar, dbar = mk3(0.f, 0.f, 0.f), xbar = mk3(0.f, 0.f, 0.f), nbar = mk3(0.f, 0.f, 0.f);
  v3 Mf = mk3(0.f, 0.f, 0.f);  // radiance beyond the hit (the field segment's far side)
  float cibar = 0.f, ctbar = 0.f, etarbar = 0.f, etaibar = 0.f, etatbar = 0.f;
  if (trunc) {
    if (sc.terminal_env) {
      // terminal mode ENV: L = A * E(d)
      v3 dd;
      v3 E = env_equirect_grad(sc.env, d, mul3(gW, s.A), &dd);
      L = mul3(s.A, E);
      Abar = mul3(gW, E);
      dbar = dd;
      Mf = E;
    } else {
      L = mk3(0.f, 0.f, 0.f);
      Abar = L;
    }
  } else {
    int2 ch = q.child[i];
    v3 Lr = mk3(0.f, 0.f, 0.f), Lt = mk3(0.f, 0.f, 0.f), drb = Lr, dtb = Lr;
    if (ch.x >= 0) {
      Lr = xyz(nxt.L[ch.x]);
      xbar += xyz(nxt.O[ch.x]);
      drb = xyz(nxt.D[ch.x]);
    }
    if (ch.y >= 0) {
      Lt = xyz(nxt.L[ch.y]);
      xbar += xyz(nxt.O[ch.y]);
      dtb = xyz(nxt.D[ch.y]);
    }
    v3 M = Lr * s.R + Lt * s.T;
    L = mul3(s.A, M);
    Abar = mul3(gW, M);
    Mf = M;
    // reflected direction u_r = d + 2 cos_i n (Eq. 3)
    v3 urb = norm_bwd(s.ur, s.dr, drb);
    dbar += urb;
    cibar += 2.f * dot(s.n, urb);
    nbar += urb * (2.f * s.cos_i);
    if (!tir) {
      // Fresnel weights (Eq. 7-8): dL/dR with T = 1 - R
      float Rbar = dot(mul3(gW, s.A), Lr - Lt);
      // refracted direction u_t = d / eta_r + (cos_i / eta_r - cos_t) n (Eq. 4-6)
      v3 utb = norm_bwd(s.ut, s.dt, dtb);
      float nu = dot(s.n, utb);
      float ier = 1.f / s.eta_r;
      dbar += utb * ier;
      etarbar += -dot(d, utb) * ier * ier - s.cos_i * ier * ier * nu;
      cibar += nu * ier;
      ctbar += -nu;
      nbar += utb * (s.cos_i * ier - s.cos_t);
      float a = s.eta_i * s.cos_i, b = s.eta_t * s.cos_t;
      float c = s.eta_i * s.cos_t, e = s.eta_t * s.cos_i;
      float rsb = Rbar * s.rs, rpb = Rbar * s.rp;
      float ab2 = (a + b) * (a + b), ce2 = (c + e) * (c + e);
      float abar = rsb * 2.f * b / ab2, bbar = -rsb * 2.f * a / ab2;
      float cbar = rpb * 2.f * e / ce2, ebar = -rpb * 2.f * c / ce2;
      cibar += abar * s.eta_i + ebar * s.eta_t;
      ctbar += bbar * s.eta_t + cbar * s.eta_i;
      etaibar += abar * s.cos_i + cbar * s.cos_t;
      etatbar += bbar * s.cos_t + ebar * s.cos_i;
      // cos_t = sqrt(1 - sin^2 t), sin^2 t = (1 - cos_i^2) / eta_r^2
      if (s.cos_t > 0.f) {
        float s2b = -ctbar / (2.f * s.cos_t);
        cibar += s2b * (-2.f * s.cos_i * ier * ier);
        etarbar += s2b * (-2.f * (1.f - s.cos_i * s.cos_i) * ier * ier * ier);
      }
    }
  }
  // IoR: entering eta_i = 1, eta_t = eta_r = eta; leaving eta_i = eta, eta_t = 1, eta_r = 1/eta
  float etabar = entering ? (etatbar + etarbar) : (etaibar - etarbar / (s.eta * s.eta));
  acc.x += etabar;
  // absorption on interior segments (Eq. 11): A = exp(-tau), tau = sigma t or
  // the grid's sum over the segment's samples
  float tbar = 0.f;
  v3 oabs = mk3(0.f, 0.f, 0.f), taubar = oabs;
  if (GRID && !entering) {
    taubar = -mul3(Abar, s.A);
    if constexpr (GRID) {
      const float tb[3] = {taubar.x, taubar.y, taubar.z};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        oabs += ts.G[c] * tb[c];
        dbar += ts.D[c] * tb[c];
        tbar += ts.T[c] * tb[c];
      }
    }
  } else if (!entering) {
    float sg0 = sc.sigma[0], sg1 = sc.sigma[1], sg2 = sc.sigma[2];
    acc.y += -Abar.x * t * s.A.x;
    acc.z += -Abar.y * t * s.A.y;
    acc.w += -Abar.z * t * s.A.z;
    tbar += -(Abar.x * sg0 * s.A.x + Abar.y * sg1 * s.A.y + Abar.z * sg2 * s.A.z);
  }
  if constexpr (FIELD) {
    if (field_seg) {
      // L = C + T M over the exterior segment [0, t]; T's effect on M is in
      // the field's backward (A = T is not used for the attenuation here)
      L = L + s.Cem;
      // the segment's radiance C + T M (A = T here)
      const v3 Lseg = s.Cem + Mf * s.A.x;
      field_segment_bwd(fdv, o, d, t, false, Lseg, gW, oabs, dbar, tbar);
      if (fseg) {
        fseg[2 * i] = make_float4(Lseg.x, Lseg.y, Lseg.z, t);
        fseg[2 * i + 1] = make_float4(gW.x, gW.y, gW.z, 1.f);  // closed segment [0, t]
      }
    }
  }
  // cos_i = -d . n
  dbar += s.n * (-cibar);
  nbar += d * (-cibar);
  // children start at x = o + t d
  v3 obar = xbar + oabs;
  dbar += xbar * t;
  tbar += dot(d, xbar);
  // shading normal n = +-normalize(m), m = sum b_k N_k (Eq. 12)
  const float sgn = entering ? 1.f : -1.f;
  v3 p0b = mk3(0.f, 0.f, 0.f), p1b = p0b, p2b = p0b;
  float b1bar = 0.f, b2bar = 0.f;
  v3 e1 = geo.p1 - geo.p0, e2 = geo.p2 - geo.p0;
  if (!degen) {
    v3 nh = normalize3(s.m);
    v3 mbar = norm_bwd(s.m, nh, nbar * sgn);
    out.m = mbar;
    b1bar += dot(geo.n1 - geo.n0, mbar);
    b2bar += dot(geo.n2 - geo.n0, mbar);
  } else {
    v3 ng = cross(e1, e2);
    v3 nh = normalize3(ng);
    v3 ngbar = norm_bwd(ng, nh, nbar * sgn);
    v3 e1b = cross(e2, ngbar), e2b = cross(ngbar, e1);
    p1b += e1b;
    p2b += e2b;
    p0b += -(e1b + e2b);
  }
  // differentiable intersection (t, b1, b2 as functions of o, d, p0, p1, p2)
  {
    v3 sv = o - geo.p0;
    v3 pv = cross(d, e2);
    float det = dot(e1, pv);
    float inv = 1.f / det;
    v3 qv = cross(sv, e1);
    float invbar = tbar * dot(e2, qv) + b1bar * dot(sv, pv) + b2bar * dot(d, qv);
    v3 e2b = qv * (tbar * inv);
    v3 qb = e2 * (tbar * inv) + d * (b2bar * inv);
    dbar += qv * (b2bar * inv);
    v3 svb = pv * (b1bar * inv);
    v3 pb = sv * (b1bar * inv);
    float detbar = -invbar * inv * inv;
    v3 e1b = pv * detbar;
    pb += e1 * detbar;
    svb += cross(e1, qb);
    e1b += cross(qb, sv);
    dbar += cross(e2, pb);
    e2b += cross(pb, d);
    obar += svb;
    p0b += -(svb + e1b + e2b);
    p1b += e1b;
    p2b += e2b;
  }
  out.f = tri < 0 ? 0 : (tri >= sc.nf ? sc.nf - 1 : tri);
  out.b1 = b1;
  out.b2 = b2;
  out.p0 = p0b;
  out.p1 = p1b;
  out.p2 = p2b;
  // the unused fourth components carry dLoss/d(optical depth) of an interior
  // segment through an absorption grid to k_grid_grad (0 elsewhere)
  cur.L[i] = make_float4(L.x, L.y, L.z, taubar.x);
  cur.O[i] = make_float4(obar.x, obar.y, obar.z, taubar.y);
  cur.D[i] = make_float4(dbar.x, dbar.y, dbar.z, taubar.z);
}

// The vertex adjoints of a generation are gathered per face without float
// atomics per hit: each hit node writes its FaceRec and takes a rank among its
// face's records (one integer atomic); a scan of the per-face counts and a
// scatter sort the nodes by face; then each face sums its records and adds
// the totals to its three vertices (18 atomics per hit face instead of 18 per
// hit).
// (the field's instantiations, whose segment replays hold some 300 registers
// a lane, are held to 256 so that two waves share a SIMD)
template <bool GRID, bool FIELD>
__global__ void __launch_bounds__(AB, FIELD ? 2 : 1) k_adjoint(SceneDev sc, Gen q, int g, const Counters* ctr,
                                                const float* grad_rgb, Adj nxt, Adj cur,
                                                FaceRec* frec, int2* fkey, uint32_t* fcnt,
                                                float4* red, float4* fseg) {
  const int64_t n = ctr->count[g];
  // each block takes one contiguous range of the generation, AB nodes a step
  const int64_t per = ((n + gridDim.x - 1) / gridDim.x + AB - 1) / AB * AB;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int64_t base = lo; base < hi; base += AB) {
    int64_t i = base + threadIdx.x;
    if (i >= hi) break;
    VtxAdj va;
    va.f = -1;
    va.m = mk3(0.f, 0.f, 0.f);
    adjoint_node<GRID, FIELD>(sc, q, i, grad_rgb, nxt, cur, acc, va, fseg);
    int2 key = make_int2(-1, 0);
    if (va.f >= 0) {
      FaceRec r;
      r.a = make_float4(va.p0.x, va.p0.y, va.p0.z, va.b1);
      r.b = make_float4(va.p1.x, va.p1.y, va.p1.z, va.b2);
      r.c = make_float4(va.p2.x, va.p2.y, va.p2.z, 0.f);
      r.m = make_float4(va.m.x, va.m.y, va.m.z, 0.f);
      frec[i] = r;
      key = make_int2(va.f, (int)atomicAdd(fcnt + va.f, 1u));
    }
    fkey[i] = key;
  }
  const float acc_eta = acc.x, acc_s0 = acc.y, acc_s1 = acc.z, acc_s2 = acc.w;
  // block reduction of the scalar gradients
  __shared__ float red_s[4][AB];
  red_s[0][threadIdx.x] = acc_eta;
  red_s[1][threadIdx.x] = acc_s0;
  red_s[2][threadIdx.x] = acc_s1;
  red_s[3][threadIdx.x] = acc_s2;
  __syncthreads();
  for (int st = AB / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int k = 0; k < 4; ++k) red_s[k][threadIdx.x] += red_s[k][threadIdx.x + st];
    __syncthreads();
  }
  // one slot per block: the final sum runs in a fixed order, so the scalar
  // gradients do not depend on the order blocks finish in
  if (threadIdx.x == 0)
    red[(size_t)g * ADJ_MAX_BLOCKS + blockIdx.x] = make_float4(red_s[0][0], red_s[1][0], red_s[2][0],
                                                               red_s[3][0]);
}

// ------------------------------------------------------------------ absorption grid gradient
// dLoss/d(grid value) of generation g's interior segments: the segment of
// node i adds tw w_j(x_k) at the 8 corner nodes j of the cell of each sample
// x_k (tw = h dLoss/d tau per channel, the same for every sample of the
// segment).  Float atomics to one address from the lanes of one instruction
// are serialized, and neighbouring rays (the lanes of a wave) mostly sample
// the same cells, so the updates are merged before they are issued: a lane
// sums the 8 corner weights of its consecutive samples that fall in the same
// cell (a run), scales them by tw into 24 values; the wave parks its lanes'
// runs in LDS; then per distinct cell among them, lanes 0-23 each sum one of
// the 24 values over the lanes of that cell and add it with one atomic.
// CELL: the sums go to per-cell records of GG_CELL floats (8 corners x 3
// channels, padded to one 128-byte line, so a cell's 24 atomics are one
// memory request), in copy blockIdx.x % copies; k_grid_gather turns the
// records into node values.  Otherwise (a grid whose records do not fit the
// scratch region) they go to the node array itself.  Control flow around the
// LDS exchange stays wave-uniform.
constexpr int GG_T = 256;
constexpr int GG_MAX_COPIES = 64;
constexpr int GG_CELL = 32;
template <bool CELL>
__global__ void __launch_bounds__(GG_T) k_grid_grad(AbsorbDev G, Gen q, int g, const Counters* ctr,
                                                    Adj cur, float* copies, int n_copies) {
  __shared__ float runs[GG_T / 64][64][25];  // per wave and lane: a run's 24 sums (+1 pad)
  const int64_t n = ctr->count[g];
  const int lane = (int)(threadIdx.x & 63u), wv = (int)(threadIdx.x >> 6);
  const int cx = G.nx - 1, cy = G.ny - 1, cz = G.nz - 1;  // cells per axis
  const size_t copy_size = CELL ? (size_t)GG_CELL * cx * cy * cz : 3 * (size_t)G.nx * G.ny * G.nz;
  float* dst = copies + (size_t)(blockIdx.x % (unsigned)n_copies) * copy_size;
  const size_t sy = 3 * (size_t)G.nx, sz = sy * (size_t)G.ny;
  const int S = G.samples;
  for (int64_t base = (int64_t)blockIdx.x * GG_T; base < n; base += (int64_t)gridDim.x * GG_T) {
    const int64_t i = base + threadIdx.x;
    v3 tb = mk3(0.f, 0.f, 0.f), o = tb, d = tb;  // tb: dLoss/d tau from the adjoint record
    float t = 0.f;
    if (i < n) {
      tb = mk3(cur.L[i].w, cur.O[i].w, cur.D[i].w);
      if (tb.x != 0.f || tb.y != 0.f || tb.z != 0.f) {
        o = xyz(q.o[i]);
        d = xyz(q.d[i]);
        t = q.hit[i].x;
      }
    }
    const bool act = tb.x != 0.f || tb.y != 0.f || tb.z != 0.f;
    const float h = t / (float)S;
    const v3 tw = tb * h;
    int k = act ? 0 : S;  // next sample of this lane
    while (__ballot(k < S)) {
      // this lane's next run: samples k, k+1, ... in one cell
      float ws[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) ws[c] = 0.f;
      int key = -1;
      while (k < S) {
        const v3 x = o + d * (h * ((float)k + 0.5f));
        const GridAxis ax = grid_axis(x.x, G.lo[0], G.scale[0], G.nx);
        const GridAxis ay = grid_axis(x.y, G.lo[1], G.scale[1], G.ny);
        const GridAxis az = grid_axis(x.z, G.lo[2], G.scale[2], G.nz);
        const int kk = (az.i * cy + ay.i) * cx + ax.i;
        if (key >= 0 && kk != key) break;
        key = kk;
        const float wy[2] = {1.f - ay.f, ay.f}, wz[2] = {1.f - az.f, az.f};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float yz = wy[c & 1] * wz[c >> 1];
          ws[2 * c] += (1.f - ax.f) * yz;
          ws[2 * c + 1] += ax.f * yz;
        }
        ++k;
      }
      const bool has = key >= 0;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        runs[wv][lane][3 * c] = tw.x * ws[c];
        runs[wv][lane][3 * c + 1] = tw.y * ws[c];
        runs[wv][lane][3 * c + 2] = tw.z * ws[c];
      }
      wave_lds_sync();
      uint64_t pending = __ballot(has);
      while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int kl = __builtin_amdgcn_readlane(key, leader);
        const uint64_t m = __ballot(has && key == kl);
        pending &= ~m;
        if (lane < 24) {
          float sum = 0.f;
          for (uint64_t mm = m; mm; mm &= mm - 1ull) sum += runs[wv][__ffsll((unsigned long long)mm) - 1][lane];
          if (CELL) {
            atomicAdd(dst + (size_t)kl * GG_CELL + lane, sum);
          } else {
            const int cc = lane / 3;  // corner (dx, dy, dz) = bits 0, 1, 2
            const int az_i = kl / (cx * cy), ay_i = (kl / cx) % cy, ax_i = kl % cx;
            atomicAdd(dst + (size_t)(az_i + (cc >> 2)) * sz + (size_t)(ay_i + ((cc >> 1) & 1)) * sy +
                          3 * (size_t)(ax_i + (cc & 1)) + lane % 3,
                      sum);
          }
        }
      }
      wave_lds_sync();
    }
  }
}

// dLoss/dtexel of generation g's equirect lookups: the lookup of node i (a
// miss, or with terminal_env a hit at the depth cap) adds gE w_k at its 4
// bilinear taps, gE = dLoss/dE per channel = grad(pixel) W (times the
// attenuation A of the last segment for a capped hit).  Merged as in
// k_grid_grad: the wave parks its lanes' 12 tap values in LDS and, per
// distinct 2 x 2 texel block among them, lanes 0-11 each sum one tap-channel
// value over the block's lanes and add it with one atomic.
__global__ void __launch_bounds__(GG_T) k_env_tex_grad(SceneDev sc, Gen q, int g, const Counters* ctr,
                                                       const float* grad_rgb) {
  const EnvDev& e = sc.env;
  __shared__ float taps[GG_T / 64][64][13];  // per wave and lane: 4 taps x 3 channels (+1 pad)
  const int64_t n = ctr->count[g];
  const int lane = (int)(threadIdx.x & 63u), wv = (int)(threadIdx.x >> 6);
  for (int64_t base = (int64_t)blockIdx.x * GG_T; base < n; base += (int64_t)gridDim.x * GG_T) {
    const int64_t i = base + threadIdx.x;
    v3 gb = mk3(0.f, 0.f, 0.f);
    bool has = false;
    v3 d = gb;
    if (i < n) {
      const uint32_t code = q.code[i];
      has = !(code & C_HIT) || (sc.terminal_env && (code & C_TRUNC));
      if (has) {
        const float4 d4 = q.d[i], w4 = q.w[i];
        d = xyz(d4);
        gb = mul3(load3(grad_rgb + 3 * __float_as_int(d4.w)), xyz(w4));
        if (sc.fd.grid && ((code & C_HIT) ? (code & C_ENTER) != 0u
                                          : !(__float_as_uint(w4.w) & RAY_INSIDE))) {
          // an exterior segment through the volumetric field: the lookup is
          // weighted by the field's transmittance
          v3 C;
          float T;
          field_segment(sc.fd, xyz(q.o[i]), d, q.hit[i].x, !(code & C_HIT), C, T);
          gb = gb * T;
        }
        if ((code & C_HIT) && !(code & C_ENTER)) {
          // capped hit reached from inside: the lookup is weighted by A
          const float t = q.hit[i].x;
          if (sc.ab.mu) {
            const v3 tau = absorb_tau(sc.ab, xyz(q.o[i]), d, t);
            gb = mul3(gb, mk3(expf(-tau.x), expf(-tau.y), expf(-tau.z)));
          } else {
            gb = mul3(gb, mk3(expf(-sc.sigma[0] * t), expf(-sc.sigma[1] * t), expf(-sc.sigma[2] * t)));
          }
        }
      }
    }
    int key = -1;
    float v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = 0.f;
    if (has) {
      EquirectTap tp;
      equirect_tap(e, d, tp, false);
      // block key: top-left texel and whether the rows differ (clamped rows coincide)
      key = ((tp.y0 << 1) | (tp.y1 != tp.y0 ? 1 : 0)) * e.W + tp.x0;
      const float gx = 1.f - tp.fx, gy = 1.f - tp.fy;
      const float w[4] = {gx * gy, tp.fx * gy, gx * tp.fy, tp.fx * tp.fy};  // (y0,x0) (y0,x1) (y1,x0) (y1,x1)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        v[3 * k] = gb.x * w[k];
        v[3 * k + 1] = gb.y * w[k];
        v[3 * k + 2] = gb.z * w[k];
      }
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) taps[wv][lane][c] = v[c];
    wave_lds_sync();
    uint64_t pending = __ballot(has);
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const int kl = __builtin_amdgcn_readlane(key, leader);
      const uint64_t m = __ballot(has && key == kl);
      pending &= ~m;
      if (lane < 12) {
        float sum = 0.f;
        for (uint64_t mm = m; mm; mm &= mm - 1ull) sum += taps[wv][__ffsll((unsigned long long)mm) - 1][lane];
        const int row = kl / e.W, x0 = kl % e.W;
        const int y0 = row >> 1, y1 = y0 + (row & 1);
        const int k = lane / 3;
        const int y = (k >> 1) ? y1 : y0, x = (k & 1) ? (x0 + 1 == e.W ? 0 : x0 + 1) : x0;
        atomicAdd(e.d_tex + ((size_t)y * e.W + x) * 3 + lane % 3, sum);
      }
    }
    wave_lds_sync();
  }
}

// d_mu from the per-cell records: node (x, y, z) is corner (dx, dy, dz) of
// cell (x - dx, y - dy, z - dz) where that cell exists; summed over corners,
// then copies, in a fixed order
__global__ void k_grid_gather(const float* copies, int n_copies, int nx, int ny, int nz, float* d_mu) {
  const int cx = nx - 1, cy = ny - 1, cz = nz - 1;
  const size_t copy_size = (size_t)GG_CELL * cx * cy * cz;
  const int64_t n = 3 * (int64_t)nx * ny * nz;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int ch = (int)(j % 3);
    const int64_t node = j / 3;
    const int x = (int)(node % nx), y = (int)((node / nx) % ny), z = (int)(node / ((int64_t)nx * ny));
    float acc = 0.f;
    for (int r = 0; r < n_copies; ++r) {
      const float* cp = copies + (size_t)r * copy_size;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int ux = x - (c & 1), uy = y - ((c >> 1) & 1), uz = z - (c >> 2);
        if (ux >= 0 && ux < cx && uy >= 0 && uy < cy && uz >= 0 && uz < cz)
          acc += cp[((size_t)(uz * cy + uy) * cx + ux) * GG_CELL + 3 * c + ch];
      }
    }
    d_mu[j] = acc;
  }
}

// ------------------------------------------------------------------ volumetric field gradient
// dLoss/d(field values) of generation g's exterior segments.  Every sample x_k
// of a segment adds fb_k w_j(x_k) at its 20 taps (fb_k: dLoss/d(feature) of
// the sample, 4 channels; the samples and fb_k as in field_segment_bwd, from
// the segment's radiance and its upstream gradient that k_adjoint left in
// fseg).  The taps of one sample fall in one grid cell (8 corners)
// and one cell of each plane (4 corners), so a sample's contributions are a
// record of 32 values for its grid cell and 16 for each plane cell.  Waves
// step through the samples together; per sample the wave parks its lanes'
// records in LDS and, per distinct cell among them, sums them and adds the
// sums with one atomic per value into that cell's record (grid records of
// FG_GREC floats, plane records of FG_PREC), in copy blockIdx.x % copies;
// k_field_gather turns the records into node values.  Neighbouring rays
// sample the same cells, so a wave's atomics shrink to a few per cell.
constexpr int FG_T = 256;
constexpr int FG_GREC = 32;  // 8 corners x 4 channels
constexpr int FG_PREC = 16;  // 4 corners x 4 channels
constexpr int FG_MAX_COPIES = 16;

__device__ __forceinline__ size_t field_rec_floats(const FieldDev& F) {
  const size_t pc = (size_t)(F.res - 1);
  return (size_t)FG_GREC * (F.nx - 1) * (F.ny - 1) * (F.nz - 1) + 3 * FG_PREC * pc * pc;
}

constexpr int FG_PARK = 52;  // per lane: up to 48 parked values, then up to 3 keys

// the wave's parked grid records (FG_GREC values and a key per lane) summed
// per distinct key and added to base + key * FG_GREC + value
__device__ __forceinline__ void merge_grid(float (*park)[FG_PARK], int key, float* base) {
  const int lane = (int)(threadIdx.x & 63u);
  park[lane][48] = __int_as_float(key);
  wave_lds_sync();
  uint64_t pending = __ballot(key >= 0);
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const int kl = __builtin_amdgcn_readlane(key, leader);
    const uint64_t m = __ballot(key == kl);
    pending &= ~m;
    if (lane < FG_GREC) {
      float sum = 0.f;
      for (uint64_t mm = m; mm; mm &= mm - 1ull) sum += park[__ffsll((unsigned long long)mm) - 1][lane];
      if (sum != 0.f) atomicAdd(base + (size_t)kl * FG_GREC + lane, sum);
    }
  }
  wave_lds_sync();
}

// the same for the three planes' records at once (plane q's FG_PREC values
// parked at 16 q, its key k[q]): lanes 16 q .. 16 q + 15 take plane q's
// distinct cells, so a pass adds up to one cell of each plane
__device__ __forceinline__ void merge_planes(float (*park)[FG_PARK], const int k[3], float* base) {
  const int lane = (int)(threadIdx.x & 63u), grp = lane >> 4, comp = lane & 15;
  uint64_t pend0 = __ballot(k[0] >= 0), pend1 = __ballot(k[1] >= 0), pend2 = __ballot(k[2] >= 0);
  wave_lds_sync();
  while (pend0 | pend1 | pend2) {
    int k0 = -1, k1 = -1, k2 = -1;
    uint64_t m0 = 0ull, m1 = 0ull, m2 = 0ull;
    if (pend0) {
      k0 = __builtin_amdgcn_readlane(k[0], __ffsll((unsigned long long)pend0) - 1);
      m0 = __ballot(k[0] == k0);
      pend0 &= ~m0;
    }
    if (pend1) {
      k1 = __builtin_amdgcn_readlane(k[1], __ffsll((unsigned long long)pend1) - 1);
      m1 = __ballot(k[1] == k1);
      pend1 &= ~m1;
    }
    if (pend2) {
      k2 = __builtin_amdgcn_readlane(k[2], __ffsll((unsigned long long)pend2) - 1);
      m2 = __ballot(k[2] == k2);
      pend2 &= ~m2;
    }
    const int kg = grp == 0 ? k0 : (grp == 1 ? k1 : (grp == 2 ? k2 : -1));
    if (kg >= 0) {
      float sum = 0.f;
      for (uint64_t mm = grp == 0 ? m0 : (grp == 1 ? m1 : m2); mm; mm &= mm - 1ull)
        sum += park[__ffsll((unsigned long long)mm) - 1][16 * grp + comp];
      if (sum != 0.f) atomicAdd(base + (size_t)kg * FG_PREC + comp, sum);
    }
  }
  wave_lds_sync();
}

__global__ void __launch_bounds__(FG_T) k_field_grad(FieldDev F, Gen q, int g, const Counters* ctr,
                                                     const float4* fseg, float* copies, int n_copies) {
  __shared__ float park[FG_T / 64][64][FG_PARK];
  const int64_t n = ctr->count[g];
  const int lane = (int)(threadIdx.x & 63u), wv = (int)(threadIdx.x >> 6);
  const int cx = F.nx - 1, cy = F.ny - 1, pc = F.res - 1;
  float* gdst = copies + (size_t)(blockIdx.x % (unsigned)n_copies) * field_rec_floats(F);
  float* pdst = gdst + (size_t)FG_GREC * cx * cy * (F.nz - 1);
  const int S = F.samples;
  for (int64_t base = (int64_t)blockIdx.x * FG_T; base < n; base += (int64_t)gridDim.x * FG_T) {
    const int64_t i = base + threadIdx.x;
    bool act = false, open = false;
    v3 o = mk3(0.f, 0.f, 0.f), d = o, Lt = o, Lb = o;
    float tend = 0.f;
    if (i < n) {
      const float4 b = fseg[2 * i + 1];
      if (b.w != 0.f) {
        const float4 a = fseg[2 * i];
        act = true;
        open = b.w > 1.5f;
        Lt = xyz(a);
        tend = a.w;
        Lb = xyz(b);
        o = xyz(q.o[i]);
        d = xyz(q.d[i]);
      }
    }
    FieldClip cl;
    cl.s0 = cl.s1 = 0.f;
    if (act && !field_clip(F, o, d, tend, open, cl)) act = false;
    const float h = act ? (cl.s1 - cl.s0) / (float)S : 0.f;
    v3 P = mk3(0.f, 0.f, 0.f);
    float Tk = 1.f;
    for (int k = 0; k < S; ++k) {
      float fb[4] = {0.f, 0.f, 0.f, 0.f};
      v3 xk = mk3(0.f, 0.f, 0.f);
      if (act) {
        xk = o + d * (cl.s0 + h * ((float)k + 0.5f));
        float f[4];
        field_feature(F, xk, f);
        const float sig = softplusf(f[0]);
        const float a = expf(-sig * h);
        const v3 c = mk3(f[1], f[2], f[3]);
        const float w = Tk * (1.f - a);
        P = P + c * w;
        const float Tn = Tk * a;
        const v3 after = Lt - P;
        const float gg = dot(Lb, c * Tn - after);
        fb[0] = h * gg / (1.f + expf(-f[0]));
        fb[1] = w * Lb.x;
        fb[2] = w * Lb.y;
        fb[3] = w * Lb.z;
        Tk = Tn;
      }
      const float xs[3] = {xk.x, xk.y, xk.z};
      FieldAxis ga[3], pa[3];
      const int nn[3] = {F.nx, F.ny, F.nz};
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        ga[ax] = field_axis(xs[ax], F.lo[ax], F.sg[ax], nn[ax]);
        pa[ax] = field_axis(xs[ax], F.lo[ax], F.sp[ax], F.res);
      }
      // the grid cell's record: corner c = (dx, dy, dz) bits 0-2, channel ch
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const float wx = (c & 1) ? ga[0].f : 1.f - ga[0].f, wy = ((c >> 1) & 1) ? ga[1].f : 1.f - ga[1].f;
        const float wz = (c >> 2) ? ga[2].f : 1.f - ga[2].f;
        const float wc = wx * wy * wz;
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) park[wv][lane][4 * c + ch] = wc * fb[ch];
      }
      merge_grid(park[wv], act ? (ga[2].i * cy + ga[1].i) * cx + ga[0].i : -1, gdst);
      // each plane's cell: (x, y), (x, z), (y, z); corner (di, dj), channel ch
      int kp[3];
#pragma unroll
      for (int qp = 0; qp < 3; ++qp) {
        const int a = qp == 2 ? 1 : 0, b = qp == 0 ? 1 : 2;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float wa = (c & 1) ? pa[a].f : 1.f - pa[a].f, wb = (c >> 1) ? pa[b].f : 1.f - pa[b].f;
#pragma unroll
          for (int ch = 0; ch < 4; ++ch) park[wv][lane][16 * qp + 4 * c + ch] = wa * wb * fb[ch];
        }
        kp[qp] = act ? (qp * pc + pa[b].i) * pc + pa[a].i : -1;
      }
      merge_planes(park[wv], kp, pdst);
    }
  }
}

// d_grid and d_planes from the cell records: a node is corner (dx, dy, dz) of
// the grid cell (x - dx, y - dy, z - dz), or corner (di, dj) of the plane
// cell (i - di, j - dj), where that cell exists; summed over corners, then
// copies, in a fixed order
__global__ void k_field_gather(FieldDev F, const float* copies, int n_copies) {
  const int nx = F.nx, ny = F.ny, nz = F.nz, res = F.res;
  const int cx = nx - 1, cy = ny - 1, cz = nz - 1, pc = res - 1;
  const size_t copy = field_rec_floats(F);
  const size_t gfl = (size_t)FG_GREC * cx * cy * cz;
  const int64_t ng = 4 * (int64_t)nx * ny * nz, np = 12 * (int64_t)res * res;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ng + np;
       j += (int64_t)gridDim.x * blockDim.x) {
    float acc = 0.f;
    if (j < ng) {
      const int ch = (int)(j & 3);
      const int64_t node = j >> 2;
      const int x = (int)(node % nx), y = (int)((node / nx) % ny), z = (int)(node / ((int64_t)nx * ny));
      for (int r = 0; r < n_copies; ++r) {
        const float* cp = copies + (size_t)r * copy;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int ux = x - (c & 1), uy = y - ((c >> 1) & 1), uz = z - (c >> 2);
          if (ux >= 0 && ux < cx && uy >= 0 && uy < cy && uz >= 0 && uz < cz)
            acc += cp[((size_t)(uz * cy + uy) * cx + ux) * FG_GREC + 4 * c + ch];
        }
      }
      F.d_grid[j] = acc;
    } else {
      const int64_t jp = j - ng;
      const int ch = (int)(jp & 3);
      const int64_t node = jp >> 2;
      const int qp = (int)(node / ((int64_t)res * res)), jj = (int)((node / res) % res), ii = (int)(node % res);
      for (int r = 0; r < n_copies; ++r) {
        const float* cp = copies + (size_t)r * copy + gfl;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int ui = ii - (c & 1), uj = jj - (c >> 1);
          if (ui >= 0 && ui < pc && uj >= 0 && uj < pc)
            acc += cp[((size_t)(qp * pc + uj) * pc + ui) * FG_PREC + 4 * c + ch];
        }
      }
      F.d_planes[jp] = acc;
    }
  }
}

// ------------------------------------------------------------------ per-face gathering
// nodes of the generation sorted by face: node i goes to off[face] + rank
__global__ void k_face_scatter(const Counters* ctr, int g, const int2* fkey, const uint32_t* off,
                               uint32_t* fidx) {
  const int64_t n = ctr->count[g];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int2 k = fkey[i];
    if (k.x >= 0) fidx[off[k.x] + (uint32_t)k.y] = (uint32_t)i;
  }
}

// Each face's records of the generation summed by a group of FG lanes and
// added to the face's running totals fg (18 floats per face: for corner k,
// the position adjoint then the vertex-normal adjoint); the group owns the
// face, so no atomics.  The face's count is reset for the next generation.
constexpr int FG = 16;
constexpr int FR_T = 256;

__global__ void __launch_bounds__(FR_T) k_face_reduce(int32_t nf, const FaceRec* frec,
                                                      const uint32_t* fidx, const uint32_t* off,
                                                      uint32_t* fcnt, float* fg) {
  const int sub = threadIdx.x % FG;
  const int64_t groups = (int64_t)gridDim.x * (FR_T / FG);
  for (int64_t f = blockIdx.x * (int64_t)(FR_T / FG) + threadIdx.x / FG; f < nf; f += groups) {
    const uint32_t b = off[f], e = off[f + 1];
    if (b == e) continue;  // the whole group agrees
    v3 p0 = mk3(0.f, 0.f, 0.f), p1 = p0, p2 = p0, n0 = p0, n1 = p0, n2 = p0;
    for (uint32_t j = b + (uint32_t)sub; j < e; j += FG) {
      const FaceRec r = frec[fidx[j]];
      p0 += xyz(r.a);
      p1 += xyz(r.b);
      p2 += xyz(r.c);
      const v3 m = xyz(r.m);
      const float b1 = r.a.w, b2 = r.b.w;
      const float b0 = 1.f - b1 - b2;
      n0 += m * b0;
      n1 += m * b1;
      n2 += m * b2;
    }
    // sum over the group's lanes
#pragma unroll
    for (int st = FG / 2; st > 0; st >>= 1) {
      p0 += mk3(__shfl_xor(p0.x, st), __shfl_xor(p0.y, st), __shfl_xor(p0.z, st));
      p1 += mk3(__shfl_xor(p1.x, st), __shfl_xor(p1.y, st), __shfl_xor(p1.z, st));
      p2 += mk3(__shfl_xor(p2.x, st), __shfl_xor(p2.y, st), __shfl_xor(p2.z, st));
      n0 += mk3(__shfl_xor(n0.x, st), __shfl_xor(n0.y, st), __shfl_xor(n0.z, st));
      n1 += mk3(__shfl_xor(n1.x, st), __shfl_xor(n1.y, st), __shfl_xor(n1.z, st));
      n2 += mk3(__shfl_xor(n2.x, st), __shfl_xor(n2.y, st), __shfl_xor(n2.z, st));
    }
    if (sub < 3) {
      const v3 pv = sub == 0 ? p0 : (sub == 1 ? p1 : p2);
      const v3 nv = sub == 0 ? n0 : (sub == 1 ? n1 : n2);
      float* q = fg + (size_t)(3 * f + sub) * 6;
      q[0] += pv.x;
      q[1] += pv.y;
      q[2] += pv.z;
      q[3] += nv.x;
      q[4] += nv.y;
      q[5] += nv.z;
    } else if (sub == 3) {
      fcnt[f] = 0u;
    }
  }
}

// after the last generation: each vertex sums the totals of the face corners
// it occupies, over its incident-face list (ascending face order, a face
// listed once per corner it holds), so no atomics and a fixed summation order
__global__ void k_vertex_gather(BvhView bv, const int32_t* F, const float* fg, float* dV, float* dN) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= bv.nv) return;
  v3 p = mk3(0.f, 0.f, 0.f), nn = p;
  int prev = -1;
  for (int k = bv.csr_off[v]; k < bv.csr_off[v + 1]; ++k) {
    const int f = bv.csr_idx[k];
    if (f == prev) continue;  // every corner of this face holding v was taken below
    prev = f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (F[3 * f + c] != v) continue;
      const float* q = fg + 6 * (3 * (int64_t)f + c);
      p += mk3(q[0], q[1], q[2]);
      nn += mk3(q[3], q[4], q[5]);
    }
  }
  dV[3 * v] += p.x;
  dV[3 * v + 1] += p.y;
  dV[3 * v + 2] += p.z;
  if (dN) {
    dN[3 * v] += nn.x;
    dN[3 * v + 1] += nn.y;
    dN[3 * v + 2] += nn.z;
  }
}

// dIoR, dsigma = ordered sums of the per-(generation, block) partials
constexpr int RED_T = 1024;  // threads of the scalar reduction (one block)

__global__ void __launch_bounds__(RED_T) k_reduce_scalars(const float4* red, int n, float* d_eta,
                                                          float* d_sigma) {
  __shared__ double sh[4][RED_T];
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    float4 v = red[i];
    a[0] += v.x;
    a[1] += v.y;
    a[2] += v.z;
    a[3] += v.w;
  }
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int st = RED_T / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *d_eta = (float)sh[0][0];
    d_sigma[0] = (float)sh[1][0];
    d_sigma[1] = (float)sh[2][0];
    d_sigma[2] = (float)sh[3][0];
  }
}

// miss list of generation g from the recorded decisions (MLP environment,
// forward and adjoint).  A block of LB threads ranks its misses in LDS and
// reserves their slots with one atomic, so the list counter sees one atomic
// per LB rays instead of one per wave.  The order of the list is irrelevant:
// every listed ray is evaluated independently.
constexpr int LB = 1024;

__global__ void __launch_bounds__(LB) k_list_misses(Gen q, int g, Counters* ctr, uint32_t* list) {
  __shared__ uint32_t wcount[LB / 64];
  __shared__ uint32_t bbase;
  const uint32_t n = ctr->count[g];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t base = (int64_t)blockIdx.x * LB; base < n; base += (int64_t)gridDim.x * LB) {
    int64_t i = base + threadIdx.x;
    bool miss = i < n && !(q.code[i] & C_HIT);
    uint64_t bm = __ballot(miss);
    if (lane == 0) wcount[wave] = (uint32_t)__popcll(bm);
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t tot = 0;
      for (int w = 0; w < LB / 64; ++w) {
        uint32_t c = wcount[w];
        wcount[w] = tot;
        tot += c;
      }
      bbase = tot ? atomicAdd(&ctr->nmiss[g], tot) : 0u;
    }
    __syncthreads();
    if (miss) list[bbase + wcount[wave] + (uint32_t)__popcll(bm & ((1ull << lane) - 1ull))] = (uint32_t)i;
    __syncthreads();
  }
}

// ------------------------------------------------------------------ normals backward (Eq. 13)
// N_v = s_v / 3, s_v = sum of unit face normals u_f, u_f = normalize(c_f),
// c_f = (p1 - p0) x (p2 - p0).
__global__ void k_nbwd_vertex(const BvhView bv, const float* dN, float4* sbar) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= bv.nv) return;
  v3 r = load3(dN + 3 * v) * (1.0f / 3.0f);
  sbar[v] = make_float4(r.x, r.y, r.z, 0.f);
}

__global__ void k_nbwd_face(const BvhView bv, const float* V, const int32_t* F, const float4* sbar,
                            float* dV) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= bv.nf) return;
  float4 u4 = bv.fn[f];
  if (u4.w == 0.f) return;
  int i0 = F[3 * f], i1 = F[3 * f + 1], i2 = F[3 * f + 2];
  v3 ub = xyz(sbar[i0]) + xyz(sbar[i1]) + xyz(sbar[i2]);
  v3 p0 = load3(V + 3 * i0), p1 = load3(V + 3 * i1), p2 = load3(V + 3 * i2);
  v3 e1 = p1 - p0, e2 = p2 - p0;
  v3 c = cross(e1, e2);
  v3 u = xyz(u4);
  v3 cb = (ub - u * dot(u, ub)) * (1.0f / len3(c));
  v3 e1b = cross(e2, cb), e2b = cross(cb, e1);
  atomic_add3(dV, i1, e1b);
  atomic_add3(dV, i2, e2b);
  atomic_add3(dV, i0, -(e1b + e2b));
}

// ------------------------------------------------------------------ env / intersect kernels
__global__ void k_env_query(EnvDev e, const float* dirs, int64_t n, float* rgb) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  v3 E = env_equirect(e, load3(dirs + 3 * i));
  rgb[3 * i] = E.x;
  rgb[3 * i + 1] = E.y;
  rgb[3 * i + 2] = E.z;
}

__global__ void k_env_query_bwd(EnvDev e, const float* dirs, int64_t n, const float* g, float* gd) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  v3 dd;
  env_equirect_grad(e, load3(dirs + 3 * i), load3(g + 3 * i), &dd);
  gd[3 * i] = dd.x;
  gd[3 * i + 1] = dd.y;
  gd[3 * i + 2] = dd.z;
}

__global__ void __launch_bounds__(TB) k_intersect(BvhView bv, const float* o, const float* d,
                                                  const int32_t* skip, int64_t n, float t_eps,
                                                  int brute, int32_t* tri, float* t, float* b) {
  __shared__ uint2 stk[DT_STACK * TB];
  __shared__ LeafQueue lq;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (brute) {
    if (i >= n) return;
  }
  const bool active = i < n;
  v3 oo = mk3(0.f, 0.f, 0.f), dd = mk3(0.f, 0.f, 1.f);
  int sk = -1;
  if (active) {
    oo = load3(o + 3 * i);
    dd = load3(d + 3 * i);
    sk = skip ? skip[i] : -1;
  }
  bool ovf = false;
  // the wave traversal needs every lane of the block's wave
  Hit h = brute ? closest_brute(bv, oo, dd, sk, t_eps)
                : closest_hit_wave<DT_STACK, false, false>(bv, active, oo, dd, sk, t_eps,
                                                           stk + threadIdx.x, TB, nullptr, 0, lq, &ovf);
  if (!active) return;
  tri[i] = ovf ? -2 : h.tri;
  t[i] = h.t;
  b[2 * i] = h.b1;
  b[2 * i + 1] = h.b2;
}

// ------------------------------------------------------------------ host helpers
dt_status make_scene(const dt_scene* sc, const dt_trace_params* p, SceneDev& s) {
  DT_REQUIRE(sc && p, "scene or params is NULL");
  DT_REQUIRE(sc->V && sc->F && sc->bvh && sc->ior && sc->sigma && sc->env,
             "scene has a NULL pointer (V, F, bvh, ior, sigma, env)");
  DT_REQUIRE(sc->nv >= 3 && sc->nf >= 1 && sc->nf <= DT_MAX_FACES && sc->nv < (1 << 30),
             "scene needs nv >= 3 and 1 <= nf <= 2^26 (got %d, %d)", sc->nv, sc->nf);
  DT_REQUIRE(p->max_depth >= 0 && p->max_depth <= DT_MAX_DEPTH, "max_depth must be in [0, %d]",
             DT_MAX_DEPTH);
  DT_REQUIRE(p->t_eps >= 0.f && p->t_eps < 1.f, "t_eps must be in [0, 1)");
  DT_REQUIRE(p->checkpoint_stride >= 1, "checkpoint_stride must be >= 1");
  DT_REQUIRE(p->queue_capacity >= 0, "queue_capacity must be >= 0");
  s.V = sc->V;
  s.F = sc->F;
  s.nv = sc->nv;
  s.nf = sc->nf;
  s.bvh = bvh_view(sc->bvh, sc->nv, sc->nf);
  s.ior = sc->ior;
  s.sigma = sc->sigma;
  memset(&s.ab, 0, sizeof(s.ab));
  if (const dt_absorption* G = sc->absorb) {
    DT_REQUIRE(G->mu, "absorption grid has a NULL mu");
    DT_REQUIRE(G->nx >= 2 && G->ny >= 2 && G->nz >= 2 && G->nx <= 1024 && G->ny <= 1024 &&
                   G->nz <= 1024,
               "absorption grid needs 2..1024 nodes per axis (got %d, %d, %d)", G->nx, G->ny, G->nz);
    DT_REQUIRE(G->samples >= 1 && G->samples <= 256, "absorption samples must be in [1, 256]");
    s.ab.mu = G->mu;
    s.ab.d_mu = G->d_mu;
    s.ab.nx = G->nx;
    s.ab.ny = G->ny;
    s.ab.nz = G->nz;
    s.ab.samples = G->samples;
    const int n[3] = {G->nx, G->ny, G->nz};
    for (int a = 0; a < 3; ++a) {
      DT_REQUIRE(G->hi[a] > G->lo[a], "absorption grid box needs hi > lo on every axis");
      s.ab.lo[a] = G->lo[a];
      s.ab.scale[a] = (float)(n[a] - 1) / (G->hi[a] - G->lo[a]);
    }
  }
  memset(&s.fd, 0, sizeof(s.fd));
  if (const dt_field* G = sc->field) {
    DT_REQUIRE(G->grid && G->planes, "field has a NULL grid or planes");
    DT_REQUIRE(G->nx >= 2 && G->ny >= 2 && G->nz >= 2 && G->res >= 2 && G->nx <= 1024 &&
                   G->ny <= 1024 && G->nz <= 1024 && G->res <= 1024,
               "field needs 2..1024 nodes per axis (got %d, %d, %d, res %d)", G->nx, G->ny, G->nz,
               G->res);
    DT_REQUIRE(G->samples >= 1 && G->samples <= 256, "field samples must be in [1, 256]");
    DT_REQUIRE((G->d_grid == nullptr) == (G->d_planes == nullptr),
               "field gradients need both d_grid and d_planes, or neither");
    s.fd.grid = G->grid;
    s.fd.planes = G->planes;
    s.fd.d_grid = G->d_grid;
    s.fd.d_planes = G->d_planes;
    s.fd.nx = G->nx;
    s.fd.ny = G->ny;
    s.fd.nz = G->nz;
    s.fd.res = G->res;
    s.fd.samples = G->samples;
    const int n[3] = {G->nx, G->ny, G->nz};
    for (int a = 0; a < 3; ++a) {
      DT_REQUIRE(G->hi[a] > G->lo[a], "field box needs hi > lo on every axis");
      s.fd.lo[a] = G->lo[a];
      s.fd.hi[a] = G->hi[a];
      s.fd.sg[a] = (float)(n[a] - 1) / (G->hi[a] - G->lo[a]);
      s.fd.sp[a] = (float)(G->res - 1) / (G->hi[a] - G->lo[a]);
    }
  }
  if (dt_status st = make_env(sc->env, s.env)) return st;
  if (s.fd.grid && s.env.kind == DT_ENV_MLP) {
    dt_set_error("a volumetric field with an MLP environment is not supported");
    return DT_ERR_UNSUPPORTED;
  }
  if (s.env.kind == DT_ENV_MLP && p->terminal_env) {
    dt_set_error("terminal_env with an MLP environment is not supported");
    return DT_ERR_UNSUPPORTED;
  }
  s.max_depth = p->max_depth;
  s.terminal_env = p->terminal_env ? 1 : 0;
  s.t_eps = p->t_eps;
  return DT_OK;
}

dt_status ray_counts(const dt_rays* r, int64_t& n_rays, int64_t& npix) {
  DT_REQUIRE(r, "rays is NULL");
  if (r->kind == DT_RAYS_EXPLICIT) {
    DT_REQUIRE(r->n >= 1 && r->n < (1ll << 31), "explicit rays need 1 <= n < 2^31");
    DT_REQUIRE(r->o && r->d, "explicit rays need o and d");
    n_rays = npix = r->n;
    return DT_OK;
  }
  DT_REQUIRE(r->kind == DT_RAYS_CAMERAS, "unknown ray kind %d", r->kind);
  DT_REQUIRE(r->n_cameras >= 1 && r->cameras, "camera rays need n_cameras >= 1 and cameras");
  DT_REQUIRE(r->n_pixels >= 1 && r->n_pixels < (1ll << 31), "n_pixels must be in [1, 2^31)");
  int64_t tot = 0;
  for (int c = 0; c < r->n_cameras; ++c) {
    const dt_camera& cam = r->cameras[c];
    DT_REQUIRE(cam.width >= 1 && cam.height >= 1, "camera %d has an empty image", c);
    DT_REQUIRE(cam.fov_deg > 0.f && cam.fov_deg < 180.f, "camera %d fov must be in (0, 180)", c);
    int64_t np = (int64_t)cam.width * cam.height;
    DT_REQUIRE(cam.pixel_offset >= 0 && cam.pixel_offset + np <= r->n_pixels,
               "camera %d pixels [%lld, %lld) exceed n_pixels %lld", c, (long long)cam.pixel_offset,
               (long long)(cam.pixel_offset + np), (long long)r->n_pixels);
    tot += np;
  }
  DT_REQUIRE(tot < (1ll << 31), "too many camera rays");
  n_rays = tot;
  npix = r->n_pixels;
  return DT_OK;
}

Gen gen_at(char* base, size_t o, size_t d, size_t w, size_t hit, size_t code, size_t child) {
  Gen g;
  g.o = o == (size_t)-1 ? nullptr : (float4*)(base + o);
  g.d = d == (size_t)-1 ? nullptr : (float4*)(base + d);
  g.w = w == (size_t)-1 ? nullptr : (float4*)(base + w);
  g.hit = hit == (size_t)-1 ? nullptr : (float4*)(base + hit);
  g.code = code == (size_t)-1 ? nullptr : (uint32_t*)(base + code);
  g.child = child == (size_t)-1 ? nullptr : (int2*)(base + child);
  return g;
}

unsigned list_grid(int64_t cap) {
  int64_t b = (cap + LB - 1) / LB;
  return (unsigned)(b < 1 ? 1 : (b > 2048 ? 2048 : b));
}

unsigned trace_grid(int64_t cap) {
  int64_t waves = (cap + 63) / 64;
  int64_t lim = TRACE_MAX_BLOCKS;  // resident waves the LDS stack allows on 256 CUs
  return (unsigned)(waves < lim ? (waves < 1 ? 1 : waves) : lim);
}

dt_status emit_rays(const dt_rays* r, Gen g0, hipStream_t s) {
  if (r->kind == DT_RAYS_EXPLICIT) {
    hipLaunchKernelGGL(k_rays_explicit, dim3(dt_blocks(r->n, 256)), dim3(256), 0, s, g0, r->o, r->d,
                       r->n);
    DT_CHECK_LAUNCH();
    return DT_OK;
  }
  int64_t base = 0;
  for (int c0 = 0; c0 < r->n_cameras; c0 += CAM_BATCH) {
    CamBatch cb;
    cb.n = r->n_cameras - c0 < CAM_BATCH ? r->n_cameras - c0 : CAM_BATCH;
    const int64_t b0 = base;
    for (int k = 0; k < cb.n; ++k) {
      const dt_camera& cam = r->cameras[c0 + k];
      if (dt_status st = make_camera(cam, c0 + k, cb.cam[k])) return st;
      cb.cam[k].base = base;
      base += (int64_t)cam.width * cam.height;
    }
    for (int k = cb.n; k < CAM_BATCH; ++k) cb.cam[k] = cb.cam[0];
    hipLaunchKernelGGL(k_raygen, dim3(dt_blocks(base - b0, 256)), dim3(256), 0, s, g0, cb, base - b0);
    DT_CHECK_LAUNCH();
  }
  return DT_OK;
}

// run generation g of the wavefront: trace, and (g < D) scan + emit
dt_status record(void* const* ev, int i, hipStream_t s) {
  if (ev && ev[i]) DT_CHECK_HIP(hipEventRecord((hipEvent_t)ev[i], s));
  return DT_OK;
}

dt_status run_generation(const SceneDev& sc, const Plan& P, int g, Gen cur, Gen nxt, Counters* ctr,
                         WorkPart* wp, unsigned long long* part_g, unsigned long long* part_other, float* rgb,
                         float* wtrunc, int32_t* flags, unsigned long long* sig, int accumulate,
                         int write_next, void* const* events, void* const* mlp_events,
                         uint32_t* miss_list, uint2* ovf, float4* att, hipStream_t s) {
  if (!sc.ab.mu && !sc.fd.grid) att = nullptr;  // the constant rate: recomputing it is cheaper
  if (dt_status st = record(events, 2 * g, s)) return st;
#define DT_TRACE(G, FL)                                                                              \
  hipLaunchKernelGGL((k_trace<G, FL>), dim3(trace_grid(P.cap[g])), dim3(TB), 0, s, sc, cur, g, ctr, part_g, \
                     rgb, wtrunc, flags, sig, accumulate, ovf, wp, att)
  if (sc.fd.grid) {
    if (sc.ab.mu) DT_TRACE(true, true); else DT_TRACE(false, true);
  } else {
    if (sc.ab.mu) DT_TRACE(true, false); else DT_TRACE(false, false);
  }
#undef DT_TRACE
  DT_CHECK_LAUNCH();
  if (dt_status st = record(events, 2 * g + 1, s)) return st;
  if (accumulate && sc.env.kind == DT_ENV_MLP) {
    hipLaunchKernelGGL(k_list_misses, dim3(list_grid(P.cap[g])), dim3(LB), 0, s, cur, g, ctr, miss_list);
    DT_CHECK_LAUNCH();
    if (dt_status st = record(mlp_events, 2 * g, s)) return st;
    if (dt_status st = mlp_trace_forward(sc.env, cur, miss_list, ctr, g, P.cap[g], rgb, s)) return st;
    if (dt_status st = record(mlp_events, 2 * g + 1, s)) return st;
  }
  if (g < P.D) {
    int64_t other_n = (P.cap[g + 1] + CHUNK - 1) / CHUNK + 1;
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, ctr, g, part_g, part_other, other_n,
                       P.cap[g + 1]);
    int64_t nch = (P.cap[g] + CHUNK - 1) / CHUNK;
#define DT_EMIT(G, FL)                                                                                 \
  hipLaunchKernelGGL((k_emit<G, FL>), dim3((unsigned)nch), dim3(EB), 0, s, sc, cur, nxt, g, ctr, part_g, \
                     P.cap[g + 1], write_next, accumulate ? flags : nullptr, att)
    if (sc.fd.grid) {
      if (sc.ab.mu) DT_EMIT(true, true); else DT_EMIT(false, true);
    } else {
      if (sc.ab.mu) DT_EMIT(true, false); else DT_EMIT(false, false);
    }
#undef DT_EMIT
    DT_CHECK_LAUNCH();
  }
  return DT_OK;
}

dt_status zero_f32(float* p, int64_t n, hipStream_t s) {
  if (!p || n <= 0) return DT_OK;
  unsigned nb = dt_blocks(n, 256);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_zero_f32, dim3(nb), dim3(256), 0, s, p, n);
  DT_CHECK_LAUNCH();
  return DT_OK;
}

dt_status zero_u64(unsigned long long* p, int64_t n, hipStream_t s) {
  if (!p || n <= 0) return DT_OK;
  unsigned nb = dt_blocks(n, 256);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_zero_u64, dim3(nb), dim3(256), 0, s, p, n);
  DT_CHECK_LAUNCH();
  return DT_OK;
}

}  // namespace

// ------------------------------------------------------------------ shared host helpers
dt_status make_env(const dt_env* env, EnvDev& e) {
  DT_REQUIRE(env, "environment descriptor is NULL");
  DT_REQUIRE(env->kind == DT_ENV_EQUIRECT || env->kind == DT_ENV_MLP, "unknown environment kind %d",
             env->kind);
  if (env->kind == DT_ENV_EQUIRECT)
    DT_REQUIRE(env->texels && env->width >= 1 && env->height >= 1 &&
                   (int64_t)env->width * env->height <= ((int64_t)1 << 29),
               "equirect environment needs texels and width, height >= 1 (at most 2^29 texels)");
  e.kind = env->kind;
  e.W = env->width;
  e.H = env->height;
  e.tex = env->texels;
  e.d_tex = env->kind == DT_ENV_EQUIRECT ? env->d_texels : nullptr;
  e.n_freq = env->n_freq;
  e.n_layers = env->n_layers;
  e.hidden = env->hidden;
  e.in_pad = env->in_pad;
  e.w = env->weights;
  e.b = env->biases;
  e.d_w = env->kind == DT_ENV_MLP ? env->d_weights : nullptr;
  e.d_b = env->kind == DT_ENV_MLP ? env->d_biases : nullptr;
  if (env->kind == DT_ENV_MLP && !mlp_supported(e)) {
    dt_set_error("environment MLP needs weights, biases, in_pad 64, hidden 64 or 128, 1-4 layers, "
                 "n_freq <= 7 (got in_pad %d hidden %d layers %d n_freq %d)",
                 env->in_pad, env->hidden, env->n_layers, env->n_freq);
    return DT_ERR_UNSUPPORTED;
  }
  DT_REQUIRE(!e.d_w == !e.d_b, "environment MLP: give both d_weights and d_biases, or neither");
  if (e.d_w && mlp_wgrad_params(e) == 0) {
    dt_set_error("environment MLP weight gradient: hidden width 64 only (got %d)", env->hidden);
    return DT_ERR_UNSUPPORTED;
  }
  return DT_OK;
}


dt_status make_camera(const dt_camera& cam, int c, CamDev& cd) {
  double e[3] = {cam.eye[0], cam.eye[1], cam.eye[2]};
  double f[3] = {cam.target[0] - e[0], cam.target[1] - e[1], cam.target[2] - e[2]};
  double fl = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  DT_REQUIRE(fl > 0.0, "camera %d: eye equals target", c);
  for (int k = 0; k < 3; ++k) f[k] /= fl;
  double up[3] = {cam.up[0], cam.up[1], cam.up[2]};
  double rt[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
  double rl = sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
  DT_REQUIRE(rl > 0.0, "camera %d: up is parallel to the view direction", c);
  for (int k = 0; k < 3; ++k) rt[k] /= rl;
  double u[3] = {rt[1] * f[2] - rt[2] * f[1], rt[2] * f[0] - rt[0] * f[2], rt[0] * f[1] - rt[1] * f[0]};
  for (int k = 0; k < 3; ++k) {
    cd.eye[k] = (float)e[k];
    cd.f[k] = (float)f[k];
    cd.r[k] = (float)rt[k];
    cd.u[k] = (float)u[k];
  }
  cd.th = (float)tan(0.5 * (double)cam.fov_deg * 3.14159265358979323846 / 180.0);
  cd.aspect = (float)((double)cam.width / (double)cam.height);
  cd.W = cam.width;
  cd.H = cam.height;
  cd.pixel_offset = cam.pixel_offset;
  cd.base = 0;
  cd.tiled = (cam.width % 8 == 0 && cam.height % 8 == 0) ? 1 : 0;
  return DT_OK;
}

dt_status chunk_scan(Counters* ctr, int g, unsigned long long* part, unsigned long long* other,
                     int64_t other_n, int64_t cap_next, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, ctr, g, part, other, other_n, cap_next);
  DT_CHECK_LAUNCH();
  return DT_OK;
}

// ------------------------------------------------------------------ C ABI
extern "C" dt_status dt_trace_bytes(const dt_trace_params* p, int64_t n_rays, int32_t nv, int32_t nf,
                                    size_t* ws_bytes, size_t* tape_bytes) {
  DT_REQUIRE(p && ws_bytes && tape_bytes, "dt_trace_bytes: NULL argument");
  DT_REQUIRE(n_rays >= 1 && n_rays < (1ll << 31), "dt_trace_bytes: n_rays must be in [1, 2^31)");
  DT_REQUIRE(nv >= 3 && nf >= 1, "dt_trace_bytes: need nv >= 3 and nf >= 1");
  DT_REQUIRE(p->max_depth >= 0 && p->max_depth <= DT_MAX_DEPTH, "max_depth must be in [0, %d]",
             DT_MAX_DEPTH);
  DT_REQUIRE(p->checkpoint_stride >= 1 && p->queue_capacity >= 0, "bad checkpoint_stride / capacity");
  Plan P;
  make_plan(p, n_rays, n_rays, nv, nf, P);
  *ws_bytes = P.ws_bytes;
  *tape_bytes = P.tape_bytes;
  return DT_OK;
}

extern "C" dt_status dt_trace_forward(const dt_scene* scene, const dt_rays* rays,
                                      const dt_trace_params* p, float* rgb, float* wtrunc,
                                      int32_t* flags, uint64_t* path_sig, int64_t* stats,
                                      void* tape, size_t tape_bytes, void* ws, size_t ws_bytes,
                                      void* stream) {
  SceneDev sc;
  if (dt_status st = make_scene(scene, p, sc)) return st;
  int64_t N, npix;
  if (dt_status st = ray_counts(rays, N, npix)) return st;
  DT_REQUIRE(rgb && ws, "dt_trace_forward: rgb and ws are required");
  Plan P;
  make_plan(p, N, npix, scene->nv, scene->nf, P);
  if (ws_bytes < P.ws_bytes) {
    dt_set_error("dt_trace_forward: workspace has %zu bytes, needs %zu", ws_bytes, P.ws_bytes);
    return DT_ERR_WORKSPACE_TOO_SMALL;
  }
  if (tape && tape_bytes < P.tape_bytes) {
    dt_set_error("dt_trace_forward: tape has %zu bytes, needs %zu", tape_bytes, P.tape_bytes);
    return DT_ERR_WORKSPACE_TOO_SMALL;
  }
  hipStream_t s = (hipStream_t)stream;
  char* W = (char*)ws;
  char* T = (char*)tape;
  Counters* ctr = (Counters*)(W + P.w_ctr);
  unsigned long long* part[2] = {(unsigned long long*)(W + P.w_part0),
                                 (unsigned long long*)(W + P.w_part1)};
  hipLaunchKernelGGL(k_init_counters, dim3(1), dim3(64), 0, s, ctr, (uint32_t)N, (WorkPart*)(W + P.w_parts));
  if (dt_status st = zero_u64(part[0], P.maxchunks + 1, s)) return st;
  if (dt_status st = zero_f32(rgb, 3 * npix, s)) return st;
  if (dt_status st = zero_f32(wtrunc, 3 * npix, s)) return st;
  if (dt_status st = zero_f32((float*)flags, npix, s)) return st;
  if (dt_status st = zero_u64((unsigned long long*)path_sig, npix, s)) return st;

  // where generation g lives during the forward pass: on the tape when it is
  // stored there, otherwise in the ping-pong scratch queues of the workspace
  auto gen_fwd = [&](int g) -> Gen {
    Gen G;
    if (T && (P.store_all || g % P.k == 0)) {
      G = gen_at(T, P.t_o[g], P.t_d[g], P.t_w[g], (size_t)-1, (size_t)-1, (size_t)-1);
    } else {
      G = gen_at(W, P.w_ro[g & 1], P.w_rd[g & 1], P.w_rw[g & 1], (size_t)-1, (size_t)-1, (size_t)-1);
    }
    if (T && P.store_all) {
      G.hit = (float4*)(T + P.t_hit[g]);
      G.code = (uint32_t*)(T + P.t_code[g]);
      G.child = (int2*)(T + P.t_child[g]);
    } else {
      G.hit = (float4*)(W + P.w_hit);
      G.code = (uint32_t*)(W + P.w_code);
      G.child = nullptr;
    }
    return G;
  };
  for (int g = 0; g <= P.D; ++g) {
    Gen cur = gen_fwd(g);
    if (g == 0)
      if (dt_status st = emit_rays(rays, cur, s)) return st;
    Gen nxt = g < P.D ? gen_fwd(g + 1) : cur;
    void* const* ev = p->timing ? p->timing->trace_events : nullptr;
    void* const* mev = p->timing ? p->timing->mlp_events : nullptr;
    if (dt_status st = run_generation(sc, P, g, cur, nxt, ctr, (WorkPart*)(W + P.w_parts), part[g & 1],
                                      part[(g + 1) & 1], rgb,
                                      wtrunc, flags, (unsigned long long*)path_sig, 1, 1, ev, mev,
                                      (uint32_t*)(W + P.w_miss), (uint2*)(W + P.w_ovf),
                                      (float4*)(W + P.w_adj[0][0]), s))
      return st;
  }
  if (T) hipLaunchKernelGGL(k_save_counters, dim3(1), dim3(64), 0, s, (Counters*)(T + P.tape_hdr), ctr);
  if (stats) hipLaunchKernelGGL(k_stats, dim3(1), dim3(64), 0, s, ctr, P.D, sc.bvh.hdr, stats);
  DT_CHECK_LAUNCH();
  return DT_OK;
}

extern "C" dt_status dt_trace_backward(const dt_scene* scene, const dt_rays* rays,
                                       const dt_trace_params* p, const float* grad_rgb,
                                       const void* tape, size_t tape_bytes, float* dV, float* d_ior,
                                       float* d_sigma, void* ws, size_t ws_bytes, void* stream) {
  SceneDev sc;
  if (dt_status st = make_scene(scene, p, sc)) return st;
  int64_t N, npix;
  if (dt_status st = ray_counts(rays, N, npix)) return st;
  DT_REQUIRE(grad_rgb && tape && dV && d_ior && d_sigma && ws,
             "dt_trace_backward: grad_rgb, tape, dV, d_ior, d_sigma and ws are required");
  Plan P;
  make_plan(p, N, npix, scene->nv, scene->nf, P);
  if (ws_bytes < P.ws_bytes || tape_bytes < P.tape_bytes) {
    dt_set_error("dt_trace_backward: workspace %zu/%zu or tape %zu/%zu bytes too small", ws_bytes,
                 P.ws_bytes, tape_bytes, P.tape_bytes);
    return DT_ERR_WORKSPACE_TOO_SMALL;
  }
  hipStream_t s = (hipStream_t)stream;
  char* W = (char*)ws;
  char* T = (char*)tape;
  Counters* ctr = (Counters*)(W + P.w_ctr);
  unsigned long long* part[2] = {(unsigned long long*)(W + P.w_part0),
                                 (unsigned long long*)(W + P.w_part1)};
  float* dN = (float*)(W + P.w_dN);
  float4* sbar = (float4*)(W + P.w_sbar);
  float4* red = (float4*)(W + P.w_red);
  FaceRec* frec = (FaceRec*)(W + P.w_frec);
  int2* fkey = (int2*)(W + P.w_fkey);
  uint32_t* fidx = (uint32_t*)(W + P.w_fidx);
  uint32_t* fcnt = (uint32_t*)(W + P.w_fcnt);
  uint32_t* foff = (uint32_t*)(W + P.w_foff);
  int32_t* fscan = (int32_t*)(W + P.w_fscan);
  float* fg = (float*)(W + P.w_fg);
  const int nred = (P.D + 1) * ADJ_MAX_BLOCKS;  // slot g * ADJ_MAX_BLOCKS + block
  hipLaunchKernelGGL(k_load_counters, dim3(1), dim3(64), 0, s, ctr, (const Counters*)(T + P.tape_hdr));
  if (dt_status st = zero_f32(dV, 3 * (int64_t)scene->nv, s)) return st;
  if (dt_status st = zero_f32(dN, 3 * (int64_t)scene->nv, s)) return st;
  if (dt_status st = zero_f32((float*)fcnt, (int64_t)scene->nf + 1, s)) return st;
  if (dt_status st = zero_f32(fg, 18 * (int64_t)scene->nf, s)) return st;
  // absorption grid: as many copies of the per-cell records as the scratch
  // region holds (at most 64)
  const int64_t gsize = sc.ab.mu ? 3 * (int64_t)sc.ab.nx * sc.ab.ny * sc.ab.nz : 0;
  const int64_t csize =
      sc.ab.mu ? (int64_t)GG_CELL * (sc.ab.nx - 1) * (int64_t)(sc.ab.ny - 1) * (sc.ab.nz - 1) : 0;
  float* gcopies = (float*)(W + P.w_gscr);
  int n_copies = 0;
  bool gcell = true;
  if (sc.ab.mu && sc.ab.d_mu) {
    const int64_t fit = (int64_t)(GG_SCRATCH / sizeof(float)) / csize;
    n_copies = (int)(fit < GG_MAX_COPIES ? fit : GG_MAX_COPIES);
    if (n_copies < 1) {
      // records larger than the scratch region: node sums straight into the caller's array
      n_copies = 1;
      gcopies = sc.ab.d_mu;
      gcell = false;
    }
    if (dt_status st = zero_f32(gcopies, gcell ? csize * n_copies : gsize, s)) return st;
  }
  if (sc.env.d_tex)
    if (dt_status st = zero_f32(sc.env.d_tex, 3 * (int64_t)sc.env.W * sc.env.H, s)) return st;
  float* mlp_part = (float*)(W + P.w_mlpg);
  if (sc.env.d_w)
    if (dt_status st = zero_f32(mlp_part, (int64_t)(mlp_wgrad_scratch_bytes() / sizeof(float)), s))
      return st;
  // volumetric field: as many copies of the per-cell records as the scratch
  // region holds (at most FG_MAX_COPIES); a field whose records do not fit has
  // its gradient added in place by the adjoint instead
  float* fcopies = (float*)(W + P.w_fscr);
  int f_copies = 0;
  float4* fseg = nullptr;
  if (sc.fd.d_grid) {
    const int64_t pc = sc.fd.res - 1;
    const int64_t rec = (int64_t)FG_GREC * (sc.fd.nx - 1) * (sc.fd.ny - 1) * (sc.fd.nz - 1) + 3 * FG_PREC * pc * pc;
    const int64_t fit = (int64_t)(FG_SCRATCH / sizeof(float)) / rec;
    f_copies = (int)(fit < FG_MAX_COPIES ? fit : FG_MAX_COPIES);
    if (f_copies >= 1) {
      fseg = (float4*)(W + P.w_fseg);
      if (dt_status st = zero_f32(fcopies, rec * f_copies, s)) return st;
    } else {
      f_copies = 0;
      if (dt_status st = zero_f32(sc.fd.d_grid, 4 * (int64_t)sc.fd.nx * sc.fd.ny * sc.fd.nz, s)) return st;
      if (dt_status st = zero_f32(sc.fd.d_planes, 12 * (int64_t)sc.fd.res * sc.fd.res, s)) return st;
    }
  }
  if (dt_status st = zero_f32((float*)red, 4 * (int64_t)nred, s)) return st;
  Adj adj[2];
  for (int b = 0; b < 2; ++b) {
    adj[b].L = (float4*)(W + P.w_adj[b][0]);
    adj[b].O = (float4*)(W + P.w_adj[b][1]);
    adj[b].D = (float4*)(W + P.w_adj[b][2]);
  }
  void* const* aev = p->timing ? p->timing->adjoint_events : nullptr;
  void* const* maev = p->timing ? p->timing->mlp_adjoint_events : nullptr;
  auto adjoint = [&](int g, Gen q) -> dt_status {
    int64_t blocks = (P.cap[g] + AB - 1) / AB;
    if (blocks > ADJ_MAX_BLOCKS) blocks = ADJ_MAX_BLOCKS;
    if (dt_status st = record(aev, 2 * g, s)) return st;
    if (sc.env.kind == DT_ENV_MLP) {
      uint32_t* ml = (uint32_t*)(W + P.w_miss);
      hipLaunchKernelGGL(k_list_misses, dim3(list_grid(P.cap[g])), dim3(LB), 0, s, q, g, ctr, ml);
      DT_CHECK_LAUNCH();
      if (dt_status st = record(maev, 2 * g, s)) return st;
      if (sc.env.d_w) {
        if (dt_status st = mlp_trace_backward_wgrad(sc.env, q, ml, ctr, g, grad_rgb, adj[g & 1], mlp_part, s))
          return st;
      } else if (dt_status st = mlp_trace_backward(sc.env, q, ml, ctr, g, P.cap[g], grad_rgb, adj[g & 1], s)) {
        return st;
      }
      if (dt_status st = record(maev, 2 * g + 1, s)) return st;
    }
#define DT_ADJ(G, FL)                                                                                  \
  hipLaunchKernelGGL((k_adjoint<G, FL>), dim3((unsigned)blocks), dim3(AB), 0, s, sc, q, g, ctr, grad_rgb,  \
                     adj[(g + 1) & 1], adj[g & 1], frec, fkey, fcnt, red, fseg)
    if (sc.fd.grid) {
      if (sc.ab.mu) DT_ADJ(true, true); else DT_ADJ(false, true);
    } else {
      if (sc.ab.mu) DT_ADJ(true, false); else DT_ADJ(false, false);
    }
#undef DT_ADJ
    if (sc.env.d_tex) {
      const int64_t eb = (P.cap[g] + GG_T - 1) / GG_T;
      hipLaunchKernelGGL(k_env_tex_grad, dim3((unsigned)(eb < 8192 ? eb : 8192)), dim3(GG_T), 0, s, sc, q, g,
                         ctr, grad_rgb);
    }
    if (fseg) {
      const int64_t fb = (P.cap[g] + FG_T - 1) / FG_T;
      hipLaunchKernelGGL(k_field_grad, dim3((unsigned)(fb < 8192 ? fb : 8192)), dim3(FG_T), 0, s, sc.fd, q, g,
                         ctr, fseg, fcopies, f_copies);
    }
    if (sc.ab.mu && sc.ab.d_mu) {
      const int64_t gb = (P.cap[g] + GG_T - 1) / GG_T;
      if (gcell)
        hipLaunchKernelGGL(k_grid_grad<true>, dim3((unsigned)(gb < 8192 ? gb : 8192)), dim3(GG_T), 0, s, sc.ab,
                           q, g, ctr, adj[g & 1], gcopies, n_copies);
      else
        hipLaunchKernelGGL(k_grid_grad<false>, dim3((unsigned)(gb < 8192 ? gb : 8192)), dim3(GG_T), 0, s,
                           sc.ab, q, g, ctr, adj[g & 1], gcopies, n_copies);
    }
    // fcnt[nf] stays 0, so foff[nf] is the total
    if (dt_status st = dt_scan_exclusive_i32((const int32_t*)fcnt, (int32_t*)foff, scene->nf + 1, fscan, s))
      return st;
    hipLaunchKernelGGL(k_face_scatter, dim3(dt_blocks(P.cap[g], 256) < 8192 ? dt_blocks(P.cap[g], 256) : 8192),
                       dim3(256), 0, s, ctr, g, fkey, foff, fidx);
    const int64_t fgroups = ((int64_t)scene->nf + FR_T / FG - 1) / (FR_T / FG);
    hipLaunchKernelGGL(k_face_reduce, dim3((unsigned)(fgroups < 8192 ? fgroups : 8192)), dim3(FR_T), 0, s,
                       scene->nf, frec, fidx, foff, fcnt, fg);
    DT_CHECK_LAUNCH();
    return record(aev, 2 * g + 1, s);
  };
  if (P.store_all) {
    for (int g = P.D; g >= 0; --g) {
      Gen q = gen_at(T, P.t_o[g], P.t_d[g], P.t_w[g], P.t_hit[g], P.t_code[g], P.t_child[g]);
      if (dt_status st = adjoint(g, q)) return st;
    }
  } else {
    // recompute each segment [g0, g0 + k) from its stored first generation
    int nseg = (P.D + P.k) / P.k;
    size_t mc = (size_t)P.maxcap;
    for (int sg = nseg - 1; sg >= 0; --sg) {
      int g0 = sg * P.k;
      int g1 = g0 + P.k - 1 < P.D ? g0 + P.k - 1 : P.D;
      Gen seg[DT_MAX_DEPTH + 1];
      for (int g = g0; g <= g1; ++g) {
        int j = g - g0;
        seg[j].o = (float4*)(W + P.w_seg_o) + mc * j;
        seg[j].d = (float4*)(W + P.w_seg_d) + mc * j;
        seg[j].w = (float4*)(W + P.w_seg_w) + mc * j;
        seg[j].hit = (float4*)(W + P.w_seg_hit) + mc * j;
        seg[j].code = (uint32_t*)(W + P.w_seg_code) + mc * j;
        seg[j].child = (int2*)(W + P.w_seg_child) + mc * j;
      }
      // generation g0 reads its rays from the tape
      seg[0].o = (float4*)(T + P.t_o[g0]);
      seg[0].d = (float4*)(T + P.t_d[g0]);
      seg[0].w = (float4*)(T + P.t_w[g0]);
      hipLaunchKernelGGL(k_reset_work, dim3(1), dim3(64), 0, s, g0, (WorkPart*)(W + P.w_parts));
      if (dt_status st = zero_u64(part[g0 & 1], P.maxchunks + 1, s)) return st;
      // adj[(g1 + 1) & 1] holds generation g1 + 1's adjoint records, which the
      // segment's first adjoint reads; adj[g1 & 1] is free until it writes
      // it, and carries the attenuation from k_trace to k_emit meanwhile
      for (int g = g0; g <= g1; ++g) {
        int j = g - g0;
        Gen nxt = g < g1 ? seg[j + 1] : seg[j];
        if (dt_status st = run_generation(sc, P, g, seg[j], nxt, ctr, (WorkPart*)(W + P.w_parts),
                                          part[g & 1], part[(g + 1) & 1],
                                          nullptr, nullptr, nullptr, nullptr, 0, g < g1 ? 1 : 0,
                                          nullptr, nullptr,
                                          (uint32_t*)(W + P.w_miss), (uint2*)(W + P.w_ovf), adj[g1 & 1].L, s))
          return st;
      }
      for (int g = g1; g >= g0; --g)
        if (dt_status st = adjoint(g, seg[g - g0])) return st;
    }
  }
  hipLaunchKernelGGL(k_reduce_scalars, dim3(1), dim3(RED_T), 0, s, red, nred, d_ior, d_sigma);
  if (sc.env.d_w)
    if (dt_status st = mlp_wgrad_reduce(sc.env, mlp_part, s)) return st;
  if (fseg) {
    const int64_t nfe = 4 * (int64_t)sc.fd.nx * sc.fd.ny * sc.fd.nz + 12 * (int64_t)sc.fd.res * sc.fd.res;
    hipLaunchKernelGGL(k_field_gather, dim3(dt_blocks(nfe, 256) < 4096 ? dt_blocks(nfe, 256) : 4096), dim3(256), 0,
                       s, sc.fd, fcopies, f_copies);
  }
  if (n_copies > 0 && gcell)
    hipLaunchKernelGGL(k_grid_gather, dim3(dt_blocks(gsize, 256) < 4096 ? dt_blocks(gsize, 256) : 4096), dim3(256),
                       0, s, gcopies, n_copies, sc.ab.nx, sc.ab.ny, sc.ab.nz, sc.ab.d_mu);
  hipLaunchKernelGGL(k_vertex_gather, dim3(dt_blocks(scene->nv, 256)), dim3(256), 0, s, sc.bvh, sc.F, fg,
                     dV, dN);
  hipLaunchKernelGGL(k_nbwd_vertex, dim3(dt_blocks(scene->nv, 256)), dim3(256), 0, s, sc.bvh, dN, sbar);
  hipLaunchKernelGGL(k_nbwd_face, dim3(dt_blocks(scene->nf, 256)), dim3(256), 0, s, sc.bvh, sc.V, sc.F,
                     sbar, dV);
  DT_CHECK_LAUNCH();
  return DT_OK;
}

extern "C" dt_status dt_env_query(const dt_env* env, const float* dirs, int64_t n, float* rgb,
                                  void* stream) {
  EnvDev e;
  if (dt_status st = make_env(env, e)) return st;
  DT_REQUIRE(dirs && rgb && n >= 0, "dt_env_query: bad arguments");
  if (n == 0) return DT_OK;
  if (e.kind == DT_ENV_MLP) return mlp_query(e, dirs, n, rgb, (hipStream_t)stream);
  hipLaunchKernelGGL(k_env_query, dim3(dt_blocks(n, 256)), dim3(256), 0, (hipStream_t)stream, e, dirs,
                     n, rgb);
  DT_CHECK_LAUNCH();
  return DT_OK;
}

extern "C" dt_status dt_env_query_backward(const dt_env* env, const float* dirs, int64_t n,
                                           const float* grad_rgb, float* grad_dirs, void* stream) {
  EnvDev e;
  if (dt_status st = make_env(env, e)) return st;
  DT_REQUIRE(dirs && grad_rgb && grad_dirs && n >= 0, "dt_env_query_backward: bad arguments");
  if (n == 0) return DT_OK;
  if (e.kind == DT_ENV_MLP)
    return mlp_query_backward(e, dirs, n, grad_rgb, grad_dirs, (hipStream_t)stream);
  hipLaunchKernelGGL(k_env_query_bwd, dim3(dt_blocks(n, 256)), dim3(256), 0, (hipStream_t)stream, e,
                     dirs, n, grad_rgb, grad_dirs);
  DT_CHECK_LAUNCH();
  return DT_OK;
}

extern "C" dt_status dt_intersect(const dt_scene* scene, const float* o, const float* d,
                                  const int32_t* skip, int64_t n, float t_eps, int32_t brute_force,
                                  int32_t* tri, float* t, float* b, void* stream) {
  DT_REQUIRE(scene && scene->bvh && o && d && tri && t && b, "dt_intersect: NULL argument");
  DT_REQUIRE(scene->nv >= 3 && scene->nf >= 1 && scene->nf <= DT_MAX_FACES,
             "dt_intersect: bad mesh size");
  DT_REQUIRE(n >= 0 && n < (1ll << 31), "dt_intersect: bad ray count");
  if (n == 0) return DT_OK;
  BvhView bv = bvh_view(scene->bvh, scene->nv, scene->nf);
  hipLaunchKernelGGL(k_intersect, dim3(dt_blocks(n, TB)), dim3(TB), 0, (hipStream_t)stream, bv, o, d,
                     skip, n, t_eps, brute_force ? 1 : 0, tri, t, b);
  DT_CHECK_LAUNCH();
  return DT_OK;
}
