// Environment MLP on bf16 matrix cores (gfx950 MFMA 16x16x32, FP32 accumulate).
//
// E(d) = head( relu(... relu(W0 gamma(u) + b0) ...) ), u = d / |d|,
// gamma(u) = [u, sin(2^k pi u), cos(2^k pi u)]_{k < n_freq}, zero-padded to 64.
// Weights are bf16 (exact MFMA operands), biases FP32.  Every activation
// vector (the encoding and each hidden layer's ReLU output) is carried as
// three bf16 vectors (the top, middle and bottom 8 significant bits of the
// FP32 value, cut by truncation, so they sum to it exactly), and each layer is
// three MFMAs (W hi + W mid + W lo) accumulated in FP32: the products of bf16
// weights and bf16 parts are exact, so a layer is as accurate as an FP32
// matrix product.  (A single bf16 rounding per activation would put steps of
// 2^-9 relative into E, and a derivative that depends on which side of a step
// a ray lands.)  The encoding takes sin(pi t), cos(pi t) of t = 2^k u, which
// is exact in FP32 (as is its reduction to a fraction of a turn), so no
// argument rounding error grows with the frequency; the hardware sine and
// cosine then add at most 1.3e-7.
//
// A block first copies the whole network into LDS (rows padded by 4 bf16 so
// the 16 rows an MFMA operand spans fall on different banks; the RGB head
// padded to 16 zero rows), then its waves loop over groups of 16 rays, so the
// weights are read from HBM once per block and every MFMA operand comes from
// LDS.  One wave evaluates 16 rays at a time.  Layers are computed transposed,
// D[out][ray] = W[out][in] * H[in][ray], so W is the MFMA A operand and the
// activations the B operand; the accumulator layout of one layer (lane l holds
// rows 4*(l/16)+j of column l%16) gives each lane four rows of a 16-row
// block, and two consecutive blocks make the eight k values a lane supplies
// to one 16x16x32 product (the weights' A operand is gathered with the same k
// pairing), so activations never leave registers.  The input gradient runs
// the same way with W^T as the A operand and the upstream gradient split into
// hi + lo (about 16 bits; the gradient tolerance is 1e-3).
#include "dt_queue.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Three-part bf16 split of an FP32 value by truncation: hi keeps the top 8
// significant bits, mid the next 8 of the (exact) remainder, lo the last 8,
// so hi + mid + lo equals the FP32 value exactly (for normal values).
struct Split3 {
  short h, m, l;
};
__device__ __forceinline__ Split3 split3(float v) {
  Split3 s;
  uint32_t a = __float_as_uint(v) & 0xFFFF0000u;
  float r = v - __uint_as_float(a);
  uint32_t b = __float_as_uint(r) & 0xFFFF0000u;
  float t = r - __uint_as_float(b);
  s.h = (short)(a >> 16);
  s.m = (short)(b >> 16);
  s.l = (short)(__float_as_uint(t) >> 16);
  return s;
}

// The encoding in the matrix cores' input order.  Lane group q of a wave holds
// input rows 16 kb + 4 q + j (kb, j < 4) of its ray, so the input rows are
// renumbered: group q < 3 carries axis q in its 16 slots s = 4 kb + j (slot 0:
// u_q; slot 1 + 2f: sin(2^f pi u_q); slot 2 + 2f: cos(2^f pi u_q); f < n_freq
// <= DT_MLP_MAX_FREQ), group 3 and unused slots are zero.  The first layer's
// weight columns are permuted to match when the network is copied to LDS.
#define DT_MLP_MAX_FREQ 7

// input column (in the caller's order: u, then per frequency sin xyz, cos xyz)
// of input row k in the matrix cores' order, or -1 for a zero row
__device__ __forceinline__ int enc_column(int k, int n_freq) {
  const int q = (k & 15) >> 2, s = ((k >> 4) << 2) | (k & 3);
  if (q == 3) return -1;
  if (s == 0) return q;
  const int f = (s - 1) >> 1;
  if (f >= n_freq) return -1;
  return 3 + 6 * f + ((s & 1) ? q : 3 + q);
}

// sin(pi 2^f u), cos(pi 2^f u) for f < n_freq by the hardware sine and cosine
// (arguments in turns: 2^(f-1) u exactly, reduced by its nearest integer,
// also exact); within 1.3e-7 of the true values over |u| <= 1, f < 7
struct EncTrig {
  float sn[DT_MLP_MAX_FREQ], cs[DT_MLP_MAX_FREQ];
};
__device__ __forceinline__ EncTrig enc_trig(float uq, int n_freq) {
  EncTrig t;
#pragma unroll
  for (int f = 0; f < DT_MLP_MAX_FREQ; ++f) {
    t.sn[f] = 0.f;
    t.cs[f] = 0.f;
    if (f < n_freq) {
      float h = uq * (float)(1 << f) * 0.5f;
      h -= rintf(h);
      t.sn[f] = __builtin_amdgcn_sinf(h);
      t.cs[f] = __builtin_amdgcn_cosf(h);
    }
  }
  return t;
}

// slot s of a lane group carrying axis value uq
__device__ __forceinline__ float enc_slot(int s, float uq, const EncTrig& t, int n_freq) {
  if (s == 0) return uq;
  const int f = (s - 1) >> 1;
  if (f >= DT_MLP_MAX_FREQ || f >= n_freq) return 0.f;
  return (s & 1) ? t.sn[f] : t.cs[f];
}

// d slot / d uq
__device__ __forceinline__ float denc_slot(int s, const EncTrig& t, int n_freq) {
  if (s == 0) return 1.f;
  const int f = (s - 1) >> 1;
  if (f >= DT_MLP_MAX_FREQ || f >= n_freq) return 0.f;
  const float w = DT_PI * (float)(1 << f);
  return (s & 1) ? w * t.cs[f] : -w * t.sn[f];
}

constexpr int IN = 64;  // padded input width
// threads per block: 8 waves share one LDS copy of a 64-wide network; the
// 128-wide one (125 KB of LDS, one block per CU) runs 4 waves of up to 512
// registers each, which its backward pass needs
template <int HID>
constexpr int mlp_threads() {
  return HID == 64 ? 512 : 256;
}

// Layout of the LDS image of a (HID, NL) network: bf16 weights row by row with
// padded row strides (layer 0: HID x (IN + 4); hidden layers: HID x (HID + 4);
// head: 16 x (HID + 4), rows 3..15 zero), then FP32 biases (NL x HID, head 16).
// For the backward, a 64-wide network also keeps transposed copies of its
// hidden-layer and first weights ([in][out], stride HID + 4), so the W^T
// operands are two 8-byte LDS reads instead of eight 2-byte ones; a 128-wide
// one has no room.
template <int HID, int NL, bool GRAD>
struct NetLds {
  static constexpr bool TRANS = GRAD && HID <= 64;
  static constexpr int LD0 = IN + 4;
  static constexpr int LDH = HID + 4;
  static constexpr int W0 = 0;
  static constexpr int WH = W0 + HID * LD0;
  static constexpr int WO = WH + (NL - 1) * HID * LDH;
  static constexpr int T0 = WO + 16 * LDH;                            // W0^T: IN x LDH
  static constexpr int TH = T0 + (TRANS ? IN * LDH : 0);              // W_L^T: HID x LDH each
  static constexpr int WEND = TH + (TRANS ? (NL - 1) * HID * LDH : 0);
  static constexpr int BOFF = (WEND * 2 + 15) / 16 * 16;  // byte offset of the biases
  static constexpr int NB = NL * HID + 16;
  static constexpr int BYTES = BOFF + NB * 4;
  static_assert(BYTES <= 160 * 1024, "network does not fit in LDS");
};

// Cooperative copy of the network (global layout: W[l] row-major [out][in],
// biases concatenated) into its LDS image; ends with a barrier.
template <int HID, int NL, bool GRAD>
__device__ __forceinline__ void load_net(const EnvDev& e, uint16_t* sw, float* sb) {
  using N = NetLds<HID, NL, GRAD>;
  const uint16_t* W = e.w;
  // first layer: columns in the matrix cores' input order
  for (int i = threadIdx.x; i < HID * IN; i += blockDim.x) {
    const int col = enc_column(i % IN, e.n_freq);
    const uint16_t v = col >= 0 ? W[(i / IN) * IN + col] : (uint16_t)0;
    sw[N::W0 + (i / IN) * N::LD0 + (i % IN)] = v;
    if (N::TRANS) sw[N::T0 + (i % IN) * N::LDH + (i / IN)] = v;
  }
  W += HID * IN;
  for (int l = 1; l < NL; ++l) {
    for (int i = threadIdx.x; i < HID * HID; i += blockDim.x) {
      sw[N::WH + (l - 1) * HID * N::LDH + (i / HID) * N::LDH + (i % HID)] = W[i];
      if (N::TRANS) sw[N::TH + (l - 1) * HID * N::LDH + (i % HID) * N::LDH + (i / HID)] = W[i];
    }
    W += HID * HID;
  }
  for (int i = threadIdx.x; i < 16 * HID; i += blockDim.x)
    sw[N::WO + (i / HID) * N::LDH + (i % HID)] = i < 3 * HID ? W[i] : (uint16_t)0;
  for (int i = threadIdx.x; i < N::NB; i += blockDim.x)
    sb[i] = i < NL * HID + 3 ? e.b[i] : 0.f;
  __syncthreads();
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

// two-part bf16 split with rounding to nearest (ties to even) of both parts:
// hi + lo carries about 17 significant bits of the value
__device__ __forceinline__ short bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
struct Split2 {
  short h, l;
};
__device__ __forceinline__ Split2 split2(float v) {
  Split2 s;
  s.h = bf16_rne(v);
  s.l = bf16_rne(v - __uint_as_float((uint32_t)(uint16_t)s.h << 16));
  return s;
}

// K = 32 operand from two K = 16 halves: slots 0..3 take k = 4q + j of the
// first 16-block, slots 4..7 k = 4q + j of the second.  A and B operands are
// always built with the same pairing, so the product sums over the same 32 k
// whatever order the matrix core walks them in.
__device__ __forceinline__ bf16x8 cat8(bf16x4 lo16, bf16x4 hi16) {
  s16x8 v = __builtin_shufflevector(lo16, hi16, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// A operand of rows r16 of a weight block in LDS: columns c0 + 4q + (0..3) and
// c0 + 16 + 4q + (0..3) of row `row` (stride ld)
__device__ __forceinline__ bf16x8 wfrag(const uint16_t* w, int row, int ld, int c0, int q) {
  bf16x4 x = *(const bf16x4*)(w + row * ld + c0 + 4 * q);
  bf16x4 y = *(const bf16x4*)(w + row * ld + c0 + 16 + 4 * q);
  return cat8(x, y);
}
// A operand of the transposed weight block: W[k][col] for the same k pairing
__device__ __forceinline__ bf16x8 wfrag_t(const uint16_t* w, int col, int ld, int k0, int q) {
  bf16x4 x, y;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    x[j] = (short)w[(k0 + 4 * q + j) * ld + col];
    y[j] = (short)w[(k0 + 16 + 4 * q + j) * ld + col];
  }
  return cat8(x, y);
}

// ------------------------------------------------------------------ weight gradient
// dLoss/dW_l = sum over rays of delta_l a_{l-1}^T and dLoss/db_l = sum of
// delta_l, with delta_l the adjoint of layer l's pre-activation and a_{l-1}
// its input (the encoding for l = 0).  The sum over rays is a matrix product
// with the rays as the contraction axis, so it runs on the matrix cores too:
// the 8 waves of a block stage their 16 rays' deltas (two bf16 parts, about
// 17 bits) and inputs (hi and mid parts of the three-part split, 16 bits) for
// one layer in LDS, feature-major with the 128 rays along a row, then every
// wave adds the products of the tiles it owns into its accumulators
// (16x16x32 products with K = 32 rays: hi*hi + hi*mid + lo*hi; bias tiles
// multiply the deltas by a ones operand).  Tiles are dealt to the waves
// round-robin, so each entry of the gradient belongs to one lane of the block;
// at the end each block adds its accumulators into its own row of partial
// sums, and a final pass sums the rows in order.  64-wide networks only (the
// 128-wide network leaves no LDS for the staging).
constexpr int WG_WAVES = 8;
constexpr int WG_RAYS = 16 * WG_WAVES;      // rays staged per round
constexpr int WG_LD = WG_RAYS + 8;          // staged row stride (bf16): rows start 16 B apart in bank order
constexpr int WG_ROWS = 64;
constexpr int WG_STAGE = 4 * WG_ROWS * WG_LD;  // delta hi, delta lo, input hi, input mid
constexpr int WG_BLOCKS = 256;              // blocks of the weight-gradient backward (rows of partials)

template <int NL>
struct WgTiles {
  // the backward visits the head (layer NL) first, then layers NL-1 .. 0;
  // layer l has ob(l) 16-row output blocks times 4 16-column input blocks
  // of weight tiles, then ob(l) bias tiles
  static constexpr int ob(int l) { return l == NL ? 1 : 4; }
  static constexpr int count(int l) { return ob(l) * 5; }
  static constexpr int first(int l) {
    int t = 0;
    for (int k = NL; k > l; --k) t += count(k);
    return t;
  }
  static constexpr int total = count(NL) + NL * count(0);
  static constexpr int slots = (total + WG_WAVES - 1) / WG_WAVES;
  // flat parameter layout (weights of every layer, then biases), 64 wide
  static constexpr int64_t n_weights = 4096 * (int64_t)NL + 192;
  static constexpr int64_t n_params = n_weights + 64 * (int64_t)NL + 3;
};

__device__ __forceinline__ bf16x8 lds8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *(const s16x8*)p);
}

// Stage layer L's deltas (rows 16 ob + 4 q + j, ob < ob(L), of this wave's
// 16 rays) and inputs (rows 16 ib + 4 q + j, ib < 4), then accumulate the
// tiles of layer L this wave owns over the block's 128 rays.  Called by every
// wave of the block the same number of times (it holds two barriers).
template <int NL>
__device__ __forceinline__ void wg_stage(uint16_t* st, int L, const bf16x4* dh, const bf16x4* dl,
                                         const bf16x4* ah, const bf16x4* am, f32x4* wacc, int wave) {
  using T = WgTiles<NL>;
  const int l = threadIdx.x & 63, q = l >> 4, r16 = l & 15;
  uint16_t* Dh = st;
  uint16_t* Dl = st + WG_ROWS * WG_LD;
  uint16_t* Ah = st + 2 * WG_ROWS * WG_LD;
  uint16_t* Am = st + 3 * WG_ROWS * WG_LD;
  const int OB = T::ob(L);
  const int col = 16 * wave + r16;
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    if (ob >= OB) break;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Dh[(16 * ob + 4 * q + j) * WG_LD + col] = (uint16_t)dh[ob][j];
      Dl[(16 * ob + 4 * q + j) * WG_LD + col] = (uint16_t)dl[ob][j];
    }
  }
#pragma unroll
  for (int ib = 0; ib < 4; ++ib)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Ah[(16 * ib + 4 * q + j) * WG_LD + col] = (uint16_t)ah[ib][j];
      Am[(16 * ib + 4 * q + j) * WG_LD + col] = (uint16_t)am[ib][j];
    }
  __syncthreads();
  const int t0 = T::first(L);
  bf16x8 ones;
#pragma unroll
  for (int k = 0; k < 8; ++k) ones[k] = (__bf16)1.0f;
#pragma unroll
  for (int tl = 0; tl < 20; ++tl) {
    if (tl >= T::count(L)) break;
    const int t = t0 + tl;
    if (t % WG_WAVES != wave) continue;
    const bool bias = tl >= OB * 4;
    const int ob = bias ? tl - OB * 4 : tl / 4;
    const int ib = tl % 4;
    f32x4 acc = wacc[t / WG_WAVES];
#pragma unroll
    for (int ks = 0; ks < WG_RAYS / 32; ++ks) {
      const int c0 = 32 * ks + 8 * q;
      const bf16x8 a_h = lds8(Dh + (16 * ob + r16) * WG_LD + c0);
      const bf16x8 a_l = lds8(Dl + (16 * ob + r16) * WG_LD + c0);
      if (bias) {
        acc = mfma32(a_h, ones, acc);
        acc = mfma32(a_l, ones, acc);
      } else {
        const bf16x8 b_h = lds8(Ah + (16 * ib + r16) * WG_LD + c0);
        const bf16x8 b_m = lds8(Am + (16 * ib + r16) * WG_LD + c0);
        acc = mfma32(a_h, b_h, acc);
        acc = mfma32(a_h, b_m, acc);
        acc = mfma32(a_l, b_h, acc);
      }
    }
    wacc[t / WG_WAVES] = acc;
  }
  __syncthreads();
}

// Add this wave's tiles into the block's row of partial sums (each entry has
// one owner lane in the block, so no atomics).  Weight (o, i) of layer 0 is
// the caller's column enc_column(i); the head keeps rows o < 3.
template <int NL>
__device__ __forceinline__ void wg_flush(const f32x4* wacc, int wave, float* part, int n_freq) {
  using T = WgTiles<NL>;
  const int l = threadIdx.x & 63, q = l >> 4, r16 = l & 15;
#pragma unroll
  for (int t = 0; t < T::total; ++t) {
    if (t % WG_WAVES != wave) continue;
    int L = NL, tl = t;
    while (tl >= T::count(L)) {
      tl -= T::count(L);
      --L;
    }
    const int OB = T::ob(L);
    const bool bias = tl >= OB * 4;
    const int ob = bias ? tl - OB * 4 : tl / 4;
    const int ib = tl % 4;
    const f32x4 acc = wacc[t / WG_WAVES];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int o = 16 * ob + 4 * q + j;
      if (L == NL && o >= 3) continue;
      int64_t k;
      if (bias) {
        if (r16 != 0) continue;
        k = T::n_weights + 64 * (int64_t)L + o;
      } else {
        int i = 16 * ib + r16;
        if (L == 0) {
          i = enc_column(i, n_freq);
          if (i < 0) continue;
        }
        k = 4096 * (int64_t)L + 64 * (int64_t)o + i;
      }
      part[k] += acc[j];
    }
  }
}

// One wave: lane l works on ray l % 16 (all four lane groups q = l / 16 carry
// the same ray).  Returns E in lanes with q == 0; when GRAD, also returns
// the direction gradient of dot(gbar, E) with respect to d (all lanes).
// Activations live in 16-row blocks in the MFMA accumulator layout (lane
// (q, r16) holds rows 4q + j of column r16); two consecutive blocks form the
// B operand of one 16x16x32 product.
template <int HID, int NL, bool GRAD, bool WG = false>
__device__ __forceinline__ v3 mlp_wave(const uint16_t* sw, const float* sb, int n_freq, v3 d,
                                       v3 gbar, v3* dbar, uint16_t* stage = nullptr,
                                       f32x4* wacc = nullptr, int wave = 0) {
  static_assert(!WG || (GRAD && HID == 64), "weight gradient: 64-wide backward only");
  using N = NetLds<HID, NL, GRAD>;
  const int l = threadIdx.x & 63, q = l >> 4, r16 = l & 15;
  constexpr int KB = HID / 16;
  float inv_len = 1.0f / sqrtf(dot(d, d));
  v3 u = d * inv_len;
  // this lane group's axis (group 3 carries zeros)
  const float uq = q == 0 ? u.x : (q == 1 ? u.y : (q == 2 ? u.z : 0.f));
  const int nfq = q == 3 ? 0 : n_freq;
  const EncTrig trig = enc_trig(uq, nfq);
  bf16x4 xh[IN / 16], xm[IN / 16], xl[IN / 16];
#pragma unroll
  for (int kb = 0; kb < IN / 16; ++kb)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Split3 p = split3(enc_slot(4 * kb + j, uq, trig, nfq));
      xh[kb][j] = p.h;
      xm[kb][j] = p.m;
      xl[kb][j] = p.l;
    }
  bf16x4 act[NL][KB];     // hi parts of every hidden layer (their signs are the ReLU masks)
  bf16x4 mi[KB], lo[KB];  // mid and lo parts of the latest hidden layer
  bf16x4 actm[WG ? NL : 1][KB];  // mid parts of every hidden layer (weight gradient)
  const float* B = sb;
  // first hidden layer, on the encoding
#pragma unroll
  for (int ob = 0; ob < KB; ++ob) {
    f32x4 acc;
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = B[ob * 16 + 4 * q + j];
#pragma unroll
    for (int kb = 0; kb < IN / 32; ++kb) {
      bf16x8 a = wfrag(sw + N::W0, ob * 16 + r16, N::LD0, kb * 32, q);
      acc = mfma32(a, cat8(xl[2 * kb], xl[2 * kb + 1]), acc);
      acc = mfma32(a, cat8(xm[2 * kb], xm[2 * kb + 1]), acc);
      acc = mfma32(a, cat8(xh[2 * kb], xh[2 * kb + 1]), acc);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Split3 p = split3(fmaxf(acc[j], 0.f));
      act[0][ob][j] = p.h;
      mi[ob][j] = p.m;
      lo[ob][j] = p.l;
      if constexpr (WG) actm[0][ob][j] = p.m;
    }
  }
  B += HID;
  // further hidden layers
#pragma unroll
  for (int L = 1; L < NL; ++L) {
    const uint16_t* WL = sw + N::WH + (L - 1) * HID * N::LDH;
    bf16x4 nmi[KB], nlo[KB];
#pragma unroll
    for (int ob = 0; ob < KB; ++ob) {
      f32x4 acc;
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = B[ob * 16 + 4 * q + j];
#pragma unroll
      for (int kb = 0; kb < KB / 2; ++kb) {
        bf16x8 a = wfrag(WL, ob * 16 + r16, N::LDH, kb * 32, q);
        acc = mfma32(a, cat8(lo[2 * kb], lo[2 * kb + 1]), acc);
        acc = mfma32(a, cat8(mi[2 * kb], mi[2 * kb + 1]), acc);
        acc = mfma32(a, cat8(act[L - 1][2 * kb], act[L - 1][2 * kb + 1]), acc);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        Split3 p = split3(fmaxf(acc[j], 0.f));
        act[L][ob][j] = p.h;
        nmi[ob][j] = p.m;
        nlo[ob][j] = p.l;
        if constexpr (WG) actm[WG ? L : 0][ob][j] = p.m;
      }
    }
#pragma unroll
    for (int ob = 0; ob < KB; ++ob) {
      mi[ob] = nmi[ob];
      lo[ob] = nlo[ob];
    }
    B += HID;
  }
  // linear RGB head (3 rows, padded to 16 zero rows)
  f32x4 out;
#pragma unroll
  for (int j = 0; j < 4; ++j) out[j] = B[4 * q + j];
#pragma unroll
  for (int kb = 0; kb < KB / 2; ++kb) {
    bf16x8 a = wfrag(sw + N::WO, r16, N::LDH, kb * 32, q);
    out = mfma32(a, cat8(lo[2 * kb], lo[2 * kb + 1]), out);
    out = mfma32(a, cat8(mi[2 * kb], mi[2 * kb + 1]), out);
    out = mfma32(a, cat8(act[NL - 1][2 * kb], act[NL - 1][2 * kb + 1]), out);
  }
  v3 E = mk3(out[0], out[1], out[2]);
  if (!GRAD) return E;

  // ---- input gradient: delta_out rows 0..2 = gbar, B layout
  bf16x4 dh0, dl0;  // delta of the head output, hi / lo parts (rows 0..2 of lane group 0)
  {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Split2 p = split2((q == 0 && j < 3) ? comp(gbar, j) : 0.f);
      dh0[j] = p.h;
      dl0[j] = p.l;
    }
  }
  if constexpr (WG) wg_stage<NL>(stage, NL, &dh0, &dl0, act[NL - 1], actm[NL - 1], wacc, wave);
  // head: delta_hidden = W_head^T delta_out (a K = 16 product over the 16
  // padded head rows), masked by the last ReLU
  bf16x4 nh[KB], nl[KB];
#pragma unroll
  for (int ib = 0; ib < KB; ++ib) {
    bf16x4 a;
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = (short)sw[N::WO + (4 * q + j) * N::LDH + ib * 16 + r16];
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma(a, dh0, acc);
    acc = mfma(a, dl0, acc);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Split2 p = split2(act[NL - 1][ib][j] > 0 ? acc[j] : 0.f);
      nh[ib][j] = p.h;
      nl[ib][j] = p.l;
    }
  }
  // hidden layers NL-1 .. 1: delta_{L-1} = W_L^T delta_L, masked by relu'(layer L-1)
#pragma unroll
  for (int L = NL - 1; L >= 1; --L) {
    if constexpr (WG) wg_stage<NL>(stage, L, nh, nl, act[L - 1], actm[WG ? L - 1 : 0], wacc, wave);
    const uint16_t* WL = sw + N::WH + (L - 1) * HID * N::LDH;
    bf16x4 th[KB], tl[KB];
#pragma unroll
    for (int ib = 0; ib < KB; ++ib) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < KB / 2; ++kb) {
        bf16x8 a;
        if constexpr (N::TRANS)
          a = wfrag(sw + N::TH + (L - 1) * HID * N::LDH, ib * 16 + r16, N::LDH, kb * 32, q);
        else
          a = wfrag_t(WL, ib * 16 + r16, N::LDH, kb * 32, q);
        acc = mfma32(a, cat8(nh[2 * kb], nh[2 * kb + 1]), acc);
        acc = mfma32(a, cat8(nl[2 * kb], nl[2 * kb + 1]), acc);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        Split2 p = split2(act[L - 1][ib][j] > 0 ? acc[j] : 0.f);
        th[ib][j] = p.h;
        tl[ib][j] = p.l;
      }
    }
#pragma unroll
    for (int ib = 0; ib < KB; ++ib) {
      nh[ib] = th[ib];
      nl[ib] = tl[ib];
    }
  }
  if constexpr (WG) wg_stage<NL>(stage, 0, nh, nl, xh, xm, wacc, wave);
  // first layer: delta_enc = W_0^T delta_0 (64 rows), then d enc / d u_q
  float gq = 0.f;
#pragma unroll
  for (int ib = 0; ib < IN / 16; ++ib) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB / 2; ++kb) {
      bf16x8 a;
      if constexpr (N::TRANS)
        a = wfrag(sw + N::T0, ib * 16 + r16, N::LDH, kb * 32, q);
      else
        a = wfrag_t(sw + N::W0, ib * 16 + r16, N::LD0, kb * 32, q);
      acc = mfma32(a, cat8(nh[2 * kb], nh[2 * kb + 1]), acc);
      acc = mfma32(a, cat8(nl[2 * kb], nl[2 * kb + 1]), acc);
    }
    // acc[j] = d loss / d (slot 4 ib + j) of ray r16 in this lane group
#pragma unroll
    for (int j = 0; j < 4; ++j) gq += acc[j] * denc_slot(4 * ib + j, trig, nfq);
  }
  // lane group q < 3 holds d / d u_q; the groups of one ray are lanes r16 + 16 q
  float gx = q == 0 ? gq : 0.f, gy = q == 1 ? gq : 0.f, gz = q == 2 ? gq : 0.f;
  gx += __shfl_xor(gx, 16);
  gy += __shfl_xor(gy, 16);
  gz += __shfl_xor(gz, 16);
  gx += __shfl_xor(gx, 32);
  gy += __shfl_xor(gy, 32);
  gz += __shfl_xor(gz, 32);
  // through u = d / |d|
  v3 gu = mk3(gx, gy, gz);
  *dbar = (gu - u * dot(u, gu)) * inv_len;
  return E;
}

// ------------------------------------------------------------------ kernels
// Every block loads the network into LDS once, then each of its waves takes
// groups of 16 consecutive items in turn; items past the count run on a dummy
// direction and write nothing.  The loops' trip counts are uniform per wave.
#define DT_MLP_PROLOGUE(GRAD)                                             \
  using N = NetLds<HID, NL, GRAD>;                                        \
  __shared__ __align__(16) unsigned char net[N::BYTES];                  \
  uint16_t* sw = (uint16_t*)net;                                          \
  float* sb = (float*)(net + N::BOFF);                                    \
  load_net<HID, NL, GRAD>(e, sw, sb);                                     \
  const int waves = mlp_threads<HID>() / 64;                              \
  const int64_t wstep = (int64_t)gridDim.x * waves * 16;                  \
  const int64_t wfirst = ((int64_t)blockIdx.x * waves + (threadIdx.x >> 6)) * 16;

// An opaque zero offset per group: the weight reads then depend on the loop
// iteration, so the compiler streams them from LDS in every group instead of
// hoisting the whole network into registers (which spills for 128-wide nets).
__device__ __forceinline__ const uint16_t* per_group(const uint16_t* sw) {
  int z = 0;
  asm volatile("" : "+s"(z));
  return sw + z;
}

template <int HID, int NL>
__global__ void __launch_bounds__(mlp_threads<HID>()) k_mlp_query(EnvDev e, const float* dirs, int64_t n,
                                                           float* rgb) {
  DT_MLP_PROLOGUE(false)
  for (int64_t w0 = wfirst; w0 < n; w0 += wstep) {
    int64_t item = w0 + (threadIdx.x & 15);
    bool valid = item < n;
    v3 d = valid ? load3(dirs + 3 * item) : mk3(0.f, 1.f, 0.f);
    v3 dummy;
    v3 E = mlp_wave<HID, NL, false>(per_group(sw), sb, e.n_freq, d, mk3(0.f, 0.f, 0.f), &dummy);
    if (valid && (threadIdx.x & 63) < 16) {
      rgb[3 * item] = E.x;
      rgb[3 * item + 1] = E.y;
      rgb[3 * item + 2] = E.z;
    }
  }
}

template <int HID, int NL>
__global__ void __launch_bounds__(mlp_threads<HID>()) k_mlp_query_bwd(EnvDev e, const float* dirs, int64_t n,
                                                               const float* g, float* gd) {
  DT_MLP_PROLOGUE(true)
  for (int64_t w0 = wfirst; w0 < n; w0 += wstep) {
    int64_t item = w0 + (threadIdx.x & 15);
    bool valid = item < n;
    v3 d = valid ? load3(dirs + 3 * item) : mk3(0.f, 1.f, 0.f);
    v3 gb = valid ? load3(g + 3 * item) : mk3(0.f, 0.f, 0.f);
    v3 db;
    mlp_wave<HID, NL, true>(per_group(sw), sb, e.n_freq, d, gb, &db);
    if (valid && (threadIdx.x & 63) < 16) {
      gd[3 * item] = db.x;
      gd[3 * item + 1] = db.y;
      gd[3 * item + 2] = db.z;
    }
  }
}

template <int HID, int NL>
__global__ void __launch_bounds__(mlp_threads<HID>()) k_mlp_trace_fwd(EnvDev e, Gen q, const uint32_t* list,
                                                               const Counters* ctr, int g, float* rgb) {
  DT_MLP_PROLOGUE(false)
  const int64_t n = ctr->nmiss[g];
  for (int64_t w0 = wfirst; w0 < n; w0 += wstep) {
    int64_t item = w0 + (threadIdx.x & 15);
    bool valid = item < n;
    uint32_t i = valid ? list[item] : 0u;
    float4 d4 = valid ? q.d[i] : make_float4(0.f, 1.f, 0.f, 0.f);
    v3 dummy;
    v3 E = mlp_wave<HID, NL, false>(per_group(sw), sb, e.n_freq, xyz(d4), mk3(0.f, 0.f, 0.f), &dummy);
    if (valid && (threadIdx.x & 63) < 16) {
      float4 w4 = q.w[i];
      int pix = __float_as_int(d4.w);
      atomicAdd(rgb + 3 * pix, w4.x * E.x);
      atomicAdd(rgb + 3 * pix + 1, w4.y * E.y);
      atomicAdd(rgb + 3 * pix + 2, w4.z * E.z);
    }
  }
}

template <int HID, int NL>
__global__ void __launch_bounds__(mlp_threads<HID>()) k_mlp_trace_bwd(EnvDev e, Gen q, const uint32_t* list,
                                                               const Counters* ctr, int g,
                                                               const float* grad_rgb, Adj cur) {
  DT_MLP_PROLOGUE(true)
  const int64_t n = ctr->nmiss[g];
  for (int64_t w0 = wfirst; w0 < n; w0 += wstep) {
    int64_t item = w0 + (threadIdx.x & 15);
    bool valid = item < n;
    uint32_t i = valid ? list[item] : 0u;
    float4 d4 = valid ? q.d[i] : make_float4(0.f, 1.f, 0.f, 0.f);
    v3 gb = mk3(0.f, 0.f, 0.f);
    if (valid) {
      float4 w4 = q.w[i];
      int pix = __float_as_int(d4.w);
      v3 gp = load3(grad_rgb + 3 * pix);
      gb = mk3(gp.x * w4.x, gp.y * w4.y, gp.z * w4.z);
    }
    v3 db;
    v3 E = mlp_wave<HID, NL, true>(per_group(sw), sb, e.n_freq, xyz(d4), gb, &db);
    if (valid && (threadIdx.x & 63) < 16) {
      cur.L[i] = make_float4(E.x, E.y, E.z, 0.f);
      cur.O[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      cur.D[i] = make_float4(db.x, db.y, db.z, 0.f);
    }
  }
}
#undef DT_MLP_PROLOGUE

// The trace adjoint of k_mlp_trace_bwd for a 64-wide network, also summing the
// weight and bias gradient: rounds of 128 listed rays per block (all waves
// take part in every round; rays past the count carry a zero adjoint), the
// block's sums added into part[blockIdx.x][...] at the end.
template <int NL>
__global__ void __launch_bounds__(16 * WG_RAYS / 4) k_mlp_trace_bwd_wg(EnvDev e, Gen q, const uint32_t* list,
                                                               const Counters* ctr, int g,
                                                               const float* grad_rgb, Adj cur,
                                                               float* part) {
  using N = NetLds<64, NL, true>;
  using T = WgTiles<NL>;
  __shared__ __align__(16) unsigned char net[N::BYTES];
  __shared__ __align__(16) uint16_t stage[WG_STAGE];
  uint16_t* sw = (uint16_t*)net;
  float* sb = (float*)(net + N::BOFF);
  load_net<64, NL, true>(e, sw, sb);
  const int wave = threadIdx.x >> 6;
  f32x4 wacc[T::slots];
#pragma unroll
  for (int k = 0; k < T::slots; ++k) wacc[k] = {0.f, 0.f, 0.f, 0.f};
  const int64_t n = ctr->nmiss[g];
  for (int64_t b0 = (int64_t)blockIdx.x * WG_RAYS; b0 < n; b0 += (int64_t)gridDim.x * WG_RAYS) {
    int64_t item = b0 + 16 * wave + (threadIdx.x & 15);
    bool valid = item < n;
    uint32_t i = valid ? list[item] : 0u;
    float4 d4 = valid ? q.d[i] : make_float4(0.f, 1.f, 0.f, 0.f);
    v3 gb = mk3(0.f, 0.f, 0.f);
    if (valid) {
      float4 w4 = q.w[i];
      int pix = __float_as_int(d4.w);
      v3 gp = load3(grad_rgb + 3 * pix);
      gb = mk3(gp.x * w4.x, gp.y * w4.y, gp.z * w4.z);
    }
    v3 db;
    v3 E = mlp_wave<64, NL, true, true>(per_group(sw), sb, e.n_freq, xyz(d4), gb, &db, stage, wacc, wave);
    if (valid && (threadIdx.x & 63) < 16) {
      cur.L[i] = make_float4(E.x, E.y, E.z, 0.f);
      cur.O[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      cur.D[i] = make_float4(db.x, db.y, db.z, 0.f);
    }
  }
  wg_flush<NL>(wacc, wave, part + (size_t)blockIdx.x * T::n_params, e.n_freq);
}

// d_w[k] (k < n_weights) and d_b[k - n_weights]: the blocks' partial sums,
// added in block order
__global__ void k_mlp_wg_reduce(const float* part, int64_t n_params, int64_t n_weights, float* d_w,
                                float* d_b) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_params;
       k += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < WG_BLOCKS; ++b) s += (double)part[(size_t)b * n_params + k];
    if (k < n_weights)
      d_w[k] = (float)s;
    else
      d_b[k - n_weights] = (float)s;
  }
}

// dispatch over the supported (hidden width, hidden layers) shapes
#define DT_MLP_SHAPES(X) X(64, 1) X(64, 2) X(64, 3) X(64, 4) X(128, 1) X(128, 2) X(128, 3) X(128, 4)

// enough blocks to cover n items (16 per wave), at most a few resident per CU
unsigned mlp_blocks(int64_t n, int threads) {
  int64_t per = threads / 4;  // 16 items per wave
  int64_t b = (n + per - 1) / per;
  const int64_t cap = 256 * 4;
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

bool mlp_supported(const EnvDev& e) {
  return e.in_pad == IN && (e.hidden == 64 || e.hidden == 128) && e.n_layers >= 1 &&
         e.n_layers <= 4 && e.n_freq >= 0 && e.n_freq <= DT_MLP_MAX_FREQ && e.w && e.b;
}

#define DT_LAUNCH(H, L, kern, grid, ...)                                                    \
  if (e.hidden == H && e.n_layers == L) {                                                   \
    hipLaunchKernelGGL((kern<H, L>), dim3(grid), dim3(mlp_threads<H>()), 0, s, __VA_ARGS__); \
    DT_CHECK_LAUNCH();                                                                      \
    return DT_OK;                                                                           \
  }

dt_status mlp_query(const EnvDev& e, const float* dirs, int64_t n, float* rgb, hipStream_t s) {
#define X(H, L) DT_LAUNCH(H, L, k_mlp_query, mlp_blocks(n, mlp_threads<H>()), e, dirs, n, rgb)
  DT_MLP_SHAPES(X)
#undef X
  dt_set_error("environment MLP shape (hidden %d, layers %d) is not supported", e.hidden, e.n_layers);
  return DT_ERR_UNSUPPORTED;
}

dt_status mlp_query_backward(const EnvDev& e, const float* dirs, int64_t n, const float* g,
                             float* gd, hipStream_t s) {
#define X(H, L) DT_LAUNCH(H, L, k_mlp_query_bwd, mlp_blocks(n, mlp_threads<H>()), e, dirs, n, g, gd)
  DT_MLP_SHAPES(X)
#undef X
  dt_set_error("environment MLP shape (hidden %d, layers %d) is not supported", e.hidden, e.n_layers);
  return DT_ERR_UNSUPPORTED;
}

dt_status mlp_trace_forward(const EnvDev& e, Gen q, const uint32_t* list, const Counters* ctr,
                            int g, int64_t cap, float* rgb, hipStream_t s) {
#define X(H, L) DT_LAUNCH(H, L, k_mlp_trace_fwd, mlp_blocks(cap, mlp_threads<H>()), e, q, list, ctr, g, rgb)
  DT_MLP_SHAPES(X)
#undef X
  dt_set_error("environment MLP shape (hidden %d, layers %d) is not supported", e.hidden, e.n_layers);
  return DT_ERR_UNSUPPORTED;
}

int64_t mlp_wgrad_params(const EnvDev& e) {
  return e.hidden == 64 ? 4096 * (int64_t)e.n_layers + 192 + 64 * (int64_t)e.n_layers + 3 : 0;
}

size_t mlp_wgrad_scratch_bytes() {
  return sizeof(float) * (size_t)WG_BLOCKS * (size_t)WgTiles<4>::n_params;
}

dt_status mlp_wgrad_reduce(const EnvDev& e, const float* part, hipStream_t s) {
  const int64_t np = mlp_wgrad_params(e);
  const int64_t nw = np - 64 * (int64_t)e.n_layers - 3;
  hipLaunchKernelGGL(k_mlp_wg_reduce, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, part, np, nw,
                     e.d_w, e.d_b);
  DT_CHECK_LAUNCH();
  return DT_OK;
}

dt_status mlp_trace_backward_wgrad(const EnvDev& e, Gen q, const uint32_t* list, const Counters* ctr,
                                   int g, const float* grad_rgb, Adj cur, float* part, hipStream_t s) {
#define X(L)                                                                                    \
  if (e.hidden == 64 && e.n_layers == L) {                                                      \
    hipLaunchKernelGGL(k_mlp_trace_bwd_wg<L>, dim3(WG_BLOCKS), dim3(16 * WG_RAYS / 4), 0, s, e, q, \
                       list, ctr, g, grad_rgb, cur, part);                                      \
    DT_CHECK_LAUNCH();                                                                          \
    return DT_OK;                                                                               \
  }
  X(1) X(2) X(3) X(4)
#undef X
  dt_set_error("environment MLP weight gradient: hidden width 64 only (got %d)", e.hidden);
  return DT_ERR_UNSUPPORTED;
}

dt_status mlp_trace_backward(const EnvDev& e, Gen q, const uint32_t* list, const Counters* ctr,
                             int g, int64_t cap, const float* grad_rgb, Adj cur, hipStream_t s) {
#define X(H, L) DT_LAUNCH(H, L, k_mlp_trace_bwd, mlp_blocks(cap, mlp_threads<H>()), e, q, list, ctr, g, grad_rgb, cur)
  DT_MLP_SHAPES(X)
#undef X
  dt_set_error("environment MLP shape (hidden %d, layers %d) is not supported", e.hidden, e.n_layers);
  return DT_ERR_UNSUPPORTED;
}
