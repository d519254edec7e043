// lbnet_kernels.hpp -- gfx950 kernels of the learned boundary upsampler.
//
// The network maps the coarse boundary samples of one box face (an R x R
// corner-aligned grid every dt steps, the SAMPLED source of the boundary
// velocity, Sec. 2-3) to the per-step 64 x 64 face field, as a residual over
// the bilinear-in-space x linear-in-time interpolation of those samples.
//
// One network sample is (face, step n in the window [t_k, t_k+1)):
//   input   S_{k-1}, S_k, S_{k+1}, S_{k+2} on the coarse grid ([4][3][R][R])
//           and the phase theta = (n - t_k) / dt
//   lift    L = corner-aligned bilinear lift of a coarse grid to 64 x 64; with
//           Sb = (1 - theta) S_k + theta S_k+1 and s the RMS of the sample's
//           4 x 3 x R x R coarse values, the 16 input channels are
//             0..2   L(Sb) / s
//             3..5   L(Duu Sb) / s    Duu, Dvv: coarse second differences
//             6..8   L(Dvv Sb) / s    (at the edge nodes: the next node's)
//             9..11  L(S_k+2 - S_k+1 - S_k + S_k-1) / s
//             12     theta
//             13, 14 4 a (1 - a), 4 b (1 - b): position of the node inside
//                    its coarse cell (a along u, b along v)
//             15     0
//   net     conv3x3(16 -> 64) ReLU, conv3x3(64 -> 64) ReLU, conv3x3(64 -> 16),
//           zero padding; input channel 15 and output channels 3..15 carry
//           zero weights
//   output  u = base + s r, base = L(Sb) (the plain interpolation)
//
// Layouts: activations NHWC bfloat16 [B][64][64][C]; device weights
// [tap][co][ci] bfloat16 (tap = 3 (dy + 1) + (dx + 1)) from FP32 master
// weights of the same layout; the backward-data weights are the same array
// with the tap mirrored and co/ci exchanged.  Products run on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation: lane l holds rows l % 16
// (A) / columns l % 16 (B) and the eight K values 8 (l / 16) .. +7; the
// accumulator holds rows 4 (l / 16) .. +3 of column l % 16.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbnet {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int NB = 256;     // threads per workgroup
constexpr int NBC = 512;    // threads per convolution workgroup: one row of a tile per wave pair
constexpr int TR = 4;       // image rows per convolution tile
constexpr int IMG = 64;     // image edge (face nodes)
constexpr int CIN = 16;     // lifted input channels (15 used)
constexpr int CH = 64;      // hidden channels
constexpr int COUT = 16;    // output channels of the last layer (3 used)
constexpr int NTAP = 9;

__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }  // round to nearest even
__device__ __forceinline__ float from_bf16(__bf16 v) { return (float)v; }

// LDS rows of C bf16 values (a pixel's channels, a weight row's input
// channels), read as 16-byte fragments: lane l takes row p0 + l % 16 and
// chunk c0 + l / 16.  A 128-bit LDS read is served 16 lanes per cycle over 64
// banks, lanes grouped within each half wave by the parity of bits 2..4 of the
// lane index ({0-3, 12-15, 20-27}, {4-11, 16-19, 28-31}; measured with the
// bank-conflict counter on the device), so rows of 128 bytes (C = 64) take
// 4-way conflicts and rows padded to 144 bytes 2-way.  With C = 64, chunk c of
// row p is stored at chunk c ^ (p & 7): the 16 lanes of every group then hit
// 16 distinct bank quads for any row offset.  Rows of 32 bytes (C = 16) are
// conflict-free as they are.  Returns the element offset of chunk c8 of row.
template <int C>
__device__ __forceinline__ int lds_at(int row, int c8) {
  static_assert(C == 16 || C == 64, "LDS rows of 16 or 64 channels");
  if constexpr (C == 64) return row * 64 + 8 * (c8 ^ (row & 7));
  else return row * C + 8 * c8;
}

// ---------------------------------------------------------------- lift
// The lift of one sample b.  coarse [B][4][3][R][R] (row v, column u),
// theta [B].  The coarse feature grids (Sb, Duu Sb, Dvv Sb, temporal
// difference) are formed in LDS first (R <= 32).
// Window mode (win.samples != NULL): the inputs of window k of a box's
// sampled face history [ns][6][R][R][3] are read from it directly: sample
// b = j * 6 + f (step t_k + j, face f) takes coarse[b][tau][c][v][u] =
// samples[clamp(k - 1 + tau)][f][v][u][c] and theta = j / dt.
struct LiftWindow {
  const float* samples;
  int ns, k, dt;
};

// The sample's coarse values into cin [12 R R] and its features into feat,
// node-major: feat[(v R + u) 12 + ch], ch = 3 grid + component (grids Sb,
// Duu Sb, Dvv Sb, temporal difference), so a node's 12 features are three
// 16-byte LDS reads
// [12 R R] (block of NT threads, red: NT doubles of LDS); returns s (the RMS
// of the coarse values, 1 if they are all zero) and theta.
template <int NT>
__device__ __forceinline__ void lift_prepare(int b, int R, const float* __restrict__ coarse,
                                             const float* __restrict__ theta, const LiftWindow& win,
                                             float* cin, float* feat, double* red, float& s_out,
                                             float& th_out) {
  const int tid = threadIdx.x, RR = R * R;
  for (int i = tid; i < 12 * RR; i += NT) {
    if (win.samples) {
      const int j = b / 6, f = b - 6 * j;
      const int tau = i / (3 * RR), rem = i - tau * 3 * RR;
      const int cc = rem / RR, vu = rem - cc * RR;
      int ks = win.k - 1 + tau;
      ks = ks < 0 ? 0 : (ks > win.ns - 1 ? win.ns - 1 : ks);
      cin[i] = win.samples[(((size_t)ks * 6 + f) * RR + vu) * 3 + cc];
    } else {
      cin[i] = coarse[(size_t)b * 12 * RR + i];
    }
  }
  __syncthreads();
  const float* c = cin;
  double ss = 0.0;
  for (int i = tid; i < 12 * RR; i += NT) ss += (double)c[i] * (double)c[i];
  red[tid] = ss;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  const double rms = sqrt(red[0] / (12.0 * RR));
  const float s = rms > 0.0 ? (float)rms : 1.0f;
  const float th = win.samples ? (float)(b / 6) / (float)win.dt : theta[b];
  // Sb and the temporal difference
  for (int i = tid; i < 3 * RR; i += NT) {
    const int cmp = i / RR, vu = i - cmp * RR;
    const float sm = c[(0 * 3 + cmp) * RR + vu], s0 = c[(1 * 3 + cmp) * RR + vu];
    const float s1 = c[(2 * 3 + cmp) * RR + vu], s2 = c[(3 * 3 + cmp) * RR + vu];
    feat[vu * 12 + 0 * 3 + cmp] = (1.0f - th) * s0 + th * s1;
    feat[vu * 12 + 3 * 3 + cmp] = (s2 - s1) - (s0 - sm);
  }
  __syncthreads();
  // second differences of Sb along u and v (edge nodes take the next node's)
  for (int i = tid; i < 3 * RR; i += NT) {
    const int cmp = i / RR, vu = i - cmp * RR;
    const int v = vu / R, u = vu - v * R;
    const float* g = feat + cmp;  // Sb of component cmp, node stride 12
    const int uc = u < 1 ? 1 : (u > R - 2 ? R - 2 : u), vc = v < 1 ? 1 : (v > R - 2 ? R - 2 : v);
    feat[vu * 12 + 1 * 3 + cmp] = R >= 3 ? g[(v * R + uc + 1) * 12] - 2.0f * g[(v * R + uc) * 12] +
                                               g[(v * R + uc - 1) * 12]
                                         : 0.0f;
    feat[vu * 12 + 2 * 3 + cmp] = R >= 3 ? g[((vc + 1) * R + u) * 12] - 2.0f * g[(vc * R + u) * 12] +
                                               g[((vc - 1) * R + u) * 12]
                                         : 0.0f;
  }
  __syncthreads();
  s_out = s;
  th_out = th;
}

// The 16 input channels of pixel (u, v) (two vectors of 8) and the lifted
// coarse field lifted[0..2] (the plain interpolation, the output's base).
__device__ __forceinline__ void lift_pixel(const float* feat, int R, float s, float th, int u, int v,
                                           bf16x8& lo, bf16x8& hi, float base3[3]) {
  // corner-aligned bilinear weights (same integer mapping as the face grid)
  const int su = u * (R - 1), sv = v * (R - 1);
  const int pu = su / (IMG - 1), pv = sv / (IMG - 1);
  const float au = (float)(su - pu * (IMG - 1)) / (float)(IMG - 1);
  const float av = (float)(sv - pv * (IMG - 1)) / (float)(IMG - 1);
  const int pu1 = pu + 1 < R ? pu + 1 : pu, pv1 = pv + 1 < R ? pv + 1 : pv;
  float c00[12], c01[12], c10[12], c11[12];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    *(float4*)&c00[4 * k] = *(const float4*)&feat[(pv * R + pu) * 12 + 4 * k];
    *(float4*)&c01[4 * k] = *(const float4*)&feat[(pv * R + pu1) * 12 + 4 * k];
    *(float4*)&c10[4 * k] = *(const float4*)&feat[(pv1 * R + pu) * 12 + 4 * k];
    *(float4*)&c11[4 * k] = *(const float4*)&feat[(pv1 * R + pu1) * 12 + 4 * k];
  }
  float lifted[12];
#pragma unroll
  for (int ch = 0; ch < 12; ch++)
    lifted[ch] = (1.0f - au) * (1.0f - av) * c00[ch] + au * (1.0f - av) * c01[ch] + (1.0f - au) * av * c10[ch] +
                 au * av * c11[ch];
#pragma unroll
  for (int ch = 0; ch < 8; ch++) lo[ch] = to_bf16(lifted[ch] / s);
#pragma unroll
  for (int ch = 8; ch < 12; ch++) hi[ch - 8] = to_bf16(lifted[ch] / s);
  hi[4] = to_bf16(th);
  hi[5] = to_bf16(4.0f * au * (1.0f - au));
  hi[6] = to_bf16(4.0f * av * (1.0f - av));
  hi[7] = to_bf16(0.0f);
#pragma unroll
  for (int k = 0; k < 3; k++) base3[k] = lifted[k];
}

// ---------------------------------------------------------------- conv
// Products with the weights as the A operand and the pixels as B: the
// accumulator of block (mb, nb) holds, in lane l, pixel 16 mb + l % 16 and
// output slots 16 nb + 4 (l / 16) + j, j = 0..3.  The weights are staged into
// LDS with their rows permuted so that slot 16 nb + 4 g + j carries channel
// co_of<CO>(slot) = 16 g + 4 nb + j: lane l then holds the 4 NBK consecutive
// channels from first_co<CO>(l) of one pixel, which leave as whole 16-byte
// (CO = 64) or 8-byte (CO = 16) vectors.
template <int CO>
__device__ __forceinline__ int co_of(int slot) {
  if constexpr (CO == 64) return 16 * ((slot & 15) >> 2) + 4 * (slot >> 4) + (slot & 3);
  else return slot;
}
template <int CO>
__device__ __forceinline__ int first_co(int lane) { return (CO == 64 ? 16 : 4) * (lane >> 4); }

// Epilogue of one pixel's NC = 4 NBK consecutive channels c0 .. c0 + NC - 1
// (v[q] = channel c0 + q) at pixel index p (b * 64 + y) * 64 + x: bias + ReLU
// -> bf16, whole 16- or 8-byte vectors.
template <int CO, int NC>
__device__ __forceinline__ void store_pixel(const float (&v)[NC], size_t p, int c0,
                                            const float* __restrict__ bias, __bf16* __restrict__ out) {
  constexpr int VS = NC >= 8 ? 8 : NC;  // bf16 values per vector access
  const size_t o = p * CO + c0;
  __bf16 h[NC];
#pragma unroll
  for (int q = 0; q < NC; q++) {
    const float t = v[q] + bias[c0 + q];
    h[q] = to_bf16(t > 0.0f ? t : 0.0f);
  }
#pragma unroll
  for (int q = 0; q < NC; q += VS) {
    if constexpr (VS == 8) *(uint4*)&out[o + q] = *(const uint4*)&h[q];
    else *(uint2*)&out[o + q] = *(const uint2*)&h[q];
  }
}

// The products of one tile row for a wave: 32 pixels (px0 ..) of output row
// y against all CO output slots of the staged weights, K = 9 CI in chunks of
// 32 (with PF, the fragments of the next two chunks load while a chunk
// multiplies; with KEEP_ORDER, the compiler may not move those loads down to
// their use, which it otherwise does: measured faster in the backward pass
// and the forward's last layer, not in its 64 -> 64 layer).  The input
// row y + dy starts at LDS pixel row_at[dy + 1] (rows of IMG + 2 pixels, zero
// halo).
template <int CI, int CO, bool PF = true, int MB = 2, int NBK = CO / 16, bool KEEP_ORDER = false>
__device__ __forceinline__ void conv_products(const __bf16* sx, const __bf16* sw, const int (&row_at)[3], int px0,
                                              int lane, f32x4 (&acc)[MB][NBK], int nb0 = 0) {
  constexpr int KCH = (NTAP * CI + 31) / 32;
#pragma unroll
  for (int mb = 0; mb < MB; mb++)
#pragma unroll
    for (int nb = 0; nb < NBK; nb++) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto frag = [&](int kc, bf16x8 (&a)[MB], bf16x8 (&bb)[NBK]) {
    const int k0 = 32 * kc + 8 * (lane >> 4);
    const bool kv = k0 < NTAP * CI;
    const int tap = kv ? k0 / CI : 0, ci = kv ? k0 - tap * CI : 0;
    const int dyi = tap / 3, dx = tap % 3 - 1;
    const int rb = dyi == 0 ? row_at[0] : (dyi == 1 ? row_at[1] : row_at[2]);
#pragma unroll
    for (int mb = 0; mb < MB; mb++) {
      const int px = px0 + 16 * mb + (lane & 15);
      a[mb] = kv ? *(const bf16x8*)&sx[lds_at<CI>(rb + px + 1 + dx, ci >> 3)] : bf16x8{};
    }
#pragma unroll
    for (int nb = 0; nb < NBK; nb++) {
      const int slot = 16 * (nb0 + nb) + (lane & 15);
      bb[nb] = kv ? *(const bf16x8*)&sw[lds_at<CI>(tap * CO + slot, ci >> 3)] : bf16x8{};
    }
  };
  auto mult = [&](const bf16x8 (&a)[MB], const bf16x8 (&bb)[NBK]) {
#pragma unroll
    for (int mb = 0; mb < MB; mb++)
#pragma unroll
      for (int nb = 0; nb < NBK; nb++)
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bb[nb], a[mb], acc[mb][nb], 0, 0, 0);
  };
  if constexpr (PF) {
    // fragments of chunks kc + 1 and kc + 2 in flight while chunk kc multiplies
    bf16x8 fa[3][MB], fb[3][NBK];
    frag(0, fa[0], fb[0]);
    if (KCH > 1) frag(1, fa[1], fb[1]);
#pragma unroll
    for (int kc = 0; kc < KCH; kc++) {
      if (kc + 2 < KCH) frag(kc + 2, fa[(kc + 2) % 3], fb[(kc + 2) % 3]);
      if constexpr (KEEP_ORDER) __builtin_amdgcn_sched_barrier(0);
      mult(fa[kc % 3], fb[kc % 3]);
    }
  } else {
#pragma unroll 2
    for (int kc = 0; kc < KCH; kc++) {
      bf16x8 a[MB], bb[NBK];
      frag(kc, a, bb);
      mult(a, bb);
    }
  }
}

// Stage the weights [tap][co][ci] into LDS with their rows in slot order.
template <int CI, int CO>
__device__ __forceinline__ void stage_weights(const __bf16* __restrict__ w, __bf16* sw, int tid) {
  for (int i = tid; i < NTAP * CO * (CI / 8); i += NBC) {
    const int row = i / (CI / 8), c8 = i - row * (CI / 8);
    const int tap = row / CO, slot = row - tap * CO;
    *(uint4*)&sw[lds_at<CI>(row, c8)] = *(const uint4*)&w[((size_t)tap * CO + co_of<CO>(slot)) * CI + 8 * c8];
  }
}

// The epilogue of a wave's tile row: pixels px0 .. px0 + 31 of image row y.
template <int CO, int MB = 2>
__device__ __forceinline__ void store_row(const f32x4 (&acc)[MB][CO / 16], int b, int y, int px0, int lane,
                                          const float* __restrict__ bias, __bf16* __restrict__ out) {
  constexpr int NBK = CO / 16, NC = 4 * NBK;
  const int c0 = first_co<CO>(lane);
#pragma unroll
  for (int mb = 0; mb < MB; mb++) {
    float v[NC];
#pragma unroll
    for (int nb = 0; nb < NBK; nb++)
#pragma unroll
      for (int j = 0; j < 4; j++) v[4 * nb + j] = acc[mb][nb][j];
    const int px = px0 + 16 * mb + (lane & 15);
    store_pixel<CO, NC>(v, ((size_t)b * IMG + y) * IMG + px, c0, bias, out);
  }
}

// ---------------------------------------------------------------- layers 2 + 3
// Layer 2 (64 -> 64, bias, ReLU) and layer 3 (64 -> 16) in one pass, so the
// layer-2 activations stay on chip.  Workgroup g takes the 64 / bands output
// rows [yb, ye) of band g % bands of image g / bands in steps of two rows:
// step s makes layer-2 rows ya, ya + 1 (ya = yb - 1 + 2 s) from layer-1 rows
// ya - 1 .. ya + 2 and then layer-3 rows ya - 1, ya (for s >= 1) from layer-2
// rows ya - 2 .. ya + 1.  Both activations live in LDS rings of four rows
// (row yy in slot (yy + 4) % 4, 66 pixels with a zero halo); the weights of
// both layers are staged once (159,744 bytes of LDS in all).  The layer-1
// rows of the next step travel in registers one step ahead.  Layer-2 rows
// outside the image are zero (layer 3's padding); the two layer-2 rows past
// each end of a band are computed by both neighbours.  Each output is the
// same chain of products (conv_products, chunks in order of increasing K) as
// a convolution of one layer at a time would compute, so the results do not
// depend on the band split or the fusion.  a2_out != NULL also stores the band's
// layer-2 rows (the backward pass reads them).  EPI3: 1 (r), 2 (r and the
// loss: dy and one partial of sum e^2 per workgroup, see loss_epilogue) or 3 (u).
struct LossOut {
  const float* truth;  // [B][64][64][3]
  float dy_scale;      // 2 / count
  __bf16* dy;          // [B][64][64][16]
  double* part;        // one partial per workgroup
};

// e = (pred - truth) / s with pred = base + s r (channels 0..2 of the fp32
// last-layer output r): the error in units of the sample's coarse RMS; the
// loss is the mean of e^2 and dy = dL/dr = 2 e / count (bf16, channels 3..15
// zero).  A lane holds channels c3 .. c3 + 3 of pixel p; returns its e^2 sum.
__device__ __forceinline__ double loss_epilogue(const float (&r)[4], int c3, size_t p, float s,
                                                const float (&bs)[3], const float (&tr)[3],
                                                const LossOut& L) {
  __bf16 d[4] = {to_bf16(0.0f), to_bf16(0.0f), to_bf16(0.0f), to_bf16(0.0f)};
  double acc = 0.0;
  if (c3 == 0) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const float pred = bs[c] + s * r[c];
      const float e = (pred - tr[c]) / s;
      acc += (double)e * (double)e;
      d[c] = to_bf16(L.dy_scale * e);
    }
  }
  *(uint2*)&L.dy[p * COUT + c3] = *(const uint2*)d;
  return acc;
}

template <int EPI3>
__global__ __launch_bounds__(NBC) void k_conv23(const __bf16* __restrict__ a1, const __bf16* __restrict__ w2,
                                                const float* __restrict__ b2, const __bf16* __restrict__ w3,
                                                const float* __restrict__ b3, __bf16* __restrict__ a2_out,
                                                void* __restrict__ out, int bands,
                                                const float* __restrict__ base,
                                                const float* __restrict__ scale, LossOut L) {
  constexpr int C = CH, RW = IMG + 2;          // channels, pixels of a staged row
  constexpr int RV = RW * (C / 8);             // 16-byte vectors of one staged row
  constexpr int XS = (2 * RV + NBC - 1) / NBC;
  __shared__ __attribute__((aligned(16))) __bf16 s_w2[NTAP * C * C];
  __shared__ __attribute__((aligned(16))) __bf16 s_w3[NTAP * COUT * C];
  __shared__ __attribute__((aligned(16))) __bf16 s_a1[4 * RW * C];
  __shared__ __attribute__((aligned(16))) __bf16 s_a2[4 * RW * C];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int b = blockIdx.x / bands, band = blockIdx.x - b * bands;
  const int rows = IMG / bands, yb = band * rows, ye = yb + rows;
  stage_weights<C, C>(w2, s_w2, tid);
  stage_weights<C, COUT>(w3, s_w3, tid);
  for (int i = tid; i < 4 * RV; i += NBC) *(uint4*)&s_a2[8 * i] = make_uint4(0u, 0u, 0u, 0u);
  uint4 xr[XS];
  auto load_rows = [&](int y) {  // layer-1 rows y, y + 1 into registers
#pragma unroll
    for (int j = 0; j < XS; j++) {
      const int v = tid + j * NBC;
      xr[j] = make_uint4(0u, 0u, 0u, 0u);
      if (v < 2 * RV) {
        const int c8 = v % (C / 8), q = v / (C / 8);
        const int xx = q % RW - 1, yy = y + q / RW;
        if (yy >= 0 && yy < IMG && xx >= 0 && xx < IMG)
          xr[j] = *(const uint4*)&a1[(((size_t)b * IMG + yy) * IMG + xx) * C + 8 * c8];
      }
    }
  };
  auto put_rows = [&](int y) {
#pragma unroll
    for (int j = 0; j < XS; j++) {
      const int v = tid + j * NBC;
      if (v < 2 * RV) {
        const int c8 = v % (C / 8), q = v / (C / 8);
        const int yy = y + q / RW;
        *(uint4*)&s_a1[lds_at<C>(((yy + 4) & 3) * RW + q % RW, c8)] = xr[j];
      }
    }
  };
  // layer-1 rows yb - 2 .. yb + 1 for step 0, rows yb + 2, yb + 3 in flight
  load_rows(yb - 2);
  put_rows(yb - 2);
  load_rows(yb);
  put_rows(yb);
  load_rows(yb + 2);
  // layer 2: wave = (row r2, pixel half, channel half); layer 3: (row r3, pixel block)
  const int r2 = wave >> 2, q = wave & 3, px2 = 32 * (q & 1), nb2 = 2 * (q >> 1);
  const int px3 = 16 * q;
  const int g = lane >> 4, c2 = 16 * g + 8 * (q >> 1);  // the 8 layer-2 channels a lane holds
  const int c3 = 4 * g;                                  // the 4 layer-3 channels a lane holds
  float bb2[8], bb3[4];                                  // their biases, loaded once
#pragma unroll
  for (int k = 0; k < 8; k++) bb2[k] = b2[c2 + k];
#pragma unroll
  for (int k = 0; k < 4; k++) bb3[k] = b3[c3 + k];
  __syncthreads();
  double lsum = 0.0;  // this lane's sum of e^2 (EPI3 2)
  const int nsteps = rows / 2 + 1;
  for (int st = 0; st < nsteps; st++) {
    const int ya = yb - 1 + 2 * st;
    {
      const int y = ya + r2;  // layer-2 row of this wave
      const int row_at[3] = {((y + 3) & 3) * RW, ((y + 4) & 3) * RW, ((y + 5) & 3) * RW};
      f32x4 acc[2][2];
      conv_products<C, C, true, 2, 2>(s_a1, s_w2, row_at, px2, lane, acc, nb2);
      const bool inside = y >= 0 && y < IMG;
#pragma unroll
      for (int mb = 0; mb < 2; mb++) {
        const int px = px2 + 16 * mb + (lane & 15);
        __bf16 h[8];
#pragma unroll
        for (int nb = 0; nb < 2; nb++)
#pragma unroll
          for (int j = 0; j < 4; j++) {
            const float t = acc[mb][nb][j] + bb2[4 * nb + j];
            h[4 * nb + j] = to_bf16(inside && t > 0.0f ? t : 0.0f);
          }
        const uint4 hv = *(const uint4*)h;
        *(uint4*)&s_a2[lds_at<C>(((y + 4) & 3) * RW + px + 1, c2 >> 3)] = hv;
        if (a2_out && y >= yb && y < ye)
          *(uint4*)&a2_out[(((size_t)b * IMG + y) * IMG + px) * C + c2] = hv;
      }
    }
    __syncthreads();  // layer-2 rows ya, ya + 1 in; layer-1 rows ya - 1, ya free
    if (st + 1 < nsteps) {
      put_rows(ya + 3);
      if (st + 2 < nsteps) load_rows(ya + 5);
    }
    if (st >= 1) {
      const int y = ya - 1 + r2;  // layer-3 row of this wave
      const int row_at[3] = {((y + 3) & 3) * RW, ((y + 4) & 3) * RW, ((y + 5) & 3) * RW};
      const size_t p = ((size_t)b * IMG + y) * IMG + px3 + (lane & 15);
      // the epilogue's inputs are loaded before the products
      float bs[3] = {0.f, 0.f, 0.f}, tr[3] = {0.f, 0.f, 0.f}, sb = 0.f;
      if (EPI3 >= 2 && g == 0) {
        sb = scale[b];
#pragma unroll
        for (int k = 0; k < 3; k++) bs[k] = base[p * 3 + k];
        if (EPI3 == 2) {
#pragma unroll
          for (int k = 0; k < 3; k++) tr[k] = L.truth[p * 3 + k];
        }
      }
      f32x4 acc[1][1];
      conv_products<C, COUT, true, 1, 1, true>(s_a2, s_w3, row_at, px3, lane, acc, 0);
      if constexpr (EPI3 == 3) {
        if (g == 0) {
#pragma unroll
          for (int k = 0; k < 3; k++) ((float*)out)[p * 3 + k] = bs[k] + sb * (acc[0][0][k] + bb3[k]);
        }
      } else {
        const float rr[4] = {acc[0][0][0] + bb3[0], acc[0][0][1] + bb3[1], acc[0][0][2] + bb3[2],
                             acc[0][0][3] + bb3[3]};
        *(float4*)&((float*)out)[p * COUT + c3] = make_float4(rr[0], rr[1], rr[2], rr[3]);
        if constexpr (EPI3 == 2) lsum += loss_epilogue(rr, c3, p, sb, bs, tr, L);
      }
    }
    __syncthreads();  // layer-1 rows of the next step in; layer-3 reads of s_a2 done
  }
  if constexpr (EPI3 == 2) {
    // the workgroup's partial: lanes, then waves, in a fixed order (the
    // layer-1 ring is free after the last barrier)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o);
    double* red = (double*)s_a1;
    if (lane == 0) red[wave] = lsum;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < NBC / 64; w++) t += red[w];
      L.part[blockIdx.x] = t;
    }
  }
}

// ---------------------------------------------------------------- backward data, layers 3 + 2
// The data gradients of layers 3 and 2 in one pass (the mirror of k_conv23):
// dz2 = [a2 > 0] (dy conv w3t) (16 -> 64) and dz1 = [a1 > 0] (dz2 conv w2t)
// (64 -> 64), bf16, no bias.  Workgroup g walks the 64 / bands rows [yb, ye)
// of band g % bands of image g / bands in steps of two rows: step s makes
// dz2 rows ya, ya + 1 (ya = yb - 1 + 2 s) from dy rows ya - 1 .. ya + 2, then
// (s >= 1) dz1 rows ya - 1, ya from dz2 rows ya - 2 .. ya + 1.  dy and dz2
// live in LDS rings of four rows (row yy in slot (yy + 4) % 4, 66 pixels with
// a zero halo); dz2 rows outside the image are zero (the padding of the second
// convolution); the band's own dz2 rows are also stored (the weight gradient
// of layer 2 reads them).  Each output is the same chain of products as a
// convolution of one layer at a time, so the results are bitwise those.
__global__ __launch_bounds__(NBC) void k_back32(const __bf16* __restrict__ dy, const __bf16* __restrict__ w3t,
                                                const __bf16* __restrict__ w2t, const __bf16* __restrict__ a2,
                                                const __bf16* __restrict__ a1, __bf16* __restrict__ dz2,
                                                __bf16* __restrict__ dz1, int bands) {
  constexpr int CA = COUT, C = CH, RW = IMG + 2;   // dy channels, hidden channels, staged row
  constexpr int RV = RW * (CA / 8);                // 16-byte vectors of one staged dy row
  constexpr int XS = (2 * RV + NBC - 1) / NBC;
  __shared__ __attribute__((aligned(16))) __bf16 s_wa[NTAP * C * CA];
  __shared__ __attribute__((aligned(16))) __bf16 s_wb[NTAP * C * C];
  __shared__ __attribute__((aligned(16))) __bf16 s_dy[4 * RW * CA];
  __shared__ __attribute__((aligned(16))) __bf16 s_dz[4 * RW * C];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int b = blockIdx.x / bands, band = blockIdx.x - b * bands;
  const int rows = IMG / bands, yb = band * rows, ye = yb + rows;
  stage_weights<CA, C>(w3t, s_wa, tid);
  stage_weights<C, C>(w2t, s_wb, tid);
  for (int i = tid; i < 4 * RW * (C / 8); i += NBC) *(uint4*)&s_dz[8 * i] = make_uint4(0u, 0u, 0u, 0u);
  uint4 xr[XS];
  auto load_rows = [&](int y) {  // dy rows y, y + 1 into registers
#pragma unroll
    for (int j = 0; j < XS; j++) {
      const int v = tid + j * NBC;
      xr[j] = make_uint4(0u, 0u, 0u, 0u);
      if (v < 2 * RV) {
        const int c8 = v % (CA / 8), q = v / (CA / 8);
        const int xx = q % RW - 1, yy = y + q / RW;
        if (yy >= 0 && yy < IMG && xx >= 0 && xx < IMG)
          xr[j] = *(const uint4*)&dy[(((size_t)b * IMG + yy) * IMG + xx) * CA + 8 * c8];
      }
    }
  };
  auto put_rows = [&](int y) {
#pragma unroll
    for (int j = 0; j < XS; j++) {
      const int v = tid + j * NBC;
      if (v < 2 * RV) {
        const int c8 = v % (CA / 8), q = v / (CA / 8);
        const int yy = y + q / RW;
        *(uint4*)&s_dy[lds_at<CA>(((yy + 4) & 3) * RW + q % RW, c8)] = xr[j];
      }
    }
  };
  load_rows(yb - 2);
  put_rows(yb - 2);
  load_rows(yb);
  put_rows(yb);
  load_rows(yb + 2);
  // both convolutions: wave = (row r, pixel half, channel half), 32 x 32 outputs
  const int r = wave >> 2, q = wave & 3, px0 = 32 * (q & 1), nb0 = 2 * (q >> 1);
  const int g = lane >> 4, c0 = 16 * g + 8 * (q >> 1);  // the 8 channels a lane holds
  // a lane's mask values (8 channels of pixel px0 + 16 mb + lane % 16 of row
  // y of m), loaded before the products that they then mask
  auto mask_load = [&](uint4 (&mv)[2], const __bf16* __restrict__ m, int y) {
#pragma unroll
    for (int mb = 0; mb < 2; mb++) {
      const int px = px0 + 16 * mb + (lane & 15);
      mv[mb] = *(const uint4*)&m[(((size_t)b * IMG + y) * IMG + px) * C + c0];
    }
  };
  // masked bf16 of those 8 channels
  auto masked = [&](const f32x4 (&acc)[2][2], int mb, const uint4 (&mvs)[2]) {
    const uint4 mv = mvs[mb];
    const __bf16* me = (const __bf16*)&mv;
    __bf16 h[8];
#pragma unroll
    for (int nb = 0; nb < 2; nb++)
#pragma unroll
      for (int j = 0; j < 4; j++)
        h[4 * nb + j] = to_bf16(from_bf16(me[4 * nb + j]) > 0.0f ? acc[mb][nb][j] : 0.0f);
    return *(const uint4*)h;
  };
  __syncthreads();
  const int nsteps = rows / 2 + 1;
  for (int st = 0; st < nsteps; st++) {
    const int ya = yb - 1 + 2 * st;
    {
      const int y = ya + r;  // dz2 row of this wave
      const int row_at[3] = {((y + 3) & 3) * RW, ((y + 4) & 3) * RW, ((y + 5) & 3) * RW};
      const bool inside = y >= 0 && y < IMG;
      uint4 mv[2] = {make_uint4(0u, 0u, 0u, 0u), make_uint4(0u, 0u, 0u, 0u)};
      if (inside) mask_load(mv, a2, y);
      f32x4 acc[2][2];
      conv_products<CA, C, true, 2, 2, true>(s_dy, s_wa, row_at, px0, lane, acc, nb0);
#pragma unroll
      for (int mb = 0; mb < 2; mb++) {
        const int px = px0 + 16 * mb + (lane & 15);
        const uint4 hv = inside ? masked(acc, mb, mv) : make_uint4(0u, 0u, 0u, 0u);
        *(uint4*)&s_dz[lds_at<C>(((y + 4) & 3) * RW + px + 1, c0 >> 3)] = hv;
        if (y >= yb && y < ye) *(uint4*)&dz2[(((size_t)b * IMG + y) * IMG + px) * C + c0] = hv;
      }
    }
    __syncthreads();  // dz2 rows ya, ya + 1 in; dy rows ya - 1, ya free
    if (st + 1 < nsteps) {
      put_rows(ya + 3);
      if (st + 2 < nsteps) load_rows(ya + 5);
    }
    if (st >= 1) {
      const int y = ya - 1 + r;  // dz1 row of this wave
      const int row_at[3] = {((y + 3) & 3) * RW, ((y + 4) & 3) * RW, ((y + 5) & 3) * RW};
      uint4 mv[2];
      mask_load(mv, a1, y);
      f32x4 acc[2][2];
      conv_products<C, C, true, 2, 2, true>(s_dz, s_wb, row_at, px0, lane, acc, nb0);
#pragma unroll
      for (int mb = 0; mb < 2; mb++) {
        const int px = px0 + 16 * mb + (lane & 15);
        *(uint4*)&dz1[(((size_t)b * IMG + y) * IMG + px) * C + c0] = masked(acc, mb, mv);
      }
    }
    __syncthreads();  // dy rows of the next step in; the reads of s_dz done
  }
}

// ---------------------------------------------------------------- head
// The lift and layer 1 (16 -> 64, bias, ReLU) in one pass: workgroup
// (sample b, band) forms the sample's coarse features once, then for each of
// its 4-row tiles lifts the six staged input rows straight into LDS (zero
// outside the image) and runs conv_products on them (so a1 is bitwise what
// a separate lift and convolution would give).  It writes
// base and s, and x0 when x0 != NULL (training reads it; inference does not).
// grid: B x bands, 16 / bands tiles per workgroup.
__global__ __launch_bounds__(NBC) void k_head(const float* __restrict__ coarse,
                                              const float* __restrict__ theta, LiftWindow win, int R,
                                              const __bf16* __restrict__ w, const float* __restrict__ bias,
                                              __bf16* __restrict__ a1, __bf16* __restrict__ x0,
                                              float* __restrict__ base, float* __restrict__ scale,
                                              int bands) {
  constexpr int CI = CIN, CO = CH;
  constexpr int SR = TR + 2;
  __shared__ __attribute__((aligned(16))) __bf16 sw[NTAP * CO * CI];
  // two lifted tiles: tile t + 1 is lifted (VALU) while tile t is multiplied
  // (MFMA), one barrier per tile
  __shared__ __attribute__((aligned(16))) __bf16 sx[2][SR * (IMG + 2) * CI];
  __shared__ double red[NBC];
  extern __shared__ __attribute__((aligned(16))) float dyn[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int b = blockIdx.x / bands, band = blockIdx.x - b * bands;
  stage_weights<CI, CO>(w, sw, tid);
  float s, th;
  lift_prepare<NBC>(b, R, coarse, theta, win, dyn, dyn + 12 * R * R, red, s, th);
  const float* feat = dyn + 12 * R * R;
  if (tid == 0 && band == 0) scale[b] = s;
  const int r = wave >> 1, px0 = (wave & 1) * 32;
  const int rows = IMG / bands, ntiles = rows / TR;
  // the tile of rows y0 .. y0 + TR - 1 lifted with a row either side
  auto lift_tile = [&](int y0, __bf16* st) {
    for (int q = tid; q < SR * (IMG + 2); q += NBC) {
      const int rr = q / (IMG + 2), xx = q - rr * (IMG + 2) - 1, yy = y0 - 1 + rr;
      uint4 lo4 = make_uint4(0u, 0u, 0u, 0u), hi4 = lo4;
      if (yy >= 0 && yy < IMG && xx >= 0 && xx < IMG) {
        bf16x8 lo, hi;
        float b3[3];
        lift_pixel(feat, R, s, th, xx, yy, lo, hi, b3);
        lo4 = __builtin_bit_cast(uint4, lo);
        hi4 = __builtin_bit_cast(uint4, hi);
        if (rr >= 1 && rr <= TR) {  // the tile's own rows
          const size_t p = ((size_t)b * IMG + yy) * IMG + xx;
          float* bo = base + p * 3;
#pragma unroll
          for (int k = 0; k < 3; k++) bo[k] = b3[k];
          if (x0) {
            *(uint4*)(x0 + p * CIN) = lo4;
            *(uint4*)(x0 + p * CIN + 8) = hi4;
          }
        }
      }
      *(uint4*)&st[lds_at<CI>(q, 0)] = lo4;
      *(uint4*)&st[lds_at<CI>(q, 1)] = hi4;
    }
  };
  lift_tile(band * rows, sx[0]);
  for (int t = 0; t < ntiles; t++) {
    // tile t is lifted; the products of tile t - 1, which read the other
    // buffer, are done
    __syncthreads();
    const int y0 = band * rows + t * TR;
    if (t + 1 < ntiles) lift_tile(y0 + TR, sx[(t + 1) & 1]);
    f32x4 acc[2][CO / 16];
    const int row_at[3] = {r * (IMG + 2), (r + 1) * (IMG + 2), (r + 2) * (IMG + 2)};
    conv_products<CI, CO, false>(sx[t & 1], sw, row_at, px0, lane, acc);
    store_row<CO>(acc, b, y0 + r, px0, lane, bias, a1);
  }
}

// ---------------------------------------------------------------- weight gradient
// dW[tap][co][ci] = sum_p dz[p][co] x[p + off(tap)][ci], db[co] = sum_p dz[p][co]
// over the image rows g, g + gridDim.x, ... of logical workgroup g; one
// partial per workgroup at part + g pstride: 9 CO CI + CO values (the weights, then the
// biases: the layout of the layer's parameters), summed in a fixed order by
// k_reduce_parts.
// Nine waves, one per tap: a wave holds all (CO/16) x (CI/16) output tiles of
// its tap, so each pixel chunk's dz and x fragments are loaded from LDS once
// and used by every tile they meet (the LDS reads per product fall by the
// tile count of a row or column).
constexpr int NBW = NTAP * 64;  // threads of the weight-gradient workgroup

typedef short s16x4 __attribute__((ext_vector_type(4)));

// Row-major LDS tiles of C = 16 or 64 bf16 channels per row, laid out so that
// the transposing reads below meet no bank conflict from any first row: one
// read serves 32 lanes per cycle, rows r .. r+3 and r+8 .. r+11 at 32 bytes
// each.  Rows of 128 bytes (C = 64) swizzle their 32-byte blocks with bits 1
// and 3 of the row; rows of 32 bytes (C = 16) move 128 bytes further every
// 8 rows (measured 2304 -> 768 and 1280 -> 768 LDS cycles per 256 reads).
template <int C>
__device__ __forceinline__ int tile_at(int row, int n) {
  static_assert(C == 16 || C == 64, "tiles of 16 or 64 channels");
  if constexpr (C == 64) {
    const int h = ((row >> 1) & 1) | (((row >> 3) & 1) << 1);
    return row * 64 + (((n >> 4) ^ h) << 4) + (n & 15);
  } else {
    return row * 16 + (row >> 3) * 64 + n;
  }
}
template <int C>
constexpr int tile_elems(int rows) { return rows * C + (C == 16 ? (rows / 8 + 1) * 64 : 0); }

// A K-major MFMA fragment from such a tile: lane l receives t[r0 + 8 (l / 16)
// + e][n0 + l % 16], e = 0..7, as the eight K values of a 16x16x32 operand.
// gfx950's transposing LDS read (ds_read_b64_tr_b16) serves each group of 16
// lanes: lane j of the group names four consecutive values S[j][0..3], and
// lane i receives S[(i >> 2) + 4 r][i & 3], r = 0..3 (measured on the
// device).  So lane j points at row r + (j >> 2), columns n0 + 4 (j & 3), and
// two reads (rows r .. r+3, r+4 .. r+7) make the fragment.
template <int C>
__device__ __forceinline__ bf16x8 tr_frag(const __bf16* t, int r0, int n0, int lane) {
  const int j = lane & 15, r = r0 + 8 * (lane >> 4) + (j >> 2), n = n0 + 4 * (j & 3);
  typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
  const s16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(t + tile_at<C>(r, n)));
  const s16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(t + tile_at<C>(r + 4, n)));
  // rows r .. r+3 in elements 0..3, r+4 .. r+7 in 4..7 (native vector types
  // only: the HIP vector structs are unions and do not carry the bits)
  return __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

template <int CI, int CO>
__global__ __launch_bounds__(NBW) void k_wgrad(const __bf16* __restrict__ x, const __bf16* __restrict__ dz,
                                              float* __restrict__ part, int pstride, int n_rows, int co_used) {
  // x rows y-1 .. y+1 and the dz row staged as they lie in memory (pixel-major,
  // channels contiguous; x with a zero pixel on either side); the products read
  // both K-major (K = pixels) through tr_frag, and the tap's dx is a row offset
  constexpr int MB = CO / 16, NBT = CI / 16;        // tiles of a tap: MB x NBT
  constexpr int XW = IMG + 2;                       // staged pixels of an x row
  constexpr int XV = 3 * XW * (CI / 8);             // 8-channel vectors of the three x rows
  constexpr int DV = IMG * (CO / 8);                // 8-channel vectors of the dz row
  constexpr int XS = (XV + NBW - 1) / NBW, DS = (DV + NBW - 1) / NBW;
  // two LDS copies of the tiles: row r + 1 is staged into one while row r is
  // multiplied from the other, one barrier per row
  __shared__ __attribute__((aligned(16))) __bf16 sdz[2][tile_elems<CO>(IMG)];     // rows px
  __shared__ __attribute__((aligned(16))) __bf16 sxr[2][tile_elems<CI>(3 * XW)];  // rows dy XW + px + 1
  // the wave's tap as a scalar: the per-wave choices below are then branches
  // around whole waves (an MFMA does not honour the execution mask)
  const int tid = threadIdx.x, lane = tid & 63, tap = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int dyi = tap / 3, dxi = tap % 3;
  f32x4 acc[MB][NBT];
#pragma unroll
  for (int mb = 0; mb < MB; mb++)
#pragma unroll
    for (int nb = 0; nb < NBT; nb++) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  // bias gradient db = dz^T 1 on the matrix cores: wave w < MB takes output
  // block w, one more product per dz fragment against a B operand of ones
  f32x4 accb = {0.f, 0.f, 0.f, 0.f};
  bf16x8 ones;
#pragma unroll
  for (int e = 0; e < 8; e++) ones[e] = (__bf16)1.0f;
  // the row after the one being staged travels in registers
  uint4 xr[XS], dr[DS];
  auto load_row = [&](int row) {
    const int b = row / IMG, y = row - b * IMG;
#pragma unroll
    for (int j = 0; j < XS; j++) {
      const int v = tid + j * NBW;
      xr[j] = make_uint4(0u, 0u, 0u, 0u);
      if (v < XV) {
        const int c8 = v % (CI / 8), q = v / (CI / 8);
        const int xx = q % XW - 1, dyr = q / XW, yy = y + dyr - 1;
        if (yy >= 0 && yy < IMG && xx >= 0 && xx < IMG)
          xr[j] = *(const uint4*)&x[(((size_t)b * IMG + yy) * IMG + xx) * CI + 8 * c8];
      }
    }
#pragma unroll
    for (int j = 0; j < DS; j++) {
      const int v = tid + j * NBW;
      dr[j] = make_uint4(0u, 0u, 0u, 0u);
      if (v < DV) dr[j] = *(const uint4*)&dz[((size_t)row * IMG) * CO + 8 * v];
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int j = 0; j < XS; j++) {
      const int v = tid + j * NBW;
      if (v < XV) *(uint4*)&sxr[buf][tile_at<CI>(v / (CI / 8), 8 * (v % (CI / 8)))] = xr[j];
    }
#pragma unroll
    for (int j = 0; j < DS; j++) {
      const int v = tid + j * NBW;
      if (v < DV) *(uint4*)&sdz[buf][tile_at<CO>(v / (CO / 8), 8 * (v % (CO / 8)))] = dr[j];
    }
  };
  // workgroups are dealt to the 8 XCDs in turn; logical index g0 gives each
  // XCD a contiguous range, so the three workgroups that share an x row read
  // it through the same L2.  Partial g0 holds rows g0, g0 + gs, ... whichever
  // workgroup runs it.
  const int gs = gridDim.x;
  const int g0 = gs % 8 == 0 ? (blockIdx.x % 8) * (gs / 8) + blockIdx.x / 8 : blockIdx.x;
  if (g0 < n_rows) {
    load_row(g0);
    stage(0);
    if (g0 + gs < n_rows) load_row(g0 + gs);
  }
  __syncthreads();
  int buf = 0;
  for (int row = g0; row < n_rows; row += gs, buf ^= 1) {
    if (row + gs < n_rows) {
      stage(buf ^ 1);  // the next row; its buffer was last read before the previous barrier
      if (row + 2 * gs < n_rows) load_row(row + 2 * gs);
    }
    const __bf16* tz = sdz[buf];
    // x row dyi, pixel p + dxi - 1 sits in tile row dyi XW + p + dxi
    const __bf16* xt = sxr[buf];
    const int xr0 = dyi * XW + dxi;
#pragma unroll
    for (int kc = 0; kc < IMG / 32; kc++) {
      bf16x8 a[MB], bv[NBT];
#pragma unroll
      for (int mb = 0; mb < MB; mb++) a[mb] = tr_frag<CO>(tz, 32 * kc, 16 * mb, lane);
#pragma unroll
      for (int nb = 0; nb < NBT; nb++) bv[nb] = tr_frag<CI>(xt, xr0 + 32 * kc, 16 * nb, lane);
#pragma unroll
      for (int mb = 0; mb < MB; mb++)
#pragma unroll
        for (int nb = 0; nb < NBT; nb++)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mb], bv[nb], acc[mb][nb], 0, 0, 0);
#pragma unroll
      for (int mb = 0; mb < MB; mb++)
        if (tap == mb) accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mb], ones, accb, 0, 0, 0);
    }
    __syncthreads();  // this row's reads done; the next row's tiles are in
  }
  float* pg = part + (size_t)g0 * pstride;
#pragma unroll
  for (int mb = 0; mb < MB; mb++)
#pragma unroll
    for (int nb = 0; nb < NBT; nb++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int co = 16 * mb + 4 * (lane >> 4) + i, ci = 16 * nb + (lane & 15);
        if (co < co_used) pg[((size_t)tap * CO + co) * CI + ci] = acc[mb][nb][i];
      }
  // every column of accb holds the sums; lanes of column 0 store them
  if (tap < MB && (lane & 15) == 0) {
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int co = 16 * tap + 4 * (lane >> 4) + i;
      if (co < co_used) pg[NTAP * CO * CI + co] = accb[i];
    }
  }
}

// Output channels of a layer that only pad its tile (the last layer's
// channels past the used ones): zero weights and biases with zero gradients,
// which the weight-gradient kernel does not store and the reduction skips.
// Weights at w_off, [tap][co][ci]; biases at b_off; channels used .. co - 1.
struct PadRows {
  int w_off, b_off, co, ci, used;
  __device__ bool skips(int i) const {
    if (i >= w_off && i < w_off + NTAP * co * ci) return ((i - w_off) / ci) % co >= used;
    return i >= b_off + used && i < b_off + co;
  }
};

// out[s][i] = sum of part[g][i] over the s-th of gridDim.y equal ranges of g,
// in increasing g (fixed order), i < n; with gridDim.y = 1 the full sum.
// Entries pad.skips(i) are not read and keep their zero in out.
__global__ void k_reduce_parts(const float* __restrict__ part, int n_parts, int n,
                               float* __restrict__ out, PadRows pad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || pad.skips(i)) return;
  const int per = (n_parts + gridDim.y - 1) / gridDim.y;
  const int g0 = blockIdx.y * per, g1 = min(n_parts, g0 + per);
  float s = 0.0f;
  // unrolled so that the loads are in flight together; the sum stays in
  // increasing g
#pragma unroll 8
  for (int g = g0; g < g1; g++) s += part[(size_t)g * n + i];
  out[(size_t)blockIdx.y * n + i] = s;
}

// u = base + s r for channels 0..2: out [B][64][64][3]
__global__ void k_combine(const float* __restrict__ r, const float* __restrict__ base,
                          const float* __restrict__ scale, int n_px, float* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_px) return;
  const float s = scale[p / (IMG * IMG)];
#pragma unroll
  for (int c = 0; c < 3; c++) out[(size_t)p * 3 + c] = base[(size_t)p * 3 + c] + s * r[(size_t)p * COUT + c];
}

// ---------------------------------------------------------------- parameters
// Adam (Kingma and Ba) on the FP32 master parameters, bias-corrected with
// step t: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps); g is the sum of
// the nseg range sums seg[s][i] in increasing s, as k_reduce_parts takes it
struct PrepLayers {
  const float* w[3];
  __bf16* wf[3];
  __bf16* wt[3];
  int co[3], ci[3];
  int off[3];  // offset of each layer's weights in the parameter vector
};

// The bf16 copies of weight i of layer l ([tap][co][ci]): the forward copy
// in the same layout, and the backward-data copy with the tap mirrored and
// co/ci exchanged.
__device__ __forceinline__ void put_weight_copies(const PrepLayers& L, int l, int i, float w) {
  const int co_n = L.co[l], ci_n = L.ci[l];
  const int tap = i / (co_n * ci_n), rem = i - tap * co_n * ci_n;
  const int co = rem / ci_n, ci = rem - co * ci_n;
  const __bf16 h = to_bf16(w);
  L.wf[l][i] = h;
  L.wt[l][((size_t)(NTAP - 1 - tap) * ci_n + ci) * co_n + co] = h;
}

// The weight gradient summed from the partials and one Adam step of each
// parameter, with the bf16 copies of the updated weights (the biases stay
// FP32), so the next forward pass needs no preparation.  One pass: a
// workgroup of 1024 threads takes 64 parameters (a wave reads 64 consecutive
// values of a partial); thread (s, j)
// sums range s of the 16 equal ranges of partials of parameter j in
// increasing order (the first stage of k_reduce_parts), and thread j the 16
// range sums in increasing order (its second stage), so the gradient is
// bitwise the two-launch reduction's.  pad.skips(i): a zero gradient.
constexpr int ADAM_RANGES = 16;
constexpr int ADAM_PARAMS = 64;  // parameters per workgroup of k_adam_parts
__global__ __launch_bounds__(ADAM_RANGES * ADAM_PARAMS) void k_adam_parts(const float* __restrict__ part, int n_parts, int n,
                                                    PadRows pad, float* __restrict__ p, float* __restrict__ m,
                                                    float* __restrict__ v, float lr, float b1, float b2,
                                                    float eps, float c1, float c2, PrepLayers L) {
  __shared__ float rs[ADAM_RANGES][ADAM_PARAMS];
  const int j = threadIdx.x % ADAM_PARAMS, sg = threadIdx.x / ADAM_PARAMS;
  const int i = blockIdx.x * ADAM_PARAMS + j;
  float sum = 0.0f;
  if (i < n && !pad.skips(i)) {
    const int per = (n_parts + ADAM_RANGES - 1) / ADAM_RANGES, g0 = sg * per, g1 = min(n_parts, g0 + per);
#pragma unroll 8
    for (int g = g0; g < g1; g++) sum += part[(size_t)g * n + i];
  }
  rs[sg][j] = sum;
  __syncthreads();
  if (threadIdx.x >= ADAM_PARAMS || i >= n) return;
  float gi = 0.0f;
#pragma unroll
  for (int s = 0; s < ADAM_RANGES; s++) gi += rs[s][j];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
#pragma unroll
  for (int l = 0; l < 3; l++) {
    const int k = i - L.off[l];
    if (k >= 0 && k < NTAP * L.co[l] * L.ci[l]) put_weight_copies(L, l, k, pi);
  }
}

// The bf16 copies of every weight (after the parameters are set).
__global__ void k_prep_weights(PrepLayers L) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int l = 0;
  while (l < 3 && i >= NTAP * L.co[l] * L.ci[l]) {
    i -= NTAP * L.co[l] * L.ci[l];
    l++;
  }
  if (l == 3) return;
  put_weight_copies(L, l, i, L.w[l][i]);
}

}  // namespace lbnet

