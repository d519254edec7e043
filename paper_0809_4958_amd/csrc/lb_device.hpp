// lb_device.hpp -- device-side data structures and per-node arithmetic of the
// fine-box lattice-Boltzmann step for gfx950.
//
// Everything is computed on deviations from rest equilibrium, d_i = f_i - w_i rho0
// (FP64 in FP64 mode, FP32 otherwise), so that the O(w_i) rest part never enters
// the rounding of the O(w_i u) signal.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbdev {

constexpr int Q = 19;
// D3Q19 directions (standard model, Sec. 3); opposite directions adjacent.
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
// opposite direction: c_OPP[i] = -c_i
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
// weight class: 0 rest (1/3), 1 axis (1/18), 2 diagonal (1/36)
constexpr int WCLS[Q] = {0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2};
constexpr double WD[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};

// Weighted-orthogonal MRT basis polynomials e_k(c) (Duenweg-Schiller-Ladd),
// evaluated at compile time; k = 0 mass, 1-3 momentum, 4 bulk, 5-9 shear,
// 10-18 ghosts.
__host__ __device__ constexpr int basis(int k, int cx, int cy, int cz) {
  const int c2 = cx * cx + cy * cy + cz * cz;
  switch (k) {
    case 0: return 1;
    case 1: return cx;
    case 2: return cy;
    case 3: return cz;
    case 4: return c2 - 1;
    case 5: return 3 * cx * cx - c2;
    case 6: return cy * cy - cz * cz;
    case 7: return cx * cy;
    case 8: return cy * cz;
    case 9: return cx * cz;
    case 10: return (3 * c2 - 5) * cx;
    case 11: return (3 * c2 - 5) * cy;
    case 12: return (3 * c2 - 5) * cz;
    case 13: return (cy * cy - cz * cz) * cx;
    case 14: return (cz * cz - cx * cx) * cy;
    case 15: return (cx * cx - cy * cy) * cz;
    case 16: return 3 * c2 * c2 - 6 * c2 + 1;
    case 17: return (2 * c2 - 3) * (3 * cx * cx - c2);
    default: return (2 * c2 - 3) * (cy * cy - cz * cz);
  }
}
// b_k = sum_i w_i e_k(c_i)^2, as exact numerator over 36
__host__ __device__ constexpr int norm36(int k) {
  int s = 0;
  for (int i = 0; i < Q; i++) {
    const int w36 = WCLS[i] == 0 ? 12 : (WCLS[i] == 1 ? 2 : 1);
    const int e = basis(k, CX[i], CY[i], CZ[i]);
    s += w36 * e * e;
  }
  return s;
}

// 1/b_k of the basis; the compile-time checks tie them to the polynomials
constexpr double INVB[Q] = {1.0, 3.0, 3.0, 3.0, 1.5, 0.75, 2.25, 9.0, 9.0, 9.0,
                            1.5, 1.5, 1.5, 4.5, 4.5, 4.5, 0.5, 0.75, 2.25};
__host__ __device__ constexpr bool invb_consistent() {
  for (int k = 0; k < Q; k++)
    if (INVB[k] * norm36(k) != 36.0) return false;
  return true;
}
static_assert(invb_consistent(), "1/b_k table does not match the basis norms");
__host__ __device__ constexpr bool basis_orthogonal() {
  for (int k = 0; k < Q; k++)
    for (int l = 0; l < k; l++) {
      int s = 0;
      for (int i = 0; i < Q; i++)
        s += (WCLS[i] == 0 ? 12 : (WCLS[i] == 1 ? 2 : 1)) * basis(k, CX[i], CY[i], CZ[i]) *
             basis(l, CX[i], CY[i], CZ[i]);
      if (s != 0) return false;
    }
  return true;
}
static_assert(basis_orthogonal(), "MRT basis is not weighted-orthogonal");

enum : int { ITEM_TILE = 0, ITEM_BOUNDARY = 1, ITEM_ROWS = 2, ITEM_FACE_ROWS = 3 };
constexpr int MAX_RECT = 12;

struct BoxDesc {
  int64_t off;          // element offset of pop[0] of this box in each population arena
  int64_t nn;           // nodes (boundary layer included)
  int nx, ny, nz, pmask;
  int bc_mode;          // 0 affine, 1 sampled, -1 none
  int bc_dt, bc_ns, bc_res;
  int64_t bc_t0;
  const void* bc;       // affine: double [ns][9]; sampled: R [ns][6][res][res][3]; learned: float ring
  int chain_first, chain_count;
  int nbnd;             // boundary nodes enumerated by boundary items
  int n_rect;           // boundary rectangles (a face, or part of one)
  int rect_face[MAX_RECT];      // face of the rectangle's nodes (-x,+x,-y,+y,-z,+z)
  int rect_cnt[MAX_RECT];       // nodes in the rectangle
  int rect_start[MAX_RECT][3];  // first node coordinate along x, y, z
  int rect_len[MAX_RECT][3];    // extent along x, y, z
  float dec[3];         // FP16 decode factor per weight class: w 2^-s
  float enc[3];         // FP16 encode factor per weight class: 2^s / w
  float s2;             // FP16 scale 2^s
  double interior;      // number of interior nodes
  int fast;             // non-periodic and 19*nn*sizeof(T) < 2^32 (32-bit offsets)
  int vec;              // interior rows handled as lane vectors (ITEM_ROWS) incl. the x-face nodes
  int ylog;             // log2 of the rows interleaved per population row (see aidx)
  int vw;               // row boxes: 32-bit words per lane vector (2 or 3)
  int xf_off;           // row boxes: first float of the box's x-face velocities, else -1
  int index;            // the box's index (random-number counters)
  int body_dt, body_ns; // accelerated-frame body force: samples every body_dt steps
  int64_t body_t0;      // step of the first sample
  const double* body;   // tracer acceleration [body_ns][3] (lattice units), NULL = none
};

struct Item {
  int box, kind;
  int x0, y0, z0;       // tile origin (node coordinates)
  int ex, ey, ez;       // tile extents; boundary: x0 = first boundary node, ex = count
};

struct ChainDesc {
  int box, first, nb, substeps, fix_com;
  int bead0;            // index of the chain's first bead among its box's beads
  double zeta, mass, fene_k, fene_r0;
  double decay;         // exp(-zeta h / mass), h = 1/substeps
  double kick;          // Langevin velocity kick sqrt(kT/m (1 - exp(-2 zeta h/m))), 0 at kT = 0
  int ai[3];            // integer part of the anchor
  double af[3];         // fractional part of the anchor
};

struct DevState {
  long long step;       // time index n of the current state
  int err_key;          // 0x7fffffff when no error; else min over (owner << 4 | code index)
  int tickets;          // k_force workgroups finished in the current step (0 between steps)
  long long pad2;
};

constexpr int ERR_NONE = 0x7fffffff;
enum : int { EC_BEAD_OUT = 1, EC_FENE = 2, EC_UNSTABLE = 3 };

// Stores of the step in FP16 round stochastically.  Rounded to nearest, a
// population that changes by less than an FP16 ulp per step keeps the same
// rounding error, of the same sign, step after step, and at neighbouring
// nodes alike; these errors feed the slow hydrodynamic modes coherently and
// grow with the flow's viscous time (u off by 6e-3 of its norm after 5,000
// steps of a 64^3 box of the batched workload, 1.3e-2 at 96^3).  Rounding up
// with probability equal to the fraction of an ulp makes every store's
// error zero-mean and independent from step to step, and the accumulation
// stops (an FP64 emulation of the same box: 1.9e-4, flat from step 100 on).
// The rounding is gfx950's v_cvt_sr_f16_f32: the top 13 bits of a random
// word are added below the last bit FP16 keeps and the rest is cut, so that
// a value rounds up with probability equal to its fraction of an FP16 ulp
// (subnormals included; rates checked on the device).  The random word of a
// store comes from a counter: the node's linear index in its box and the
// step index, mixed by the 32-bit MurmurHash3 finaliser (Appleby), plus a
// Weyl increment per direction.  The state upload and the re-layout of a
// checkpoint round to nearest (exact values there).
__device__ __forceinline__ unsigned dither_node(unsigned node, unsigned step) {
  unsigned h = node * 0x9E3779B1u + step * 0x85EBCA77u;
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}
__device__ __forceinline__ unsigned dither_pop(unsigned h, int i) {
  return h + (unsigned)i * 0x9E3779B9u;
}

typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));

template <int S> struct Store;
template <> struct Store<0> {
  using T = double;   // storage
  using R = double;   // compute
  __device__ static R dec(T v, float) { return v; }
  __device__ static T enc(R v, float) { return v; }
  __device__ static T enc(R v, float, unsigned) { return v; }
  __device__ static T keep(R v, unsigned) { return v; }
};
template <> struct Store<1> {
  using T = float;
  using R = float;
  __device__ static R dec(T v, float) { return v; }
  __device__ static T enc(R v, float) { return v; }
  __device__ static T enc(R v, float, unsigned) { return v; }
  __device__ static T keep(R v, unsigned) { return v; }
};
template <> struct Store<2> {
  using T = _Float16;
  using R = float;
  // product rounded to FP32 in both directions, never fused into a
  // neighbouring add or conversion: every kernel (pulled or in-place reads,
  // state upload, readout) then decodes and encodes a value identically
  __device__ static R dec(T v, float k) {
#pragma clang fp contract(off)
    return (float)v * k;
  }
  // round to nearest (state upload, re-layout)
  __device__ static T enc(R v, float k) {
#pragma clang fp contract(off)
    return (_Float16)(v * k);
  }
  // stochastic rounding with the random word r (top 13 bits used)
  __device__ static T enc(R v, float k, unsigned r) {
#pragma clang fp contract(off)
    const float x = v * k;
    h16x2 o = {};
    o = __builtin_amdgcn_cvt_sr_f16_f32(o, x, r, false);
    return o[0];
  }
  // a value the collision already produced in storage units, (f/w - rho0) 2^s
  __device__ static T keep(R x, unsigned r) {
    h16x2 o = {};
    o = __builtin_amdgcn_cvt_sr_f16_f32(o, x, r, false);
    return o[0];
  }
  // the same into a packed pair: with fresh, the low half starts a new word
  // (the high half follows); otherwise the other half is kept
  __device__ static void keep_into(unsigned& word, bool hi, R x, unsigned r, bool fresh) {
    if (hi || !fresh) {
      h16x2 o = __builtin_bit_cast(h16x2, word);
      o = hi ? __builtin_amdgcn_cvt_sr_f16_f32(o, x, r, true)
             : __builtin_amdgcn_cvt_sr_f16_f32(o, x, r, false);
      word = __builtin_bit_cast(unsigned, o);
    } else {
      h16x2 o = {};
      o = __builtin_amdgcn_cvt_sr_f16_f32(o, x, r, false);
      word = __builtin_bit_cast(unsigned, o);
    }
  }
};

template <typename R>
__device__ __forceinline__ R wgt(int i) { return (R)WD[WCLS[i]]; }

// w_c x without the bias of a rounded weight.  In FP32 the weights 1/3, 1/18
// and 1/36 round up by 3.0e-8, 7.5e-9 and 7.5e-9 of themselves: multiplied
// into every post-collision population, that same-signed factor would scale
// the conserved mass and momentum on every step and build up over the flow's
// relaxation time (1e-5 of the velocity over 10^4 steps of a 128^3 box).  The
// residual w_c - (float)w_c, added by a fused multiply-add, cancels it (CW:
// FP32 storage).  In FP64 the weights' rounding (1e-17) is left alone, and in
// FP16 storage the half-precision rounding of every stored value (2^-11) is
// far larger than the bias, so the step keeps the plain product there.
constexpr float WF[3] = {(float)WD[0], (float)WD[1], (float)WD[2]};
constexpr float WLO[3] = {(float)(WD[0] - (double)WF[0]), (float)(WD[1] - (double)WF[1]),
                          (float)(WD[2] - (double)WF[2])};
template <typename R, bool CW>
__host__ __device__ __forceinline__ constexpr R wmul(int c, R x) {
  if constexpr (CW && sizeof(R) == 4) {
    return __builtin_fmaf(x, WF[c], x * WLO[c]);
  } else {
    return (R)WD[c] * x;
  }
}

// 1/rho: exact division in FP64, the hardware reciprocal (1 ulp) in FP32
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Equilibrium deviation f_eq_i(rho, u) - w_i rho0 = w_i [drho + rho(3 cu + 9/2 cu^2 - 3/2 u^2)]
template <typename R, bool CW = false>
__device__ __forceinline__ void eq_dev(R drho, R rho, R ux, R uy, R uz, R out[Q]) {
  const R uu = ux * ux + uy * uy + uz * uz;
  const R base = drho - (R)1.5 * rho * uu;
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const R cu = (R)CX[i] * ux + (R)CY[i] * uy + (R)CZ[i] * uz;
    out[i] = wmul<R, CW>(WCLS[i], base + rho * cu * ((R)3.0 + (R)4.5 * cu));
  }
}

// Collision of one node in deviation form.  d[] in: pre-collision deviations,
// out: post-collision deviations.  g: force density of this step.
template <typename R, int COLL, bool CW = false>
__device__ __forceinline__ void collide(R d[Q], R gx, R gy, R gz, R rho0, R omega, R om_bulk,
                                        R om_ghost) {
  R drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 0; i < Q; i++) {
    drho += d[i];
    if (CX[i]) jx += (R)CX[i] * d[i];
    if (CY[i]) jy += (R)CY[i] * d[i];
    if (CZ[i]) jz += (R)CZ[i] * d[i];
  }
  const R rho = rho0 + drho;
  const R inv = (R)1 / rho;
  const R ux = (jx + (R)0.5 * gx) * inv;
  const R uy = (jy + (R)0.5 * gy) * inv;
  const R uz = (jz + (R)0.5 * gz) * inv;
  if (COLL == 0) {
    // BGK with Guo forcing
    R eq[Q];
    eq_dev<R, CW>(drho, rho, ux, uy, uz, eq);
    const R ug = ux * gx + uy * gy + uz * gz;
    const R fpre = (R)1 - (R)0.5 * omega;
#pragma unroll
    for (int i = 0; i < Q; i++) {
      const R cu = (R)CX[i] * ux + (R)CY[i] * uy + (R)CZ[i] * uz;
      const R cg = (R)CX[i] * gx + (R)CY[i] * gy + (R)CZ[i] * gz;
      const R F = wmul<R, CW>(WCLS[i], (R)3 * (cg - ug) + (R)9 * cu * cg);
      d[i] = d[i] - omega * (d[i] - eq[i]) + fpre * F;
    }
  } else {
    // MRT: moments of the deviations (equal to those of f for k >= 1)
    R m[Q];
#pragma unroll
    for (int k = 4; k < Q; k++) {
      R s = 0;
#pragma unroll
      for (int i = 0; i < Q; i++) {
        const int e = basis(k, CX[i], CY[i], CZ[i]);
        if (e == 1) s += d[i];
        else if (e == -1) s -= d[i];
        else if (e != 0) s += (R)e * d[i];
      }
      m[k] = s;
    }
    // equilibrium moments of f_eq(rho, u) and forcing moments of (u g + g u)
    const R uu = ux * ux + uy * uy + uz * uz;
    const R ug = ux * gx + uy * gy + uz * gz;
    R meq[10], mf[10];
    meq[4] = rho * uu;
    meq[5] = rho * ((R)3 * ux * ux - uu);
    meq[6] = rho * (uy * uy - uz * uz);
    meq[7] = rho * ux * uy;
    meq[8] = rho * uy * uz;
    meq[9] = rho * ux * uz;
    mf[4] = (R)2 * ug;
    mf[5] = (R)2 * ((R)3 * ux * gx - ug);
    mf[6] = (R)2 * (uy * gy - uz * gz);
    mf[7] = ux * gy + uy * gx;
    mf[8] = uy * gz + uz * gy;
    mf[9] = ux * gz + uz * gx;
    R ms[Q];
    ms[0] = drho;
    ms[1] = jx + gx;
    ms[2] = jy + gy;
    ms[3] = jz + gz;
    {
      const R gb = (R)1 - om_bulk;
      ms[4] = meq[4] + gb * (m[4] - meq[4]) + (R)0.5 * ((R)1 + gb) * mf[4];
      const R gs = (R)1 - omega;
      const R hs = (R)0.5 * ((R)1 + gs);
#pragma unroll
      for (int k = 5; k < 10; k++) ms[k] = meq[k] + gs * (m[k] - meq[k]) + hs * mf[k];
      const R gg = (R)1 - om_ghost;
#pragma unroll
      for (int k = 10; k < Q; k++) ms[k] = gg * m[k];
    }
#pragma unroll
    for (int k = 0; k < Q; k++) ms[k] *= (R)INVB[k];
    // back transform f_i = w_i sum_k e_k(c_i) ms_k
#pragma unroll
    for (int i = 0; i < Q; i++) {
      R s = 0;
#pragma unroll
      for (int k = 0; k < Q; k++) {
        const int e = basis(k, CX[i], CY[i], CZ[i]);
        if (e == 1) s += ms[k];
        else if (e == -1) s -= ms[k];
        else if (e != 0) s += (R)e * ms[k];
      }
      d[i] = wmul<R, CW>(WCLS[i], s);
    }
  }
}

// ---------------------------------------------------------------------------
// Thermal fluctuations.  Counter-based random numbers: Philox4x32-10 (Salmon,
// Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC
// 2011) -- ten rounds of two 32 x 32 -> 64-bit products mixed into the 128-bit
// counter under a 64-bit key bumped by the Weyl constants -- and the map of
// 32 random bits to a uniform number on (-sqrt 3, sqrt 3), mean 0, variance 1.
__device__ __forceinline__ void philox4x32(unsigned (&c)[4], unsigned k0, unsigned k1) {
#pragma unroll
  for (int r = 0; r < 10; r++) {
    // each product whole (one v_mad_u64_u32, not a low and a high multiply)
    const unsigned long long p0 = (unsigned long long)0xD2511F53u * c[0];
    const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c[2];
    const unsigned lo0 = (unsigned)p0, hi0 = (unsigned)(p0 >> 32);
    const unsigned lo1 = (unsigned)p1, hi1 = (unsigned)(p1 >> 32);
    const unsigned n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ double unit_uniform(unsigned u) {
  return ((double)u - 2147483647.5) * (1.7320508075688772 / 2147483648.0);
}

// What a node's collision adds to the plain step: the accelerated-frame force
// density -rho a (Sec. 2) and, when mu = 3 kT > 0, the fluctuating collision;
// its random numbers come from the Philox counter (node, box, step, draw 0..3).
template <typename R>
struct Ext {
  R ax, ay, az;
  R mu;
  unsigned k0, k1;
  unsigned node, box, step;
};

// the 16 unit-variance numbers of a node (modes 4..18 use the first 15)
template <typename R>
__device__ __forceinline__ void mode_noise(const Ext<R>& e, R (&r)[16]) {
#pragma unroll
  for (unsigned dd = 0; dd < 4; dd++) {
    unsigned c[4] = {e.node, e.box, e.step, dd};
    philox4x32(c, e.k0, e.k1);
#pragma unroll
    for (int q = 0; q < 4; q++) r[4 * dd + q] = (R)unit_uniform(c[q]);
  }
}

// ---------------------------------------------------------------------------
// MRT in pair form.  Directions come in opposite pairs (2p-1, 2p), p = 1..9,
// with representative velocities (1,0,0) (0,1,0) (0,0,1) (1,1,0) (1,-1,0)
// (1,0,1) (1,0,-1) (0,1,1) (0,1,-1).  Even basis polynomials see the pair sum
// s_p = d_{2p-1} + d_{2p}, odd ones the difference a_p = d_{2p-1} - d_{2p}, and
// the moments of the weighted-orthogonal basis share partial sums; the
// compile-time checks below tie these hand-written transforms to basis().
template <typename R>
__host__ __device__ constexpr void mrt_forward(const R d[Q], R m[Q]) {
  R s[10] = {}, a[10] = {};
  for (int p = 1; p <= 9; p++) {
    s[p] = d[2 * p - 1] + d[2 * p];
    a[p] = d[2 * p - 1] - d[2 * p];
  }
  const R Sa = s[1] + s[2] + s[3];
  const R Sd = s[4] + s[5] + s[6] + s[7] + s[8] + s[9];
  m[0] = d[0] + Sa + Sd;
  const R Ax = a[4] + a[5] + a[6] + a[7];
  const R Ay = a[4] - a[5] + a[8] + a[9];
  const R Az = a[6] - a[7] + a[8] - a[9];
  m[1] = a[1] + Ax;
  m[2] = a[2] + Ay;
  m[3] = a[3] + Az;
  m[4] = Sd - d[0];
  const R X = (s[1] + s[1]) - s[2] - s[3];
  const R Y = (s[4] + s[5] + s[6] + s[7]) - (s[8] + s[9]) - (s[8] + s[9]);
  m[5] = X + Y;
  m[17] = Y - X;
  const R P = s[2] - s[3];
  const R Rr = s[4] + s[5] - s[6] - s[7];
  m[6] = P + Rr;
  m[18] = Rr - P;
  m[7] = s[4] - s[5];
  m[8] = s[8] - s[9];
  m[9] = s[6] - s[7];
  m[16] = d[0] - Sa - Sa + Sd;
  m[10] = Ax - a[1] - a[1];
  m[11] = Ay - a[2] - a[2];
  m[12] = Az - a[3] - a[3];
  m[13] = a[4] + a[5] - a[6] - a[7];
  m[14] = a[5] - a[4] + a[8] + a[9];
  m[15] = a[6] - a[7] - a[8] + a[9];
}

// Back transform of moments already divided by b_k: d_i = w_i sum_k e_k(c_i) M_k.
// GZ: the nine ghost moments are zero (not read).  WS: d_i / w_i scaled by sc
// (the FP16 storage units) instead: the weights of the transform and the
// storage's 1/w_i cancel, and the stored value needs no product of its own.
template <typename R, bool GZ, bool CW = false, bool WS = false>
__host__ __device__ constexpr void mrt_backward(const R M[Q], R d[Q], R sc = R(1)) {
  auto wout = [&](int c, R x) -> R {
    if constexpr (WS) return x * sc;
    else return wmul<R, CW>(c, x);
  };
  const R g10 = GZ ? R(0) : M[10], g11 = GZ ? R(0) : M[11], g12 = GZ ? R(0) : M[12];
  const R g13 = GZ ? R(0) : M[13], g14 = GZ ? R(0) : M[14], g15 = GZ ? R(0) : M[15];
  const R g16 = GZ ? R(0) : M[16], g17 = GZ ? R(0) : M[17], g18 = GZ ? R(0) : M[18];
  d[0] = wout(0, M[0] - M[4] + g16);
  const R E1 = M[0] + (M[5] + M[5]) - (g16 + g16) - (g17 + g17);
  const R O1 = M[1] - (g10 + g10);
  const R E2 = M[0] - M[5] + M[6] - (g16 + g16) + g17 - g18;
  const R O2 = M[2] - (g11 + g11);
  const R E3 = M[0] - M[5] - M[6] - (g16 + g16) + g17 + g18;
  const R O3 = M[3] - (g12 + g12);
  const R Bd = M[0] + M[4] + g16;           // common to the six diagonal pairs
  const R C45 = Bd + M[5] + M[6] + g17 + g18;
  const R C67 = Bd + M[5] - M[6] + g17 - g18;
  const R C89 = Bd - (M[5] + M[5]) - (g17 + g17);
  const R E4 = C45 + M[7], E5 = C45 - M[7];
  const R E6 = C67 + M[9], E7 = C67 - M[9];
  const R E8 = C89 + M[8], E9 = C89 - M[8];
  const R x10 = M[1] + g10, y11 = M[2] + g11, z12 = M[3] + g12;
  const R O4 = x10 + y11 + g13 - g14;
  const R O5 = x10 - y11 + g13 + g14;
  const R O6 = x10 + z12 - g13 + g15;
  const R O7 = x10 - z12 - g13 - g15;
  const R O8 = y11 + z12 + g14 - g15;
  const R O9 = y11 - z12 + g14 + g15;
  d[1] = wout(1, E1 + O1);
  d[2] = wout(1, E1 - O1);
  d[3] = wout(1, E2 + O2);
  d[4] = wout(1, E2 - O2);
  d[5] = wout(1, E3 + O3);
  d[6] = wout(1, E3 - O3);
  d[7] = wout(2, E4 + O4);
  d[8] = wout(2, E4 - O4);
  d[9] = wout(2, E5 + O5);
  d[10] = wout(2, E5 - O5);
  d[11] = wout(2, E6 + O6);
  d[12] = wout(2, E6 - O6);
  d[13] = wout(2, E7 + O7);
  d[14] = wout(2, E7 - O7);
  d[15] = wout(2, E8 + O8);
  d[16] = wout(2, E8 - O8);
  d[17] = wout(2, E9 + O9);
  d[18] = wout(2, E9 - O9);
}

__host__ __device__ constexpr bool pair_forward_matches_basis() {
  for (int i = 0; i < Q; i++) {
    double d[Q] = {}, m[Q] = {};
    d[i] = 1.0;
    mrt_forward<double>(d, m);
    for (int k = 0; k < Q; k++)
      if (m[k] != (double)basis(k, CX[i], CY[i], CZ[i])) return false;
  }
  return true;
}
__host__ __device__ constexpr bool pair_backward_matches_basis() {
  for (int k = 0; k < Q; k++) {
    double M[Q] = {}, d[Q] = {};
    M[k] = 1.0;
    mrt_backward<double, false>(M, d);
    for (int i = 0; i < Q; i++) {
      const double want = WD[WCLS[i]] * basis(k, CX[i], CY[i], CZ[i]);
      const double diff = d[i] - want;
      if (diff > 1e-15 || diff < -1e-15) return false;
    }
  }
  return true;
}
static_assert(pair_forward_matches_basis(), "pair-form forward transform != basis");
static_assert(pair_backward_matches_basis(), "pair-form back transform != basis");

// MRT collision in pair form on deviations (moments of d equal those of f for
// k >= 1; m_0 is the density deviation).  GZ: ghost relaxation rate 1.
// NOISE: the fluctuating collision (Duenweg, Schiller and Ladd): every relaxed
// mode k >= 4 gains sqrt(mu rho b_k (1 - gamma_k^2)) r_k, which keeps its
// fluctuations at the equilibrium variance mu rho b_k (mu = 3 kT); the ghosts
// are then formed whatever GZ says.
template <typename R, bool GZ, bool NOISE = false, bool CW = false, bool WS = false>
__device__ __forceinline__ void collide_mrt_pairs(R d[Q], R gx, R gy, R gz, R rho0, R omega,
                                                  R om_bulk, R om_ghost,
                                                  const Ext<R>* ext = nullptr, R sc = R(1)) {
  R m[Q];
  mrt_forward<R>(d, m);
  const R drho = m[0];
  const R rho = rho0 + drho;
  const R inv = recip(rho);
  const R ux = (m[1] + (R)0.5 * gx) * inv;
  const R uy = (m[2] + (R)0.5 * gy) * inv;
  const R uz = (m[3] + (R)0.5 * gz) * inv;
  const R uu = ux * ux + uy * uy + uz * uz;
  const R ug = ux * gx + uy * gy + uz * gz;
  R M[Q];
  M[0] = drho;
  M[1] = (m[1] + gx) * (R)3;
  M[2] = (m[2] + gy) * (R)3;
  M[3] = (m[3] + gz) * (R)3;
  const R gb = (R)1 - om_bulk, hb = (R)0.5 * ((R)1 + gb);
  const R gs = (R)1 - omega, hs = (R)0.5 * ((R)1 + gs);
  {
    const R eq = rho * uu;
    M[4] = (eq + gb * (m[4] - eq) + hb * ((R)2 * ug)) * (R)1.5;
  }
  {
    const R eq = rho * ((R)3 * ux * ux - uu);
    M[5] = (eq + gs * (m[5] - eq) + hs * ((R)2 * ((R)3 * ux * gx - ug))) * (R)0.75;
  }
  {
    const R eq = rho * (uy * uy - uz * uz);
    M[6] = (eq + gs * (m[6] - eq) + hs * ((R)2 * (uy * gy - uz * gz))) * (R)2.25;
  }
  {
    const R eq = rho * ux * uy;
    M[7] = (eq + gs * (m[7] - eq) + hs * (ux * gy + uy * gx)) * (R)9;
  }
  {
    const R eq = rho * uy * uz;
    M[8] = (eq + gs * (m[8] - eq) + hs * (uy * gz + uz * gy)) * (R)9;
  }
  {
    const R eq = rho * ux * uz;
    M[9] = (eq + gs * (m[9] - eq) + hs * (ux * gz + uz * gx)) * (R)9;
  }
  if constexpr (NOISE) {
    const R gg = (R)1 - om_ghost;
#pragma unroll
    for (int k = 10; k < Q; k++) M[k] = GZ ? (R)0 : gg * m[k] * (R)INVB[k];
    R r[16];
    mode_noise<R>(*ext, r);
    const R mr = ext->mu * rho;
    const R ab = sqrt(mr * ((R)1 - gb * gb)), as = sqrt(mr * ((R)1 - gs * gs)),
            ag = sqrt(mr * ((R)1 - gg * gg));
    // noise of mode k, divided by b_k like the relaxed moments: a r_k / sqrt(b_k)
    M[4] += ab * r[0] * (R)sqrt(INVB[4]);
#pragma unroll
    for (int k = 5; k < 10; k++) M[k] += as * r[k - 4] * (R)sqrt(INVB[k]);
#pragma unroll
    for (int k = 10; k < Q; k++) M[k] += ag * r[k - 4] * (R)sqrt(INVB[k]);
    mrt_backward<R, false, CW, WS>(M, d, sc);
  } else {
    if (!GZ) {
      const R gg = (R)1 - om_ghost;
#pragma unroll
      for (int k = 10; k < Q; k++) M[k] = gg * m[k] * (R)INVB[k];
    }
    mrt_backward<R, GZ, CW, WS>(M, d, sc);
  }
}

// Arena layout: pop[z][y / Y][i][y % Y][x] (x fastest), Y = 2^ylog.  The
// 19 population rows of a block of Y consecutive y lines are adjacent, and
// each population's Y rows are contiguous, so that a population row of a
// block spans whole 128-byte lines when nx is short (Y = 1 gives
// pop[z][y][i][x]).  The populations a node pulls lie in at most nine
// neighbouring lines (y - c_y, z - c_z).
__host__ __device__ __forceinline__ int64_t aidx(const BoxDesc& b, int i, int x, int y, int z) {
  const int Y = 1 << b.ylog;
  return (((int64_t)z * (b.ny >> b.ylog) + (y >> b.ylog)) * Q + i) * ((int64_t)b.nx << b.ylog) +
         (int64_t)(y & (Y - 1)) * b.nx + x;
}

// Neighbour coordinate with wrap on periodic axes.
__device__ __forceinline__ int wrapc(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// How a buffer holds the pre-collision state of t_n:
//   LAYOUT_PULL   post-collision populations of t_{n-1} at their source node:
//                 f_i(x) = A[x - c_i][i] (two buffers; boundary slots hold the
//                 boundary equilibrium)
//   LAYOUT_PLACE  in place: f_i(x) = A[x][i] (a state just uploaded, or the
//                 single buffer of in-place streaming after an odd step)
//   LAYOUT_SWAP   post-collision populations of t_{n-1} in the opposite slot
//                 of their source node: f_i(x) = A[x - c_i][OPP[i]] (in-place
//                 streaming after an even step)
enum : int { LAYOUT_PULL = 0, LAYOUT_PLACE = 1, LAYOUT_SWAP = 2 };

// Layout of the single buffer of in-place streaming at time index n: even
// steps read in place and write each node's results into its opposite slots,
// odd steps read those and write the next in-place state.
__host__ __device__ __forceinline__ int aa_layout(long long n) {
  return (n & 1) ? LAYOUT_SWAP : LAYOUT_PLACE;
}

// Pre-collision deviations of node (x, y, z) at t_n from a buffer of the given
// layout (PER: periodic axes wrap).
template <int S, bool PER>
__device__ __forceinline__ void load_pre(const typename Store<S>::T* __restrict__ src,
                                         const BoxDesc& b, int x, int y, int z, int layout,
                                         typename Store<S>::R d[Q]) {
  using St = Store<S>;
  if (layout == LAYOUT_PLACE) {
#pragma unroll
    for (int i = 0; i < Q; i++) d[i] = St::dec(src[aidx(b, i, x, y, z)], b.dec[WCLS[i]]);
    return;
  }
  const bool swap = layout == LAYOUT_SWAP;
#pragma unroll
  for (int i = 0; i < Q; i++) {
    int sx = x - CX[i], sy = y - CY[i], sz = z - CZ[i];
    if (PER) {
      if (b.pmask & 1) sx = wrapc(sx, b.nx);
      if (b.pmask & 2) sy = wrapc(sy, b.ny);
      if (b.pmask & 4) sz = wrapc(sz, b.nz);
    }
    d[i] = St::dec(src[aidx(b, swap ? OPP[i] : i, sx, sy, sz)], b.dec[WCLS[i]]);
  }
}

}  // namespace lbdev
