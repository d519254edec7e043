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

enum : int { ITEM_TILE = 0, ITEM_BOUNDARY = 1 };

struct BoxDesc {
  int64_t off;          // element offset of pop[0] of this box in each population arena
  int64_t nn;           // nodes (boundary layer included)
  int nx, ny, nz, pmask;
  int bc_mode;          // 0 affine, 1 sampled, -1 none
  int bc_dt, bc_ns, bc_res;
  int64_t bc_t0;
  const void* bc;       // affine: double [ns][9]; sampled: T [ns][6][res][res][3]
  int chain_first, chain_count;
  int nbnd;             // boundary nodes of this box
  int face_cnt[6];      // nodes per face in enumeration order
  int face_start[6][3]; // start coordinate of each face's node ranges
  int face_len[6][3];   // extent of each face along x, y, z
  float dec[3];         // FP16 decode factor per weight class: w 2^-s
  float enc[3];         // FP16 encode factor per weight class: 2^s / w
  double interior;      // number of interior nodes
};

struct Item {
  int box, kind;
  int x0, y0, z0;       // tile origin (node coordinates)
  int ex, ey, ez;       // tile extents; boundary: x0 = first boundary node, ex = count
};

struct ChainDesc {
  int box, first, nb, substeps, fix_com, pad;
  double zeta, mass, fene_k, fene_r0;
  double decay;         // exp(-zeta h / mass), h = 1/substeps
  int ai[3];            // integer part of the anchor
  double af[3];         // fractional part of the anchor
};

struct DevState {
  long long step;       // time index n of the current state
  int err_key;          // 0x7fffffff when no error; else min over (owner << 4 | code index)
  int pad;
  unsigned int done;    // workgroups finished in the current fused launch
  unsigned int pad2;
};

constexpr int ERR_NONE = 0x7fffffff;
enum : int { EC_BEAD_OUT = 1, EC_FENE = 2, EC_UNSTABLE = 3 };

template <int S> struct Store;
template <> struct Store<0> {
  using T = double;   // storage
  using R = double;   // compute
  __device__ static R dec(T v, float) { return v; }
  __device__ static T enc(R v, float) { return v; }
};
template <> struct Store<1> {
  using T = float;
  using R = float;
  __device__ static R dec(T v, float) { return v; }
  __device__ static T enc(R v, float) { return v; }
};
template <> struct Store<2> {
  using T = _Float16;
  using R = float;
  __device__ static R dec(T v, float k) { return (float)v * k; }
  __device__ static T enc(R v, float k) { return (_Float16)(v * k); }
};

template <typename R>
__device__ __forceinline__ R wgt(int i) { return (R)WD[WCLS[i]]; }

// Equilibrium deviation f_eq_i(rho, u) - w_i rho0 = w_i [drho + rho(3 cu + 9/2 cu^2 - 3/2 u^2)]
template <typename R>
__device__ __forceinline__ void eq_dev(R drho, R rho, R ux, R uy, R uz, R out[Q]) {
  const R uu = ux * ux + uy * uy + uz * uz;
  const R base = drho - (R)1.5 * rho * uu;
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const R cu = (R)CX[i] * ux + (R)CY[i] * uy + (R)CZ[i] * uz;
    out[i] = wgt<R>(i) * (base + rho * cu * ((R)3.0 + (R)4.5 * cu));
  }
}

// Collision of one node in deviation form.  d[] in: pre-collision deviations,
// out: post-collision deviations.  g: force density of this step.
template <typename R, int COLL>
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
    eq_dev<R>(drho, rho, ux, uy, uz, eq);
    const R ug = ux * gx + uy * gy + uz * gz;
    const R fpre = (R)1 - (R)0.5 * omega;
#pragma unroll
    for (int i = 0; i < Q; i++) {
      const R cu = (R)CX[i] * ux + (R)CY[i] * uy + (R)CZ[i] * uz;
      const R cg = (R)CX[i] * gx + (R)CY[i] * gy + (R)CZ[i] * gz;
      const R F = wgt<R>(i) * ((R)3 * (cg - ug) + (R)9 * cu * cg);
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
      d[i] = wgt<R>(i) * s;
    }
  }
}

// Neighbour coordinate with wrap on periodic axes.
__device__ __forceinline__ int wrapc(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Pre-collision deviations of node (x, y, z) at t_n: pulled from the
// post-collision buffer of t_{n-1} (boundary slots hold the boundary
// equilibrium), or read in place when the buffer holds a pre-collision state.
template <int S, bool PER>
__device__ __forceinline__ void load_pre(const typename Store<S>::T* __restrict__ src,
                                         const BoxDesc& b, int x, int y, int z, bool pre,
                                         typename Store<S>::R d[Q]) {
  using St = Store<S>;
  const int64_t nn = b.nn;
  if (pre) {
    const int node = (z * b.ny + y) * b.nx + x;
#pragma unroll
    for (int i = 0; i < Q; i++) d[i] = St::dec(src[i * nn + node], b.dec[WCLS[i]]);
    return;
  }
#pragma unroll
  for (int i = 0; i < Q; i++) {
    int sx = x - CX[i], sy = y - CY[i], sz = z - CZ[i];
    if (PER) {
      if (b.pmask & 1) sx = wrapc(sx, b.nx);
      if (b.pmask & 2) sy = wrapc(sy, b.ny);
      if (b.pmask & 4) sz = wrapc(sz, b.nz);
    }
    const int node = (sz * b.ny + sy) * b.nx + sx;
    d[i] = St::dec(src[i * nn + node], b.dec[WCLS[i]]);
  }
}

}  // namespace lbdev
