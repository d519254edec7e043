// lb_vort_kernels.hpp -- vorticity of the fine box, the quantity the paper
// compares with the DNS (Sec. 3, Figs. 1 and 2: |omega| averaged over a
// control volume around the tracer).
//
//   k_vort      |curl u| of u = j/rho at t_n (pre-collision moments) by
//               second-order central differences, (d u_c/d x_a)(q) =
//               (u_c(q + e_a) - u_c(q - e_a)) / 2, summed over a control
//               volume (FP64 partial per workgroup), optionally stored per node.
//               A workgroup walks a 16 x 16 (x, y) tile through a slab of
//               planes; u of the tile plus a one-node halo is kept for three
//               consecutive planes in an LDS ring, so each node's populations
//               are loaded (18/16)^2 ~ 1.27 times and the z neighbours are
//               reused from LDS.  Moments and differences in FP64 whatever
//               the storage: the stored populations are the only rounding.
//   k_vort_sum  one workgroup: the partials of each volume in a fixed order.
#pragma once
#include "lb_kernels.hpp"

namespace lbdev {

constexpr int VT = 16;   // tile edge (x and y), one node per thread
constexpr int VH = VT + 2;

struct VortArgs {
  BoxDesc b;
  const void* src;      // the box's populations in the current arena
  int pre;              // layout of the arena (LAYOUT_PULL, LAYOUT_PLACE or LAYOUT_SWAP)
  double rho0;
  int lo[3], hi[3];     // control volume, inclusive node ranges
  int tx, ty, zslab;    // tiles along x and y, planes per workgroup
  double* partials;     // [grid] sum of |omega| over each workgroup's nodes
  double* field;        // [nz][ny][nx] |omega| per node, or NULL
};

template <int S, bool PER>
__global__ __launch_bounds__(VT * VT) void k_vort(VortArgs A) {
  using St = Store<S>;
  using T = typename St::T;
  using R = typename St::R;
  __shared__ double su[3][VH][VH][3];
  __shared__ double red[VT * VT / 64];
  const int tid = threadIdx.x;
  const BoxDesc& b = A.b;
  const int per_slab = A.tx * A.ty;
  const int tile = blockIdx.x % per_slab, slab = blockIdx.x / per_slab;
  const int x0 = A.lo[0] + VT * (tile % A.tx), y0 = A.lo[1] + VT * (tile / A.tx);
  const int z0 = A.lo[2] + slab * A.zslab;
  const int z1 = min(A.hi[2], z0 + A.zslab - 1);
  const T* src = (const T*)A.src;
  double acc = 0.0;
  for (int z = z0 - 1; z <= z1 + 1; z++) {
    const int slot = (z - (z0 - 1)) % 3;
    for (int p = tid; p < VH * VH; p += VT * VT) {
      const int lx = p % VH, ly = p / VH;
      int x = x0 - 1 + lx, y = y0 - 1 + ly, zz = z;
      if (x > A.hi[0] + 1 || y > A.hi[1] + 1) continue;
      if (PER) {
        if (b.pmask & 1) x = wrapc(x, b.nx);
        if (b.pmask & 2) y = wrapc(y, b.ny);
        if (b.pmask & 4) zz = wrapc(zz, b.nz);
      }
      R d[Q];
      load_pre<S, PER>(src, b, x, y, zz, A.pre, d);
      double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
      for (int i = 0; i < Q; i++) {
        const double v = (double)d[i];
        drho += v;
        if (CX[i]) jx += (double)CX[i] * v;
        if (CY[i]) jy += (double)CY[i] * v;
        if (CZ[i]) jz += (double)CZ[i] * v;
      }
      const double inv = 1.0 / (A.rho0 + drho);
      su[slot][ly][lx][0] = jx * inv;
      su[slot][ly][lx][1] = jy * inv;
      su[slot][ly][lx][2] = jz * inv;
    }
    __syncthreads();
    const int zc = z - 1;
    if (zc >= z0) {
      const int tx = tid % VT, ty = tid / VT;
      const int x = x0 + tx, y = y0 + ty;
      if (x <= A.hi[0] && y <= A.hi[1]) {
        const int sm = (zc - 1 - (z0 - 1)) % 3, s0 = (zc - (z0 - 1)) % 3, sp = slot;
        const int lx = tx + 1, ly = ty + 1;
        double du[3][3];  // du[c][a] = d u_c / d x_a
#pragma unroll
        for (int c = 0; c < 3; c++) {
          du[c][0] = 0.5 * (su[s0][ly][lx + 1][c] - su[s0][ly][lx - 1][c]);
          du[c][1] = 0.5 * (su[s0][ly + 1][lx][c] - su[s0][ly - 1][lx][c]);
          du[c][2] = 0.5 * (su[sp][ly][lx][c] - su[sm][ly][lx][c]);
        }
        const double wx = du[2][1] - du[1][2];
        const double wy = du[0][2] - du[2][0];
        const double wz = du[1][0] - du[0][1];
        const double w = sqrt(wx * wx + wy * wy + wz * wz);
        acc += w;
        if (A.field) A.field[((int64_t)zc * b.ny + y) * b.nx + x] = w;
      }
    }
    __syncthreads();
  }
  acc = wave_sum(acc);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < VT * VT / 64; w++) s += red[w];
    A.partials[blockIdx.x] = s;
  }
}

// Sums of the workgroup partials of each volume, in a fixed order:
// thread t adds partials t, t + 256, ... of its volume, then a fixed tree.
// off[v] .. off[v+1] are volume v's partials; out[v] = sum / count[v].
__global__ __launch_bounds__(WG) void k_vort_sum(const double* __restrict__ partials,
                                                 const int* __restrict__ off,
                                                 const double* __restrict__ count, int n_vol,
                                                 double* __restrict__ out) {
  __shared__ double red[WG];
  const int tid = threadIdx.x;
  for (int v = 0; v < n_vol; v++) {
    double s = 0.0;
    for (int k = off[v] + tid; k < off[v + 1]; k += WG) s += partials[k];
    red[tid] = s;
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) out[v] = red[0] / count[v];
    __syncthreads();
  }
}

}  // namespace lbdev
