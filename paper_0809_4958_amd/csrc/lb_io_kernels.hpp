// lb_io_kernels.hpp -- gfx950 kernels around the fused step: the per-step
// finalisation, state upload and readout, and the stream-copy probe.
//
//   k_finalize  one workgroup at the end of a step (check steps, or contexts
//               without chains; otherwise k_force ends the step): reduces the
//               check partials in a fixed order per box, checks finiteness,
//               advances the step counter.
//   k_set_pre / k_read / k_read_sites / k_read_beads   state upload and readout.
//   k_copy      16-byte stream copy in contiguous per-workgroup chunks (HBM
//               ceiling probe).
#pragma once
#include "lb_kernels.hpp"

namespace lbdev {

// One workgroup after the fused step: per-box fixed-order sums of the item
// partials (on check steps), finiteness check, device step advance.  Runs as
// its own launch so that the fused kernel needs no device-wide fences.
__global__ __launch_bounds__(WG) void k_finalize(LbArgs A) {
  const int tid = threadIdx.x;
  put_stamp(A.stamp_after);
  if (A.st->err_key != ERR_NONE) return;
  const long long step = A.st->step;
  const bool check = A.reduce_every > 0 && ((step + 1) % A.reduce_every) == 0;
  __shared__ int s_bad;
  if (tid == 0) s_bad = 0x7fffffff;
  __syncthreads();
  if (check) {
    for (int bx = tid; bx < A.n_boxes; bx += WG) {
      double s[4] = {0.0, 0.0, 0.0, 0.0};
      for (int q = A.check_off[bx]; q < A.check_off[bx + 1]; q++) {
#pragma unroll
        for (int m = 0; m < 4; m++) s[m] += A.partials[4 * q + m];
      }
      const double M = A.rho0 * A.boxes[bx].interior + s[0];
      double* mm = A.mass_mom + 5 * bx;
      mm[0] = (double)(step + 1);
      mm[1] = M;
      mm[2] = s[1];
      mm[3] = s[2];
      mm[4] = s[3];
      if (!(isfinite(M) && isfinite(s[1]) && isfinite(s[2]) && isfinite(s[3]))) atomicMin(&s_bad, bx);
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (s_bad != 0x7fffffff)
      A.st->err_key = (s_bad << 4) | EC_UNSTABLE;
    else if (A.advance)
      A.st->step = step + 1;
  }
}

// ------------------------------------------------------- state upload
// pre-collision state of one box from FP64 populations [19][nn] (mode 0), from
// the equilibrium of a velocity field u[nn][3] (mode 1), rest (mode 2), or FP64
// deviations f_i - w_i rho0 [19][nn] (mode 3)
// swap: write the LAYOUT_SWAP image of that state (in-place streaming at an
// odd time index): f_i(x) of every interior node x into slot OPP[i] of node
// x - c_i (each slot has one writer); other slots are left as they are.
template <int S>
__global__ __launch_bounds__(WG) void k_set_pre(BoxDesc b, typename Store<S>::T* __restrict__ dst,
                                                const double* __restrict__ in, int mode, double rho0,
                                                int swap) {
  using St = Store<S>;
  using R = typename St::R;
  const int64_t nn = b.nn;
  for (int64_t node = (int64_t)blockIdx.x * WG + threadIdx.x; node < nn;
       node += (int64_t)gridDim.x * WG) {
    const int x = (int)(node % b.nx);
    const int y = (int)((node / b.nx) % b.ny);
    const int z = (int)(node / ((int64_t)b.nx * b.ny));
    R d[Q];
    if (!is_interior(b, x, y, z) || mode == 2) {
#pragma unroll
      for (int i = 0; i < Q; i++) d[i] = 0;
    } else if (mode == 0) {
#pragma unroll
      for (int i = 0; i < Q; i++) d[i] = (R)(in[i * nn + node] - WD[WCLS[i]] * rho0);
    } else if (mode == 3) {
#pragma unroll
      for (int i = 0; i < Q; i++) d[i] = (R)in[i * nn + node];
    } else {
      // deviation of f_eq(rho0, u): computed in FP64 then rounded once
      double ud[3] = {in[3 * node], in[3 * node + 1], in[3 * node + 2]};
      double eq[Q];
      eq_dev<double>(0.0, rho0, ud[0], ud[1], ud[2], eq);
#pragma unroll
      for (int i = 0; i < Q; i++) d[i] = (R)eq[i];
    }
    if (swap) {
      if (!is_interior(b, x, y, z)) continue;
#pragma unroll
      for (int i = 0; i < Q; i++) {
        int sx = x - CX[i], sy = y - CY[i], sz = z - CZ[i];
        if (b.pmask & 1) sx = wrapc(sx, b.nx);
        if (b.pmask & 2) sy = wrapc(sy, b.ny);
        if (b.pmask & 4) sz = wrapc(sz, b.nz);
        dst[aidx(b, OPP[i], sx, sy, sz)] = St::enc(d[i], b.enc[WCLS[i]]);
      }
      continue;
    }
#pragma unroll
    for (int i = 0; i < Q; i++) dst[aidx(b, i, x, y, z)] = St::enc(d[i], b.enc[WCLS[i]]);
  }
}

// ------------------------------------------------------------ readout
// what: 0 populations [19][nn], 1 rho [nn], 2 u [nn][3], 3 deviations [19][nn];
// pre: the layout of the buffer (LAYOUT_PULL, LAYOUT_PLACE or LAYOUT_SWAP)
template <int S, bool PER>
__global__ __launch_bounds__(WG) void k_read(BoxDesc b, const typename Store<S>::T* __restrict__ src,
                                             double* __restrict__ out, int what, int pre, double rho0) {
  using R = typename Store<S>::R;
  const int64_t nn = b.nn;
  for (int64_t node = (int64_t)blockIdx.x * WG + threadIdx.x; node < nn;
       node += (int64_t)gridDim.x * WG) {
    const int x = (int)(node % b.nx);
    const int y = (int)((node / b.nx) % b.ny);
    const int z = (int)(node / ((int64_t)b.nx * b.ny));
    double f[Q];
    if (is_interior(b, x, y, z)) {
      R d[Q];
      load_pre<S, PER>(src, b, x, y, z, pre, d);
#pragma unroll
      for (int i = 0; i < Q; i++) f[i] = WD[WCLS[i]] * rho0 + (double)d[i];
      if (what == 0) {
#pragma unroll
        for (int i = 0; i < Q; i++) out[i * nn + node] = f[i];
      } else if (what == 3) {
#pragma unroll
        for (int i = 0; i < Q; i++) out[i * nn + node] = (double)d[i];
      } else {
        double drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
        for (int i = 0; i < Q; i++) {
          drho += (double)d[i];
          jx += CX[i] * (double)d[i];
          jy += CY[i] * (double)d[i];
          jz += CZ[i] * (double)d[i];
        }
        const double rho = rho0 + drho;
        if (what == 1) {
          out[node] = rho;
        } else {
          out[3 * node] = jx / rho;
          out[3 * node + 1] = jy / rho;
          out[3 * node + 2] = jz / rho;
        }
      }
    } else {
      if (what == 0) {
#pragma unroll
        for (int i = 0; i < Q; i++) out[i * nn + node] = WD[WCLS[i]] * rho0;
      } else if (what == 3) {
#pragma unroll
        for (int i = 0; i < Q; i++) out[i * nn + node] = 0.0;
      } else if (what == 1) {
        out[node] = rho0;
      } else {
        out[3 * node] = out[3 * node + 1] = out[3 * node + 2] = 0.0;
      }
    }
  }
}

template <int S, bool PER>
__global__ __launch_bounds__(WG) void k_read_sites(BoxDesc b, const typename Store<S>::T* __restrict__ src,
                                                   const int* __restrict__ xyz, int n,
                                                   double* __restrict__ out, int pre, double rho0) {
  using R = typename Store<S>::R;
  const int k = blockIdx.x * WG + threadIdx.x;
  if (k >= n) return;
  R d[Q];
  load_pre<S, PER>(src, b, xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2], pre, d);
#pragma unroll
  for (int i = 0; i < Q; i++) out[Q * k + i] = WD[WCLS[i]] * rho0 + (double)d[i];
}

// bead positions/velocities of one parity buffer back to absolute FP64 coordinates
template <typename R>
__global__ void k_read_beads(const ChainDesc* __restrict__ chains, int c0, int c1,
                             const R* __restrict__ buf, double* __restrict__ out, int add_anchor) {
  int o = 0;
  for (int c = c0; c < c1; c++) {
    const ChainDesc ch = chains[c];
    for (int j = threadIdx.x; j < ch.nb; j += blockDim.x)
      for (int a = 0; a < 3; a++) {
        double v = (double)buf[3 * (ch.first + j) + a];
        if (add_anchor) v = (double)ch.ai[a] + (ch.af[a] + v);
        out[3 * (o + j) + a] = v;
      }
    o += ch.nb;
  }
}

// stream copy with 16-byte accesses, four independent loads in flight per
// thread, non-temporal stores (HBM ceiling probe); n is a multiple of
// 4 * WG * gridDim.x or the tail is copied one vector at a time
__global__ __launch_bounds__(WG) void k_copy(const uint4* __restrict__ src_, uint4* __restrict__ dst_,
                                             size_t n, size_t per_block) {
  typedef unsigned v4 __attribute__((ext_vector_type(4)));
  const v4* __restrict__ src = (const v4*)src_;
  v4* __restrict__ dst = (v4*)dst_;
  // each workgroup streams its own contiguous chunk of per_block vectors
  const size_t b0 = (size_t)blockIdx.x * per_block;
  const size_t b1 = b0 + per_block < n ? b0 + per_block : n;
  size_t i = b0 + threadIdx.x;
  for (; i + 3 * WG < b1; i += 4 * WG) {
    const v4 a = src[i], b = src[i + WG], c = src[i + 2 * WG], d = src[i + 3 * WG];
    __builtin_nontemporal_store(a, &dst[i]);
    __builtin_nontemporal_store(b, &dst[i + WG]);
    __builtin_nontemporal_store(c, &dst[i + 2 * WG]);
    __builtin_nontemporal_store(d, &dst[i + 3 * WG]);
  }
  for (; i < b1; i += WG) __builtin_nontemporal_store(src[i], &dst[i]);
}

}  // namespace lbdev
