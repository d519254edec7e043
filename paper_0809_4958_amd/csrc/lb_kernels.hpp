// lb_kernels.hpp -- gfx950 kernels of the fine-box lattice-Boltzmann step.
//
//   k_chain   one workgroup per chain (one wavefront when the chains have at
//             most 64 beads): trilinear interpolation of the fluid
//             velocity at each bead from the pre-collision moments, the MD
//             substeps (FENE, exact friction update, centre-of-mass pin) and
//             the spreading records (stencil base, fractional offsets,
//             friction impulse) plus the chain's stencil bounding box.
//   k_lb      the fused step over a work list: interior rows and tiles do
//             pull streaming, collide and store (periodic boxes also gather
//             the spread force of their chains); boundary items store the
//             boundary equilibrium populations that point into the interior.
//   k_force   after k_lb, one workgroup per chain of a non-periodic box: the
//             nodes of the chain's stencil box collide again with the spread
//             force gathered from the records (fixed bead order, no atomics);
//             on steps without a check pass its last workgroup ends the step.
//   k_check   on check steps: FP64 partial sums of the interior's mass and
//             momentum at t_{n+1} from the arena k_lb wrote; k_finalize
//             (lb_io_kernels.hpp) adds them per box.
#pragma once
#include "lb_device.hpp"

namespace lbdev {

constexpr int WG = 256;
constexpr int MAX_SLOTS = 4;   // tile plane positions per thread (ex*ey <= 1024)
constexpr int MAX_BOX_CHAINS = 64;
// Cache-policy bits of the row items' population loads and stores (0, or the
// non-temporal hint 2): every population is written once per step and read
// only in the next, so the stores stream past the caches (measured +6% on the
// batched FP16 step); non-temporal loads measured slower.  Build-time choices,
// like LB_MIN_WAVES (when defined, it overrides the per-variant wave counts of
// lb_min_waves for every FP32/FP16 step kernel).
#ifndef LB_LOAD_POLICY
#define LB_LOAD_POLICY 0
#endif
#ifndef LB_STORE_POLICY
#define LB_STORE_POLICY 2
#endif

// Timing inside captured graphs: thread 0 of workgroup 0 (dispatched first)
// records the constant-rate device clock (hipDeviceAttributeWallClockRate kHz)
// when its kernel starts, with a vector store; p = NULL records nothing.
__device__ __forceinline__ void put_stamp(long long* p) {
  if (p && blockIdx.x == 0 && threadIdx.x == 0) *p = wall_clock64();
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Value of another lane through a DPP move: CTRL the pattern, ROWS the
// 16-lane rows written; lanes whose source is outside the pattern, and rows
// not written, read 0
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_get(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, true));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_get(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), CTRL, ROWS, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, ROWS, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float lane63(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ double lane63(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// N sums over the 64 lanes at once, returned to every lane, in one fixed
// order with register-to-register lane moves (DPP): within each 16-lane row
// lane i adds lane i-1, i-2, i-4, i-8 (shifts in, zero at the row start), so
// lane 15 of a row holds the row's sum; then rows 1 and 3 add lane 15 of the
// row before, rows 2 and 3 add lane 31, and lane 63 holds the total.  Called
// with every lane active.
template <typename R, int N>
__device__ __forceinline__ void wave_sums(R (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; k++) v[k] += dpp_get<0x111, 0xf>(v[k]);  // row_shr:1
#pragma unroll
  for (int k = 0; k < N; k++) v[k] += dpp_get<0x112, 0xf>(v[k]);  // row_shr:2
#pragma unroll
  for (int k = 0; k < N; k++) v[k] += dpp_get<0x114, 0xf>(v[k]);  // row_shr:4
#pragma unroll
  for (int k = 0; k < N; k++) v[k] += dpp_get<0x118, 0xf>(v[k]);  // row_shr:8
#pragma unroll
  for (int k = 0; k < N; k++) v[k] += dpp_get<0x142, 0xa>(v[k]);  // row_bcast:15
#pragma unroll
  for (int k = 0; k < N; k++) v[k] += dpp_get<0x143, 0xc>(v[k]);  // row_bcast:31
#pragma unroll
  for (int k = 0; k < N; k++) v[k] = lane63(v[k]);
}

// x-face boundary velocities of one work item by one wavefront (defined with
// k_xface below)
template <int S>
__device__ __forceinline__ void xface_wave(const BoxDesc* __restrict__ boxes,
                                           const int4* __restrict__ items, int item,
                                           float* __restrict__ xface, DevState* __restrict__ st,
                                           long long* stamp);

// ---------------------------------------------------------------- chain
// CB threads per chain (one per bead): 64 when no chain has more than 64
// beads (one wavefront: the MD substeps exchange values by cross-lane
// operations, with no barriers), else 256 (through LDS).
// Workgroups n_chains and up compute the x-face boundary velocities of the
// step instead (CB / 64 work items each), so the two independent pieces of
// work before the fused step share one launch and run side by side.
template <int S, bool PER, int CB, bool TH = false>
__global__ __launch_bounds__(CB, 3) void k_chain(const BoxDesc* __restrict__ boxes,
                                              const ChainDesc* __restrict__ chains,
                                              const typename Store<S>::T* __restrict__ a0,
                                              const typename Store<S>::T* __restrict__ a1,
                                              double* __restrict__ pos,
                                              double* __restrict__ vel,
                                              int total_beads, int4* __restrict__ rec_base,
                                              double* __restrict__ rec_d,
                                              double* __restrict__ rec_dp,
                                              int* __restrict__ bbox, DevState* __restrict__ st,
                                              double rho0_d, int pre, long long* stamp,
                                              int n_chains, const int4* __restrict__ xf_items,
                                              int n_xf_items, float* __restrict__ xface,
                                              unsigned key0, unsigned key1) {
  // Chain arithmetic in FP64 for every storage.  The friction impulses of a
  // chain's beads are dominated by their bond forces, which cancel between
  // neighbouring beads on the nodes the spreading shares: the node force is
  // a small difference of large terms, and FP32 impulses and stencil weights
  // cost 1e-4 of the fluid velocity near 32 collapsed 256-bead chains over
  // 2,000 steps (FP32 storage, against 5e-8 without chains).
  using R = double;
  using RP = typename Store<S>::R;
  const int ci = blockIdx.x;
  if (ci >= n_chains) {
    const int item = (ci - n_chains) * (CB / 64) +
                     __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    if (item < n_xf_items) xface_wave<S>(boxes, xf_items, item, xface, st, nullptr);
    return;
  }
  // inputs read before the timestamp store (see k_check)
  const ChainDesc c = chains[ci];
  const BoxDesc b = boxes[c.box];
  const bool latched = __hip_atomic_load(&st->err_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ERR_NONE;
  put_stamp(stamp);
  if (latched) return;
  const R rho0 = (R)rho0_d;
  const long long step = st->step;
  const int par = (int)(step & 1);
  const typename Store<S>::T* src = (par ? a1 : a0) + b.off;
  const int j = threadIdx.x;
  const bool act = j < c.nb;
  const int gj = c.first + j;

  __shared__ R spx[CB], spy[CB], spz[CB];
  __shared__ R bfx[CB], bfy[CB], bfz[CB];
  __shared__ R red[3][CB];
  __shared__ int sflag;
  __shared__ int sbox[6];
  if (j == 0) {
    sflag = 0;
    sbox[0] = sbox[1] = sbox[2] = 0x7fffffff;
    sbox[3] = sbox[4] = sbox[5] = -0x7fffffff;
  }
  R rx = 0, ry = 0, rz = 0, vx = 0, vy = 0, vz = 0;
  const size_t pin = (size_t)par * total_beads * 3, pout = (size_t)(par ^ 1) * total_beads * 3;
  if (act) {
    rx = pos[pin + 3 * gj];
    ry = pos[pin + 3 * gj + 1];
    rz = pos[pin + 3 * gj + 2];
    vx = vel[pin + 3 * gj];
    vy = vel[pin + 3 * gj + 1];
    vz = vel[pin + 3 * gj + 2];
  }
  __syncthreads();

  // stencil at t_n: R = anchor + rel, anchor split into integer + fractional parts
  int base[3] = {0, 0, 0};
  R dl[3] = {0, 0, 0};
  if (act) {
    const R rr[3] = {rx, ry, rz};
    const int n3[3] = {b.nx, b.ny, b.nz};
    bool out = false;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      const R r = (R)c.af[a] + rr[a];
      const R fl = floor(r);
      base[a] = c.ai[a] + (int)fl;
      dl[a] = r - fl;
      if (!((b.pmask >> a) & 1)) {
        if (base[a] < 1 || base[a] + 1 > n3[a] - 2) out = true;
      } else {
        base[a] = ((base[a] % n3[a]) + n3[a]) % n3[a];
      }
    }
    if (out) atomicOr(&sflag, 1);
  }
  __syncthreads();
  if (sflag) {
    if (j == 0) atomicMin(&st->err_key, (ci << 4) | EC_BEAD_OUT);
    return;
  }

  // fluid velocity at the bead: sum over the 8 corners of weight x j/rho, in
  // corner order, four corners at a time (their loads in flight together).
  // All eight at once took 214 VGPRs.  The kernel is compiled for three
  // waves per SIMD (168 VGPRs with the FP64 chain arithmetic, a few spilled),
  // so that the x-face waves sharing its launch run three per SIMD, not two
  // (measured 27.6 against 30.2 us for the launch on the batch).
  R ux = 0, uy = 0, uz = 0;
  if (act) {
#pragma unroll 1
    for (int half = 0; half < 2; half++)
#pragma unroll
    for (int c4 = 0; c4 < 4; c4++) {
      const int cc = 4 * half + c4;
      const int o0 = cc & 1, o1 = (cc >> 1) & 1, o2 = (cc >> 2) & 1;
      int qx = base[0] + o0, qy = base[1] + o1, qz = base[2] + o2;
      if (PER) {
        if (b.pmask & 1) qx = wrapc(qx, b.nx);
        if (b.pmask & 2) qy = wrapc(qy, b.ny);
        if (b.pmask & 4) qz = wrapc(qz, b.nz);
      }
      const R w = (o0 ? dl[0] : (R)1 - dl[0]) * (o1 ? dl[1] : (R)1 - dl[1]) *
                  (o2 ? dl[2] : (R)1 - dl[2]);
      RP d[Q];
      load_pre<S, PER>(src, b, qx, qy, qz, pre == 2 ? aa_layout(step) : pre, d);
      R drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
      for (int i = 0; i < Q; i++) {
        drho += d[i];
        if (CX[i]) jx += (R)CX[i] * d[i];
        if (CY[i]) jy += (R)CY[i] * d[i];
        if (CZ[i]) jz += (R)CZ[i] * d[i];
      }
      const R wr = w / (rho0 + drho);
      ux += wr * jx;
      uy += wr * jy;
      uz += wr * jz;
    }
  }

  // MD substeps.  With one wavefront per chain (CB = 64) the neighbour's
  // position, the neighbour's bond force, the FENE overflow flag and the
  // centre-of-mass sums move between lanes by cross-lane operations, with no
  // barriers (the sums in the fixed DPP order of wave_sums); otherwise
  // through LDS (a fixed-order tree).
  constexpr bool WAVE = CB == 64;
  const R h = (R)1 / (R)c.substeps;
  const R decay = (R)c.decay;
  const R mass = (R)c.mass, fk = (R)c.fene_k;
  const R r02 = (R)(c.fene_r0 * c.fene_r0);
  // reciprocals once: the substeps' dependent chain then holds one division
  // (the FENE factor) instead of five
  const R izeta = (R)1 / (R)c.zeta, ir02 = (R)1 / r02, inb = (R)1 / (R)c.nb;
  // FENE force of the bond to the next bead (separation e); false when the
  // bond has reached its maximum extension
  auto fene = [&](R ex, R ey, R ez, R& fx, R& fy, R& fz) -> bool {
    const R r2 = ex * ex + ey * ey + ez * ez;
    if (r2 >= r02) return false;
    const R fac = fk / ((R)1 - r2 * ir02);
    fx = fac * ex;
    fy = fac * ey;
    fz = fac * ez;
    return true;
  };
  R dpx = 0, dpy = 0, dpz = 0;
  bool overflow = false;
  for (int s = 0; s < c.substeps; s++) {
    R fx = 0, fy = 0, fz = 0;  // bond j -> j+1
    R gx = 0, gy = 0, gz = 0;  // bond j-1 -> j
    if constexpr (WAVE) {
      // next bead's position (wave_shl:1: lane j reads lane j+1)
      const R qx = dpp_get<0x130, 0xf>(rx), qy = dpp_get<0x130, 0xf>(ry),
              qz = dpp_get<0x130, 0xf>(rz);
      bool bad = false;
      if (act && j + 1 < c.nb) bad = !fene(qx - rx, qy - ry, qz - rz, fx, fy, fz);
      if (__any(bad)) {
        overflow = true;
        break;
      }
      // previous bead's bond force (wave_shr:1: lane j reads lane j-1)
      gx = dpp_get<0x138, 0xf>(fx);
      gy = dpp_get<0x138, 0xf>(fy);
      gz = dpp_get<0x138, 0xf>(fz);
    } else {
      spx[j] = rx;
      spy[j] = ry;
      spz[j] = rz;
      __syncthreads();
      if (act && j + 1 < c.nb && !fene(spx[j + 1] - rx, spy[j + 1] - ry, spz[j + 1] - rz, fx, fy, fz))
        atomicOr(&sflag, 2);
      bfx[j] = fx;
      bfy[j] = fy;
      bfz[j] = fz;
      __syncthreads();
      if (sflag) {
        overflow = true;
        break;
      }
      if (j > 0) {
        gx = bfx[j - 1];
        gy = bfy[j - 1];
        gz = bfz[j - 1];
      }
    }
    if (act) {
      R Fx = fx, Fy = fy, Fz = fz;
      if (j > 0) {
        Fx -= gx;
        Fy -= gy;
        Fz -= gz;
      }
      const R tx = ux + Fx * izeta, ty = uy + Fy * izeta, tz = uz + Fz * izeta;
      R nvx = tx + (vx - tx) * decay, nvy = ty + (vy - ty) * decay, nvz = tz + (vz - tz) * decay;
      if constexpr (TH) {
        // Langevin noise of the exact friction update: the Ornstein-Uhlenbeck
        // kick of the substep, from the Philox counter (bead index in the box,
        // box, step, 16 + substep)
        unsigned cc[4] = {(unsigned)(c.bead0 + j), (unsigned)b.index, (unsigned)step, 16u + (unsigned)s};
        philox4x32(cc, key0, key1);
        const double kick = c.kick;
        nvx += (R)(kick * unit_uniform(cc[0]));
        nvy += (R)(kick * unit_uniform(cc[1]));
        nvz += (R)(kick * unit_uniform(cc[2]));
      }
      dpx += mass * (nvx - vx) - Fx * h;
      dpy += mass * (nvy - vy) - Fy * h;
      dpz += mass * (nvz - vz) - Fz * h;
      vx = nvx;
      vy = nvy;
      vz = nvz;
      rx += h * vx;
      ry += h * vy;
      rz += h * vz;
    }
    if (c.fix_com && WAVE) {
      // fixed-order sums of velocity and relative position, all six at once
      // (the position sum does not depend on the velocity correction)
      R t[6] = {act ? vx : (R)0, act ? vy : (R)0, act ? vz : (R)0,
                act ? rx : (R)0, act ? ry : (R)0, act ? rz : (R)0};
      wave_sums(t);
      vx -= t[0] * inb;
      vy -= t[1] * inb;
      vz -= t[2] * inb;
      rx -= t[3] * inb;
      ry -= t[4] * inb;
      rz -= t[5] * inb;
    } else if (c.fix_com) {
      // fixed-order tree sums of velocity and relative position
#pragma unroll 1
      for (int pass = 0; pass < 2; pass++) {
        R sx = act ? (pass ? rx : vx) : (R)0;
        R sy = act ? (pass ? ry : vy) : (R)0;
        R sz = act ? (pass ? rz : vz) : (R)0;
        red[0][j] = sx;
        red[1][j] = sy;
        red[2][j] = sz;
        __syncthreads();
        for (int o = CB / 2; o > 0; o >>= 1) {
          if (j < o) {
            red[0][j] += red[0][j + o];
            red[1][j] += red[1][j + o];
            red[2][j] += red[2][j + o];
          }
          __syncthreads();
        }
        sx = red[0][0];
        sy = red[1][0];
        sz = red[2][0];
        __syncthreads();
        const R mx = sx * inb, my = sy * inb, mz = sz * inb;
        if (pass == 0) {
          vx -= mx;
          vy -= my;
          vz -= mz;
        } else {
          rx -= mx;
          ry -= my;
          rz -= mz;
        }
      }
    }
    if constexpr (!WAVE) __syncthreads();
  }
  if (overflow) {
    if (j == 0) atomicMin(&st->err_key, (ci << 4) | EC_FENE);
    return;
  }
  if (act) {
    pos[pout + 3 * gj] = rx;
    pos[pout + 3 * gj + 1] = ry;
    pos[pout + 3 * gj + 2] = rz;
    vel[pout + 3 * gj] = vx;
    vel[pout + 3 * gj + 1] = vy;
    vel[pout + 3 * gj + 2] = vz;
    rec_base[gj] = make_int4(base[0], base[1], base[2], 0);
    rec_d[3 * gj] = dl[0];
    rec_d[3 * gj + 1] = dl[1];
    rec_d[3 * gj + 2] = dl[2];
    rec_dp[3 * gj] = dpx;
    rec_dp[3 * gj + 1] = dpy;
    rec_dp[3 * gj + 2] = dpz;
    atomicMin(&sbox[0], base[0]);
    atomicMin(&sbox[1], base[1]);
    atomicMin(&sbox[2], base[2]);
    atomicMax(&sbox[3], base[0] + 1);
    atomicMax(&sbox[4], base[1] + 1);
    atomicMax(&sbox[5], base[2] + 1);
  }
  __syncthreads();
  if (j == 0) {
    if (b.pmask) {
      // wrapped stencils: every tile of the box checks this chain
      bbox[6 * ci + 0] = 0;
      bbox[6 * ci + 1] = 0;
      bbox[6 * ci + 2] = 0;
      bbox[6 * ci + 3] = b.nx - 1;
      bbox[6 * ci + 4] = b.ny - 1;
      bbox[6 * ci + 5] = b.nz - 1;
    } else {
      for (int a = 0; a < 6; a++) bbox[6 * ci + a] = sbox[a];
    }
  }
}

// ----------------------------------------------------- boundary helpers
// Velocity u_b of boundary node q on face f at step n (Sec. 2-3): affine
// u_b = A(t_n)(q - x_c) or bilinear on the face x linear in time.
// The time part, the same for every node of a box at step n: the samples k,
// k1 and the weight th of the second (two = false: k alone).
template <typename R>
struct BcTime {
  long long k, k1;
  bool two;
  R th;
};

template <typename R>
__device__ __forceinline__ BcTime<R> bc_time(const BoxDesc& b, long long n) {
  long long rel = n - b.bc_t0;
  if (rel < 0) rel = 0;
  long long k = rel / b.bc_dt;
  long long rem = rel - k * b.bc_dt;
  long long k1 = k + 1;  // second sample of the linear time weight
  if (b.bc_mode == 2) {
    // learned: ring of n_samples slots
    k %= b.bc_ns;
    k1 = (k + 1) % b.bc_ns;
  } else if (k >= b.bc_ns) {
    k = b.bc_ns - 1;
    rem = 0;
  }
  BcTime<R> tm;
  tm.k = k;
  tm.k1 = k1;
  tm.two = rem > 0 && (b.bc_mode == 2 || k1 < b.bc_ns);
  tm.th = (R)rem / (R)b.bc_dt;
  return tm;
}

// The space part at node q of face f, given the time part of the step.
template <typename R>
__device__ __forceinline__ void boundary_velocity(const BoxDesc& b, int f, const int q[3],
                                                  const BcTime<R>& tm, R u[3]) {
  const long long k = tm.k, k1 = tm.k1;
  const bool two = tm.two;
  const R th = tm.th;
  if (b.bc_mode == 0) {
    const double* A0 = (const double*)b.bc + 9 * k;
    const double* A1 = A0 + 9;
    const R rx = (R)q[0] - (R)0.5 * (R)(b.nx - 1);
    const R ry = (R)q[1] - (R)0.5 * (R)(b.ny - 1);
    const R rz = (R)q[2] - (R)0.5 * (R)(b.nz - 1);
#pragma unroll
    for (int a = 0; a < 3; a++) {
      R m0 = (R)A0[3 * a], m1 = (R)A0[3 * a + 1], m2 = (R)A0[3 * a + 2];
      if (two) {
        m0 = ((R)1 - th) * m0 + th * (R)A1[3 * a];
        m1 = ((R)1 - th) * m1 + th * (R)A1[3 * a + 1];
        m2 = ((R)1 - th) * m2 + th * (R)A1[3 * a + 2];
      }
      u[a] = m0 * rx + m1 * ry + m2 * rz;
    }
    return;
  }
  const int a = f >> 1;
  const int au = (a == 0) ? 1 : 0;
  const int av = (a == 2) ? 1 : 2;
  const int n3[3] = {b.nx, b.ny, b.nz};
  const int nu = n3[au], nv = n3[av];
  const int Rr = b.bc_res;
  // cell and fraction in exact integer arithmetic, 32-bit (lb_set_boundary
  // keeps (n - 1)(res - 1) below 2^31): a per-lane 64-bit division costs
  // an order of magnitude more instructions
  const unsigned du = (unsigned)(nu - 1), dv = (unsigned)(nv - 1);
  const unsigned su = (unsigned)q[au] * (unsigned)(Rr - 1), sv = (unsigned)q[av] * (unsigned)(Rr - 1);
  const unsigned pu = su / du, pv = sv / dv;
  const int p = (int)pu, qq = (int)pv;
  const R al = (R)(int)(su - pu * du) / (R)(nu - 1);
  const R be = (R)(int)(sv - pv * dv) / (R)(nv - 1);
  const int p1 = p + 1 < Rr ? p + 1 : p, q1 = qq + 1 < Rr ? qq + 1 : qq;
  // the three components of a grid point are adjacent: one vector load per
  // corner (scattered gathers are limited by the address rate, not bytes)
  struct V3 {
    R c[3];
  };
  const V3* Sb = (const V3*)b.bc;
  const size_t fs = (size_t)Rr * Rr;
  R v0[3], v1[3] = {0, 0, 0};
#pragma unroll
  for (int t = 0; t < 2; t++) {
    if (t == 1 && !two) break;
    const V3* Sk = Sb + ((size_t)(t ? k1 : k) * 6 + f) * fs;
    R* out = t ? v1 : v0;
    const V3 s00 = Sk[(size_t)qq * Rr + p], s01 = Sk[(size_t)qq * Rr + p1];
    const V3 s10 = Sk[(size_t)q1 * Rr + p], s11 = Sk[(size_t)q1 * Rr + p1];
#pragma unroll
    for (int cmp = 0; cmp < 3; cmp++)
      out[cmp] = ((R)1 - al) * ((R)1 - be) * s00.c[cmp] + al * ((R)1 - be) * s01.c[cmp] +
                 ((R)1 - al) * be * s10.c[cmp] + al * be * s11.c[cmp];
  }
#pragma unroll
  for (int cmp = 0; cmp < 3; cmp++) u[cmp] = two ? ((R)1 - th) * v0[cmp] + th * v1[cmp] : v0[cmp];
}

__device__ __forceinline__ bool is_interior(const BoxDesc& b, int x, int y, int z) {
  return ((b.pmask & 1) || (x >= 1 && x <= b.nx - 2)) && ((b.pmask & 2) || (y >= 1 && y <= b.ny - 2)) &&
         ((b.pmask & 4) || (z >= 1 && z <= b.nz - 2));
}

struct LbArgs {
  const BoxDesc* boxes;
  const Item* items;
  const int* order;        // [n_entries], -1 = empty slot
  int n_entries;
  void* a0;
  void* a1;
  const ChainDesc* chains;
  const int4* rec_base;
  const void* rec_d;
  const void* rec_dp;
  const int* bbox;
  DevState* st;
  double* partials;        // [n_check][4] mass/momentum partials of k_check
  const int4* check_items; // k_check workgroups: box, first plane, end plane
  const int* check_off;    // [n_boxes + 1] first k_check workgroup of each box
  double* mass_mom;        // [n_boxes][5]
  long long* stamp_first;  // timed graphs: start of the step's first kernel,
  long long* stamp_lb;     // of k_lb,
  long long* stamp_after;  // and of the first kernel after k_lb (else NULL)
  float* xface;            // x-face velocities of the row boxes at t_n (k_xface)
  const int4* xf_items;    // x-face work items (one wavefront each): box, first node, count
  int n_xf_items;
  int n_boxes;
  int reduce_every;
  double rho0, omega, om_bulk, om_ghost;
  int pre;
  int advance;
  double kT;               // thermal fluctuations (fluctuating MRT) when > 0
  unsigned key0, key1;     // Philox key of the context's random numbers
  int aa;                  // in-place streaming on one buffer (a0 == a1): tile items only
};

// Collision dispatcher: 0 BGK, 1 MRT, 2 MRT with ghost rate 1.  CW: the
// lattice weights applied with their FP32 residual (FP32 storage).
// WS: the post-collision values come out in FP16 storage units,
// d_i 2^s / w_i with 2^s = sc (the MRT back transform then applies no weights)
template <typename R, int COLL, bool CW = false, bool WS = false>
__device__ __forceinline__ void collide_any(R d[Q], R gx, R gy, R gz, R rho0, R omega, R omb,
                                            R omg, R sc = R(1)) {
  if (COLL == 0) {
    collide<R, 0, CW>(d, gx, gy, gz, rho0, omega, omb, omg);
    if constexpr (WS) {
#pragma unroll
      for (int i = 0; i < Q; i++) d[i] *= sc * (R)(WCLS[i] == 0 ? 3 : (WCLS[i] == 1 ? 18 : 36));
    }
  } else if (COLL == 1) {
    collide_mrt_pairs<R, false, false, CW, WS>(d, gx, gy, gz, rho0, omega, omb, omg, nullptr, sc);
  } else {
    collide_mrt_pairs<R, true, false, CW, WS>(d, gx, gy, gz, rho0, omega, omb, omg, nullptr, sc);
  }
}

// whether the step of storage S applies the weights with their residual
template <int S>
constexpr bool comp_weights() { return S == 1; }

// Tracer acceleration of a box at step n (accelerated-frame body force,
// Sec. 2): linear in time between samples, in FP64 like the samples.
template <typename R>
__device__ __forceinline__ void body_accel(const BoxDesc& b, long long n, R& ax, R& ay, R& az) {
  ax = ay = az = (R)0;
  if (!b.body) return;
  long long rel = n - b.body_t0;
  if (rel < 0) rel = 0;
  long long k = rel / b.body_dt, rem = rel - k * b.body_dt;
  if (k >= b.body_ns) {
    k = b.body_ns - 1;
    rem = 0;
  }
  const double* a0 = b.body + 3 * k;
  if (rem > 0 && k + 1 < b.body_ns) {
    const double th = (double)rem / (double)b.body_dt;
    ax = (R)((1.0 - th) * a0[0] + th * a0[3]);
    ay = (R)((1.0 - th) * a0[1] + th * a0[4]);
    az = (R)((1.0 - th) * a0[2] + th * a0[5]);
  } else {
    ax = (R)a0[0];
    ay = (R)a0[1];
    az = (R)a0[2];
  }
}

// The per-step part of a box's collision extensions (node counter set per node).
template <typename R>
__device__ __forceinline__ Ext<R> make_ext(const LbArgs& A, const BoxDesc& b, long long step) {
  Ext<R> e;
  body_accel<R>(b, step, e.ax, e.ay, e.az);
  e.mu = (R)(3.0 * A.kT);
  e.k0 = A.key0;
  e.k1 = A.key1;
  e.node = 0u;
  e.box = (unsigned)b.index;
  e.step = (unsigned)step;
  return e;
}

// Collision with the extensions: the force density of the chains g plus the
// body force -rho a (rho the node's pre-collision density), and the
// fluctuating collision when mu > 0 (MRT only).
template <typename R, int COLL, bool CW = false, bool WS = false>
__device__ __forceinline__ void collide_ext(R d[Q], R gx, R gy, R gz, R rho0, R omega, R omb,
                                            R omg, const Ext<R>& e, R sc = R(1)) {
  R drho = 0;
#pragma unroll
  for (int i = 0; i < Q; i++) drho += d[i];
  const R rho = rho0 + drho;
  gx -= rho * e.ax;
  gy -= rho * e.ay;
  gz -= rho * e.az;
  if (COLL != 0 && e.mu > (R)0)
    collide_mrt_pairs<R, COLL == 2, true, CW, WS>(d, gx, gy, gz, rho0, omega, omb, omg, &e, sc);
  else
    collide_any<R, COLL, CW, WS>(d, gx, gy, gz, rho0, omega, omb, omg, sc);
}

// Spread force g(x) = - sum_j w_jx dP_j at node (x, y, z): chains whose stencil
// box overlaps the tile (cmask), beads in fixed order, no atomics.
// UNROLL: beads whose records are loaded together (1 inside the fused step,
// where registers are short)
template <typename R, bool PER, int UNROLL>
__device__ __forceinline__ void gather_force(const LbArgs& A, const BoxDesc& b,
                                             unsigned long long cmask, int x, int y, int z, R& gx,
                                             R& gy, R& gz) {
  // records and sums in FP64 (the bead impulses cancel on shared nodes),
  // rounded to the collision's precision once
  const double* rd = (const double*)A.rec_d;
  const double* rp = (const double*)A.rec_dp;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int c = 0; c < b.chain_count && c < MAX_BOX_CHAINS; c++) {
    if (!((cmask >> c) & 1ull)) continue;
    const int gc = b.chain_first + c;
    const int* bb = A.bbox + 6 * gc;
    if (z < bb[2] || z > bb[5]) continue;
    if (!(x >= bb[0] && x <= bb[3] && y >= bb[1] && y <= bb[4])) continue;
    const ChainDesc& ch = A.chains[gc];
    // no branch per bead (a bead whose stencil misses the node subtracts a
    // selected zero), so the record loads of consecutive beads overlap
#pragma unroll UNROLL
    for (int jb = ch.first; jb < ch.first + ch.nb; jb++) {
      const int4 bs = A.rec_base[jb];
      int ox = x - bs.x, oy = y - bs.y, oz = z - bs.z;
      if (PER) {
        if ((b.pmask & 1) && ox < 0) ox += b.nx;
        if ((b.pmask & 2) && oy < 0) oy += b.ny;
        if ((b.pmask & 4) && oz < 0) oz += b.nz;
      }
      const bool hit = (unsigned)ox <= 1u && (unsigned)oy <= 1u && (unsigned)oz <= 1u;
      const double w = (ox ? rd[3 * jb] : 1.0 - rd[3 * jb]) *
                       (oy ? rd[3 * jb + 1] : 1.0 - rd[3 * jb + 1]) *
                       (oz ? rd[3 * jb + 2] : 1.0 - rd[3 * jb + 2]);
      const double px = rp[3 * jb], py = rp[3 * jb + 1], pz = rp[3 * jb + 2];
      sx -= hit ? w * px : 0.0;
      sy -= hit ? w * py : 0.0;
      sz -= hit ? w * pz : 0.0;
    }
  }
  gx += (R)sx;
  gy += (R)sy;
  gz += (R)sz;
}

// Interior tile of a non-periodic box whose population groups (0..9 and
// 10..18) each span less than 4 GiB: every load is one 32-bit offset add on
// a per-thread node offset plus a scalar (uniform) group base.
template <int S, int COLL, int BS, bool EXT>
__device__ __forceinline__ void tile_fast(const LbArgs& A, const BoxDesc& b, const Item& it,
                                          const typename Store<S>::T* src,
                                          typename Store<S>::T* dst, bool pre, long long step,
                                          typename Store<S>::R rho0,
                                          typename Store<S>::R omega, typename Store<S>::R omb,
                                          typename Store<S>::R omg) {
  using St = Store<S>;
  using T = typename St::T;
  using R = typename St::R;
  constexpr unsigned SB = sizeof(T);
  const unsigned nx = (unsigned)b.nx, ny = (unsigned)b.ny;
  const unsigned rs = (unsigned)Q * nx;   // row-block stride (elements)
  const unsigned ps = rs * ny;            // plane stride
  const char* __restrict__ s0 = (const char*)src;
  char* __restrict__ d0 = (char*)dst;
  unsigned so[Q], doff[Q];
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const int delta = pre ? 0 : CX[i] + CY[i] * (int)rs + CZ[i] * (int)ps;
    so[i] = (unsigned)i * nx * SB - (unsigned)delta * SB;
    doff[i] = (unsigned)i * nx * SB;
  }
  const float dc0 = b.dec[0], dc1 = b.dec[1], dc2 = b.dec[2];
  const R sc = (R)b.s2;
  const int plane = it.ex * it.ey;
  Ext<R> ext{};
  if constexpr (EXT) ext = make_ext<R>(A, b, step);
#pragma unroll 1
  for (int p = threadIdx.x; p < plane; p += BS) {
    const int x = it.x0 + p % it.ex;
    const int y = it.y0 + p / it.ex;
    unsigned voff = (((unsigned)it.z0 * ny + (unsigned)y) * rs + (unsigned)x) * SB;
#pragma unroll 1
    for (int z = it.z0; z < it.z0 + it.ez; z++, voff += ps * SB) {
      R d[Q];
#pragma unroll
      for (int i = 0; i < Q; i++) {
        const T v = *(const T*)(s0 + (voff + so[i]));
        const float k = WCLS[i] == 0 ? dc0 : (WCLS[i] == 1 ? dc1 : dc2);
        d[i] = St::dec(v, k);
      }
      if constexpr (EXT) {
        ext.node = ((unsigned)z * ny + (unsigned)y) * nx + (unsigned)x;
        collide_ext<R, COLL, comp_weights<S>(), S == 2>(d, (R)0, (R)0, (R)0, rho0, omega, omb, omg, ext, sc);
      } else {
        collide_any<R, COLL, comp_weights<S>(), S == 2>(d, (R)0, (R)0, (R)0, rho0, omega, omb, omg, sc);
      }
      const unsigned hn = dither_node(((unsigned)z * ny + (unsigned)y) * nx + (unsigned)x, (unsigned)step);
#pragma unroll
      for (int i = 0; i < Q; i++) {
        *(T*)(d0 + (voff + doff[i])) = St::keep(d[i], dither_pop(hn, i));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Row items: each lane owns V consecutive nodes of one x-row, held as W 32-bit
// words (V = 2W FP16 or W FP32 values), and moves every population with one
// aligned W-word load and one W-word store.  The interior rows (y, z) of a box
// (1 <= y <= ny-2, 1 <= z <= nz-2), each cut into L = nx / V lane groups, are
// numbered consecutively, and a workgroup walks BS consecutive groups per
// iteration, so rows may straddle wavefronts and every lane is busy for any
// nx divisible by V.  The pull's +-1 shift in x is an element selection
// inside the lane's vector plus one element of the neighbouring group: a lane
// shuffle inside the wavefront, or a direct load for the first and last lane
// of a wavefront.  The groups holding x = 0 or x = nx-1 store the boundary
// equilibrium of that node (face -x or +x), so every store is a full vector.
template <int S, int W>
struct RowVec {
  using T = typename Store<S>::T;
  static constexpr int EPW = 4 / (int)sizeof(T);  // elements per 32-bit word
  static constexpr int V = W * EPW;               // nodes per lane
};

// Buffer resource over [base, base + bytes) (raw, stride 0; gfx9 word 3):
// a lane addresses it with one 32-bit offset, a population with a scalar
// offset, and accesses past the end read zero / are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, long long bytes) {
  const int n = bytes >= 0xffffffffLL ? (int)0xffffffffu : (int)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, n, 0x00020000);
}

template <int W>
__device__ __forceinline__ void vload(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff,
                                      unsigned (&w)[W]) {
  if constexpr (W == 1) {
    w[0] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, soff, LB_LOAD_POLICY);
  } else if constexpr (W == 2) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, soff, LB_LOAD_POLICY);
    w[0] = v[0];
    w[1] = v[1];
  } else if constexpr (W == 3) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b96(r, (int)voff, soff, LB_LOAD_POLICY);
    w[0] = v[0];
    w[1] = v[1];
    w[2] = v[2];
  } else {
    static_assert(W == 4, "row vectors are 1 to 4 words");
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, soff, LB_LOAD_POLICY);
    w[0] = v[0];
    w[1] = v[1];
    w[2] = v[2];
    w[3] = v[3];
  }
}

template <int W>
__device__ __forceinline__ void vstore(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff,
                                       const unsigned (&w)[W]) {
  if constexpr (W == 1) {
    __builtin_amdgcn_raw_buffer_store_b32(w[0], r, (int)voff, soff, LB_STORE_POLICY);
  } else if constexpr (W == 2) {
    __attribute__((ext_vector_type(2))) unsigned v;
    v[0] = w[0];
    v[1] = w[1];
    __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)voff, soff, LB_STORE_POLICY);
  } else if constexpr (W == 3) {
    __attribute__((ext_vector_type(3))) unsigned v;
    v[0] = w[0];
    v[1] = w[1];
    v[2] = w[2];
    __builtin_amdgcn_raw_buffer_store_b96(v, r, (int)voff, soff, LB_STORE_POLICY);
  } else {
    __attribute__((ext_vector_type(4))) unsigned v;
    v[0] = w[0];
    v[1] = w[1];
    v[2] = w[2];
    v[3] = w[3];
    __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)voff, soff, LB_STORE_POLICY);
  }
}

// element e of a lane's words, e in [-1, V]: -1 is the left neighbour's last
// element (held in the high bits of `left`), V the right neighbour's first
// (low bits of `right`)
template <int S, int W>
__device__ __forceinline__ typename Store<S>::T velem(const unsigned (&w)[W], unsigned left,
                                                      unsigned right, int e) {
  using T = typename Store<S>::T;
  constexpr int V = RowVec<S, W>::V;
  if constexpr (sizeof(T) == 2) {
    unsigned short h;
    if (e == -1) h = (unsigned short)(left >> 16);
    else if (e == V) h = (unsigned short)(right & 0xffffu);
    else h = (unsigned short)((e & 1) ? (w[e >> 1] >> 16) : (w[e >> 1] & 0xffffu));
    return __builtin_bit_cast(T, h);
  } else {
    const unsigned u = e == -1 ? left : (e == V ? right : w[e]);
    return __builtin_bit_cast(T, u);
  }
}

// Encode a value into element e of a lane vector: FP16 rounds stochastically
// straight into its half of the packed word, the other half kept (the x-face
// node of a row overwrites an element after its neighbour's).
template <int S, int W>
__device__ __forceinline__ void vput_enc(unsigned (&w)[W], int e, typename Store<S>::R v, float k,
                                         unsigned r) {
  if constexpr (S == 2) {
#pragma clang fp contract(off)
    Store<2>::keep_into(w[e >> 1], (e & 1) != 0, v * k, r, false);
  } else {
    w[e] = __builtin_bit_cast(unsigned, Store<S>::enc(v, k, r));
  }
}
// the same for a value already in storage units (collide_any with WS), the
// elements written in order (element 2j starts word j)
template <int S, int W>
__device__ __forceinline__ void vput_keep(unsigned (&w)[W], int e, typename Store<S>::R x,
                                          unsigned r) {
  if constexpr (S == 2) {
    Store<2>::keep_into(w[e >> 1], (e & 1) != 0, x, r, true);
  } else {
    w[e] = __builtin_bit_cast(unsigned, Store<S>::keep(x, r));
  }
}

template <int S, int W>
__device__ __forceinline__ void vput(unsigned (&w)[W], int e, typename Store<S>::T val) {
  using T = typename Store<S>::T;
  if constexpr (sizeof(T) == 2) {
    const unsigned h = (unsigned)__builtin_bit_cast(unsigned short, val);
    unsigned& word = w[e >> 1];
    word = (e & 1) ? ((word & 0xffffu) | (h << 16)) : ((word & 0xffff0000u) | h);
  } else {
    w[e] = __builtin_bit_cast(unsigned, val);
  }
}

template <int S, int W, int COLL, bool PRE, int BS, bool EXT>
__device__ __forceinline__ void tile_rows(const LbArgs& A, const BoxDesc& b, const Item& it,
                                          const typename Store<S>::T* src,
                                          typename Store<S>::T* dst, long long step,
                                          typename Store<S>::R rho0,
                                          typename Store<S>::R omega, typename Store<S>::R omb,
                                          typename Store<S>::R omg) {
  using St = Store<S>;
  using T = typename St::T;
  using R = typename St::R;
  constexpr int V = RowVec<S, W>::V;
  constexpr int SB = (int)sizeof(T);
  const int nx = b.nx, ny = b.ny, nyi = b.ny - 2;
  const int L = nx / V;                            // lane groups per row
  const int nxb = nx * SB;                         // bytes per population row
  const int yl = b.ylog, ym = (1 << b.ylog) - 1;
  const int pib = nxb << yl;                       // bytes per population in a block of Y rows
  const int bkb = Q * pib;                         // bytes per block of Y rows
  const long long psb = (long long)Q * nxb * ny;   // bytes per plane
  const long long box_bytes = psb * b.nz;
  const int g_last = L * nyi * (b.nz - 2) - 1;     // last group of the box
  const int q_end = it.x0 + it.ex;
  const float dc0 = b.dec[0], dc1 = b.dec[1], dc2 = b.dec[2];
  const float ec0 = b.enc[0], ec1 = b.enc[1], ec2 = b.enc[2];
  const R sc = (R)b.s2;
  const int lane = (int)(threadIdx.x & 63);
  const unsigned lane_l = (unsigned)(lane - 1) & 63u, lane_r = (unsigned)(lane + 1) & 63u;
  // population i of the node sits at vo[c_y] + soff(i) from the iteration's
  // base plane (one plane below its first row): offsets >= 0; vo holds the
  // lane's line offsets for y - c_y, c_y = 1, 0, -1
  const int ps = (int)psb;
  auto ybytes = [&](int yy) { return (yy >> yl) * bkb + (yy & ym) * nxb; };
  Ext<R> ext{};
  if constexpr (EXT) ext = make_ext<R>(A, b, step);
#pragma unroll 1
  for (int qb = it.x0; qb < q_end; qb += BS) {
    const int zf = 1 + (qb / L) / nyi;             // first plane of this iteration
    const long long base = (long long)(zf - 1) * psb;
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc((const char*)src + base, box_bytes - base);
    const __amdgpu_buffer_rsrc_t rdst = make_rsrc((const char*)dst + base, box_bytes - base);
    const int q = qb + (int)threadIdx.x;
    const bool act = q < q_end;
    // groups past the item still load real data (their own group, or the last
    // group of the box): the last active lane's right neighbour may be one
    const int qq = q < g_last ? q : g_last;
    const int row = qq / L;
    const int c = qq - row * L;
    const int zi = row / nyi;
    const int y = 1 + row - zi * nyi, z = 1 + zi;
    const int x0 = c * V;
    const int zrel = (z - zf) * ps + x0 * SB;
    const unsigned vo[3] = {(unsigned)(zrel + ybytes(y - 1)), (unsigned)(zrel + ybytes(y)),
                            (unsigned)(zrel + ybytes(y + 1))};   // indexed 1 - c_y
    const unsigned voff = vo[1];
    unsigned raw[Q][W];
#pragma unroll
    for (int i = 0; i < Q; i++) {
      const int so = i * pib + (PRE ? ps : (1 - CZ[i]) * ps);
      vload<W>(rsrc, PRE ? voff : vo[1 - CY[i]], so, raw[i]);
    }
    // boundary velocity of the lane's x-face node (first or last lane group of
    // a row; L >= 2, so at most one), written by k_xface for this step and
    // loaded together with the populations
    const bool xface = act && (c == 0 || c == L - 1);
    const int xside = c == 0 ? 0 : 1;
    float xu[3] = {0.0f, 0.0f, 0.0f};
    if (xface) {
      const float* xf = A.xface + b.xf_off + 3 * ((xside * (b.nz - 2) + (z - 1)) * nyi + (y - 1));
      xu[0] = xf[0];
      xu[1] = xf[1];
      xu[2] = xf[2];
    }
    // neighbour elements of the populations shifted in x
    unsigned left[Q], right[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) {
      left[i] = 0u;
      right[i] = 0u;
      if (!PRE && CX[i] == 1) left[i] = __shfl(raw[i][W - 1], (int)lane_l, 64);
      if (!PRE && CX[i] == -1) right[i] = __shfl(raw[i][0], (int)lane_r, 64);
    }
    if (!PRE) {
      // first / last lane of the wavefront: the neighbour group sits in
      // another wavefront; load its element directly (in bounds: c > 0 means
      // x0 - 1 >= 0, c < L - 1 means x0 + V <= nx - 1)
      if (lane == 0 && c != 0) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
          if (CX[i] != 1) continue;
          const int so = i * pib + (1 - CZ[i]) * ps - SB;
          const int vl = (int)vo[1 - CY[i]];
          if constexpr (SB == 2)
            left[i] = (unsigned)__builtin_amdgcn_raw_buffer_load_b16(rsrc, vl, so, 0) << 16;
          else
            left[i] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, vl, so, 0);
        }
      }
      if (lane == 63 && c != L - 1) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
          if (CX[i] != -1) continue;
          const int so = i * pib + (1 - CZ[i]) * ps + V * SB;
          const int vr = (int)vo[1 - CY[i]];
          if constexpr (SB == 2)
            right[i] = (unsigned)__builtin_amdgcn_raw_buffer_load_b16(rsrc, vr, so, 0);
          else
            right[i] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, vr, so, 0);
        }
      }
    }
    unsigned out[Q][W];
#pragma unroll
    for (int k = 0; k < V; k++) {
      R d[Q];
#pragma unroll
      for (int i = 0; i < Q; i++) {
        const int e = PRE ? k : k - CX[i];
        const float kd = WCLS[i] == 0 ? dc0 : (WCLS[i] == 1 ? dc1 : dc2);
        d[i] = St::dec(velem<S, W>(raw[i], left[i], right[i], e), kd);
      }
      const int x = x0 + k;
      if constexpr (EXT) {
        ext.node = ((unsigned)z * (unsigned)ny + (unsigned)y) * (unsigned)nx + (unsigned)x;
        collide_ext<R, COLL, comp_weights<S>(), S == 2>(d, (R)0, (R)0, (R)0, rho0, omega, omb, omg, ext, sc);
      } else {
        collide_any<R, COLL, comp_weights<S>(), S == 2>(d, (R)0, (R)0, (R)0, rho0, omega, omb, omg, sc);
      }
      const unsigned hn =
          dither_node(((unsigned)z * (unsigned)ny + (unsigned)y) * (unsigned)nx + (unsigned)x, (unsigned)step);
#pragma unroll
      for (int i = 0; i < Q; i++) {
        const float ke = WCLS[i] == 0 ? ec0 : (WCLS[i] == 1 ? ec1 : ec2);
        vput_keep<S, W>(out[i], k, d[i], dither_pop(hn, i));
      }
    }
    // x-face nodes of this row: boundary equilibrium at t_n (faces -x, +x)
    if (xface) {
      R eq[Q];
      eq_dev<R>((R)0, rho0, xu[0], xu[1], xu[2], eq);
      const unsigned xn = xside == 0 ? 0u : (unsigned)(nx - 1);
      const unsigned hx =
          dither_node(((unsigned)z * (unsigned)ny + (unsigned)y) * (unsigned)nx + xn, (unsigned)step);
      // element indices stay compile-time constants (registers, not scratch)
      if (xside == 0) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
          const float ke = WCLS[i] == 0 ? ec0 : (WCLS[i] == 1 ? ec1 : ec2);
          vput_enc<S, W>(out[i], 0, eq[i], ke, dither_pop(hx, i));
        }
      } else {
#pragma unroll
        for (int i = 0; i < Q; i++) {
          const float ke = WCLS[i] == 0 ? ec0 : (WCLS[i] == 1 ? ec1 : ec2);
          vput_enc<S, W>(out[i], V - 1, eq[i], ke, dither_pop(hx, i));
        }
      }
    }
    if (act) {
#pragma unroll
      for (int i = 0; i < Q; i++) vstore<W>(rdst, voff, i * pib + ps, out[i]);
    }
  }
}

// Face rows of a row box: the rows y = 0, y = ny-1 (1 <= z <= nz-2) and all
// rows of the planes z = 0, z = nz-1, cut into the same lane groups, numbered
// plane z = 0 (rows y = 0..ny-1), plane z = nz-1, then for each interior z its
// rows y = 0 and y = ny-1.  Every node takes the boundary equilibrium at t_n
// with the face of lowest index it lies on (-x, +x, -y, +y, -z, +z); a row
// stores, one W-word vector each, the populations whose target line
// (y + c_y, z + c_z) is an interior line -- the only ones ever read.
template <int S, int W, int BS>
__device__ __forceinline__ void face_rows(const BoxDesc& b, const Item& it,
                                          typename Store<S>::T* dst, long long step,
                                          typename Store<S>::R rho0) {
  using St = Store<S>;
  using R = typename St::R;
  constexpr int V = RowVec<S, W>::V;
  constexpr int SB = (int)sizeof(typename St::T);
  const int nx = b.nx, ny = b.ny, nz = b.nz;
  const int L = nx / V;
  const long long nxb = (long long)nx * SB, psb = Q * nxb * ny;
  const int yl = b.ylog, ym = (1 << b.ylog) - 1;
  const long long pib = nxb << yl, bkb = Q * pib;
  const float ec0 = b.enc[0], ec1 = b.enc[1], ec2 = b.enc[2];
  const int q_end = it.x0 + it.ex;
  const BcTime<R> tm = bc_time<R>(b, step);
#pragma unroll 1
  for (int q = it.x0 + (int)threadIdx.x; q < q_end; q += BS) {
    const int fr = q / L;
    const int c = q - fr * L;
    int y, z;
    if (fr < ny) {
      y = fr;
      z = 0;
    } else if (fr < 2 * ny) {
      y = fr - ny;
      z = nz - 1;
    } else {
      const int k = fr - 2 * ny;
      z = 1 + (k >> 1);
      y = (k & 1) ? ny - 1 : 0;
    }
    const int x0 = c * V;
    unsigned out[Q][W];
#pragma unroll
    for (int k = 0; k < V; k++) {
      const int x = x0 + k;
      const int f = x == 0 ? 0 : (x == nx - 1 ? 1 : (y == 0 ? 2 : (y == ny - 1 ? 3 : (z == 0 ? 4 : 5))));
      const int qn[3] = {x, y, z};
      R u[3];
      boundary_velocity<R>(b, f, qn, tm, u);
      R eq[Q];
      eq_dev<R>((R)0, rho0, u[0], u[1], u[2], eq);
      const unsigned hn =
          dither_node(((unsigned)z * (unsigned)ny + (unsigned)y) * (unsigned)nx + (unsigned)x, (unsigned)step);
#pragma unroll
      for (int i = 0; i < Q; i++) {
        const float ke = WCLS[i] == 0 ? ec0 : (WCLS[i] == 1 ? ec1 : ec2);
        vput_enc<S, W>(out[i], k, eq[i], ke, dither_pop(hn, i));
      }
    }
    char* row = (char*)dst + (long long)z * psb + (long long)(y >> yl) * bkb + (long long)(y & ym) * nxb +
                (long long)x0 * SB;
#pragma unroll
    for (int i = 0; i < Q; i++) {
      // only populations that stream into an interior line are ever read
      const int ty = y + CY[i], tz = z + CZ[i];
      if (ty < 1 || ty > ny - 2 || tz < 1 || tz > nz - 2) continue;
      char* p = row + i * pib;
      if constexpr (W == 1) *(unsigned*)p = out[i][0];
      else if constexpr (W == 2) *(uint2*)p = make_uint2(out[i][0], out[i][1]);
      else if constexpr (W == 3) *(uint3*)p = make_uint3(out[i][0], out[i][1], out[i][2]);
      else *(uint4*)p = make_uint4(out[i][0], out[i][1], out[i][2], out[i][3]);
    }
  }
}

// Interior tile, general addressing (periodic axes wrap, any box size).
// In-place streaming (aa): an even step reads each node in place and writes
// f*_i into its own slot OPP[i]; an odd step reads those (LAYOUT_SWAP) and
// writes f*_i into slot i of node x + c_i, where the next even step reads it
// in place.  Each slot is read and written by one node only.
template <int S, int COLL, bool PER, int BS, bool EXT>
__device__ __forceinline__ void tile_generic(const LbArgs& A, const BoxDesc& b, const Item& it,
                                             const typename Store<S>::T* src,
                                             typename Store<S>::T* dst, int layout, bool aa,
                                             long long step,
                                             unsigned long long cmask, typename Store<S>::R rho0,
                                             typename Store<S>::R omega, typename Store<S>::R omb,
                                             typename Store<S>::R omg) {
  using St = Store<S>;
  using R = typename St::R;
  const int plane = it.ex * it.ey;
  const R sc = (R)b.s2;
  Ext<R> ext{};
  if constexpr (EXT) ext = make_ext<R>(A, b, step);
#pragma unroll 1
  for (int p = threadIdx.x; p < plane; p += BS) {
    const int x = it.x0 + p % it.ex;
    const int y = it.y0 + p / it.ex;
#pragma unroll 1
    for (int z = it.z0; z < it.z0 + it.ez; z++) {
      R d[Q];
      load_pre<S, PER>(src, b, x, y, z, layout, d);
      R gx = 0, gy = 0, gz = 0;
      if (cmask) gather_force<R, PER, 1>(A, b, cmask, x, y, z, gx, gy, gz);
      if constexpr (EXT) {
        ext.node = (unsigned)(((int64_t)z * b.ny + y) * b.nx + x);
        collide_ext<R, COLL, comp_weights<S>(), S == 2>(d, gx, gy, gz, rho0, omega, omb, omg, ext, sc);
      } else {
        collide_any<R, COLL, comp_weights<S>(), S == 2>(d, gx, gy, gz, rho0, omega, omb, omg, sc);
      }
      const unsigned hn = dither_node((unsigned)(((int64_t)z * b.ny + y) * b.nx + x), (unsigned)step);
      if (aa && !(step & 1)) {
#pragma unroll
        for (int i = 0; i < Q; i++)
          dst[aidx(b, OPP[i], x, y, z)] = St::keep(d[i], dither_pop(hn, i));
      } else if (aa) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
          int tx = x + CX[i], ty = y + CY[i], tz = z + CZ[i];
          if (PER) {
            if (b.pmask & 1) tx = wrapc(tx, b.nx);
            if (b.pmask & 2) ty = wrapc(ty, b.ny);
            if (b.pmask & 4) tz = wrapc(tz, b.nz);
          }
          dst[aidx(b, i, tx, ty, tz)] = St::keep(d[i], dither_pop(hn, i));
        }
      } else {
#pragma unroll
        for (int i = 0; i < Q; i++)
          dst[aidx(b, i, x, y, z)] = St::keep(d[i], dither_pop(hn, i));
      }
    }
  }
}

// ----------------------------------------------------------- fused step

// Resident waves per SIMD the step kernel is compiled for: the most that fit
// without spilling (VGPRs per lane: 512 / waves).  FP64 BGK 2 (197-228 VGPRs),
// MRT 3 (147-150), MRT with ghost rate 1 4 (124-127); FP32 3-4 (94-122); FP16
// MRT 3 (101-144), FP16 BGK 2 (127-178).  Left to itself the allocator lands
// just above a boundary and runs one wave fewer, measured 5-11% slower.
constexpr int lb_min_waves(int S, int COLL) {
  return S == 0 ? (COLL == 0 ? 2 : (COLL == 1 ? 3 : 4))
#ifdef LB_MIN_WAVES
                : LB_MIN_WAVES;
#else
                : (S == 1 ? (COLL == 0 ? 3 : 4) : (COLL == 0 ? 2 : 3));
#endif
}

// The extended collision (body force, thermal noise) holds more registers:
// its instantiations ask for two resident waves per SIMD.
constexpr int lb_min_waves_ext(int S, int COLL, bool EXT) { return EXT ? 2 : lb_min_waves(S, COLL); }

// AA: the instantiation for in-place streaming on boxes without periodic
// axes (no row items, no stores of the two-buffer step); the periodic
// instantiation takes either streaming from A.aa.
template <int S, int COLL, bool PER, int BS = WG, bool EXT = false, bool AA = false>
__global__ __launch_bounds__(BS, lb_min_waves_ext(S, COLL, EXT)) void k_lb(LbArgs A) {
  using St = Store<S>;
  using T = typename St::T;
  using R = typename St::R;

  const int tid = threadIdx.x;
  put_stamp(A.stamp_first);
  put_stamp(A.stamp_lb);
  const bool skip =
      __hip_atomic_load(&A.st->err_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ERR_NONE;
  if (skip) return;  // uniform: the latch is set before this launch or not at all
  const long long step = A.st->step;
  const int par = (int)(step & 1);
  const R rho0 = (R)A.rho0, omega = (R)A.omega, omb = (R)A.om_bulk, omg = (R)A.om_ghost;
  const T* __restrict__ srcA = (const T*)(par ? A.a1 : A.a0);
  T* __restrict__ dstA = (T*)(par ? A.a0 : A.a1);
  const bool pre = A.pre != 0;
  const bool aa = AA || (PER && A.aa);

  for (int e = blockIdx.x; e < A.n_entries; e += gridDim.x) {
    const int ii = A.order[e];
    if (ii < 0) continue;
    const Item it = A.items[ii];
    const BoxDesc& b = A.boxes[it.box];
    const T* __restrict__ src = srcA + b.off;
    T* __restrict__ dst = dstA + b.off;

    if (it.kind == ITEM_ROWS) {
      // row boxes are never periodic: their chains couple in k_force
      if constexpr (S != 0 && !PER && !AA) {
#define LB_ROWS(PR)                                                                    \
  do {                                                                                 \
    if (b.vw == 3)                                                                     \
      tile_rows<S, 3, COLL, PR, BS, EXT>(A, b, it, src, dst, step, rho0, omega, omb, omg); \
    else                                                                               \
      tile_rows<S, 2, COLL, PR, BS, EXT>(A, b, it, src, dst, step, rho0, omega, omb, omg); \
  } while (0)
        if (pre) LB_ROWS(true);
        else LB_ROWS(false);
#undef LB_ROWS
      }
    } else if (it.kind == ITEM_FACE_ROWS) {
      if constexpr (S != 0 && !PER && !AA) {
        if (b.vw == 3) face_rows<S, 3, BS>(b, it, dst, step, rho0);
        else face_rows<S, 2, BS>(b, it, dst, step, rho0);
      }
    } else if (it.kind == ITEM_TILE) {
      // chains whose stencil box overlaps this tile, periodic boxes only (the
      // chains of the other boxes couple in k_force)
      unsigned long long cmask = 0;
      const bool gather = (PER && b.pmask) || aa;
      for (int c = 0; gather && c < b.chain_count && c < MAX_BOX_CHAINS; c++) {
        const int* bb = A.bbox + 6 * (b.chain_first + c);
        const bool ov = bb[0] <= it.x0 + it.ex - 1 && bb[3] >= it.x0 && bb[1] <= it.y0 + it.ey - 1 &&
                        bb[4] >= it.y0 && bb[2] <= it.z0 + it.ez - 1 && bb[5] >= it.z0;
        if (ov) cmask |= 1ull << c;
      }
      if (!PER && !AA && b.fast) {
        tile_fast<S, COLL, BS, EXT>(A, b, it, src, dst, pre, step, rho0, omega, omb, omg);
      } else {
        const int layout = aa ? aa_layout(step) : (pre ? LAYOUT_PLACE : LAYOUT_PULL);
        tile_generic<S, COLL, PER, BS, EXT>(A, b, it, src, dst, layout, aa, step, cmask, rho0,
                                            omega, omb, omg);
      }
    } else {
      // boundary chunk: equilibrium at rho0 and u_b(t_n) for the populations
      // that stream into the interior
      const BcTime<R> tm = bc_time<R>(b, step);
      for (int k = it.x0 + tid; k < it.x0 + it.ex; k += BS) {
        int r = 0, kk = k;
        while (r < b.n_rect - 1 && kk >= b.rect_cnt[r]) {
          kk -= b.rect_cnt[r];
          r++;
        }
        const int f = b.rect_face[r];
        const int lx = b.rect_len[r][0], ly = b.rect_len[r][1];
        int q[3];
        q[0] = b.rect_start[r][0] + kk % lx;
        q[1] = b.rect_start[r][1] + (kk / lx) % ly;
        q[2] = b.rect_start[r][2] + kk / (lx * ly);
        R u[3];
        boundary_velocity<R>(b, f, q, tm, u);
        R eq[Q];
        eq_dev<R>((R)0, rho0, u[0], u[1], u[2], eq);
        const unsigned hn =
            dither_node((unsigned)(((int64_t)q[2] * b.ny + q[1]) * b.nx + q[0]), (unsigned)step);
#pragma unroll
        for (int i = 1; i < Q; i++) {
          int tx = q[0] + CX[i], ty = q[1] + CY[i], tz = q[2] + CZ[i];
          if (PER) {
            if (b.pmask & 1) tx = wrapc(tx, b.nx);
            if (b.pmask & 2) ty = wrapc(ty, b.ny);
            if (b.pmask & 4) tz = wrapc(tz, b.nz);
          }
          if (!is_interior(b, tx, ty, tz)) continue;
          // in-place streaming: an even step leaves the population in the
          // node's opposite slot, an odd step in slot i of the target node
          const T v = St::enc(eq[i], b.enc[WCLS[i]], dither_pop(hn, i));
          if (aa && !(step & 1))
            dst[aidx(b, OPP[i], q[0], q[1], q[2])] = v;
          else if (aa)
            dst[aidx(b, i, tx, ty, tz)] = v;
          else
            dst[aidx(b, i, q[0], q[1], q[2])] = v;
        }
      }
    }
  }
}

// ----------------------------------------------------------- x-face velocities
// Before the fused step: the boundary velocity u_b(y, t_n) of every x-face node
// of the interior rows of the row boxes (faces -x and +x, interior y and z), so
// that the row lanes that own those nodes read three floats instead of
// evaluating the boundary source with dependent loads.  Node k of a box:
// k = side (ny-2)(nz-2) + (z-1)(ny-2) + (y-1), velocity at xface[xf_off + 3k].
// ------------------------------------------------------------ chain forcing
// Chains of non-periodic boxes couple to the fluid in a pass of their own,
// right after the fused step: the interior nodes of each chain's stencil box
// collide again from the same pre-collision populations (the fused step reads
// one buffer and writes the other, so they are intact), now with the spread
// force of every chain of the box whose stencil box holds the node (Guo
// forcing, the same collision), and overwrite what the fused step stored
// there.  The fused step then never gathers spread force for these boxes.
// Where the stencil boxes of two chains overlap, both workgroups compute the
// node and store the same values.  One workgroup per chain.  On steps that
// have no check pass it also ends the step (step index advance), which then
// needs no launch of its own.
template <int S, int COLL, bool PER, bool EXT = false>
__global__ __launch_bounds__(WG) void k_force(LbArgs A) {
  using St = Store<S>;
  using T = typename St::T;
  using R = typename St::R;
  const int gc = blockIdx.x;
  // inputs read before the timestamp store (see k_check)
  const bool latched =
      __hip_atomic_load(&A.st->err_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ERR_NONE;
  const long long step = A.st->step;
  const ChainDesc ch = A.chains[gc];
  const BoxDesc b = A.boxes[ch.box];
  int bb[6];
#pragma unroll
  for (int a = 0; a < 6; a++) bb[a] = A.bbox[6 * gc + a];
  put_stamp(A.stamp_after);
  if (latched) return;  // uniform: set before this launch or not at all
  if (!b.pmask) {       // periodic boxes gather inside the fused step
    const int par = (int)(step & 1);
    const T* __restrict__ src = (const T*)(par ? A.a1 : A.a0) + b.off;
    T* __restrict__ dst = (T*)(par ? A.a0 : A.a1) + b.off;
    const R rho0 = (R)A.rho0, omega = (R)A.omega, omb = (R)A.om_bulk, omg = (R)A.om_ghost;
    const R sc = (R)b.s2;
    const unsigned long long all =
        b.chain_count >= MAX_BOX_CHAINS ? ~0ull : (1ull << b.chain_count) - 1ull;
    const int lx = bb[3] - bb[0] + 1, ly = bb[4] - bb[1] + 1, lz = bb[5] - bb[2] + 1;
    const int n = (lx > 0 && ly > 0 && lz > 0) ? lx * ly * lz : 0;
#pragma unroll 1
    for (int p = threadIdx.x; p < n; p += WG) {
      const int x = bb[0] + p % lx, y = bb[1] + (p / lx) % ly, z = bb[2] + p / (lx * ly);
      if (!is_interior(b, x, y, z)) continue;
      R d[Q];
      load_pre<S, PER>(src, b, x, y, z, A.pre != 0, d);
      R gx = 0, gy = 0, gz = 0;
      gather_force<R, PER, 4>(A, b, all, x, y, z, gx, gy, gz);
      if constexpr (EXT) {
        // the same body force and noise k_lb gave the node (same counter)
        Ext<R> ext = make_ext<R>(A, b, step);
        ext.node = (unsigned)(((int64_t)z * b.ny + y) * b.nx + x);
        collide_ext<R, COLL, comp_weights<S>(), S == 2>(d, gx, gy, gz, rho0, omega, omb, omg, ext, sc);
      } else {
        collide_any<R, COLL, comp_weights<S>(), S == 2>(d, gx, gy, gz, rho0, omega, omb, omg, sc);
      }
      const unsigned hn = dither_node((unsigned)(((int64_t)z * b.ny + y) * b.nx + x), (unsigned)step);
#pragma unroll
      for (int i = 0; i < Q; i++)
        dst[aidx(b, i, x, y, z)] = St::keep(d[i], dither_pop(hn, i));
    }
  }
  // On steps without a check pass (advance set) the last workgroup to take a
  // ticket ends the step instead of a separate launch: every workgroup has
  // read the step index before its ticket, and nothing is published for
  // another workgroup, so no fence is needed.
  if (A.advance) {
    __syncthreads();
    if (threadIdx.x == 0 && atomicAdd(&A.st->tickets, 1) == (int)gridDim.x - 1) {
      atomicExch(&A.st->tickets, 0);
      A.st->step = step + 1;
    }
  }
}

constexpr int XF_NODES = 4;  // x-face nodes per lane
constexpr int XF_ITEM = XF_NODES * 64;  // nodes per x-face work item (one wavefront)

template <int S>
__device__ __forceinline__ void xface_wave(const BoxDesc* __restrict__ boxes,
                                           const int4* __restrict__ items, int item,
                                           float* __restrict__ xface, DevState* __restrict__ st,
                                           long long* stamp) {
  using R = typename Store<S>::R;
  // inputs read before the timestamp store (see k_check)
  const bool latched =
      __hip_atomic_load(&st->err_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ERR_NONE;
  const long long step = st->step;
  const int4 w = items[item];  // box, first node, node count
  const BoxDesc b = boxes[w.x];
  put_stamp(stamp);
  if (latched) return;
  const int lane = (int)threadIdx.x & 63;
  const int nyi = b.ny - 2, plane = nyi * (b.nz - 2);
  const BcTime<R> tm = bc_time<R>(b, step);
  // XF_NODES independent nodes per lane, unrolled so that their sample loads
  // are in flight together
#pragma unroll
  for (int j = 0; j < XF_NODES; j++) {
    const int k = w.y + lane + j * 64;
    if (k >= w.y + w.z) break;
    const int side = k / plane, r = k - side * plane;
    const int zi = r / nyi, yi = r - zi * nyi;
    const int q[3] = {side == 0 ? 0 : b.nx - 1, 1 + yi, 1 + zi};
    R u[3];
    boundary_velocity<R>(b, side, q, tm, u);
    // one 12-byte store per lane: a wavefront writes 768 contiguous bytes
    struct F3 {
      float c[3];
    };
    *(F3*)(xface + b.xf_off + 3 * k) = F3{{(float)u[0], (float)u[1], (float)u[2]}};
  }
}

// x-face velocities alone (boxes without chains, readout, autotuner trials):
// WG / 64 work items per workgroup, one per wavefront
template <int S>
__global__ __launch_bounds__(WG) void k_xface(LbArgs A) {
  const int item = (int)blockIdx.x * (WG / 64) + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  if (item >= A.n_xf_items) return;
  xface_wave<S>(A.boxes, A.xf_items, item, A.xface, A.st, A.stamp_first);
}

// ----------------------------------------------------------- mass / momentum
// On check steps ((n+1) % K == 0), after the fused step: the interior's mass
// and momentum at t_{n+1}, i.e. every stored population of the arena just
// written whose target node x + c_i is interior (FP64).  Workgroup w covers
// the planes [cz0, cz1) of box cbox, one FP64 partial of each sum per
// workgroup (wave shuffle -> LDS, fixed order); k_finalize adds the partials
// of a box in workgroup order.  A separate pass, so the step itself is the
// same arithmetic on every step.
template <int S, bool PER>
__global__ __launch_bounds__(WG) void k_check(LbArgs A) {
  using St = Store<S>;
  using T = typename St::T;
  __shared__ double sred[4][WG / 64];
  const int tid = threadIdx.x, w = blockIdx.x;
  // everything read before the timestamp store, which the compiler cannot
  // tell apart from the descriptor tables (after it, they would be re-read per
  // lane instead of through scalar loads)
  const bool latched =
      __hip_atomic_load(&A.st->err_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ERR_NONE;
  const long long step = A.st->step;
  const int4 cw = A.check_items[w];  // box, first plane, end plane
  const BoxDesc b = A.boxes[cw.x];
  put_stamp(A.stamp_after);
  if (latched) return;
  if (!(A.reduce_every > 0 && ((step + 1) % A.reduce_every) == 0)) return;
  const int par = (int)(step & 1);
  const T* __restrict__ arena = (const T*)(par ? A.a0 : A.a1) + b.off;  // written by this step
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (!A.aa && !PER && b.nx % 8 == 0) {
    // chunks of 8 consecutive nodes of a row, every population read as
    // 16-byte vectors (rows start 16-byte aligned: box offsets are multiples
    // of 128 elements and 8 nodes span 16 bytes or a multiple of it).  The
    // node's own populations are always inside the box, so all of them are
    // loaded before any is tested (no load waits behind a branch); selects,
    // not products, drop the ones that stream out of the fluid, so that
    // whatever a boundary node holds in them never enters a sum.
    constexpr int NV = 8 * (int)sizeof(T) / 16;
    const int cpr = b.nx / 8;
    const int n_chunks = (cw.z - cw.y) * b.ny * cpr;
    for (int p = tid; p < n_chunks; p += WG) {
      const int row = p / cpr, c = p - row * cpr;
      const int zz = row / b.ny, y = row - zz * b.ny, z = cw.y + zz;
      const int x0 = 8 * c;
      uint4 raw[Q][NV];
#pragma unroll
      for (int i = 0; i < Q; i++) {
        const uint4* src = (const uint4*)(arena + aidx(b, i, x0, y, z));
#pragma unroll
        for (int q = 0; q < NV; q++) raw[i][q] = src[q];
      }
#pragma unroll
      for (int i = 0; i < Q; i++) {
        const int ty = y + CY[i], tz = z + CZ[i];
        const bool row_in = ty >= 1 && ty <= b.ny - 2 && tz >= 1 && tz <= b.nz - 2;
        const T* v = (const T*)raw[i];
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < 8; k++) {
          const int tx = x0 + k + CX[i];
          const double d = (double)St::dec(v[k], b.dec[WCLS[i]]);
          sum += (tx >= 1 && tx <= b.nx - 2) ? d : 0.0;
        }
        sum = row_in ? sum : 0.0;
        acc[0] += sum;
        if (CX[i]) acc[1] += CX[i] * sum;
        if (CY[i]) acc[2] += CY[i] * sum;
        if (CZ[i]) acc[3] += CZ[i] * sum;
      }
    }
  } else {
    // node by node; a slab holds fewer than 2^31 nodes (32-bit indices);
    // loads first and selects after, as above
    const int n_slab = (cw.z - cw.y) * b.ny * b.nx;
    for (int p = tid; p < n_slab; p += WG) {
      const int row = p / b.nx, x = p - row * b.nx;
      const int zz = row / b.ny, y = row - zz * b.ny, z = cw.y + zz;
      T raw[Q];
#pragma unroll
      for (int i = 0; i < Q; i++) raw[i] = arena[aidx(b, i, x, y, z)];
      // where slot i of this node streams to, and along which direction:
      // two buffers and an in-place even step (slot OPP[i] holds f*_OPP[i],
      // moving along -c_i) move it on, an in-place odd step left it in place
      const int mv = A.aa ? ((step & 1) ? 0 : -1) : 1;
      const int dir = A.aa && !(step & 1) ? -1 : 1;
#pragma unroll
      for (int i = 0; i < Q; i++) {
        int tx = x + mv * CX[i], ty = y + mv * CY[i], tz = z + mv * CZ[i];
        if (PER) {
          if (b.pmask & 1) tx = wrapc(tx, b.nx);
          if (b.pmask & 2) ty = wrapc(ty, b.ny);
          if (b.pmask & 4) tz = wrapc(tz, b.nz);
        }
        const double d = (double)St::dec(raw[i], b.dec[WCLS[i]]);
        const double v = is_interior(b, tx, ty, tz) ? d : 0.0;
        acc[0] += v;
        if (CX[i]) acc[1] += dir * CX[i] * v;
        if (CY[i]) acc[2] += dir * CY[i] * v;
        if (CZ[i]) acc[3] += dir * CZ[i] * v;
      }
    }
  }
#pragma unroll
  for (int m = 0; m < 4; m++) {
    const double v = wave_sum(acc[m]);
    if ((tid & 63) == 0) sred[m][tid >> 6] = v;
  }
  __syncthreads();
  if (tid < 4) {
    double s = 0.0;
    for (int k = 0; k < WG / 64; k++) s += sred[tid][k];
    A.partials[4 * w + tid] = s;
  }
}

}  // namespace lbdev
