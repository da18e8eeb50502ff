// Fused pull-stream / boundary / wall-model / MRT-Smagorinsky collision
// kernel for the D3Q19 channel (Algorithm 1 of Xue, Yao, Davidson,
// arXiv 2304.04214), plus the initialisation, import/export, stream-only and
// copy kernels.
//
// Population layout: 64-node bricks.  The 19 populations of the 64 nodes
// (x, y, 64 zc .. 64 zc + 63) are one contiguous block of 19 x 64 elements,
// and bricks are ordered (x, zc, y): element (i, x, y, z) sits at
// ((x zc_n + z/64) ny + y) 1216 + 64 i + z%64.  A wave (64 lanes) owns one
// brick: its 19 stores are one contiguous 4864-byte (float) run, and its pulls
// come from the 3 x 3 neighbouring (x, y) bricks plus one element of the
// z-neighbouring bricks for the +-1 z shifts.
//
// Mapping: one thread per node.  A block is 4 consecutive y rows (4 waves) of
// one (x, z-chunk).  x and y are wave-uniform (scalar registers), so every
// boundary decision is a scalar select and each population load is
// scalar base + per-lane column offset.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "stream.h"



namespace lbm {
namespace {

// Reichardt wall force of a first off-wall cell (Sec. II.C, Eq. (16)-(21)):
// base vector from the tangential part of u_2, projected speed u_hat, u_tau
// from a fixed number of Newton steps on u_tau u+(y u_tau / nu0) = |u_hat|,
// F_w = -sign(u_hat) rho u_tau^2 e_x.  The wall normal is along y.
//
// With the line-averaged model (wall_line set) u_tau is the signed value of
// the cell's wall line, computed by wall_line_kernel from the z-mean of u_hat.
__device__ __forceinline__ void wall_force(const CollideArgs& a, float rho, float uwx, float uwz, float u2x,
                                           float u2z, float& fx, float& fz, float& ut_out, int w, int x) {
  fx = 0.f;
  fz = 0.f;
  ut_out = 0.f;
  const float line = a.wall_line ? a.wall_line[w * a.nx + x] : 0.f;
  if (a.wall_line) ut_out = fabsf(line);
  const float tn2 = u2x * u2x + u2z * u2z;
  if (!(tn2 > 0.f)) return;
  const float itn = 1.f / sqrtf(tn2);
  const float ex = u2x * itn, ez = u2z * itn;
  if (a.wall_line) {
    const float tw = (line > 0.f ? -1.f : 1.f) * rho * line * line;
    fx = tw * ex;
    fz = tw * ez;
    return;
  }
  const float uhat = uwx * ex + uwz * ez;
  if (uhat == 0.f) return;
  const float ut = newton_utau(a, fabsf(uhat));
  const float tw = (uhat > 0.f ? -1.f : 1.f) * rho * ut * ut;
  fx = tw * ex;
  fz = tw * ez;
  ut_out = ut;
}

// MRT collision with Guo forcing in moment space and the Smagorinsky
// relaxation time (Sec. II.A-II.B, Eq. (6)-(15)), written as
// f* = f + M^-1 delta with delta_k = -s_k (m_k - m_eq_k) + (1 - s_k/2) F_k.
// The moment transform uses the even/odd split of the basis over the
// opposite-direction pairs (i, 18 - i).  Returns the force-corrected velocity.
//
// DEV: f holds the deviations h_i = f_i - w_i and is updated as h* = h + M^-1
// delta; pr are the pair sums of h and rhoh = rho - 1.  The weights add only
// to m_0 = rho, m_1 (-11) and m_2 (3), which enter through e_1 and e_2.
template <bool FORCE, bool DEV = false>
__device__ __forceinline__ void collide(const CollideArgs& a, const Tau0& t0, float f[Q], const Pairs& pr, float rho,
                                        float jx, float jy, float jz, float Fx, float Fy, float Fz, float& ux,
                                        float& uy, float& uz, float rhoh = 0.f) {
  const float* s = pr.s;
  const float* d = pr.d;
  const float f9 = f[9];
  const float A = pr.A;
  const float Bx = pr.Bx;
  const float T04 = s[0] + s[4], T26 = s[2] + s[6], T1357 = s[1] + s[3] + s[5] + s[7];
  const float m1 = 8.f * A - 11.f * Bx - 30.f * f9;
  const float m2 = A - 4.f * Bx + 12.f * f9;
  const float m9 = 2.f * (s[8] - T04) + T1357 - T26;
  const float m10 = -2.f * T04 + T1357 + 2.f * T26 - 4.f * s[8];
  const float m11 = (s[5] + s[6] + s[7]) - (s[1] + s[2] + s[3]);
  const float m12 = (s[5] + s[7] - 2.f * s[6]) - (s[1] + s[3] - 2.f * s[2]);
  const float m13 = s[5] - s[7], m14 = s[0] - s[4], m15 = s[1] - s[3];
  const float m4 = (d[3] + d[7]) - (d[1] + d[5]) + 4.f * d[8];
  const float m6 = d[4] - (d[0] + d[5] + d[7]) + 4.f * d[6];
  const float m8 = 4.f * d[2] - (d[0] + d[1] + d[3] + d[4]);
  const float m16 = (d[1] + d[7]) - (d[3] + d[5]);
  const float m17 = (d[4] + d[5] + d[7]) - d[0];
  const float m18 = (d[0] + d[4]) - (d[1] + d[3]);

  // Eq. (11): rho u = j + F/2;  Eq. (8) equilibria (with the readings of m2, m4,6,8)
  const float ir = rcp_fast(rho);
  const float px = FORCE ? jx + 0.5f * Fx : jx;
  const float py = FORCE ? jy + 0.5f * Fy : jy;
  const float pz = FORCE ? jz + 0.5f * Fz : jz;
  ux = px * ir;
  uy = py * ir;
  uz = pz * ir;
  const float uxx = ux * ux, uyy = uy * uy, uzz = uz * uz, uu = uxx + uyy + uzz;
  const float e1 = DEV ? m1 + 11.f * rhoh - 19.f * rho * uu : m1 - rho * (19.f * uu - 11.f);
  const float e2 = DEV ? m2 - 3.f * rhoh + 5.5f * rho * uu : m2 - rho * (3.f - 5.5f * uu);
  const float e4 = m4 + (2.f / 3.f) * px;
  const float e6 = m6 + (2.f / 3.f) * py;
  const float e8 = m8 + (2.f / 3.f) * pz;
  const float q9 = rho * (2.f * uxx - uyy - uzz);
  const float q11 = rho * (uyy - uzz);
  const float e9 = m9 - q9, e10 = m10 + 0.5f * q9;
  const float e11 = m11 - q11, e12 = m12 + 0.5f * q11;
  const float e13 = m13 - px * uy, e14 = m14 - py * uz, e15 = m15 - px * uz;

  // Sec. II.B: Pi_neq from the non-equilibrium moments, Q^(1/2) = |Pi_neq|,
  // tau_eff = tau0/2 + sqrt(tau0^2 + 18 sqrt(2) C_smag Q^(1/2) / rho)/2
  const float dc2 = e1 * (1.f / 19.f);
  const float pxx = (e9 + dc2) * (1.f / 3.f);
  const float pyy = 0.5f * (dc2 - pxx + e11), pzz = 0.5f * (dc2 - pxx - e11);
  const float q2 = pxx * pxx + pyy * pyy + pzz * pzz + 2.f * (e13 * e13 + e14 * e14 + e15 * e15);
  const float tau = 0.5f * t0.tau0 + 0.5f * sqrt_fast(t0.tau0sq + a.smag * sqrt_fast(q2) * ir);
  const float sv = rcp_fast(tau);
  const float hv = 1.f - 0.5f * sv;

  // Guo forcing moments M Fbar = (1/rho) d m_eq/du . F
  float F1 = 0.f, F2 = 0.f, F4 = 0.f, F6 = 0.f, F8 = 0.f, F9 = 0.f, F10 = 0.f, F11 = 0.f, F12 = 0.f;
  float F13 = 0.f, F14 = 0.f, F15 = 0.f;
  if (FORCE) {
    const float uF = ux * Fx + uy * Fy + uz * Fz;
    F1 = 38.f * uF;
    F2 = -11.f * uF;
    F4 = (-2.f / 3.f) * Fx;
    F6 = (-2.f / 3.f) * Fy;
    F8 = (-2.f / 3.f) * Fz;
    F9 = 2.f * (2.f * ux * Fx - uy * Fy - uz * Fz);
    F10 = -0.5f * F9;
    F11 = 2.f * (uy * Fy - uz * Fz);
    F12 = -0.5f * F11;
    F13 = ux * Fy + uy * Fx;
    F14 = uy * Fz + uz * Fy;
    F15 = ux * Fz + uz * Fx;
  }
  // delta_k / D_k
  const float a1 = FORCE ? -a.rs[1] * e1 + a.rf[1] * F1 : -a.rs[1] * e1;
  const float a2 = FORCE ? -a.rs[2] * e2 + a.rf[2] * F2 : -a.rs[2] * e2;
  const float a9 = (FORCE ? -sv * e9 + hv * F9 : -sv * e9) * (1.f / 36.f);
  const float a10 = FORCE ? -a.rs[10] * e10 + a.rf[10] * F10 : -a.rs[10] * e10;
  const float a11 = (FORCE ? -sv * e11 + hv * F11 : -sv * e11) * (1.f / 12.f);
  const float a12 = FORCE ? -a.rs[12] * e12 + a.rf[12] * F12 : -a.rs[12] * e12;
  const float a13 = (FORCE ? -sv * e13 + hv * F13 : -sv * e13) * 0.25f;
  const float a14 = (FORCE ? -sv * e14 + hv * F14 : -sv * e14) * 0.25f;
  const float a15 = (FORCE ? -sv * e15 + hv * F15 : -sv * e15) * 0.25f;
  const float b3 = 0.1f * Fx, b5 = 0.1f * Fy, b7 = 0.1f * Fz;
  const float b4 = FORCE ? -a.rs[4] * e4 + a.rf[4] * F4 : -a.rs[4] * e4;
  const float b6 = FORCE ? -a.rs[6] * e6 + a.rf[6] * F6 : -a.rs[6] * e6;
  const float b8 = FORCE ? -a.rs[8] * e8 + a.rf[8] * F8 : -a.rs[8] * e8;
  const float b16 = -a.rs[16] * m16, b17 = -a.rs[17] * m17, b18 = -a.rs[18] * m18;

  // f* = f + M^T diag(1/D) delta, assembled per opposite pair
  const float P = 8.f * a1 + a2, Qx = -11.f * a1 - 4.f * a2, R9 = -30.f * a1 + 12.f * a2;
  const float b910 = a9 + a10, c1112 = a11 + a12;
  const float h = 2.f * a10 - a9, kk = 2.f * a12 - a11;
  float E[9], O[9];
  E[0] = P - 2.f * b910 + a14;
  E[4] = P - 2.f * b910 - a14;
  E[1] = P + b910 - c1112 + a15;
  E[3] = P + b910 - c1112 - a15;
  E[5] = P + b910 + c1112 + a13;
  E[7] = P + b910 + c1112 - a13;
  E[2] = Qx + h + kk;
  E[6] = Qx + h - kk;
  E[8] = Qx + 2.f * a9 - 4.f * a10;
  const float B34 = FORCE ? b3 + b4 : b4, B56 = FORCE ? b5 + b6 : b6, B78 = FORCE ? b7 + b8 : b8;
  O[0] = -B56 - B78 - b17 + b18;
  O[4] = B56 - B78 + b17 + b18;
  O[1] = -B34 - B78 + b16 - b18;
  O[3] = B34 - B78 - b16 - b18;
  O[5] = -B34 - B56 - b16 + b17;
  O[7] = B34 - B56 + b16 + b17;
  O[2] = 4.f * b8 - (FORCE ? b7 : 0.f);
  O[6] = 4.f * b6 - (FORCE ? b5 : 0.f);
  O[8] = 4.f * b4 - (FORCE ? b3 : 0.f);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const float lo = f[k], hi = f[18 - k];
    f[k] = lo + E[k] + O[k];
    f[18 - k] = hi + E[k] - O[k];
  }
  f[9] = f9 + R9;
}

// Node of the calling thread: block = 4 consecutive y rows of one (x, z-chunk),
// blocks ordered like the bricks (y-groups fastest, then z-chunks, then x).
struct Node {
  int x, y, zci, base, gy, lane, z;
  bool owned, active;
};
__device__ __forceinline__ Node decode(const CollideArgs& a) {
  Node n;
  const int L = blockIdx.x;
  n.gy = L % a.yg;
  const int rest = L / a.yg;
  n.zci = rest % a.zc;
  n.x = rest / a.zc;
  n.lane = threadIdx.x & (ZT - 1);
  n.base = min(YROWS * n.gy, a.ny - YROWS);
  n.y = n.base + uni(threadIdx.x >> 6);
  n.owned = n.y >= YROWS * n.gy;  // rows shared with the previous group (ragged ny) are helpers only
  const int zraw = n.zci * ZT + n.lane;
  n.active = zraw < a.nz;
  n.z = n.active ? zraw : a.nz - 1;  // inactive lanes compute a valid node and store nothing
  return n;
}

// Boundary rules, wall model, collision, store and statistics of one node
// whose pulled populations are in f (Algorithm 1 for one cell).
// The outlet and inlet rules of an open channel on the pulled populations f
// of node (x, y, z); store: write the outlet history of the step.
template <bool F16>
__device__ __forceinline__ void x_rules(const CollideArgs& a, int x, int y, int z, const Col& col, float f[Q],
                                        bool store) {
  const bool inflow = a.xbc == LBM_X_INFLOW;
  if (inflow && x == a.nx - 1) {  // convective outlet for c_x < 0
    const Geo g2 = make_geo(a, x - 1, y);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int i = OUT5[k];
      const float up = pull_dir<F16>(a, g2, i, col, 0.f);
      const int hidx = (k * a.ny + y) * a.nz + z;
      const float v = a.out_wh * a.hist_in[hidx] + a.out_wu * up;
      f[i] = v;
      if (store) a.hist_out[hidx] = v;
    }
  }
  if (inflow && x == 0) inlet_regularize(a, y, z, f);
}

// NT: non-temporal population stores (see CollideArgs::nt_store).
template <bool F16, bool NT = true>
__device__ __forceinline__ void node_update(const CollideArgs& a, int x, int y, int z, int lane, int base, int zci,
                                            bool owned, bool active, const Col& col, float f[Q],
                                            float (*lds_u2)[2][ZT]) {
  x_rules<F16>(a, x, y, z, col, f, active && owned);

  // density and momentum before the force (Eq. (10)-(11)), summed directly
  // so that the collision's pair sums are not live across the wall force
  float rho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    rho += f[i];
    if (CX[i]) jx += CX[i] * f[i];
    if (CY[i]) jy += CY[i] * f[i];
    if (CZ[i]) jz += CZ[i] * f[i];
  }

  float Fx = 0.f, Fy = 0.f, Fz = 0.f;
  bool force = a.has_g != 0;
  if (force) {
    Fx = rho * a.g[0];
    Fy = rho * a.g[1];
    Fz = rho * a.g[2];
  }
  if (a.wall_model) {
    const bool bot = base == 0, top = base == a.ny - YROWS;
    if (bot || top) {  // block-uniform: the block holds a wall row and its neighbour
      const float ir = 1.f / rho;
      if (bot && y == 1) {
        lds_u2[0][0][lane] = jx * ir;
        lds_u2[0][1][lane] = jz * ir;
      }
      if (top && y == a.ny - 2) {
        lds_u2[1][0][lane] = jx * ir;
        lds_u2[1][1][lane] = jz * ir;
      }
      __syncthreads();
      const bool wb = bot && y == 0, wt = top && y == a.ny - 1;
      if (wb || wt) {
        const int w = wb ? 0 : 1;
        float fwx, fwz, ut;
        wall_force(a, rho, jx * ir, jz * ir, lds_u2[w][0][lane], lds_u2[w][1][lane], fwx, fwz, ut, w, x);
        Fx += fwx;
        Fz += fwz;
        force = true;
        if (a.wall_acc) {  // wall statistics: sum over the wave's z of u_tau (FP64, one writer per slot)
          double v = active ? (double)ut : 0.0;
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, ZT);
          if (lane == 0) a.wall_acc[((size_t)w * a.nx + x) * a.zc + zci] += v;
        }
      }
    }
  }

  float ux, uy, uz;
  const Tau0 t0 = tau0_of_x(a, x);
  const Pairs pr = make_pairs(f);
  if (force)
    collide<true>(a, t0, f, pr, rho, jx, jy, jz, Fx, Fy, Fz, ux, uy, uz);
  else
    collide<false>(a, t0, f, pr, rho, jx, jy, jz, 0.f, 0.f, 0.f, ux, uy, uz);

  if (!(rho > 0.f && rho < 1e30f)) atomicOr(a.err, ERRBIT_NONFINITE);

  if (active && owned) {
    char* p = const_cast<char*>(row_ptr<F16>(a.dst, rowpart(a, x, y)));
#pragma unroll
    for (int i = 0; i < Q; ++i)
      Pop<F16>::template stp<NT>(p + i * ZT * Pop<F16>::ES, i, col.b0, f[i], ref_off(a, i, y));
  }

  if (a.stats_on) {
    const int p = a.plane_of_x[x];
    if (p >= 0 && owned) {
      const bool on = active;
      double v[9];
      const double dx = ux, dy = uy, dz = uz;
      v[0] = on ? dx : 0.0;
      v[1] = on ? dy : 0.0;
      v[2] = on ? dz : 0.0;
      v[3] = on ? dx * dx : 0.0;
      v[4] = on ? dy * dy : 0.0;
      v[5] = on ? dz * dz : 0.0;
      v[6] = on ? dx * dy : 0.0;
      v[7] = on ? dx * dz : 0.0;
      v[8] = on ? dy * dz : 0.0;
#pragma unroll
      for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, ZT);
      if (lane == 0) {
        double* s = a.stats + (((size_t)p * a.ny + y) * a.zc + zci) * 9;
#pragma unroll
        for (int k = 0; k < 9; ++k) s[k] += v[k];
      }
    }
  }
}

// With FP16 storage the collide-stream step runs as two kernels over
// disjoint block sets (a block = 4 consecutive y rows of one (x, z-chunk)):
//  * bulk blocks (every block away from the inlet, outlet and statistics
//    planes): interior blocks, whose 3 x 3 source rows all lie inside the
//    lattice, and the y-groups holding a wall row, in one lean kernel that
//    keeps few registers and many waves in flight to hide HBM latency;
//  * boundary blocks (inlet and outlet planes, sampled statistics planes):
//    the general kernel with every rule of Algorithm 1.
// On lattices up to FUSED_MAX_NODES the two lists run as one launch
// (collide_fused_kernel).  With FP32 storage the general kernel takes every
// block.  All read s_n and write disjoint nodes of s_{n+1}.  Each walks a
// block list (columns (x, y-group) dealt to the XCDs by xcd_order).

// A block whose 3 x 3 source rows all lie inside the lattice (see the
// block lists): plain shifted pulls, no boundary rule.
// dref / dpull: the reference offsets (REF), passed as restrict kernel
// arguments so that their loads need not be ordered after the stores.
template <bool F16, bool FORCE, bool REF>
__device__ __forceinline__ void plain_block(const CollideArgs& a, int x, int zci, int gy,
                                            const float* __restrict__ dref, const float* __restrict__ dpull) {
  const int lane = threadIdx.x & (ZT - 1);
  const int base = min(YROWS * gy, a.ny - YROWS);
  const int y = base + uni(threadIdx.x >> 6);
  const bool owned = y >= YROWS * gy;
  const int zraw = zci * ZT + lane;
  const bool active = zraw < a.nz;
  const int z = active ? zraw : a.nz - 1;
  const Col col = make_col<F16>(a, z);
  const Geo g = make_geo(a, x, y);
  typename Pop<F16>::Raw r[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const uint32_t cs = CZ[i] == 1 ? col.bm : (CZ[i] == -1 ? col.bp : col.b0);
    r[i] = Pop<F16>::raw(row_ptr<F16>(a.src, rowpart(a, g.xs[CX[i] + 1], g.ys[CY[i] + 1]) + (uint32_t)i * ZT), cs);
  }
  // FP16 storage computes on the deviations h = f - w directly (no w added on
  // load or subtracted on store); FP32 storage on the populations.
  float f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (!F16)
      f[i] = Pop<F16>::cvt(i, r[i], 0.f);
    else if (REF)
      f[i] = Pop<true>::cvt_dev(r[i], dpull[y * Q + i]);  // wave-uniform row: scalar loads
    else
      f[i] = Pop<true>::cvt_dev(r[i]);
  }
  const Pairs pr = make_pairs(f);
  const float rhoh = pr.A + pr.Bx + f[9];  // sum of h (F16) or rho (F32)
  const float rho = F16 ? 1.f + rhoh : rhoh;
  const float jx = (pr.d[3] + pr.d[7]) - (pr.d[1] + pr.d[5] + pr.d[8]);
  const float jy = pr.d[4] - (pr.d[0] + pr.d[5] + pr.d[6] + pr.d[7]);
  const float jz = -(pr.d[0] + pr.d[1] + pr.d[2] + pr.d[3] + pr.d[4]);
  float ux, uy, uz;
  const Tau0 t0 = tau0_of_x(a, x);
  if (FORCE)
    collide<true, F16>(a, t0, f, pr, rho, jx, jy, jz, rho * a.g[0], rho * a.g[1], rho * a.g[2], ux, uy, uz, rhoh);
  else
    collide<false, F16>(a, t0, f, pr, rho, jx, jy, jz, 0.f, 0.f, 0.f, ux, uy, uz, rhoh);
  if (!(rho > 0.f && rho < 1e30f)) atomicOr(a.err, ERRBIT_NONFINITE);
  if (active && owned) {
    char* p = const_cast<char*>(row_ptr<F16>(a.dst, rowpart(a, x, y)));
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (F16 && REF)
        Pop<true>::stp_dev<true>(p + i * ZT * Pop<F16>::ES, col.b0, f[i], dref[y * Q + i]);
      else if (F16)
        Pop<true>::stp_dev<true>(p + i * ZT * Pop<F16>::ES, col.b0, f[i]);
      else
        Pop<F16>::template stp<true>(p + i * ZT * Pop<F16>::ES, i, col.b0, f[i], 0.f);
    }
  }
}

// A y-group holding a wall row, away from the inlet, outlet and statistics
// planes: the plain block's data flow plus the wall rules of the pull and
// the wall model (the wall row's neighbour velocity through LDS).  Density
// and momentum are summed directly so that the pair sums of the collision
// are not live across the Newton solve (fewer registers).
template <bool F16, bool REF>
__device__ __forceinline__ void wall_block(const CollideArgs& a, int x, int zci, int gy, float (*lds_u2)[2][ZT],
                                           const float* __restrict__ dref) {

  const int lane = threadIdx.x & (ZT - 1);
  const int base = min(YROWS * gy, a.ny - YROWS);
  const int y = base + uni(threadIdx.x >> 6);
  const bool owned = y >= YROWS * gy;
  const int zraw = zci * ZT + lane;
  const bool active = zraw < a.nz;
  const int z = active ? zraw : a.nz - 1;
  const Col col = make_col<F16>(a, z);
  const Geo g = make_geo(a, x, y);
  typename Pop<F16>::Raw r[Q];
  issue_pulls<F16>(a, g, col, r);  // every x source exists; the y walls redirect
  float f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (!F16)
      f[i] = Pop<F16>::cvt(i, r[i], 0.f);
    else if (REF)
      f[i] = Pop<true>::cvt_dev(r[i], pull_ref(a, g, i));
    else
      f[i] = Pop<true>::cvt_dev(r[i]);
  }
  // density and momentum first; the pair sums of the collision are formed
  // after the wall force, so they are not live across the Newton solve
  float rhoh = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    rhoh += f[i];
    if (CX[i]) jx += CX[i] * f[i];
    if (CY[i]) jy += CY[i] * f[i];
    if (CZ[i]) jz += CZ[i] * f[i];
  }
  const float rho = F16 ? 1.f + rhoh : rhoh;
  float Fx = rho * a.g[0], Fy = rho * a.g[1], Fz = rho * a.g[2];
  if (a.wall_model) {
    const bool bot = base == 0, top = base == a.ny - YROWS;
    const float ir = 1.f / rho;
    if (bot && y == 1) {
      lds_u2[0][0][lane] = jx * ir;
      lds_u2[0][1][lane] = jz * ir;
    }
    if (top && y == a.ny - 2) {
      lds_u2[1][0][lane] = jx * ir;
      lds_u2[1][1][lane] = jz * ir;
    }
    __syncthreads();
    const bool wb = bot && y == 0, wt = top && y == a.ny - 1;
    if (wb || wt) {
      const int w = wb ? 0 : 1;
      float fwx, fwz, ut;
      wall_force(a, rho, jx * ir, jz * ir, lds_u2[w][0][lane], lds_u2[w][1][lane], fwx, fwz, ut, w, x);
      Fx += fwx;
      Fz += fwz;
      if (a.wall_acc) {
        double v = active ? (double)ut : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, ZT);
        if (lane == 0) a.wall_acc[((size_t)w * a.nx + x) * a.zc + zci] += v;
      }
    }
  }
  float ux, uy, uz;
  const Pairs pr = make_pairs(f);
  collide<true, F16>(a, tau0_of_x(a, x), f, pr, rho, jx, jy, jz, Fx, Fy, Fz, ux, uy, uz, rhoh);
  if (!(rho > 0.f && rho < 1e30f)) atomicOr(a.err, ERRBIT_NONFINITE);
  if (active && owned) {
    char* p = const_cast<char*>(row_ptr<F16>(a.dst, rowpart(a, x, y)));
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (F16 && REF)
        Pop<true>::stp_dev<true>(p + i * ZT * Pop<F16>::ES, col.b0, f[i], dref[y * Q + i]);
      else if (F16)
        Pop<true>::stp_dev<true>(p + i * ZT * Pop<F16>::ES, col.b0, f[i]);
      else
        Pop<F16>::template stp<true>(p + i * ZT * Pop<F16>::ES, i, col.b0, f[i], 0.f);
    }
  }
}

// Interior and wall blocks (block-uniform choice): the lean kernel, so it
// keeps few registers and many waves in flight to hide HBM latency.
template <bool F16, bool FORCE, bool REF>
__global__ __launch_bounds__(BLOCK) void collide_bulk_kernel(CollideArgs a, const int* __restrict__ blist,
                                                             const float* __restrict__ dref,
                                                             const float* __restrict__ dpull) {
  __shared__ float lds_u2[2][2][ZT];
  const int e = blist[blockIdx.x];
  if (e < 0) return;  // padding of the XCD-ordered list (whole block: no barrier is skipped by part of it)
  int x, zci, gy;
  block_coords(a, e, x, zci, gy);
  const int base = min(YROWS * gy, a.ny - YROWS);
  if (a.ywall != LBM_Y_PERIODIC && (base == 0 || base == a.ny - YROWS))
    wall_block<F16, REF>(a, x, zci, gy, lds_u2, dref);
  else
    plain_block<F16, FORCE, REF>(a, x, zci, gy, dref, dpull);
}

template <bool F16, bool NT = true>
__global__ __launch_bounds__(BLOCK) void collide_general_kernel(CollideArgs a, const int* __restrict__ blist) {
  __shared__ float lds_u2[2][2][ZT];
  const int e = blist[blockIdx.x];
  if (e < 0) return;  // padding of the XCD-ordered list (whole block: no barrier is skipped by part of it)
  int x, zci, gy;
  block_coords(a, e, x, zci, gy);
  const int lane = threadIdx.x & (ZT - 1);
  const int base = min(YROWS * gy, a.ny - YROWS);
  const int y = base + uni(threadIdx.x >> 6);
  const bool owned = y >= YROWS * gy;  // rows shared with the previous group (ragged ny) are helpers only
  const int zraw = zci * ZT + lane;
  const bool active = zraw < a.nz;
  const int z = active ? zraw : a.nz - 1;  // inactive lanes compute a valid node and store nothing
  const Col col = make_col<F16>(a, z);
  const Geo g = make_geo(a, x, y);
  typename Pop<F16>::Raw r[Q];
  issue_pulls<F16>(a, g, col, r);
  float f[Q];
  convert_pulls<F16>(a, g, r, f);
  node_update<F16, NT>(a, x, y, z, lane, base, zci, owned, active, col, f, lds_u2);
}

// FP16 storage on lattices up to FUSED_MAX_NODES: both block lists in one
// launch, the general blocks (gl, n_gen entries) first so that their longer
// work overlaps the bulk blocks (bl).  Held to 64 VGPRs (8 waves per SIMD, as
// the bulk kernel; the general path spills a few).  A separate general launch
// costs a fixed ~10 us (its blocks run alone as a latency-bound wave), more
// than the fused kernel's slower bulk path on small lattices, less on large.
template <bool F16, bool FORCE, bool REF>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8)))
void collide_fused_kernel(CollideArgs a, const int* __restrict__ gl, int n_gen, const int* __restrict__ bl,
                          const float* __restrict__ dref, const float* __restrict__ dpull) {
  __shared__ float lds_u2[2][2][ZT];
  const int b = (int)blockIdx.x;
  if (b < n_gen) {  // a general block (block-uniform)
    const int e = gl[b];
    if (e < 0) return;  // padding of the XCD-ordered list (whole block)
    int x, zci, gy;
    block_coords(a, e, x, zci, gy);
    const int lane = threadIdx.x & (ZT - 1);
    const int base = min(YROWS * gy, a.ny - YROWS);
    const int y = base + uni(threadIdx.x >> 6);
    const bool owned = y >= YROWS * gy;
    const int zraw = zci * ZT + lane;
    const bool active = zraw < a.nz;
    const int z = active ? zraw : a.nz - 1;
    const Col col = make_col<F16>(a, z);
    const Geo g = make_geo(a, x, y);
    typename Pop<F16>::Raw r[Q];
    issue_pulls<F16>(a, g, col, r);
    float f[Q];
    convert_pulls<F16>(a, g, r, f);
    node_update<F16>(a, x, y, z, lane, base, zci, owned, active, col, f, lds_u2);
    return;
  }
  const int e = bl[b - n_gen];
  if (e < 0) return;
  int x, zci, gy;
  block_coords(a, e, x, zci, gy);
  const int base = min(YROWS * gy, a.ny - YROWS);
  if (a.ywall != LBM_Y_PERIODIC && (base == 0 || base == a.ny - YROWS))
    wall_block<F16, REF>(a, x, zci, gy, lds_u2, dref);
  else
    plain_block<F16, FORCE, REF>(a, x, zci, gy, dref, dpull);
}

// Pre-force velocity (u_x, u_z) of node (x, y, z) after streaming and the
// boundary rules, as node_update forms it.
template <bool F16>
__device__ __forceinline__ void pre_force_uxz(const CollideArgs& a, int x, int y, int z, const Col& col, float& ux,
                                              float& uz) {
  const Geo g = make_geo(a, x, y);
  typename Pop<F16>::Raw r[Q];
  issue_pulls<F16>(a, g, col, r);
  float f[Q];
  convert_pulls<F16>(a, g, r, f);
  x_rules<F16>(a, x, y, z, col, f, false);
  const Pairs pr = make_pairs(f);
  const float rho = pr.A + pr.Bx + f[9];
  const float jx = (pr.d[3] + pr.d[7]) - (pr.d[1] + pr.d[5] + pr.d[8]);
  const float jz = -(pr.d[0] + pr.d[1] + pr.d[2] + pr.d[3] + pr.d[4]);
  const float ir = 1.f / rho;
  ux = jx * ir;
  uz = jz * ir;
}

// Line-averaged wall model: one block per wall line (x, wall).  Its four
// waves sum u_hat = u_w . e_x (Eq. (19), 0 where u_2 has no tangential part)
// over z in FP64 in a fixed order; the line's u_tau solves Eq. (20) for the
// mean's magnitude and is stored with the mean's sign.
template <bool F16>
__global__ __launch_bounds__(BLOCK) void wall_line_kernel(CollideArgs a, float* line) {
  __shared__ double part[BLOCK / ZT];
  const int x = blockIdx.x, w = blockIdx.y;
  const int yw = w ? a.ny - 1 : 0, y2 = w ? a.ny - 2 : 1;
  const int lane = threadIdx.x & (ZT - 1), wave = uni(threadIdx.x >> 6);
  double acc = 0.0;
  for (int zci = wave; zci < a.zc; zci += BLOCK / ZT) {
    const int zraw = zci * ZT + lane;
    const bool active = zraw < a.nz;
    const int z = active ? zraw : a.nz - 1;
    const Col col = make_col<F16>(a, z);
    float uwx, uwz, u2x, u2z;
    pre_force_uxz<F16>(a, x, yw, z, col, uwx, uwz);
    pre_force_uxz<F16>(a, x, y2, z, col, u2x, u2z);
    const float tn2 = u2x * u2x + u2z * u2z;
    float uh = 0.f;
    if (tn2 > 0.f) {
      const float itn = 1.f / sqrtf(tn2);
      uh = uwx * (u2x * itn) + uwz * (u2z * itn);
    }
    acc += active ? (double)uh : 0.0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, ZT);
  if (lane == 0) part[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < BLOCK / ZT; ++k) s += part[k];
    const float ub = (float)(s / a.nz);
    const float ut = ub != 0.f ? newton_utau(a, fabsf(ub)) : 0.f;
    line[w * a.nx + x] = ub > 0.f ? ut : -ut;
  }
}

// Pull with the wall rules only (debug map); unset populations are -1.
__global__ __launch_bounds__(BLOCK) void stream_only_kernel(CollideArgs a) {
  const Node nd = decode(a);
  if (!nd.active || !nd.owned) return;
  const Col col = make_col<false>(a, nd.z);
  const Geo g = make_geo(a, nd.x, nd.y);
  const uint32_t row = rowpart(a, nd.x, nd.y);
#pragma unroll
  for (int i = 0; i < Q; ++i) Pop<false>::st_plain(a.dst, i, row + (uint32_t)i * ZT + col.c0, pull_dir<false>(a, g, i, col, -1.f), 0.f);
}

// f_i = f_eq_i(rho, u) + eps w_i pert_i from SoA node fields [.][N], N = (x ny + y) nz + z,
// in the precision T of the inputs (float or double), rounded once to the
// storage: FP32 populations, or with FP16 storage the deviation f - w - r
// formed in T.
template <bool F16, typename T>
__global__ __launch_bounds__(BLOCK) void init_kernel(CollideArgs a, float* hist, const T* rho, const T* u,
                                                     const T* pert, T eps) {
  const Node nd = decode(a);
  if (!nd.active || !nd.owned) return;
  const int N = a.nx * a.ny * a.nz;
  const int n = (nd.x * a.ny + nd.y) * a.nz + nd.z;
  const T r = rho ? rho[n] : T(1);
  const T ux = u[n], uy = u[N + n], uz = u[2 * N + n];
  const T uu15 = T(1.5) * (ux * ux + uy * uy + uz * uz);
  const uint32_t e0 = rowpart(a, nd.x, nd.y) + colpart(a, nd.z);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const T cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
    T v = (T)WD[i] * r * (T(1) + T(3) * cu + T(4.5) * cu * cu - uu15);
    if (pert) v += eps * (T)WD[i] * pert[(size_t)i * N + n];
    const float ref = ref_off(a, i, nd.y);
    if (F16 && sizeof(T) == 8)
      static_cast<_Float16*>(a.dst)[e0 + (uint32_t)i * ZT] = (_Float16)(float)((v - WD[i]) - (T)ref);
    else
      Pop<F16>::st_plain(a.dst, i, e0 + (uint32_t)i * ZT, (float)v, ref);
    if (hist && nd.x == a.nx - 1) {
#pragma unroll
      for (int k = 0; k < 5; ++k)
        if (OUT5[k] == i) hist[(k * a.ny + nd.y) * a.nz + nd.z] = (float)v;
    }
  }
}

// State (bricks) -> float SoA [19][N].
template <bool F16>
__global__ __launch_bounds__(BLOCK) void export_kernel(CollideArgs a, float* out) {
  const Node nd = decode(a);
  if (!nd.active || !nd.owned) return;
  const size_t N = (size_t)a.nx * a.ny * a.nz;
  const size_t n = ((size_t)nd.x * a.ny + nd.y) * a.nz + nd.z;
  const uint32_t e0 = rowpart(a, nd.x, nd.y) + colpart(a, nd.z);
#pragma unroll
  for (int i = 0; i < Q; ++i) out[(size_t)i * N + n] = Pop<F16>::ld_plain(a.src, i, e0 + (uint32_t)i * ZT, ref_off(a, i, nd.y));
}

// Float SoA [19][N] -> state (bricks), rounded to the storage type.
template <bool F16>
__global__ __launch_bounds__(BLOCK) void import_kernel(CollideArgs a, const float* in) {
  const Node nd = decode(a);
  if (!nd.active || !nd.owned) return;
  const size_t N = (size_t)a.nx * a.ny * a.nz;
  const size_t n = ((size_t)nd.x * a.ny + nd.y) * a.nz + nd.z;
  const uint32_t e0 = rowpart(a, nd.x, nd.y) + colpart(a, nd.z);
#pragma unroll
  for (int i = 0; i < Q; ++i)
    Pop<F16>::st_plain(a.dst, i, e0 + (uint32_t)i * ZT, in[(size_t)i * N + n], ref_off(a, i, nd.y));
}

// FP16 storage reference offsets r_i(y) = f_eq_i(1, u_ref(y)) - w_i (second-order
// equilibrium, FP64, stored as float); u_ref == nullptr gives r = 0.
__device__ double dref_value(const double* u_ref, int ny, int y, int i) {
#pragma clang fp contract(off)  // plain multiplies and adds: reproducible off the device
  const double ux = u_ref[y], uy = u_ref[ny + y], uz = u_ref[2 * ny + y];
  const double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
  return WD[i] * (3.0 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy + uz * uz));
}

// dref[y][i] = r_i(y); dpull[y][i] = r_i of the row a plain pull of direction i
// reads into row y (y - c_y, periodic in y like the plain pull rows).
__global__ void dref_kernel(const double* u_ref, int ny, float* dref, float* dpull) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ny * Q) return;
  const int y = k / Q, i = k % Q;
  const int ys = (y - CY[i] + ny) % ny;
  dref[k] = (float)dref_value(u_ref, ny, y, i);
  dpull[k] = (float)dref_value(u_ref, ny, ys, i);
}

// The current FP16 state re-encoded in place from offsets dold to dnew (either
// may be null: 0).
__global__ __launch_bounds__(BLOCK) void recode_kernel(CollideArgs a, _Float16* state, const float* dold,
                                                       const float* dnew) {
  const Node nd = decode(a);
  if (!nd.active || !nd.owned) return;
  const uint32_t e0 = rowpart(a, nd.x, nd.y) + colpart(a, nd.z);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float ro = dold ? dold[nd.y * Q + i] : 0.f, rn = dnew ? dnew[nd.y * Q + i] : 0.f;
    _Float16& h = state[e0 + (uint32_t)i * ZT];
    h = (_Float16)(((float)h + ro) - rn);
  }
}

// One 16-byte vector per thread, non-temporal load and store (the bandwidth
// reference of the benchmark: 6.54-6.58 TB/s for 2-11 GiB, against 6.20-6.36
// with plain loads and 5.6-6.1 with 2-8 vectors per thread).  The pull kernels
// keep plain loads: each source row is read by up to nine destination rows,
// which must hit in L2.
typedef float vec4f __attribute__((ext_vector_type(4)));
__global__ void copy_kernel(const vec4f* __restrict__ src, vec4f* __restrict__ dst, int64_t n4) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n4) __builtin_nontemporal_store(__builtin_nontemporal_load(src + k), dst + k);
}

}  // namespace

// Kernel arguments of a launch reading buffer src and writing buffer dst.
void fill_args(lbm_ctx* h, CollideArgs& a, int src, int dst) {
  const lbm_config& c = h->cfg;
  a.src = h->f[src];
  a.dst = h->f[dst];
  a.hist_in = h->hist[src];
  a.hist_out = h->hist[dst];
  a.u_in = h->stg_bound ? h->stg.u_in : nullptr;
  a.stats = h->d_stats;
  a.wall_acc = h->stats_on ? h->d_wall_acc : nullptr;
  a.wall_line = nullptr;
  a.dref = h->d_dref;
  a.dpull = h->d_dpull;
  a.plane_of_x = h->d_plane_of_x;
  a.err = h->d_err;
  a.nx = c.nx;
  a.ny = c.ny;
  a.nz = c.nz;
  a.zc = h->zc;
  a.yg = h->yg;
  a.nblocks = h->nblocks;
  a.ywall = c.ywall;
  a.xbc = c.xbc;
  a.wall_model = c.wall_model;
  a.wall_law = c.wall_law;
  a.newton_iters = c.newton_iters;
  a.stats_on = h->stats_on && h->d_stats != nullptr;
  // FP32 population stores bypass the caches (non-temporal) unless both state
  // buffers fit in the Infinity Cache with room to spare: then the next step
  // reads the state the last one wrote from there.  (FP16 storage measured
  // no gain from cached stores: it always stores non-temporally.)
  a.nt_store = h->cfg.storage == LBM_STORE_F16DEV ||
               2 * 4 * (int64_t)Q * h->cfg.nx * h->cfg.ny * h->zc * ZT > NT_STORE_MIN_BYTES;
  a.has_g = (c.g[0] != 0.0 || c.g[1] != 0.0 || c.g[2] != 0.0) ? 1 : 0;
  a.tau0 = (float)c.tau0;
  a.tau0sq = (float)(c.tau0 * c.tau0);
  a.smag = (float)(18.0 * std::sqrt(2.0) * c.cs_smag * c.cs_smag);
  for (int k = 0; k < 3; ++k) a.g[k] = (float)c.g[k];
  const double nu0 = (c.tau0 - 0.5) / 3.0;
  a.nu0 = (float)nu0;
  a.inv_nu0 = (float)(1.0 / nu0);
  a.y_wall = (float)c.y_wall;
  a.kappa = (float)c.kappa;
  a.inv_kappa = (float)(1.0 / c.kappa);
  a.b_reich = (float)c.b_reich;
  if (c.outlet == LBM_OUTLET_ZERO_GRADIENT) {
    a.out_wh = 0.f;
    a.out_wu = 1.f;
  } else {  // convective: (f^prev + U_c f(x-1)) / (1 + U_c)
    a.out_wh = (float)(1.0 / (1.0 + c.u_conv));
    a.out_wu = (float)(c.u_conv / (1.0 + c.u_conv));
  }
  a.sponge_x0 = c.sponge_cells > 0 ? c.nx - c.sponge_cells : c.nx;
  a.sponge_inv_len = c.sponge_cells > 0 ? (float)(1.0 / c.sponge_cells) : 0.f;
  a.sponge_dnu = c.sponge_cells > 0 ? (float)(c.sponge_nu - nu0) : 0.f;
  for (int k = 0; k < Q; ++k) {
    a.rs[k] = (float)(c.s[k] / DNORM[k]);
    a.rf[k] = (float)((1.0 - 0.5 * c.s[k]) / DNORM[k]);
  }
}


// The line-averaged u_tau of the step a describes, into h->d_wall_line (a
// no-op unless that model is configured); a.wall_line then points there.
hipError_t launch_wall_line(lbm_ctx* h, CollideArgs& a, hipStream_t stream) {
  const lbm_config& c = h->cfg;
  if (c.wall_avg != LBM_WALL_AVG_LINE || !c.wall_model || c.ywall == LBM_Y_PERIODIC) return hipSuccess;
  if (!h->d_wall_line) {
    hipError_t e = hipMalloc(&h->d_wall_line, sizeof(float) * 2 * c.nx);
    if (e != hipSuccess) return e;
  }
  dim3 grid(c.nx, 2);
  if (c.storage == LBM_STORE_F16DEV)
    wall_line_kernel<true><<<grid, BLOCK, 0, stream>>>(a, h->d_wall_line);
  else
    wall_line_kernel<false><<<grid, BLOCK, 0, stream>>>(a, h->d_wall_line);
  a.wall_line = h->d_wall_line;
  return hipGetLastError();
}

// The bulk kernel variant for the storage, the body force and the FP16
// reference offsets.
void launch_bulk_kernel(lbm_ctx* h, const CollideArgs& a, bool f16, hipStream_t stream) {
  const int n = h->n_int;
  const int* bl = h->d_blist_int;
  if (h->fused) {
    const int ng = h->n_bnd, nt = ng + n;
    const int* gl = h->d_blist_bnd;
    if (nt == 0) return;
    if (a.dref) {
      if (a.has_g)
        collide_fused_kernel<true, true, true><<<nt, BLOCK, 0, stream>>>(a, gl, ng, bl, a.dref, a.dpull);
      else
        collide_fused_kernel<true, false, true><<<nt, BLOCK, 0, stream>>>(a, gl, ng, bl, a.dref, a.dpull);
    } else {
      if (a.has_g)
        collide_fused_kernel<true, true, false><<<nt, BLOCK, 0, stream>>>(a, gl, ng, bl, a.dref, a.dpull);
      else
        collide_fused_kernel<true, false, false><<<nt, BLOCK, 0, stream>>>(a, gl, ng, bl, a.dref, a.dpull);
    }
    return;
  }
  if (n == 0) return;
  if (!f16) {
    if (a.has_g)
      collide_bulk_kernel<false, true, false><<<n, BLOCK, 0, stream>>>(a, bl, a.dref, a.dpull);
    else
      collide_bulk_kernel<false, false, false><<<n, BLOCK, 0, stream>>>(a, bl, a.dref, a.dpull);
  } else if (a.dref) {
    if (a.has_g)
      collide_bulk_kernel<true, true, true><<<n, BLOCK, 0, stream>>>(a, bl, a.dref, a.dpull);
    else
      collide_bulk_kernel<true, false, true><<<n, BLOCK, 0, stream>>>(a, bl, a.dref, a.dpull);
  } else {
    if (a.has_g)
      collide_bulk_kernel<true, true, false><<<n, BLOCK, 0, stream>>>(a, bl, a.dref, a.dpull);
    else
      collide_bulk_kernel<true, false, false><<<n, BLOCK, 0, stream>>>(a, bl, a.dref, a.dpull);
  }
}

// The general blocks of one step: one dispatch per x-chunk of the list (the
// chunks update disjoint nodes from s_n, so their order is free).
void launch_edge_kernels(lbm_ctx* h, const CollideArgs& a, hipStream_t stream) {
  const bool f16 = h->cfg.storage == LBM_STORE_F16DEV;
  for (size_t k = 0; k + 1 < h->bnd_off.size(); ++k) {
    const int n = h->bnd_off[k + 1] - h->bnd_off[k];
    const int* bl = h->d_blist_bnd + h->bnd_off[k];
    if (n <= 0) continue;
    if (f16)
      collide_general_kernel<true><<<n, BLOCK, 0, stream>>>(a, bl);
    else if (a.nt_store)
      collide_general_kernel<false, true><<<n, BLOCK, 0, stream>>>(a, bl);
    else
      collide_general_kernel<false, false><<<n, BLOCK, 0, stream>>>(a, bl);
  }
}

// The step's line u_tau (line-averaged wall model; also when no general block
// exists, e.g. a periodic channel with FP16 storage) and the general blocks
// (unless the fused kernel takes them with the bulk blocks).
hipError_t launch_boundary(lbm_ctx* h, int src, int dst, hipStream_t stream, const float* u_in) {
  CollideArgs a;
  fill_args(h, a, src, dst);
  if (u_in) a.u_in = u_in;
  hipError_t e = launch_wall_line(h, a, stream);
  if (e != hipSuccess || h->n_bnd == 0 || h->fused) return e;
  launch_edge_kernels(h, a, stream);
  return hipGetLastError();
}

// One step between caller buffers (statistics off), on one stream: the
// boundary and bulk block lists with FP16 storage, the single list with FP32.
hipError_t launch_step_explicit(lbm_ctx* h, const void* src, void* dst, const float* hist_in, float* hist_out,
                                const float* u_in, hipStream_t stream) {
  CollideArgs a;
  fill_args(h, a, h->cur, h->cur);
  a.src = src;
  a.dst = dst;
  a.hist_in = hist_in;
  a.hist_out = hist_out;
  a.u_in = u_in;
  a.stats_on = 0;
  a.wall_acc = nullptr;
  const bool f16 = h->cfg.storage == LBM_STORE_F16DEV;
  hipError_t e = launch_wall_line(h, a, stream);
  if (e != hipSuccess) return e;
  if (!h->fused) launch_edge_kernels(h, a, stream);
  launch_bulk_kernel(h, a, f16, stream);
  return hipGetLastError();
}

// The bulk blocks of one step (with the general blocks when fused; u_in, when
// given, replaces the bound inlet plane).  With the line-averaged wall model
// the step's line u_tau must already be in h->d_wall_line on this stream
// (launch_boundary).
hipError_t launch_bulk(lbm_ctx* h, int src, int dst, hipStream_t stream, const float* u_in) {
  CollideArgs a;
  fill_args(h, a, src, dst);
  if (u_in) a.u_in = u_in;
  if (h->cfg.wall_avg == LBM_WALL_AVG_LINE && h->cfg.wall_model && h->cfg.ywall != LBM_Y_PERIODIC)
    a.wall_line = h->d_wall_line;
  launch_bulk_kernel(h, a, h->cfg.storage == LBM_STORE_F16DEV, stream);
  return hipGetLastError();
}

// Arrange a list of blocks for dispatch.  Blocks are handed to the 8 XCDs
// round-robin (block b runs on XCD b mod 8), and each XCD has its own L2.
// The only cache lines two blocks share are the edge lines of the +-1 z
// shifts between z-neighbouring bricks of one (x, y-group) column, so every
// column is given to one XCD and its z-chunks run back to back there.
// Columns go to XCDs in turn, each class of column (heavy[c]: wall groups,
// whose blocks take longer) with its own turn, so that every XCD gets its
// share of both; queues are padded with -1 (empty block).
std::vector<int> xcd_order(const std::vector<int>& entries, int zc, const std::vector<char>* heavy) {
  constexpr int NX = 8;
  std::vector<std::vector<int>> q(NX);
  const size_t ncol = entries.size() / zc;
  size_t turn[2] = {0, 0};
  for (size_t c = 0; c < ncol; ++c) {
    const int k = heavy ? ((*heavy)[c] ? 1 : 0) : 0;
    const size_t xcd = turn[k]++ % NX;
    for (int j = 0; j < zc; ++j) q[xcd].push_back(entries[c * zc + j]);
  }
  size_t len = 0;
  for (auto& v : q) len = std::max(len, v.size());
  std::vector<int> out(len * NX, -1);
  for (int k = 0; k < NX; ++k)
    for (size_t j = 0; j < q[k].size(); ++j) out[j * NX + k] = q[k][j];
  return out;
}

// Split the blocks (x, z-chunk, y-group) into bulk and boundary lists,
// each ordered by xcd_order (see collide_bulk_kernel / collide_general_kernel).
// The planes of plane_of_x (the attached statistics planes) are boundary
// blocks whether or not statistics are being accumulated: the two kernels
// round FP16 deviations differently (the bulk kernel computes on deviations),
// and a recompute with statistics off must reproduce the forward run.
// With FP32 storage the boundary list (all blocks) is cut into x-chunks of
// about CHUNK_BLOCKS blocks, each ordered by xcd_order on its own, since
// every chunk is a dispatch of its own.
hipError_t build_block_lists(lbm_ctx* h, const std::vector<int>& plane_of_x) {
  const lbm_config& c = h->cfg;
  std::vector<int> in, bd;
  std::vector<char> in_heavy;  // per bulk column: a wall group
  in.reserve((size_t)c.nx * h->zc * h->yg);
  int64_t int_nodes = 0;
  const bool split = h->split;
  // columns (x, y-group) in memory order, each with its zc z-chunks
  for (int x = 0; x < c.nx; ++x) {
    // statistics planes (attached, accumulating or not) take the general kernel
    const bool xb = (c.xbc == LBM_X_INFLOW && (x == 0 || x == c.nx - 1)) || plane_of_x[x] >= 0;
    for (int gy = 0; gy < h->yg; ++gy) {
      const int base = std::min(YROWS * gy, c.ny - YROWS);
      const bool bulk_block = split && !xb;  // wall groups take the bulk kernel's wall branch
      if (bulk_block) in_heavy.push_back(c.ywall != LBM_Y_PERIODIC && (base == 0 || base == c.ny - YROWS));
      for (int zc = 0; zc < h->zc; ++zc) {
        const int e = (x * h->zc + zc) * h->yg + gy;
        (bulk_block ? in : bd).push_back(e);
        if (bulk_block) {
          const int owned_rows = YROWS - (YROWS * gy - base);
          const int lanes = std::min(ZT, c.nz - ZT * zc);
          int_nodes += (int64_t)owned_rows * lanes;
        }
      }
    }
  }
  in = xcd_order(in, h->zc, &in_heavy);
  // bd is in memory order (x-major), so an x-range is a contiguous run of it
  int nchunk = 1;
  if (!split) nchunk = (int)std::max<int64_t>(1, std::llround((double)h->nblocks / CHUNK_BLOCKS));
  const int planes = (c.nx + std::min(nchunk, c.nx) - 1) / std::min(nchunk, c.nx);
  const int per_plane = h->zc * h->yg;
  {
    std::vector<int> out;
    h->bnd_off.assign(1, 0);
    size_t i = 0;
    for (int x0 = 0; x0 < c.nx; x0 += planes) {
      std::vector<int> part;
      while (i < bd.size() && bd[i] / per_plane < x0 + planes) part.push_back(bd[i++]);
      if (part.empty()) continue;
      part = xcd_order(part, h->zc);
      out.insert(out.end(), part.begin(), part.end());
      h->bnd_off.push_back((int)out.size());
    }
    bd.swap(out);
  }
  h->chunk_planes = planes;
  hipError_t err;
  for (int k = 0; k < 2; ++k) {
    std::vector<int>& v = k == 0 ? in : bd;
    int** d = k == 0 ? &h->d_blist_int : &h->d_blist_bnd;
    int* cap = k == 0 ? &h->cap_int : &h->cap_bnd;
    if (*cap < (int)v.size() || !*d) {
      if (*d && (err = hipFree(*d)) != hipSuccess) return err;
      *d = nullptr;
      if ((err = hipMalloc(d, sizeof(int) * std::max<size_t>(v.size(), 1))) != hipSuccess) return err;
      *cap = (int)std::max<size_t>(v.size(), 1);
    }
    if (!v.empty() && (err = hipMemcpy(*d, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice)) != hipSuccess)
      return err;
  }
  h->n_int = (int)in.size();
  h->n_bnd = (int)bd.size();
  h->int_nodes = int_nodes;
  return hipSuccess;
}

hipError_t launch_stream_only(lbm_ctx* h, int src, int dst) {
  CollideArgs a;
  fill_args(h, a, src, dst);
  stream_only_kernel<<<h->nblocks, BLOCK, 0, h->stream>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_init_t(lbm_ctx* h, const T* rho, const T* u, const T* pert, T eps) {
  CollideArgs a;
  fill_args(h, a, h->cur, h->cur);
  float* hist = h->cfg.xbc == LBM_X_INFLOW ? h->hist[h->cur] : nullptr;
  if (h->cfg.storage == LBM_STORE_F16DEV)
    init_kernel<true, T><<<h->nblocks, BLOCK, 0, h->stream>>>(a, hist, rho, u, pert, eps);
  else
    init_kernel<false, T><<<h->nblocks, BLOCK, 0, h->stream>>>(a, hist, rho, u, pert, eps);
  return hipGetLastError();
}

hipError_t launch_init(lbm_ctx* h, const float* rho, const float* u, const float* pert, float eps) {
  return launch_init_t(h, rho, u, pert, eps);
}

hipError_t launch_init(lbm_ctx* h, const double* rho, const double* u, const double* pert, double eps) {
  return launch_init_t(h, rho, u, pert, eps);
}

hipError_t launch_export(lbm_ctx* h, float* out) {
  CollideArgs a;
  fill_args(h, a, h->cur, h->cur);
  if (h->cfg.storage == LBM_STORE_F16DEV)
    export_kernel<true><<<h->nblocks, BLOCK, 0, h->stream>>>(a, out);
  else
    export_kernel<false><<<h->nblocks, BLOCK, 0, h->stream>>>(a, out);
  return hipGetLastError();
}

hipError_t launch_import(lbm_ctx* h, const float* in) {
  CollideArgs a;
  fill_args(h, a, h->cur, h->cur);
  if (h->cfg.storage == LBM_STORE_F16DEV)
    import_kernel<true><<<h->nblocks, BLOCK, 0, h->stream>>>(a, in);
  else
    import_kernel<false><<<h->nblocks, BLOCK, 0, h->stream>>>(a, in);
  return hipGetLastError();
}

// Replace the FP16 storage reference (u_ref: device double [3][ny], or null
// for none) and re-encode the current state.  Synchronises the stream.
hipError_t launch_set_reference(lbm_ctx* h, const double* u_ref) {
  const int ny = h->cfg.ny;
  if (!u_ref && !h->d_dref) return hipSuccess;  // no reference before or after
  float* dnew = nullptr;  // [ny][19] offsets, then [ny][19] pull offsets
  hipError_t e = hipSuccess;
  if (u_ref) {
    if ((e = hipMalloc(&dnew, sizeof(float) * 2 * ny * Q)) != hipSuccess) return e;
    dref_kernel<<<(ny * Q + 255) / 256, 256, 0, h->stream>>>(u_ref, ny, dnew, dnew + ny * Q);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    CollideArgs a;
    fill_args(h, a, h->cur, h->cur);
    recode_kernel<<<h->nblocks, BLOCK, 0, h->stream>>>(a, static_cast<_Float16*>(h->f[h->cur]), h->d_dref, dnew);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {  // the handle keeps its old reference
    if (dnew) (void)hipFree(dnew);
    return e;
  }
  if (h->d_dref && (e = hipFree(h->d_dref)) != hipSuccess) return e;
  h->d_dref = dnew;
  h->d_dpull = dnew ? dnew + ny * Q : nullptr;
  return hipSuccess;
}

// Float bricks <-> float SoA [19][N] for adjoint fields (always FP32).
hipError_t launch_field_export(lbm_ctx* h, const float* bricks, float* soa) {
  CollideArgs a;
  fill_args(h, a, h->cur, h->cur);
  a.src = bricks;
  export_kernel<false><<<h->nblocks, BLOCK, 0, h->stream>>>(a, soa);
  return hipGetLastError();
}

hipError_t launch_field_import(lbm_ctx* h, const float* soa, float* bricks) {
  CollideArgs a;
  fill_args(h, a, h->cur, h->cur);
  a.dst = bricks;
  import_kernel<false><<<h->nblocks, BLOCK, 0, h->stream>>>(a, soa);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t s) {
  const int64_t n4 = bytes / 16;
  const int64_t nb = (n4 + 255) / 256;
  if (nb < 1 || nb > 0x7fffffff) return hipErrorInvalidValue;
  copy_kernel<<<(unsigned)nb, 256, 0, s>>>(static_cast<const vec4f*>(src), static_cast<vec4f*>(dst), n4);
  return hipGetLastError();
}

}  // namespace lbm
