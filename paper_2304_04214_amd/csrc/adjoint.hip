// Discrete adjoint of the fused collide-stream step (the transpose of the
// linearised Algorithm 1 step of Xue, Yao, Davidson, arXiv 2304.04214), for
// gradients of statistics losses with respect to the STG amplitude scalings
// s_b (Sec. III.A, Eq. (22)-(25)) and the Smagorinsky constant C_s
// (Sec. II.B, Eq. (13)-(15)).
//
// Formulation.  Node X of step n -> n+1 pulls 19 values of s_n (Eq. (3) with
// the wall rules), applies its boundary rules, the wall force and the
// collision.  Every element of s_n is pulled by at most one node, so the
// adjoint of the pull is a scatter to the same addresses, with no conflicts:
// a thread recomputes its node's forward step from s_n, pulls
// lam_{n+1}(X) back through the collision, the wall force and the boundary
// rules to its 19 pulled values, and stores each at the address it was pulled
// from.  Couplings between nodes beyond the pull:
//  * wall model: a first off-wall cell reads the velocity of the next row;
//    its sensitivity goes back to that row through LDS (the block holds both);
//  * line-averaged wall model: every first off-wall cell of a wall line
//    (x, wall) takes the line's u_tau, a function of the z-mean of u_hat over
//    the line.  A first launch over the wall blocks stops each wall cell's
//    adjoint at dL/d(line u_tau) and sums it per line chunk; the main launch
//    then gives every cell of the line its share through the mean;
//  * convective outlet: the outlet node at x = nx-1 reads the pulled values of
//    the node at nx-2.  The thread of node (nx-2, y, z) does the outlet node
//    (nx-1, y, z) first, stores dL/dhist_n and adds the outlet node's
//    sensitivity to its upstream term to its own c_x < 0 values.
// Elements of s_n that no node pulls (on the x = 0 and x = nx-1 planes of an
// open channel) are set to zero by the thread of the node that holds them.
//
// The Newton solve for u_tau is differentiated through its converged root
// (implicit function theorem), not through the truncated iteration.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "internal.h"
#include "stream.h"

namespace lbm {
namespace {

// Moments (M v)_k of a population vector in the Appendix A.1 basis, from its
// opposite-pair sums and differences.
__device__ __forceinline__ void moments(const float v[Q], float m[Q]) {
  const Pairs p = make_pairs(v);
  const float* s = p.s;
  const float* d = p.d;
  const float T04 = s[0] + s[4], T26 = s[2] + s[6], T1357 = s[1] + s[3] + s[5] + s[7];
  m[0] = p.A + p.Bx + v[9];
  m[1] = 8.f * p.A - 11.f * p.Bx - 30.f * v[9];
  m[2] = p.A - 4.f * p.Bx + 12.f * v[9];
  m[3] = (d[3] + d[7]) - (d[1] + d[5] + d[8]);
  m[4] = (d[3] + d[7]) - (d[1] + d[5]) + 4.f * d[8];
  m[5] = d[4] - (d[0] + d[5] + d[6] + d[7]);
  m[6] = d[4] - (d[0] + d[5] + d[7]) + 4.f * d[6];
  m[7] = -(d[0] + d[1] + d[2] + d[3] + d[4]);
  m[8] = 4.f * d[2] - (d[0] + d[1] + d[3] + d[4]);
  m[9] = 2.f * (s[8] - T04) + T1357 - T26;
  m[10] = -2.f * T04 + T1357 + 2.f * T26 - 4.f * s[8];
  m[11] = (s[5] + s[6] + s[7]) - (s[1] + s[2] + s[3]);
  m[12] = (s[5] + s[7] - 2.f * s[6]) - (s[1] + s[3] - 2.f * s[2]);
  m[13] = s[5] - s[7];
  m[14] = s[0] - s[4];
  m[15] = s[1] - s[3];
  m[16] = (d[1] + d[7]) - (d[3] + d[5]);
  m[17] = (d[4] + d[5] + d[7]) - d[0];
  m[18] = (d[0] + d[4]) - (d[1] + d[3]);
}

// g += M^T nu, assembled per opposite pair (the transpose of moments()).
__device__ __forceinline__ void add_mt(float g[Q], const float nu[Q]) {
  const float P = nu[0] + 8.f * nu[1] + nu[2], Qx = nu[0] - 11.f * nu[1] - 4.f * nu[2];
  const float b910 = nu[9] + nu[10], c1112 = nu[11] + nu[12];
  const float h = 2.f * nu[10] - nu[9], kk = 2.f * nu[12] - nu[11];
  float E[9], O[9];
  E[0] = P - 2.f * b910 + nu[14];
  E[4] = P - 2.f * b910 - nu[14];
  E[1] = P + b910 - c1112 + nu[15];
  E[3] = P + b910 - c1112 - nu[15];
  E[5] = P + b910 + c1112 + nu[13];
  E[7] = P + b910 + c1112 - nu[13];
  E[2] = Qx + h + kk;
  E[6] = Qx + h - kk;
  E[8] = Qx + 2.f * nu[9] - 4.f * nu[10];
  const float B34 = nu[3] + nu[4], B56 = nu[5] + nu[6], B78 = nu[7] + nu[8];
  O[0] = -B56 - B78 - nu[17] + nu[18];
  O[4] = B56 - B78 + nu[17] + nu[18];
  O[1] = -B34 - B78 + nu[16] - nu[18];
  O[3] = B34 - B78 - nu[16] - nu[18];
  O[5] = -B34 - B56 - nu[16] + nu[17];
  O[7] = B34 - B56 + nu[16] + nu[17];
  O[2] = 4.f * nu[8] - nu[7];
  O[6] = 4.f * nu[6] - nu[5];
  O[8] = 4.f * nu[4] - nu[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    g[k] += E[k] + O[k];
    g[18 - k] += E[k] - O[k];
  }
  g[9] += nu[0] - 30.f * nu[1] + 12.f * nu[2];
}

// Adjoint of the regularised inlet (inlet_regularize): gb holds dL/d(inlet
// populations) on entry and dL/d(pulled populations) on return (zero for
// c_x > 0, which the rule does not read); ub receives dL/du_in.
__device__ __forceinline__ void inlet_adjoint(float rin, float ux, float uy, float uz, float gb[Q], float& ubx,
                                              float& uby, float& ubz) {
  // dL/dPi_neq
  float Pxx = 0.f, Pyy = 0.f, Pzz = 0.f, Pxy = 0.f, Pyz = 0.f, Pxz = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float c = 4.5f * (float)WD[i] * gb[i];
    Pxx += (CX[i] * CX[i] - 1.f / 3.f) * c;
    Pyy += (CY[i] * CY[i] - 1.f / 3.f) * c;
    Pzz += (CZ[i] * CZ[i] - 1.f / 3.f) * c;
    Pxy += (2 * CX[i] * CY[i]) * c;
    Pyz += (2 * CY[i] * CZ[i]) * c;
    Pxz += (2 * CX[i] * CZ[i]) * c;
  }
  const float uu15 = 1.5f * (ux * ux + uy * uy + uz * uz);
  const float i1u = 1.f / (1.f - ux);
  float rb = 0.f;
  ubx = uby = ubz = 0.f;
  float fb[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    // dL/df_neq_i (c_x <= 0 only enter Pi_neq, the c_x < 0 ones twice)
    float feqb = gb[i];
    fb[i] = 0.f;
    if (CX[i] <= 0) {
      const float fnb = (CX[i] * CX[i] - 1.f / 3.f) * Pxx + (CY[i] * CY[i] - 1.f / 3.f) * Pyy +
                        (CZ[i] * CZ[i] - 1.f / 3.f) * Pzz + (CX[i] * CY[i]) * Pxy + (CY[i] * CZ[i]) * Pyz +
                        (CX[i] * CZ[i]) * Pxz;
      const float mult = CX[i] == 0 ? 1.f : 2.f;
      fb[i] = mult * fnb;
      feqb -= mult * fnb;
    }
    // f_eq_i = w_i rin (1 + 3 cu + 4.5 cu^2 - 1.5 uu)
    const float cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
    const float wr = (float)WD[i] * feqb;
    rb += wr * (1.f + 3.f * cu + 4.5f * cu * cu - uu15);
    const float t = wr * rin * (3.f + 9.f * cu);
    ubx += t * CX[i] - wr * rin * 3.f * ux;
    uby += t * CY[i] - wr * rin * 3.f * uy;
    ubz += t * CZ[i] - wr * rin * 3.f * uz;
  }
  // rin = (rho_0 + 2 rho_-) / (1 - u_x)
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (CX[i] == 0) fb[i] += rb * i1u;
    if (CX[i] == -1) fb[i] += 2.f * rb * i1u;
    gb[i] = fb[i];
  }
  ubx += rb * rin * i1u;
}

// Whether this block scatters row y (block y-group gy, first row base).  The
// block that scatters a row must hold every term of its adjoint: with the
// wall model, row ny-2 receives the top wall row's sensitivity, so it belongs
// to the top block even where ragged ny puts it in another group.
__device__ __forceinline__ bool row_owned(const CollideArgs& a, int y, int gy, int base) {
  if (a.wall_model && y == a.ny - 2) return base == a.ny - YROWS;
  return y >= YROWS * gy;
}

// Per-block state of the adjoint kernel.
struct AdjLds {
  float u2[2][2][ZT];  // forward: (u_x, u_z) of rows 1 and ny-2
  float g2[2][2][ZT];  // reverse: dL/d(u_x, u_z) of those rows, from the wall rows
  double part[YROWS];
  float gup[5][BLOCK];  // outlet node's U_c dL/dhist_n, for the node upstream of it
};

// The adjoint of one node (x, y, z) of the calling thread (see the file
// comment).  L.gup (the thread's slot): on the outlet plane (x = nx-1)
// receives U_c dL/dhist_n of the c_x < 0 populations; on the plane x = nx-2 it
// is added to them.  csb: the node's dL/dC_s is added.  Block-uniform x;
// contains __syncthreads.
//
// PROBE (line-averaged model only): stop after the wall force and store the
// wave's sum of dL/d(line u_tau) of the wall rows in A.line_part.
// REF (FP16 storage relative to a reference profile): dref / dpull are the
// reference offsets of the stored rows and of the plain pulls' source rows,
// passed as restrict kernel arguments so that their scalar loads are not
// ordered after stores (the values of a.dref / a.dpull).
template <bool F16, bool REF, bool PROBE = false>
__device__ __forceinline__ void node_adjoint(const AdjointArgs& A, AdjLds& L, int x, int y, int z, int lane,
                                             int base, int zci, bool own, bool active, float& csb,
                                             const float* __restrict__ dref, const float* __restrict__ dpull) {
  const CollideArgs& a = A.c;
  const bool mine = own && active;
  const Col col = make_col<F16>(a, z);
  const Geo g = make_geo(a, x, y);
  typename Pop<F16>::Raw r[Q];
  issue_pulls<F16>(a, g, col, r);
  const uint32_t erow = rowpart(a, x, y) + col.c0;
  float f[Q];
  if (!F16 || !REF) {
    convert_pulls<F16>(a, g, r, f);
  } else if (interior(g)) {  // wave-uniform: plain pulls, offsets of the source rows y - c_y
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = Pop<F16>::cvt(i, r[i], dpull[y * Q + i]);
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      int plane, ysrc;
      pull_plane_row(a, g, i, plane, ysrc);
      f[i] = pull_ok(a, g, i) ? Pop<F16>::cvt(i, r[i], dref[ysrc * Q + plane]) : 0.f;
    }
  }

  // ---- forward recompute: boundary rules ----
  const bool inflow = a.xbc == LBM_X_INFLOW;
  const bool outlet = inflow && x == a.nx - 1, inlet = inflow && x == 0;
  if (outlet) {
    const Geo g2 = make_geo(a, x - 1, y);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int i = OUT5[k];
      const float up = pull_dir<F16>(a, g2, i, col, 0.f);
      f[i] = a.out_wh * a.hist_in[(k * a.ny + y) * a.nz + z] + a.out_wu * up;
    }
  }
  float rin = 0.f;
  if (inlet) rin = inlet_regularize(a, y, z, f);

  // ---- forward recompute: density, momentum, wall force ----
  const Pairs pr = make_pairs(f);
  const float rho = pr.A + pr.Bx + f[9];
  const float jx = (pr.d[3] + pr.d[7]) - (pr.d[1] + pr.d[5] + pr.d[8]);
  const float jy = pr.d[4] - (pr.d[0] + pr.d[5] + pr.d[6] + pr.d[7]);
  const float jz = -(pr.d[0] + pr.d[1] + pr.d[2] + pr.d[3] + pr.d[4]);
  float Fx = rho * a.g[0], Fy = rho * a.g[1], Fz = rho * a.g[2];
  const bool bot = base == 0, top = base == a.ny - YROWS;
  const bool wblock = a.wall_model && (bot || top);  // block-uniform
  const bool wrow = wblock && ((bot && y == 0) || (top && y == a.ny - 1));
  const bool nrow = wblock && ((bot && y == 1) || (top && y == a.ny - 2));
  const int wslot = (bot && y <= 1) ? 0 : 1;
  bool wact = false, wbas = false;  // force applied; base vector defined
  // wall state kept for the reverse sweep: e_x, 1/|t|, the signed u_tau (the
  // force is -rho wsu |wsu| e_x), d(u_tau u+)/du_tau and the pre-force u_w
  float wex = 0.f, wez = 0.f, witn = 0.f, wsu = 0.f, wdg = 1.f, uwx = 0.f, uwz = 0.f;
  if (wblock) {
    const float iw = 1.f / rho;  // pre-force velocities j / rho of the wall model
    uwx = jx * iw;
    uwz = jz * iw;
    if (nrow) {
      L.u2[wslot][0][lane] = uwx;
      L.u2[wslot][1][lane] = uwz;
    }
    __syncthreads();
    if (wrow) {
      const float u2x = L.u2[wslot][0][lane], u2z = L.u2[wslot][1][lane];
      const float tn2 = u2x * u2x + u2z * u2z;
      if (tn2 > 0.f && a.wall_line) {  // line-averaged: the line's signed u_tau
        wbas = true;
        witn = 1.f / sqrtf(tn2);
        wex = u2x * witn;
        wez = u2z * witn;
        wsu = a.wall_line[wslot * a.nx + x];
        if (wsu != 0.f) {
          wact = true;
          const float wtw = -rho * wsu * fabsf(wsu);
          Fx += wtw * wex;
          Fz += wtw * wez;
          const float yp = a.y_wall * fabsf(wsu) * a.inv_nu0;
          float up, dup;
          wall_law(a, yp, up, dup);
          wdg = up + yp * dup;  // d(u_tau u+)/du_tau at the line's root
        }
      } else if (tn2 > 0.f) {
        wbas = true;
        witn = 1.f / sqrtf(tn2);
        wex = u2x * witn;
        wez = u2z * witn;
        const float uhat = uwx * wex + uwz * wez;
        if (uhat != 0.f) {
          wact = true;
          const float ut = newton_utau(a, fabsf(uhat));
          wsu = uhat > 0.f ? ut : -ut;
          const float wtw = -rho * wsu * ut;
          Fx += wtw * wex;
          Fz += wtw * wez;
          const float yp = a.y_wall * ut * a.inv_nu0;
          float up, dup;
          wall_law(a, yp, up, dup);
          wdg = up + yp * dup;  // d(u_tau u+)/du_tau at the root
        }
      }
    }
  }

  // ---- forward recompute: collision quantities (as in collide()) ----
  float ml[Q];
  moments(f, ml);
  const float ir = rcp_fast(rho);
  const float px = jx + 0.5f * Fx, py = jy + 0.5f * Fy, pz = jz + 0.5f * Fz;
  const float ux = px * ir, uy = py * ir, uz = pz * ir;
  const float uxx = ux * ux, uyy = uy * uy, uzz = uz * uz, uu = uxx + uyy + uzz;
  const float e1 = ml[1] - rho * (19.f * uu - 11.f);
  const float q9 = rho * (2.f * uxx - uyy - uzz);
  const float q11 = rho * (uyy - uzz);
  const float e9 = ml[9] - q9;
  const float e11 = ml[11] - q11;
  const float e13 = ml[13] - px * uy, e14 = ml[14] - py * uz, e15 = ml[15] - px * uz;
  const float dc2 = e1 * (1.f / 19.f);
  const float pxx = (e9 + dc2) * (1.f / 3.f);
  const float pyy = 0.5f * (dc2 - pxx + e11), pzz = 0.5f * (dc2 - pxx - e11);
  const float q2 = pxx * pxx + pyy * pyy + pzz * pzz + 2.f * (e13 * e13 + e14 * e14 + e15 * e15);
  const float Qh = sqrt_fast(q2);
  const Tau0 t0 = tau0_of_x(a, x);
  const float rr = sqrt_fast(t0.tau0sq + a.smag * Qh * ir);
  const float tau = 0.5f * t0.tau0 + 0.5f * rr;
  const float sv = rcp_fast(tau);
  const float hv = 1.f - 0.5f * sv;
  const float F9 = 2.f * (2.f * ux * Fx - uy * Fy - uz * Fz);
  const float F11 = 2.f * (uy * Fy - uz * Fz);
  const float F13 = ux * Fy + uy * Fx, F14 = uy * Fz + uz * Fy, F15 = ux * Fz + uz * Fx;

  // ---- reverse: collision ----
  // lambda_{n+1}(X) is loaded here rather than with the pulls, so that it holds
  // no registers through the forward recompute, and is not kept past its
  // moments: the rows of M are orthogonal with M M^T = D, so lambda =
  // M^T D^-1 (M lambda) and dL/df = lambda + M^T nu = M^T (D^-1 M lambda + nu),
  // with D^-1 M lambda folded into nu once the cotangents nu_k have been read.
  float lam[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) lam[i] = A.lam_next[erow + (uint32_t)i * ZT];
  moments(lam, ml);  // (M lambda)_k; delta_k / D_k enters f*, so mu_k = (M lambda)_k / D_k
  float nu[Q];       // dL/dm (moment-space cotangent of the pre-collision populations)
  nu[1] = -a.rs[1] * ml[1];
  nu[2] = -a.rs[2] * ml[2];
  nu[4] = -a.rs[4] * ml[4];
  nu[6] = -a.rs[6] * ml[6];
  nu[8] = -a.rs[8] * ml[8];
  nu[10] = -a.rs[10] * ml[10];
  nu[12] = -a.rs[12] * ml[12];
  // nu_16..18 are not read below: fold at once
  nu[16] = 0.125f * ml[16] - a.rs[16] * ml[16];
  nu[17] = 0.125f * ml[17] - a.rs[17] * ml[17];
  nu[18] = 0.125f * ml[18] - a.rs[18] * ml[18];
  // (D^-1 M lambda)_k of the conserved moments
  const float lam0 = ml[0] * (1.f / 19.f), lam3 = 0.1f * ml[3], lam5 = 0.1f * ml[5], lam7 = 0.1f * ml[7];
  const float Fb1 = a.rf[1] * ml[1], Fb2 = a.rf[2] * ml[2], Fb4 = a.rf[4] * ml[4], Fb6 = a.rf[6] * ml[6];
  const float Fb8 = a.rf[8] * ml[8], Fb10 = a.rf[10] * ml[10], Fb12 = a.rf[12] * ml[12];
  const float mu9 = ml[9] * (1.f / 36.f), mu11 = ml[11] * (1.f / 12.f);
  const float mu13 = 0.25f * ml[13], mu14 = 0.25f * ml[14], mu15 = 0.25f * ml[15];
  nu[9] = -sv * mu9;
  nu[11] = -sv * mu11;
  nu[13] = -sv * mu13;
  nu[14] = -sv * mu14;
  nu[15] = -sv * mu15;
  const float Fb9 = hv * mu9, Fb11 = hv * mu11, Fb13 = hv * mu13, Fb14 = hv * mu14, Fb15 = hv * mu15;
  // viscous rate 1/tau_eff -> tau_eff -> Q^(1/2), rho and C_s
  const float svb = -(mu9 * (e9 + 0.5f * F9) + mu11 * (e11 + 0.5f * F11) + mu13 * (e13 + 0.5f * F13) +
                      mu14 * (e14 + 0.5f * F14) + mu15 * (e15 + 0.5f * F15));
  const float taub = -svb * sv * sv;
  const float Xb = taub * 0.25f * rcp_fast(rr);
  const float Qhb = Xb * a.smag * ir;
  float rhob = -Xb * a.smag * Qh * ir * ir;
  if (mine) csb += Xb * Qh * ir * A.dsmag;
  const float q2b = Qh > 0.f ? 0.5f * Qhb * rcp_fast(Qh) : 0.f;
  {
    const float pxxb = 2.f * q2b * pxx, pyyb = 2.f * q2b * pyy, pzzb = 2.f * q2b * pzz;
    nu[13] += 4.f * q2b * e13;
    nu[14] += 4.f * q2b * e14;
    nu[15] += 4.f * q2b * e15;
    const float Pt = pxxb - 0.5f * (pyyb + pzzb);
    const float dc2b = 0.5f * (pyyb + pzzb) + Pt * (1.f / 3.f);
    nu[11] += 0.5f * (pyyb - pzzb);
    nu[9] += Pt * (1.f / 3.f);
    nu[1] += dc2b * (1.f / 19.f);
  }
  // equilibrium moments as functions of rho and p = rho u (e_k = m_k - m_eq_k)
  const float q9b = -nu[9] + 0.5f * nu[10], q11b = -nu[11] + 0.5f * nu[12];
  float pxb = -38.f * ux * nu[1] + 11.f * ux * nu[2] + (2.f / 3.f) * nu[4] + 4.f * ux * q9b - uy * nu[13] -
              uz * nu[15];
  float pyb = -38.f * uy * nu[1] + 11.f * uy * nu[2] + (2.f / 3.f) * nu[6] - 2.f * uy * q9b + 2.f * uy * q11b -
              ux * nu[13] - uz * nu[14];
  float pzb = -38.f * uz * nu[1] + 11.f * uz * nu[2] + (2.f / 3.f) * nu[8] - 2.f * uz * q9b - 2.f * uz * q11b -
              uy * nu[14] - ux * nu[15];
  rhob += (19.f * uu + 11.f) * nu[1] - (3.f + 5.5f * uu) * nu[2] - (2.f * uxx - uyy - uzz) * q9b -
          (uyy - uzz) * q11b + ux * uy * nu[13] + uy * uz * nu[14] + ux * uz * nu[15];
  // last read of nu_1..15: fold D^-1 M lambda
  nu[1] += (1.f / 2394.f) * ml[1];
  nu[2] += (1.f / 252.f) * ml[2];
  nu[4] += (1.f / 40.f) * ml[4];
  nu[6] += (1.f / 40.f) * ml[6];
  nu[8] += (1.f / 40.f) * ml[8];
  nu[10] += (1.f / 72.f) * ml[10];
  nu[12] += (1.f / 24.f) * ml[12];
  nu[9] += mu9;
  nu[11] += mu11;
  nu[13] += mu13;
  nu[14] += mu14;
  nu[15] += mu15;
  // Guo force moments F_k(u, F); the conserved moments 3, 5, 7 gain F itself
  const float uFb = 38.f * Fb1 - 11.f * Fb2;
  const float A9 = Fb9 - 0.5f * Fb10, A11 = Fb11 - 0.5f * Fb12;
  float uxb = uFb * Fx + 4.f * A9 * Fx + Fb13 * Fy + Fb15 * Fz;
  float uyb = uFb * Fy - 2.f * A9 * Fy + 2.f * A11 * Fy + Fb13 * Fx + Fb14 * Fz;
  float uzb = uFb * Fz - 2.f * A9 * Fz - 2.f * A11 * Fz + Fb14 * Fy + Fb15 * Fx;
  float Fxb = uFb * ux - (2.f / 3.f) * Fb4 + 4.f * A9 * ux + Fb13 * uy + Fb15 * uz + lam3;
  float Fyb = uFb * uy - (2.f / 3.f) * Fb6 - 2.f * A9 * uy + 2.f * A11 * uy + Fb13 * ux + Fb14 * uz + lam5;
  float Fzb = uFb * uz - (2.f / 3.f) * Fb8 - 2.f * A9 * uz - 2.f * A11 * uz + Fb14 * uy + Fb15 * ux + lam7;
  // statistics source: d/du of sum_k coef_k (u, v, w, uu, vv, ww, uv, uw, vw)
  if (A.coef) {
    const int p = a.plane_of_x[x];
    if (p >= 0) {
      const float* c = A.coef + ((size_t)p * a.ny + y) * 9;
      uxb += c[0] + 2.f * c[3] * ux + c[6] * uy + c[7] * uz;
      uyb += c[1] + 2.f * c[4] * uy + c[6] * ux + c[8] * uz;
      uzb += c[2] + 2.f * c[5] * uz + c[7] * ux + c[8] * uy;
    }
  }
  // u = p / rho, p = j + F / 2, F = rho g + F_w
  pxb += uxb * ir;
  pyb += uyb * ir;
  pzb += uzb * ir;
  rhob -= (uxb * ux + uyb * uy + uzb * uz) * ir;
  float jxb = pxb, jyb = pyb, jzb = pzb;
  Fxb += 0.5f * pxb;
  Fyb += 0.5f * pyb;
  Fzb += 0.5f * pzb;
  rhob += Fxb * a.g[0] + Fyb * a.g[1] + Fzb * a.g[2];

  // ---- reverse: wall force F_w = -sign(u_hat) rho u_tau^2 e ----
  if (wblock) {
    float u2xb = 0.f, u2zb = 0.f;
    if (a.wall_line) {
      float exb = 0.f, ezb = 0.f, uhb = 0.f, lb = 0.f;
      if (wact) {  // rho and e_x of the cell itself; u_tau of the line
        const float twb = Fxb * wex + Fzb * wez;
        const float wtw = -rho * wsu * fabsf(wsu);
        exb = wtw * Fxb;
        ezb = wtw * Fzb;
        rhob -= twb * wsu * fabsf(wsu);  // d tw / d rho = tw / rho
        lb = -2.f * twb * rho * fabsf(wsu);  // d tw / d line = 2 tw / line
      }
      if constexpr (PROBE) {
        if (wrow) {  // wave-uniform: the whole wave reduces
          double v = (active && wact) ? (double)lb : 0.0;
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, ZT);
          if (lane == 0) A.line_part[((size_t)wslot * a.nx + x) * a.zc + zci] = v;
        }
        return;
      }
      if (wact) {
        double s = 0.0;  // dL/d(line u_tau): the line's chunks in order
        for (int k = 0; k < a.zc; ++k) s += A.line_part[((size_t)wslot * a.nx + x) * a.zc + k];
        uhb = (float)s / (wdg * (float)a.nz);  // d line / d mean = 1 / wdg; d mean / d u_hat = 1 / nz
      }
      if (wbas) {  // u_hat = u_w . e_x of this cell entered the line's mean
        const float iw = 1.f / rho;
        exb += uhb * uwx;
        ezb += uhb * uwz;
        const float uwxb = uhb * wex, uwzb = uhb * wez;
        jxb += uwxb * iw;
        jzb += uwzb * iw;
        rhob -= (uwxb * uwx + uwzb * uwz) * iw;
        const float ed = wex * exb + wez * ezb;  // e = t / |t|
        u2xb = (exb - wex * ed) * witn;
        u2zb = (ezb - wez * ed) * witn;
      }
    } else if (wact) {
      const float twb = Fxb * wex + Fzb * wez;
      const float ut = fabsf(wsu), wtw = -rho * wsu * ut;
      const float iw = 1.f / rho;
      float exb = wtw * Fxb, ezb = wtw * Fzb;
      rhob -= twb * wsu * ut;  // d tw / d rho = tw / rho
      // d tw / du_tau = 2 tw / u_tau; du_tau/d|u_hat| = 1 / wdg; d|u_hat|/du_hat = sign(u_hat)
      const float uhb = -2.f * twb * rho * ut / wdg;
      exb += uhb * uwx;
      ezb += uhb * uwz;
      const float uwxb = uhb * wex, uwzb = uhb * wez;
      jxb += uwxb * iw;
      jzb += uwzb * iw;
      rhob -= (uwxb * uwx + uwzb * uwz) * iw;
      const float ed = wex * exb + wez * ezb;  // e = t / |t|
      u2xb = (exb - wex * ed) * witn;
      u2zb = (ezb - wez * ed) * witn;
    }
    if (wrow) {
      L.g2[wslot][0][lane] = u2xb;
      L.g2[wslot][1][lane] = u2zb;
    }
    __syncthreads();
    if (nrow) {  // this row's pre-force velocity fed the wall row's base vector
      const float gx = L.g2[wslot][0][lane], gz = L.g2[wslot][1][lane];
      const float iw = 1.f / rho;
      jxb += gx * iw;
      jzb += gz * iw;
      rhob -= (gx * uwx + gz * uwz) * iw;
    }
  }
  if constexpr (PROBE) return;

  // ---- dL/d(post-boundary populations) = M^T (D^-1 M lambda + nu) ----
  nu[0] = lam0 + rhob;
  nu[3] = lam3 + jxb;
  nu[5] = lam5 + jyb;
  nu[7] = lam7 + jzb;
#pragma unroll
  for (int i = 0; i < Q; ++i) lam[i] = 0.f;
  add_mt(lam, nu);
  float* gb = lam;

  // ---- reverse: boundary rules ----
  if (outlet) {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int i = OUT5[k];
      const int hidx = (k * a.ny + y) * a.nz + z;
      const float t = gb[i] + A.eta_next[hidx];  // hist_{n+1} holds these populations
      if (mine) A.eta_prev[hidx] = a.out_wh * t;
      L.gup[k][threadIdx.x] = a.out_wu * t;
      gb[i] = 0.f;
    }
  }
  if (inflow && x == a.nx - 2) {  // values the outlet node read through its upstream term
#pragma unroll
    for (int k = 0; k < 5; ++k) gb[OUT5[k]] += L.gup[k][threadIdx.x];
  }
  const Col cl = make_col<false>(a, z);
  char* lp = reinterpret_cast<char*>(A.lam_prev);
  if (inlet) {
    const int pl = a.ny * a.nz, o = y * a.nz + z;
    const float uix = a.u_in[o], uiy = a.u_in[pl + o], uiz = a.u_in[2 * pl + o];
    float ubx, uby, ubz;
    inlet_adjoint(rin, uix, uiy, uiz, gb, ubx, uby, ubz);
    if (mine) {
      A.g_uin[o] = ubx;
      A.g_uin[pl + o] = uby;
      A.g_uin[2 * pl + o] = ubz;
    }
    // dL/ds_b: sum over the row of g_uin . (a v'), per wave (FP64, fixed order)
    double v = mine ? (double)ubx * A.fluct[o] + (double)uby * A.fluct[pl + o] + (double)ubz * A.fluct[2 * pl + o]
                    : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, ZT);
    if (lane == 0 && own) A.amp_part[y * a.zc + zci] += v;  // one writer per entry and step
  }
  // Populations of an open channel's end planes that no node pulls (c_x = -1
  // at x = 0, c_x = +1 at x = nx-1) are zero; the only other writer of such an
  // element is this thread's own bounce-back scatter below, which follows.
  if (mine && (inlet || outlet)) {
    const int cxz = inlet ? -1 : 1;
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (CX[i] == cxz)
        *reinterpret_cast<float*>(lp + (size_t)(rowpart(a, x, y) + (uint32_t)i * ZT) * 4u + cl.b0) = 0.f;
  }

  // ---- scatter to the addresses the pulls read ----
  if (mine) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int cx = CX[i], cy = CY[i], cz = CZ[i];
      uint32_t cs = cz == 1 ? cl.bm : (cz == -1 ? cl.bp : cl.b0);
      int plane = i, xsrc = g.xs[cx + 1], ysrc = g.ys[cy + 1];
      if (cy != 0) {
        const bool out = g.yout[cy + 1];
        const bool bb = out && a.ywall == LBM_Y_BOUNCEBACK;
        plane = out ? (bb ? opp(i) : REFLY[i]) : i;
        xsrc = bb ? g.x : xsrc;
        ysrc = out ? g.y : ysrc;
        cs = bb ? cl.b0 : cs;
      }
      if (pull_ok(a, g, i))
        *reinterpret_cast<float*>(lp + (size_t)(rowpart(a, xsrc, ysrc) + (uint32_t)plane * ZT) * 4u + cs) = gb[i];
    }
  }
}

// One thread per node; a block is 4 consecutive y rows of one (x, z-chunk),
// the block entry blist[blockIdx.x] (adjoint_list: the planes x = 0 and
// x = nx-2 of an open channel first, so that their longer work overlaps the
// rest; -1 pads).  Each block at nx-2 first does the outlet node of its
// (y, z) (x = nx-1), whose dL/dhist feeds its own c_x < 0 values.
// Held to 96 VGPRs: 5 waves per SIMD instead of 4, at the cost of one spilled
// VGPR with FP16 states and 11 with FP32 states (measured faster for both).
template <bool F16, bool REF>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(5)))
void adjoint_kernel(AdjointArgs A, const int* __restrict__ blist, const float* __restrict__ dref,
                    const float* __restrict__ dpull) {
  __shared__ AdjLds L;
  const CollideArgs& a = A.c;
  const int e = blist[blockIdx.x];
  if (e < 0) return;  // block-uniform
  const bool open = a.xbc == LBM_X_INFLOW;
  int x0, zci, gy;
  block_coords(a, e, x0, zci, gy);
  const int lane = threadIdx.x & (ZT - 1);
  const int w = uni(threadIdx.x >> 6);
  const int base = min(YROWS * gy, a.ny - YROWS);
  const int y = base + w;
  const int zraw = zci * ZT + lane;
  const bool active = zraw < a.nz;
  const int z = active ? zraw : a.nz - 1;  // inactive lanes compute a valid node and store nothing
  const bool own = row_owned(a, y, gy, base);
  float csb = 0.f;
  if (open && x0 == a.nx - 2) {  // block-uniform
    node_adjoint<F16, REF>(A, L, a.nx - 1, y, z, lane, base, zci, own, active, csb, dref, dpull);
    __syncthreads();  // LDS reuse by the second node
  }
  node_adjoint<F16, REF>(A, L, x0, y, z, lane, base, zci, own, active, csb, dref, dpull);
  // dL/dC_s of the block (fixed-order FP64 reduction)
  double c = (double)csb;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, ZT);
  if (lane == 0) L.part[w] = c;
  __syncthreads();
  if (threadIdx.x == 0) A.cs_part[e] += ((L.part[0] + L.part[1]) + L.part[2]) + L.part[3];  // one writer per step
}

// Line-averaged wall model: the wall blocks (y-groups 0 and yg-1 of every
// (x, z-chunk)) store dL/d(line u_tau) per wall-line chunk; every chunk of
// every line is written, so the main launch reads no stale sums.
template <bool F16, bool REF>
__global__ __launch_bounds__(BLOCK) void adjoint_line_probe_kernel(AdjointArgs A, const float* __restrict__ dref,
                                                                  const float* __restrict__ dpull) {
  __shared__ AdjLds L;
  const CollideArgs& a = A.c;
  const int ng = a.yg > 1 ? 2 : 1;
  const int b = (int)blockIdx.x;
  const int k = b % ng, zci = (b / ng) % a.zc, x = b / (ng * a.zc);
  const int gy = k == 0 ? 0 : a.yg - 1;
  const int lane = threadIdx.x & (ZT - 1);
  const int base = min(YROWS * gy, a.ny - YROWS);
  const int y = base + uni(threadIdx.x >> 6);
  const int zraw = zci * ZT + lane;
  const bool active = zraw < a.nz;
  const int z = active ? zraw : a.nz - 1;
  float csb = 0.f;
  node_adjoint<F16, REF, true>(A, L, x, y, z, lane, base, zci, row_owned(a, y, gy, base), active, csb, dref,
                               dpull);
}

// grad[n_bins] += the accumulated per-block dL/dC_s (fixed-order tree), and
// grad[b] += the accumulated inlet-row partial sums of bin b (rows, then
// z-chunks, in order).  The accumulators are cleared for the next sweep.
__global__ __launch_bounds__(256) void adjoint_finalize_kernel(double* cs_part, int nparts, double* amp_part, int zc,
                                                               const int* bin_of_y, int ny, int n_bins,
                                                               double* grad) {
  __shared__ double part[256];
  __shared__ double rows[LBM_ADJ_MAX_NY];
  __shared__ int bins[LBM_ADJ_MAX_NY];
  double s = 0.0;
  for (int k = threadIdx.x; k < nparts; k += 256) {
    s += cs_part[k];
    cs_part[k] = 0.0;
  }
  part[threadIdx.x] = s;
  if (amp_part)
    for (int y = threadIdx.x; y < ny; y += 256) {
      double r = 0.0;
      for (int c = 0; c < zc; ++c) {
        r += amp_part[y * zc + c];
        amp_part[y * zc + c] = 0.0;
      }
      rows[y] = r;
      const int by = bin_of_y[y];
      bins[y] = by < 0 ? 0 : (by >= n_bins ? n_bins - 1 : by);  // clamped like the STG binding
    }
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[n_bins] += part[0];
  if (amp_part)
    for (int bn = threadIdx.x; bn < n_bins; bn += 256) {
      double acc = 0.0;
      for (int y = 0; y < ny; ++y)
        if (bins[y] == bn) acc += rows[y];
      grad[bn] += acc;
    }
}

}  // namespace

// Block entries whose partial sums the accumulators hold: x = 0 .. nx-2 of
// an open channel (the plane nx-2 includes the outlet plane), all blocks of a
// periodic one.
int adjoint_blocks(const lbm_ctx* h) {
  return h->cfg.xbc == LBM_X_INFLOW ? (h->cfg.nx - 1) * h->zc * h->yg : h->nblocks;
}

// Dispatch order of the adjoint's block entries, built on the first adjoint
// step: the open channel's planes x = 0 and x = nx-2, then the other columns
// (x, y-group) dealt to the XCDs by xcd_order, the y-groups holding a wall row
// (longer work) with their own turn.  Columns whole on one XCD also keep the
// partial cache lines of the +-1 z scatters of neighbouring z-chunks in one L2.
hipError_t adjoint_list(lbm_ctx* h) {
  if (h->d_ablist) return hipSuccess;
  const lbm_config& c = h->cfg;
  const bool open = c.xbc == LBM_X_INFLOW;
  const bool walls = c.ywall != LBM_Y_PERIODIC;
  std::vector<int> ends, rest;
  std::vector<char> heavy;
  for (int x = 0; x < (open ? c.nx - 1 : c.nx); ++x) {
    const bool end = open && (x == 0 || x == c.nx - 2);
    for (int gy = 0; gy < h->yg; ++gy) {
      if (!end) heavy.push_back(walls && (gy == 0 || gy == h->yg - 1));
      for (int zci = 0; zci < h->zc; ++zci) (end ? ends : rest).push_back((x * h->zc + zci) * h->yg + gy);
    }
  }
  rest = xcd_order(rest, h->zc, &heavy);
  ends.insert(ends.end(), rest.begin(), rest.end());
  hipError_t err;
  if ((err = hipMalloc(&h->d_ablist, sizeof(int) * ends.size())) != hipSuccess) return err;
  if ((err = hipMemcpy(h->d_ablist, ends.data(), sizeof(int) * ends.size(), hipMemcpyHostToDevice)) != hipSuccess) {
    (void)hipFree(h->d_ablist);
    h->d_ablist = nullptr;
    return err;
  }
  h->n_ablist = (int)ends.size();
  return hipSuccess;
}

// One launch over all block entries of adjoint_blocks() (in adjoint_list's
// order); the inlet plane at t_next, unless given, is computed first.
// With the line-averaged wall model the step's line u_tau is recomputed from
// s_n and the inlet plane, and the probe launch runs before the main one.
hipError_t launch_adjoint(lbm_ctx* h, const AdjointArgs& args, int storage_f16, double t_next, bool fill_inlet,
                          float* u_in, float* fluct) {
  hipError_t e;
  if (fill_inlet && (e = launch_stg_fill(h, t_next, h->stream, fluct, u_in)) != hipSuccess) return e;
  AdjointArgs A = args;
  if ((e = launch_wall_line(h, A.c, h->stream)) != hipSuccess) return e;
  if (A.c.wall_line) {
    const lbm_config& c = h->cfg;
    if (!h->d_line_part && (e = hipMalloc(&h->d_line_part, sizeof(double) * 2 * c.nx * h->zc)) != hipSuccess)
      return e;
    A.line_part = h->d_line_part;
    const int nprobe = c.nx * h->zc * (h->yg > 1 ? 2 : 1);
    if (storage_f16 && A.c.dref)
      adjoint_line_probe_kernel<true, true><<<nprobe, BLOCK, 0, h->stream>>>(A, A.c.dref, A.c.dpull);
    else if (storage_f16)
      adjoint_line_probe_kernel<true, false><<<nprobe, BLOCK, 0, h->stream>>>(A, nullptr, nullptr);
    else
      adjoint_line_probe_kernel<false, false><<<nprobe, BLOCK, 0, h->stream>>>(A, nullptr, nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = adjoint_list(h)) != hipSuccess) return e;
  if (storage_f16 && A.c.dref)
    adjoint_kernel<true, true><<<h->n_ablist, BLOCK, 0, h->stream>>>(A, h->d_ablist, A.c.dref, A.c.dpull);
  else if (storage_f16)
    adjoint_kernel<true, false><<<h->n_ablist, BLOCK, 0, h->stream>>>(A, h->d_ablist, nullptr, nullptr);
  else
    adjoint_kernel<false, false><<<h->n_ablist, BLOCK, 0, h->stream>>>(A, h->d_ablist, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_adjoint_reduce(lbm_ctx* h, double* grad) {
  const bool bins = h->cfg.xbc == LBM_X_INFLOW && h->stg_bound;
  adjoint_finalize_kernel<<<1, 256, 0, h->stream>>>(h->d_cs_part, adjoint_blocks(h), bins ? h->d_amp_part : nullptr,
                                                    h->zc, bins ? h->stg.bin_of_y : nullptr, h->cfg.ny,
                                                    bins ? h->stg.n_bins : 0, grad);
  return hipGetLastError();
}

}  // namespace lbm
