// Device-side building blocks shared by the forward collide-stream kernels
// and the adjoint kernels: population storage, the 64-node brick addressing,
// the pull geometry with the wall rules, opposite-pair sums and the wall-law
// Newton solve.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

#include <type_traits>

namespace lbm {

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Population storage: float, or half deviations h_i = f_i - w_i - r_i(y),
// where r_i(y) is the optional per-row reference offset of the storage
// (f_eq(1, U(y)) - w_i for a reference velocity profile U(y); 0 without one).
// The `ref` arguments carry r of the stored plane and row; float storage
// ignores them.
template <bool F16>
struct Pop;
// Loads take a wave-uniform element offset `row` (scalar) and a per-lane byte
// offset `cb`, so the address is scalar base + 32-bit vector offset.
template <>
struct Pop<false> {
  static constexpr uint32_t ES = 4;
  using Raw = float;
  __device__ static __forceinline__ Raw raw(const char* p, uint32_t off) {
    return *reinterpret_cast<const float*>(p + off);
  }
  __device__ static __forceinline__ float cvt(int, Raw r, float) { return r; }
  // p: wave-uniform byte pointer; off: per-lane byte offset (+ a constant)
  __device__ static __forceinline__ float ldp(const char* p, int, uint32_t off, float) {
    return *reinterpret_cast<const float*>(p + off);
  }
  // NT: non-temporal store (see CollideArgs::nt_store)
  template <bool NT>
  __device__ static __forceinline__ void stp(char* p, int, uint32_t off, float v, float) {
    if constexpr (NT)
      __builtin_nontemporal_store(v, reinterpret_cast<float*>(p + off));
    else
      *reinterpret_cast<float*>(p + off) = v;
  }
  __device__ static __forceinline__ void st_plain(void* base, int, uint32_t e, float v, float) {
    static_cast<float*>(base)[e] = v;
  }
  __device__ static __forceinline__ float ld_plain(const void* base, int, uint32_t e, float) {
    return static_cast<const float*>(base)[e];
  }
};
template <>
struct Pop<true> {
  static constexpr uint32_t ES = 2;
  using Raw = uint32_t;  // the 16-bit pattern of h_i
  __device__ static __forceinline__ Raw raw(const char* p, uint32_t off) {
    return *reinterpret_cast<const unsigned short*>(p + off);
  }
  __device__ static __forceinline__ float cvt(int i, Raw r, float ref) {
    return ((float)WD[i] + ref) + (float)__builtin_bit_cast(_Float16, (unsigned short)r);
  }
  // f = w_i + r_i + h_i
  __device__ static __forceinline__ float ldp(const char* p, int i, uint32_t off, float ref) {
    return ((float)WD[i] + ref) + (float)*reinterpret_cast<const _Float16*>(p + off);
  }
  // h_i = f - w_i - r_i rounded to nearest even half
  template <bool NT>
  __device__ static __forceinline__ void stp(char* p, int i, uint32_t off, float v, float ref) {
    stp_dev<NT>(p, off, (v - (float)WD[i]) - ref);
  }
  // The deviation from the weights f_i - w_i = h_i + r_i (kernels that compute
  // on deviations).
  __device__ static __forceinline__ float cvt_dev(Raw r) { return (float)__builtin_bit_cast(_Float16, (unsigned short)r); }
  __device__ static __forceinline__ float cvt_dev(Raw r, float ref) { return cvt_dev(r) + ref; }
  template <bool NT>
  __device__ static __forceinline__ void stp_dev(char* p, uint32_t off, float h, float ref) {
    stp_dev<NT>(p, off, h - ref);
  }
  template <bool NT>
  __device__ static __forceinline__ void stp_dev(char* p, uint32_t off, float h) {
    const unsigned short hb = __builtin_bit_cast(unsigned short, (_Float16)h);
    if constexpr (NT)
      __builtin_nontemporal_store(hb, reinterpret_cast<unsigned short*>(p + off));
    else
      *reinterpret_cast<unsigned short*>(p + off) = hb;
  }
  __device__ static __forceinline__ void st_plain(void* base, int i, uint32_t e, float v, float ref) {
    static_cast<_Float16*>(base)[e] = (_Float16)((v - (float)WD[i]) - ref);
  }
  __device__ static __forceinline__ float ld_plain(const void* base, int i, uint32_t e, float ref) {
    return ((float)WD[i] + ref) + (float)static_cast<const _Float16*>(base)[e];
  }
};

// Reference offset r_j(y) of stored plane j in row y (wave-uniform: a scalar
// load), 0 without a reference profile.
__device__ __forceinline__ float ref_off(const CollideArgs& a, int j, int y) {
  return a.dref ? a.dref[y * Q + j] : 0.f;
}

// Byte pointer to the start of the (x, y) brick row of a buffer (wave-uniform).
template <bool F16>
__device__ __forceinline__ const char* row_ptr(const void* base, uint32_t rowp) {
  return static_cast<const char*>(base) + (size_t)rowp * Pop<F16>::ES;
}

// Wave-uniform source rows of one node row (x, y).
struct Geo {
  int x, y;
  int xs[3];
  bool xok[3];  // index c_x + 1: source x = x - c_x and whether it lies in the lattice
  int ys[3];
  bool yout[3];  // index c_y + 1: source y and whether it lies beyond a wall
};

__device__ __forceinline__ Geo make_geo(const CollideArgs& a, int x, int y) {
  Geo g;
  g.x = x;
  g.y = y;
#pragma unroll
  for (int c = -1; c <= 1; ++c) {
    int s = x - c;
    bool ok = true;
    if (a.xbc == LBM_X_PERIODIC) {
      s = s < 0 ? s + a.nx : (s >= a.nx ? s - a.nx : s);
    } else {
      ok = s >= 0 && s < a.nx;
      s = s < 0 ? 0 : (s >= a.nx ? a.nx - 1 : s);
    }
    g.xs[c + 1] = s;
    g.xok[c + 1] = ok;
    int t = y - c;
    bool out = t < 0 || t >= a.ny;
    if (a.ywall == LBM_Y_PERIODIC) {
      t = t < 0 ? t + a.ny : (t >= a.ny ? t - a.ny : t);
      out = false;
    } else {
      t = t < 0 ? 0 : (t >= a.ny ? a.ny - 1 : t);
    }
    g.ys[c + 1] = t;
    g.yout[c + 1] = out;
  }
  return g;
}

constexpr uint32_t BRICK = Q * ZT;  // elements per 64-node brick

// Element offset contributed by (x, y) (wave-uniform) and by z (per lane).
__device__ __forceinline__ uint32_t rowpart(const CollideArgs& a, int x, int y) {
  return ((uint32_t)x * (uint32_t)(a.zc * a.ny) + (uint32_t)y) * BRICK;
}
__device__ __forceinline__ uint32_t colpart(const CollideArgs& a, int z) {
  return (uint32_t)(z >> 6) * (uint32_t)a.ny * BRICK + (uint32_t)(z & (ZT - 1));
}

// Column offsets of z and of its periodic neighbours z - 1 and z + 1, in
// elements and (times the element size) in bytes.
struct Col {
  uint32_t c0, b0, bm, bp;
};
template <bool F16>
__device__ __forceinline__ Col make_col(const CollideArgs& a, int z) {
  const int zm = z == 0 ? a.nz - 1 : z - 1;
  const int zp = z == a.nz - 1 ? 0 : z + 1;
  constexpr uint32_t es = Pop<F16>::ES;
  const uint32_t c0 = colpart(a, z);
  return Col{c0, c0 * es, colpart(a, zm) * es, colpart(a, zp) * es};
}

// Pull of direction i into node (g.x, g.y, z) with the wall rules
// (Eq. (3); halfway bounce-back or specular slip at the y walls).  Sources
// outside the x range (inlet unknowns, outlet) give `unset`.  The source plane,
// row and z are chosen by selects (scalar for plane and row) and the load is
// always issued from a valid address, so the 19 loads of a node form one
// straight-line batch.  Opposite and mirrored directions share w_i.
template <bool F16>
__device__ __forceinline__ float pull_dir(const CollideArgs& a, const Geo& g, int i, const Col& col, float unset) {
  const int cx = CX[i], cy = CY[i], cz = CZ[i];
  const uint32_t cs = cz == 1 ? col.bm : (cz == -1 ? col.bp : col.b0);
  int plane = i, xsrc = g.xs[cx + 1], ysrc = g.ys[cy + 1];
  uint32_t csrc = cs;
  bool ok = g.xok[cx + 1];
  if (cy != 0) {
    const bool out = g.yout[cy + 1];
    const bool bb = out && a.ywall == LBM_Y_BOUNCEBACK;
    plane = out ? (bb ? opp(i) : REFLY[i]) : i;
    xsrc = bb ? g.x : xsrc;
    ysrc = out ? g.y : ysrc;
    csrc = bb ? col.b0 : cs;
    ok = bb ? true : ok;
  }
  const char* p = row_ptr<F16>(a.src, rowpart(a, xsrc, ysrc) + (uint32_t)plane * ZT);
  const float v = Pop<F16>::ldp(p, i, csrc, ref_off(a, plane, ysrc));
  return ok ? v : unset;
}

// Whether the pulled source of direction i exists (false only for sources
// outside the x range: inlet unknowns and the outlet's c_x < 0 directions).
__device__ __forceinline__ bool pull_ok(const CollideArgs& a, const Geo& g, int i) {
  const int cx = CX[i], cy = CY[i];
  if (cy != 0 && g.yout[cy + 1] && a.ywall == LBM_Y_BOUNCEBACK) return true;
  return g.xok[cx + 1];
}

// A row whose 3 x 3 source rows all lie inside the lattice: no wall, inlet or
// outlet rule applies and the pulls are plain shifted loads.
__device__ __forceinline__ bool interior(const Geo& g) {
  return g.xok[0] && g.xok[2] && !g.yout[0] && !g.yout[2];
}

// Issue the 19 pull loads of node row g (raw storage values, no conversion),
// so that they can be in flight while another row is being collided.
template <bool F16>
__device__ __forceinline__ void issue_pulls(const CollideArgs& a, const Geo& g, const Col& col,
                                            typename Pop<F16>::Raw r[Q]) {
  if (interior(g)) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const uint32_t cs = CZ[i] == 1 ? col.bm : (CZ[i] == -1 ? col.bp : col.b0);
      r[i] = Pop<F16>::raw(row_ptr<F16>(a.src, rowpart(a, g.xs[CX[i] + 1], g.ys[CY[i] + 1]) + (uint32_t)i * ZT), cs);
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int cx = CX[i], cy = CY[i], cz = CZ[i];
      const uint32_t cs = cz == 1 ? col.bm : (cz == -1 ? col.bp : col.b0);
      int plane = i, xsrc = g.xs[cx + 1], ysrc = g.ys[cy + 1];
      uint32_t csrc = cs;
      if (cy != 0) {
        const bool out = g.yout[cy + 1];
        const bool bb = out && a.ywall == LBM_Y_BOUNCEBACK;
        plane = out ? (bb ? opp(i) : REFLY[i]) : i;
        xsrc = bb ? g.x : xsrc;
        ysrc = out ? g.y : ysrc;
        csrc = bb ? col.b0 : cs;
      }
      r[i] = Pop<F16>::raw(row_ptr<F16>(a.src, rowpart(a, xsrc, ysrc) + (uint32_t)plane * ZT), csrc);
    }
  }
}

// Stored plane and source row of the pull of direction i into row g (the
// wall rules of issue_pulls); wave-uniform.
__device__ __forceinline__ void pull_plane_row(const CollideArgs& a, const Geo& g, int i, int& plane, int& ysrc) {
  const int cy = CY[i];
  plane = i;
  ysrc = g.ys[cy + 1];
  if (cy != 0 && g.yout[cy + 1]) {
    plane = a.ywall == LBM_Y_BOUNCEBACK ? opp(i) : REFLY[i];
    ysrc = g.y;
  }
}

// Reference offset of the value the pull of direction i reads.
__device__ __forceinline__ float pull_ref(const CollideArgs& a, const Geo& g, int i) {
  int plane, ysrc;
  pull_plane_row(a, g, i, plane, ysrc);
  return ref_off(a, plane, ysrc);
}

// Populations from the raw loads; sources outside the x range give 0.
template <bool F16>
__device__ __forceinline__ void convert_pulls(const CollideArgs& a, const Geo& g, const typename Pop<F16>::Raw r[Q],
                                              float f[Q]) {
  if (interior(g)) {
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = Pop<F16>::cvt(i, r[i], ref_off(a, i, g.ys[CY[i] + 1]));
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = pull_ok(a, g, i) ? Pop<F16>::cvt(i, r[i], pull_ref(a, g, i)) : 0.f;
  }
}

// Sums and differences over the opposite pairs (i, 18 - i); density and
// momentum follow from them (Eq. (10)-(11)).
struct Pairs {
  float s[9], d[9], A, Bx;
};
__device__ __forceinline__ Pairs make_pairs(const float f[Q]) {
  Pairs p;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    p.s[k] = f[k] + f[18 - k];
    p.d[k] = f[k] - f[18 - k];
  }
  p.A = p.s[0] + p.s[1] + p.s[3] + p.s[4] + p.s[5] + p.s[7];
  p.Bx = p.s[2] + p.s[6] + p.s[8];
  return p;
}

__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }


__device__ __forceinline__ void block_coords(const CollideArgs& a, int e, int& x, int& zci, int& gy) {
  gy = e % a.yg;
  const int r = e / a.yg;
  zci = r % a.zc;
  x = r / a.zc;
}

// Molecular relaxation time of plane x (wave-uniform): tau0, or inside the
// outlet sponge 1/2 + 3 nu(x), nu(x) = nu0 + (nu_s - nu0) r^2,
// r = (x - x0 + 1) / L (Sec. IV.A names the sponge; the ramp is a reading).
struct Tau0 {
  float tau0, tau0sq;
};
__device__ __forceinline__ Tau0 tau0_of_x(const CollideArgs& a, int x) {
  if (x < a.sponge_x0) return Tau0{a.tau0, a.tau0sq};
  const float r = (float)(x - a.sponge_x0 + 1) * a.sponge_inv_len;
  const float t = 0.5f + 3.f * (a.nu0 + a.sponge_dnu * r * r);
  return Tau0{t, t * t};
}

// e^x through the hardware base-2 exponential (about 1 ulp; results below
// the normal range flush to 0, where the Reichardt terms are negligible).
__device__ __forceinline__ float exp_hw(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }

// log(1 + x), x > -1, from the hardware base-2 logarithm with the correction
// for the rounding of 1 + x (Goldberg): log(u) x / (u - 1), u = fl(1 + x), and
// x itself where u rounds to 1.  About 2 ulp, also for small x.
__device__ __forceinline__ float log1p_hw(float x) {
  const float u = 1.f + x, d = u - 1.f;
  const float l = __builtin_amdgcn_logf(u) * 0.693147180559945309f;
  return d == 0.f ? x : l * (x * rcp_fast(d));
}

// Reichardt law u+ and du+/dy+ (Sec. II.C, Eq. (16)) in FP32 from hardware
// transcendentals: e^(-y+/11) - 1 by its Taylor series up to t^6 where
// |t| = y+/11 < 0.3 (truncation below 2e-7 relative) so that small y+ loses no
// digits, log1p as above.  u+ within about 4e-7 relative of the exact law and
// u_tau of the Newton solve within about 2e-7 for y+ from 1e-4 to 1e4 (the
// library's expf / log1pf / expm1f cost five times the instructions, and the
// solve runs in every wall cell of every step).
__device__ __forceinline__ void reichardt(const CollideArgs& a, float yp, float& up, float& dup) {
  const float t = yp * (-1.f / 11.f);
  const float e1 = exp_hw(t), e3 = exp_hw(yp * (-1.f / 3.f));
  const float em1s =
      t * (1.f + t * (0.5f + t * ((1.f / 6.f) + t * ((1.f / 24.f) + t * ((1.f / 120.f) + t * (1.f / 720.f))))));
  const float em1 = t > -0.3f ? em1s : e1 - 1.f;
  up = log1p_hw(a.kappa * yp) * a.inv_kappa - a.b_reich * (em1 + yp * (1.f / 11.f) * e3);
  dup = rcp_fast(1.f + a.kappa * yp) + a.b_reich * ((e1 - e3) * (1.f / 11.f) + yp * (1.f / 33.f) * e3);
}

// Musker's explicit law of the wall (the alternative Sec. II.C names):
// u+ = 5.424 atan((2y+ - 8.15)/16.7) + log10((y+ + 10.6)^9.6 / (y+^2 - 8.15y+ + 86)^2) + C,
// C = -3.5113 so that u+(0) = 0 (the rounded -3.52 often printed leaves -0.0087 at the
// wall and no positive u_tau root below y+ = 0.009).
__device__ __forceinline__ void musker(float yp, float& up, float& dup) {
  constexpr float LOG10E = 0.43429448190325182f;
  const float t = (2.f * yp - 8.15f) * (1.f / 16.7f);
  const float q = yp * yp - 8.15f * yp + 86.f;  // > 0 for every y+
  // differences from y+ = 0 (atan(t) - atan(t0) = atan2(t - t0, 1 + t t0)): u+(0) = 0
  // exactly and no term cancels at small y+
  constexpr float T0 = -8.15f / 16.7f;
  up = 5.424f * atan2f(yp * (2.f / 16.7f), 1.f + T0 * t) +
       (9.6f * log1pf(yp * (1.f / 10.6f)) - 2.f * log1pf(yp * (yp - 8.15f) * (1.f / 86.f))) * LOG10E;
  dup = 5.424f * (2.f / 16.7f) / (1.f + t * t) + LOG10E * (9.6f / (yp + 10.6f) - 2.f * (2.f * yp - 8.15f) / q);
}

// The configured law of the wall (wave-uniform switch).
__device__ __forceinline__ void wall_law(const CollideArgs& a, float yp, float& up, float& dup) {
  if (a.wall_law == LBM_WALL_MUSKER)
    musker(yp, up, dup);
  else
    reichardt(a, yp, up, dup);
}

// u_tau from a fixed number of Newton steps on u_tau u+(y u_tau / nu0) = ua
// (Sec. II.C, Eq. (20)), started from the viscous-sublayer estimate.
__device__ __forceinline__ float newton_utau(const CollideArgs& a, float ua) {
  float ut = sqrt_fast(a.nu0 * ua * rcp_fast(a.y_wall));
  for (int it = 0; it < a.newton_iters; ++it) {
    const float yp = a.y_wall * ut * a.inv_nu0;
    float up, dup;
    wall_law(a, yp, up, dup);
    ut -= (ut * up - ua) * rcp_fast(up + yp * dup);  // the steps' own rounding is corrected by the next
  }
  return ut;
}

// Regularised inlet populations (Sec. III.A, Eq. (26)-(31)): Zou-He density
// from the known c_x <= 0 populations, second-order equilibrium at u_in, and
// the non-equilibrium part rebuilt from Pi_neq with the unknown c_x > 0
// non-equilibrium populations taken equal to their opposites.  Returns the
// inlet density.
__device__ __forceinline__ float inlet_regularize(const CollideArgs& a, int y, int z, float f[Q]) {
  const int pl = a.ny * a.nz, o = y * a.nz + z;
  const float ux = a.u_in[o], uy = a.u_in[pl + o], uz = a.u_in[2 * pl + o];
  float rho0 = 0.f, rhom = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (CX[i] == 0) rho0 += f[i];
    if (CX[i] == -1) rhom += f[i];
  }
  const float rin = (rho0 + 2.f * rhom) / (1.f - ux);
  const float uu15 = 1.5f * (ux * ux + uy * uy + uz * uz);
  float feq[Q];
  float pxx = 0.f, pyy = 0.f, pzz = 0.f, pxy = 0.f, pyz = 0.f, pxz = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
    feq[i] = (float)WD[i] * rin * (1.f + 3.f * cu + 4.5f * cu * cu - uu15);
    if (CX[i] <= 0) {
      const float fn = (CX[i] == 0 ? 1.f : 2.f) * (f[i] - feq[i]);
      pxx += (CX[i] * CX[i] - 1.f / 3.f) * fn;
      pyy += (CY[i] * CY[i] - 1.f / 3.f) * fn;
      pzz += (CZ[i] * CZ[i] - 1.f / 3.f) * fn;
      pxy += (CX[i] * CY[i]) * fn;
      pyz += (CY[i] * CZ[i]) * fn;
      pxz += (CX[i] * CZ[i]) * fn;
    }
  }
  const float tr3 = (pxx + pyy + pzz) * (1.f / 3.f);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float cpc = CX[i] * CX[i] * pxx + CY[i] * CY[i] * pyy + CZ[i] * CZ[i] * pzz +
                      2.f * (CX[i] * CY[i] * pxy + CY[i] * CZ[i] * pyz + CX[i] * CZ[i] * pxz);
    f[i] = feq[i] + 4.5f * (float)WD[i] * (cpc - tr3);
  }
  return rin;
}

}  // namespace lbm
