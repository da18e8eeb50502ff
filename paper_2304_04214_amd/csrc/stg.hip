// Synthetic turbulence generator for the inlet plane (Sec. III.A,
// Eq. (22)-(25); Algorithm 1 steps 3-5) and the Reichardt mean inflow.
//
// Binding precomputes the time-independent tables: mode amplitudes
// sqrt(6 q) sigma, the spanwise phase factors (cos, sin)(k d_z z) reduced in
// FP64, the Cholesky factors a(y) of R(y) and the per-row scalings s_b.
// Filling evaluates, per step, the (y, t)-dependent phase
// k d_y (y + 1/2) + omega t + phi in FP64 (reduced mod 2 pi), and combines it
// with the spanwise factor by angle addition, so the FP32 cosines never see a
// large argument.  The mode sum itself is FP32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "internal.h"

// Scratch of the allocation-free inlet fill (stg_inlet_fill_noalloc): the STG
// tables of one call (the inputs' binding, as the handle's tables hold it for
// stg_inlet_fill).  One copy per device, held until the process ends; every
// call on a device uses that device's copy.  Host code never uses this name
// as an address: lbm::noalloc_scratch_setup looks up each device's address.
static __device__ __align__(256) unsigned char scratch[lbm::NOALLOC_STG_BYTES];

namespace lbm {
namespace {

constexpr double TWO_PI = 6.283185307179586476925286766559;
constexpr float MACH_LIMIT = 0.17320508075688773f;  // 0.3 c_s, c_s = 1/sqrt(3)

__global__ void stg_bind_kernel(lbm_stg s, StgTables t, int ny, int nz, int* err) {
  const bool rows = s.k_rans != nullptr;  // per-row spectrum: sqrt(6 q^n(y)) lives in rowamp
  const int N = s.n_modes;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nzN = (int64_t)N * nz;
  if (k < nzN) {
    const int n = (int)(k / nz), z = (int)(k % nz);
    const double ph = fmod(s.kmag[n] * s.d[2 * N + n] * (double)z, TWO_PI);
    double sn, cs;
    sincos(ph, &sn, &cs);
    t.trigz[k] = make_float2((float)cs, (float)sn);
    return;
  }
  const int64_t k2 = k - nzN;
  if (k2 < N) {
    const int n = (int)k2;
    const double a = rows ? 1.0 : sqrt(6.0 * s.q[n]);  // Eq. (25): sqrt(6) sqrt(q^n)
    for (int c = 0; c < 3; ++c) t.amp3[c * N + n] = (float)(a * s.sigma[c * N + n]);
    t.ky[n] = s.kmag[n] * s.d[N + n];
    return;
  }
  const int64_t k3 = k2 - N;
  if (k3 < ny) {
    const int y = (int)k3;
    // Eq. (24): lower Cholesky factor of R (FP64), a11 a21 a22 a31 a32 a33.
    // A row whose R is not symmetric positive definite (a pivot R11,
    // R22 - a21^2 or R33 - a31^2 - a32^2 not positive, or a non-finite entry)
    // is reported (LBM_ERR_ARG at the next lbm_sync) and gets a zero factor.
    const double R11 = s.R[y], R21 = s.R[ny + y], R22 = s.R[2 * ny + y];
    const double R31 = s.R[3 * ny + y], R32 = s.R[4 * ny + y], R33 = s.R[5 * ny + y];
    double a11 = 0.0, a21 = 0.0, a22 = 0.0, a31 = 0.0, a32 = 0.0, a33 = 0.0;
    bool ok = R11 > 0.0 && isfinite(R11) && isfinite(R21) && isfinite(R22) && isfinite(R31) && isfinite(R32) &&
              isfinite(R33);
    if (ok) {
      a11 = sqrt(R11);
      a21 = R21 / a11;
      a31 = R31 / a11;
      const double p22 = R22 - a21 * a21;
      ok = p22 > 0.0;
      if (ok) {
        a22 = sqrt(p22);
        a32 = (R32 - a21 * a31) / a22;
        const double p33 = R33 - a31 * a31 - a32 * a32;
        ok = p33 > 0.0;
        if (ok) a33 = sqrt(p33);
      }
    }
    if (!ok) {
      a11 = a21 = a22 = a31 = a32 = a33 = 0.0;
      atomicOr(err, ERRBIT_STG_TABLE);
    }
    t.chol[y] = (float)a11;
    t.chol[ny + y] = (float)a21;
    t.chol[2 * ny + y] = (float)a22;
    t.chol[3 * ny + y] = (float)a31;
    t.chol[4 * ny + y] = (float)a32;
    t.chol[5 * ny + y] = (float)a33;
    int b = s.bin_of_y[y];
    b = b < 0 ? 0 : (b >= s.n_bins ? s.n_bins - 1 : b);  // out-of-range bins are clamped
    t.sb[y] = (float)s.amp_bin[b];
    for (int c = 0; c < 3; ++c) t.urans[c * ny + y] = (float)s.u_rans[c * ny + y];
  }
}

// Per-row weights of the modified von Karman spectrum (Sec. III.A, Eq. (25),
// the spectrum of the cited STG) from the row's RANS k, omega and wall
// distance: one block per inlet row; FP64 throughout, the row sum reduced in
// a fixed order; rowamp[y][n] = sqrt(6 q^n(y)).
__device__ double spectrum_weight(const lbm_stg& s, int n, double ke, double keta, double kcut) {
  const int N = s.n_modes;
  double dk = 1.0;
  if (N > 1) {
    const int lo = n > 0 ? n - 1 : 0, hi = n < N - 1 ? n + 1 : N - 1;
    dk = (s.kmag[hi] - s.kmag[lo]) / (hi - lo);
  }
  const double k = s.kmag[n], r = k / ke;
  const double r2 = r * r;
  const double a = 12.0 * k / keta, c = 4.0 * fmax(k - 0.9 * kcut, 0.0) / kcut;
  return r2 * r2 * pow(1.0 + 2.4 * r2, -17.0 / 6.0) * exp(-a * a - c * c * c) * dk;
}

__global__ __launch_bounds__(256) void stg_spectrum_kernel(lbm_stg s, float* rowamp, int ny, double nu, int* err) {
  __shared__ double red[256];
  const int y = blockIdx.x, N = s.n_modes;
  const double CMU = 0.09, CL = 3.0;
  const double k = s.k_rans[y], om = s.omega_rans[y];
  bool bad = !(k > 0.0) || !(om > 0.0) || !isfinite(k) || !isfinite(om);
  const double dw = fmin(y + 0.5, ny - y - 0.5);
  const double le = fmin(2.0 * dw, CL * sqrt(k) / (CMU * om));  // energy-containing eddy length
  const double eta = sqrt(sqrt(nu * nu * nu / (CMU * k * om)));  // Kolmogorov length
  const double ke = TWO_PI / le, keta = TWO_PI / eta, kcut = TWO_PI / 2.0;  // l_cut = 2 cells
  double part = 0.0;
  for (int n = threadIdx.x; n < N; n += 256) {
    if (n > 0 && !(s.kmag[n] > s.kmag[n - 1])) bad = true;
    part += spectrum_weight(s, n, ke, keta, kcut);
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double sum = red[0];
  if (!(sum > 0.0)) bad = true;
  for (int n = threadIdx.x; n < N; n += 256)
    rowamp[(int64_t)y * N + n] = (float)sqrt(6.0 * spectrum_weight(s, n, ke, keta, kcut) / sum);
  if (bad) atomicOr(err, ERRBIT_STG_TABLE);
}

// One block per (inlet row y, 64 spanwise nodes, step); its four waves each
// sum a quarter of the modes, and the partial sums are added in a fixed order.
// Step j = blockIdx.z has time time0 + j.  With ring ==
// nullptr the plane goes to s.u_in / s.fluct; otherwise to plane j of ring /
// fring, and the plane of step last_j also to s.u_in / s.fluct.
__global__ __launch_bounds__(256) void stg_fill_kernel(lbm_stg s, StgTables t, int ny, int nz, double time0,
                                                       int* err, float* ring, float* fring, int last_j,
                                                       PlaneDst dst) {
  __shared__ float2 rowph[LBM_MAX_MODES];
  __shared__ float amp[3][LBM_MAX_MODES];
  __shared__ float part[3][3][64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int y = blockIdx.y;
  const int zr = blockIdx.x * 64 + lane;
  const int z = zr < nz ? zr : nz - 1;
  const int N = s.n_modes;
  const int j = blockIdx.z;
  const double time = time0 + j;
  // (y, t)-dependent phase of every mode, FP64 then reduced to [0, 2 pi)
  for (int n = threadIdx.x; n < N; n += 256) {
    const double ph = fmod(t.ky[n] * (y + 0.5) + s.omega[n] * time + s.phi[n], TWO_PI);
    double sn, cs;
    sincos(ph, &sn, &cs);
    rowph[n] = make_float2((float)cs, (float)sn);
    const float r = t.rowamp ? t.rowamp[(int64_t)y * N + n] : 1.f;
    amp[0][n] = t.amp3[n] * r;
    amp[1][n] = t.amp3[N + n] * r;
    amp[2][n] = t.amp3[2 * N + n] * r;
  }
  __syncthreads();
  float v0 = 0.f, v1 = 0.f, v2 = 0.f;
  const float2* tz = t.trigz + z;
  // wave w sums the contiguous mode range [n0, n1)
  const int n0 = (N * w) >> 2, n1 = (N * (w + 1)) >> 2;
#pragma unroll 8
  for (int n = n0; n < n1; ++n) {
    const float2 a = rowph[n];
    const float2 b = tz[(int64_t)n * nz];
    const float c = a.x * b.x - a.y * b.y;  // cos(alpha + beta)
    v0 += amp[0][n] * c;
    v1 += amp[1][n] * c;
    v2 += amp[2][n] * c;
  }
  if (w > 0) {
    part[w - 1][0][lane] = v0;
    part[w - 1][1][lane] = v1;
    part[w - 1][2][lane] = v2;
  }
  __syncthreads();
  if (w != 0 || zr >= nz) return;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v0 += part[k][0][lane];
    v1 += part[k][1][lane];
    v2 += part[k][2][lane];
  }
  // Eq. (23): u' = a v' with the lower-triangular Cholesky factor; Eq. (22)
  const float a11 = t.chol[y], a21 = t.chol[ny + y], a22 = t.chol[2 * ny + y];
  const float a31 = t.chol[3 * ny + y], a32 = t.chol[4 * ny + y], a33 = t.chol[5 * ny + y];
  const float p0 = a11 * v0;
  const float p1 = a21 * v0 + a22 * v1;
  const float p2 = a31 * v0 + a32 * v1 + a33 * v2;
  const float sb = t.sb[y];
  const int o = y * nz + z, pl = ny * nz;
  const float ux = t.urans[y] + sb * p0;
  const float uy = t.urans[ny + y] + sb * p1;
  const float uz = t.urans[2 * ny + y] + sb * p2;
  float* u = nullptr;
  float* f = nullptr;
  if (dst.u[0]) {  // per-step destinations (block-uniform)
    u = dst.u[j];
    f = dst.f[j];
  } else if (ring) {
    u = ring + (size_t)j * 3 * pl;
    f = fring ? fring + (size_t)j * 3 * pl : nullptr;
  }
  const bool bound = u == nullptr || j == last_j;
  if (u) {
    u[o] = ux;
    u[pl + o] = uy;
    u[2 * pl + o] = uz;
    if (f) {
      f[o] = p0;
      f[pl + o] = p1;
      f[2 * pl + o] = p2;
    }
  }
  if (bound) {
    s.u_in[o] = ux;
    s.u_in[pl + o] = uy;
    s.u_in[2 * pl + o] = uz;
    if (s.fluct) {
      s.fluct[o] = p0;
      s.fluct[pl + o] = p1;
      s.fluct[2 * pl + o] = p2;
    }
  }
  if (!(fabsf(ux) < MACH_LIMIT)) atomicOr(err, ERRBIT_MACH);
}

// Reichardt law with the constants of the configuration (Sec. II.C, Eq. (16)).
__global__ void inflow_reichardt_kernel(double* u, int ny, double u_tau, double nu0, double kappa, double B) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= ny) return;
  const double d = fmin(y + 0.5, ny - y - 0.5);
  const double yp = d * u_tau / nu0;
  const double up = log1p(kappa * yp) / kappa - B * (expm1(-yp / 11.0) + (yp / 11.0) * exp(-yp / 3.0));
  u[y] = u_tau * up;
  u[ny + y] = 0.0;
  u[2 * ny + y] = 0.0;
}

template <class T>
hipError_t grow(T** p, int* cap, int need) {
  if (*p && *cap >= need) return hipSuccess;
  if (*p) {
    hipError_t e = hipFree(*p);
    if (e != hipSuccess) return e;
    *p = nullptr;
  }
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)need);
  if (e == hipSuccess) *cap = need;
  return e;
}

}  // namespace

hipError_t launch_stg_bind(lbm_ctx* h, const lbm_stg* s) {
  const int N = s->n_modes, ny = h->cfg.ny, nz = h->cfg.nz;
  StgTables& t = h->tab;
  hipError_t e;
  if ((e = grow(&t.trigz, &t.cap_trigz, N * nz)) != hipSuccess) return e;
  if ((e = grow(&t.amp3, &t.cap_amp3, 3 * N)) != hipSuccess) return e;
  if ((e = grow(&t.ky, &t.cap_ky, N)) != hipSuccess) return e;
  if ((e = grow(&t.chol, &t.cap_chol, 6 * ny)) != hipSuccess) return e;
  if ((e = grow(&t.sb, &t.cap_sb, ny)) != hipSuccess) return e;
  if ((e = grow(&t.urans, &t.cap_urans, 3 * ny)) != hipSuccess) return e;
  t.n_modes = N;
  const int64_t total = (int64_t)N * nz + N + ny;
  const int nb = (int)((total + 255) / 256);
  t.rowamp = nullptr;
  stg_bind_kernel<<<nb, 256, 0, h->stream>>>(*s, t, ny, nz, h->d_err);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (s->k_rans) {
    if ((e = grow(&t.rowamp_buf, &t.cap_rowamp, ny * N)) != hipSuccess) return e;
    t.rowamp = t.rowamp_buf;
    stg_spectrum_kernel<<<ny, 256, 0, h->stream>>>(*s, t.rowamp_buf, ny, (h->cfg.tau0 - 0.5) / 3.0, h->d_err);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// fluct and u_in, when given, replace the bound outputs (the fluctuation a v'
// and the inlet velocity plane).
hipError_t launch_stg_fill(lbm_ctx* h, double time, hipStream_t stream, float* fluct, float* u_in) {
  const int ny = h->cfg.ny, nz = h->cfg.nz;
  dim3 grid((nz + 63) / 64, ny);
  lbm_stg s = h->stg;
  if (fluct) s.fluct = fluct;
  if (u_in) s.u_in = u_in;
  stg_fill_kernel<<<grid, 256, 0, stream>>>(s, h->tab, ny, nz, time, h->d_err, nullptr, nullptr, -1, PlaneDst{});
  return hipGetLastError();
}

// The inlet planes of nb consecutive steps (times time0 .. time0 + nb - 1) in
// one launch, into plane j of ring (and fring); the plane of step last_j
// (-1: none) also goes to the bound u_in / fluct.
hipError_t launch_stg_fill_batch(lbm_ctx* h, double time0, int nb, hipStream_t stream, float* ring, float* fring,
                                 int last_j) {
  const int ny = h->cfg.ny, nz = h->cfg.nz;
  dim3 grid((nz + 63) / 64, ny, nb);
  stg_fill_kernel<<<grid, 256, 0, stream>>>(h->stg, h->tab, ny, nz, time0, h->d_err, ring, fring, last_j,
                                            PlaneDst{});
  return hipGetLastError();
}

// The inlet planes of nb <= STG_BATCH consecutive steps (times time0 ..
// time0 + nb - 1) in one launch, plane j to dst.u[j] and a v' to dst.f[j]
// (both non-null for j < nb); the bound outputs are not written.
hipError_t launch_stg_fill_to(lbm_ctx* h, double time0, int nb, hipStream_t stream, const PlaneDst& dst) {
  const int ny = h->cfg.ny, nz = h->cfg.nz;
  dim3 grid((nz + 63) / 64, ny, nb);
  stg_fill_kernel<<<grid, 256, 0, stream>>>(h->stg, h->tab, ny, nz, time0, h->d_err, nullptr, nullptr, -1, dst);
  return hipGetLastError();
}

namespace {

// Device address of `scratch` per device, looked up once (lbm_create, with the
// device current).
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch[MAX_DEVICES] = {};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Byte offsets of the tables in the scratch (each 256-byte aligned) and their
// total: trigz [N][nz] float2, amp3 [3][N] float, ky [N] double, chol [6][ny],
// sb [ny], urans [3][ny] float, rowamp [ny][N] float with the per-row spectrum.
struct NoallocLayout {
  size_t trigz, amp3, ky, chol, sb, urans, rowamp, total;
};
NoallocLayout noalloc_layout(int n_modes, int ny, int nz, bool rows) {
  NoallocLayout L;
  size_t o = 0;
  L.trigz = o;
  o += align256(sizeof(float2) * (size_t)n_modes * nz);
  L.amp3 = o;
  o += align256(sizeof(float) * 3 * (size_t)n_modes);
  L.ky = o;
  o += align256(sizeof(double) * (size_t)n_modes);
  L.chol = o;
  o += align256(sizeof(float) * 6 * (size_t)ny);
  L.sb = o;
  o += align256(sizeof(float) * (size_t)ny);
  L.urans = o;
  o += align256(sizeof(float) * 3 * (size_t)ny);
  L.rowamp = o;
  if (rows) o += align256(sizeof(float) * (size_t)ny * n_modes);
  L.total = o;
  return L;
}

}  // namespace

hipError_t noalloc_scratch_setup(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch[device] = p;
  return hipSuccess;
}

size_t noalloc_stg_bytes(const lbm_ctx* h, const lbm_stg* s) {
  return noalloc_layout(s->n_modes, h->cfg.ny, h->cfg.nz, s->k_rans != nullptr).total;
}

// stg_inlet_fill with the inputs bound into the device's scratch instead of the
// handle's tables: the same bind, spectrum and fill kernels, no allocation.
// The caller has checked noalloc_stg_bytes <= NOALLOC_STG_BYTES.
hipError_t launch_stg_fill_noalloc(lbm_ctx* h, const lbm_stg* s, double time) {
  if (h->device < 0 || h->device >= MAX_DEVICES) return hipErrorInvalidDevice;
  char* base;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = static_cast<char*>(g_scratch[h->device]);
  }
  if (!base) return hipErrorInvalidSymbol;
  const int N = s->n_modes, ny = h->cfg.ny, nz = h->cfg.nz;
  const bool rows = s->k_rans != nullptr;
  const NoallocLayout L = noalloc_layout(N, ny, nz, rows);
  if (L.total > NOALLOC_STG_BYTES) return hipErrorInvalidValue;
  StgTables t;
  t.n_modes = N;
  t.trigz = reinterpret_cast<float2*>(base + L.trigz);
  t.amp3 = reinterpret_cast<float*>(base + L.amp3);
  t.ky = reinterpret_cast<double*>(base + L.ky);
  t.chol = reinterpret_cast<float*>(base + L.chol);
  t.sb = reinterpret_cast<float*>(base + L.sb);
  t.urans = reinterpret_cast<float*>(base + L.urans);
  t.rowamp = nullptr;
  const int64_t total = (int64_t)N * nz + N + ny;
  stg_bind_kernel<<<(int)((total + 255) / 256), 256, 0, h->stream>>>(*s, t, ny, nz, h->d_err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (rows) {
    float* rowamp = reinterpret_cast<float*>(base + L.rowamp);
    stg_spectrum_kernel<<<ny, 256, 0, h->stream>>>(*s, rowamp, ny, (h->cfg.tau0 - 0.5) / 3.0, h->d_err);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    t.rowamp = rowamp;
  }
  dim3 grid((nz + 63) / 64, ny);
  stg_fill_kernel<<<grid, 256, 0, h->stream>>>(*s, t, ny, nz, time, h->d_err, nullptr, nullptr, -1, PlaneDst{});
  return hipGetLastError();
}

hipError_t launch_inflow_reichardt(lbm_ctx* h, double u_tau, double* u_rans) {
  const int ny = h->cfg.ny;
  const double nu0 = (h->cfg.tau0 - 0.5) / 3.0;
  inflow_reichardt_kernel<<<(ny + 63) / 64, 64, 0, h->stream>>>(u_rans, ny, u_tau, nu0, h->cfg.kappa,
                                                                 h->cfg.b_reich);
  return hipGetLastError();
}

}  // namespace lbm
