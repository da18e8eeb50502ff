// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/lbm.h"
#include "lattice.h"

namespace lbm {

// Bits of the device error word.
constexpr int ERRBIT_MACH = 1;
constexpr int ERRBIT_NONFINITE = 2;
constexpr int ERRBIT_STG_TABLE = 4;  // invalid STG inputs: R not positive definite, per-row spectrum (kmag order, k, omega)

constexpr int ZT = 64;     // z-lanes per wave (one wave = one (x, y) row segment)
constexpr int YROWS = 4;   // rows (waves) per collide block
constexpr int BLOCK = ZT * YROWS;
constexpr int STG_BATCH = 32;  // steps whose inlet planes one STG launch computes
constexpr int64_t FUSED_MAX_NODES = int64_t(1) << 24;  // FP16: one fused collide launch up to this size
// FP32 storage: each step's general-kernel blocks go out as one dispatch per
// range of x-planes holding about this many blocks (whole planes; a lattice of
// up to 1.5x this many blocks is one dispatch).  On lattices of tens of
// millions of nodes this holds the pull at about 0.75 of HBM peak where one
// dispatch over all blocks reaches 0.69-0.70; the FP16 bulk kernel gains
// nothing from it and keeps one dispatch.
constexpr int CHUNK_BLOCKS = 30000;
// FP32 state buffers together larger than this: non-temporal population
// stores (the 256 MB Infinity Cache cannot hold the state from one step to
// the next).
constexpr int64_t NT_STORE_MIN_BYTES = int64_t(192) << 20;
// Static device scratch of stg_inlet_fill_noalloc (per device, for the process
// lifetime): the STG tables of one call must fit.
constexpr size_t NOALLOC_STG_BYTES = size_t(4) << 20;
// Largest ny the adjoint supports (its bin reduction stages rows in LDS).
#define LBM_ADJ_MAX_NY 4096

// Arguments of the fused collide-stream kernel (passed by value).
struct CollideArgs {
  const void* src;  // state s_n (64-node bricks, see collide.hip)
  void* dst;        // state s_{n+1}
  const float* hist_in;   // [5][ny][nz]
  float* hist_out;        // [5][ny][nz]
  const float* u_in;      // [3][ny][nz]
  double* stats;          // [n_planes][ny][zc][9]
  double* wall_acc;       // [2][nx][zc] sums of u_tau in the first off-wall rows, or null
  const float* wall_line; // [2][nx] signed u_tau of each wall line (line-averaged model), or null
  const float* dref;      // [ny][19] FP16 storage reference offsets r_i(y), or null (r = 0)
  const float* dpull;     // [ny][19] r of the value a plain (wall-free) pull of direction i reads into row y
  const int* plane_of_x;  // [nx], -1 when not sampled
  int* err;
  int nx, ny, nz, zc, yg, nblocks;
  int nt_store;           // 1: non-temporal population stores (all but small FP32 lattices)
  int ywall, xbc, wall_model, newton_iters, stats_on, has_g, wall_law;
  float tau0, tau0sq, smag;  // smag = 18 sqrt(2) C_s^2
  float g[3];
  float nu0, inv_nu0, y_wall, kappa, inv_kappa, b_reich;
  float out_wh, out_wu;  // outlet rule f_i = out_wh f_i^prev + out_wu f_i(x-1) for c_x < 0
  int sponge_x0;                 // first sponge plane (nx: no sponge)
  float sponge_inv_len, sponge_dnu;  // 1 / sponge_cells, sponge_nu - nu0
  float rs[Q], rf[Q];  // s_k / D_k and (1 - s_k/2) / D_k for the fixed-rate moments
};

// Arguments of the adjoint kernels (passed by value).  c holds the forward
// arguments with src = s_n, hist_in = its outlet history and u_in = the inlet
// plane at t_{n+1}; dst, hist_out and stats are unused.
struct AdjointArgs {
  CollideArgs c;
  const float* lam_next;  // dL/ds_{n+1}, float bricks
  float* lam_prev;        // dL/ds_n, float bricks
  const float* eta_next;  // dL/dhist_{n+1} [5][ny][nz]
  float* eta_prev;        // dL/dhist_n [5][ny][nz]
  const float* coef;      // [n_planes][ny][9] statistics weights, or null
  float* g_uin;           // dL/du_in [3][ny][nz]
  const float* fluct;     // a v' of the inlet plane [3][ny][nz]
  double* cs_part;        // [blocks] per-block dL/dC_s
  double* amp_part;       // [ny][zc] per inlet-row-chunk sum of g_uin . fluct
  double* line_part;      // [2][nx][zc] per wall-line chunk dL/d(line u_tau) (line-averaged model)
  float dsmag;            // d(18 sqrt(2) C_s^2)/dC_s
};

// Per-step destinations of a batch of inlet planes (u_in and a v' of step j
// of the batch), passed by value; u[0] == nullptr: not used.
struct PlaneDst {
  float* u[STG_BATCH];
  float* f[STG_BATCH];
};

struct StgTables {
  int n_modes = 0;
  int cap_trigz = 0, cap_amp3 = 0, cap_ky = 0, cap_chol = 0, cap_sb = 0, cap_urans = 0, cap_rowamp = 0;
  float* amp3 = nullptr;    // [3][N] sqrt(6 q) sigma; sigma alone with the per-row spectrum
  float* rowamp_buf = nullptr;    // [ny][N] allocation behind rowamp
  const float* rowamp = nullptr;  // [ny][N] sqrt(6 q^n(y)) with the per-row spectrum, else null
  double* ky = nullptr;     // [N] kmag d_y
  float2* trigz = nullptr;  // [N][nz] (cos, sin)(kmag d_z z mod 2 pi)
  float* chol = nullptr;    // [6][ny]
  float* sb = nullptr;      // [ny] amplitude scaling of each row
  float* urans = nullptr;   // [3][ny]
};

}  // namespace lbm

struct lbm_ctx {
  lbm_config cfg{};
  hipStream_t stream = nullptr;  // caller's stream: every call's work is ordered on it
  int device = 0;
  void* f[2] = {nullptr, nullptr};
  float* hist[2] = {nullptr, nullptr};
  int cur = 0;
  int64_t time = 0;
  int64_t N = 0;
  int zc = 0, yg = 0, nblocks = 0;
  int* d_err = nullptr;
  int* d_plane_of_x = nullptr;
  int* d_blist_int = nullptr;  // bulk / boundary collide block lists
  int* d_blist_bnd = nullptr;
  int n_int = 0, n_bnd = 0, cap_int = 0, cap_bnd = 0;
  // Offsets of the x-chunks of d_blist_bnd (chunks + 1 entries; one chunk
  // except with FP32 storage on large lattices), and the x-planes per chunk.
  std::vector<int> bnd_off;
  int chunk_planes = 0;
  int64_t int_nodes = 0;  // nodes updated by one bulk launch
  // FP16 storage: boundary blocks in the general kernel, then the bulk blocks
  // in a lean kernel; on lattices up to FUSED_MAX_NODES both in one fused
  // launch.  FP32 storage is HBM-bound with the general kernel alone: one
  // launch over all blocks.
  bool split = false;
  bool fused = false;
  double* d_stats = nullptr;
  double* d_wall_acc = nullptr;  // [2][nx][zc], with the wall model
  float* d_wall_line = nullptr;  // [2][nx] line-averaged u_tau of the current step
  double* d_line_part = nullptr; // [2][nx][zc] adjoint partial sums of the line model
  float* d_dref = nullptr;       // [ny][19] FP16 storage reference offsets (null: none)
  float* d_dpull = nullptr;      // [ny][19] the same, of the plain pulls' source rows
  int n_planes = 0;
  std::vector<int> plane_of_x;  // host copy of d_plane_of_x
  int stats_on = 0;
  int64_t n_samples = 0;
  bool stg_bound = false;
  lbm_stg stg{};
  lbm::StgTables tab;
  // adjoint scratch (allocated on the first adjoint step)
  double* d_cs_part = nullptr;  // [nblocks] dL/dC_s per block, accumulated over adjoint steps
  double* d_amp_part = nullptr; // [ny][zc] dL/ds_b partials per inlet row chunk, accumulated
  float* d_fluct = nullptr;     // [3][ny][nz], when the bound STG inputs have no fluct buffer
  float* d_guin = nullptr;      // [3][ny][nz], when the caller passes no g_uin
  float* d_uin_ring = nullptr;  // [STG_BATCH][3][ny][nz] inlet planes of the steps of one batch
  float* d_fl_ring = nullptr;   // the same for a v', when the bound STG inputs keep it
  int* d_ablist = nullptr;      // [n_ablist] adjoint block entries in dispatch order (-1 pads)
  int n_ablist = 0;
  int timing = 0;
  std::vector<hipEvent_t> ev;  // pairs (start, stop) of timed launches
  int64_t ev_used = 0;
  double timed_ms = 0.0;
  int64_t timed_launches = 0;
};

namespace lbm {
// collide.hip
// u_in, when given, replaces the bound inlet plane.
hipError_t launch_boundary(lbm_ctx* h, int src, int dst, hipStream_t stream, const float* u_in = nullptr);
hipError_t launch_bulk(lbm_ctx* h, int src, int dst, hipStream_t stream, const float* u_in = nullptr);
hipError_t build_block_lists(lbm_ctx* h, const std::vector<int>& plane_of_x);
hipError_t launch_stream_only(lbm_ctx* h, int src, int dst);
hipError_t launch_init(lbm_ctx* h, const float* rho, const float* u, const float* pert, float eps);
hipError_t launch_init(lbm_ctx* h, const double* rho, const double* u, const double* pert, double eps);
hipError_t launch_export(lbm_ctx* h, float* out);
hipError_t launch_import(lbm_ctx* h, const float* in);
hipError_t launch_set_reference(lbm_ctx* h, const double* u_ref);
hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t s);
void fill_args(lbm_ctx* h, CollideArgs& a, int src, int dst);
hipError_t launch_wall_line(lbm_ctx* h, CollideArgs& a, hipStream_t stream);
// Entries of columns (x, y-group) of zc z-chunks each, in column order, dealt
// to the 8 XCDs column by column; -1 pads the result.
std::vector<int> xcd_order(const std::vector<int>& entries, int zc, const std::vector<char>* heavy = nullptr);
hipError_t launch_field_export(lbm_ctx* h, const float* bricks, float* soa);
hipError_t launch_field_import(lbm_ctx* h, const float* soa, float* bricks);
// adjoint.hip
hipError_t launch_adjoint(lbm_ctx* h, const AdjointArgs& args, int storage_f16, double t_next, bool fill_inlet,
                          float* u_in, float* fluct);
hipError_t launch_step_explicit(lbm_ctx* h, const void* src, void* dst, const float* hist_in, float* hist_out,
                                const float* u_in, hipStream_t stream);
hipError_t launch_adjoint_reduce(lbm_ctx* h, double* grad);
// stg.hip
hipError_t launch_stg_bind(lbm_ctx* h, const lbm_stg* s);
hipError_t launch_stg_fill(lbm_ctx* h, double t, hipStream_t stream, float* fluct = nullptr, float* u_in = nullptr);
hipError_t launch_stg_fill_batch(lbm_ctx* h, double time0, int nb, hipStream_t stream, float* ring, float* fring,
                                 int last_j);
hipError_t launch_stg_fill_to(lbm_ctx* h, double time0, int nb, hipStream_t stream, const PlaneDst& dst);
hipError_t launch_inflow_reichardt(lbm_ctx* h, double u_tau, double* u_rans);
// The static scratch of stg_inlet_fill_noalloc: per-device address lookup (once per
// device, that device current), the bytes a binding needs, the fill itself.
hipError_t noalloc_scratch_setup(int device);
size_t noalloc_stg_bytes(const lbm_ctx* h, const lbm_stg* s);
hipError_t launch_stg_fill_noalloc(lbm_ctx* h, const lbm_stg* s, double time);
}  // namespace lbm
