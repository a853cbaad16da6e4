// Internal declarations shared by the host plan (pb3_host.cpp) and the
// kernel launchers (pb3_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pb3.h"

namespace pb3 {

constexpr int kReduceSlices = 32;
constexpr int kWindowBlocks = 256;  // PB3_WINDOW_SCRATCH = 2 + 2 * kWindowBlocks doubles

// Stage indices for the optional per-kernel timing.
enum Stage {
  ST_FWD_Z = 0,
  ST_FWD_Y,
  ST_FWD_X,
  ST_POWER,
  ST_INV_X,
  ST_INV_Y,
  ST_INV_Z,
  ST_CONTRACT,
  ST_REDUCE,
  ST_COUNT
};

// One work tile of the per-bin inverse passes: bin b, first column.
struct BinTile {
  int32_t bin;
  int32_t col0;
};

// Geometry of bin b's pruned spectrum: kx in [-knegx, kposx], ky in
// [-knegy, kposy], kz in [0, kzn) (the positive side one shorter than the
// negative where it reaches the Nyquist index).
struct BinGeom {
  int32_t knegx, kposx;  // x extent
  int32_t knegy, kposy;  // y extent
  int32_t ly;            // knegy + kposy + 1
  int32_t kzn;           // number of kz planes
  int32_t n2lo, n2hi;    // cubic box: the bin's modes are n2lo <= |n|^2 < n2hi (n2lo < 0: use the per-mode table)
  int64_t a1_off;        // float2 offset of this bin's x-pass output  [Mx][ly][kzn]
  int64_t a2_off;        // float2 offset of this bin's y-pass output  [Mx][My][kzn]
};

// A device tile table for one inverse pass and the tile width it was built for.
struct TileSet {
  BinTile* d;
  int n;
  int tb;
};

// Jobs of one plan launched together (grid z = job index, at most kMaxJobs):
// their inputs and outputs by value, and the byte stride between their
// workspaces.  A single call is one job with stride 0.
constexpr int kMaxJobs = 8;
struct JobIO {
  const float* delta[kMaxJobs];
  double* pk[kMaxJobs];
  double* bk[kMaxJobs];
  const float* window;  // optional (single job): the forward pass transforms window * delta
};

struct DeviceTables {
  int8_t* bin3 = nullptr;         // bin of every compact mode [Lcx][Lcy][Kz] (int8, -1 outside), then one -1
  int32_t* modes = nullptr;       // compact D index of every binned half-spectrum mode (bit 31: weight 1)
  int32_t* chunk = nullptr;       // power chunks: (bin, start, end) triples
  int32_t* chunk_first = nullptr; // per bin: index of its first chunk (n_bins + 1 entries)
  int32_t* xtile_first = nullptr; // per bin: index of its first inverse-x tile (n_bins + 1 entries)
  BinGeom* geom = nullptr;        // per bin
  BinTile* tiles = nullptr;       // all FP32 inverse-pass tiles (x, then y, then z)
  int32_t* trip_all = nullptr;    // candidate triplets (3 ints each), simple contraction
  int32_t* out_map = nullptr;     // per kept triplet: index into one work-group's MFMA partial vector
  int32_t* out_map_ab = nullptr;  // the same for pairs against separate column fields (multipoles)
  int32_t* out_inv = nullptr;     // per element of a partial vector: the kept triplet read there, or -1
  double* inv_counts = nullptr;   // per kept triplet: scale / T
  double* pk_scale = nullptr;     // per bin: V / (N_pix^2 N_b)
  float2* tw_n[3] = {};           // W_{N_i}^j, j < N_i, per axis x, y, z
  float2* tw_m[3] = {};           // W_{M_i}^j
  double2* tw_m_d[3] = {};        // FP64 twiddles for the count pass
  double* nmodes_d = nullptr;      // masked power: N_b as double (made on first use)
  double* pml_inv = nullptr;       // multipoles: per bin, inverse discrete Fisher x V / N_pix^2 [nb][n_ell^2]
  int32_t* ml_trips = nullptr;     // multipoles: (a, b, l nb + c) per l and kept triplet
  double* ml_fac = nullptr;        // multipoles: (2l + 1) V^2 M^6 / (N^9 T) per l and kept triplet
  int32_t* ml_map = nullptr;       // multipoles: identity map over kept triplets
  // weighted estimator (pb3_plan_set_weights); all null when unweighted
  float* win_inv = nullptr;        // 1 / sinc(pi k / N_i)^p, k in [-N_i/2, N_i/2], axes x, y, z back to back
  float* pfid_inv = nullptr;       // 1 / P_fid over integer |n|^2 (lut_len entries)
  double* pfid_inv_d = nullptr;    // same in FP64 (weighted triangle counts)
  double* mode_w = nullptr;        // per power mode: 1 / (m^2 P_fid^2)
  double* bk_bias = nullptr;       // per kept triplet: shot-noise bispectrum
  double* bk_mix = nullptr;        // bispectrum multipole Fisher: per kept triplet [n_ell][n_ell] (else null)
};

struct Workspace {
  void* base = nullptr;
  size_t bytes = 0;
  bool owned = false;
  float2* f1 = nullptr;     // [Nx][Ny][Kz]
  float2* f2 = nullptr;     // [Nx][Lcy][Kz]
  float2* dc = nullptr;     // [Lcx][Lcy][Kz]
  float2* a1 = nullptr;     // per-bin x-pass outputs
  float2* a2 = nullptr;     // per-bin y-pass outputs
  float* g = nullptr;       // [nb][Mx My Mz] (separate z pass only)
  float* part = nullptr;    // contraction partials [work-group][tile*256]
  double* rsl = nullptr;    // reduction slices [kReduceSlices][tile*256]
  double* ppart = nullptr;  // power partials (per chunk of a bin's mode list, or per inverse-x tile)
};

// Execution context of one launch sequence: job 0's workspace, the stride
// to the next job's, the number of jobs and their I/O.
struct Exec {
  Workspace ws;
  size_t wstride = 0;
  int n_jobs = 1;
  JobIO io{};
};

}  // namespace pb3

struct pb3_plan {
  // geometry: Nx x Ny x Nz cells on an Lx x Ly x Lz box
  int Nx = 0, Ny = 0, Nz = 0;
  double Lx = 0, Ly = 0, Lz = 0;
  bool aniso = false;          // box sides differ: bins on FP64 k^2 in h/Mpc (else integer |n|^2)
  unsigned flags = 0;
  int nb = 0;
  int nb_pad = 0;  // bins rounded up to the contraction's 16-bin groups
  std::vector<double> edges;   // k_f units (cubic box) or h/Mpc (anisotropic box)
  std::vector<int64_t> thr;    // cubic box: smallest |n|^2 in bin b (thr[nb]: first |n|^2 above the top)
  int Kx = 0, Ky = 0, Kzt = 0; // max |n_i| over binned modes, per axis
  bool fullx = false, fully = false, fullz = false;  // compact extent == whole axis
  int Kcx = 0, Kcy = 0;        // centred offsets of the compact x / y index
  int Lcx = 0, Lcy = 0;        // compact x / y lengths
  int Kz = 0;                  // compact z length
  int Mx = 0, My = 0, Mz = 0;  // contraction grid
  double kf2[3] = {0, 0, 0};   // (2 pi / L_i)^2
  double msc[3] = {1, 1, 1};   // multipole scales: k_f,i^2 / k_f,z^2 (all exactly 1 for a cubic box)
  std::vector<int8_t> bin3;    // bin of every compact mode [Lcx][Lcy][Kz], then a trailing -1
  bool fused = false;          // inverse z pass fused into the contraction (no G in HBM)
  bool fused_ok = false;       // the fused kernel supports this plan
  int lmax = 0;                // highest multipole (0, 2 or 4)
  bool weighted = false;       // pb3_plan_set_weights was called
  int window_order = 0;        // pixel window deconvolved (0 none, 1 NGP, 2 CIC, 3 TSC)
  double nbar = 0;             // number density for the shot-noise terms (0: none)
  double pk_shift = 0;         // subtracted from P (shot noise 1 / nbar)
  std::vector<double> pfid;    // P_fid over integer |n|^2 (weighted plans)
  std::vector<double> pml_inv; // per bin inverse discrete Fisher of the power multipoles, x V / N_pix^2
  std::vector<double> bk_mix;  // bispectrum multipole Fisher mixing per kept triplet [n_ell][n_ell] (or empty)
  int tuned = 0;               // launch shape: 0 default, 1 from the autotune cache, 2 measured
  int lut_len = 0;             // cubic box: bin of |n|^2 for |n|^2 < lut_len
  std::vector<int8_t> lut;
  std::vector<int64_t> nmodes;
  std::vector<double> kmean;
  std::vector<pb3::BinGeom> geom;
  int64_t a1_len = 0, a2_len = 0;  // float2 counts
  std::vector<int32_t> trip_all;   // candidates (a,b,c)
  std::vector<int32_t> trip;       // kept
  std::vector<double> counts;      // kept T
  std::vector<int32_t> modes;
  std::vector<int32_t> chunks;
  int n_chunks = 0;
  std::vector<int32_t> chunk_first;
  pb3::TileSet tx{}, ty{}, tz{};   // FP32 inverse-pass tiles (device)
  // contraction
  int contract_wgs = 0;        // partial vectors (accumulation chunks) of the contraction
  int part_len = 0;            // floats per partial vector of the bispectrum's contraction (its MFMA tiles * 256)
  int part_len_ab = 0;         // the same for pairs against separate column fields (multipoles)
  int n_cu = 0;                // compute units of the plan's device
  pb3_precision last_prec = PB3_FP32;
  bool device = false;
  int device_id = 0;
  pb3::DeviceTables d;
  pb3::Workspace ws;
  // timing: ring of event pairs, slot = call index mod kTimingRing
  static constexpr int kTimingRing = 256;
  std::vector<hipEvent_t> ev;              // [ring][stage][2]
  std::vector<uint8_t> ev_used;            // [ring][stage]
  long n_calls = 0;                        // calls since the last reset
  hipStream_t last_stream = nullptr;
};

namespace pb3 {

// cells of the data grid and of the contraction grid
inline size_t npix(const pb3_plan& p) { return (size_t)p.Nx * p.Ny * p.Nz; }
inline size_t mpix(const pb3_plan& p) { return (size_t)p.Mx * p.My * p.Mz; }
// compact spectrum entries
inline size_t ncompact(const pb3_plan& p) { return (size_t)p.Lcx * p.Lcy * p.Kz; }

void set_error(const std::string& msg);
pb3_status hip_fail(hipError_t e, const char* what);
// Every device allocation of the library goes through dev_malloc.  Test
// hook: with PB3_FAIL_ALLOC_AT=n in the environment, the n-th allocation
// counted from when that value was first seen fails with
// hipErrorOutOfMemory (a changed value restarts the count; text after the
// number is ignored).
hipError_t dev_malloc(void** ptr, size_t bytes);

// plan workspace (pb3_host.cpp): size and layout at base
size_t workspace_bytes(const pb3_plan* p);
Workspace carve(const pb3_plan* p, void* base, size_t bytes);
pb3_status check_prec(pb3_precision prec);
// PB3_EINVAL unless p is 8-byte aligned (what names the argument in the error)
pb3_status check_field_ptr(const void* p, const char* what);
// the whole launch sequence of one plan for the jobs of x, on stream s
pb3_status enqueue(const pb3_plan& p, const Exec& x, bool do_pk, bool do_bk, pb3_precision prec, hipStream_t s);
int launches_per_sequence(const pb3_plan& p, bool do_pk, bool do_bk);

// kernel launchers (pb3_kernels.hip); all return hipGetLastError()
hipError_t launch_fwd_z(const pb3_plan& p, const Exec& x, hipStream_t s);
hipError_t launch_fwd_y(const pb3_plan& p, const Exec& x, hipStream_t s);
hipError_t launch_fwd_x(const pb3_plan& p, const Exec& x, hipStream_t s);
// final = false leaves the per-bin sums to launch_reduce(..., with_pk = true).
hipError_t launch_power(const pb3_plan& p, const Exec& x, hipStream_t s, bool final);
hipError_t launch_inv_x(const pb3_plan& p, const Exec& x, hipStream_t s, double* ppart = nullptr);
hipError_t launch_inv_y(const pb3_plan& p, const Exec& x, hipStream_t s);
hipError_t launch_inv_z(const pb3_plan& p, const Exec& x, hipStream_t s);
hipError_t launch_contract(const pb3_plan& p, const Exec& x, pb3_precision prec, hipStream_t s);
// with_pk: also the power spectrum's per-bin sums (after launch_power(..., false)).
hipError_t launch_reduce(const pb3_plan& p, const Exec& x, hipStream_t s, bool with_pk, bool pk_folded);
// With both spectra of an unweighted plan, the power spectrum's per-bin
// sums are taken by the inverse x pass (one FP64 partial per tile) and
// finished in the reduction's launch.
bool power_folded(const pb3_plan& p, bool do_pk, bool do_bk);
int n_x_tiles(const pb3_plan& p);
// window moments and P / <w^2>, B / <w^3> (scratch: 2 + 2 kWindowBlocks doubles;
// scratch[0..1] receive <w^2>, <w^3>)
hipError_t launch_window(long n, const float* w, double* pk, int nb, double* bk, int nt, double* scratch,
                         hipStream_t s);
// FP64 triangle counts on the contraction grid: writes raw M^6 sum HHH for
// every candidate triplet into counts_out (host), using temporary memory.
// With the plan's P_fid weights set, the weighted counts sum 1/(P_1 P_2 P_3);
// q_out (may be null) receives the shot-noise sums of the weighted estimator
// sum over closed triangles of 1/(P_2 P_3) + 1/(P_1 P_3) + 1/(P_1 P_2).
pb3_status compute_counts_fp64(pb3_plan& p, std::vector<double>& counts_out, std::vector<double>* q_out = nullptr);
pb3_status compute_bk_mixing(pb3_plan& p, std::vector<double>& mix_out);
// masked power spectrum with the Monte Carlo Fisher matrix (pb3_kernels.hip)
size_t masked_workspace_bytes(const pb3_plan& p);
// multipoles (pb3_kernels.hip)
size_t multipoles_workspace_bytes(const pb3_plan& p);
pb3_status run_multipoles(pb3_plan& p, const float* delta, double* pk_out, double* bk_out, pb3_precision prec,
                          void* workspace, hipStream_t s);
pb3_status run_masked_power(pb3_plan& p, const float* data, const float* window, const float* const* grfs, int n_grf,
                            double* pk_out, double* f_out, void* workspace, hipStream_t s);
// bispectrum with the Monte Carlo linear term (pb3_kernels.hip)
size_t linear_workspace_bytes(const pb3_plan& p, int n_sim);
pb3_status run_bispectrum_linear(pb3_plan& p, const float* data, const float* const* sims, int n_sim, double* bk_out,
                                 pb3_precision prec, void* workspace, hipStream_t s);
// MFMA contraction (contract_mfma.hip): tiles for nq 16-bin groups, the
// partial-vector index of triplet (a, b, c) (-1 if not produced), launch
// ab = true: every pair a <= b against columns c (separate column fields);
// ab = false: the bispectrum's layout (pairs inside a 16-bin group)
int mfma_tiles(bool ab, int nb);
int mfma_locate(bool ab, int nb, int a, int b, int c);
hipError_t launch_contract_mfma(const pb3_plan& p, const Exec& x, bool mixed, hipStream_t s);
// pairs of the fields g against columns of the fields gc (nb bins each, M^3
// voxels; gc == nullptr: g itself) into x.ws.part.  ab = true: every pair
// a <= b against columns c >= its group (mixed precision only; the
// multipoles), else the bispectrum's layout (gc must be null).
hipError_t launch_contract_cols(const pb3_plan& p, const Exec& x, const float* g, const float* gc, bool mixed,
                                bool ab, hipStream_t s);
int mfma_grid(int nq, int n_cu);
// fused inverse z pass + contraction (contract_mfma.hip)
bool fused_supported(int nq, int m);
int fused_grid(int nq, int m, long mvox, int n_cu);
hipError_t launch_zcontract(const pb3_plan& p, const Exec& x, bool mixed, hipStream_t s);
// inverse passes (fft_passes.hip) on FP32 (dbl = false) or FP64 lines;
// unit = the shell indicator instead of Theta_b D (count pass, FP64 only);
// n_jobs jobs whose buffers are wstride bytes apart
// weighted: apply the plan's window / P_fid weights (estimator fields);
// unit_w: per-|n|^2 weight of the unit fields (count pass, may be null);
// ppart: FP32 unweighted spectra only, one FP64 power partial per tile (may be null)
// (the FP32 or FP64 twiddles of the axis are the plan's)
// Angular weight of the FP64 unit fields: L_l1(mu) L_l2(mu) u_x^ex u_y^ey u_z^ez
// with u = k / |k| and mu = u_z (all zero: no angular weight).  A mode with
// a Nyquist component (|k_i| = h_i, half the grid) takes the average over its
// representatives +-h_i, so an odd power of that component gives zero.
struct AngW {
  int l1 = 0, l2 = 0, ex = 0, ey = 0, ez = 0;
  int hx = -1, hy = -1, hz = -1;
};
hipError_t run_inv_x(const pb3_plan& p, bool dbl, bool unit, const float2* dc, void* a1, const TileSet& ts,
                     int n_jobs, size_t wstride, hipStream_t s, int ell = 0, const double* unit_w = nullptr,
                     bool weighted = false, AngW aw = AngW{}, double* ppart = nullptr);
hipError_t run_inv_y(const pb3_plan& p, bool dbl, const void* a1, void* a2, const TileSet& ts, int n_jobs,
                     size_t wstride, hipStream_t s);
hipError_t run_inv_z(const pb3_plan& p, bool dbl, const void* a2, void* gout, const TileSet& ts, int n_jobs,
                     size_t wstride, hipStream_t s);
// z round trip of the masked power spectrum's Monte Carlo: per bin, the inverse z
// pass, times the window, then the forward z pass kept at kz < Kz (full grid,
// z lengths of the half-length form)
bool zround_supported(const pb3_plan& p);
hipError_t run_zround(const pb3_plan& p, const float2* a2, const float* window, float2* f1, hipStream_t s);
// tile widths of the inverse passes for FP32 (dbl = false) or FP64 lines
int tile_width_x(int M, bool dbl);
int tile_width_z(int M, bool dbl);
// per-bin tile tables of the three inverse passes (host): x pass (row jy,
// chunk of tbxy columns), y pass (x-plane, chunk), z pass tbz lines
void build_tiles(const pb3_plan& p, int tbxy, int tbz, std::vector<BinTile>& vx, std::vector<BinTile>& vy,
                 std::vector<BinTile>& vz);

}  // namespace pb3
