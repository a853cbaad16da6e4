// Host side of the MI355X polyspectrum library: plan construction (bins,
// triplets, contraction grid, tables, triangle counts), workspace
// management and the C ABI declared in include/pb3.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include <unistd.h>

#include "pb3_internal.h"

namespace pb3 {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

pb3_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? PB3_ENOMEM : PB3_EDEVICE;
}

hipError_t dev_malloc(void** ptr, size_t bytes) {
  static std::mutex mu;
  static std::string seen;
  static long count = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    const char* v = std::getenv("PB3_FAIL_ALLOC_AT");
    const std::string cur = v ? v : "";
    if (cur != seen) {
      seen = cur;
      count = 0;
    }
    const long at = cur.empty() ? 0 : std::atol(cur.c_str());
    if (at > 0 && ++count == at) {
      *ptr = nullptr;
      return hipErrorOutOfMemory;
    }
  }
  return hipMalloc(ptr, bytes);
}

static bool len_supported(int n) {
  static const int ok[] = {16, 24, 32, 48, 64, 96, 128, 192, 256, 384};
  for (int v : ok)
    if (v == n) return true;
  return false;
}

// smallest supported length strictly above lo and not above hi (0 if none)
static int smallest_len_above(int lo, int hi) {
  static const int ok[] = {16, 24, 32, 48, 64, 96, 128, 192, 256, 384};
  for (int v : ok)
    if (v > lo && v <= hi) return v;
  return 0;
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

void build_tiles(const pb3_plan& p, int tbxy, int tbz, std::vector<BinTile>& vx, std::vector<BinTile>& vy,
                 std::vector<BinTile>& vz) {
  vx.clear();
  vy.clear();
  vz.clear();
  for (int b = 0; b < p.nb; ++b) {
    const BinGeom& g = p.geom[b];
    // x pass: chunks of the flattened (jy, kz) columns; y pass: of the flattened (x, kz) columns
    for (int c = 0; c < g.ly * g.kzn; c += tbxy) vx.push_back(BinTile{b, c});
    for (int c = 0; c < p.Mx * g.kzn; c += tbxy) vy.push_back(BinTile{b, c});
    int nz = p.Mx * p.My;
    for (int c = 0; c < nz; c += tbz) vz.push_back(BinTile{b, c});
  }
}

// FP64 twiddle table W_n^j = exp(-2 pi i j / n), j < n
static std::vector<double> twiddles(int n) {
  std::vector<double> w(2 * (size_t)n);
  for (int j = 0; j < n; ++j) {
    // exact angles via the reduced fraction j/n; sin/cos of multiples of pi/2 exact
    double a = -2.0 * M_PI * (double)j / (double)n;
    double c = std::cos(a), s = std::sin(a);
    if (4 * j % n == 0) {
      int q = 4 * j / n;
      c = (q == 0) ? 1.0 : (q == 2) ? -1.0 : 0.0;
      s = (q == 1) ? -1.0 : (q == 3) ? 1.0 : 0.0;
    }
    w[2 * j] = c;
    w[2 * j + 1] = s;
  }
  return w;
}

template <typename T> static pb3_status dalloc(T** ptr, size_t count) {
  hipError_t e = dev_malloc((void**)ptr, sizeof(T) * (count ? count : 1));
  if (e != hipSuccess) {
    *ptr = nullptr;
    set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
    return PB3_ENOMEM;
  }
  return PB3_OK;
}

template <typename T> static pb3_status upload(T** ptr, const T* src, size_t count) {
  pb3_status st = dalloc(ptr, count);
  if (st != PB3_OK) return st;
  if (count == 0) return PB3_OK;
  hipError_t e = hipMemcpy(*ptr, src, sizeof(T) * count, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  return PB3_OK;
}

static pb3_status upload_twiddles_f(float2** out, int n) {
  std::vector<double> w = twiddles(n);
  std::vector<float2> f(n);
  for (int j = 0; j < n; ++j) f[j] = make_float2((float)w[2 * j], (float)w[2 * j + 1]);
  return upload(out, f.data(), f.size());
}

static pb3_status upload_twiddles_d(double2** out, int n) {
  std::vector<double> w = twiddles(n);
  std::vector<double2> f(n);
  for (int j = 0; j < n; ++j) f[j] = make_double2(w[2 * j], w[2 * j + 1]);
  return upload(out, f.data(), f.size());
}

static void free_device(pb3_plan* p) {
  DeviceTables& d = p->d;
  void* ptrs[] = {d.bin3,      d.modes,      d.chunk,     d.chunk_first, d.geom,      d.tiles,     d.trip_all,
                  d.out_map,   d.inv_counts, d.pk_scale,  d.tw_n[0],     d.tw_n[1],   d.tw_n[2],   d.tw_m[0],
                  d.tw_m[1],   d.tw_m[2],    d.tw_m_d[0], d.tw_m_d[1],   d.tw_m_d[2], d.nmodes_d,  d.pml_inv,
                  d.ml_trips,  d.ml_fac,     d.ml_map,    d.win_inv,     d.pfid_inv,  d.pfid_inv_d, d.mode_w,
                  d.bk_bias,   d.bk_mix,     d.out_map_ab, d.xtile_first, d.out_inv};
  for (void* q : ptrs)
    if (q) hipFree(q);
  d = DeviceTables{};
  if (p->ws.owned && p->ws.base) hipFree(p->ws.base);
  p->ws = Workspace{};
  for (hipEvent_t e : p->ev)
    if (e) hipEventDestroy(e);
  p->ev.clear();
}

// ------------------------------------------------------------ host plan
static pb3_status build_host(pb3_plan* p, const int grid[3], const double box[3], const double* edges, int n_edges,
                             unsigned flags) {
  if (!grid || !box || !edges) {
    set_error("null argument");
    return PB3_EINVAL;
  }
  for (int a = 0; a < 3; ++a) {
    if (grid[a] <= 0 || grid[a] % 2) {
      set_error("grid lengths must be positive and even");
      return PB3_EINVAL;
    }
    if (!len_supported(grid[a])) {
      set_error("grid length " + std::to_string(grid[a]) +
                " not implemented (supported: 16..384 of the form 2^a 3^b)");
      return PB3_EUNSUPPORTED;
    }
    if (!(box[a] > 0) || !std::isfinite(box[a])) {
      set_error("box sides must be positive");
      return PB3_EINVAL;
    }
  }
  if ((long)grid[0] * grid[1] * grid[2] > (1L << 31) - 1) {
    set_error("more than 2^31 - 1 grid cells not implemented");
    return PB3_EUNSUPPORTED;
  }
  if (n_edges < 2) {
    set_error("need at least two bin edges");
    return PB3_EINVAL;
  }
  p->Nx = grid[0];
  p->Ny = grid[1];
  p->Nz = grid[2];
  p->Lx = box[0];
  p->Ly = box[1];
  p->Lz = box[2];
  p->aniso = !(box[0] == box[1] && box[0] == box[2]);
  p->flags = flags;
  if (p->aniso && !(flags & PB3_FLAG_EDGES_HMPC)) {
    set_error("a box with unequal sides needs bin edges in h/Mpc (PB3_FLAG_EDGES_HMPC)");
    return PB3_EINVAL;
  }
  if (flags & PB3_FLAG_BK_FISHER) {
    if (!(flags & (PB3_FLAG_LMAX2 | PB3_FLAG_LMAX4)) || (flags & PB3_FLAG_POWER_ONLY)) {
      set_error("PB3_FLAG_BK_FISHER needs bispectrum multipoles (PB3_FLAG_LMAX2 or PB3_FLAG_LMAX4, not power-only)");
      return PB3_EINVAL;
    }
    if (p->aniso) {
      set_error("the bispectrum multipole Fisher matrix is implemented for boxes with equal sides");
      return PB3_EUNSUPPORTED;
    }
  }
  for (int a = 0; a < 3; ++a) {
    const double kf = 2.0 * M_PI / box[a];
    p->kf2[a] = kf * kf;
  }
  for (int a = 0; a < 3; ++a) p->msc[a] = p->kf2[a] / p->kf2[2];
  const double kf = 2.0 * M_PI / p->Lx;  // cubic box: the k_f of every axis
  p->edges.resize(n_edges);
  for (int i = 0; i < n_edges; ++i) {
    double e = edges[i];
    if (!std::isfinite(e) || e < 0) {
      set_error("bin edges must be finite and non-negative");
      return PB3_EINVAL;
    }
    if ((flags & PB3_FLAG_EDGES_HMPC) && !p->aniso) {
      e /= kf;
      double h = std::round(2.0 * e) / 2.0;
      if (std::fabs(e - h) <= 1e-9 * std::max(1.0, std::fabs(e))) e = h;
    }
    p->edges[i] = e;
    if (i > 0 && !(p->edges[i] > p->edges[i - 1])) {
      set_error("bin edges must be strictly increasing");
      return PB3_EINVAL;
    }
  }
  const int nb = n_edges - 1;
  if (nb > 48) {
    set_error("more than 48 bins not implemented");
    return PB3_EUNSUPPORTED;
  }
  p->nb = nb;
  p->nb_pad = (nb + 15) / 16 * 16;
  const int Ng[3] = {p->Nx, p->Ny, p->Nz};
  // Bin membership.  Cubic box: integer thresholds, |n|^2 in bin b <=>
  // thr[b] <= |n|^2 < thr[b+1].  Anisotropic box: the FP64 value
  // k^2 = (kf2x nx^2 + kf2y ny^2) + kf2z nz^2 against e_b^2 (h/Mpc), in that
  // order of operations.
  std::vector<double> e2(nb + 1);
  for (int i = 0; i <= nb; ++i) e2[i] = p->edges[i] * p->edges[i];
  if (!p->aniso) {
    p->thr.resize(nb + 1);
    for (int i = 0; i <= nb; ++i) {
      int64_t t = (int64_t)std::ceil(e2[i]);
      // guard against e2 just above an integer through rounding of the square
      while (t > 0 && (double)(t - 1) >= e2[i]) --t;
      while ((double)t < e2[i]) ++t;
      p->thr[i] = t;
    }
  }
  // largest |n_i| with the single-axis mode n_i e_i below the top edge (kb
  // below the edge of bin b's upper side), clamped to the Nyquist index
  auto axis_max = [&](int a, int b_top) -> int {
    int k = 0;
    if (!p->aniso) {
      const int64_t top = p->thr[b_top] - 1;  // largest |n|^2 inside
      if (top < 0) return -1;
      k = (int)std::floor(std::sqrt((double)top));
      while ((int64_t)(k + 1) * (k + 1) <= top) ++k;
      while ((int64_t)k * k > top) --k;
    } else {
      if (!(e2[b_top] > 0.0)) return -1;
      k = 0;
      while (k < Ng[a] / 2 && p->kf2[a] * ((double)(k + 1) * (double)(k + 1)) < e2[b_top]) ++k;
    }
    return std::min(k, Ng[a] / 2);
  };
  p->Kx = axis_max(0, nb);
  p->Ky = axis_max(1, nb);
  p->Kzt = axis_max(2, nb);
  if (p->Kx < 0 || p->Ky < 0 || p->Kzt < 0) {
    set_error("the top bin edge is zero");
    return PB3_EINVAL;
  }
  p->fullx = p->Kx >= p->Nx / 2;
  p->fully = p->Ky >= p->Ny / 2;
  p->fullz = p->Kzt >= p->Nz / 2;
  p->Kcx = p->fullx ? p->Nx / 2 : p->Kx;
  p->Lcx = p->fullx ? p->Nx : 2 * p->Kx + 1;
  p->Kcy = p->fully ? p->Ny / 2 : p->Ky;
  p->Lcy = p->fully ? p->Ny : 2 * p->Ky + 1;
  p->Kz = p->fullz ? p->Nz / 2 + 1 : p->Kzt + 1;
  // contraction grid per axis: an alias-free smaller grid when 3 K_i < N_i
  p->Mx = p->Nx;
  p->My = p->Ny;
  p->Mz = p->Nz;
  if (!(flags & PB3_FLAG_FULL_GRID)) {
    int m;
    if (3 * p->Kx < p->Nx && (m = smallest_len_above(3 * p->Kx, p->Nx))) p->Mx = m;
    if (3 * p->Ky < p->Ny && (m = smallest_len_above(3 * p->Ky, p->Ny))) p->My = m;
    if (3 * p->Kzt < p->Nz && (m = smallest_len_above(3 * p->Kzt, p->Nz))) p->Mz = m;
  }
  // cubic box: bin lookup by |n|^2
  if (!p->aniso) {
    const int64_t kk = (int64_t)p->Kcx * p->Kcx + (int64_t)p->Kcy * p->Kcy + (int64_t)(p->Kz - 1) * (p->Kz - 1);
    p->lut_len = (int)kk + 1;
    p->lut.assign(p->lut_len, (int8_t)-1);
    for (int64_t n2 = 0; n2 < p->lut_len; ++n2)
      for (int b = 0; b < nb; ++b)
        if (n2 >= p->thr[b] && n2 < p->thr[b + 1]) p->lut[n2] = (int8_t)b;
  }
  auto bin_of = [&](int kx, int ky, int kz) -> int {
    if (!p->aniso) {
      const int64_t n2 = (int64_t)kx * kx + (int64_t)ky * ky + (int64_t)kz * kz;
      return n2 < p->lut_len ? p->lut[n2] : -1;
    }
    double k2 = p->kf2[0] * (double)((int64_t)kx * kx) + p->kf2[1] * (double)((int64_t)ky * ky);
    k2 = k2 + p->kf2[2] * (double)((int64_t)kz * kz);
    if (k2 < e2[0] || !(k2 < e2[nb])) return -1;
    int b = (int)(std::upper_bound(e2.begin(), e2.end(), k2) - e2.begin()) - 1;
    return b;
  };
  // modes of the compact half spectrum, per bin
  std::vector<std::vector<int32_t>> per(nb);
  p->nmodes.assign(nb, 0);
  p->bin3.assign(ncompact(*p) + 1, (int8_t)-1);  // a trailing "no bin" entry
  p->lmax = (flags & PB3_FLAG_LMAX4) ? 4 : (flags & PB3_FLAG_LMAX2) ? 2 : 0;
  const int ne = p->lmax / 2 + 1;
  std::vector<double> msum((size_t)nb * ne * ne, 0.0);  // per bin: sum over its modes of L_i L_j
  std::vector<double> ksum(nb, 0.0);
  const double* ms = p->msc;
  for (int cx = 0; cx < p->Lcx; ++cx) {
    int kx = cx - p->Kcx;
    for (int cy = 0; cy < p->Lcy; ++cy) {
      int ky = cy - p->Kcy;
      for (int kz = 0; kz < p->Kz; ++kz) {
        const int b = bin_of(kx, ky, kz);
        if (b < 0) continue;
        const bool self = (kz == 0) || (p->fullz && kz == p->Nz / 2);
        const int32_t idx = (int32_t)(((int64_t)cx * p->Lcy + cy) * p->Kz + kz);
        p->bin3[idx] = (int8_t)b;
        per[b].push_back(self ? (int32_t)(idx | 0x80000000u) : idx);
        const int w = self ? 1 : 2;
        p->nmodes[b] += w;
        if (!p->aniso) {
          ksum[b] += w * std::sqrt((double)((int64_t)kx * kx + (int64_t)ky * ky + (int64_t)kz * kz)) * kf;
        } else {
          double k2 = p->kf2[0] * (double)((int64_t)kx * kx) + p->kf2[1] * (double)((int64_t)ky * ky);
          k2 = k2 + p->kf2[2] * (double)((int64_t)kz * kz);
          ksum[b] += w * std::sqrt(k2);
        }
        if (ne > 1) {
          // mu^2 = k_z^2 / k^2 (integer arithmetic for a cubic box, whose scales are 1)
          const double den = ms[0] * kx * kx + ms[1] * ky * ky + ms[2] * kz * kz;
          const double m2 = den > 0 ? ms[2] * kz * kz / den : 0.0;
          const double L[3] = {1.0, 1.5 * m2 - 0.5, (35.0 * m2 * m2 - 30.0 * m2 + 3.0) / 8.0};
          for (int i = 0; i < ne; ++i)
            for (int j = 0; j < ne; ++j) msum[((size_t)b * ne + i) * ne + j] += w * L[i] * L[j];
        }
      }
    }
  }
  for (int b = 0; b < nb; ++b) {
    if (p->nmodes[b] == 0) {
      set_error("bin " + std::to_string(b) + " contains no grid modes");
      return PB3_EINVAL;
    }
  }
  p->kmean.resize(nb);
  for (int b = 0; b < nb; ++b) p->kmean[b] = ksum[b] / (double)p->nmodes[b];
  // power multipoles: per bin, the inverse of the discrete Fisher matrix
  // (1/2) sum_n L_i L_j (its 1/2 cancels the numerator's), times V / N_pix^2
  if (ne > 1) {
    const double np = (double)p->Nx * p->Ny * p->Nz;
    const double sc = p->Lx * p->Ly * p->Lz / (np * np);
    p->pml_inv.assign((size_t)nb * ne * ne, 0.0);
    for (int b = 0; b < nb; ++b) {
      double a[3][6] = {};
      for (int i = 0; i < ne; ++i) {
        for (int j = 0; j < ne; ++j) a[i][j] = msum[((size_t)b * ne + i) * ne + j];
        a[i][ne + i] = 1.0;
      }
      for (int k = 0; k < ne; ++k) {  // Gauss-Jordan with partial pivoting
        int pr = k;
        for (int r = k + 1; r < ne; ++r)
          if (std::fabs(a[r][k]) > std::fabs(a[pr][k])) pr = r;
        if (std::fabs(a[pr][k]) < 1e-9 * (double)p->nmodes[b]) {
          set_error("bin " + std::to_string(b) + " has too few mode directions to separate the multipoles");
          return PB3_EINVAL;
        }
        for (int c = 0; c < 2 * ne; ++c) std::swap(a[k][c], a[pr][c]);
        const double d = a[k][k];
        for (int c = 0; c < 2 * ne; ++c) a[k][c] /= d;
        for (int r = 0; r < ne; ++r)
          if (r != k) {
            const double f = a[r][k];
            for (int c = 0; c < 2 * ne; ++c) a[r][c] -= f * a[k][c];
          }
      }
      for (int i = 0; i < ne; ++i)
        for (int j = 0; j < ne; ++j) p->pml_inv[((size_t)b * ne + i) * ne + j] = sc * a[i][ne + j];
    }
  }
  p->modes.clear();
  p->chunks.clear();
  const int CH = 1024;
  for (int b = 0; b < nb; ++b) {
    int start = (int)p->modes.size();
    p->modes.insert(p->modes.end(), per[b].begin(), per[b].end());
    int end = (int)p->modes.size();
    for (int s = start; s < end; s += CH) {
      p->chunks.push_back(b);
      p->chunks.push_back(s);
      p->chunks.push_back(std::min(end, s + CH));
    }
  }
  p->n_chunks = (int)(p->chunks.size() / 3);
  p->chunk_first.assign(nb + 1, 0);
  for (int c = 0, b = 0; b <= nb; ++b) {
    while (c < p->n_chunks && p->chunks[3 * c] < b) ++c;
    p->chunk_first[b] = c;
  }
  // per-bin spectrum rectangles and intermediate offsets
  p->geom.resize(nb);
  int64_t o1 = 0, o2 = 0;
  for (int b = 0; b < nb; ++b) {
    const int kbx = axis_max(0, b + 1), kby = axis_max(1, b + 1), kbz = axis_max(2, b + 1);
    BinGeom g{};
    g.knegx = std::max(kbx, 0);
    g.kposx = (p->fullx && kbx == p->Nx / 2) ? p->Nx / 2 - 1 : std::max(kbx, 0);
    g.knegy = std::max(kby, 0);
    g.kposy = (p->fully && kby == p->Ny / 2) ? p->Ny / 2 - 1 : std::max(kby, 0);
    g.ly = g.knegy + g.kposy + 1;
    g.kzn = std::max(kbz, 0) + 1;
    g.n2lo = p->aniso ? -1 : (int32_t)p->thr[b];
    g.n2hi = p->aniso ? -1 : (int32_t)p->thr[b + 1];
    g.a1_off = o1;
    g.a2_off = o2;
    o1 += (int64_t)p->Mx * g.ly * g.kzn;
    o2 += (int64_t)p->Mx * p->My * g.kzn;
    p->geom[b] = g;
  }
  p->a1_len = o1;
  p->a2_len = o2;
  // triangle-valid triplets, c fastest
  p->trip_all.clear();
  for (int a = 0; a < nb; ++a)
    for (int b = a; b < nb; ++b)
      for (int c = b; c < nb; ++c)
        if (p->edges[c] < p->edges[a + 1] + p->edges[b + 1]) {
          p->trip_all.push_back(a);
          p->trip_all.push_back(b);
          p->trip_all.push_back(c);
        }
  if (flags & PB3_FLAG_POWER_ONLY) p->trip_all.clear();
  if (p->trip_all.size() / 3 > 8192) {
    set_error("more than 8192 triplets not implemented");
    return PB3_EUNSUPPORTED;
  }
  p->trip = p->trip_all;
  p->fused_ok = !(flags & PB3_FLAG_POWER_ONLY) && fused_supported(p->nb_pad / 16, p->Mz);
  p->fused = !(flags & PB3_FLAG_NO_FUSION) && p->fused_ok;
  p->contract_wgs = 512;
  p->part_len = (flags & PB3_FLAG_POWER_ONLY) ? 0 : mfma_tiles(false, p->nb) * 256;
  p->part_len_ab = (flags & PB3_FLAG_POWER_ONLY) || p->lmax == 0 ? 0 : mfma_tiles(true, p->nb) * 256;
  return PB3_OK;
}

// floats per partial vector of the longer of the two contraction layouts
static size_t part_max(const pb3_plan& p) { return (size_t)std::max(p.part_len, p.part_len_ab); }

int n_x_tiles(const pb3_plan& p) {
  const int tb = tile_width_x(p.Mx, false);
  if (tb <= 0) return 0;
  int n = 0;
  for (int b = 0; b < p.nb && b < (int)p.geom.size(); ++b) n += (p.geom[b].ly * p.geom[b].kzn + tb - 1) / tb;
  return n;
}
// power partials: one per chunk of the mode lists, or one per inverse-x tile
static size_t ppart_len(const pb3_plan& p) { return (size_t)std::max({p.n_chunks, n_x_tiles(p), 1}); }

bool power_folded(const pb3_plan& p, bool do_pk, bool do_bk) {
  return do_pk && do_bk && !p.trip.empty() && !p.d.mode_w && !p.d.win_inv && !p.d.pfid_inv;
}

size_t workspace_bytes(const pb3_plan* p) {
  size_t b = 0;
  const size_t A = 256;
  b += align_up(sizeof(float2) * (size_t)p->Nx * p->Ny * p->Kz, A);
  b += align_up(sizeof(float2) * (size_t)p->Nx * p->Lcy * p->Kz, A);
  b += align_up(sizeof(float2) * ncompact(*p), A);
  b += align_up(sizeof(float2) * (size_t)p->a1_len, A);
  b += align_up(sizeof(float2) * (size_t)p->a2_len, A);
  const bool has_g = !p->fused && !(p->flags & PB3_FLAG_POWER_ONLY);
  b += has_g ? align_up(sizeof(float) * (size_t)p->nb * mpix(*p), A) : 0;
  b += align_up(sizeof(float) * (size_t)p->contract_wgs * part_max(*p), A);
  b += align_up(sizeof(double) * ppart_len(*p), A);
  b += align_up(sizeof(double) * (size_t)kReduceSlices * part_max(*p), A);
  return b;
}

Workspace carve(const pb3_plan* p, void* base, size_t bytes) {
  Workspace w;
  w.base = base;
  w.bytes = bytes;
  w.owned = false;
  char* c = (char*)base;
  const size_t A = 256;
  auto take = [&](size_t n) {
    char* r = c;
    c += align_up(n, A);
    return (void*)r;
  };
  w.f1 = (float2*)take(sizeof(float2) * (size_t)p->Nx * p->Ny * p->Kz);
  w.f2 = (float2*)take(sizeof(float2) * (size_t)p->Nx * p->Lcy * p->Kz);
  w.dc = (float2*)take(sizeof(float2) * ncompact(*p));
  w.a1 = (float2*)take(sizeof(float2) * (size_t)p->a1_len);
  w.a2 = (float2*)take(sizeof(float2) * (size_t)p->a2_len);
  const bool has_g = !p->fused && !(p->flags & PB3_FLAG_POWER_ONLY);
  w.g = has_g ? (float*)take(sizeof(float) * (size_t)p->nb * mpix(*p)) : nullptr;
  w.part = (float*)take(sizeof(float) * (size_t)p->contract_wgs * part_max(*p));
  w.ppart = (double*)take(sizeof(double) * ppart_len(*p));
  w.rsl = (double*)take(sizeof(double) * (size_t)kReduceSlices * part_max(*p));
  return w;
}

static void carve_workspace(pb3_plan* p, void* base, size_t bytes, bool owned) {
  p->ws = carve(p, base, bytes);
  p->ws.owned = owned;
}



static pb3_status ensure_workspace(pb3_plan* p) {
  if (p->ws.base) return PB3_OK;
  if (p->flags & PB3_FLAG_EXT_WORKSPACE) {
    set_error("plan needs a bound workspace (PB3_FLAG_EXT_WORKSPACE)");
    return PB3_EINVAL;
  }
  size_t bytes = workspace_bytes(p);
  void* base = nullptr;
  hipError_t e = dev_malloc(&base, bytes);
  if (e != hipSuccess) {
    set_error("workspace hipMalloc of " + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
    return PB3_ENOMEM;
  }
  carve_workspace(p, base, bytes, true);
  return PB3_OK;
}

// ------------------------------------------------------------ autotune
// Launch-shape choice per plan: the inverse z pass fused into the
// contraction or separate, and the number of contraction work-groups
// (multiples of the CU count).  Each candidate runs the whole bispectrum
// path a few times on a zero field; the fastest median wins, except that the
// default shape is kept unless another is more than 2% faster.  Results are
// cached in a text file (PB3_AUTOTUNE_CACHE) keyed by device architecture,
// grid, contraction grid and the bin thresholds.
static std::string tune_key(const pb3_plan* p) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, p->device_id) == hipSuccess) arch = prop.gcnArchName;
  std::ostringstream k;
  k << arch << " N" << p->Nx << "x" << p->Ny << "x" << p->Nz << " M" << p->Mx << "x" << p->My << "x" << p->Mz;
  if (p->aniso) {
    k << " L" << p->Lx << "x" << p->Ly << "x" << p->Lz << " e";
    for (double e : p->edges) k << ":" << e;
  } else {
    k << " thr";
    for (int64_t t : p->thr) k << ":" << t;
  }
  return k.str();
}

static bool tune_lookup(const std::string& path, const std::string& key, int& fused, int& wgs) {
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    size_t bar = line.rfind(" | ");
    if (bar == std::string::npos || line.compare(0, bar, key) != 0 || bar != key.size()) continue;
    std::istringstream v(line.substr(bar + 3));
    int a = -1, b = -1;
    if (v >> a >> b && (a == 0 || a == 1) && b > 0) {
      fused = a;
      wgs = b;
      found = true;  // the last entry for a key wins
    }
  }
  return found;
}

// ------------------------------------------------------------ plan cache
// The data-independent artefacts of a plan, the triangle counts T of every
// candidate triplet (eq. N-ell-def at l = 0) and, with PB3_FLAG_BK_FISHER,
// the multipole mixing blocks, can be kept on disk: with PB3_PLAN_CACHE
// naming a directory, plan creation reads them from a file keyed by the
// device architecture, the grids, the bins (and the box when its sides
// differ), and writes that file after computing them.  A file whose key,
// length or checksum does not match is ignored and rewritten.  Weighted
// sums (pb3_plan_set_weights) depend on the caller's P_fid and are not
// cached.
static uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = (const unsigned char*)data;
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

static std::string cache_file(const char* dir, const std::string& key, const char* what) {
  char name[64];
  std::snprintf(name, sizeof name, "/pb3_%s_%016llx.bin", what, (unsigned long long)fnv1a(key.data(), key.size()));
  return std::string(dir) + name;
}

static const char kCacheMagic[] = "PB3PLAN1";

static bool cache_read(const std::string& key, const char* what, std::vector<double>& v, size_t n) {
  const char* dir = std::getenv("PB3_PLAN_CACHE");
  if (!dir || !*dir) return false;
  std::ifstream f(cache_file(dir, key, what), std::ios::binary);
  if (!f) return false;
  std::string magic, k, w;
  if (!std::getline(f, magic) || magic != kCacheMagic || !std::getline(f, k) || k != key || !std::getline(f, w) ||
      w != what)
    return false;
  uint64_t len = 0, sum = 0;
  if (!f.read((char*)&len, sizeof len) || len != n) return false;
  std::vector<double> t(n);
  if (n && !f.read((char*)t.data(), sizeof(double) * n)) return false;
  if (!f.read((char*)&sum, sizeof sum)) return false;
  uint64_t h = fnv1a(key.data(), key.size());
  h = fnv1a(t.data(), sizeof(double) * n, h);
  if (h != sum) return false;
  v.swap(t);
  return true;
}

static void cache_write(const std::string& key, const char* what, const std::vector<double>& v) {
  const char* dir = std::getenv("PB3_PLAN_CACHE");
  if (!dir || !*dir) return;
  const std::string path = cache_file(dir, key, what);
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
    if (!f) return;
    const uint64_t len = v.size();
    uint64_t h = fnv1a(key.data(), key.size());
    h = fnv1a(v.data(), sizeof(double) * v.size(), h);
    f << kCacheMagic << "\n" << key << "\n" << what << "\n";
    f.write((const char*)&len, sizeof len);
    f.write((const char*)v.data(), sizeof(double) * v.size());
    f.write((const char*)&h, sizeof h);
    if (!f) {
      f.close();
      std::remove(tmp.c_str());
      return;
    }
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());  // whole files only
}

static pb3_status autotune(pb3_plan* p, int n_cu) {
  const char* path = std::getenv("PB3_AUTOTUNE_CACHE");
  const std::string key = tune_key(p);
  int c_fused = -1, c_wgs = -1;
  if (path && tune_lookup(path, key, c_fused, c_wgs) && (!c_fused || p->fused_ok)) {
    p->fused = c_fused == 1;
    p->contract_wgs = c_wgs;
    p->tuned = 1;
    return PB3_OK;
  }
  struct Cand {
    bool fused;
    int wgs;
  };
  std::vector<Cand> cands;
  const int nq = p->nb_pad / 16;
  if (p->fused_ok) {
    const int base = fused_grid(nq, p->Mz, (long)mpix(*p), n_cu);
    for (int mult : {1, 2}) cands.push_back({true, base * mult});
  }
  for (int mult : {1, 2, 3, 4}) cands.push_back({false, n_cu * mult});
  // scratch: the largest workspace, a zero field and outputs
  size_t ws_max = 0;
  const bool keep_fused = p->fused;
  const int keep_wgs = p->contract_wgs;
  for (const Cand& c : cands) {
    p->fused = c.fused;
    p->contract_wgs = c.wgs;
    ws_max = std::max(ws_max, workspace_bytes(p));
  }
  p->fused = keep_fused;
  p->contract_wgs = keep_wgs;
  const size_t n3 = npix(*p);
  const int nt = (int)(p->trip.size() / 3);
  void *ws = nullptr, *fld = nullptr, *bk = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  pb3_status st = PB3_OK;
  hipError_t e;
  if ((e = dev_malloc(&ws, ws_max)) != hipSuccess || (e = dev_malloc(&fld, sizeof(float) * n3)) != hipSuccess ||
      (e = dev_malloc(&bk, sizeof(double) * std::max(nt, 1))) != hipSuccess) {
    st = PB3_ENOMEM;
    set_error("autotune allocation failed");
  }
  if (st == PB3_OK && ((e = hipMemset(fld, 0, sizeof(float) * n3)) != hipSuccess ||
                       (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess))
    st = hip_fail(e, "autotune set-up");
  float best = 1e30f, def_ms = -1.f;
  Cand pick{keep_fused, keep_wgs};
  for (size_t ci = 0; ci < cands.size() && st == PB3_OK; ++ci) {
    p->fused = cands[ci].fused;
    p->contract_wgs = cands[ci].wgs;
    Exec x;
    x.ws = carve(p, ws, ws_max);
    x.io.delta[0] = (const float*)fld;
    x.io.bk[0] = (double*)bk;
    std::vector<float> ms;
    for (int r = 0; r < 4 && st == PB3_OK; ++r) {
      if ((e = hipEventRecord(e0, nullptr)) != hipSuccess) {
        st = hip_fail(e, "hipEventRecord");
        break;
      }
      st = enqueue(*p, x, false, true, PB3_MIXED_BF16X3, nullptr);
      if (st != PB3_OK) break;
      if ((e = hipEventRecord(e1, nullptr)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) {
        st = hip_fail(e, "autotune timing");
        break;
      }
      float t = 0.f;
      hipEventElapsedTime(&t, e0, e1);
      if (r > 0) ms.push_back(t);  // the first run warms up
    }
    if (st != PB3_OK) break;
    std::sort(ms.begin(), ms.end());
    const float med = ms[ms.size() / 2];
    if (cands[ci].fused == keep_fused && cands[ci].wgs == keep_wgs) def_ms = med;
    if (med < best) {
      best = med;
      pick = cands[ci];
    }
  }
  // keep the default shape unless another is clearly faster (the medians of
  // nearly equal shapes swap from run to run)
  if (st == PB3_OK && def_ms > 0.f && best > 0.98f * def_ms) {
    pick = Cand{keep_fused, keep_wgs};
    best = def_ms;
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(ws);
  hipFree(fld);
  hipFree(bk);
  if (st != PB3_OK) return st;
  p->fused = pick.fused;
  p->contract_wgs = pick.wgs;
  p->tuned = 2;
  if (path) {
    std::ofstream f(path, std::ios::app);
    if (f) f << key << " | " << (pick.fused ? 1 : 0) << " " << pick.wgs << " " << best << "\n";
  }
  return PB3_OK;
}

static pb3_status build_device(pb3_plan* p) {
  pb3_status st;
  hipError_t e = hipGetDevice(&p->device_id);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  int n_cu = 0;
  e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, p->device_id);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  p->n_cu = n_cu;
  p->contract_wgs = p->fused ? fused_grid(p->nb_pad / 16, p->Mz, (long)mpix(*p), n_cu) : mfma_grid(p->nb_pad / 16, n_cu);
  DeviceTables& d = p->d;
  if ((st = upload(&d.bin3, p->bin3.data(), p->bin3.size())) != PB3_OK) return st;
  if ((st = upload(&d.modes, p->modes.data(), p->modes.size())) != PB3_OK) return st;
  if ((st = upload(&d.chunk, p->chunks.data(), p->chunks.size())) != PB3_OK) return st;
  if ((st = upload(&d.chunk_first, p->chunk_first.data(), p->chunk_first.size())) != PB3_OK) return st;
  if ((st = upload(&d.geom, p->geom.data(), p->geom.size())) != PB3_OK) return st;
  if ((st = upload(&d.trip_all, p->trip_all.data(), p->trip_all.size())) != PB3_OK) return st;
  const int Ng[3] = {p->Nx, p->Ny, p->Nz}, Mg[3] = {p->Mx, p->My, p->Mz};
  for (int a = 0; a < 3; ++a) {
    if ((st = upload_twiddles_f(&d.tw_n[a], Ng[a])) != PB3_OK) return st;
    if ((st = upload_twiddles_f(&d.tw_m[a], Mg[a])) != PB3_OK) return st;
    if ((st = upload_twiddles_d(&d.tw_m_d[a], Mg[a])) != PB3_OK) return st;
  }
  // FP32 inverse-pass tiles
  int tbx = tile_width_x(p->Mx, false), tbz = tile_width_z(p->Mz, false);
  if (tbx <= 0 || tbz <= 0) {
    set_error("contraction grid not implemented");
    return PB3_EUNSUPPORTED;
  }
  std::vector<BinTile> vx, vy, vz;
  build_tiles(*p, tbx, tbz, vx, vy, vz);
  std::vector<BinTile> all(vx);
  all.insert(all.end(), vy.begin(), vy.end());
  all.insert(all.end(), vz.begin(), vz.end());
  if ((st = upload(&d.tiles, all.data(), all.size())) != PB3_OK) return st;
  p->tx = TileSet{d.tiles, (int)vx.size(), tbx};
  {
    // the inverse-x tiles are in bin order: per bin, the index of its first
    std::vector<int32_t> xf(p->nb + 1, (int32_t)vx.size());
    for (int t = (int)vx.size() - 1; t >= 0; --t) xf[vx[t].bin] = t;
    for (int b = p->nb - 1; b >= 0; --b) xf[b] = std::min(xf[b], xf[b + 1]);
    if ((st = upload(&d.xtile_first, xf.data(), xf.size())) != PB3_OK) return st;
  }
  p->ty = TileSet{d.tiles + vx.size(), (int)vy.size(), tbx};
  p->tz = TileSet{d.tiles + vx.size() + vy.size(), (int)vz.size(), tbz};
  // power normalisation V / (N_pix^2 N_b)
  const double V = p->Lx * p->Ly * p->Lz;
  const double n3 = (double)p->Nx * p->Ny * p->Nz;
  std::vector<double> pks(p->nb);
  for (int b = 0; b < p->nb; ++b) pks[b] = V / (n3 * n3 * (double)p->nmodes[b]);
  if ((st = upload(&d.pk_scale, pks.data(), pks.size())) != PB3_OK) return st;
  // triangle counts in FP64 on the contraction grid
  std::vector<double> raw;
  const int n_cand = (int)(p->trip_all.size() / 3);
  const std::string ckey = tune_key(p);
  if (!(p->flags & PB3_FLAG_POWER_ONLY) && !cache_read(ckey, "counts", raw, (size_t)n_cand)) {
    if ((st = compute_counts_fp64(*p, raw)) != PB3_OK) return st;
    cache_write(ckey, "counts", raw);
  }
  p->trip.clear();
  p->counts.clear();
  std::vector<int32_t> map, map_ab;
  std::vector<double> fac;
  const double m3 = (double)p->Mx * p->My * p->Mz;
  const double scale = V * V * (m3 * m3) / (n3 * n3 * n3);
  for (int t = 0; t < n_cand; ++t) {
    double T = std::nearbyint(raw[t]);
    if (std::fabs(raw[t] - T) > 1e-3) {
      set_error("triangle count not integral (" + std::to_string(raw[t]) + ")");
      return PB3_EDEVICE;
    }
    if (T <= 0) {
      if (p->flags & PB3_FLAG_STRICT) {
        set_error("a triangle-valid triplet has no closed triangle on the grid");
        return PB3_EINVAL;
      }
      continue;
    }
    for (int k = 0; k < 3; ++k) p->trip.push_back(p->trip_all[3 * t + k]);
    p->counts.push_back(T);
    const int a = p->trip_all[3 * t], b = p->trip_all[3 * t + 1], c = p->trip_all[3 * t + 2];
    int loc = mfma_locate(false, p->nb, a, b, c);
    if (loc < 0 || loc >= p->part_len) {
      set_error("internal: triplet not covered by the contraction tiles");
      return PB3_EDEVICE;
    }
    map.push_back(loc);
    if (p->part_len_ab > 0) {
      loc = mfma_locate(true, p->nb, a, b, c);
      if (loc < 0 || loc >= p->part_len_ab) {
        set_error("internal: triplet not covered by the column-field contraction tiles");
        return PB3_EDEVICE;
      }
      map_ab.push_back(loc);
    }
    fac.push_back(scale / T);
  }
  if ((st = upload(&d.out_map, map.data(), map.size())) != PB3_OK) return st;
  {
    // the inverse map: the reduction's slice sums are stored in triplet order
    std::vector<int32_t> inv((size_t)p->part_len, -1);
    for (size_t t = 0; t < map.size(); ++t) inv[(size_t)map[t]] = (int32_t)t;
    if ((st = upload(&d.out_inv, inv.data(), inv.size())) != PB3_OK) return st;
  }
  if (!map_ab.empty() && (st = upload(&d.out_map_ab, map_ab.data(), map_ab.size())) != PB3_OK) return st;
  if ((st = upload(&d.inv_counts, fac.data(), fac.size())) != PB3_OK) return st;
  if (p->lmax > 0) {
    const int ne = p->lmax / 2 + 1, nt = (int)(p->trip.size() / 3);
    std::vector<int32_t> mt, mm(nt);
    std::vector<double> mf;
    for (int l = 0; l < ne; ++l)
      for (int t = 0; t < nt; ++t) {
        mt.push_back(p->trip[3 * t]);
        mt.push_back(p->trip[3 * t + 1]);
        mt.push_back(l * p->nb + p->trip[3 * t + 2]);
        mf.push_back((4 * l + 1) * fac[t]);  // (2 ell + 1) with ell = 2 l
      }
    for (int t = 0; t < nt; ++t) mm[t] = t;
    if ((st = upload(&d.pml_inv, p->pml_inv.data(), p->pml_inv.size())) != PB3_OK) return st;
    if ((st = upload(&d.ml_trips, mt.data(), mt.size())) != PB3_OK) return st;
    if ((st = upload(&d.ml_fac, mf.data(), mf.size())) != PB3_OK) return st;
    if ((st = upload(&d.ml_map, mm.data(), mm.size())) != PB3_OK) return st;
    if (p->flags & PB3_FLAG_BK_FISHER) {
      const std::string mkey = ckey + " lmax" + std::to_string(p->lmax);
      if (!cache_read(mkey, "mixing", p->bk_mix, (size_t)nt * ne * ne)) {
        if ((st = compute_bk_mixing(*p, p->bk_mix)) != PB3_OK) return st;
        cache_write(mkey, "mixing", p->bk_mix);
      }
      if ((st = upload(&d.bk_mix, p->bk_mix.data(), p->bk_mix.size())) != PB3_OK) return st;
    }
  }
  if (p->flags & PB3_FLAG_STAGE_TIMING) {
    p->ev.assign((size_t)pb3_plan::kTimingRing * ST_COUNT * 2, nullptr);
    p->ev_used.assign((size_t)pb3_plan::kTimingRing * ST_COUNT, 0);
    for (auto& ev : p->ev) {
      e = hipEventCreate(&ev);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
  }
  p->device = true;
  if ((p->flags & PB3_FLAG_AUTOTUNE) && !(p->flags & PB3_FLAG_POWER_ONLY)) return autotune(p, n_cu);
  return PB3_OK;
}

// run one stage, bracketed by events when timing is on
template <typename F> static pb3_status stage(pb3_plan* p, int id, hipStream_t s, const char* name, F&& fn) {
  const bool timed = !p->ev.empty();
  const size_t slot = (size_t)(p->n_calls % pb3_plan::kTimingRing) * ST_COUNT + id;
  if (timed) {
    hipError_t e = hipEventRecord(p->ev[2 * slot], s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  }
  hipError_t e = fn();
  if (e != hipSuccess) return hip_fail(e, name);
  if (timed) {
    e = hipEventRecord(p->ev[2 * slot + 1], s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    p->ev_used[slot] = 1;
  }
  return PB3_OK;
}

static pb3_status check_ready(pb3_plan* p) {
  if (!p) {
    set_error("null plan");
    return PB3_EINVAL;
  }
  if (!p->device) {
    set_error("plan has no device state (created with PB3_FLAG_HOST_ONLY)");
    return PB3_EINVAL;
  }
  int dev = -1;
  hipGetDevice(&dev);
  if (dev != p->device_id) {
    set_error("plan was created on another device");
    return PB3_EINVAL;
  }
  return ensure_workspace(p);
}

// The launch sequence of one plan over the jobs of x (all stages on
// stream s).  wrap(stage, name, fn) runs fn, optionally timed.
template <typename W>
static pb3_status enqueue_w(const pb3_plan& p, const Exec& x, bool do_pk, bool do_bk, pb3_precision prec,
                            hipStream_t s, W&& wrap) {
  pb3_status st;
  // with both spectra, the power spectrum's per-bin sums run in the reduction's launch; for
  // unweighted plans the inverse x pass takes the sums over the modes it gathers anyway
  const bool merge = do_pk && do_bk && !p.trip.empty();
  const bool fold = power_folded(p, do_pk, do_bk);
  if ((st = wrap(ST_FWD_Z, "fwd_z", [&] { return launch_fwd_z(p, x, s); })) != PB3_OK) return st;
  if ((st = wrap(ST_FWD_Y, "fwd_y", [&] { return launch_fwd_y(p, x, s); })) != PB3_OK) return st;
  if ((st = wrap(ST_FWD_X, "fwd_x", [&] { return launch_fwd_x(p, x, s); })) != PB3_OK) return st;
  if (do_pk && !fold) {
    if ((st = wrap(ST_POWER, "power", [&] { return launch_power(p, x, s, !merge); })) != PB3_OK) return st;
  }
  if (do_bk) {
    if ((st = wrap(ST_INV_X, "inv_x", [&] { return launch_inv_x(p, x, s, fold ? x.ws.ppart : nullptr); })) !=
        PB3_OK)
      return st;
    if ((st = wrap(ST_INV_Y, "inv_y", [&] { return launch_inv_y(p, x, s); })) != PB3_OK) return st;
    if (p.fused) {
      if ((st = wrap(ST_CONTRACT, "contract",
                     [&] { return launch_zcontract(p, x, prec == PB3_MIXED_BF16X3, s); })) != PB3_OK)
        return st;
    } else {
      if ((st = wrap(ST_INV_Z, "inv_z", [&] { return launch_inv_z(p, x, s); })) != PB3_OK) return st;
      if ((st = wrap(ST_CONTRACT, "contract", [&] { return launch_contract(p, x, prec, s); })) != PB3_OK) return st;
    }
    if ((st = wrap(ST_REDUCE, "reduce", [&] { return launch_reduce(p, x, s, merge, fold); })) != PB3_OK) return st;
  }
  return PB3_OK;
}

pb3_status enqueue(const pb3_plan& p, const Exec& x, bool do_pk, bool do_bk, pb3_precision prec, hipStream_t s) {
  return enqueue_w(p, x, do_pk, do_bk, prec, s, [](int, const char* name, auto&& fn) -> pb3_status {
    hipError_t e = fn();
    return e == hipSuccess ? PB3_OK : hip_fail(e, name);
  });
}

// kernel launches of one enqueue (for reporting)
int launches_per_sequence(const pb3_plan& p, bool do_pk, bool do_bk) {
  int n = 3;
  if (do_pk && !power_folded(p, do_pk, do_bk)) n += (do_bk && !p.trip.empty()) ? 1 : 2;
  if (do_bk) {
    n += 2 + 2;
    if (p.fused) n += 1;
    else n += 1 + ((p.nb_pad / 16) >= 2 ? 3 : 1);
  }
  return n;
}

// Field pointers: the forward z pass reads pairs of float32 values.
pb3_status check_field_ptr(const void* p, const char* what) {
  if (((uintptr_t)p & 7u) != 0) {
    set_error(std::string(what) + " must be 8-byte aligned");
    return PB3_EINVAL;
  }
  return PB3_OK;
}

pb3_status check_prec(pb3_precision prec) {
  if (prec != PB3_FP32 && prec != PB3_MIXED_BF16X3) {
    set_error("unknown precision");
    return PB3_EINVAL;
  }
  return PB3_OK;
}

static pb3_status run(pb3_plan* p, const float* delta, double* pk, double* bk, pb3_precision prec, hipStream_t s) {
  pb3_status st = check_ready(p);
  if (st != PB3_OK) return st;
  if (!delta || (!pk && !bk)) {
    set_error("null device pointer");
    return PB3_EINVAL;
  }
  if ((st = check_field_ptr(delta, "delta")) != PB3_OK) return st;
  if (bk && (p->flags & PB3_FLAG_POWER_ONLY)) {
    set_error("plan was created with PB3_FLAG_POWER_ONLY (no bispectrum tables)");
    return PB3_EINVAL;
  }
  if ((st = check_prec(prec)) != PB3_OK) return st;
  if (!p->ev.empty()) {
    size_t slot = (size_t)(p->n_calls % pb3_plan::kTimingRing) * ST_COUNT;
    std::fill(p->ev_used.begin() + slot, p->ev_used.begin() + slot + ST_COUNT, 0);
  }
  p->last_stream = s;
  Exec x;
  x.ws = p->ws;
  x.io.delta[0] = delta;
  x.io.pk[0] = pk;
  x.io.bk[0] = bk;
  st = enqueue_w(*p, x, pk != nullptr, bk != nullptr, prec, s,
                 [&](int id, const char* name, auto&& fn) { return stage(p, id, s, name, fn); });
  if (st != PB3_OK) return st;
  p->last_prec = prec;
  ++p->n_calls;
  return PB3_OK;
}

}  // namespace pb3

using namespace pb3;

extern "C" {

pb3_status pb3_plan_create(const int grid[3], const double box[3], const double* edges, int n_edges, unsigned flags,
                           pb3_plan** out) {
  if (!out) {
    set_error("null output pointer");
    return PB3_EINVAL;
  }
  *out = nullptr;
  pb3_plan* p = new (std::nothrow) pb3_plan();
  if (!p) {
    set_error("host allocation failed");
    return PB3_ENOMEM;
  }
  pb3_status st = build_host(p, grid, box, edges, n_edges, flags);
  if (st == PB3_OK && !(flags & PB3_FLAG_HOST_ONLY)) st = build_device(p);
  if (st != PB3_OK) {
    free_device(p);
    delete p;
    return st;
  }
  *out = p;
  return PB3_OK;
}

pb3_status pb3_plan_destroy(pb3_plan* plan) {
  if (!plan) return PB3_OK;
  free_device(plan);
  delete plan;
  return PB3_OK;
}

size_t pb3_plan_workspace_bytes(const pb3_plan* plan) { return plan ? workspace_bytes(plan) : 0; }

pb3_status pb3_plan_bind_workspace(pb3_plan* plan, void* dev, size_t bytes) {
  if (!plan || !dev) {
    set_error("null argument");
    return PB3_EINVAL;
  }
  size_t need = workspace_bytes(plan);
  if (bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return PB3_ENOMEM;
  }
  if (((uintptr_t)dev) % 256) {
    set_error("workspace must be 256-byte aligned");
    return PB3_EINVAL;
  }
  if (plan->ws.owned && plan->ws.base) hipFree(plan->ws.base);
  carve_workspace(plan, dev, bytes, false);
  return PB3_OK;
}

int pb3_n_bins(const pb3_plan* plan) { return plan ? plan->nb : 0; }
int pb3_n_triplets(const pb3_plan* plan) { return plan ? (int)(plan->trip.size() / 3) : 0; }
int pb3_grid(const pb3_plan* plan) { return plan ? plan->Nx : 0; }
int pb3_contract_grid(const pb3_plan* plan) { return plan ? plan->Mx : 0; }

pb3_status pb3_grid3(const pb3_plan* plan, int* grid_out, int* contract_out) {
  if (!plan || (!grid_out && !contract_out)) {
    set_error("null argument");
    return PB3_EINVAL;
  }
  if (grid_out) {
    grid_out[0] = plan->Nx;
    grid_out[1] = plan->Ny;
    grid_out[2] = plan->Nz;
  }
  if (contract_out) {
    contract_out[0] = plan->Mx;
    contract_out[1] = plan->My;
    contract_out[2] = plan->Mz;
  }
  return PB3_OK;
}

pb3_status pb3_plan_launch_shape(const pb3_plan* plan, int* fused_out, int* contract_wgs_out, int* tuned_out) {
  if (!plan) {
    set_error("null plan");
    return PB3_EINVAL;
  }
  if (fused_out) *fused_out = plan->fused ? 1 : 0;
  if (contract_wgs_out) *contract_wgs_out = plan->contract_wgs;
  if (tuned_out) *tuned_out = plan->tuned;
  return PB3_OK;
}

pb3_status pb3_get_bins(const pb3_plan* plan, double* edges_kf_out, double* kmean_out, int64_t* n_modes_out) {
  if (!plan) {
    set_error("null plan");
    return PB3_EINVAL;
  }
  if (edges_kf_out) std::copy(plan->edges.begin(), plan->edges.end(), edges_kf_out);
  if (kmean_out) std::copy(plan->kmean.begin(), plan->kmean.end(), kmean_out);
  if (n_modes_out) std::copy(plan->nmodes.begin(), plan->nmodes.end(), n_modes_out);
  return PB3_OK;
}

pb3_status pb3_get_triplets(const pb3_plan* plan, int32_t* abc_out) {
  if (!plan || !abc_out) {
    set_error("null argument");
    return PB3_EINVAL;
  }
  std::copy(plan->trip.begin(), plan->trip.end(), abc_out);
  return PB3_OK;
}

pb3_status pb3_norm(const pb3_plan* plan, int64_t* n_modes_out, double* counts_out) {
  if (!plan) {
    set_error("null plan");
    return PB3_EINVAL;
  }
  if (!plan->device) {
    set_error("triangle counts need a device plan");
    return PB3_EINVAL;
  }
  if (n_modes_out) std::copy(plan->nmodes.begin(), plan->nmodes.end(), n_modes_out);
  if (counts_out) std::copy(plan->counts.begin(), plan->counts.end(), counts_out);
  return PB3_OK;
}

pb3_status pb3_power(pb3_plan* plan, const float* delta_dev, double* pk_dev, void* stream) {
  if (!pk_dev) {
    set_error("null output pointer");
    return PB3_EINVAL;
  }
  return run(plan, delta_dev, pk_dev, nullptr, PB3_FP32, (hipStream_t)stream);
}

pb3_status pb3_bispectrum(pb3_plan* plan, const float* delta_dev, double* bk_dev, pb3_precision prec, void* stream) {
  if (!bk_dev) {
    set_error("null output pointer");
    return PB3_EINVAL;
  }
  return run(plan, delta_dev, nullptr, bk_dev, prec, (hipStream_t)stream);
}

pb3_status pb3_polyspectra(pb3_plan* plan, const float* delta_dev, double* pk_dev, double* bk_dev, pb3_precision prec,
                           void* stream) {
  return run(plan, delta_dev, pk_dev, bk_dev, prec, (hipStream_t)stream);
}

pb3_status pb3_window_normalize(const pb3_plan* plan, const float* w_dev, double* pk_dev, double* bk_dev,
                                double* scratch_dev, void* stream) {
  if (!plan || !w_dev || !scratch_dev || (!pk_dev && !bk_dev)) {
    set_error("null argument");
    return PB3_EINVAL;
  }
  if (!plan->device) {
    set_error("plan has no device state (created with PB3_FLAG_HOST_ONLY)");
    return PB3_EINVAL;
  }
  const long n = (long)npix(*plan);
  hipError_t e = launch_window(n, w_dev, pk_dev, plan->nb, bk_dev, (int)(plan->trip.size() / 3), scratch_dev,
                               (hipStream_t)stream);
  return e == hipSuccess ? PB3_OK : hip_fail(e, "window normalisation");
}

size_t pb3_masked_power_workspace_bytes(const pb3_plan* plan) { return plan ? masked_workspace_bytes(*plan) : 0; }

size_t pb3_bispectrum_linear_workspace_bytes(const pb3_plan* plan, int n_sim) {
  return (plan && n_sim >= 1) ? linear_workspace_bytes(*plan, n_sim) : 0;
}

pb3_status pb3_bispectrum_linear(pb3_plan* plan, const float* data_dev, const float* const* sims_dev, int n_sim,
                                 double* bk_dev, pb3_precision prec, void* workspace_dev, size_t workspace_bytes_,
                                 void* stream) {
  if (!plan || !data_dev || !sims_dev || !bk_dev || !workspace_dev) {
    set_error("null argument");
    return PB3_EINVAL;
  }
  if (check_field_ptr(data_dev, "data") != PB3_OK) return PB3_EINVAL;
  for (int i = 0; i < n_sim; ++i)
    if (sims_dev[i] && check_field_ptr(sims_dev[i], "each simulation") != PB3_OK) return PB3_EINVAL;
  if (!plan->device) {
    set_error("plan has no device state (created with PB3_FLAG_HOST_ONLY)");
    return PB3_EINVAL;
  }
  if (plan->flags & PB3_FLAG_POWER_ONLY) {
    set_error("plan was created with PB3_FLAG_POWER_ONLY (no bispectrum tables)");
    return PB3_EINVAL;
  }
  if (plan->weighted) {
    set_error("the linear term takes unit weights (plan has pb3_plan_set_weights)");
    return PB3_EINVAL;
  }
  if (n_sim < 1) {
    set_error("at least one field is needed for the linear term");
    return PB3_EINVAL;
  }
  for (int i = 0; i < n_sim; ++i)
    if (!sims_dev[i]) {
      set_error("null field");
      return PB3_EINVAL;
    }
  pb3_status st = check_prec(prec);
  if (st != PB3_OK) return st;
  const size_t need = linear_workspace_bytes(*plan, n_sim);
  if (workspace_bytes_ < need || ((uintptr_t)workspace_dev) % 256) {
    set_error("workspace too small or not 256-byte aligned: need " + std::to_string(need) + " bytes");
    return PB3_ENOMEM;
  }
  int dev = -1;
  hipGetDevice(&dev);
  if (dev != plan->device_id) {
    set_error("plan was created on another device");
    return PB3_EINVAL;
  }
  return run_bispectrum_linear(*plan, data_dev, sims_dev, n_sim, bk_dev, prec, workspace_dev, (hipStream_t)stream);
}

pb3_status pb3_masked_power(pb3_plan* plan, const float* data_dev, const float* window_dev,
                            const float* const* grfs_dev, int n_grf, double* pk_dev, double* fisher_dev,
                            void* workspace_dev, size_t workspace_bytes_, void* stream) {
  if (!plan || !data_dev || !window_dev || !grfs_dev || !pk_dev || !workspace_dev) {
    set_error("null argument");
    return PB3_EINVAL;
  }
  if (check_field_ptr(data_dev, "data") != PB3_OK || check_field_ptr(window_dev, "window") != PB3_OK)
    return PB3_EINVAL;
  for (int i = 0; i < n_grf; ++i)
    if (grfs_dev[i] && check_field_ptr(grfs_dev[i], "each random field") != PB3_OK) return PB3_EINVAL;
  if (!plan->device) {
    set_error("plan has no device state (created with PB3_FLAG_HOST_ONLY)");
    return PB3_EINVAL;
  }
  if (plan->Mx != plan->Nx || plan->My != plan->Ny || plan->Mz != plan->Nz) {
    set_error("the masked power spectrum needs the full grid (create the plan with PB3_FLAG_FULL_GRID)");
    return PB3_EINVAL;
  }
  if (plan->weighted) {
    set_error("the masked power spectrum takes unit weights (plan has pb3_plan_set_weights)");
    return PB3_EINVAL;
  }
  if (n_grf < 1) {
    set_error("at least one random field is needed");
    return PB3_EINVAL;
  }
  for (int i = 0; i < n_grf; ++i)
    if (!grfs_dev[i]) {
      set_error("null random field");
      return PB3_EINVAL;
    }
  if (plan->nb > 48) {
    set_error("the masked power spectrum is implemented for at most 48 bins");
    return PB3_EUNSUPPORTED;
  }
  if (plan->Nx != plan->Ny || plan->Ny != plan->Nz || plan->aniso) {
    set_error("the masked power spectrum is implemented for cubic grids and boxes");
    return PB3_EUNSUPPORTED;
  }
  if (workspace_bytes_ < masked_workspace_bytes(*plan) || ((uintptr_t)workspace_dev) % 256) {
    set_error("workspace too small or not 256-byte aligned: need " +
              std::to_string(masked_workspace_bytes(*plan)) + " bytes");
    return PB3_ENOMEM;
  }
  int dev = -1;
  hipGetDevice(&dev);
  if (dev != plan->device_id) {
    set_error("plan was created on another device");
    return PB3_EINVAL;
  }
  return run_masked_power(*plan, data_dev, window_dev, grfs_dev, n_grf, pk_dev, fisher_dev, workspace_dev,
                          (hipStream_t)stream);
}

int pb3_n_ell(const pb3_plan* plan) { return plan ? plan->lmax / 2 + 1 : 0; }

pb3_status pb3_multipole_mixing(const pb3_plan* plan, double* mix_out) {
  if (!plan || !mix_out) {
    set_error("null argument");
    return PB3_EINVAL;
  }
  if (!(plan->flags & PB3_FLAG_BK_FISHER) || plan->bk_mix.empty()) {
    set_error("the plan has no bispectrum multipole Fisher matrix (device plan with PB3_FLAG_BK_FISHER)");
    return PB3_EINVAL;
  }
  std::copy(plan->bk_mix.begin(), plan->bk_mix.end(), mix_out);
  return PB3_OK;
}

int pb3_weights_table_len(const pb3_plan* plan) { return (plan && !plan->aniso) ? (int)plan->thr[plan->nb] : 0; }

pb3_status pb3_plan_set_weights(pb3_plan* plan, int window_order, const double* pfid, int n_pfid, double nbar) {
  if (!plan || !plan->device) {
    set_error("weights need a device plan");
    return PB3_EINVAL;
  }
  pb3_plan* p = plan;
  if (p->weighted) {
    set_error("weights are already set on this plan");
    return PB3_EINVAL;
  }
  if (p->aniso) {
    set_error("weights take P_fid over integer |n|^2: a box with equal sides is needed");
    return PB3_EUNSUPPORTED;
  }
  if (p->flags & PB3_FLAG_BK_FISHER) {
    set_error("weights are not implemented with the bispectrum multipole Fisher matrix (PB3_FLAG_BK_FISHER)");
    return PB3_EUNSUPPORTED;
  }
  if (window_order < 0 || window_order > 3 || !(nbar >= 0.0)) {
    set_error("window order must be 0..3 and nbar >= 0");
    return PB3_EINVAL;
  }
  const int need = (int)p->thr[p->nb];  // first |n|^2 above the top bin
  if (pfid) {
    if (n_pfid < need) {
      set_error("P_fid table too short: need " + std::to_string(need) + " entries (|n|^2 = 0.." +
                std::to_string(need - 1) + ")");
      return PB3_EINVAL;
    }
    for (int j = 1; j < need; ++j)
      if (!(pfid[j] > 0.0)) {
        set_error("P_fid must be positive at every binned |n|^2");
        return PB3_EINVAL;
      }
  }
  if (nbar > 0.0 && !pfid && !(p->flags & PB3_FLAG_POWER_ONLY)) {
    set_error("the bispectrum shot-noise term needs a P_fid table (it serves as the power model)");
    return PB3_EINVAL;
  }
  const double V = p->Lx * p->Ly * p->Lz, n3 = (double)p->Nx * p->Ny * p->Nz;
  // 1D window inverse per component (axes x, y, z back to back, k in
  // [-N_i/2, N_i/2] at off[i] + k) and 1 / P_fid per |n|^2
  const int Ng[3] = {p->Nx, p->Ny, p->Nz};
  const int off[3] = {p->Nx / 2, p->Nx + 1 + p->Ny / 2, p->Nx + p->Ny + 2 + p->Nz / 2};
  std::vector<double> winv((size_t)p->Nx + p->Ny + p->Nz + 3, 1.0);
  for (int a = 0; a < 3; ++a)
    for (int k = -Ng[a] / 2; k <= Ng[a] / 2; ++k) {
      if (window_order == 0 || k == 0) continue;
      const double x = M_PI * k / Ng[a];
      winv[off[a] + k] = std::pow(x / std::sin(x), window_order);
    }
  std::vector<double> pf(p->lut_len, 1.0);
  if (pfid)
    for (int j = 0; j < p->lut_len && j < n_pfid; ++j) pf[j] = pfid[j] > 0.0 ? pfid[j] : 1.0;
  std::vector<float> winv_f(winv.begin(), winv.end()), pinv_f(p->lut_len);
  std::vector<double> pinv_d(p->lut_len);
  for (int j = 0; j < p->lut_len; ++j) {
    pinv_d[j] = 1.0 / pf[j];
    pinv_f[j] = (float)pinv_d[j];
  }
  // power: per-mode weight 1 / (m^2 P_fid^2) and the weighted Fisher per bin
  const int nb = p->nb, ne = p->lmax / 2 + 1;
  std::vector<double> mw(p->modes.size()), fish(nb, 0.0), msum((size_t)nb * ne * ne, 0.0);
  for (int c = 0; c < p->n_chunks; ++c) {
    const int b = p->chunks[3 * c];
    for (int i = p->chunks[3 * c + 1]; i < p->chunks[3 * c + 2]; ++i) {
      const int32_t m = p->modes[i];
      const int idx = m & 0x7fffffff, w = m < 0 ? 1 : 2;
      const int kz = idx % p->Kz, cxy = idx / p->Kz;
      const int ky = cxy % p->Lcy - p->Kcy, kx = cxy / p->Lcy - p->Kcx;
      const int64_t n2 = (int64_t)kx * kx + (int64_t)ky * ky + (int64_t)kz * kz;
      const double wi = winv[off[0] + kx] * winv[off[1] + ky] * winv[off[2] + kz];
      const double q = 1.0 / pf[n2];
      mw[i] = wi * wi * q * q;
      fish[b] += w * q * q;
      if (ne > 1) {
        const double m2 = n2 > 0 ? (double)kz * kz / (double)n2 : 0.0;
        const double L[3] = {1.0, 1.5 * m2 - 0.5, (35.0 * m2 * m2 - 30.0 * m2 + 3.0) / 8.0};
        for (int a = 0; a < ne; ++a)
          for (int bb = 0; bb < ne; ++bb) msum[((size_t)b * ne + a) * ne + bb] += w * q * q * L[a] * L[bb];
      }
    }
  }
  std::vector<double> pks(nb);
  for (int b = 0; b < nb; ++b) pks[b] = V / (n3 * n3 * fish[b]);
  std::vector<double> pml(p->pml_inv);
  if (ne > 1) {  // weighted discrete Fisher of the power multipoles
    const double sc = V / (n3 * n3);
    for (int b = 0; b < nb; ++b) {
      double a[3][6] = {};
      for (int i = 0; i < ne; ++i) {
        for (int j = 0; j < ne; ++j) a[i][j] = msum[((size_t)b * ne + i) * ne + j];
        a[i][ne + i] = 1.0;
      }
      for (int k = 0; k < ne; ++k) {
        int pr = k;
        for (int r = k + 1; r < ne; ++r)
          if (std::fabs(a[r][k]) > std::fabs(a[pr][k])) pr = r;
        for (int c = 0; c < 2 * ne; ++c) std::swap(a[k][c], a[pr][c]);
        const double dd = a[k][k];
        for (int c = 0; c < 2 * ne; ++c) a[k][c] /= dd;
        for (int r = 0; r < ne; ++r)
          if (r != k) {
            const double f = a[r][k];
            for (int c = 0; c < 2 * ne; ++c) a[r][c] -= f * a[k][c];
          }
      }
      for (int i = 0; i < ne; ++i)
        for (int j = 0; j < ne; ++j) pml[((size_t)b * ne + i) * ne + j] = sc * a[i][ne + j];
    }
  }
  // Everything that can fail on allocation comes first, into new tables;
  // the plan changes only once all of it has succeeded.
  pb3_status st;
  DeviceTables& d = p->d;
  float *t_win = nullptr, *t_pinv = nullptr;
  double *t_pinv_d = nullptr, *t_mw = nullptr, *t_bias = nullptr;
  auto drop = [&](pb3_status r) {
    for (void* q : {(void*)t_win, (void*)t_pinv, (void*)t_pinv_d, (void*)t_mw, (void*)t_bias})
      if (q) hipFree(q);
    return r;
  };
  if ((window_order != 0 && (st = upload(&t_win, winv_f.data(), winv_f.size())) != PB3_OK) ||
      (pfid && (st = upload(&t_pinv, pinv_f.data(), pinv_f.size())) != PB3_OK) ||
      (pfid && (st = upload(&t_pinv_d, pinv_d.data(), pinv_d.size())) != PB3_OK) ||
      (st = upload(&t_mw, mw.data(), mw.size())) != PB3_OK)
    return drop(st);
  const bool with_bk = !(p->flags & PB3_FLAG_POWER_ONLY) && !p->trip.empty();
  const int nt = (int)(p->trip.size() / 3);
  std::vector<double> fac, bias, counts(p->counts);
  if (with_bk) {
    // bispectrum: weighted triangle sums N_0 = sum 1/(P1 P2 P3), the shot-noise sums
    std::vector<double> n0, q;
    d.pfid_inv_d = t_pinv_d;  // the count pass reads the weights from the plan's tables
    st = compute_counts_fp64(*p, n0, nbar > 0.0 ? &q : nullptr);
    d.pfid_inv_d = nullptr;
    if (st != PB3_OK) return drop(st);
    const double m3 = (double)p->Mx * p->My * p->Mz;
    const double scale = V * V * (m3 * m3) / (n3 * n3 * n3);
    for (int t = 0, kept = 0; t < (int)(p->trip_all.size() / 3) && kept < nt; ++t) {
      if (p->trip_all[3 * t] != p->trip[3 * kept] || p->trip_all[3 * t + 1] != p->trip[3 * kept + 1] ||
          p->trip_all[3 * t + 2] != p->trip[3 * kept + 2])
        continue;  // dropped (no closed triangle)
      fac.push_back(scale / n0[t]);
      bias.push_back(nbar > 0.0 ? q[t] / n0[t] / nbar - 2.0 / (nbar * nbar) : 0.0);
      counts[kept] = n0[t];
      ++kept;
    }
    if ((int)fac.size() != nt) {
      set_error("internal: weighted triangle sums do not match the triplet list");
      return drop(PB3_EDEVICE);
    }
    if (nbar > 0.0 && (st = upload(&t_bias, bias.data(), bias.size())) != PB3_OK) return drop(st);
  }
  // commit
  hipError_t e = hipMemcpy(d.pk_scale, pks.data(), sizeof(double) * nb, hipMemcpyHostToDevice);
  if (e == hipSuccess && ne > 1)
    e = hipMemcpy(d.pml_inv, pml.data(), sizeof(double) * pml.size(), hipMemcpyHostToDevice);
  std::vector<double> mf;
  if (e == hipSuccess && with_bk) {
    e = hipMemcpy(d.inv_counts, fac.data(), sizeof(double) * nt, hipMemcpyHostToDevice);
    if (e == hipSuccess && p->lmax > 0) {
      for (int l = 0; l < ne; ++l)
        for (int t = 0; t < nt; ++t) mf.push_back((4 * l + 1) * fac[t]);
      e = hipMemcpy(d.ml_fac, mf.data(), sizeof(double) * mf.size(), hipMemcpyHostToDevice);
    }
  }
  if (e != hipSuccess) return drop(hip_fail(e, "hipMemcpy"));
  d.win_inv = t_win;
  d.pfid_inv = t_pinv;
  d.pfid_inv_d = t_pinv_d;
  d.mode_w = t_mw;
  if (t_bias) d.bk_bias = t_bias;
  p->pfid = std::move(pf);
  p->pml_inv = std::move(pml);
  p->counts = std::move(counts);
  p->window_order = window_order;
  p->nbar = nbar;
  p->pk_shift = nbar > 0.0 ? 1.0 / nbar : 0.0;
  p->weighted = true;
  return PB3_OK;
}

size_t pb3_multipoles_workspace_bytes(const pb3_plan* plan) {
  return (plan && plan->lmax > 0) ? multipoles_workspace_bytes(*plan) : 0;
}

pb3_status pb3_multipoles(pb3_plan* plan, const float* delta_dev, double* pk_dev, double* bk_dev, pb3_precision prec,
                          void* workspace_dev, size_t workspace_bytes_, void* stream) {
  if (!plan || !delta_dev || (!pk_dev && !bk_dev) || !workspace_dev) {
    set_error("null argument");
    return PB3_EINVAL;
  }
  if (check_field_ptr(delta_dev, "delta") != PB3_OK) return PB3_EINVAL;
  if (!plan->device || plan->lmax == 0) {
    set_error("multipoles need a device plan created with PB3_FLAG_LMAX2 or PB3_FLAG_LMAX4");
    return PB3_EINVAL;
  }
  if (bk_dev && (plan->flags & PB3_FLAG_POWER_ONLY)) {
    set_error("plan was created with PB3_FLAG_POWER_ONLY (no bispectrum tables)");
    return PB3_EINVAL;
  }
  if (workspace_bytes_ < multipoles_workspace_bytes(*plan) || ((uintptr_t)workspace_dev) % 256) {
    set_error("workspace too small or not 256-byte aligned: need " +
              std::to_string(multipoles_workspace_bytes(*plan)) + " bytes");
    return PB3_ENOMEM;
  }
  int dev = -1;
  hipGetDevice(&dev);
  if (dev != plan->device_id) {
    set_error("plan was created on another device");
    return PB3_EINVAL;
  }
  pb3_status pst = check_prec(prec);
  if (pst != PB3_OK) return pst;
  return run_multipoles(*plan, delta_dev, pk_dev, bk_dev, prec, workspace_dev, (hipStream_t)stream);
}

static const char* kStageNames[ST_COUNT] = {"fwd_z", "fwd_y", "fwd_x",    "power", "inv_x",
                                            "inv_y", "inv_z", "contract", "reduce"};

const char* pb3_stage_name(int stage) {
  if (stage < 0 || stage >= ST_COUNT) return "";
  return kStageNames[stage];
}

pb3_status pb3_stage_times(pb3_plan* plan, float* ms_out, int* counts_out, int capacity, int* n_out) {
  if (!plan || !ms_out) {
    set_error("null argument");
    return PB3_EINVAL;
  }
  if (plan->ev.empty()) {
    set_error("plan was not created with PB3_FLAG_STAGE_TIMING");
    return PB3_EINVAL;
  }
  const int n = std::min(capacity, (int)ST_COUNT);
  const long calls = std::min<long>(plan->n_calls, pb3_plan::kTimingRing);
  for (int i = 0; i < n; ++i) {
    double sum = 0.0;
    int cnt = 0;
    for (long c = 0; c < calls; ++c) {
      size_t slot = (size_t)((plan->n_calls - 1 - c) % pb3_plan::kTimingRing) * ST_COUNT + i;
      if (!plan->ev_used[slot]) continue;
      hipError_t e = hipEventSynchronize(plan->ev[2 * slot + 1]);
      if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, plan->ev[2 * slot], plan->ev[2 * slot + 1]);
      if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
      sum += ms;
      ++cnt;
    }
    ms_out[i] = cnt ? (float)(sum / cnt) : 0.f;
    if (counts_out) counts_out[i] = cnt;
  }
  if (n_out) *n_out = n;
  return PB3_OK;
}

pb3_status pb3_stage_timing_reset(pb3_plan* plan) {
  if (!plan) {
    set_error("null plan");
    return PB3_EINVAL;
  }
  plan->n_calls = 0;
  std::fill(plan->ev_used.begin(), plan->ev_used.end(), 0);
  return PB3_OK;
}

const char* pb3_status_string(pb3_status s) {
  switch (s) {
    case PB3_OK: return "ok";
    case PB3_EINVAL: return "invalid argument";
    case PB3_ENOMEM: return "out of memory";
    case PB3_EDEVICE: return "device error";
    case PB3_EUNSUPPORTED: return "unsupported";
    case PB3_EBUSY: return "busy";
  }
  return "unknown status";
}

const char* pb3_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
