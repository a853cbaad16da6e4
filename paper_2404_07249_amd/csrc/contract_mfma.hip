// Triplet contraction on the matrix cores (gfx950).
//
// S_abc = sum_x G_a(x) G_b(x) G_c(x) for all pairs (a <= b) against all c,
// as a GEMM  C[pair][c] += A[pair][x] B[x][c]  with the voxels x as the
// reduction dimension.  The pair products A = G_a G_b are formed on the fly
// in registers and never stored.
//
// Lane layout (wave of 64, lane = 16 g + i): lane (i, g) holds, for every
// 16-bin group q, the field of bin 16 q + i at its voxels (8 per K-step of
// 32).  That is exactly the B operand of the MFMA for column block q, and
// the A operand of a 16-row pair block is one multiplication away: row i
// of block (p, q, s) is the pair (16 p + i, 16 q + ((i - s) mod 16)), whose
// second factor arrives from lane (i - s) mod 16 of the same row of 16
// lanes through a DPP row rotation.  Rotations s = 0..8 cover every
// unordered pair inside one 16-bin group (s = 8 twice), s = 0..15 every
// pair across two groups.  Column blocks below the pair's larger group
// (c < b) are skipped.
//
// Mixed precision: A and B are split into bf16 hi + lo (hi by round to
// nearest even, lo = x - hi exactly in FP32, then rounded), and each tile
// takes hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 with FP32
// accumulation.  FP32: v_mfma_f32_16x16x4_f32 on the unsplit values.
//
// Each wave accumulates its K-steps in FP32 registers over one chunk of
// voxels; the chunk's tiles are written as one FP32 partial vector (summed
// over a group's waves in LDS in a fixed order when a group has several),
// and the fixed-order FP64 reduction over chunks follows.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "fft_dev.h"
#include "job.h"
#include "pb3_internal.h"

namespace pb3 {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;
typedef float f2_t __attribute__((ext_vector_type(2)));
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2_t;

// Tile layouts.  A pair block (p, q, s) is 16 pair rows: row i pairs bin
// 16 p + i with bin 16 q + ((i - s) mod 16); a tile is a pair block against
// one 16-bin column block; cmask holds the block's column blocks.
//   kLayoutAB: every pair a <= b (p <= q; s = 0..8 inside a group, 0..15
//     across two), columns c >= 16 q.  Every triplet is read at (pair
//     (a, b), column c), as the column operand must be for the multipoles,
//     whose Legendre weight sits on the c leg.
//   kLayoutDiag: only the pairs inside one group (p = q).  S_abc is
//     symmetric, and a triplet a <= b <= c always has two bins in one group
//     when there are at most two groups (with three, the triplets with a,
//     b, c in groups 0, 1, 2 take the cross blocks (0, 1, s) against column
//     block 2).  A triplet with two bins in group p and one in group q != p
//     is read at the pair in p against column block q, so blocks (p, p, s)
//     take every other group's column block.  A triplet with all three bins
//     in group p: their positions cut the 16-cycle into three arcs that sum
//     to 16, so some pair is at most 5 apart, and it is read at that pair;
//     blocks (p, p, s) take their own column block only for s <= 5 (with
//     one group, blocks s = 6..8 are not formed at all).  At two groups
//     this is 18 pair blocks and 30 tiles instead of 34 and 43: fewer pair
//     products to form and split on the VALU, fewer MFMAs.
//   kLayoutDiag8, kLayoutDiag4: kLayoutDiag for plans whose last group
//     holds at most 8 or 4 real bins (the rest are zero padding).  Its pairs
//     are then at most r - 1 apart (r = 8 or 4), so only blocks s < r are
//     formed for it, and its one-group triplets, whose closest pair is at
//     most (r - 1) / 2 apart, need its own column block only for those s.
//     At 17-20 bins this is 13 pair blocks and 21 tiles, at 21-24 bins 17
//     and 27, instead of 18 and 30.
constexpr int kLayoutAB = 0, kLayoutDiag = 1, kLayoutDiag8 = 2, kLayoutDiag4 = 3;
constexpr int kDiagOwnMaxS = 5;  // largest pair separation a one-group triplet needs (16 / 3 rounded down)

// Real bins the last group of a Diag layout may hold, and its pair blocks
// (separations 0 .. n-1) and the separations that take its own column block.
constexpr int diag_cap(int L) { return L == kLayoutDiag4 ? 4 : L == kLayoutDiag8 ? 8 : 16; }
constexpr int diag_min(int a, int b) { return a < b ? a : b; }
constexpr int diag_blocks(int L, int nq, int p) {
  const int r = p == nq - 1 ? diag_cap(L) : 16;
  return nq == 1 ? diag_min(kDiagOwnMaxS, (r - 1) / 2) + 1 : diag_min(9, r);
}
constexpr int diag_own_max(int L, int nq, int p) {
  const int r = p == nq - 1 ? diag_cap(L) : 16;
  return diag_min(kDiagOwnMaxS, (r - 1) / 2);
}

struct PairBlock {
  int p, q, s;
  unsigned cmask;
};

constexpr unsigned all_cols(int nq) { return (1u << nq) - 1u; }
constexpr unsigned cols_from(int nq, int q) { return all_cols(nq) & ~((1u << q) - 1u); }

constexpr PairBlock pair_block(int L, int nq, int k) {
  if (L == kLayoutAB) {
    for (int p = 0; p < nq; ++p)
      for (int q = p; q < nq; ++q) {
        int ns = (p == q) ? 9 : 16;
        if (k < ns) return PairBlock{p, q, k, cols_from(nq, q)};
        k -= ns;
      }
  } else {
    // group 0, then (nq == 3) the cross blocks of groups 0 and 1, then the
    // other groups
    for (int p = 0; p < nq; ++p) {
      const int ns = diag_blocks(L, nq, p);
      if (k < ns)
        return PairBlock{p, p, k, k <= diag_own_max(L, nq, p) ? all_cols(nq) : all_cols(nq) & ~(1u << p)};
      k -= ns;
      if (p == 0 && nq == 3) {
        if (k < 16) return PairBlock{0, 1, k, 1u << 2};
        k -= 16;
      }
    }
  }
  return PairBlock{-1, -1, -1, 0u};
}
constexpr int n_pair_blocks(int L, int nq) {
  if (L == kLayoutAB) return nq * 9 + (nq * (nq - 1) / 2) * 16;
  int n = nq == 3 ? 16 : 0;
  for (int p = 0; p < nq; ++p) n += diag_blocks(L, nq, p);
  return n;
}
constexpr int popc(unsigned m) { return m ? (int)(m & 1u) + popc(m >> 1) : 0; }
// tiles (pair block x column block) in pair blocks [0, k)
constexpr int tiles_before(int L, int nq, int k) {
  int t = 0;
  for (int j = 0; j < k; ++j) t += popc(pair_block(L, nq, j).cmask);
  return t;
}
constexpr int n_tiles(int L, int nq) { return tiles_before(L, nq, n_pair_blocks(L, nq)); }
// tile offset of column block cb within its pair block
constexpr int col_rank(unsigned cmask, int cb) { return popc(cmask & ((1u << cb) - 1u)); }

// Pair-block ranges processed by one launch ("group") of the tile-staged
// kernel; at most ~54 tiles of accumulators per launch.
constexpr int n_groups(int L, int nq) { return nq <= 2 ? 1 : (L == kLayoutAB ? 3 : 2); }
constexpr int group_begin(int L, int nq, int g) {
  if (nq <= 2) return g == 0 ? 0 : n_pair_blocks(L, nq);
  if (L == kLayoutAB) {
    // nq == 3 pair blocks in order: (0,0)9 (0,1)16 (0,2)16 (1,1)9 (1,2)16 (2,2)9
    // tiles per block: 3, 2, 1, 2, 1, 1 -> groups of 43, 32, 43 tiles
    return g == 0 ? 0 : g == 1 ? 9 + 8 : g == 2 ? 9 + 16 + 16 : n_pair_blocks(L, nq);
  }
  // (0,0) 6 x 3 + 3 x 2, (0,1) 16 x 1: 40 tiles, then (1,1) and (2,2): at most 48 tiles
  return g == 0 ? 0 : g == 1 ? diag_blocks(L, nq, 0) + 16 : n_pair_blocks(L, nq);
}

__device__ __forceinline__ float ror16(float x, int s) {
  switch (s) {
    case 1: return __builtin_amdgcn_update_dpp(0.0f, x, 0x121, 0xf, 0xf, true);
    case 2: return __builtin_amdgcn_update_dpp(0.0f, x, 0x122, 0xf, 0xf, true);
    case 3: return __builtin_amdgcn_update_dpp(0.0f, x, 0x123, 0xf, 0xf, true);
    case 4: return __builtin_amdgcn_update_dpp(0.0f, x, 0x124, 0xf, 0xf, true);
    case 5: return __builtin_amdgcn_update_dpp(0.0f, x, 0x125, 0xf, 0xf, true);
    case 6: return __builtin_amdgcn_update_dpp(0.0f, x, 0x126, 0xf, 0xf, true);
    case 7: return __builtin_amdgcn_update_dpp(0.0f, x, 0x127, 0xf, 0xf, true);
    case 8: return __builtin_amdgcn_update_dpp(0.0f, x, 0x128, 0xf, 0xf, true);
    case 9: return __builtin_amdgcn_update_dpp(0.0f, x, 0x129, 0xf, 0xf, true);
    case 10: return __builtin_amdgcn_update_dpp(0.0f, x, 0x12a, 0xf, 0xf, true);
    case 11: return __builtin_amdgcn_update_dpp(0.0f, x, 0x12b, 0xf, 0xf, true);
    case 12: return __builtin_amdgcn_update_dpp(0.0f, x, 0x12c, 0xf, 0xf, true);
    case 13: return __builtin_amdgcn_update_dpp(0.0f, x, 0x12d, 0xf, 0xf, true);
    case 14: return __builtin_amdgcn_update_dpp(0.0f, x, 0x12e, 0xf, 0xf, true);
    case 15: return __builtin_amdgcn_update_dpp(0.0f, x, 0x12f, 0xf, 0xf, true);
    default: return x;
  }
}

// Split 8 FP32 values into bf16 hi (round to nearest even) and bf16 lo of
// the FP32 residual x - hi.  The residual is exactly representable; it is
// formed by v_dot2_f32_bf16 as x + (-1) * hi + 0 * hi' with the selector
// pairs sel.lo = (-1, 0) and sel.hi = (0, -1).  The selectors arrive as
// kernel arguments so that the compiler cannot fold them into an inline
// constant (whose packed-bf16 reading differs).
struct SplitSel {
  bf16x2_t lo, hi;
};

__device__ __forceinline__ void split8(const float* v, bf16x8_t& hi, bf16x8_t& lo, const SplitSel& sel) {
#pragma unroll
  for (int j = 0; j < 8; j += 2) {
    f2_t pv = {v[j], v[j + 1]};
    bf16x2_t h = __builtin_convertvector(pv, bf16x2_t);
    hi[j] = h[0];
    hi[j + 1] = h[1];
    f2_t r;
    r.x = __builtin_amdgcn_fdot2_f32_bf16(h, sel.lo, v[j], false);
    r.y = __builtin_amdgcn_fdot2_f32_bf16(h, sel.hi, v[j + 1], false);
    bf16x2_t l = __builtin_convertvector(r, bf16x2_t);
    lo[j] = l[0];
    lo[j + 1] = l[1];
  }
}

template <int NQ, int L, bool MIXED, int K, int K1, int T0>
__device__ __forceinline__ void do_blocks(const float (&gv)[NQ][8], const bf16x8_t (&bh)[NQ], const bf16x8_t (&bl)[NQ],
                                          f32x4_t* acc, const SplitSel& sel) {
#pragma clang fp contract(off)
  if constexpr (K < K1) {
    constexpr PairBlock pb = pair_block(L, NQ, K);
    constexpr int tb = tiles_before(L, NQ, K) - T0;
    float a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = gv[pb.p][j] * ror16(gv[pb.q][j], pb.s);
    if constexpr (MIXED) {
      bf16x8_t ah, al;
      split8(a, ah, al, sel);
#pragma unroll
      for (int cb = 0; cb < NQ; ++cb) {
        if ((pb.cmask >> cb) & 1u) {
          const int t = tb + col_rank(pb.cmask, cb);
          f32x4_t c = acc[t];
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[cb], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[cb], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[cb], c, 0, 0, 0);
          acc[t] = c;
        }
      }
      do_blocks<NQ, L, MIXED, K + 1, K1, T0>(gv, bh, bl, acc, sel);
    } else {
      // FP32: interleave this block's MFMA chains with the next block's so
      // consecutive MFMAs do not wait on the same accumulator
      constexpr bool PAIRED = K + 1 < K1;
      constexpr PairBlock pn = pair_block(L, NQ, PAIRED ? K + 1 : K);
      constexpr int tn = tiles_before(L, NQ, PAIRED ? K + 1 : K) - T0;
      float an[8];
      if constexpr (PAIRED) {
#pragma unroll
        for (int j = 0; j < 8; ++j) an[j] = gv[pn.p][j] * ror16(gv[pn.q][j], pn.s);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
#pragma unroll
        for (int cb = 0; cb < NQ; ++cb)
          if ((pb.cmask >> cb) & 1u) {
            const int t = tb + col_rank(pb.cmask, cb);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], gv[cb][j], acc[t], 0, 0, 0);
          }
        if constexpr (PAIRED) {
#pragma unroll
          for (int cb = 0; cb < NQ; ++cb)
            if ((pn.cmask >> cb) & 1u) {
              const int t = tn + col_rank(pn.cmask, cb);
              acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(an[j], gv[cb][j], acc[t], 0, 0, 0);
            }
        }
      }
      do_blocks<NQ, L, MIXED, (PAIRED ? K + 2 : K + 1), K1, T0>(gv, bh, bl, acc, sel);
    }
  }
}

// Pair blocks [k0, k1) are shared out between NG wave groups that stream
// the same voxels; boundaries balance an estimated cost per block (its
// split on the VALU plus its tiles on the matrix core).
constexpr int block_cost(int L, int nq, int k) { return 96 + 48 * popc(pair_block(L, nq, k).cmask); }
// (boundary g: the block edge whose running cost is nearest g/ng of the total)
constexpr int group_bound(int L, int nq, int k0, int k1, int ng, int g) {
  if (g <= 0) return k0;
  if (g >= ng) return k1;
  int total = 0;
  for (int k = k0; k < k1; ++k) total += block_cost(L, nq, k);
  int acc = 0, best = k0, best_err = total * ng + 1;
  for (int k = k0; k <= k1; ++k) {
    const int err = acc * ng > total * g ? acc * ng - total * g : total * g - acc * ng;
    if (err < best_err) {
      best_err = err;
      best = k;
    }
    if (k < k1) acc += block_cost(L, nq, k);
  }
  return best;
}
// union of the column blocks and of the row groups of pair blocks [b, e)
constexpr unsigned range_cols(int L, int nq, int b, int e) {
  unsigned m = 0u;
  for (int k = b; k < e; ++k) m |= pair_block(L, nq, k).cmask;
  return m;
}
constexpr unsigned range_rows(int L, int nq, int b, int e) {
  unsigned m = 0u;
  for (int k = b; k < e; ++k) m |= (1u << pair_block(L, nq, k).p) | (1u << pair_block(L, nq, k).q);
  return m;
}

// One launch covers pair blocks [K0, K1) (tiles [T0, T1)), shared out
// between kGroups groups of kWavesPerGroup waves.  Work-group w takes the
// voxels [w*vpw, (w+1)*vpw) in tiles of kTileVox voxels: each tile of all
// bins is loaded once per work-group into LDS (double-buffered, the next
// tile's global loads in flight during the current tile's math) together
// with its bf16 hi/lo split, then every group contracts it for its own
// pair blocks, wave w of a group taking voxels [32 w, 32 w + 32) of the
// tile.  part: [n_wg][n_tiles_total*256] FP32.
constexpr int kGroups = 4, kWavesPerGroup = 2, kContractThreads = 64 * kGroups * kWavesPerGroup;
constexpr int kTileVox = 32 * kWavesPerGroup;
constexpr int kPitchF = kTileVox + 4;  // floats per bin row of the staged tile
constexpr int kPitchH = kTileVox + 8;  // bf16 per bin row of the staged split

template <int NQ> struct TileStage {
  float f[16 * NQ * kPitchF];
  __bf16 hi[16 * NQ * kPitchH];
  __bf16 lo[16 * NQ * kPitchH];
};

template <int NQ, int L, int K0, int K1, int G> struct GroupRange {
  static constexpr int b = group_bound(L, NQ, K0, K1, kGroups, G);
  static constexpr int e = group_bound(L, NQ, K0, K1, kGroups, G + 1);
  static constexpr int t0 = tiles_before(L, NQ, b) - tiles_before(L, NQ, K0);  // offset in this launch's tiles
  static constexpr int nt = tiles_before(L, NQ, e) - tiles_before(L, NQ, b);
  static constexpr unsigned cols = range_cols(L, NQ, b, e);  // column blocks used
  static constexpr unsigned rows = range_rows(L, NQ, b, e);  // groups whose FP32 fields form the pairs
};

template <int NQ, int L, bool MIXED, int K0, int K1, int G, int NTMAX>
__device__ __forceinline__ void contract_tile(const TileStage<NQ>& st, int i, int grp, int wig, f32x4_t (&acc)[NTMAX],
                                              const SplitSel& sel) {
  using R = GroupRange<NQ, L, K0, K1, G>;
  float gv[NQ][8];
  bf16x8_t bh[NQ], bl[NQ];
  const int off = 32 * wig + 8 * grp;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (((R::rows | (MIXED ? 0u : R::cols)) >> q) & 1u) {
      const float4* pf = reinterpret_cast<const float4*>(st.f + (16 * q + i) * kPitchF + off);
      float4 x0 = pf[0], x1 = pf[1];
      gv[q][0] = x0.x; gv[q][1] = x0.y; gv[q][2] = x0.z; gv[q][3] = x0.w;
      gv[q][4] = x1.x; gv[q][5] = x1.y; gv[q][6] = x1.z; gv[q][7] = x1.w;
    }
    if constexpr (MIXED) {
      if ((R::cols >> q) & 1u) {
        bh[q] = *reinterpret_cast<const bf16x8_t*>(st.hi + (16 * q + i) * kPitchH + off);
        bl[q] = *reinterpret_cast<const bf16x8_t*>(st.lo + (16 * q + i) * kPitchH + off);
      }
    }
  }
  do_blocks<NQ, L, MIXED, R::b, R::e, tiles_before(L, NQ, R::b)>(gv, bh, bl, acc, sel);
}

template <int NQ, int L, int K0, int K1, int G, int NTMAX>
__device__ __forceinline__ void reduce_group(float* red, const f32x4_t (&acc)[NTMAX], int w, int i, int grp) {
  using R = GroupRange<NQ, L, K0, K1, G>;
  float* r = red + R::t0 * 256;
#pragma unroll
  for (int t = 0; t < R::nt; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int idx = t * 256 + (4 * grp + q) * 16 + i;
      r[idx] = (w == 0) ? acc[t][q] : r[idx] + acc[t][q];
    }
}

// Single-wave groups: the wave's tiles go straight from its accumulators to
// the chunk's partial vector (the same layout reduce_group builds), and the
// accumulators restart at zero.
template <int NQ, int L, int K0, int K1, int G, int NTMAX>
__device__ __forceinline__ void flush_group(float* __restrict__ dst, f32x4_t (&acc)[NTMAX], int i, int grp) {
  using R = GroupRange<NQ, L, K0, K1, G>;
  float* r = dst + R::t0 * 256;
#pragma unroll
  for (int t = 0; t < R::nt; ++t) {
#pragma unroll
    for (int q = 0; q < 4; ++q) r[t * 256 + (4 * grp + q) * 16 + i] = acc[t][q];
    acc[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  }
}

template <int NQ, int L, int K0, int K1> constexpr int max_group_tiles() {
  int m = GroupRange<NQ, L, K0, K1, 0>::nt;
  m = GroupRange<NQ, L, K0, K1, 1>::nt > m ? GroupRange<NQ, L, K0, K1, 1>::nt : m;
  m = GroupRange<NQ, L, K0, K1, 2>::nt > m ? GroupRange<NQ, L, K0, K1, 2>::nt : m;
  m = GroupRange<NQ, L, K0, K1, 3>::nt > m ? GroupRange<NQ, L, K0, K1, 3>::nt : m;
  return m < 1 ? 1 : m;
}

// Cooperative load of one voxel tile (all 16*NQ bins) into registers.
template <int NQ> struct TileRegs {
  static constexpr int N4 = 16 * NQ * kTileVox / 4;  // float4 per tile
  static constexpr int PER = (N4 + kContractThreads - 1) / kContractThreads;
  float4 v[PER];
};

// Bins at or above nb (the padding of the last 16-bin group) are zero
// fields and are not read.
template <int NQ>
__device__ __forceinline__ void tile_load(const float* __restrict__ g, long mvox, long v0, int nb,
                                          TileRegs<NQ>& r) {
#pragma unroll
  for (int k = 0; k < TileRegs<NQ>::PER; ++k) {
    int e = threadIdx.x + k * kContractThreads;
    if (e < TileRegs<NQ>::N4) {
      int bin = e / (kTileVox / 4), c4 = e % (kTileVox / 4);
      r.v[k] = bin < nb ? *reinterpret_cast<const float4*>(g + (size_t)bin * mvox + v0 + 4 * c4)
                        : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
}

// The FP32 rows (pair factors) come from r, the bf16 column operand from
// rc: the same fields for the bispectrum, the Legendre-weighted fields
// for its multipoles.
template <int NQ, bool MIXED>
__device__ __forceinline__ void tile_store(TileStage<NQ>& st, const TileRegs<NQ>& r, const TileRegs<NQ>& rc,
                                           const SplitSel& sel) {
#pragma unroll
  for (int k = 0; k < TileRegs<NQ>::PER; ++k) {
    int e = threadIdx.x + k * kContractThreads;
    if (e < TileRegs<NQ>::N4) {
      int bin = e / (kTileVox / 4), c4 = e % (kTileVox / 4);
      *reinterpret_cast<float4*>(st.f + bin * kPitchF + 4 * c4) = r.v[k];
      if constexpr (MIXED) {
        float x[8] = {rc.v[k].x, rc.v[k].y, rc.v[k].z, rc.v[k].w, 0.f, 0.f, 0.f, 0.f};
        bf16x8_t h8, l8;
        split8(x, h8, l8, sel);
        __bf16* ph = st.hi + bin * kPitchH + 4 * c4;
        __bf16* pl = st.lo + bin * kPitchH + 4 * c4;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          ph[j] = h8[j];
          pl[j] = l8[j];
        }
      }
    }
  }
}

template <int NQ, int L, bool MIXED, int K0, int K1>
__global__ void __launch_bounds__(kContractThreads) k_contract_mfma(const float* __restrict__ g, long mvox, long vpw,
                                                                    float* __restrict__ part, int part_len,
                                                                    unsigned sel_lo, unsigned sel_hi,
                                                                    size_t wstride, int nb,
                                                                    const float* __restrict__ gc) {
  static_assert(kGroups == 4, "group dispatch below assumes four groups");
  const bool cols = gc != nullptr;  // separate column fields (mixed precision only)
  g = job_ptr(g, wstride);
  part = job_ptr(part, wstride);
  constexpr int T0 = tiles_before(L, NQ, K0);
  constexpr int T1 = tiles_before(L, NQ, K1);
  constexpr int NTMAX = max_group_tiles<NQ, L, K0, K1>();
  constexpr int RED = (T1 - T0) * 256;
  constexpr int STAGE_FLOATS = (2 * sizeof(TileStage<NQ>) + 3) / 4;
  __shared__ __align__(16) float smem[RED > STAGE_FLOATS ? RED : STAGE_FLOATS];
  TileStage<NQ>* stage = reinterpret_cast<TileStage<NQ>*>(smem);
  float* red = smem;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int gi = wave / kWavesPerGroup, wig = wave % kWavesPerGroup;
  const int i = lane & 15, grp = lane >> 4;
  f32x4_t acc[NTMAX];
#pragma unroll
  for (int t = 0; t < NTMAX; ++t) acc[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  SplitSel sel;
  __builtin_memcpy(&sel.lo, &sel_lo, 4);
  __builtin_memcpy(&sel.hi, &sel_hi, 4);
  const long vb = (long)blockIdx.x * vpw;
  long ve = vb + vpw;
  if (ve > mvox) ve = mvox;
  const int n_tiles_wg = ve > vb ? (int)((ve - vb) / kTileVox) : 0;
  TileRegs<NQ> regs, regc;
  if (n_tiles_wg > 0) {
    tile_load<NQ>(g, mvox, vb, nb, regs);
    if (cols) tile_load<NQ>(gc, mvox, vb, nb, regc);
    tile_store<NQ, MIXED>(stage[0], regs, cols ? regc : regs, sel);
  }
  __syncthreads();
  for (int m = 0; m < n_tiles_wg; ++m) {
    const bool more = m + 1 < n_tiles_wg;
    if (more) {
      tile_load<NQ>(g, mvox, vb + (long)(m + 1) * kTileVox, nb, regs);
      if (cols) tile_load<NQ>(gc, mvox, vb + (long)(m + 1) * kTileVox, nb, regc);
    }
    const TileStage<NQ>& cur = stage[m & 1];
    switch (gi) {
      case 0: contract_tile<NQ, L, MIXED, K0, K1, 0>(cur, i, grp, wig, acc, sel); break;
      case 1: contract_tile<NQ, L, MIXED, K0, K1, 1>(cur, i, grp, wig, acc, sel); break;
      case 2: contract_tile<NQ, L, MIXED, K0, K1, 2>(cur, i, grp, wig, acc, sel); break;
      default: contract_tile<NQ, L, MIXED, K0, K1, 3>(cur, i, grp, wig, acc, sel); break;
    }
    if (more) tile_store<NQ, MIXED>(stage[(m + 1) & 1], regs, cols ? regc : regs, sel);
    __syncthreads();
  }
  // fixed-order sum of the waves of each group in LDS (reuses the stage)
  for (int w = 0; w < kWavesPerGroup; ++w) {
    if (wig == w) {
      switch (gi) {
        case 0: reduce_group<NQ, L, K0, K1, 0>(red, acc, w, i, grp); break;
        case 1: reduce_group<NQ, L, K0, K1, 1>(red, acc, w, i, grp); break;
        case 2: reduce_group<NQ, L, K0, K1, 2>(red, acc, w, i, grp); break;
        default: reduce_group<NQ, L, K0, K1, 3>(red, acc, w, i, grp); break;
      }
    }
    __syncthreads();
  }
  float* dst = part + (size_t)blockIdx.x * part_len + (size_t)T0 * 256;
  for (int e = threadIdx.x; e < RED; e += kContractThreads) dst[e] = red[e];
}

template <int NQ, int L, bool MIXED, int G>
static hipError_t launch_group(const float* g, long mvox, int n_wg, long vpw, float* part, int part_len, int n_jobs,
                               size_t wstride, int nb, const float* gc, hipStream_t s) {
  constexpr int K0 = group_begin(L, NQ, G), K1 = group_begin(L, NQ, G + 1);
  // bf16 pairs (element 0 in the low half): (-1, 0) and (0, -1)
  const unsigned sel_lo = 0x0000BF80u, sel_hi = 0xBF800000u;
  hipLaunchKernelGGL((k_contract_mfma<NQ, L, MIXED, K0, K1>), dim3(n_wg, 1, n_jobs), dim3(kContractThreads), 0, s, g,
                     mvox, vpw, part, part_len, sel_lo, sel_hi, wstride, nb, gc);
  return hipGetLastError();
}

template <int NQ, int L, bool MIXED>
static hipError_t launch_nq(const float* g, long mvox, int n_wg, long vpw, float* part, int part_len, int n_jobs,
                            size_t wstride, int nb, const float* gc, hipStream_t s) {
  hipError_t e = launch_group<NQ, L, MIXED, 0>(g, mvox, n_wg, vpw, part, part_len, n_jobs, wstride, nb, gc, s);
  if constexpr (n_groups(L, NQ) > 1) {
    if (e == hipSuccess)
      e = launch_group<NQ, L, MIXED, 1>(g, mvox, n_wg, vpw, part, part_len, n_jobs, wstride, nb, gc, s);
  }
  if constexpr (n_groups(L, NQ) > 2) {
    if (e == hipSuccess)
      e = launch_group<NQ, L, MIXED, 2>(g, mvox, n_wg, vpw, part, part_len, n_jobs, wstride, nb, gc, s);
  }
  return e;
}

// ===================================================================
// Fused inverse z pass + contraction.
//
// Work-group w takes whole z-lines (x, y) of the contraction grid, lines
// [w*lpw, (w+1)*lpw).  Besides its contraction waves it has 4 producer
// waves: while the contraction waves work on line m from one LDS stage, the
// producers build line m+1 in the other: for every bin pair (b, b+1) one
// complex M-point inverse FFT of F_b + i F_{b+1} (each extended by
// Hermitian symmetry from the y-pass output kz < kzn_b) gives G_b and
// G_{b+1} on the line as real and imaginary parts; the rows are scaled by
// 1/M^3, written to the stage and split into bf16 hi/lo there.  The
// filtered fields therefore never go to HBM.  Each FFT lives inside one
// wavefront, so producers synchronise per wave and only the per-line
// work-group barrier couples them to the contraction waves.
// Contraction waves per group: in mixed precision one (4 waves beside the
// 4 producers; 8 waves per work-group leave each wave the registers of two
// waves per SIMD, so neither the FFT nor the tile accumulators spill, where
// two per group spill and run slower); in FP32 two, whose second wave hides
// the dependent chains of the 8x more numerous FP32 MFMAs.
constexpr int kProducerThreads = 256;
constexpr int fused_waves(bool mixed) { return mixed ? 1 : 2; }
constexpr int fused_consumers(bool mixed) { return 64 * kGroups * fused_waves(mixed); }
constexpr int fused_threads(bool mixed) { return fused_consumers(mixed) + kProducerThreads; }

template <int NQ, int M> struct LineStage {
  static constexpr int PF = M + 4, PH = M + 8;
  float f[16 * NQ * PF];
  __bf16 hi[16 * NQ * PH];
  __bf16 lo[16 * NQ * PH];
};

template <int NQ, int L, bool MIXED, int K0, int K1, int G, int M, int NTMAX>
__device__ __forceinline__ void contract_line_group(const LineStage<NQ, M>& st, int i, int grp, int wig,
                                                    f32x4_t (&acc)[NTMAX], const SplitSel& sel) {
  using R = GroupRange<NQ, L, K0, K1, G>;
  constexpr int PF = LineStage<NQ, M>::PF, PH = LineStage<NQ, M>::PH;
  for (int ks = wig; ks < M / 32; ks += fused_waves(MIXED)) {
    const int off = 32 * ks + 8 * grp;
    float gv[NQ][8];
    bf16x8_t bh[NQ], bl[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      if (((R::rows | (MIXED ? 0u : R::cols)) >> q) & 1u) {
        const float4* pf = reinterpret_cast<const float4*>(st.f + (16 * q + i) * PF + off);
        float4 x0 = pf[0], x1 = pf[1];
        gv[q][0] = x0.x; gv[q][1] = x0.y; gv[q][2] = x0.z; gv[q][3] = x0.w;
        gv[q][4] = x1.x; gv[q][5] = x1.y; gv[q][6] = x1.z; gv[q][7] = x1.w;
      }
      if constexpr (MIXED) {
        if ((R::cols >> q) & 1u) {
          bh[q] = *reinterpret_cast<const bf16x8_t*>(st.hi + (16 * q + i) * PH + off);
          bl[q] = *reinterpret_cast<const bf16x8_t*>(st.lo + (16 * q + i) * PH + off);
        }
      }
    }
    do_blocks<NQ, L, MIXED, R::b, R::e, tiles_before(L, NQ, R::b)>(gv, bh, bl, acc, sel);
  }
}

// The producer's line factorisation M = R1 x R2: phase 1 runs R2 lanes of
// R1-point DFTs, phase 2 R1 lanes of R2-point DFTs, in a slot of 8 or 16
// lanes.  At M = 96 the default 16 x 6 gives each loading lane a 16-point
// DFT and 16 inputs with 10 of the slot's lanes idle; 8 x 12 halves the
// loads and twiddles per lane.
constexpr int zr1(int m) { return m == 96 ? 8 : fft2_r1(m); }
constexpr int zr2(int m) { return m / zr1(m); }
constexpr int zthreads(int m) { return (zr1(m) > zr2(m) ? zr1(m) : zr2(m)) <= 8 ? 8 : 16; }
static_assert(zr1(192) <= 16 && zr2(192) <= 16 && zr1(96) * zr2(96) == 96, "producer slots of at most 16 lanes");

// Producer side.  The 256 producer threads form slots of zthreads(M)
// lanes; slot t transforms the bin pair (2t, 2t + 1) of every line, packed
// as one complex line F_2t + i F_2t+1 (both real after the transform).
// The pair's geometry is read once.  In mixed precision the raw inputs of
// the next line are fetched into registers while the current line is
// transformed; the FP32 groups (12 waves, fewer registers per wave) fetch
// each line just before its transform.
template <int M> struct PairSrc {
  static constexpr int R1 = zr1(M), R2 = zr2(M);
  const float2* x0;  // bin 2t's y-pass output, lines of s0 planes
  const float2* x1;  // bin 2t + 1's (bin 2t's when there is none)
  int s0, s1;
  int k0n, k1n;      // kz planes of each bin (k1n = 0: no second bin)
  bool on;           // the slot holds a pair
  float2 r0[R1], r1[R1];
};

template <int M>
__device__ __forceinline__ void pair_init(PairSrc<M>& ps, const float2* a2, const BinGeom* __restrict__ geom,
                                          int nb, int slot, bool live) {
  const int npairs = (nb + 1) / 2;
  ps.on = live && slot < npairs;
  ps.x0 = ps.x1 = a2;
  ps.s0 = ps.s1 = ps.k0n = ps.k1n = 0;
  if (ps.on) {
    const BinGeom g0 = geom[2 * slot];
    const bool has1 = 2 * slot + 1 < nb;
    const BinGeom g1 = has1 ? geom[2 * slot + 1] : g0;
    ps.x0 = a2 + g0.a2_off;
    ps.x1 = a2 + g1.a2_off;
    ps.s0 = g0.kzn;
    ps.s1 = g1.kzn;
    ps.k0n = g0.kzn;
    ps.k1n = has1 ? g1.kzn : 0;
  }
}

// Which inputs j of a phase-1 lane (plane n = tl + R2 j, tl < R2) can be
// nonzero when every bin keeps fewer than KB planes (kzn <= KB - 1; KB = 0:
// no bound): plane n itself (n < kzn) or its mirror M - n (M - n < kzn).
// On an alias-free contraction grid (M > 3 K) kzn <= M / 3 + 1, so at
// M = 192 inputs j = 0..5 can only be direct planes, j = 10..15 only
// mirrored ones, and j = 6..9 are always zero: no load, no select.
template <int M, int KB> struct PlaneKinds {
  static constexpr int R2 = zr2(M);
  // without a bound (KB = 0, the full grid) a bin keeps at most M / 2 + 1
  // planes, so only the inputs j around n = M / 2 can be either
  static constexpr int B = KB > 0 ? KB : M / 2 + 2;
  static constexpr bool direct(int j) { return R2 * j < B; }
  static constexpr bool mirror(int j) { return M - R2 * j - (R2 - 1) < B; }
};

// Raw inputs of one line for a phase-1 lane: plane n = tl + R2 j comes from
// plane n (n < kzn) or, conjugated when combined, from plane M - n
// (M - n < kzn) of the half-spectrum; otherwise it is zero.  The plane
// bounds are re-read on each call, so that no comparison derived from them
// is kept across the line loop (the compiler would hold them as lane masks
// in scalar registers and spill those).
// MASKED (the FP32 groups, short of registers): loads under lane masks
// leave the zero planes zero.  Otherwise every lane loads, which suits
// fetching a line ahead: an input that can only be a direct plane or only a
// mirrored one reads a zero kept in global memory when it is past the bin's
// planes, so the combine needs no select (11% fewer producer instructions
// than selecting after the load); an input that can be either (around
// n = M / 2 on the full grid) selects, with plane 0 standing in for zero.
// zero input of the fused producer (read only)
__device__ float2 kZeroPlane[1];

template <int M, bool MASKED, int KB>
__device__ __forceinline__ void pair_fetch(PairSrc<M>& ps, long line, int tl) {
  using PK = PlaneKinds<M, KB>;
  constexpr int R1 = PairSrc<M>::R1, R2 = PairSrc<M>::R2;
  if (!ps.on || tl >= R2) return;
  const float2* p0 = ps.x0 + line * ps.s0;
  const float2* p1 = ps.x1 + line * ps.s1;
  int k0n = ps.k0n, k1n = ps.k1n;
  asm volatile("" : "+v"(k0n), "+v"(k1n));
#pragma unroll
  for (int j = 0; j < R1; ++j) {
    const int k = tl + R2 * j, m = M - k;
    const bool d = PK::direct(j), r = PK::mirror(j);
    if (!d && !r) continue;  // never loaded, never read
    if constexpr (MASKED) {
      float2 a = make_float2(0.f, 0.f), c = make_float2(0.f, 0.f);
      if (d && k < k0n) a = p0[k];
      else if (r && m < k0n) a = p0[m];
      if (d && k < k1n) c = p1[k];
      else if (r && m < k1n) c = p1[m];
      ps.r0[j] = a;
      ps.r1[j] = c;
    } else if (d != r) {
      // a direct-only or mirror-only input: past the bin's planes it reads
      // the zero constant, so the combine needs no select
      const int i0 = d ? k : m;
      const float2* q0 = i0 < k0n ? p0 + i0 : kZeroPlane;
      const float2* q1 = i0 < k1n ? p1 + i0 : kZeroPlane;
      ps.r0[j] = *q0;
      ps.r1[j] = *q1;
    } else {
      ps.r0[j] = p0[(d && k < k0n) ? k : ((r && m < k0n) ? m : 0)];
      ps.r1[j] = p1[(d && k < k1n) ? k : ((r && m < k1n) ? m : 0)];
    }
  }
}

// Build the stage for one line from the fetched inputs; next >= 0 starts the
// fetch of that line once phase 1 has taken these.
template <int NQ, bool MIXED, int M, bool MASKED, int KB>
__device__ __forceinline__ void produce_line(LineStage<NQ, M>& st, PairSrc<M>& ps, long next, const float2* tws,
                                             float2* scr, int slot, int tl, float scale, const SplitSel& sel) {
  using PK = PlaneKinds<M, KB>;
  constexpr int R1 = zr1(M), R2 = zr2(M);
  constexpr int PF = LineStage<NQ, M>::PF, PH = LineStage<NQ, M>::PH;
  if (!ps.on) return;
  const int b0 = 2 * slot, b1 = 2 * slot + 1;
  int k0n = ps.k0n, k1n = ps.k1n;  // re-read per line (see pair_fetch)
  asm volatile("" : "+v"(k0n), "+v"(k1n));
  fft2_line_wave<M, 1, zr1(M)>(
      scr + slot * R1 * (R2 + 1), tl, tws,
      [&](int j, int k) {
        const bool d = PK::direct(j), r = PK::mirror(j);
        if (!d && !r) return make_float2(0.f, 0.f);
        float2 a = ps.r0[j], c = ps.r1[j];
        if (!MASKED && d != r) {
          // zero past the planes (see pair_fetch); mirrored inputs are conjugated
          if (d) return make_float2(a.x - c.y, a.y + c.x);
          return make_float2(a.x + c.y, c.x - a.y);
        }
        if constexpr (MASKED) {
          if (!d || k >= k0n) a.y = -a.y;  // mirrored plane (or zero)
          if (!d || k >= k1n) c.y = -c.y;
        } else {
          const int m = M - k;
          const bool a_d = d && k < k0n, c_d = d && k < k1n;
          const bool a_r = r && m < k0n, c_r = r && m < k1n;
          if (!a_d) a = a_r ? make_float2(a.x, -a.y) : make_float2(0.f, 0.f);
          if (!c_d) c = c_r ? make_float2(c.x, -c.y) : make_float2(0.f, 0.f);
        }
        return make_float2(a.x - c.y, a.y + c.x);  // F_b + i F_{b+1}
      },
      [&]() {
        if (next >= 0) pair_fetch<M, MASKED, KB>(ps, next, tl);
      },
      [&](int k1, const float2 (&u)[R2]) {
#pragma unroll
        for (int k2 = 0; k2 < R2; k2 += 2) {
          const int z0 = k1 + R1 * k2, z1 = z0 + R1;
          float r0 = u[k2].x * scale, r1 = u[k2 + 1].x * scale;
          float i0 = u[k2].y * scale, i1 = u[k2 + 1].y * scale;
          st.f[b0 * PF + z0] = r0;
          st.f[b0 * PF + z1] = r1;
          st.f[b1 * PF + z0] = i0;
          st.f[b1 * PF + z1] = i1;
          if constexpr (MIXED) {
            float rv[8] = {r0, r1, i0, i1, 0.f, 0.f, 0.f, 0.f};
            bf16x8_t h8, l8;
            split8(rv, h8, l8, sel);
            st.hi[b0 * PH + z0] = h8[0];
            st.hi[b0 * PH + z1] = h8[1];
            st.hi[b1 * PH + z0] = h8[2];
            st.hi[b1 * PH + z1] = h8[3];
            st.lo[b0 * PH + z0] = l8[0];
            st.lo[b0 * PH + z1] = l8[1];
            st.lo[b1 * PH + z0] = l8[2];
            st.lo[b1 * PH + z1] = l8[3];
          }
        }
      });
}

// KB: every bin keeps fewer than KB z planes (0: no bound; see PlaneKinds).
template <int NQ, int L, bool MIXED, int M, int KB>
__global__ void __launch_bounds__(fused_threads(MIXED)) k_zcontract(const float2* __restrict__ a2,
                                                             const BinGeom* __restrict__ geom, int nb,
                                                             const float2* __restrict__ tw, float scale, long lpw,
                                                             float* __restrict__ part, int part_len, unsigned sel_lo,
                                                             unsigned sel_hi, size_t wstride, long nlines, int cpw,
                                                             int n_chunks) {
  a2 = job_ptr(a2, wstride);
  part = job_ptr(part, wstride);
  constexpr int K0 = 0, K1 = n_pair_blocks(L, NQ);
  constexpr int NT = n_tiles(L, NQ);
  constexpr int NTMAX = max_group_tiles<NQ, L, K0, K1>();
  constexpr int TL = zthreads(M), NSLOT = kProducerThreads / TL;
  static_assert(2 * NSLOT >= 16 * NQ, "one bin pair per producer slot");
  constexpr int STAGE_BYTES = (int)sizeof(LineStage<NQ, M>);
  constexpr int RED_BYTES = NT * 256 * 4;
  constexpr int MAIN = 2 * STAGE_BYTES > RED_BYTES ? 2 * STAGE_BYTES : RED_BYTES;
  __shared__ __align__(16) unsigned char smem[MAIN];
  __shared__ float2 tws[M];
  __shared__ float2 scr[NSLOT * zr1(M) * (zr2(M) + 1)];
  LineStage<NQ, M>* stage = reinterpret_cast<LineStage<NQ, M>*>(smem);
  float* red = reinterpret_cast<float*>(smem);
  const int tid = threadIdx.x;
  constexpr int FW = fused_waves(MIXED), NTHR = fused_threads(MIXED), NCON = fused_consumers(MIXED);
  const bool producer = tid >= NCON;
  const int lane = tid & 63, wave = tid >> 6;
  SplitSel sel;
  __builtin_memcpy(&sel.lo, &sel_lo, 4);
  __builtin_memcpy(&sel.hi, &sel_hi, 4);
  // zero both stages (rows of padding bins stay zero), twiddles to LDS
  for (int e = tid; e < 2 * STAGE_BYTES / 4; e += NTHR) reinterpret_cast<float*>(smem)[e] = 0.f;
  for (int e = tid; e < M; e += NTHR) tws[e] = tw[e];
  __syncthreads();
  // chunks [c0, c0 + cc) of lpw lines each, one partial vector per chunk
  // (several chunks per work-group only with single-wave groups)
  const int c0 = blockIdx.x * cpw;
  const int cc = n_chunks - c0 < cpw ? n_chunks - c0 : cpw;
  const long l0 = (long)c0 * lpw;
  long l1 = (long)(c0 + cc) * lpw;
  if (l1 > nlines) l1 = nlines;
  const int n = l1 > l0 ? (int)(l1 - l0) : 0;
  constexpr int TAIL = FW == 1 ? 0 : FW;  // barriers of the LDS sum of a group's waves
  // Producer and consumer waves run separate loops, so that neither holds
  // the other's registers, with the same barrier count (1 + n + TAIL).
  if (producer) {
    const int pslot = (tid - NCON) / TL, ptl = (tid - NCON) % TL;
    PairSrc<M> ps;
    pair_init<M>(ps, a2, geom, nb, pslot, n > 0);
    constexpr bool AHEAD = MIXED;  // fetch a line ahead (see PairSrc)
    if (ps.on) {
      pair_fetch<M, !AHEAD, KB>(ps, l0, ptl);
      produce_line<NQ, MIXED, M, !AHEAD, KB>(stage[0], ps, AHEAD && n > 1 ? l0 + 1 : -1, tws, scr, pslot, ptl,
                                             scale, sel);
    }
    __syncthreads();
    for (int m = 0; m < n; ++m) {
      if (m + 1 < n) {
        if constexpr (!AHEAD) pair_fetch<M, true, KB>(ps, l0 + m + 1, ptl);
        produce_line<NQ, MIXED, M, !AHEAD, KB>(stage[(m + 1) & 1], ps, AHEAD && m + 2 < n ? l0 + m + 2 : -1, tws,
                                               scr, pslot, ptl, scale, sel);
      }
      __syncthreads();
    }
    for (int w = 0; w < TAIL; ++w) __syncthreads();
  } else {
    const int gi = wave / FW, wig = wave % FW;
    const int i = lane & 15, grp = lane >> 4;
    f32x4_t acc[NTMAX];
#pragma unroll
    for (int t = 0; t < NTMAX; ++t) acc[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    __syncthreads();
    int gm = 0;  // line index within the work-group (stage parity)
    for (int c = 0; c < cc; ++c) {
      const long cl0 = (long)(c0 + c) * lpw;
      long cl1 = cl0 + lpw;
      if (cl1 > nlines) cl1 = nlines;
      const int nc = cl1 > cl0 ? (int)(cl1 - cl0) : 0;
      for (int m = 0; m < nc; ++m, ++gm) {
        const LineStage<NQ, M>& cur = stage[gm & 1];
        switch (gi) {
          case 0: contract_line_group<NQ, L, MIXED, K0, K1, 0, M>(cur, i, grp, wig, acc, sel); break;
          case 1: contract_line_group<NQ, L, MIXED, K0, K1, 1, M>(cur, i, grp, wig, acc, sel); break;
          case 2: contract_line_group<NQ, L, MIXED, K0, K1, 2, M>(cur, i, grp, wig, acc, sel); break;
          default: contract_line_group<NQ, L, MIXED, K0, K1, 3, M>(cur, i, grp, wig, acc, sel); break;
        }
        __syncthreads();
      }
      if constexpr (FW == 1) {
        float* dst = part + (size_t)(c0 + c) * part_len;
        switch (gi) {
          case 0: flush_group<NQ, L, K0, K1, 0>(dst, acc, i, grp); break;
          case 1: flush_group<NQ, L, K0, K1, 1>(dst, acc, i, grp); break;
          case 2: flush_group<NQ, L, K0, K1, 2>(dst, acc, i, grp); break;
          default: flush_group<NQ, L, K0, K1, 3>(dst, acc, i, grp); break;
        }
      }
    }
    // fixed-order sum of the waves of each group in LDS (reuses the stages)
    for (int w = 0; w < TAIL; ++w) {
      if (wig == w) {
        switch (gi) {
          case 0: reduce_group<NQ, L, K0, K1, 0>(red, acc, w, i, grp); break;
          case 1: reduce_group<NQ, L, K0, K1, 1>(red, acc, w, i, grp); break;
          case 2: reduce_group<NQ, L, K0, K1, 2>(red, acc, w, i, grp); break;
          default: reduce_group<NQ, L, K0, K1, 3>(red, acc, w, i, grp); break;
        }
      }
      __syncthreads();
    }
  }
  if constexpr (FW > 1) {
    float* dst = part + (size_t)c0 * part_len;
    for (int e = tid; e < NT * 256; e += NTHR) dst[e] = red[e];
  }
}

template <int NQ, int L, bool MIXED, int M>
static hipError_t launch_fused_m(const pb3_plan& p, const Exec& x, hipStream_t s) {
  const long nlines = (long)p.Mx * p.My;  // z lines of length M = Mz
  const long lpw = (nlines + p.contract_wgs - 1) / p.contract_wgs;
  const unsigned sel_lo = 0x0000BF80u, sel_hi = 0xBF800000u;
  const float scale = (float)(1.0 / ((double)p.Mx * p.My * p.Mz));
  // With single-wave groups a work-group takes up to 4 consecutive chunks
  // (one start-up per CU instead of one per chunk) while the grid still
  // covers every CU; the partial vectors are the same.
  int cpw = 1;
  if (fused_waves(MIXED) == 1 && p.n_cu > 0)
    while (cpw < 4 && p.contract_wgs % (2 * cpw) == 0 && p.contract_wgs / (2 * cpw) >= p.n_cu) cpw *= 2;
  const int n_wg = (p.contract_wgs + cpw - 1) / cpw;
  // every bin keeps at most Kz planes; on an alias-free grid Kz <= M / 3 + 1,
  // and on any grid Kz <= M / 2 + 1 (the producer's plane kinds assume it)
  constexpr int KB = M / 3 + 2;
  if (p.Kz > M / 2 + 1) return hipErrorInvalidValue;
  if (p.Kz < KB)
    hipLaunchKernelGGL((k_zcontract<NQ, L, MIXED, M, KB>), dim3(n_wg, 1, x.n_jobs), dim3(fused_threads(MIXED)), 0, s,
                       x.ws.a2, p.d.geom, p.nb, p.d.tw_m[2], scale, lpw, x.ws.part, p.part_len, sel_lo, sel_hi,
                       x.wstride, nlines, cpw, p.contract_wgs);
  else
    hipLaunchKernelGGL((k_zcontract<NQ, L, MIXED, M, 0>), dim3(n_wg, 1, x.n_jobs), dim3(fused_threads(MIXED)), 0, s,
                       x.ws.a2, p.d.geom, p.nb, p.d.tw_m[2], scale, lpw, x.ws.part, p.part_len, sel_lo, sel_hi,
                       x.wstride, nlines, cpw, p.contract_wgs);
  return hipGetLastError();
}

template <int NQ, int L, bool MIXED>
static hipError_t launch_fused_nq(const pb3_plan& p, const Exec& x, hipStream_t s) {
  switch (p.Mz) {
    case 32: return launch_fused_m<NQ, L, MIXED, 32>(p, x, s);
    case 64: return launch_fused_m<NQ, L, MIXED, 64>(p, x, s);
    case 96: return launch_fused_m<NQ, L, MIXED, 96>(p, x, s);
    case 128: return launch_fused_m<NQ, L, MIXED, 128>(p, x, s);
    case 192: return launch_fused_m<NQ, L, MIXED, 192>(p, x, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NQ, int L>
static hipError_t launch_fused_l(const pb3_plan& p, const Exec& x, bool mixed, hipStream_t s) {
  return mixed ? launch_fused_nq<NQ, L, true>(p, x, s) : launch_fused_nq<NQ, L, false>(p, x, s);
}

// Accumulation chunks (partial vectors) of the fused kernel: enough that
// each covers about kFusedVoxPerWg voxels, between one and four times the
// resident work-group count.  Each chunk's FP32 MFMA accumulators then sum
// a bounded number of products (at 256^3 x 30 bins, 1024 chunks: max
// |dB|/A 1.8e-7 in mixed precision against 5.5e-7 with 256), at a few per
// cent more time for the extra partial vectors.
constexpr long kFusedVoxPerWg = 6912;
int fused_grid(int nq, int m, long mvox, int n_cu) {
  int per = 1;
  hipError_t e = hipErrorInvalidValue;
  const void* fn = nullptr;
  if (nq == 1) {
    constexpr int L = kLayoutDiag;
    fn = m == 32 ? (const void*)k_zcontract<1, L, true, 32, 0> : m == 64 ? (const void*)k_zcontract<1, L, true, 64, 0>
       : m == 96 ? (const void*)k_zcontract<1, L, true, 96, 0> : m == 128 ? (const void*)k_zcontract<1, L, true, 128, 0>
                 : (const void*)k_zcontract<1, L, true, 192, 0>;
  } else {
    constexpr int L = kLayoutDiag;
    fn = m == 32 ? (const void*)k_zcontract<2, L, true, 32, 0> : m == 64 ? (const void*)k_zcontract<2, L, true, 64, 0>
       : m == 96 ? (const void*)k_zcontract<2, L, true, 96, 0> : m == 128 ? (const void*)k_zcontract<2, L, true, 128, 0>
                 : (const void*)k_zcontract<2, L, true, 192, 0>;
  }
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, fused_threads(true), 0);
  if (e != hipSuccess || per < 1) per = 1;
  if (per > 4) per = 4;
  const long base = (long)n_cu * per;
  const long want = (mvox + kFusedVoxPerWg - 1) / kFusedVoxPerWg;
  const long mult = std::min<long>(4, std::max<long>(1, (want + base - 1) / base));
  return (int)(base * mult);
}

bool fused_supported(int nq, int m) {
  return nq >= 1 && nq <= 2 && (m == 32 || m == 64 || m == 96 || m == 128 || m == 192);
}

// The bispectrum's tile layout for nb bins: trimmed when the last 16-bin
// group holds at most 8 or 4 real bins.
static int diag_layout(int nb) {
  const int nq = (nb + 15) / 16, r = nb - 16 * (nq - 1);
  return r <= 4 ? kLayoutDiag4 : r <= 8 ? kLayoutDiag8 : kLayoutDiag;
}

hipError_t launch_zcontract(const pb3_plan& p, const Exec& x, bool mixed, hipStream_t s) {
  const int nq = p.nb_pad / 16, l = diag_layout(p.nb);
  if (nq == 1)
    return l == kLayoutDiag4   ? launch_fused_l<1, kLayoutDiag4>(p, x, mixed, s)
           : l == kLayoutDiag8 ? launch_fused_l<1, kLayoutDiag8>(p, x, mixed, s)
                               : launch_fused_l<1, kLayoutDiag>(p, x, mixed, s);
  if (nq == 2)
    return l == kLayoutDiag4   ? launch_fused_l<2, kLayoutDiag4>(p, x, mixed, s)
           : l == kLayoutDiag8 ? launch_fused_l<2, kLayoutDiag8>(p, x, mixed, s)
                               : launch_fused_l<2, kLayoutDiag>(p, x, mixed, s);
  return hipErrorInvalidValue;
}

int mfma_tiles(bool ab, int nb) {
  const int nq = (nb + 15) / 16;
  const int L = ab ? kLayoutAB : diag_layout(nb);
  return nq >= 1 && nq <= 3 ? n_tiles(L, nq) : -1;
}

// Partial-vector index of triplet (a, b, c), a <= b <= c: its tile, row and
// column (-1 if the layout does not produce it).  kLayoutAB reads it at
// (pair (a, b), column c).  kLayoutDiag: all three in one group, at the
// pair of the smallest separation against the third bin; else at (pair
// (a, b), column c) when a and b share a group, at (pair (b, c), column a)
// when b and c do, and (three groups) at the cross pair (a, b) against c.
int mfma_locate(bool ab, int nb, int a, int b, int c) {
  const int nq = (nb + 15) / 16;
  const int L = ab ? kLayoutAB : diag_layout(nb);
  int x = a, y = b, z = c;
  auto sep = [](int u, int v) {  // cyclic separation of two positions in a 16-bin group
    const int d = ((u - v) % 16 + 16) % 16;
    return d <= 8 ? d : 16 - d;
  };
  if (!ab) {
    if (a / 16 == b / 16 && b / 16 == c / 16) {
      // all in one group: the pair at the smallest separation (at most 5)
      const int sab = sep(a, b), sac = sep(a, c), sbc = sep(b, c);
      if (sac < sab && sac <= sbc) {
        y = c;
        z = b;
      } else if (sbc < sab && sbc < sac) {
        x = b;
        y = c;
        z = a;
      }
    } else if (a / 16 != b / 16 && b / 16 == c / 16) {
      x = b;
      y = c;
      z = a;
    }
  }
  const int p = x / 16, q = y / 16, ix = x % 16, iy = y % 16;
  int row, s;
  if (p == q) {
    const int d = ((ix - iy) % 16 + 16) % 16;
    if (d <= 8) {
      row = ix;
      s = d;
    } else {
      row = iy;
      s = 16 - d;
    }
  } else {
    row = ix;
    s = ((ix - iy) % 16 + 16) % 16;
  }
  const int cb = z / 16, col = z % 16;
  const int npb = n_pair_blocks(L, nq);
  for (int k = 0; k < npb; ++k) {
    const PairBlock pb = pair_block(L, nq, k);
    if (pb.p == p && pb.q == q && pb.s == s) {
      if (!((pb.cmask >> cb) & 1u)) return -1;
      return (tiles_before(L, nq, k) + col_rank(pb.cmask, cb)) * 256 + row * 16 + col;
    }
  }
  return -1;
}

// Work-groups that fill the device once: CUs x resident 8-wave groups.
int mfma_grid(int nq, int n_cu) {
  int per = 1;
  hipError_t e = hipErrorInvalidValue;
  constexpr int L = kLayoutDiag;
  switch (nq) {
    case 1:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per, (const void*)k_contract_mfma<1, L, true, 0, group_begin(L, 1, 1)>, kContractThreads, 0);
      break;
    case 2:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per, (const void*)k_contract_mfma<2, L, true, 0, group_begin(L, 2, 1)>, kContractThreads, 0);
      break;
    default:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per, (const void*)k_contract_mfma<3, L, true, 0, group_begin(L, 3, 1)>, kContractThreads, 0);
      break;
  }
  if (e != hipSuccess || per < 1) per = 1;
  if (per > 4) per = 4;
  return n_cu * per;
}

hipError_t launch_contract_mfma(const pb3_plan& p, const Exec& x, bool mixed, hipStream_t s) {
  return launch_contract_cols(p, x, x.ws.g, nullptr, mixed, false, s);
}

// ab = false (the bispectrum): kLayoutDiag into partial vectors of
// p.part_len floats; ab = true (column fields gc, or the fields g
// themselves when gc is null): kLayoutAB into vectors of p.part_len_ab.

hipError_t launch_contract_cols(const pb3_plan& p, const Exec& x, const float* g, const float* gc, bool mixed,
                                bool ab, hipStream_t s) {
  if ((gc && !ab) || (gc && !mixed)) return hipErrorInvalidValue;  // column fields: bf16 operand, layout AB
  const long mvox = (long)mpix(p);
  const int nq = p.nb_pad / 16;
  const int n_wg = p.contract_wgs;
  long vpw = (mvox + n_wg - 1) / n_wg;
  vpw = (vpw + kTileVox - 1) / kTileVox * kTileVox;
  float* part = x.ws.part;
  const int nj = x.n_jobs;
  const size_t ws = x.wstride;
  if (ab) {
    if (!mixed) return hipErrorInvalidValue;
    constexpr int L = kLayoutAB;
    const int pl = p.part_len_ab;
    switch (nq) {
      case 1: return launch_nq<1, L, true>(g, mvox, n_wg, vpw, part, pl, nj, ws, p.nb, gc, s);
      case 2: return launch_nq<2, L, true>(g, mvox, n_wg, vpw, part, pl, nj, ws, p.nb, gc, s);
      case 3: return launch_nq<3, L, true>(g, mvox, n_wg, vpw, part, pl, nj, ws, p.nb, gc, s);
      default: return hipErrorInvalidValue;
    }
  }
  const int pl = p.part_len, l = diag_layout(p.nb);
  auto run = [&](auto lc) -> hipError_t {
    constexpr int L = decltype(lc)::value;
    switch (nq) {
      case 1: return mixed ? launch_nq<1, L, true>(g, mvox, n_wg, vpw, part, pl, nj, ws, p.nb, gc, s)
                           : launch_nq<1, L, false>(g, mvox, n_wg, vpw, part, pl, nj, ws, p.nb, gc, s);
      case 2: return mixed ? launch_nq<2, L, true>(g, mvox, n_wg, vpw, part, pl, nj, ws, p.nb, gc, s)
                           : launch_nq<2, L, false>(g, mvox, n_wg, vpw, part, pl, nj, ws, p.nb, gc, s);
      case 3: return mixed ? launch_nq<3, L, true>(g, mvox, n_wg, vpw, part, pl, nj, ws, p.nb, gc, s)
                           : launch_nq<3, L, false>(g, mvox, n_wg, vpw, part, pl, nj, ws, p.nb, gc, s);
      default: return hipErrorInvalidValue;
    }
  };
  if (l == kLayoutDiag4) return run(std::integral_constant<int, kLayoutDiag4>{});
  if (l == kLayoutDiag8) return run(std::integral_constant<int, kLayoutDiag8>{});
  return run(std::integral_constant<int, kLayoutDiag>{});
}

}  // namespace pb3
