// SBMT hot path for MI355X (gfx950): bitmap -> boundary -> exact per-triangle
// classification -> canonical class -> template lookup -> closed mesh
// (arXiv 2602.19474, Sec. 3.3, Alg. 1, Alg. 2, App. G).
//
// Every kernel serves one image or a batch of images: a kernel's blocks are
// numbered across the images of the call and mapped back to (image, local
// block) through a prefix table of per-image block counts.
//
// Kernels
//   k_coarsen  block-majority coarse raster as packed bits, with a background ring
//   k_count    per tile (RB rows x kCB owners): owners whose 3x3 sample window
//              is uniform, or that no boundary segment reaches, are counted at
//              once; the others ("slow" owners) are appended to a record list
//   k_slow     every slow owner of the call, densely: exact classification
//              (Alg. 1), class and rotation (Sec. 3.3.3), a 16-byte record, and
//              its counts added to its row segment
//   k_scan_*   exclusive prefix sum of the per-segment counts -> output offsets
//   k_emit     per tile: owner counts and their prefix sums in LDS (with a
//              one-row, one-column halo for neighbour ids), then FP64
//              vertices, int32 triangles and u8 class codes (Alg. 2)
//   k_fused    the whole classify-scan-emit path in one persistent launch:
//              workgroups take full-width row bands in ticket order, publish
//              their counts and find their output offsets by a decoupled
//              look-back over earlier bands of the same image
//
// The output order is fixed by the owner numbering and does not depend on
// the tile shape, the strategy or the batch.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/sbmt.h"

#define SBMT_CONST __constant__
#include "sbmt_tables.h"
#define SBMT_HD __device__ __forceinline__
#include "sbmt_device.h"

namespace sbmt {

SBMT_HD int lut_key(int code) { return sbmt_lut_key[code]; }
SBMT_HD int lut_nfg(int cls) { return sbmt_lut_nfg[cls]; }
SBMT_HD int lut_ntri(int cls) { return sbmt_lut_ntri[cls]; }
SBMT_HD uint32_t lut_tri(int cls, int j) { return sbmt_lut_tri[cls][j]; }

// Block segment table of each device (see block_tab), written by k_block_table
// when a handle is created on the device.
__device__ uint4 g_blocktab[1024];
SBMT_HD uint4 block_tab(int i) { return g_blocktab[i]; }

__global__ void __launch_bounds__(256) k_block_table() {
  const int s9 = blockIdx.x * 256 + threadIdx.x;
  if (s9 >= 512) return;
  uint4 A, B;
  block_table_entry((uint32_t)s9, A, B);
  g_blocktab[2 * s9] = A;
  g_blocktab[2 * s9 + 1] = B;
}

constexpr int kThreads = 256;
constexpr int kCB = 256;               // owners per row segment (one per thread)
constexpr int kScanThreads = 512;  // 2048 segments per scan block: more blocks in flight than 4096
constexpr int kScanChunk = 4 * kScanThreads;
constexpr int kWinRows = 16, kWinWords = 16;  // LDS window of the coarse raster per tile
constexpr int64_t kMaxRecords = 0x7ffffffeLL;  // records of a call
constexpr int kMaxBandChunks = 64;             // fused path: row segments per band
constexpr int kSlowBlocks = 2048;              // dense slow pass: blocks of its grid-stride loop
constexpr int kDenseLists = 64;                // dense slow lists (tile mod 64), each with its own counter
constexpr int kSizeWords = SBMT_SIZE_WORDS;    // per-image sizes record
constexpr int kSegSlots = 64;                  // partial segment counts per image (spread atomics)
constexpr int kRowPad = 20;                    // row-table entries past the last grid row (tile and halo rows)

// One image of a call, as the kernels see it.
struct Img {
  Geo g;
  const uint8_t* bm;  // bitmap rows (device)
  uint32_t* bits;     // coarse raster, (CH + 2 kRing) rows of wpr words
  uint16_t* omap;     // [NK][NI] owner map of the multi-kernel path, see map_code
  RowT* rows;         // [NK + kRowPad] per grid row data of the exact predicates (row_table_entry)
  uint32_t* cols;     // [NI][2] per grid column and row parity: window column Clo + 8 | x0 << 24 | x1 << 28
  int64_t seg0;       // first row segment of the image in the call's segment arrays
  int64_t band0;      // first band of the image (fused path, 4-row numbering)
  int64_t halo0;      // first word of the image's halo rows (fused path)
  double* verts;
  int32_t* tris;
  uint8_t* codes;
  int64_t vcap, tcap;  // output capacities in rows
};

// Scratch shared by the images of a call.
struct Shared {
  int4* seg_cnt;                    // [nseg] (nv, nt, ncut, 0) of owners counted in k_count
  unsigned long long* seg_slow;     // [nseg] slow-owner counts nv | nt << 21 | ncut << 42
  longlong4* seg_off;               // [nseg + 1] exclusive (v, t, cut) over the call; [nseg] = totals
  longlong4* blk;                   // [nblk] scan block sums
  unsigned long long* ctr;          // [8] 1: band ticket
  int* imgerr;                      // [n] protocol violation seen
  int64_t* sizes;                   // [n][kSizeWords] n_vertices, n_triangles, n_cut, status, n_segments
  unsigned long long* segacc;       // [n][kSegSlots] partial boundary-segment counts
  SlowRec* rec;                     // slow-owner records, tcap per count tile
  uint32_t* dense;                  // [kDenseLists][dcap] indices into rec of the queued slow owners
  unsigned long long* dctr;         // [kDenseLists] entries of each list
  int* tile_n;                      // [count tiles] slow owners queued by each tile
  unsigned long long* band;         // [nbands] fused path look-back words
  int64_t tcap, nseg, nbands, dcap;
  int nblk, n;
};

// Block -> image maps.  OneSrc carries the single image by value; ManySrc
// reads the image table of the workspace and a per-kernel prefix table of
// block counts.
struct OneSrc {
  Img d;
  __device__ __forceinline__ int find(int64_t b, const int64_t*, int64_t& local) const {
    local = b;
    return 0;
  }
  __device__ __forceinline__ const Img& img(int) const { return d; }
};

struct ManySrc {
  const Img* d;
  int n;
  __device__ __forceinline__ int find(int64_t b, const int64_t* tab, int64_t& local) const {
    int lo = 0, hi = n - 1;  // largest i with tab[i] <= b
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tab[mid] <= b) lo = mid;
      else hi = mid - 1;
    }
    local = b - tab[lo];
    return lo;
  }
  __device__ __forceinline__ const Img& img(int i) const { return d[i]; }
};

SBMT_HD unsigned long long pack_counts(uint32_t info) {
  return (unsigned long long)info_nv(info) | ((unsigned long long)info_nt(info) << 21) |
         ((unsigned long long)info_ncut(info) << 42);
}

// Owner map of the multi-kernel path, two bytes per owner: bits 0-14 of the
// info word (vertex, crossing counts, chain vertices, triangle counts) and bit
// 15 = slow.  Owners that are not slow have no chain vertex, so their bit 7
// carries the inside bit instead.  k_count writes every owner's code (slow
// ones with a record as a bare 0x8000), k_slow the codes of its owners.
SBMT_HD uint32_t map_code(uint32_t info) {
  return info_slow(info) ? (info & 0xffffu) : ((info & 0x7f7fu) | ((uint32_t)info_fg(info) << 7));
}
SBMT_HD uint32_t map_info(uint32_t code) {
  return (code & 0x8000u) ? code : ((code & 0x7f7fu) | (((code >> 7) & 1u) << 16));
}

// Owner frame without the samples: what emission needs of a slow owner.
SBMT_HD Frame owner_place(const Geo& g, int k, int i, int Rlo) {
  Frame f;
  f.k = k;
  f.i = i;
  f.o = k & 1;
  f.X = g.X0 + 4 * g.h * i + 2 * g.h * f.o;
  f.Rlo = Rlo;
  f.Clo = clo_of(g, f.X);
  f.s9 = 0;
  return f;
}

// Inclusive scan over the 64 lanes of a wave with DPP row shifts and row
// broadcasts (lanes without a source add 0).
__device__ __forceinline__ int wave_incl_scan_dpp(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
  return x;
}

// ---------------------------------------------------------------------------
// Coarse raster: bit (R + ring, C + ringC) = [2 * #fg pixels of block (R, C) >= s^2].
// A block covers kCoarsenRows stored rows and 256 stored columns.  Its pixel
// rectangle is read with aligned 16-byte loads (a load never leaves the page
// of the bytes it is for) and folded into per-pixel-row bit masks in LDS;
// then one lane per sample counts its s x s block with popcounts and the
// samples of a wave are packed by a ballot.  Samples outside the image (the
// ring) are background.
// Blocks per image: ceil(wpr / 8) x ceil((CH + 2 ring) / kCoarsenRows).
// ---------------------------------------------------------------------------
constexpr int kCoarsenRows = 8;
constexpr int kCoarsenMaxS = 9;
constexpr int kCoarsenWords = (256 * kCoarsenMaxS + 15 + kCoarsenMaxS + 31) / 32 + 2;  // mask words per pixel row

// Stride 2 with 16-byte aligned rows: four lanes make one raster word, each
// from one aligned 16-byte load of the two pixel rows of its 8 samples; a
// 2 x 2 block is foreground iff at least two of its pixels are (both of a
// pair, or one of each pair).
__device__ __forceinline__ void coarsen_s2(const Img& d, const Geo& g, int bx, int ry) {
  auto nz4 = [](uint32_t w) {  // bit j = byte j is nonzero
    uint32_t t = (((w & 0x7f7f7f7fu) + 0x7f7f7f7fu) | w) & 0x80808080u;
    t >>= 7;
    return (t | (t >> 7) | (t >> 14) | (t >> 21)) & 15u;
  };
  auto load16 = [&](int y, int x) -> uint32_t {  // nonzero bits of pixels x .. x+15 of row y (0 outside)
    if (y < 0 || y >= g.H || x + 16 <= 0 || x >= g.W) return 0u;
    const uint8_t* row = d.bm + (int64_t)y * g.stride;
    if (x >= 0 && x + 16 <= g.W) {
      const uint4 v = *reinterpret_cast<const uint4*>(row + x);
      return nz4(v.x) | (nz4(v.y) << 4) | (nz4(v.z) << 8) | (nz4(v.w) << 12);
    }
    uint32_t m = 0;  // the chunk at the row's end
    for (int j = 0; j < 16; ++j)
      if (x + j >= 0 && x + j < g.W && row[x + j]) m |= 1u << j;
    return m;
  };
  const int task = threadIdx.x >> 2, part = threadIdx.x & 3;
  const int rr = ry * kCoarsenRows + (task >> 3), w = 8 * bx + (task & 7);  // stored row, raster word
  const int C0 = 32 * w - kRingC + 8 * part, R = rr - kRing;                  // first coarse column, coarse row
  uint32_t bits = 0;
  if (R >= 0 && R < g.CH) {
    const uint32_t T = load16(2 * R, 2 * C0), B = load16(2 * R + 1, 2 * C0);
    uint32_t m = ((T & (T >> 1)) | (B & (B >> 1)) | ((T | (T >> 1)) & (B | (B >> 1)))) & 0x5555u;
    m = (m | (m >> 1)) & 0x3333u;
    m = (m | (m >> 2)) & 0x0f0fu;
    m = (m | (m >> 4)) & 0x00ffu;
    bits = m << (8 * part);
  }
  // the four lanes of a word OR their bytes together (quad permutations)
  bits |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)bits, 0xb1, 0xf, 0xf, false);  // quad_perm [1,0,3,2]
  bits |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)bits, 0x4e, 0xf, 0xf, false);  // quad_perm [2,3,0,1]
  if (part == 0 && rr < g.CH + 2 * kRing && w < g.wpr) d.bits[(int64_t)rr * g.wpr + w] = bits;
}

template <class Src>
__global__ void __launch_bounds__(256) k_coarsen(Src src, const int64_t* __restrict__ tab, Shared sh) {
  __shared__ uint32_t mask[kCoarsenRows * kCoarsenMaxS][kCoarsenWords];
  int64_t local;
  const int ii = src.find(blockIdx.x, tab, local);
  const Img& d = src.img(ii);
  const Geo g = d.g;
  const int nbx = (g.wpr + 7) / 8;
  const int bx = (int)local % nbx, ry = (int)local / nbx;  // block index of an image: 32 bits
  if (blockIdx.x == 0 && threadIdx.x < 8) sh.ctr[threadIdx.x] = 0;
  if (local == 0 && threadIdx.x == 0) sh.imgerr[ii] = 0;
  // look-back words and size slots of the fused path start at zero
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < sh.nbands; q += (int64_t)gridDim.x * blockDim.x)
    sh.band[q] = 0ull;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < kSizeWords * (int64_t)sh.n;
       q += (int64_t)gridDim.x * blockDim.x)
    sh.sizes[q] = 0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < kSegSlots * (int64_t)sh.n;
       q += (int64_t)gridDim.x * blockDim.x)
    sh.segacc[q] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x < kDenseLists) sh.dctr[threadIdx.x] = 0ull;
  if (g.s == 2 && (((uintptr_t)d.bm | (uintptr_t)g.stride) & 15u) == 0) {  // uniform per image
    coarsen_s2(d, g, (int)local % nbx, (int)local / nbx);
    return;
  }
  const int s = g.s;
  const int rr0 = ry * kCoarsenRows;                 // first stored row
  const int C0 = 256 * bx - kRingC;                  // first coarse column of the block
  const int R0 = rr0 - kRing;                        // first coarse row
  const int xa = s * max(C0, 0), xb = min(s * (C0 + 256), g.W);  // pixel columns
  const int pa = s * max(R0, 0), pb = min(s * (R0 + kCoarsenRows), g.H);  // pixel rows
  const int npr = max(pb - pa, 0);
  const int nw = (xb - xa + 15 + s + 31) / 32 + 2;
  for (int t = threadIdx.x; t < npr * nw; t += blockDim.x) mask[t / nw][t - (t / nw) * nw] = 0u;
  __syncthreads();
  if (xb > xa && npr > 0) {
    // 16-byte chunks covering bytes xa .. xb-1 of each pixel row; bit
    // (x - xa + 15) of the row mask = pixel x is foreground
    const int nchm = (xb - xa + 15) / 16 + 1;  // chunks per row, at most
    for (int t = threadIdx.x; t < npr * nchm; t += blockDim.x) {
      const int pr = t / nchm, q = t - pr * nchm;
      const uint8_t* row = d.bm + (int64_t)(pa + pr) * g.stride;
      const uintptr_t lo = ((uintptr_t)(row + xa)) & ~(uintptr_t)15;
      const uintptr_t hi = ((uintptr_t)(row + xb - 1)) & ~(uintptr_t)15;
      if (lo + 16 * (uintptr_t)q <= hi) {
        const uint4 v = *reinterpret_cast<const uint4*>(lo + 16 * (uintptr_t)q);
        const int rel = (int)((lo + 16 * (uintptr_t)q) - (uintptr_t)(row + xa));  // pixel of byte 0, minus xa
        // bit j = byte j is nonzero (four bytes per word at once), then only
        // the bytes of pixels xa .. xb-1 are kept
        auto nz4 = [](uint32_t w) {
          uint32_t t = (((w & 0x7f7f7f7fu) + 0x7f7f7f7fu) | w) & 0x80808080u;
          t >>= 7;
          return (t | (t >> 7) | (t >> 14) | (t >> 21)) & 15u;
        };
        const int blo = max(0, -rel), bhi = min(16, xb - xa - rel);
        const uint32_t inmask = bhi > blo ? (((1u << bhi) - 1u) & ~((1u << blo) - 1u)) : 0u;
        const uint32_t bits = (nz4(v.x) | (nz4(v.y) << 4) | (nz4(v.z) << 8) | (nz4(v.w) << 12)) & inmask;
        if (bits) {
          const int p = rel + 15;  // >= 0
          const uint64_t sh64 = (uint64_t)bits << (p & 31);
          atomicOr(&mask[pr][p >> 5], (uint32_t)sh64);
          if (sh64 >> 32) atomicOr(&mask[pr][(p >> 5) + 1], (uint32_t)(sh64 >> 32));
        }
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int cc = 256 * bx + threadIdx.x;  // stored column
  const int C = cc - kRingC;
  const int nrows = g.CH + 2 * kRing;
  for (int r = 0; r < kCoarsenRows; ++r) {
    const int rr = rr0 + r;
    if (rr >= nrows) break;
    const int R = rr - kRing;
    int fg = 0;
    if (C >= 0 && C < g.CW && R >= 0 && R < g.CH) {
      const int x0 = s * C - xa + 15;  // bit of the block's first pixel
      int cnt = 0;
      for (int dr = 0; dr < s; ++dr) {
        const int pr = s * R + dr - pa;
        if (pa + pr >= g.H) break;
        const uint64_t m = (uint64_t)mask[pr][x0 >> 5] | ((uint64_t)mask[pr][(x0 >> 5) + 1] << 32);
        cnt += __builtin_popcountll((m >> (x0 & 31)) & ((1ull << s) - 1ull));
      }
      fg = 2 * cnt >= s * s;
    }
    const unsigned long long mm = __ballot(fg);
    if ((lane & 63) < 2 && (cc & ~63) / 32 + lane < g.wpr)
      d.bits[(int64_t)rr * g.wpr + (cc & ~63) / 32 + lane] = (uint32_t)(mm >> (32 * lane));
  }
}

// Boundary segments of each image: a marching-squares cell has one segment per
// foreground->background step of its corners in positive order, and every pair
// of 4-adjacent samples is walked once in each direction by the two cells that
// share it, so the count is the number of 4-adjacent sample pairs that differ
// (ring included).  A block sums a run of stored raster rows (the image's rows
// split over as many blocks as it has 16-row grid bands), one thread per word.
template <class Src>
__global__ void __launch_bounds__(256) k_segcount(Src src, const int64_t* __restrict__ tab, Shared sh) {
  __shared__ int part[256 / 64];
  int64_t local;
  const int ii = src.find(blockIdx.x, tab, local);
  const Img& d = src.img(ii);
  const Geo g = d.g;
  const int nb = (g.NK + 15) / 16;
  const int nrows = g.CH + 2 * kRing;
  const int rpb = (nrows + nb - 1) / nb;
  const int r0 = (int)local * rpb, r1 = min(r0 + rpb, nrows);
  // the row table: grid rows 16 local .. 16 local + 15 (the last block also
  // the padding rows past the grid)
  {
    const int k0 = 16 * (int)local, k1 = (int)local == nb - 1 ? g.NK + kRowPad : k0 + 16;
    for (int k = k0 + (int)threadIdx.x; k < k1; k += 256) d.rows[k] = row_table_entry(g, k);
  }
  // the column table: window column and x reach of column i in rows of parity o
  for (int j = (int)local * 256 + (int)threadIdx.x; j < 2 * g.NI; j += nb * 256) {
    const int i = j >> 1, o = j & 1;
    const int X = g.X0 + 4 * g.h * i + 2 * g.h * o, Clo = clo_of(g, X);
    int x0, x1;
    owner_xreach(g, X, Clo, x0, x1);
    d.cols[j] = (uint32_t)(Clo + 8) | ((uint32_t)x0 << 24) | ((uint32_t)x1 << 28);
  }
  int n = 0;
  for (int t = threadIdx.x; t < (r1 - r0) * g.wpr; t += 256) {
    const int rr = r0 + t / g.wpr, w = t - (t / g.wpr) * g.wpr;
    const uint32_t* row = d.bits + (int64_t)rr * g.wpr;
    const uint32_t x = row[w], xn = w + 1 < g.wpr ? row[w + 1] : 0u;
    const uint32_t xd = rr + 1 < nrows ? row[g.wpr + w] : 0u;
    n += __builtin_popcount(x ^ ((x >> 1) | (xn << 31))) + __builtin_popcount(x ^ xd);
  }
  n = __builtin_amdgcn_readlane(wave_incl_scan_dpp(n), 63);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int tot = part[0] + part[1] + part[2] + part[3];
    // one atomic per block, spread over the image's slots (summed by segment_total)
    if (tot) atomicAdd(&sh.segacc[kSegSlots * (int64_t)ii + (blockIdx.x & (kSegSlots - 1))], (unsigned long long)tot);
  }
}

__device__ __forceinline__ long long segment_total(const Shared& sh, int ii) {
  long long t = 0;
  for (int j = 0; j < kSegSlots; ++j) t += (long long)sh.segacc[kSegSlots * (int64_t)ii + j];
  return t;
}

// Stage the coarse-raster window of a tile (cell rows rlo .. rhi, owner
// columns cfirst .. clast) in LDS; returns the view.  Sizes are checked on the
// host (tile_window_fits).
__device__ __forceinline__ Bits stage_window(const Geo& g, const uint32_t* __restrict__ bits, uint32_t* win, int rlo,
                                             int rhi, int cfirst, int clast) {
  const int x0 = g.X0 + 4 * g.h * cfirst, x1 = g.X0 + 4 * g.h * clast + 2 * g.h;
  const int wlo = (clo_of(g, x0) + kRingC) >> 5;
  const int whi = ((clo_of(g, x1) + 2 + kRingC) >> 5) + 1;
  const int nw = whi - wlo + 1, nr = rhi - rlo + 1;
  // t / nw as a multiply by ceil(2^16 / nw): exact for t * nw < 2^16
  // (t < kWinRows * kWinWords, nw <= kWinWords)
  const uint32_t inv = (65536u + (uint32_t)nw - 1u) / (uint32_t)nw;
  for (int t = threadIdx.x; t < nr * nw; t += blockDim.x) {
    const int r = (int)(((uint32_t)t * inv) >> 16), w = t - r * nw;
    win[r * nw + w] = bits[(int64_t)(rlo + r) * g.wpr + wlo + w];
  }
  Bits b;
  b.p = win;
  b.wpr = nw;
  b.rr0 = rlo;
  b.cc0 = 32 * wlo;
  return b;
}

// Popcount of the bits of m below this lane.
__device__ __forceinline__ int lanes_below(unsigned long long m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    T u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}

// ---------------------------------------------------------------------------
// Count one tile: rows k0 .. k0+RB-1, owners c0 .. c0+kCB-1.  Uniform windows
// are counted from one bit; the other owners are checked against the
// segments of their block: quiet ones (no segment reaches them) are counted
// here, slow ones get a slot in the tile's record region (their position is
// written into it for the dense classification) or, beyond the region's
// capacity, keep the queued mark for k_slow.  Every owner's code goes to the
// owner map; the per-row counts of the owners counted here go to acc_out.
// ---------------------------------------------------------------------------
template <int RB>
struct CountLds {
  int acc[RB][4];
  uint32_t u0[RB][kWinWords], u1[RB][kWinWords];  // uniform-window masks per row
  alignas(8) uint16_t code[RB][kCB];
  int rowR[RB];
  uint32_t rowp[RB];     // row_info of each row (reach in y, row signs)
  uint32_t xc[2][kCB];   // per column and row parity: Clo - (window's first column) | x0 << 16 | x1 << 20
  uint16_t q1[RB * kCB];  // non-uniform owners, RB * 64 entries per wave
  uint16_t q2[RB * kCB];
  int2 wacc[kThreads / 64][RB];  // per wave and row: vertices and triangles of its uniform owners
  int qn[kThreads / 64];         // per wave: entries in q1
  int n2;
  unsigned dbase;
  uint32_t win[kWinRows * kWinWords];
};

// Rows k0 .. k0+RB-1 of column block cb.  With hdst, the codes of the last
// row go to hdst[c] instead of the owner map (the persistent kernel counts
// the first row of the next band that way without writing it).  Slow owners
// beyond the record region keep the queued mark (0x8000) for k_slow (the
// persistent kernel's regions hold every owner of a tile), which keeps this
// routine free of the classification's registers.
template <int RB, bool kDense = false>
__device__ __forceinline__ void count_tile(const Img& d, const Geo& g, int ii, int64_t tile, int k0, int cb,
                                           const Shared& sh, CountLds<RB>& L, int4* acc_out,
                                           uint16_t* __restrict__ hdst) {
  const int c0 = cb * kCB;
  const int lane = threadIdx.x & 63;
  if (threadIdx.x < RB) {
    // the row table holds every row a tile reaches (kRowPad rows past the grid)
    const RowT& rt = d.rows[k0 + threadIdx.x];
    L.rowR[threadIdx.x] = rt.R;
    L.rowp[threadIdx.x] = rt.pk;
    L.acc[threadIdx.x][0] = L.acc[threadIdx.x][1] = L.acc[threadIdx.x][2] = L.acc[threadIdx.x][3] = 0;
  }
  if (threadIdx.x == 0) L.n2 = 0;
  __syncthreads();
  const int klast = min(k0 + RB, g.NK) - 1;
  const Bits bw = stage_window(g, d.bits, L.win, L.rowR[0] + kRing, L.rowR[klast - k0] + 2 + kRing, c0,
                               min(c0 + kCB, g.NI) - 1);
  __syncthreads();
  const uint32_t inv = (65536u + (uint32_t)bw.wpr - 1u) / (uint32_t)bw.wpr;  // as in stage_window
  for (int t = threadIdx.x; t < (klast - k0 + 1) * bw.wpr; t += kThreads) {
    const int r = (int)(((uint32_t)t * inv) >> 16), w = t - r * bw.wpr;
    window_masks_word(bw, L.rowR[r] + kRing, w, L.u0[r][w], L.u1[r][w]);
  }
  __syncthreads();
  // uniform windows, one owner per thread; the others are queued.  A thread
  // keeps its column, so its window column depends only on the row parity.
  const int c = c0 + threadIdx.x;
  int wcol[2];
  const uint2 ce = c < g.NI ? reinterpret_cast<const uint2*>(d.cols)[c] : make_uint2(8u, 0u);
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    const uint32_t e = o ? ce.y : ce.x;
    wcol[o] = (int)(e & 0xffffffu) - 8 + kRingC - bw.cc0;
    L.xc[o][threadIdx.x] = (uint32_t)wcol[o] | (((e >> 24) & 15u) << 16) | ((e >> 28) << 20);
  }
  // away from the grid edges both owned triangles exist for every owner, so a
  // uniform owner's counts are constants and a row's sums are popcounts
  const bool interior = k0 + RB < g.NK && c0 >= 1 && c0 + kCB < g.NI;
  const bool both = (g.flags & 1u) != 0;
  const uint32_t code_fg = map_code(fast_info_k(g, k0, c0 + 1, 1)), code_bg = map_code(fast_info_k(g, k0, c0 + 1, 0));
  // each wave queues its non-uniform owners in its own part of q1 (ballot and
  // mbcnt, no atomics) and keeps its rows' counts of uniform owners in
  // registers (lane r those of row r), handed over in wacc
  uint16_t* const qw = L.q1 + (threadIdx.x >> 6) * (RB * 64);
  int qn = 0, rv = 0, rt = 0;
  for (int r = 0; r < RB; ++r) {
    const int k = k0 + r;
    if (k >= g.NK) break;  // uniform
    int kind = 1;          // positions beyond the grid: no owner, nothing counted
    if (c < g.NI) {
      const int wc = wcol[k & 1], w = wc >> 5, sh = wc & 31;
      kind = (int)((L.u0[r][w] >> sh) & 1u) | ((int)((L.u1[r][w] >> sh) & 1u) << 1);
    }
    // a non-uniform owner's code is written again below
    int nv, nt;
    if (interior) {
      L.code[r][threadIdx.x] = (uint16_t)(kind == 2 ? code_fg : code_bg);
      // vertices: one per counted owner; triangles: two
      nv = (int)__popcll(__ballot(both ? kind != 0 : kind == 2));
      nt = 2 * nv;
    } else {
      int p = 0;  // vertices | triangles << 16
      if (c < g.NI && kind != 0) {
        const uint32_t fi = fast_info_k(g, k, c, kind >> 1);
        p = info_nv(fi) | (info_nt(fi) << 16);
        L.code[r][threadIdx.x] = (uint16_t)map_code(fi);
      }
      p = __builtin_amdgcn_readlane(wave_incl_scan_dpp(p), 63);
      nv = p & 0xffff;
      nt = p >> 16;
    }
    const unsigned long long mnu = __ballot(kind == 0);
    if (kind == 0) qw[qn + lanes_below(mnu)] = (uint16_t)(r * kCB + threadIdx.x);
    qn += (int)__popcll(mnu);
    rv = lane == r ? nv : rv;
    rt = lane == r ? nt : rt;
  }
  if (lane < RB) L.wacc[threadIdx.x >> 6][lane] = make_int2(rv, rt);
  if (lane == 0) L.qn[threadIdx.x >> 6] = qn;
  __syncthreads();
  if (threadIdx.x < RB) {
    int sv = 0, st = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
      sv += L.wacc[w][threadIdx.x].x;
      st += L.wacc[w][threadIdx.x].y;
    }
    atomicAdd(&L.acc[threadIdx.x][0], sv);
    atomicAdd(&L.acc[threadIdx.x][1], st);
  }
  static_assert(kThreads / 64 == 4, "four waves");
  const int p1 = L.qn[0], p2 = p1 + L.qn[1], p3 = p2 + L.qn[2], n1 = p3 + L.qn[3];
  // non-uniform windows: quiet owners (no segment reaches them) or slow ones
  for (int q = threadIdx.x; q < n1; q += kThreads) {
    const int w = (q >= p1) + (q >= p2) + (q >= p3);
    const int e = L.q1[w * (RB * 64) + q - (w == 0 ? 0 : (w == 1 ? p1 : (w == 2 ? p2 : p3)))];
    const int r = e / kCB, col = e - r * kCB, c = c0 + col;
    const int k = k0 + r;
    const uint32_t xc = L.xc[k & 1][col];
    const Frame f = owner_frame_at(g, bw, k, c, L.rowR[r], (int)(xc & 0xffffu) - kRingC + bw.cc0);
    uint32_t fi = 0;
    if (needs_slow(g, f, (int)((xc >> 16) & 15u), (int)((xc >> 20) & 15u), L.rowp[r], fi)) {
      L.q2[atomicAdd(&L.n2, 1)] = (uint16_t)e;
      L.code[r][e - r * kCB] = 0x8000;
    } else {
      L.code[r][e - r * kCB] = (uint16_t)map_code(fi);
      atomicAdd(&L.acc[r][0], info_nv(fi));
      atomicAdd(&L.acc[r][1], info_nt(fi));
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sh.tile_n[tile] = L.n2;
    // list tile mod kDenseLists, so that no counter takes every tile's atomic
    if (kDense && L.n2)
      L.dbase = (unsigned)((tile & (kDenseLists - 1)) * sh.dcap +
                           (int64_t)atomicAdd(&sh.dctr[tile & (kDenseLists - 1)],
                                              (unsigned long long)min((int64_t)L.n2, sh.tcap)));
  }
  if (kDense) __syncthreads();
  for (int q = threadIdx.x; q < L.n2; q += kThreads) {
    const int e = L.q2[q], r = e / kCB, c = c0 + (e - r * kCB);
    const int k = k0 + r;
    if (q < sh.tcap) {
      // the owner's position for the dense pass
      sh.rec[tile * sh.tcap + q].x = (uint64_t)c | ((uint64_t)k << 24) | ((uint64_t)ii << 48);
      if (kDense) sh.dense[L.dbase + q] = (uint32_t)(tile * sh.tcap + q);
    }
  }
  __syncthreads();
  // the tile's owner codes, four per lane and row
  for (int t = threadIdx.x; t < RB * (kCB / 4); t += kThreads) {
    const int r = t / (kCB / 4), c = c0 + 4 * (t - r * (kCB / 4));
    const int k = k0 + r;
    if (k >= g.NK || c >= g.NI) continue;
    const bool to_h = hdst != nullptr && r == RB - 1;
    uint16_t* dst = to_h ? hdst + c : d.omap + (int64_t)k * g.NI + c;
    const uint16_t* src = &L.code[r][c - c0];
    if (!to_h && c + 4 <= g.NI && ((((int64_t)k * g.NI + c) & 3) == 0)) {
      *reinterpret_cast<uint2*>(dst) = *reinterpret_cast<const uint2*>(src);
    } else {
      for (int u = 0; u < 4 && c + u < g.NI; ++u) dst[u] = src[u];
    }
  }
  __syncthreads();
  if (threadIdx.x < RB && k0 + (int)threadIdx.x < g.NK) {
    const int r = threadIdx.x;
    acc_out[r] = make_int4(L.acc[r][0], L.acc[r][1], L.acc[r][2], L.acc[r][3]);
    if (L.acc[r][3]) atomicOr(&sh.imgerr[ii], 1);
  }
}

// Eight waves per SIMD: the target also caps the scalar registers (a few
// spill to vector lanes), which an uncapped build exceeds.
template <class Src, int RB>
__global__ void __launch_bounds__(kThreads, 8) k_count(Src src, const int64_t* __restrict__ tab, Shared sh) {
  __shared__ CountLds<RB> L;
  __shared__ int4 out[RB];
  int64_t local;
  const int ii = src.find(blockIdx.x, tab, local);
  const Img& d = src.img(ii);
  const Geo g = d.g;
  const int cb = (int)local % g.NCB, ky = (int)local / g.NCB;  // tile index of an image: 32 bits
  count_tile<RB, true>(d, g, ii, (int64_t)blockIdx.x, ky * RB, cb, sh, L, out, nullptr);
  __syncthreads();
  const int k = ky * RB + (int)threadIdx.x;
  if (threadIdx.x < RB && k < g.NK) sh.seg_cnt[d.seg0 + (int64_t)k * g.NCB + cb] = out[threadIdx.x];
}

// ---------------------------------------------------------------------------
// Slow owners with a record, densely: one lane per entry of the lists the count
// tiles filled (in whatever order their atomics ran), so that waves are full
// whatever the spread of slow owners over tiles.  Each record carries the
// owner's position and its row's cell row; the classification replaces it in
// place (with the owner's place in its tile in the spare bits 48..63) and the
// owner's code goes to the owner map.  Held to 64 VGPRs (eight waves per
// SIMD): faster than the 78 it takes unbounded (six waves).
// ---------------------------------------------------------------------------
template <class Src, int RB>
__global__ void __launch_bounds__(kThreads, 8) k_slow_dense(Src src, Shared sh) {
  __shared__ int64_t pre[kDenseLists + 1];
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int l = 0; l < kDenseLists; ++l) {
      pre[l] = t;
      t += (int64_t)sh.dctr[l];
    }
    pre[kDenseLists] = t;
  }
  __syncthreads();
  const int64_t n = pre[kDenseLists];
  for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < n; j += (int64_t)gridDim.x * kThreads) {
    int lo = 0, hi = kDenseLists - 1;  // list: largest l with pre[l] <= j
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= j) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t idx = sh.dense[lo * sh.dcap + (j - pre[lo])];
    const SlowRec P = sh.rec[idx];
    const int k = (int)((P.x >> 24) & 0xffffffu), c = (int)(P.x & 0xffffffu), ii = (int)(P.x >> 48);
    const Img& d = src.img(ii);
    const Geo g = d.g;
    Bits b;
    b.p = d.bits;
    b.wpr = g.wpr;
    b.rr0 = 0;
    b.cc0 = 0;
    const RowT& rt = d.rows[k];
    const Frame f = owner_frame(g, b, k, c, rt.R);
    Slow sr;
    slow_classify(g, f, rt, d.rows[k + 1].FL, sr);
    SlowRec R = pack_slow(sr);
    R.x |= (uint64_t)(((k & (RB - 1)) << 8) | (c & (kCB - 1))) << 48;
    sh.rec[idx] = R;
    d.omap[(int64_t)k * g.NI + c] = (uint16_t)map_code(sr.info);
    if (info_err(sr.info)) atomicOr(&sh.imgerr[ii], 1);
  }
}

// ---------------------------------------------------------------------------
// Per count tile, after the dense pass: the per-row sums of its slow owners'
// counts (from their records), and the slow owners beyond its record region
// (the tile queued more than the region holds; they still carry the queued
// mark 0x8000), classified here without a record.
// ---------------------------------------------------------------------------
template <class Src, int RB>
__global__ void __launch_bounds__(64) k_slow_tiles(Src src, const int64_t* __restrict__ tab, Shared sh) {
  __shared__ unsigned long long acc[RB];
  __shared__ uint32_t hasrec[RB * kCB / 32];
  __shared__ int rowR[RB];
  const int64_t tile = blockIdx.x;
  const int64_t nq = sh.tile_n[tile];
  const bool over = nq > sh.tcap;  // uniform
  const int nrec = (int)min(nq, sh.tcap);
  int64_t local;
  const int ii = src.find(blockIdx.x, tab, local);
  const Img& d = src.img(ii);
  const Geo g = d.g;
  const int cb = (int)local % g.NCB, ky = (int)local / g.NCB;  // tile index of an image: 32 bits
  if (threadIdx.x < RB) {
    acc[threadIdx.x] = 0ull;
    if (over) rowR[threadIdx.x] = d.rows[ky * RB + threadIdx.x].R;
  }
  if (over)
    for (int t = threadIdx.x; t < RB * kCB / 32; t += 64) hasrec[t] = 0u;
  __syncthreads();
  // owners with a record (classified by the dense pass: their place is in
  // bits 48..63)
  for (int q = threadIdx.x; q < nrec; q += 64) {
    const SlowRec R = sh.rec[tile * sh.tcap + q];
    atomicAdd(&acc[(int)(R.x >> 56)], pack_counts(R.info));
    if (over) {
      const int e = (int)(R.x >> 56) * kCB + (int)((R.x >> 48) & 255u);
      atomicOr(&hasrec[e >> 5], 1u << (e & 31));
    }
  }
  __syncthreads();
  if (!over) {
    const int k = ky * RB + (int)threadIdx.x;
    if (threadIdx.x < RB && k < g.NK) sh.seg_slow[d.seg0 + (int64_t)k * g.NCB + cb] = acc[threadIdx.x];
    return;
  }
  Bits b;
  b.p = d.bits;
  b.wpr = g.wpr;
  b.rr0 = 0;
  b.cc0 = 0;
  for (int e = threadIdx.x; e < RB * kCB; e += 64) {
    const int r = e / kCB, k = ky * RB + r, c = cb * kCB + (e - r * kCB);
    if (k >= g.NK || c >= g.NI || ((hasrec[e >> 5] >> (e & 31)) & 1u)) continue;
    if (d.omap[(int64_t)k * g.NI + c] != 0x8000u) continue;
    const Frame f = owner_frame(g, b, k, c, rowR[r]);
    Slow sr;
    slow_classify(g, f, d.rows[k], d.rows[k + 1].FL, sr);
    d.omap[(int64_t)k * g.NI + c] = (uint16_t)map_code(sr.info);
    atomicAdd(&acc[r], pack_counts(sr.info));
    if (info_err(sr.info)) atomicOr(&sh.imgerr[ii], 1);
  }
  __syncthreads();
  const int k = ky * RB + (int)threadIdx.x;
  if (threadIdx.x < RB && k < g.NK) sh.seg_slow[d.seg0 + (int64_t)k * g.NCB + cb] = acc[threadIdx.x];
}

// ---------------------------------------------------------------------------
// Exclusive scan of the per-segment (nv, nt, ncut) over the whole call.
// ---------------------------------------------------------------------------
// block-wide exclusive scan of (a, b) over kScanThreads threads; returns totals
__device__ void block_excl_scan2(long long& a, long long& b, long long* sa, long long* sb, long long& ta,
                                 long long& tb) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  long long ia = wave_incl_scan(a, lane), ib = wave_incl_scan(b, lane);
  if (lane == 63) {
    sa[wv] = ia;
    sb[wv] = ib;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int nw = blockDim.x >> 6;
    long long xa = threadIdx.x < nw ? sa[threadIdx.x] : 0, xb = threadIdx.x < nw ? sb[threadIdx.x] : 0;
    long long ya = wave_incl_scan(xa, lane), yb = wave_incl_scan(xb, lane);
    if (threadIdx.x < nw) {
      sa[threadIdx.x] = ya - xa;
      sb[threadIdx.x] = yb - xb;
    }
    if (threadIdx.x == nw - 1) {
      sa[32] = ya;
      sb[32] = yb;
    }
  }
  __syncthreads();
  a = ia - a + sa[wv];
  b = ib - b + sb[wv];
  ta = sa[32];
  tb = sb[32];
  __syncthreads();
}

__device__ __forceinline__ void seg_counts(const Shared& sh, int64_t j, long long& a, long long& b, long long& c) {
  const int4 v = sh.seg_cnt[j];
  const unsigned long long s = sh.seg_slow[j];
  a = v.x + (long long)(s & 0x1fffffull);
  b = v.y + (long long)((s >> 21) & 0x1fffffull);
  c = v.z + (long long)(s >> 42);
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(Shared sh) {
  __shared__ long long sa[33], sb[33];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  long long a = 0, b = 0, c = 0;
  for (int q = 0; q < 4; ++q) {
    const int64_t j = base + (int64_t)threadIdx.x * 4 + q;
    if (j < sh.nseg) {
      long long x, y, z;
      seg_counts(sh, j, x, y, z);
      a += x;
      b += y;
      c += z;
    }
  }
  long long ta, tb, tc, dummy;
  block_excl_scan2(a, b, sa, sb, ta, tb);
  long long z = 0;
  block_excl_scan2(c, z, sa, sb, tc, dummy);
  if (threadIdx.x == 0) sh.blk[blockIdx.x] = make_longlong4(ta, tb, tc, 0);
}

__global__ void __launch_bounds__(kScanThreads) k_scan_blocks(Shared sh) {
  __shared__ long long sa[33], sb[33];
  long long ra = 0, rb = 0, rc = 0;
  for (int base = 0; base < sh.nblk; base += kScanThreads) {
    const int j = base + threadIdx.x;
    longlong4 v = j < sh.nblk ? sh.blk[j] : make_longlong4(0, 0, 0, 0);
    long long a = v.x, b = v.y, ta, tb;
    block_excl_scan2(a, b, sa, sb, ta, tb);
    long long c = v.z, z = 0, tc, dd;
    block_excl_scan2(c, z, sa, sb, tc, dd);
    if (j < sh.nblk) sh.blk[j] = make_longlong4(ra + a, rb + b, rc + c, 0);
    ra += ta;
    rb += tb;
    rc += tc;
  }
  if (threadIdx.x == 0) sh.seg_off[sh.nseg] = make_longlong4(ra, rb, rc, 0);
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(Shared sh) {
  __shared__ long long sa[33], sb[33];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  long long va[4], vb[4], vc[4];
  long long a = 0, b = 0, c = 0;
  for (int q = 0; q < 4; ++q) {
    const int64_t j = base + (int64_t)threadIdx.x * 4 + q;
    va[q] = vb[q] = vc[q] = 0;
    if (j < sh.nseg) seg_counts(sh, j, va[q], vb[q], vc[q]);
    a += va[q];
    b += vb[q];
    c += vc[q];
  }
  long long ta, tb, tc, dd;
  block_excl_scan2(a, b, sa, sb, ta, tb);
  long long z = 0;
  block_excl_scan2(c, z, sa, sb, tc, dd);
  const longlong4 bo = sh.blk[blockIdx.x];
  a += bo.x;
  b += bo.y;
  c += bo.z;
  for (int q = 0; q < 4; ++q) {
    const int64_t j = base + (int64_t)threadIdx.x * 4 + q;
    if (j < sh.nseg) sh.seg_off[j] = make_longlong4(a, b, c, 0);
    a += va[q];
    b += vb[q];
    c += vc[q];
  }
}

// Per-image sizes and status from the scanned offsets (one thread per image).
template <class Src>
__device__ __forceinline__ void image_totals(const Img& d, const Shared& sh, long long& nv, long long& nt,
                                             long long& nc) {
  const int64_t nsegi = (int64_t)d.g.NK * d.g.NCB;
  const longlong4 a = sh.seg_off[d.seg0], b = sh.seg_off[d.seg0 + nsegi];
  nv = b.x - a.x;
  nt = b.y - a.y;
  nc = b.z - a.z;
}

__device__ __forceinline__ int64_t image_status(const Img& d, int err, long long nv, long long nt) {
  if (err) return SBMT_E_PROTOCOL;
  if (nv > 0x7fffffffLL) return SBMT_E_INDEX_OVERFLOW;
  if (nv > d.vcap || nt > d.tcap) return SBMT_E_CAPACITY;
  return SBMT_OK;
}

template <class Src>
__global__ void k_sizes(Src src, Shared sh, int64_t* __restrict__ user) {
  const int ii = blockIdx.x * blockDim.x + threadIdx.x;
  if (ii >= sh.n) return;
  const Img& d = src.img(ii);
  long long nv, nt, nc;
  image_totals<Src>(d, sh, nv, nt, nc);
  const int64_t st = image_status(d, sh.imgerr[ii], nv, nt);
  int64_t* o = sh.sizes + kSizeWords * (int64_t)ii;
  o[0] = nv;
  o[1] = nt;
  o[2] = nc;
  o[3] = st;
  o[4] = segment_total(sh, ii);
  if (user) {
    int64_t* u = user + kSizeWords * (int64_t)ii;
    u[0] = nv;
    u[1] = nt;
    u[2] = nc;
    u[3] = st;
    u[4] = o[4];
  }
}

// ---------------------------------------------------------------------------
// Emission of one tile: rows k0 .. k0+RB-1, owners c0 .. c0+kCB-1.
//   1. owner codes of the tile plus a one-row / one-column halo (from the
//      owner map) and the tile's slow-owner records;
//   2. prefix sums of the counts of every row in LDS plus the segment bases
//      give each owner's first vertex and triangle id and its neighbours' ids;
//   3. fast and quiet owners are emitted (a vertex per thread, each wave's
//      triangles in output order), then the slow owners of the tile densely
//      from their records (those without a record: see kEmitMissing).
// bv[0..RB] (image-local first vertex of each row's segment, row RB = the halo
// row) and tb[0..RB-1] (first triangle) come from the caller: written before
// the call (the persistent kernel) or by the `bases` callback.
// ---------------------------------------------------------------------------
template <int RB>
struct EmitLds {
  static constexpr int W = kCB + 2;  // columns c0-1 .. c0+kCB
  static constexpr int kSlowChunk = 128;  // slow-owner records staged at a time
  static constexpr int kSlowItems = 10;   // outputs of one kind per record, at most
  uint16_t info[RB + 1][W];  // owner codes (0 outside the grid)
  int16_t voff[RB + 1][W];   // first vertex of each owner, from bv of its row
  int16_t toff[RB][W];       // first triangle of each owner, from tb of its row
  uint32_t hasrec[RB * kCB / 32];
  int rowR[RB + 1];
  double rowy[RB + 1];  // lat_y of each row
  int bv[RB + 1];
  long long tb[RB];
  int rowv[RB + 1];  // vertices of each row's kCB owners
  union {
    struct {
      SlowRec srec[kSlowChunk];
      uint16_t sitem[kSlowChunk * kSlowItems];  // record | output number << 8
    } r;
    uint32_t stage[4][kThreads / 64][64];  // strip emission: a wave's triangles by output slot (a, b, c, tag)
  } x;
  uint16_t lut[15 * 3 * 2 * 5];              // emission table of the side mode
  uint8_t tslot[kThreads / 64][128];         // per wave: fast triangle rank -> lane << 1 | which
  int swt[kThreads / 64];
};

// Ids an owner of an emission tile needs (row r, LDS column col = owner
// column - c0 + 1, row parity o_), from the codes and offsets in LDS.
template <int RB>
__device__ __forceinline__ Nb tile_nb(const EmitLds<RB>& L, int r, int col, uint32_t f, int o_) {
  Nb nb;
  const int bv0 = L.bv[r], bv1 = L.bv[r + 1];
  nb.vid = bv0 + L.voff[r][col];
  nb.id_vr = bv0 + L.voff[r][col + 1];
  nb.id_vdl = bv1 + L.voff[r + 1][col + o_ - 1];
  nb.id_vdr = bv1 + L.voff[r + 1][col + o_];
  nb.b0 = nb.vid + info_self(f);
  nb.b1 = nb.b0 + info_n(f, 0);
  nb.b2 = nb.b1 + info_n(f, 1);
  const uint32_t fr = map_info(L.info[r][col + 1]);
  nb.b3 = nb.id_vr + info_self(fr) + info_n(fr, 0);
  const uint32_t fl = map_info(L.info[r + 1][col + o_ - 1]);
  nb.b4 = nb.id_vdl + info_self(fl);
  nb.bI = nb.b2 + info_n(f, 2);
  return nb;
}

// Slow owners of an emission tile from their records, kSlowChunk records at a
// time: the records and the lists of their output vertices and triangles go to
// LDS, then one lane writes one output (records of the halo row are skipped:
// the band below emits them).  Record q is held by thread q mod kThreads in
// held0 / held1 (q / kThreads = 0, 1) while q < kHold * kThreads.  Needs the tile's codes,
// offsets, row bases, cell rows and emission table in L.
constexpr int kHold = 2;
template <int RB>
__device__ __forceinline__ void emit_records(const Img& d, const Geo& g, int k0, int c0, int64_t tile,
                                             const Shared& sh, EmitLds<RB>& L, const SlowRec held0,
                                             const SlowRec held1, int nrec) {
  constexpr int kChunk = EmitLds<RB>::kSlowChunk;
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  Out out;
  out.v = d.verts;
  out.t = d.tris;
  out.c = d.codes;
  out.vbase = 0;
  out.tbase = 0;
  for (int ch = 0; ch * kChunk < nrec; ++ch) {
    const int qi = threadIdx.x & (kChunk - 1);
    const int q = ch * kChunk + qi;
    bool mine = false;
    int cnt = 0;  // vertices | triangles << 16
    if ((int)threadIdx.x / kChunk == ch % (kThreads / kChunk) && q < nrec) {
      const int j = ch / (kThreads / kChunk);
      SlowRec R;
      if (j < kHold) {
        // field by field, so that held[] stays in registers
        static_assert(kHold == 2, "two held records per thread");
        R.info = j == 0 ? held0.info : held1.info;
        R.tri = j == 0 ? held0.tri : held1.tri;
        R.x = j == 0 ? held0.x : held1.x;
      } else {
        R = sh.rec[tile * sh.tcap + q];
      }
      L.x.r.srec[qi] = R;
      mine = (int)(R.x >> 56) < RB;
      if (mine) cnt = info_nv(R.info) | (info_nt(R.info) << 16);
    }
    const int incl = wave_incl_scan_dpp(cnt);
    if (lane == 63) L.swt[wv] = incl;
    __syncthreads();
    int before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
      const int tw = L.swt[w];
      before += w < wv ? tw : 0;
      total += tw;
    }
    const int excl = before + incl - cnt;
    for (int i = 0; i < (cnt & 0xffff); ++i) L.x.r.sitem[(excl & 0xffff) + i] = (uint16_t)(qi | (i << 8));
    __syncthreads();
    for (int it = threadIdx.x; it < (total & 0xffff); it += kThreads) {
      const int item = L.x.r.sitem[it];
      const SlowRec R = L.x.r.srec[item & 255];
      const int r = (int)(R.x >> 56), col = (int)((R.x >> 48) & 255u) + 1;
      const Frame f = owner_place(g, k0 + r, c0 + col - 1, L.rowR[r]);
      emit_slow_vertex(g, f, R, item >> 8, L.bv[r] + L.voff[r][col], L.rowy[r], L.rowy[r + 1], out);
    }
    __syncthreads();
    for (int i = 0; i < (cnt >> 16); ++i) L.x.r.sitem[(excl >> 16) + i] = (uint16_t)(qi | (i << 8));
    __syncthreads();
    for (int it = threadIdx.x; it < (total >> 16); it += kThreads) {
      const int item = L.x.r.sitem[it];
      const SlowRec R = L.x.r.srec[item & 255];
      const int r = (int)(R.x >> 56), col = (int)((R.x >> 48) & 255u) + 1;
      const Nb nb = tile_nb(L, r, col, map_info(L.info[r][col]), (k0 + r) & 1);
      emit_slow_triangle(g, R, item >> 8, nb, L.tb[r] + L.toff[r][col], out, L.lut);
    }
    __syncthreads();
  }
}

// Owner info comes from the owner map (row RB, the halo row, from hcodes when
// given), slow owners' emission data from the records of count tile `tile`
// (each record carries the owner's place in the tile; records of the halo
// row, which the persistent kernel keeps in the same region, are skipped).
// What is emitted:
//   kEmitAll      everything, every slow owner from its record (the persistent
//                 kernel, whose record regions hold every owner of a tile);
//   kEmitRecords  fast and quiet owners and the slow owners with a record;
//   kEmitMissing  only the slow owners without a record (the count tile's
//                 record region was full; the count pass classified them).
constexpr int kEmitAll = 0, kEmitRecords = 1, kEmitMissing = 2;
// `bases(L)` fills L.bv[0..RB] and L.tb[0..RB-1] (see above); it is called
// once the tile's other loads are issued, so that its latency overlaps theirs.
template <int RB, int kMode = kEmitAll, class Bases>
__device__ __forceinline__ void emit_tile(const Img& d, const Geo& g, int k0, int cb, int64_t tile, const Shared& sh,
                                          EmitLds<RB>& L, const uint16_t* __restrict__ hcodes, Bases&& bases) {
  constexpr int W = EmitLds<RB>::W;
  constexpr int kLut = 15 * 3 * 2 * 5;
  static_assert(kLut <= 2 * kThreads, "two table entries per thread");
  const int c0 = cb * kCB;
  if (threadIdx.x <= RB) {  // read after step 2
    L.rowR[threadIdx.x] = d.rows[k0 + threadIdx.x].R;
    L.rowy[threadIdx.x] = lat_y(g, k0 + threadIdx.x);
  }
  Bits bw;
  bw.p = d.bits;
  bw.wpr = g.wpr;
  bw.rr0 = 0;
  bw.cc0 = 0;
  // 1. every wave loads the owner codes of its rows (wave w: rows w, w + 4,
  // ...; lane = column within each block of 64, lanes 0 and 1 also the
  // columns c0-1 and c0+kCB) and the tile's records, all loads first so that
  // their latencies overlap
  // the wave index is uniform: its rows' addresses are computed once per wave
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int kWaves = kThreads / 64;
  constexpr int kRowsW = (RB + 1 + kWaves - 1) / kWaves;
  constexpr int kU = kCB / 64;
  uint32_t codes[kRowsW][kU], edge[kRowsW];
  SlowRec held[kHold];
  bool hv[kHold];
  const int nrec = (int)min((int64_t)sh.tile_n[tile], sh.tcap);
  // 0xffff marks a position outside the grid (no owner code has all bits set)
  auto load_code = [&](int rr, int c) -> uint32_t {
    const int k = k0 + rr;
    if (k >= g.NK || c < 0 || c >= g.NI) return 0xffffu;
    return (rr == RB && hcodes) ? (uint32_t)hcodes[c] : (uint32_t)d.omap[(int64_t)k * g.NI + c];
  };
#pragma unroll
  for (int m = 0; m < kRowsW; ++m) {
    const int rr = wv + kWaves * m;
#pragma unroll
    for (int u = 0; u < kU; ++u) codes[m][u] = rr <= RB ? load_code(rr, c0 + 64 * u + lane) : 0xffffu;
    edge[m] = (rr <= RB && lane < 2) ? load_code(rr, lane == 0 ? c0 - 1 : c0 + kCB) : 0xffffu;
  }
#pragma unroll
  for (int j = 0; j < kHold; ++j) {
    const int q = threadIdx.x + j * kThreads;
    hv[j] = kMode != kEmitMissing && q < nrec;
    if (hv[j]) held[j] = sh.rec[tile * sh.tcap + q];
  }
  // the emission table of the side mode, to LDS in step 2
  const uint16_t* lt = (g.flags & 1u) ? &sbmt_lut_emit[0][0][0][0] : &sbmt_lut_emit_fg[0][0][0][0];
  const uint16_t lut0 = lt[threadIdx.x];
  const uint16_t lut1 = threadIdx.x + kThreads < kLut ? lt[threadIdx.x + kThreads] : 0;
  bases(L);
  // 2. per row: owner codes into LDS and the prefix sums, in four blocks of 64
  // consecutive columns (a DPP wave scan each; vertex and triangle counts of
  // a row segment stay below 2^16: packed)
  L.lut[threadIdx.x] = lut0;
  if (threadIdx.x + kThreads < kLut) L.lut[threadIdx.x + kThreads] = lut1;
#pragma unroll
  for (int m = 0; m < kRowsW; ++m) {
    const int rr = wv + kWaves * m;
    if (rr > RB) break;  // uniform per wave
    int carry = 0;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int col = 1 + 64 * u + lane;
      const uint32_t cd = codes[m][u];
      const uint32_t cv = cd != 0xffffu ? cd : 0u;
      L.info[rr][col] = (uint16_t)cv;
      // counts straight from the code: bit 7 is a chain vertex in a slow
      // owner's code and the inside bit in the others'
      const int p = __builtin_popcount(cv & ((cv & 0x8000u) ? 0x1ffu : 0x17fu)) |
                    ((int)(((cv >> 9) & 7u) + ((cv >> 12) & 7u)) << 16);
      const int incl = wave_incl_scan_dpp(p);
      const int e = carry + incl - p;
      L.voff[rr][col] = (int16_t)(e & 0xffff);
      if (rr < RB) L.toff[rr][col] = (int16_t)(e >> 16);
      carry += __builtin_amdgcn_readlane(incl, 63);
    }
    const uint32_t fe = edge[m] != 0xffffu ? map_info(edge[m]) : 0u;
    if (lane < 2) L.info[rr][lane == 0 ? 0 : W - 1] = (uint16_t)(edge[m] != 0xffffu ? edge[m] : 0u);
    const int nv_left = __builtin_amdgcn_readlane(info_nv(fe), 0);
    if (lane == 0) {
      L.voff[rr][0] = (int16_t)(-nv_left);
      L.voff[rr][W - 1] = (int16_t)(carry & 0xffff);
      L.rowv[rr] = carry & 0xffff;
    }
  }
  __syncthreads();
  auto neighbours = [&](int r, int col, uint32_t f, int o_) { return tile_nb(L, r, col, f, o_); };
  // 3. fast and quiet owners: each thread writes the vertex of its owner; the
  // wave's triangles are written in output order, lane j the j-th (so that a
  // store covers consecutive triangles); then the slow owners of the tile
  // from their records.
  const bool both = (g.flags & 1u) != 0;
  Out out;
  out.v = d.verts;
  out.t = d.tris;
  out.c = d.codes;
  out.vbase = 0;
  out.tbase = 0;
  for (int r = 0; r < RB && kMode != kEmitMissing; ++r) {
    const int k = k0 + r;
    if (k >= g.NK) break;
    const int o_ = k & 1;
    const int col = 1 + threadIdx.x;
    const int c = c0 + threadIdx.x;
    // the row segment's outputs start at uniform addresses: 32-bit offsets
    // from them (a row segment holds fewer than 2^16 of each)
    const int bvr = __builtin_amdgcn_readfirstlane(L.bv[r]), bvn = __builtin_amdgcn_readfirstlane(L.bv[r + 1]);
    const long long tbr = L.tb[r];
    const int64_t tbs = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(tbr >> 32)) << 32) |
                                  (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)tbr));
    char* const vrow = reinterpret_cast<char*>(d.verts + 2 * (int64_t)bvr);
    char* const trow = reinterpret_cast<char*>(d.tris + 3 * tbs);
    uint8_t* const crow = d.codes + tbs;
    const uint32_t f = c < g.NI ? map_info(L.info[r][col]) : 0u;
    const bool fast = c < g.NI && !info_slow(f);
    if (fast && info_self(f)) {
      double2 v;
      v.x = lat_x(g, g.X0 + 4 * g.h * c + 2 * g.h * o_);
      v.y = L.rowy[r];
      *reinterpret_cast<double2*>(vrow + (uint32_t)L.voff[r][col] * 16u) = v;
    }
    // ranks of the wave's fast triangles (at most two per owner)
    const int ntb = fast ? info_ntb(f) : 0, nf = ntb + (fast ? info_nta(f) : 0);
    const int incl = wave_incl_scan_dpp(nf);
    const int tot = __builtin_amdgcn_readlane(incl, 63), ex = incl - nf;
    uint8_t* const slot = L.tslot[wv];
    if (ntb) slot[ex] = (uint8_t)(lane << 1);
    if (nf > ntb) slot[ex + ntb] = (uint8_t)((lane << 1) | 1);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // at most two triangles per lane (ranks lane and lane + 64), their LDS
    // reads issued together and both kinds of triangle selected, not branched
    int e2[2];
    bool h2[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      h2[q] = lane + 64 * q < tot;
      e2[q] = h2[q] ? slot[lane + 64 * q] : 0;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = e2[q];
      const int ocol = 64 * wv + 1 + (e >> 1);
      const uint32_t of = map_info(L.info[r][ocol]);
      const int tof = L.toff[r][ocol];
      const int va = L.voff[r][ocol], vr = L.voff[r][ocol + 1];
      const int vdl = L.voff[r + 1][ocol + o_ - 1], vdr = L.voff[r + 1][ocol + o_];
      const bool second = (e & 1) != 0;
      const uint32_t u = (uint32_t)(uint16_t)tof + (second ? (uint32_t)info_ntb(of) : 0u);
      Tri3 t3;
      t3.a = bvr + va;
      t3.b = second ? bvr + vr : bvn + vdr;
      t3.c = bvn + (second ? vdr : vdl);
      if (h2[q]) {
        *reinterpret_cast<Tri3*>(trow + u * 12u) = t3;
        crow[u] = both && !info_fg(of) ? 0x80 : 0;
      }
    }
    // the next row's ranks reuse the slots
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // 4. slow owners from their records
  if (kMode != kEmitMissing) emit_records<RB>(d, g, k0, c0, tile, sh, L, held[0], held[1], nrec);
  __syncthreads();
  if (kMode == kEmitMissing) {
    // slow owners beyond the tile's record region were classified by the
    // count pass without a record: mark the recorded ones, classify the rest
    for (int t = threadIdx.x; t < RB * kCB / 32; t += kThreads) L.hasrec[t] = 0u;
    __syncthreads();
    for (int q = threadIdx.x; q < nrec; q += kThreads) {
      const int pos = (int)(sh.rec[tile * sh.tcap + q].x >> 48);
      if ((pos >> 8) >= RB) continue;
      const int e = (pos >> 8) * kCB + (pos & 255);
      atomicOr(&L.hasrec[e >> 5], 1u << (e & 31));
    }
    __syncthreads();
    for (int e = threadIdx.x; e < RB * kCB; e += kThreads) {
      const int r = e / kCB, col = e - r * kCB + 1;
      if (!info_slow(map_info(L.info[r][col])) || ((L.hasrec[e >> 5] >> (e & 31)) & 1u)) continue;
      const int k = k0 + r, c = c0 + col - 1;
      const Frame fr = owner_frame(g, bw, k, c, L.rowR[r]);
      Slow sr;
      slow_classify(g, fr, d.rows[k], d.rows[k + 1].FL, sr);
      const Nb nb = neighbours(r, col, map_info(L.info[r][col]), k & 1);
      emit_slow(g, fr, pack_slow(sr), nb, L.tb[r] + L.toff[r][col], out, L.lut);
    }
  }
}

// One count tile of the multi-kernel path: its image, the bases of its row
// segments, then emit_tile.
template <class Src, int RB, int kMode>
__device__ __forceinline__ void emit_count_tile(const Src& src, const int64_t* __restrict__ tab, const Shared& sh,
                                                int64_t tile, EmitLds<RB>& L) {
  int64_t local;
  const int ii = src.find(tile, tab, local);
  const Img& d = src.img(ii);
  const Geo g = d.g;
  long long nv, nt, nc;
  image_totals<Src>(d, sh, nv, nt, nc);
  if (image_status(d, sh.imgerr[ii], nv, nt) != SBMT_OK) return;  // uniform per block
  const int cb = (int)local % g.NCB, ky = (int)local / g.NCB;  // tile index of an image: 32 bits
  const int64_t nsegi = (int64_t)g.NK * g.NCB;
  const longlong4 base = sh.seg_off[d.seg0];
  emit_tile<RB, kMode>(d, g, ky * RB, cb, tile, sh, L, nullptr, [&](EmitLds<RB>& E) {
    if (threadIdx.x <= RB) {
      const int k = ky * RB + threadIdx.x;
      const longlong4 o = sh.seg_off[d.seg0 + (k < g.NK ? (int64_t)k * g.NCB + cb : nsegi)];
      E.bv[threadIdx.x] = (int)(o.x - base.x);
      if (threadIdx.x < RB) E.tb[threadIdx.x] = o.y - base.y;
    }
  });
}

// ---------------------------------------------------------------------------
// Emission of one count tile by strips (the multi-kernel path).  Wave w takes
// the owners c0 + 64 w + lane of every row of the tile and walks down the rows.
// A vertex id is the prefix of the vertex counts along its row (owner
// numbering), so the wave holds the prefixes of rows r and r+1 in registers
// and a fast owner's triangles need no lookup: vid(k, i+1) = vid(k, i) +
// nv(k, i), and the row below gives vid(k+1, i+o) and, one lane to the left,
// vid(k+1, i+o-1).  The tile's codes and offsets also go to LDS, where the slow
// owners, emitted afterwards from their records, find their neighbours' ids.
// ---------------------------------------------------------------------------
template <int RB>
struct StripLds {
  EmitLds<RB> e;
  int wtot[RB + 1][kThreads / 64];         // packed counts (nv | nt << 16) of each strip's rows
  int lastnv[RB + 1][kThreads / 64 + 1];   // nv of the owner left of each strip ([0]: column c0 - 1)
};

__device__ __forceinline__ int packed_counts(uint32_t cv) {
  // bit 7 is a chain vertex in a slow owner's code and the inside bit in the others'
  return __builtin_popcount(cv & ((cv & 0x8000u) ? 0x1ffu : 0x17fu)) |
         ((int)(((cv >> 9) & 7u) + ((cv >> 12) & 7u)) << 16);
}

template <class Src, int RB>
// At most 64 VGPRs: eight workgroups per compute unit.
__global__ void __launch_bounds__(kThreads, 8) k_emit(Src src, const int64_t* __restrict__ tab, Shared sh) {
  __shared__ StripLds<RB> S;
  EmitLds<RB>& L = S.e;
  constexpr int W = EmitLds<RB>::W;
  constexpr int kWaves = kThreads / 64;
  constexpr int kLut = 15 * 3 * 2 * 5;
  static_assert(kLut <= 2 * kThreads, "two table entries per thread");
  const int64_t tile = blockIdx.x;
  int64_t local;
  const int ii = src.find(tile, tab, local);
  const Img& d = src.img(ii);
  const Geo g = d.g;
  {
    long long nv, nt, nc;
    image_totals<Src>(d, sh, nv, nt, nc);
    if (image_status(d, sh.imgerr[ii], nv, nt) != SBMT_OK) return;  // uniform per block
  }
  const int cb = (int)local % g.NCB, ky = (int)local / g.NCB;  // tile index of an image: 32 bits
  const int k0 = ky * RB, c0 = cb * kCB;
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int col = 1 + 64 * wv + lane;  // LDS column
  const int c = c0 + 64 * wv + lane;
  const int nrec = (int)min((int64_t)sh.tile_n[tile], sh.tcap);
  // 1. loads first, so that their latencies overlap: the strip's codes in every
  // row (row RB is the row below the tile), the halo columns c0 - 1 and
  // c0 + kCB, the tile's records, the emission table, the row bases
  uint32_t code[RB + 1];
#pragma unroll
  for (int r = 0; r <= RB; ++r)
    code[r] = (k0 + r < g.NK && c < g.NI) ? (uint32_t)d.omap[(int64_t)(k0 + r) * g.NI + c] : 0u;
  uint32_t hcode = 0;
  const int hr = threadIdx.x >> 1, hside = threadIdx.x & 1;
  if (threadIdx.x < 2 * (RB + 1)) {
    const int hc = hside ? c0 + kCB : c0 - 1;
    if (k0 + hr < g.NK && hc >= 0 && hc < g.NI) hcode = d.omap[(int64_t)(k0 + hr) * g.NI + hc];
  }
  SlowRec held[kHold];
#pragma unroll
  for (int j = 0; j < kHold; ++j) {
    const int q = threadIdx.x + j * kThreads;
    if (q < nrec) held[j] = sh.rec[tile * sh.tcap + q];
  }
  const uint16_t* lt = (g.flags & 1u) ? &sbmt_lut_emit[0][0][0][0] : &sbmt_lut_emit_fg[0][0][0][0];
  const uint16_t lut0 = lt[threadIdx.x];
  const uint16_t lut1 = threadIdx.x + kThreads < kLut ? lt[threadIdx.x + kThreads] : 0;
  if (threadIdx.x <= RB) {
    const int k = k0 + threadIdx.x;
    const int64_t nsegi = (int64_t)g.NK * g.NCB;
    const longlong4 base = sh.seg_off[d.seg0];
    const longlong4 o = sh.seg_off[d.seg0 + (k < g.NK ? (int64_t)k * g.NCB + cb : nsegi)];
    L.bv[threadIdx.x] = (int)(o.x - base.x);
    if (threadIdx.x < RB) L.tb[threadIdx.x] = o.y - base.y;
    L.rowR[threadIdx.x] = d.rows[k].R;
    L.rowy[threadIdx.x] = lat_y(g, k);
  }
  L.lut[threadIdx.x] = lut0;
  if (threadIdx.x + kThreads < kLut) L.lut[threadIdx.x + kThreads] = lut1;
  L.x.stage[3][wv][lane] = 0u;  // staging slots start empty
  if (threadIdx.x < 2 * (RB + 1)) {
    L.info[hr][hside ? W - 1 : 0] = (uint16_t)hcode;
    if (!hside) {
      const int nvl = packed_counts(hcode) & 0xffff;
      S.lastnv[hr][0] = nvl;
      L.voff[hr][0] = (int16_t)(-nvl);
    }
  }
  // 2. per row: packed counts, their prefix along the strip (a DPP wave scan),
  // the strip's totals to LDS; vertex and triangle counts of a row segment stay
  // below 2^16
  int incl[RB + 1];
  const bool both = (g.flags & 1u) != 0;
#pragma unroll
  for (int r = 0; r <= RB; ++r) {
    const int p = packed_counts(code[r]);
    if (!both && __ballot((code[r] & 0x8000u) != 0u) == 0ull) {
      // no slow owner in the strip's row: a fast owner emits its vertex and
      // both triangles iff it is inside, so the prefix is a count of inside bits
      const int nb = lanes_below(__ballot((code[r] & 1u) != 0u)) + (int)(code[r] & 1u);
      incl[r] = nb | (nb << 17);
    } else {
      incl[r] = wave_incl_scan_dpp(p);
    }
    if (lane == 63) {
      S.wtot[r][wv] = incl[r];
      S.lastnv[r][wv + 1] = p & 0xffff;
    }
    L.info[r][col] = (uint16_t)code[r];
  }
  __syncthreads();
  // prefix of the strips to the left (uniform per wave), the row segment's totals
  int sb[RB + 1];
#pragma unroll
  for (int r = 0; r <= RB; ++r) {
    int before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const int tw = S.wtot[r][w];
      before += w < wv ? tw : 0;
      total += tw;
    }
    sb[r] = __builtin_amdgcn_readfirstlane(before);
    if (threadIdx.x == 0) L.voff[r][W - 1] = (int16_t)(total & 0xffff);
  }
  // 3. fast owners row by row: the vertex of the owner, then its triangles
  // (Tb, then Ta), written at their offsets; offsets go to LDS for step 4
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int k = k0 + r;
    if (k >= g.NK) break;  // uniform
    const int o = k & 1;
    const uint32_t cv = code[r];
    const int pn = packed_counts(code[r + 1]);
    const int exn = sb[r + 1] + incl[r + 1] - pn, inn = sb[r + 1] + incl[r + 1];
    if (r == RB - 1) L.voff[RB][col] = (int16_t)(exn & 0xffff);
    if (__ballot(cv != 0u) == 0ull) {
      // nothing in the strip's row (no vertex, no triangle, no slow owner):
      // every owner's offsets are the strip's first ones
      L.voff[r][col] = (int16_t)(sb[r] & 0xffff);
      L.toff[r][col] = (int16_t)(sb[r] >> 16);
      continue;
    }
    const int p = packed_counts(cv);
    const int ex = sb[r] + incl[r] - p;  // within the row segment: vertices | triangles << 16
    L.voff[r][col] = (int16_t)(ex & 0xffff);
    L.toff[r][col] = (int16_t)(ex >> 16);
    // vertex count of the owner left of this one in the row below (one lane to
    // the left; lane 0 from the strip to the left)
    int nvl = __builtin_amdgcn_update_dpp(0, pn & 0xffff, 0x138, 0xf, 0xf, false);  // wave_shr:1
    const int nvl0 = S.lastnv[r + 1][wv];
    nvl = lane == 0 ? nvl0 : nvl;
    const int bvr = __builtin_amdgcn_readfirstlane(L.bv[r]), bvn = __builtin_amdgcn_readfirstlane(L.bv[r + 1]);
    const long long tbr = L.tb[r];
    const int64_t tbs = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(tbr >> 32)) << 32) |
                                  (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)tbr));
    char* const vrow = reinterpret_cast<char*>(d.verts + 2 * (int64_t)bvr);
    char* const trow = reinterpret_cast<char*>(d.tris + 3 * tbs);
    uint8_t* const crow = d.codes + tbs;
    const bool fast = (cv & 0x8000u) == 0u;
    if (fast && (cv & 1u)) {
      double2 v;
      v.x = lat_x(g, g.X0 + 4 * g.h * c + 2 * g.h * o);
      v.y = L.rowy[r];
      *reinterpret_cast<double2*>(vrow + (uint32_t)(ex & 0xffff) * 16u) = v;
    }
    const int ntb = fast ? (int)((cv >> 9) & 7u) : 0, nta = fast ? (int)((cv >> 12) & 7u) : 0;
    const int vid = bvr + (ex & 0xffff);
    const int vr = bvr + ((sb[r] + incl[r]) & 0xffff);
    const int vdl = bvn + (exn & 0xffff) - (o ? 0 : nvl);
    const int vdr = bvn + ((o ? inn : exn) & 0xffff);
    // the triangles go to LDS at their slot relative to the strip's first
    // triangle of the row (slow owners' slots stay empty), 64 slots at a time;
    // lane j then writes slot j, so that a store covers consecutive triangles
    const uint32_t tag = 1u | ((both && !((cv >> 7) & 1u)) ? 0x8000u : 0u);
    const int s0 = sb[r] >> 16;                                  // the strip's first triangle
    const int ns = __builtin_amdgcn_readlane(incl[r], 63) >> 16;  // the strip's triangles in this row
    const int q0 = (ex >> 16) - s0;
    uint32_t* const sa = L.x.stage[0][wv];
    uint32_t* const sb2 = L.x.stage[1][wv];
    uint32_t* const sc = L.x.stage[2][wv];
    uint32_t* const sw = L.x.stage[3][wv];
    for (int base = 0; base < ns; base += 64) {  // uniform
      const int qa = q0 - base, qb = qa + ntb;
      if (ntb && qa >= 0 && qa < 64) {
        sa[qa] = (uint32_t)vid;
        sb2[qa] = (uint32_t)vdr;
        sc[qa] = (uint32_t)vdl;
        sw[qa] = tag;
      }
      if (nta && qb >= 0 && qb < 64) {
        sa[qb] = (uint32_t)vid;
        sb2[qb] = (uint32_t)vr;
        sc[qb] = (uint32_t)vdr;
        sw[qb] = tag;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const uint32_t ew = sw[lane];
      if (ew) {
        const uint32_t u = (uint32_t)(s0 + base + lane);
        Tri3 t3;
        t3.a = (int)sa[lane];
        t3.b = (int)sb2[lane];
        t3.c = (int)sc[lane];
        *reinterpret_cast<Tri3*>(trow + u * 12u) = t3;
        if (both) crow[u] = (uint8_t)(ew >> 8);  // foreground mode: the codes are filled below
        sw[lane] = 0u;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  // foreground mode: every fast triangle has code 0 (an uncut foreground
  // triangle), so each row segment's codes are first set to 0 with 16-byte
  // stores (bytes at the unaligned ends); the slow owners' sub-triangles get
  // their codes in step 4, after the barrier
  if (!both) {
    for (int r = wv; r < RB; r += kWaves) {
      if (k0 + r >= g.NK) break;  // uniform
      int n = 0;  // triangles of the row segment (the strip totals were written before step 2's barrier)
#pragma unroll
      for (int w = 0; w < kWaves; ++w) n += S.wtot[r][w] >> 16;
      uint8_t* const p0 = d.codes + L.tb[r];
      uint8_t* const p1 = p0 + n;
      uint8_t* const a0 = reinterpret_cast<uint8_t*>(((uintptr_t)p0 + 15) & ~(uintptr_t)15);
      uint8_t* const a1 = reinterpret_cast<uint8_t*>((uintptr_t)p1 & ~(uintptr_t)15);
      if (a0 >= a1) {
        if (lane < n) p0[lane] = 0;  // fewer than 32 bytes
      } else {
        if (lane < a0 - p0) p0[lane] = 0;
        if (lane >= 16 && lane - 16 < p1 - a1) a1[lane - 16] = 0;
        for (uint8_t* q = a0 + 16 * lane; q < a1; q += 1024) *reinterpret_cast<uint4*>(q) = make_uint4(0u, 0u, 0u, 0u);
      }
    }
  }
  __syncthreads();
  // 4. slow owners from their records
  emit_records<RB>(d, g, k0, c0, tile, sh, L, held[0], held[1], nrec);
}

// Slow owners without a record: the tiles whose count pass queued more slow
// owners than their record region holds, found among kThreads tiles per
// block and emitted one after the other (rare: the region is sized for the
// usual share of slow owners).
template <class Src, int RB>
__global__ void __launch_bounds__(kThreads) k_emit_missing(Src src, const int64_t* __restrict__ tab, Shared sh,
                                                           int64_t ntile) {
  __shared__ EmitLds<RB> L;
  __shared__ unsigned long long over[kThreads / 64];
  const int64_t t0 = (int64_t)blockIdx.x * kThreads;
  const int64_t t = t0 + threadIdx.x;
  const unsigned long long b = __ballot(t < ntile && sh.tile_n[t] > sh.tcap);
  if ((threadIdx.x & 63) == 0) over[threadIdx.x >> 6] = b;
  __syncthreads();
  for (int w = 0; w < kThreads / 64; ++w) {
    for (unsigned long long m = over[w]; m; m &= m - 1) {  // the same value in every lane
      emit_count_tile<Src, RB, kEmitMissing>(src, tab, sh, t0 + 64 * w + __builtin_ctzll(m), L);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Fused persistent path.  A workgroup repeatedly takes the next band (RB
// full-width rows of one image) in ticket order and
//   1. counts its row segments and those of the halo row below it, queueing
//      slow owners in the tiles' record regions (the halo row's codes go to a
//      per-band row of scratch: the band below writes the owner map there);
//   2. classifies the band's slow owners densely, adding their counts;
//   3. publishes the band's (n_v, n_t) and finds its offsets by a decoupled
//      look-back over the bands of the same image: earlier tickets only, which
//      are running or done and publish without waiting, so every wait ends;
//   4. emits its tiles left to right with the per-row segment bases.
// Bands that would not fit the output capacity skip their writes; the last
// band of an image writes the image's sizes and status.
// ---------------------------------------------------------------------------
constexpr unsigned long long kLbAgg = 1ull << 62, kLbIncl = 2ull << 62;
SBMT_HD unsigned long long lb_word(unsigned long long flag, long long v, long long t) {
  return flag | ((unsigned long long)t << 31) | (unsigned long long)v;
}

template <int RB>
struct FusedLds {
  union {
    CountLds<RB + 1> c;
    EmitLds<RB> e;
  } u;
  int4 acc[RB + 1];                  // per-row counts of the chunk just counted
  int2 cnt[kMaxBandChunks][RB + 1];  // per chunk and row: (nv, nt); later the image-local bases
  int cn[kMaxBandChunks + 1];        // records per chunk, then their prefix
  long long ticket;
  int ncut, err;
};

template <int RB>
__global__ void __launch_bounds__(kThreads, 3) k_fused(ManySrc src, const int64_t* __restrict__ tab,
                                                       const int64_t* __restrict__ ttab, Shared sh, int64_t nbands,
                                                       uint16_t* __restrict__ halo) {
  __shared__ FusedLds<RB> F;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) F.ticket = (long long)atomicAdd(&sh.ctr[1], 1ull);
    __syncthreads();
    const long long t = F.ticket;
    if (t >= nbands) break;
    int64_t j;
    const int ii = src.find(t, tab, j);
    const Img& d = src.img(ii);
    const Geo g = d.g;
    const int nb = (g.NK + RB - 1) / RB;
    const int k0 = (int)j * RB;
    uint16_t* hcode = halo + d.halo0 + j * (int64_t)g.NI;  // codes of row k0 + RB
    const int64_t tile0 = ttab[ii] + j * g.NCB;             // count tile of chunk 0
    if (threadIdx.x == 0) F.ncut = F.err = 0;
    // 1. counts of rows k0 .. k0+RB chunk by chunk (the last row is the halo
    // row: its codes go to hcode, the owner map keeps the next band's own)
    for (int cb = 0; cb < g.NCB; ++cb) {
      __syncthreads();
      if (threadIdx.x <= RB) F.acc[threadIdx.x] = make_int4(0, 0, 0, 0);
      // records hold every owner of the band tile (checked on the host), so no
      // slow owner is ever classified here
      count_tile<RB + 1>(d, g, ii, tile0 + cb, k0, cb, sh, F.u.c, F.acc, hcode);
      __syncthreads();
      if (threadIdx.x <= RB) F.cnt[cb][threadIdx.x] = make_int2(F.acc[threadIdx.x].x, F.acc[threadIdx.x].y);
      if (threadIdx.x == 0) {
        F.cn[cb] = (int)min((int64_t)F.u.c.n2, sh.tcap);
        for (int r = 0; r < RB; ++r) F.ncut += F.acc[r].z;
      }
    }
    __syncthreads();
    // 2. the band's recorded slow owners, densely
    if (threadIdx.x == 0) {
      int s = 0;
      for (int cb = 0; cb < g.NCB; ++cb) {
        const int n = F.cn[cb];
        F.cn[cb] = s;
        s += n;
      }
      F.cn[g.NCB] = s;
    }
    __syncthreads();
    const int nslow = F.cn[g.NCB];
    for (int q = threadIdx.x; q < nslow; q += kThreads) {
      int lo = 0, hi = g.NCB - 1;  // chunk: largest cb with cn[cb] <= q
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (F.cn[mid] <= q) lo = mid;
        else hi = mid - 1;
      }
      const int64_t idx = (tile0 + lo) * sh.tcap + (q - F.cn[lo]);
      const uint64_t p = sh.rec[idx].x;
      const int k = (int)((p >> 24) & 0xffffffu), c = (int)(p & 0xffffffu);
      const int r = k - k0;
      Bits b;
      b.p = d.bits;
      b.wpr = g.wpr;
      b.rr0 = 0;
      b.cc0 = 0;
      const Frame f = owner_frame(g, b, k, c, d.rows[k].R);
      Slow sr;
      slow_classify(g, f, d.rows[k], d.rows[k + 1].FL, sr);
      SlowRec R = pack_slow(sr);
      R.x |= (uint64_t)((r << 8) | (c - lo * kCB)) << 48;
      sh.rec[idx] = R;
      if (r < RB) d.omap[(int64_t)k * g.NI + c] = (uint16_t)map_code(sr.info);
      else hcode[c] = (uint16_t)map_code(sr.info);
      atomicAdd(&F.cnt[lo][r].x, info_nv(sr.info));
      atomicAdd(&F.cnt[lo][r].y, info_nt(sr.info));
      if (r < RB) atomicAdd(&F.ncut, info_ncut(sr.info));
      if (info_err(sr.info)) F.err = 1;
    }
    __syncthreads();
    // 3. band totals, look-back, per-row segment bases
    if (threadIdx.x == 0) {
      long long av = 0, at = 0;
      for (int cb = 0; cb < g.NCB; ++cb)
        for (int r = 0; r < RB; ++r) {
          av += F.cnt[cb][r].x;
          at += F.cnt[cb][r].y;
        }
      if (F.err) atomicOr(&sh.imgerr[ii], 1);
      if (F.ncut) atomicAdd((unsigned long long*)&sh.sizes[kSizeWords * (int64_t)ii + 2], (unsigned long long)F.ncut);
      unsigned long long* w = sh.band + d.band0 + j;
      long long pv = 0, pt = 0;
      if (j == 0) {
        __hip_atomic_store(w, lb_word(kLbIncl, av, at), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        __hip_atomic_store(w, lb_word(kLbAgg, av, at), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        for (int64_t p = j - 1; p >= 0; --p) {
          unsigned long long x;
          for (;;) {
            x = __hip_atomic_load(sh.band + d.band0 + p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            if (x >> 62) break;
            __builtin_amdgcn_s_sleep(2);
          }
          pv += (long long)(x & 0x7fffffffull);
          pt += (long long)((x >> 31) & 0x7fffffffull);
          if ((x >> 62) == 2ull) break;
        }
        __hip_atomic_store(w, lb_word(kLbIncl, pv + av, pt + at), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
      // rows of the band in order, chunks in order within a row; the halo row
      // starts where the band ends
      long long v = pv, tt = pt;
      for (int r = 0; r < RB; ++r)
        for (int cb = 0; cb < g.NCB; ++cb) {
          const int2 x = F.cnt[cb][r];
          F.cnt[cb][r] = make_int2((int)v, (int)tt);
          v += x.x;
          tt += x.y;
        }
      F.cnt[0][RB].x = (int)v;  // first vertex of the halo row's first segment
      if (j == nb - 1) {
        // last band of the image: its end is the image total
        const int st = (int)image_status(d, atomicOr(&sh.imgerr[ii], 0), v, tt);
        sh.sizes[kSizeWords * (int64_t)ii + 0] = v;
        sh.sizes[kSizeWords * (int64_t)ii + 1] = tt;
        sh.sizes[kSizeWords * (int64_t)ii + 3] = st;
        sh.sizes[kSizeWords * (int64_t)ii + 4] = segment_total(sh, ii);
      }
      // write only if the band's vertex and triangle ranges fit
      F.err = (v > d.vcap || tt > d.tcap || v > 0x7fffffffLL || atomicOr(&sh.imgerr[ii], 0)) ? 1 : 0;
    }
    __syncthreads();
    if (F.err) continue;
    // 4. emission, tiles left to right; the halo row's bases follow the row
    int hv = F.cnt[0][RB].x;
    for (int cb = 0; cb < g.NCB; ++cb) {
      EmitLds<RB>& E = F.u.e;
      __syncthreads();
      if (threadIdx.x < RB) {
        E.bv[threadIdx.x] = F.cnt[cb][threadIdx.x].x;
        E.tb[threadIdx.x] = F.cnt[cb][threadIdx.x].y;
      }
      if (threadIdx.x == RB) E.bv[RB] = hv;
      emit_tile<RB>(d, g, k0, cb, tile0 + cb, sh, E, hcode, [](EmitLds<RB>&) {});
      __syncthreads();
      hv += E.rowv[RB];
    }
  }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
// grid_h = p / U, U = 2^q (q <= 8), reduced; the coarse stride is the smallest
// s with s^2 > 2 h^2.
static bool parse_grid_h(double grid_h, int* p, int* q) {
  if (!(grid_h > 0.0) || grid_h > 6.0) return false;
  const double g256 = grid_h * 256.0;
  if (g256 != __builtin_floor(g256)) return false;
  int pp = (int)g256, qq = 8;
  while (qq > 0 && (pp & 1) == 0) {
    pp >>= 1;
    --qq;
  }
  *p = pp;
  *q = qq;
  return true;
}

static int stride_for(int p, int U) {
  int s = 1;
  while ((int64_t)s * s * U * U <= 2LL * p * p) ++s;
  return s;
}

static bool grid_h_supported(int p, int U) {
  // the owner parallelogram (width 1.5 h) must fit two coarse cells: 3h <= 2s
  return p >= 1 && p <= 6 * U && 3 * p <= 2 * stride_for(p, U) * U;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Host copies of the exact row-cell rule, used to check before any launch that
// every 3x3 sample window the kernels read lies inside the stored raster.
static int host_z3sign(int64_t a, int64_t b) {
  if (a >= 0 && b >= 0) return (a | b) != 0 ? 1 : 0;
  if (a <= 0 && b <= 0) return -1;
  __int128 a2 = (__int128)a * a, b2 = (__int128)3 * b * b;
  return a > 0 ? (a2 > b2 ? 1 : -1) : (b2 > a2 ? 1 : -1);
}
static int64_t host_floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  return (a % b != 0 && a < 0) ? q - 1 : q;
}
static int64_t host_row_cell(int64_t k, int p, int s, int U) {
  int64_t kp = k * p;
  int64_t R = host_floordiv(kp * 17320 / (10000LL * U) - s - 1, 2 * s);
  while (host_z3sign(-(int64_t)U * (2 * s * R + s + 1), kp) < 0) --R;
  while (host_z3sign(-(int64_t)U * (2 * s * (R + 1) + s + 1), kp) >= 0) ++R;
  return R;
}

constexpr int kMaxTileRows = 16;  // largest RB instantiated
static bool tile_window_fits(const Geo& g) {
  // rows: the cell rows of kMaxTileRows + 1 grid rows plus the 3x3 window;
  // words: the cell columns of kCB + 2 owners plus the window and one spare word
  const double h = (double)g.h / g.U;
  const double rows = ((kMaxTileRows + 1) * h * 0.8660254037844386) / g.s + 5;
  const double words = ((kCB + 2) * h / g.s + 4) / 32.0 + 3;
  return rows <= kWinRows && words <= kWinWords;
}

static bool windows_in_bounds(const Geo& g) {
  const int64_t rlo_min = host_row_cell(0, g.h, g.s, g.U), rlo_max = host_row_cell(g.NK - 1, g.h, g.s, g.U);
  const int64_t xmin = g.X0, xmax = (int64_t)g.X0 + 4LL * g.h * (g.NI - 1) + 2LL * g.h;
  const int64_t clo_min = host_floordiv(xmin - 2 * g.h - 2LL * (g.s - 1) * g.U, 4LL * g.s * g.U);
  const int64_t clo_max = host_floordiv(xmax - 2 * g.h - 2LL * (g.s - 1) * g.U, 4LL * g.s * g.U);
  // rows Rlo .. Rlo+2 and bit columns Clo .. Clo+2 (plus one spare word) are read
  return rlo_min + kRing >= 0 && rlo_max + 2 + kRing < g.CH + 2 * kRing && clo_min + kRingC >= 0 &&
         ((clo_max + 2 + kRingC) >> 5) + 1 < g.wpr;
}

static sbmt_status make_geo(const sbmt_image* img, Geo* out, bool need_ptr) {
  if (!img) return SBMT_E_INVALID_ARG;
  if (img->width < 0 || img->height < 0) return SBMT_E_INVALID_ARG;
  if ((int64_t)img->width > (1 << 20) || (int64_t)img->height > (1 << 20)) return SBMT_E_INVALID_ARG;
  if (img->width > 0 && img->height > 0 && ((need_ptr && img->bitmap == nullptr) || img->row_stride < img->width))
    return SBMT_E_INVALID_ARG;
  if (img->flags & ~1u) return SBMT_E_INVALID_ARG;
  int p = 0, q = 0;
  if (!parse_grid_h(img->grid_h, &p, &q) || !grid_h_supported(p, 1 << q)) return SBMT_E_UNSUPPORTED_GRID_H;
  Geo g;
  g.W = img->width;
  g.H = img->height;
  g.stride = img->row_stride;
  g.h = p;
  g.q = q;
  g.U = 1 << q;
  g.s = stride_for(p, g.U);
  // exact predicates in 64-bit integers need |a|, |b| < 2^31: 16 s U^2 (side + ring) < 2^31
  const int64_t side = std::max<int64_t>(g.W, g.H) + 2 * g.s + 16;
  if ((__int128)16 * g.s * g.U * g.U * side >= ((__int128)1 << 31)) return SBMT_E_UNSUPPORTED_GRID_H;
  g.CW = (g.W + g.s - 1) / g.s;
  g.CH = (g.H + g.s - 1) / g.s;
  // rows 0..m with m the smallest m >= 1 such that 3 m^2 h^2 > (2 s CH + 1)^2
  const __int128 rhs = (__int128)g.U * g.U * (2LL * g.s * g.CH + 1) * (2LL * g.s * g.CH + 1);
  int64_t m = (int64_t)((2.0 * g.s * g.CH + 1) * g.U / (p * 1.7320508075688772)) - 2;
  if (m < 1) m = 1;
  while ((__int128)3 * m * m * p * p <= rhs) ++m;
  while (m > 1 && (__int128)3 * (m - 1) * (m - 1) * p * p > rhs) --m;
  if (m + 1 >= (1LL << 24)) return SBMT_E_INVALID_ARG;
  g.NK = (int32_t)(m + 1);
  // x of vertex (0, 0), odd; the last column lies right of x = s CW - 1/2
  g.X0 = g.U == 1 ? -2 * p - 3 : -(2 * p + 3 * g.U) - 1;
  const int64_t ni = (4LL * g.U * g.s * g.CW - 2LL * g.U - g.X0) / (4LL * p) + 2;
  if (ni >= (1LL << 24)) return SBMT_E_INVALID_ARG;
  g.NI = (int32_t)ni;
  g.NCB = (g.NI + kCB - 1) / kCB;
  g.wpr = (kRingC + g.CW + kRing + 31) / 32 + 1;
  g.flags = img->flags;
  g.inv4s = 1.0f / (float)(4 * g.s);
  g.xscale = 0.25 / (double)g.U;
  g.invU = 1.0 / (double)g.U;
  if (!windows_in_bounds(g) || !tile_window_fits(g)) return SBMT_E_INVALID_ARG;
  // owner positions in record lists: 24 bits per coordinate
  if (g.NK >= (1 << 24) || g.NI >= (1 << 24)) return SBMT_E_INVALID_ARG;
  *out = g;
  return SBMT_OK;
}

static int rb_index(int rb) { return rb == 4 ? 0 : (rb == 8 ? 1 : (rb == 16 ? 2 : -1)); }
static const int kRBs[3] = {4, 8, 16};

// Workspace of a call on n images: shared scratch, then per-image regions.
struct CallLayout {
  int n = 0;
  std::vector<Geo> g;
  std::vector<size_t> off_bits, off_omap, off_rows, off_cols;
  std::vector<int64_t> seg0, band0, halo0;  // band0, halo0 for the smallest fused band height
  std::vector<int64_t> tab;           // [1 + 3 + 3][n + 1]: coarsen blocks, tiles per RB, bands per RB
  int64_t nseg = 0, owners = 0, rcap = 0, nbands_max = 0, halo_words = 0, ntiles_max = 0;
  int64_t tcap[3] = {0, 0, 0};  // records per count tile, per tile height
  int64_t dcap[3] = {0, 0, 0};  // entries per dense list, per tile height
  int nblk = 0;
  size_t off_ctr, off_dctr, off_imgerr, off_sizes, off_segacc, off_desc, off_tab, off_cnt, off_slow, off_segoff, off_blk, off_rec,
      off_dense, off_tilen, off_band, off_halo, total;
  bool fused_ok = true;  // per-image counts fit the fused path's int32 bases and band width
};

static int64_t* tab_row(CallLayout& L, int which) { return L.tab.data() + (size_t)which * (L.n + 1); }

static sbmt_status make_call_layout(const sbmt_image* imgs, int n, int64_t record_cap, bool need_ptr,
                                    CallLayout* out) {
  if (n < 1 || n > 65535 || !imgs) return SBMT_E_INVALID_ARG;
  CallLayout& L = *out;
  L.n = n;
  L.g.resize(n);
  L.off_bits.resize(n);
  L.off_omap.resize(n);
  L.off_rows.resize(n);
  L.off_cols.resize(n);
  L.seg0.resize(n);
  L.band0.resize(n);
  L.halo0.resize(n);
  L.tab.assign((size_t)7 * (n + 1), 0);
  for (int i = 0; i < n; ++i) {
    sbmt_status st = make_geo(&imgs[i], &L.g[i], need_ptr);
    if (st != SBMT_OK) return st;
  }
  for (int i = 0; i < n; ++i) {
    const Geo& g = L.g[i];
    L.seg0[i] = L.nseg;
    L.nseg += (int64_t)g.NK * g.NCB;
    L.owners += (int64_t)g.NK * g.NI;
    const int64_t cblk = (int64_t)((g.wpr + 7) / 8) * ((g.CH + 2 * kRing + kCoarsenRows - 1) / kCoarsenRows);
    tab_row(L, 0)[i + 1] = tab_row(L, 0)[i] + cblk;
    for (int r = 0; r < 3; ++r) {
      const int64_t rows = (g.NK + kRBs[r] - 1) / kRBs[r];
      tab_row(L, 1 + r)[i + 1] = tab_row(L, 1 + r)[i] + rows * g.NCB;
      tab_row(L, 4 + r)[i + 1] = tab_row(L, 4 + r)[i] + rows;
    }
    L.band0[i] = tab_row(L, 4)[i];
    L.halo0[i] = L.halo_words;
    L.halo_words += (int64_t)((g.NK + 3) / 4) * g.NI;
    // a band's counts are kept as int32 image-local offsets: 10 triangles per
    // owner bound the image's triangles
    if (g.NCB > kMaxBandChunks || 10LL * g.NK * g.NI > 0x7fffffffLL) L.fused_ok = false;
  }
  L.nbands_max = tab_row(L, 4)[n];
  // records: by default half of each tile's owners (the slow fraction reaches
  // about a third at grid_h = 4 on fine structures); an explicit cap is
  // shared evenly by the tiles
  for (int r = 0; r < 3; ++r) L.ntiles_max = std::max(L.ntiles_max, tab_row(L, 1 + r)[n]);
  if (record_cap == 0) {
    for (int r = 0; r < 3; ++r) L.rcap = std::max(L.rcap, tab_row(L, 1 + r)[n] * (int64_t)(kRBs[r] * kCB / 2));
  } else if (record_cap < 0) {
    // room for every owner of a persistent-kernel band tile (its rows and halo row)
    for (int r = 0; r < 2; ++r) L.rcap = std::max(L.rcap, tab_row(L, 1 + r)[n] * (int64_t)((kRBs[r] + 1) * kCB));
  } else {
    L.rcap = std::max<int64_t>(record_cap, 0);
  }
  if (L.rcap > kMaxRecords) L.rcap = kMaxRecords;
  for (int r = 0; r < 3; ++r) {
    const int64_t nt = tab_row(L, 1 + r)[n];
    L.tcap[r] = L.rcap / std::max<int64_t>(nt, 1);
    // tile t feeds list t mod kDenseLists: at most ceil(nt / kDenseLists) tiles a list
    L.dcap[r] = (nt + kDenseLists - 1) / kDenseLists * L.tcap[r];
  }
  // lists in use: min(tiles, kDenseLists); at most rcap + (kDenseLists - 1) tcap entries
  int64_t dmax = 0;
  for (int r = 0; r < 3; ++r)
    dmax = std::max(dmax, std::min<int64_t>(tab_row(L, 1 + r)[n], kDenseLists) * L.dcap[r]);
  L.nblk = (int)((L.nseg + kScanChunk - 1) / kScanChunk);
  size_t off = 0;
  L.off_ctr = off;
  off = align256(off + 8 * sizeof(unsigned long long));
  L.off_dctr = off;
  off = align256(off + kDenseLists * sizeof(unsigned long long));
  L.off_imgerr = off;
  off = align256(off + (size_t)n * sizeof(int));
  L.off_sizes = off;
  off = align256(off + (size_t)n * kSizeWords * sizeof(int64_t));
  L.off_segacc = off;
  off = align256(off + (size_t)n * kSegSlots * sizeof(unsigned long long));
  L.off_desc = off;
  off = align256(off + (size_t)n * sizeof(Img));
  L.off_tab = off;
  off = align256(off + L.tab.size() * sizeof(int64_t));
  L.off_cnt = off;
  off = align256(off + (size_t)L.nseg * sizeof(int4));
  L.off_slow = off;
  off = align256(off + (size_t)L.nseg * sizeof(unsigned long long));
  L.off_segoff = off;
  off = align256(off + (size_t)(L.nseg + 1) * sizeof(longlong4));
  L.off_blk = off;
  off = align256(off + (size_t)L.nblk * sizeof(longlong4));
  L.off_rec = off;
  off = align256(off + (size_t)L.rcap * sizeof(SlowRec));
  L.off_dense = off;
  off = align256(off + (size_t)dmax * sizeof(uint32_t));
  L.off_tilen = off;
  off = align256(off + (size_t)L.ntiles_max * sizeof(int));
  L.off_band = off;
  off = align256(off + (size_t)L.nbands_max * sizeof(unsigned long long));
  L.off_halo = off;
  off = align256(off + (size_t)L.halo_words * sizeof(uint16_t));
  for (int i = 0; i < n; ++i) {
    const Geo& g = L.g[i];
    L.off_bits[i] = off;
    off = align256(off + (size_t)(g.CH + 2 * kRing) * g.wpr * 4);
    L.off_omap[i] = off;
    off = align256(off + (size_t)g.NK * g.NI * 2);
    L.off_rows[i] = off;
    off = align256(off + (size_t)(g.NK + kRowPad) * sizeof(RowT));
    L.off_cols[i] = off;
    off = align256(off + (size_t)g.NI * 2 * sizeof(uint32_t));
  }
  L.total = off;
  return SBMT_OK;
}

static Shared shared_of(const CallLayout& L, void* ws, int rbi) {
  char* b = (char*)ws;
  Shared s;
  s.seg_cnt = (int4*)(b + L.off_cnt);
  s.seg_slow = (unsigned long long*)(b + L.off_slow);
  s.seg_off = (longlong4*)(b + L.off_segoff);
  s.blk = (longlong4*)(b + L.off_blk);
  s.ctr = (unsigned long long*)(b + L.off_ctr);
  s.imgerr = (int*)(b + L.off_imgerr);
  s.sizes = (int64_t*)(b + L.off_sizes);
  s.segacc = (unsigned long long*)(b + L.off_segacc);
  s.rec = (SlowRec*)(b + L.off_rec);
  s.dense = (uint32_t*)(b + L.off_dense);
  s.dctr = (unsigned long long*)(b + L.off_dctr);
  s.dcap = L.dcap[rbi];
  s.band = (unsigned long long*)(b + L.off_band);
  s.tile_n = (int*)(b + L.off_tilen);
  s.tcap = L.tcap[rbi];
  s.nseg = L.nseg;
  s.nbands = L.nbands_max;
  s.nblk = L.nblk;
  s.n = L.n;
  return s;
}

static Img img_of(const CallLayout& L, int i, const sbmt_image& im, void* ws, const sbmt_outputs* o) {
  char* b = (char*)ws;
  Img d;
  memset(&d, 0, sizeof(d));
  d.g = L.g[i];
  d.bm = im.bitmap;
  d.bits = (uint32_t*)(b + L.off_bits[i]);
  d.omap = (uint16_t*)(b + L.off_omap[i]);
  d.rows = (RowT*)(b + L.off_rows[i]);
  d.cols = (uint32_t*)(b + L.off_cols[i]);
  d.seg0 = L.seg0[i];
  d.band0 = L.band0[i];
  d.halo0 = L.halo0[i];
  if (o) {
    d.verts = o->verts;
    d.tris = o->tris;
    d.codes = o->codes;
    d.vcap = o->vert_cap;
    d.tcap = o->tri_cap;
  }
  return d;
}

template <class Src>
static sbmt_status launch_front(const CallLayout& L, const Src& src, const int64_t* dtab, const Shared& sh, int rbi,
                                hipStream_t st) {
  const int64_t* t0 = dtab;
  const int64_t* tt = dtab ? dtab + (size_t)(1 + rbi) * (L.n + 1) : nullptr;
  const int64_t ncb = L.tab[(size_t)0 * (L.n + 1) + L.n];
  const int64_t ntile = L.tab[(size_t)(1 + rbi) * (L.n + 1) + L.n];
  if (ncb > 0x7fffffffLL || ntile > 0x7fffffffLL) return SBMT_E_INVALID_ARG;
  hipLaunchKernelGGL(k_coarsen<Src>, dim3((unsigned)ncb), dim3(256), 0, st, src, t0, sh);
  const int64_t nsb = L.tab[(size_t)6 * (L.n + 1) + L.n];  // 16-row bands: segment-count blocks
  hipLaunchKernelGGL(k_segcount<Src>, dim3((unsigned)nsb), dim3(256), 0, st, src,
                     dtab ? dtab + (size_t)6 * (L.n + 1) : nullptr, sh);
  switch (kRBs[rbi]) {
    case 4: hipLaunchKernelGGL((k_count<Src, 4>), dim3((unsigned)ntile), dim3(kThreads), 0, st, src, tt, sh); break;
    case 8: hipLaunchKernelGGL((k_count<Src, 8>), dim3((unsigned)ntile), dim3(kThreads), 0, st, src, tt, sh); break;
    default: hipLaunchKernelGGL((k_count<Src, 16>), dim3((unsigned)ntile), dim3(kThreads), 0, st, src, tt, sh); break;
  }
  // the dense pass: a grid-stride loop over the queued records (at most rcap)
  const dim3 gd((unsigned)std::max<int64_t>(1, std::min<int64_t>((L.rcap + kThreads - 1) / kThreads, kSlowBlocks)));
  switch (kRBs[rbi]) {
    case 4:
      hipLaunchKernelGGL((k_slow_dense<Src, 4>), gd, dim3(kThreads), 0, st, src, sh);
      hipLaunchKernelGGL((k_slow_tiles<Src, 4>), dim3((unsigned)ntile), dim3(64), 0, st, src, tt, sh);
      break;
    case 8:
      hipLaunchKernelGGL((k_slow_dense<Src, 8>), gd, dim3(kThreads), 0, st, src, sh);
      hipLaunchKernelGGL((k_slow_tiles<Src, 8>), dim3((unsigned)ntile), dim3(64), 0, st, src, tt, sh);
      break;
    default:
      hipLaunchKernelGGL((k_slow_dense<Src, 16>), gd, dim3(kThreads), 0, st, src, sh);
      hipLaunchKernelGGL((k_slow_tiles<Src, 16>), dim3((unsigned)ntile), dim3(64), 0, st, src, tt, sh);
      break;
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3(L.nblk), dim3(kScanThreads), 0, st, sh);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanThreads), 0, st, sh);
  hipLaunchKernelGGL(k_scan_apply, dim3(L.nblk), dim3(kScanThreads), 0, st, sh);
  return hipGetLastError() == hipSuccess ? SBMT_OK : SBMT_E_DEVICE;
}

template <class Src>
static sbmt_status launch_sizes(const CallLayout& L, const Src& src, const Shared& sh, int64_t* user, hipStream_t st) {
  hipLaunchKernelGGL(k_sizes<Src>, dim3((L.n + 255) / 256), dim3(256), 0, st, src, sh, user);
  return hipGetLastError() == hipSuccess ? SBMT_OK : SBMT_E_DEVICE;
}

template <class Src>
static sbmt_status launch_emit(const CallLayout& L, const Src& src, const int64_t* dtab, const Shared& sh, int rbi,
                               hipStream_t st) {
  const int64_t* tt = dtab ? dtab + (size_t)(1 + rbi) * (L.n + 1) : nullptr;
  const int64_t ntile = L.tab[(size_t)(1 + rbi) * (L.n + 1) + L.n];
  if (ntile > 0x7fffffffLL) return SBMT_E_INVALID_ARG;
  const dim3 gm((unsigned)((ntile + kThreads - 1) / kThreads));
  switch (kRBs[rbi]) {
    case 4:
      hipLaunchKernelGGL((k_emit<Src, 4>), dim3((unsigned)ntile), dim3(kThreads), 0, st, src, tt, sh);
      hipLaunchKernelGGL((k_emit_missing<Src, 4>), gm, dim3(kThreads), 0, st, src, tt, sh, ntile);
      break;
    case 8:
      hipLaunchKernelGGL((k_emit<Src, 8>), dim3((unsigned)ntile), dim3(kThreads), 0, st, src, tt, sh);
      hipLaunchKernelGGL((k_emit_missing<Src, 8>), gm, dim3(kThreads), 0, st, src, tt, sh, ntile);
      break;
    default:
      hipLaunchKernelGGL((k_emit<Src, 16>), dim3((unsigned)ntile), dim3(kThreads), 0, st, src, tt, sh);
      hipLaunchKernelGGL((k_emit_missing<Src, 16>), gm, dim3(kThreads), 0, st, src, tt, sh, ntile);
      break;
  }
  return hipGetLastError() == hipSuccess ? SBMT_OK : SBMT_E_DEVICE;
}



__global__ void k_copy_sizes(const int64_t* __restrict__ s, int64_t n4, int64_t* __restrict__ user) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n4) user[q] = s[q];
}

#include "sbmt_pre.h"


}  // namespace sbmt


using namespace sbmt;

// Pinned host buffers are allocated once per size class and recycled, so that
// creating and destroying batch objects in a serving loop never calls the
// (device-synchronising) pinned allocator after warm-up.
struct PinnedPool {
  std::vector<std::vector<void*>> free_;  // per size class 2^(12 + j) bytes
  std::vector<void*> all_;
  void* get(size_t bytes, int* cls) {
    int j = 0;
    while (((size_t)4096 << j) < bytes) ++j;
    *cls = j;
    if ((int)free_.size() <= j) free_.resize(j + 1);
    if (!free_[j].empty()) {
      void* p = free_[j].back();
      free_[j].pop_back();
      return p;
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, (size_t)4096 << j, hipHostMallocDefault) != hipSuccess) return nullptr;
    all_.push_back(p);
    return p;
  }
  void put(void* p, int cls) {
    if (p) free_[cls].push_back(p);
  }
  void release() {
    for (void* p : all_) (void)hipHostFree(p);
    all_.clear();
    free_.clear();
  }
};

// Scratch of the allocation-free entry point: the workspace of one image, in
// a file-scope device array (every GPU the library runs on holds its own copy
// until the process ends).  Host code never uses the array's name as an
// address: each handle looks up its device's copy once, at creation.
static __device__ __align__(256) unsigned char scratch[SBMT_NOALLOC_SCRATCH_BYTES];

struct sbmt_context {
  int device;
  int cus;
  long long* pinned;  // 8 x int64 (one sizes record)
  PinnedPool pool;
  void* scratch_ptr;  // this device's copy of `scratch`
};

struct sbmt_batch_s {
  sbmt_context* ctx;
  std::vector<sbmt_image> imgs;
  CallLayout L;
  sbmt_tuning tune;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  unsigned char* stage = nullptr;  // pinned: descriptors + tables
  size_t stage_bytes = 0;
  int64_t* psizes = nullptr;       // pinned: n x 4
  int stage_cls = 0, psizes_cls = 0;
  int count_rbi = -1;  // tile height of the last count pass (emission must use the same tiles)
};

static void host_sizes_of(const int64_t* w, sbmt_sizes* out) {
  out->n_vertices = w[0];
  out->n_triangles = w[1];
  out->n_cut = w[2];
  out->n_segments = w[4];
}

// The persistent kernel runs only where every band tile's slow owners fit its
// record region (band rows plus the halo row): its record-overflow branch (the
// count pass classifying owners without a record, emission classifying them
// again) faulted the GPU once in testing without a cause found, so it is kept
// unreachable and such tunings run the multi-kernel path.
static bool fused_records_fit(const CallLayout& L, int tile_rows) {
  const int rbi = rb_index(tile_rows);
  return L.fused_ok && rbi >= 0 && L.tcap[rbi] >= (int64_t)(tile_rows + 1) * kCB;
}

static bool tuning_valid(const sbmt_tuning* t) {
  if (t->strategy != SBMT_STRATEGY_MULTI && t->strategy != SBMT_STRATEGY_FUSED) return false;
  if (rb_index(t->tile_rows) < 0) return false;
  if (t->strategy == SBMT_STRATEGY_FUSED && t->tile_rows == 16) return false;
  if (t->groups_per_cu < 0 || t->groups_per_cu > 16) return false;
  return true;
}

static sbmt_tuning default_tuning() {
  sbmt_tuning t;
  memset(&t, 0, sizeof(t));
  t.strategy = SBMT_STRATEGY_MULTI;
  t.tile_rows = 8;
  t.groups_per_cu = 0;
  t.record_cap = 0;
  return t;
}

extern "C" {

sbmt_status sbmt_create(int device, sbmt_handle* out) {
  if (!out) return SBMT_E_INVALID_ARG;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SBMT_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return SBMT_E_DEVICE;
  sbmt_context* c = new (std::nothrow) sbmt_context();
  if (!c) return SBMT_E_DEVICE;
  c->device = device;
  if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->cus < 1)
    c->cus = 256;
  // the device address of this device's scratch array (the device is current)
  if (hipGetSymbolAddress(&c->scratch_ptr, HIP_SYMBOL(scratch)) != hipSuccess || c->scratch_ptr == nullptr) {
    delete c;
    return SBMT_E_DEVICE;
  }
  if (hipHostMalloc((void**)&c->pinned, 8 * sizeof(long long), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return SBMT_E_DEVICE;
  }
  // this device's block segment table (idempotent; finished before any use)
  hipLaunchKernelGGL(k_block_table, dim3(2), dim3(256), 0, 0);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipHostFree(c->pinned);
    delete c;
    return SBMT_E_DEVICE;
  }
  *out = c;
  return SBMT_OK;
}

sbmt_status sbmt_destroy(sbmt_handle h) {
  if (!h) return SBMT_E_INVALID_ARG;
  if (h->pinned) (void)hipHostFree(h->pinned);
  h->pool.release();
  delete h;
  return SBMT_OK;
}

sbmt_status sbmt_query(const sbmt_image* img, sbmt_layout* out) {
  CallLayout L;
  sbmt_status st = make_call_layout(img, 1, 0, false, &L);
  if (st != SBMT_OK) return st;
  if (out) {
    out->stride_s = L.g[0].s;
    out->coarse_w = L.g[0].CW;
    out->coarse_h = L.g[0].CH;
    out->grid_rows = L.g[0].NK;
    out->grid_cols = L.g[0].NI;
    out->workspace_bytes = L.total;
  }
  return SBMT_OK;
}

static sbmt_status single_prepare(const sbmt_image* img, void* workspace, size_t ws_bytes, CallLayout* L) {
  sbmt_status st = make_call_layout(img, 1, 0, true, L);
  if (st != SBMT_OK) return st;
  if (!workspace || ws_bytes < L->total) return SBMT_E_WORKSPACE;
  return SBMT_OK;
}

sbmt_status sbmt_plan(sbmt_handle h, const sbmt_image* img, void* workspace, size_t ws_bytes, sbmt_sizes* out,
                      void* stream) {
  if (!h || !out) return SBMT_E_INVALID_ARG;
  CallLayout L;
  sbmt_status st = single_prepare(img, workspace, ws_bytes, &L);
  if (st != SBMT_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const Shared sh = shared_of(L, workspace, 1);
  OneSrc src;
  src.d = img_of(L, 0, *img, workspace, nullptr);
  if ((st = launch_front(L, src, nullptr, sh, 1, s)) != SBMT_OK) return st;
  if ((st = launch_sizes(L, src, sh, nullptr, s)) != SBMT_OK) return st;
  if (hipMemcpyAsync(h->pinned, sh.sizes, kSizeWords * sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess)
    return SBMT_E_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return SBMT_E_DEVICE;
  if (h->pinned[3] == SBMT_E_PROTOCOL) return SBMT_E_PROTOCOL;
  host_sizes_of((const int64_t*)h->pinned, out);
  if (out->n_vertices > 0x7fffffffLL) return SBMT_E_INDEX_OVERFLOW;
  return SBMT_OK;
}

sbmt_status sbmt_run(sbmt_handle h, const sbmt_image* img, void* workspace, size_t ws_bytes, double* verts,
                     int32_t* tris, uint8_t* codes, void* stream) {
  if (!h) return SBMT_E_INVALID_ARG;
  CallLayout L;
  sbmt_status st = single_prepare(img, workspace, ws_bytes, &L);
  if (st != SBMT_OK) return st;
  const Shared sh = shared_of(L, workspace, 1);
  // the plan's totals bound every write; capacities are the totals themselves
  sbmt_outputs o;
  o.verts = verts;
  o.tris = tris;
  o.codes = codes;
  o.vert_cap = INT64_MAX;
  o.tri_cap = INT64_MAX;
  OneSrc src;
  src.d = img_of(L, 0, *img, workspace, &o);
  return launch_emit(L, src, nullptr, sh, 1, (hipStream_t)stream);
}

sbmt_status sbmt_mesh_async(sbmt_handle h, const sbmt_image* img, void* workspace, size_t ws_bytes, double* verts,
                            int64_t vert_cap, int32_t* tris, uint8_t* codes, int64_t tri_cap, int64_t* sizes_dev,
                            void* stream) {
  if (!h || !sizes_dev || vert_cap < 0 || tri_cap < 0) return SBMT_E_INVALID_ARG;
  CallLayout L;
  sbmt_status st = single_prepare(img, workspace, ws_bytes, &L);
  if (st != SBMT_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const Shared sh = shared_of(L, workspace, 1);
  sbmt_outputs o;
  o.verts = verts;
  o.tris = tris;
  o.codes = codes;
  o.vert_cap = vert_cap;
  o.tri_cap = tri_cap;
  OneSrc src;
  src.d = img_of(L, 0, *img, workspace, &o);
  if ((st = launch_front(L, src, nullptr, sh, 1, s)) != SBMT_OK) return st;
  if ((st = launch_emit(L, src, nullptr, sh, 1, s)) != SBMT_OK) return st;
  return launch_sizes(L, src, sh, sizes_dev, s);
}

sbmt_status sbmt_mesh_noalloc(sbmt_handle h, const sbmt_image* img, double* verts, int64_t vert_cap, int32_t* tris,
                              uint8_t* codes, int64_t tri_cap, int64_t* sizes_dev, void* stream) {
  if (!h || !h->scratch_ptr) return SBMT_E_INVALID_ARG;
  CallLayout L;
  sbmt_status st = make_call_layout(img, 1, 0, true, &L);
  if (st != SBMT_OK) return st;
  if (L.total > (size_t)SBMT_NOALLOC_SCRATCH_BYTES) return SBMT_E_WORKSPACE;
  // the same launches as sbmt_mesh_async, on the device's scratch array
  return sbmt_mesh_async(h, img, h->scratch_ptr, (size_t)SBMT_NOALLOC_SCRATCH_BYTES, verts, vert_cap, tris, codes,
                         tri_cap, sizes_dev, stream);
}

// ---------------------------------------------------------------------------
// Batches.
// ---------------------------------------------------------------------------
sbmt_status sbmt_batch_create(sbmt_handle h, const sbmt_image* imgs, int32_t n, const sbmt_tuning* tuning,
                              size_t* ws_bytes, sbmt_batch* out) {
  if (!h || !out || !imgs || n < 1) return SBMT_E_INVALID_ARG;
  sbmt_tuning t = tuning ? *tuning : default_tuning();
  if (!tuning_valid(&t) || t.record_cap < 0) return SBMT_E_INVALID_ARG;
  sbmt_batch_s* b = new (std::nothrow) sbmt_batch_s();
  if (!b) return SBMT_E_DEVICE;
  b->ctx = h;
  b->imgs.assign(imgs, imgs + n);
  // a batch created for the persistent kernel with the default record count
  // gets records for every owner of its band tiles
  const int64_t rc = (t.strategy == SBMT_STRATEGY_FUSED && t.record_cap == 0) ? -1 : t.record_cap;
  sbmt_status st = make_call_layout(imgs, n, rc, true, &b->L);
  if (st != SBMT_OK) {
    delete b;
    return st;
  }
  if (t.strategy == SBMT_STRATEGY_FUSED && !fused_records_fit(b->L, t.tile_rows)) t.strategy = SBMT_STRATEGY_MULTI;
  b->tune = t;
  b->stage_bytes = b->L.off_cnt - b->L.off_desc;
  b->stage = (unsigned char*)h->pool.get(b->stage_bytes, &b->stage_cls);
  b->psizes = (int64_t*)h->pool.get((size_t)n * kSizeWords * sizeof(int64_t), &b->psizes_cls);
  if (!b->stage || !b->psizes) {
    h->pool.put(b->stage, b->stage_cls);
    h->pool.put(b->psizes, b->psizes_cls);
    delete b;
    return SBMT_E_DEVICE;
  }
  if (ws_bytes) *ws_bytes = b->L.total;
  *out = b;
  return SBMT_OK;
}

sbmt_status sbmt_batch_destroy(sbmt_batch b) {
  if (!b) return SBMT_E_INVALID_ARG;
  b->ctx->pool.put(b->stage, b->stage_cls);
  b->ctx->pool.put(b->psizes, b->psizes_cls);
  delete b;
  return SBMT_OK;
}

sbmt_status sbmt_batch_bind(sbmt_batch b, void* workspace, size_t ws_bytes, const sbmt_outputs* outs, void* stream) {
  if (!b) return SBMT_E_INVALID_ARG;
  if (!workspace || ws_bytes < b->L.total) return SBMT_E_WORKSPACE;
  if (outs)
    for (int i = 0; i < b->L.n; ++i)
      if (outs[i].vert_cap < 0 || outs[i].tri_cap < 0) return SBMT_E_INVALID_ARG;
  const CallLayout& L = b->L;
  unsigned char* st = b->stage;
  memset(st, 0, b->stage_bytes);
  Img* desc = (Img*)(st + (L.off_desc - L.off_desc));
  for (int i = 0; i < L.n; ++i) desc[i] = img_of(L, i, b->imgs[i], workspace, outs ? &outs[i] : nullptr);
  memcpy(st + (L.off_tab - L.off_desc), L.tab.data(), L.tab.size() * sizeof(int64_t));
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync((char*)workspace + L.off_desc, st, b->stage_bytes, hipMemcpyHostToDevice, s) != hipSuccess)
    return SBMT_E_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return SBMT_E_DEVICE;
  b->ws = workspace;
  b->ws_bytes = ws_bytes;
  return SBMT_OK;
}

static ManySrc many_of(const sbmt_batch_s* b) {
  ManySrc m;
  m.d = (const Img*)((char*)b->ws + b->L.off_desc);
  m.n = b->L.n;
  return m;
}
static const int64_t* dtab_of(const sbmt_batch_s* b) { return (const int64_t*)((char*)b->ws + b->L.off_tab); }

sbmt_status sbmt_batch_plan(sbmt_batch b, sbmt_sizes* out, void* stream) {
  if (!b || !out) return SBMT_E_INVALID_ARG;
  if (!b->ws) return SBMT_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const Shared sh = shared_of(b->L, b->ws, rb_index(b->tune.tile_rows));
  const ManySrc src = many_of(b);
  sbmt_status st = launch_front(b->L, src, dtab_of(b), sh, rb_index(b->tune.tile_rows), s);
  if (st != SBMT_OK) return st;
  b->count_rbi = rb_index(b->tune.tile_rows);
  if ((st = launch_sizes(b->L, src, sh, nullptr, s)) != SBMT_OK) return st;
  const size_t bytes = (size_t)b->L.n * kSizeWords * sizeof(int64_t);
  if (hipMemcpyAsync(b->psizes, sh.sizes, bytes, hipMemcpyDeviceToHost, s) != hipSuccess) return SBMT_E_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return SBMT_E_DEVICE;
  sbmt_status worst = SBMT_OK;
  for (int i = 0; i < b->L.n; ++i) {
    host_sizes_of(b->psizes + kSizeWords * i, &out[i]);
    const int64_t sti = b->psizes[kSizeWords * i + 3];
    if (sti == SBMT_E_PROTOCOL) worst = SBMT_E_PROTOCOL;
    if (sti == SBMT_E_INDEX_OVERFLOW && worst == SBMT_OK) worst = SBMT_E_INDEX_OVERFLOW;
  }
  return worst;
}

sbmt_status sbmt_batch_plan_async(sbmt_batch b, void* stream) {
  if (!b) return SBMT_E_INVALID_ARG;
  if (!b->ws) return SBMT_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const Shared sh = shared_of(b->L, b->ws, rb_index(b->tune.tile_rows));
  const ManySrc src = many_of(b);
  sbmt_status st = launch_front(b->L, src, dtab_of(b), sh, rb_index(b->tune.tile_rows), s);
  if (st != SBMT_OK) return st;
  b->count_rbi = rb_index(b->tune.tile_rows);
  if ((st = launch_sizes(b->L, src, sh, nullptr, s)) != SBMT_OK) return st;
  const size_t bytes = (size_t)b->L.n * kSizeWords * sizeof(int64_t);
  if (hipMemcpyAsync(b->psizes, sh.sizes, bytes, hipMemcpyDeviceToHost, s) != hipSuccess) return SBMT_E_DEVICE;
  return SBMT_OK;
}

sbmt_status sbmt_batch_host_sizes(sbmt_batch b, sbmt_sizes* out, int64_t* status) {
  if (!b || !out) return SBMT_E_INVALID_ARG;
  for (int i = 0; i < b->L.n; ++i) {
    host_sizes_of(b->psizes + kSizeWords * i, &out[i]);
    if (status) status[i] = b->psizes[kSizeWords * i + 3];
  }
  return SBMT_OK;
}

sbmt_status sbmt_batch_emit(sbmt_batch b, int64_t* sizes_dev, void* stream) {
  if (!b) return SBMT_E_INVALID_ARG;
  if (!b->ws) return SBMT_E_WORKSPACE;
  if (b->count_rbi < 0) return SBMT_E_INVALID_ARG;  // nothing planned
  hipStream_t s = (hipStream_t)stream;
  const Shared sh = shared_of(b->L, b->ws, b->count_rbi);
  const ManySrc src = many_of(b);
  sbmt_status st = launch_emit(b->L, src, dtab_of(b), sh, b->count_rbi, s);
  if (st != SBMT_OK) return st;
  return launch_sizes(b->L, src, sh, sizes_dev, s);
}

static int fused_groups(const sbmt_batch_s* b) {
  const int gpc = b->tune.groups_per_cu > 0 ? b->tune.groups_per_cu : (b->tune.tile_rows == 4 ? 6 : 4);
  const int64_t nb = b->L.tab[(size_t)(4 + rb_index(b->tune.tile_rows)) * (b->L.n + 1) + b->L.n];
  return (int)std::min<int64_t>(nb, (int64_t)gpc * b->ctx->cus);
}

sbmt_status sbmt_batch_mesh(sbmt_batch b, int64_t* sizes_dev, void* stream) {
  if (!b) return SBMT_E_INVALID_ARG;
  if (!b->ws) return SBMT_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const CallLayout& L = b->L;
  const int rbi = rb_index(b->tune.tile_rows);
  const Shared sh = shared_of(L, b->ws, rbi);
  const ManySrc src = many_of(b);
  const int64_t* dtab = dtab_of(b);
  if (b->tune.strategy == SBMT_STRATEGY_MULTI || !fused_records_fit(L, b->tune.tile_rows)) {
    b->count_rbi = rbi;
    sbmt_status st = launch_front(L, src, dtab, sh, rbi, s);
    if (st != SBMT_OK) return st;
    if ((st = launch_emit(L, src, dtab, sh, rbi, s)) != SBMT_OK) return st;
    return launch_sizes(L, src, sh, sizes_dev, s);
  }
  const int64_t ncb = L.tab[(size_t)L.n];
  if (ncb > 0x7fffffffLL) return SBMT_E_INVALID_ARG;
  hipLaunchKernelGGL(k_coarsen<ManySrc>, dim3((unsigned)ncb), dim3(256), 0, s, src, dtab, sh);
  hipLaunchKernelGGL(k_segcount<ManySrc>, dim3((unsigned)L.tab[(size_t)6 * (L.n + 1) + L.n]), dim3(256), 0, s, src,
                     dtab + (size_t)6 * (L.n + 1), sh);
  const int64_t nbands = L.tab[(size_t)(4 + rbi) * (L.n + 1) + L.n];
  const int64_t* btab = dtab + (size_t)(4 + rbi) * (L.n + 1);
  uint16_t* halo = (uint16_t*)((char*)b->ws + L.off_halo);
  const int64_t* ttab = dtab + (size_t)(1 + rbi) * (L.n + 1);
  const int grid = fused_groups(b);
  if (b->tune.tile_rows == 4)
    hipLaunchKernelGGL((k_fused<4>), dim3(grid), dim3(kThreads), 0, s, src, btab, ttab, sh, nbands, halo);
  else
    hipLaunchKernelGGL((k_fused<8>), dim3(grid), dim3(kThreads), 0, s, src, btab, ttab, sh, nbands, halo);
  if (sizes_dev) {
    const int64_t n4 = kSizeWords * (int64_t)L.n;
    hipLaunchKernelGGL(k_copy_sizes, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s, (const int64_t*)sh.sizes,
                       n4, sizes_dev);
  }
  return hipGetLastError() == hipSuccess ? SBMT_OK : SBMT_E_DEVICE;
}

sbmt_status sbmt_batch_sizes(sbmt_batch b, sbmt_sizes* out, int64_t* status, void* stream) {
  if (!b || !out) return SBMT_E_INVALID_ARG;
  if (!b->ws) return SBMT_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = (size_t)b->L.n * kSizeWords * sizeof(int64_t);
  if (hipMemcpyAsync(b->psizes, (char*)b->ws + b->L.off_sizes, bytes, hipMemcpyDeviceToHost, s) != hipSuccess)
    return SBMT_E_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return SBMT_E_DEVICE;
  for (int i = 0; i < b->L.n; ++i) {
    host_sizes_of(b->psizes + kSizeWords * i, &out[i]);
    if (status) status[i] = b->psizes[kSizeWords * i + 3];
  }
  return SBMT_OK;
}

sbmt_status sbmt_batch_get_tuning(sbmt_batch b, sbmt_tuning* out) {
  if (!b || !out) return SBMT_E_INVALID_ARG;
  *out = b->tune;
  return SBMT_OK;
}

sbmt_status sbmt_batch_set_tuning(sbmt_batch b, const sbmt_tuning* t) {
  if (!b || !t) return SBMT_E_INVALID_ARG;
  sbmt_tuning x = *t;
  if (!tuning_valid(&x)) return SBMT_E_INVALID_ARG;
  if (x.record_cap != b->tune.record_cap) return SBMT_E_INVALID_ARG;  // fixed by the layout
  if (x.strategy == SBMT_STRATEGY_FUSED && !fused_records_fit(b->L, x.tile_rows)) return SBMT_E_INVALID_ARG;
  b->tune = x;
  return SBMT_OK;
}

// Autotuner: time every candidate tuning on this batch (one warm-up and
// `reps` timed runs of the whole path, HIP events on `stream`) and keep the
// fastest.  Outputs must be bound; they are overwritten.
sbmt_status sbmt_batch_tune(sbmt_batch b, int32_t reps, sbmt_tuning* best, float* best_ms, void* stream) {
  if (!b || reps < 1) return SBMT_E_INVALID_ARG;
  if (!b->ws) return SBMT_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  std::vector<sbmt_tuning> cand;
  for (int rb : {4, 8, 16}) {
    sbmt_tuning t = b->tune;
    t.strategy = SBMT_STRATEGY_MULTI;
    t.tile_rows = rb;
    t.groups_per_cu = 0;
    cand.push_back(t);
  }
  for (int rb : {4, 8})
    for (int gpc : {1, 2, 3}) {
      if (!fused_records_fit(b->L, rb)) continue;
      sbmt_tuning t = b->tune;
      t.strategy = SBMT_STRATEGY_FUSED;
      t.tile_rows = rb;
      t.groups_per_cu = gpc;
      cand.push_back(t);
    }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return SBMT_E_DEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return SBMT_E_DEVICE;
  }
  const sbmt_tuning saved = b->tune;
  float bestt = 1e30f;
  sbmt_tuning bt = saved;
  sbmt_status result = SBMT_OK;
  for (const sbmt_tuning& t : cand) {
    b->tune = t;
    sbmt_status st = sbmt_batch_mesh(b, nullptr, stream);
    if (st == SBMT_OK && hipEventRecord(e0, s) != hipSuccess) st = SBMT_E_DEVICE;
    for (int r = 0; r < reps && st == SBMT_OK; ++r) st = sbmt_batch_mesh(b, nullptr, stream);
    if (st == SBMT_OK && hipEventRecord(e1, s) != hipSuccess) st = SBMT_E_DEVICE;
    if (st == SBMT_OK && hipEventSynchronize(e1) != hipSuccess) st = SBMT_E_DEVICE;
    float ms = 0.f;
    if (st == SBMT_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = SBMT_E_DEVICE;
    if (st != SBMT_OK) {
      result = st;
      break;
    }
    ms /= (float)reps;
    if (ms < bestt) {
      bestt = ms;
      bt = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->tune = result == SBMT_OK ? bt : saved;
  if (best) *best = b->tune;
  if (best_ms) *best_ms = bestt;
  return result;
}

int32_t sbmt_num_classes(void) { return SBMT_NUM_CLASSES; }

int32_t sbmt_class_code(int32_t class_id) {
  static const int32_t codes[] = {SBMT_CLASS_CODES_INIT};
  if (class_id < 1 || class_id > SBMT_NUM_CLASSES) return -1;
  return codes[class_id];
}

sbmt_status sbmt_pre_query(const sbmt_image* img, size_t* workspace_bytes, int64_t* vert_bound, int64_t* tri_bound) {
  PreLayout P;
  sbmt_status st = pre_layout(img, false, &P);
  if (st != SBMT_OK) return st;
  if (workspace_bytes) *workspace_bytes = P.total;
  if (vert_bound) *vert_bound = P.nown + P.nmid;
  if (tri_bound) *tri_bound = 4 * P.nown;
  return SBMT_OK;
}

// Arguments of the preprocessing kernels over workspace w (layout PL).
static PreArgs pre_args(const PreLayout& PL, char* w, double a, double b, double c) {
  PreArgs P;
  P.a = a;
  P.b = b;
  P.c = c;
  P.verts = nullptr;
  P.on_polyline = nullptr;
  P.tris = nullptr;
  P.vcap = P.tcap = 0;
  P.mid = (uint8_t*)(w + PL.off_mid);
  P.split = (int32_t*)(w + PL.off_split);
  P.flags = (uint8_t*)(w + PL.off_flags);
  P.ins_base = (int64_t*)(w + PL.off_ins);
  P.counts = (int64_t*)(w + PL.off_counts);
  P.snap_mid = (int32_t*)(w + PL.off_snap);
  P.rcount = PL.off_rcount ? (uint32_t*)(w + PL.off_rcount) : nullptr;
  P.rtri = PL.off_rtri ? (uint32_t*)(w + PL.off_rtri) : nullptr;
  P.rbase = PL.off_rbase ? (int64_t*)(w + PL.off_rbase) : nullptr;
  P.gsizes = (const int64_t*)(w + PL.off_out);
  P.otris = nullptr;
  P.ocodes = nullptr;
  P.otcap = 0;
  P.overts = nullptr;
  P.ovcap = 0;
  P.used = PL.off_used ? (uint8_t*)(w + PL.off_used) : nullptr;
  P.usedcap = PL.off_used ? PL.nown + PL.nmid : 0;
  P.vmap = PL.off_vmap ? (int32_t*)(w + PL.off_vmap) : nullptr;
  P.vbsum = PL.off_vbsum ? (int64_t*)(w + PL.off_vbsum) : nullptr;
  P.nused = PL.off_nused ? (int64_t*)(w + PL.off_nused) : nullptr;
  P.tlist = PL.off_tlist ? (int32_t*)(w + PL.off_tlist) : nullptr;
  P.rtbase = PL.off_rtbase ? (int64_t*)(w + PL.off_rtbase) : nullptr;
  P.cbase = PL.off_cbase ? (int32_t*)(w + PL.off_cbase) : nullptr;
  P.cblk = PL.off_cblk ? (int64_t*)(w + PL.off_cblk) : nullptr;
  P.cstore = PL.off_cstore ? (uint32_t*)(w + PL.off_cstore) : nullptr;
  P.ccap = PL.off_cstore ? PL.ccap : 0;
  return P;
}
// Steps 1-3 (the grid, with its triangles when `triangles`), then the sizes
// record at PL.off_out.
static sbmt_status pre_launch_grid(const PreLayout& PL, const OneSrc& src, const PreArgs& P, const Shared& sh, char* w,
                                   bool triangles, hipStream_t s) {
  const Geo& g = PL.L.g[0];
  const int64_t ncb = PL.L.tab[PL.L.n];
  const int64_t nseg = PL.L.nseg;
  const int64_t nwb = ((int64_t)(g.CH + 1) * g.wpr + 255) / 256;  // raster words of rows -1 .. CH - 1
  const int nchunk = (g.NI + kPreQuad - 1) / kPreQuad;  // 1024-vertex chunks of a lattice row
  const int64_t nqb = (nseg + 3) / 4;                    // four row segments (waves) per block
  if ((int64_t)g.NK * nchunk > 0x7fffffffLL) return SBMT_E_INVALID_ARG;
  if (ncb > 0x7fffffffLL || nseg > 0x7fffffffLL || nwb > 0x7fffffffLL) return SBMT_E_INVALID_ARG;
  hipLaunchKernelGGL(k_coarsen<OneSrc>, dim3((unsigned)ncb), dim3(256), 0, s, src, (const int64_t*)nullptr, sh);
  hipLaunchKernelGGL(k_pre_clear, dim3(1024), dim3(256), 0, s, P, PL.nmid);
  hipLaunchKernelGGL(k_pre_lattice, dim3((unsigned)(g.NK * nchunk)), dim3(256), 0, s, src, P, nchunk);
  hipLaunchKernelGGL(k_pre_snap, dim3((unsigned)nwb), dim3(256), 0, s, src, P);
  hipLaunchKernelGGL(k_pre_repel, dim3((unsigned)nwb), dim3(256), 0, s, src, P);
  hipLaunchKernelGGL(k_pre_split, dim3((unsigned)nwb), dim3(256), 0, s, src, P);
  hipLaunchKernelGGL(k_pre_count, dim3((unsigned)nqb), dim3(256), 0, s, src, P, sh);
  hipLaunchKernelGGL(k_scan_reduce, dim3(PL.L.nblk), dim3(kScanThreads), 0, s, sh);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanThreads), 0, s, sh);
  hipLaunchKernelGGL(k_scan_apply, dim3(PL.L.nblk), dim3(kScanThreads), 0, s, sh);
  hipLaunchKernelGGL(k_pre_inserted, dim3((unsigned)nqb), dim3(256), 0, s, src, P, sh);
  if (triangles) hipLaunchKernelGGL(k_pre_triangles, dim3((unsigned)nqb), dim3(256), 0, s, src, P, sh);
  hipLaunchKernelGGL(k_pre_sizes, dim3(1), dim3(1), 0, s, src, P, sh, (int64_t*)(w + PL.off_out));
  return hipGetLastError() == hipSuccess ? SBMT_OK : SBMT_E_DEVICE;
}
static sbmt_status pre_read_sizes(sbmt_handle h, const int64_t* dev, int n, int64_t* counts, hipStream_t s) {
  if (hipMemcpyAsync(h->pinned, dev, n * sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return SBMT_E_DEVICE;
  for (int j = 0; j < n; ++j) counts[j] = h->pinned[j];
  return SBMT_OK;
}

sbmt_status sbmt_preprocess(sbmt_handle h, const sbmt_image* img, double a, double b, double c, void* workspace,
                            size_t ws_bytes, double* verts, uint8_t* on_polyline, int64_t vert_cap, int32_t* tris,
                            int64_t tri_cap, int64_t* counts, void* stream) {
  if (!h || !counts || vert_cap < 0 || tri_cap < 0) return SBMT_E_INVALID_ARG;
  if ((vert_cap > 0 && (!verts || !on_polyline)) || (tri_cap > 0 && !tris)) return SBMT_E_INVALID_ARG;
  PreLayout PL;
  sbmt_status st = pre_layout(img, true, &PL);
  if (st != SBMT_OK) return st;
  const Geo& g = PL.L.g[0];
  if (!pre_thresholds_ok(a, b, c, (double)g.h / g.U)) return SBMT_E_INVALID_ARG;
  if (!workspace || ws_bytes < PL.total) return SBMT_E_WORKSPACE;
  // every vertex of the lattice needs room before the kernels write it
  if (vert_cap < PL.nown) return SBMT_E_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)workspace;
  const Shared sh = shared_of(PL.L, workspace, 1);
  OneSrc src;
  src.d = img_of(PL.L, 0, *img, workspace, nullptr);
  PreArgs P = pre_args(PL, w, a, b, c);
  P.verts = verts;
  P.on_polyline = on_polyline;
  P.tris = tris;
  P.vcap = vert_cap;
  P.tcap = tri_cap;
  if ((st = pre_launch_grid(PL, src, P, sh, w, true, s)) != SBMT_OK) return st;
  if ((st = pre_read_sizes(h, (const int64_t*)(w + PL.off_out), 6, counts, s)) != SBMT_OK) return st;
  return (sbmt_status)counts[5];
}

sbmt_status sbmt_pre_mesh_query(const sbmt_image* img, size_t* workspace_bytes, int64_t* grid_vert_bound) {
  PreLayout P;
  sbmt_status st = pre_layout(img, false, &P, true);
  if (st != SBMT_OK) return st;
  if (workspace_bytes) *workspace_bytes = P.total;
  if (grid_vert_bound) *grid_vert_bound = P.nown + P.nmid;
  return SBMT_OK;
}

sbmt_status sbmt_preprocess_mesh(sbmt_handle h, const sbmt_image* img, double a, double b, double c, void* workspace,
                                 size_t ws_bytes, double* verts, int64_t vert_cap, int32_t* tris, uint8_t* codes,
                                 int64_t tri_cap, int64_t* counts, void* stream) {
  if (!h || !counts || vert_cap < 0 || tri_cap < 0) return SBMT_E_INVALID_ARG;
  if ((vert_cap > 0 && !verts) || (tri_cap > 0 && (!tris || !codes))) return SBMT_E_INVALID_ARG;
  PreLayout PL;
  sbmt_status st = pre_layout(img, true, &PL, true);
  if (st != SBMT_OK) return st;
  const Geo& g = PL.L.g[0];
  if (!pre_thresholds_ok(a, b, c, (double)g.h / g.U)) return SBMT_E_INVALID_ARG;
  if (!workspace || ws_bytes < PL.total) return SBMT_E_WORKSPACE;
  if (PL.nown + PL.nmid > 0x7fffffffLL) return SBMT_E_INDEX_OVERFLOW;  // grid vertex indices in 32 bits
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)workspace;
  const Shared sh = shared_of(PL.L, workspace, 1);
  OneSrc src;
  src.d = img_of(PL.L, 0, *img, workspace, nullptr);
  PreArgs P = pre_args(PL, w, a, b, c);
  // the grid goes to the workspace; the mesh keeps the grid vertices its
  // triangles use, then the new ones
  P.verts = (double*)(w + PL.off_gverts);
  P.on_polyline = (uint8_t*)(w + PL.off_onp);
  P.vcap = PL.nown + PL.nmid;
  P.overts = verts;
  P.ovcap = vert_cap;
  P.otris = tris;
  P.ocodes = codes;
  P.otcap = tri_cap;
  if ((st = pre_launch_grid(PL, src, P, sh, w, false, s)) != SBMT_OK) return st;
  const int64_t nqb = (PL.L.nseg + 3) / 4;
  int64_t* out2 = (int64_t*)(w + PL.off_out2);
  const Geo& gg = PL.L.g[0];
  const int64_t nwb = ((int64_t)(gg.CH + 1) * gg.wpr + 255) / 256;
  // grid-stride passes: as many blocks as run at once on the device
  const int ncu = std::max(h->cus, 1);
  auto resident = [ncu](auto* k) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(k), 256, 0) != hipSuccess ||
        nb < 1)
      nb = 2;
    return dim3((unsigned)(nb * ncu));
  };
  hipLaunchKernelGGL(k_pre_mesh_touch, dim3((unsigned)nwb), dim3(256), 0, s, src, P);
  // the touched owners' list: counts per row segment, their offsets, the list
  hipLaunchKernelGGL(k_pre_mesh_tcount, dim3((unsigned)nqb), dim3(256), 0, s, src, P, sh);
  hipLaunchKernelGGL(k_scan_reduce, dim3(PL.L.nblk), dim3(kScanThreads), 0, s, sh);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanThreads), 0, s, sh);
  hipLaunchKernelGGL(k_scan_apply, dim3(PL.L.nblk), dim3(kScanThreads), 0, s, sh);
  hipLaunchKernelGGL(k_pre_mesh_count, dim3((unsigned)nqb), dim3(256), 0, s, src, P, sh);
  hipLaunchKernelGGL(k_pre_mesh_probe_owner, resident(&k_pre_mesh_probe_owner), dim3(256), 0, s, src, P, sh);
  // slots of the cut triangles' kept outputs, then their counts
  if (PL.ncblk > 0x7fffffffLL) return SBMT_E_INVALID_ARG;
  hipLaunchKernelGGL(k_pre_cut_count, dim3((unsigned)PL.ncblk), dim3(256), 0, s, P, sh);
  hipLaunchKernelGGL(k_pre_cut_top, dim3(1), dim3(256), 0, s, P, PL.ncblk);
  hipLaunchKernelGGL(k_pre_cut_apply, dim3((unsigned)PL.ncblk), dim3(256), 0, s, P, sh);
  hipLaunchKernelGGL(k_pre_mesh_cut_count, resident(&k_pre_mesh_cut_count), dim3(256), 0, s, src, P, sh);
  // the output counts per row segment and their offsets
  hipLaunchKernelGGL(k_pre_mesh_segsum, dim3((unsigned)nqb), dim3(256), 0, s, src, P, sh);
  hipLaunchKernelGGL(k_scan_reduce, dim3(PL.L.nblk), dim3(kScanThreads), 0, s, sh);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanThreads), 0, s, sh);
  hipLaunchKernelGGL(k_scan_apply, dim3(PL.L.nblk), dim3(kScanThreads), 0, s, sh);
  if (PL.nvblk > 0x7fffffffLL) return SBMT_E_INVALID_ARG;
  hipLaunchKernelGGL(k_pre_vscan_count, dim3((unsigned)PL.nvblk), dim3(256), 0, s, P);
  hipLaunchKernelGGL(k_pre_vscan_top, dim3(1), dim3(256), 0, s, P, PL.nvblk);
  hipLaunchKernelGGL(k_pre_vscan_apply, dim3((unsigned)PL.nvblk), dim3(256), 0, s, P);
  hipLaunchKernelGGL(k_pre_mesh_vbase, dim3((unsigned)nqb), dim3(256), 0, s, src, P, sh);
  hipLaunchKernelGGL(k_pre_mesh_edge_verts, resident(&k_pre_mesh_edge_verts), dim3(256), 0, s, src, P);
  hipLaunchKernelGGL(k_pre_mesh_inner_verts, resident(&k_pre_mesh_inner_verts), dim3(256), 0, s, src, P);
  hipLaunchKernelGGL(k_pre_mesh_triangles, dim3((unsigned)nqb), dim3(256), 0, s, src, P, sh);
  hipLaunchKernelGGL(k_pre_mesh_whole_tris, resident(&k_pre_mesh_whole_tris), dim3(256), 0, s, src, P);
  hipLaunchKernelGGL(k_pre_mesh_cut_tris, resident(&k_pre_mesh_cut_tris), dim3(256), 0, s, src, P);
  hipLaunchKernelGGL(k_pre_mesh_sizes, dim3(1), dim3(1), 0, s, P, sh, out2);
  if (hipGetLastError() != hipSuccess) return SBMT_E_DEVICE;
  if ((st = pre_read_sizes(h, out2, 8, counts, s)) != SBMT_OK) return st;
  return (sbmt_status)counts[5];
}

const char* sbmt_status_string(sbmt_status s) {
  switch (s) {
    case SBMT_OK: return "ok";
    case SBMT_E_INVALID_ARG: return "invalid argument";
    case SBMT_E_UNSUPPORTED_GRID_H: return "unsupported grid_h (p/2^q up to 6 with 3h <= 2s, q <= 8, and 16 s 4^q side < 2^31)";
    case SBMT_E_INDEX_OVERFLOW: return "vertex count exceeds int32";
    case SBMT_E_WORKSPACE: return "workspace missing or too small";
    case SBMT_E_DEVICE: return "HIP runtime error";
    case SBMT_E_PROTOCOL: return "inadmissible local boundary pattern";
    case SBMT_E_CAPACITY: return "mesh larger than the output capacity";
  }
  return "unknown status";
}

}  // extern "C"
