// SBMT hot path for MI355X (gfx950): bitmap -> boundary -> exact per-triangle
// classification -> canonical class -> template lookup -> closed mesh
// (arXiv 2602.19474, Sec. 3.3, Alg. 1, Alg. 2, App. G).
//
// Kernels
//   k_coarsen  block-majority coarse raster as packed bits, with a background ring
//   k_count    per row segment (row k, CB owners): classify every owner, sum
//              vertex/triangle counts (plan)
//   k_scan_*   exclusive prefix sum of the per-segment counts -> output offsets
//   k_emit     per tile (RB rows x CB owners): re-classify, prefix-sum the owner
//              counts in LDS (with a one-row, one-column halo for neighbour ids),
//              write FP64 vertices, int32 triangles and u8 class codes
//
// The output order is fixed by the owner numbering and does not depend on
// the tile shape.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

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
SBMT_HD uint32_t lut_emit(int cls, int rot, int t, int j) { return sbmt_lut_emit[cls][rot][t][j]; }

constexpr int kThreads = 256;
constexpr int kCB = 256;          // owners per row segment
constexpr int kOPT = kCB / kThreads;  // owners per thread per row
constexpr int kRB = 8;            // rows per emission tile
constexpr int kRec = 192;         // slow-owner records kept in LDS per emission tile
constexpr int kScanThreads = 1024;
constexpr int kScanChunk = 4 * kScanThreads;


struct Work {
  uint32_t* bits;
  int4* seg_cnt;       // [nseg] (nv, nt, ncut, err)
  longlong2* seg_off;  // [nseg] exclusive (vertex, triangle) offsets
  longlong4* blk;      // [nblk] scan block sums / offsets
  long long* tot;      // [8] nv, nt, ncut, err
};


// ---------------------------------------------------------------------------
// Coarse raster: bit (R + ring, C + ringC) = [2 * #fg pixels of block (R, C) >= s^2].
// One lane per sample; a wave covers 64 consecutive stored columns and packs
// them with a ballot; samples outside the image (the ring) are background.
// grid (ceil(32 wpr / 256), CH + 2 ring), 256 threads.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_coarsen(Geo g, const uint8_t* __restrict__ bm, uint32_t* __restrict__ bits,
                                                 long long* __restrict__ tot) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int gw = blockIdx.x * 4 + wv;  // 64-bit group of the stored row
  const int rr = blockIdx.y;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 8) tot[threadIdx.x] = 0;
  const int R = rr - kRing;
  const int C = 64 * gw + lane - kRingC;
  int fg = 0;
  if (R >= 0 && R < g.CH && C >= 0 && C < g.CW) {
    const int s = g.s;
    const int r0 = s * R, r1 = min(r0 + s, g.H);
    const int c0 = s * C, c1 = min(c0 + s, g.W);
    int cnt = 0;
    for (int r = r0; r < r1; ++r) {
      const uint8_t* row = bm + (int64_t)r * g.stride;
      for (int c = c0; c < c1; ++c) cnt += row[c] != 0;
    }
    fg = 2 * cnt >= s * s;
  }
  const unsigned long long m = __ballot(fg);
  const int w = 2 * gw + lane;
  if (lane < 2 && w < g.wpr) bits[(int64_t)rr * g.wpr + w] = (uint32_t)(m >> (32 * lane));
}

// Stage the coarse-raster window of a tile (grid rows k0 .. k0 + nk - 1, owner
// columns cfirst .. clast) in LDS; returns the view.  Sizes are checked on the
// host (tile_window_fits).
constexpr int kWinRows = 16, kWinWords = 16;

__device__ __forceinline__ Bits stage_window(const Geo& g, const uint32_t* __restrict__ bits, uint32_t* win, int rlo, int rhi,
                             int cfirst, int clast) {
  const int x0 = g.X0 + 4 * g.h * cfirst, x1 = g.X0 + 4 * g.h * clast + 2 * g.h;
  const int wlo = (clo_of(g, x0) + kRingC) >> 5;
  const int whi = ((clo_of(g, x1) + 2 + kRingC) >> 5) + 1;
  const int nw = whi - wlo + 1, nr = rhi - rlo + 1;
  for (int t = threadIdx.x; t < nr * nw; t += blockDim.x) {
    const int r = t / nw, w = t - r * nw;
    win[r * nw + w] = bits[(int64_t)(rlo + r) * g.wpr + wlo + w];
  }
  Bits b;
  b.p = win;
  b.wpr = nw;
  b.rr0 = rlo;
  b.cc0 = 32 * wlo;
  return b;
}

__device__ __forceinline__ int wave_sum(int v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Plan: classify every owner of kRB row segments and sum the counts per
// segment.  Owners whose window is not uniform are queued in LDS for the whole
// tile and classified densely afterwards.
// grid (NCB, ceil(NK / kRB)), kThreads threads, kOPT owners per thread per row.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_count(Geo g, const uint32_t* __restrict__ bits_g,
                                                    int4* __restrict__ seg_cnt, long long* __restrict__ tot) {
  __shared__ int acc[kRB][4];
  __shared__ int rowR[kRB];
  __shared__ uint16_t q1[kRB * kCB];
  __shared__ uint16_t q2[kRB * kCB];
  __shared__ int n1, n2;
  __shared__ uint32_t win[kWinRows * kWinWords];
  const int cb = blockIdx.x;
  const int k0 = blockIdx.y * kRB;
  const int c0 = cb * kCB;
  const int lane = threadIdx.x & 63;
  if (threadIdx.x < kRB) {
    rowR[threadIdx.x] = row_cell(k0 + threadIdx.x, g.h, g.s);
    acc[threadIdx.x][0] = acc[threadIdx.x][1] = acc[threadIdx.x][2] = acc[threadIdx.x][3] = 0;
  }
  if (threadIdx.x == 0) n1 = n2 = 0;
  __syncthreads();
  const int klast = min(k0 + kRB, g.NK) - 1;
  const Bits bw = stage_window(g, bits_g, win, rowR[0] + kRing, rowR[klast - k0] + 2 + kRing, c0,
                               min(c0 + kCB, g.NI) - 1);
  __syncthreads();
  // uniform windows, one owner per thread; the others are queued
  for (int r = 0; r < kRB; ++r) {
    const int k = k0 + r;
    if (k >= g.NK) break;
    int nv = 0, nt = 0;
    for (int j = 0; j < kOPT; ++j) {
      const int c = c0 + j * kThreads + threadIdx.x;
      if (c >= g.NI) continue;
      const Frame f = owner_frame(g, bw, k, c, rowR[r]);
      if (frame_uniform(f)) {
        const uint32_t fi = fast_info(g, f);
        nv += info_nv(fi);
        nt += info_nt(fi);
      } else {
        q1[atomicAdd(&n1, 1)] = (uint16_t)(r * kCB + (c - c0));
      }
    }
    nv = wave_sum(nv);
    nt = wave_sum(nt);
    if (lane == 0 && (nv | nt)) { atomicAdd(&acc[r][0], nv); atomicAdd(&acc[r][1], nt); }
  }
  __syncthreads();
  // non-uniform windows: quiet owners (no segment reaches them) or slow ones
  for (int q = threadIdx.x; q < n1; q += kThreads) {
    const int e = q1[q], r = e / kCB, c = c0 + (e - r * kCB);
    const Frame f = owner_frame(g, bw, k0 + r, c, rowR[r]);
    uint32_t fi = 0;
    if (needs_slow(g, f, fi)) {
      q2[atomicAdd(&n2, 1)] = (uint16_t)e;
    } else {
      atomicAdd(&acc[r][0], info_nv(fi));
      atomicAdd(&acc[r][1], info_nt(fi));
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < n2; q += kThreads) {
    const int e = q2[q], r = e / kCB, c = c0 + (e - r * kCB);
    const Frame f = owner_frame(g, bw, k0 + r, c, rowR[r]);
    Slow sr;
    slow_classify(g, f, sr);
    atomicAdd(&acc[r][0], info_nv(sr.info));
    atomicAdd(&acc[r][1], info_nt(sr.info));
    atomicAdd(&acc[r][2], info_ncut(sr.info));
    if (info_err(sr.info)) atomicOr(&acc[r][3], 1);
  }
  __syncthreads();
  if (threadIdx.x < kRB && k0 + (int)threadIdx.x < g.NK) {
    const int r = threadIdx.x;
    seg_cnt[(int64_t)(k0 + r) * g.NCB + cb] = make_int4(acc[r][0], acc[r][1], acc[r][2], acc[r][3]);
    if (acc[r][3]) atomicOr((unsigned long long*)&tot[3], 1ull);
  }
}

// ---------------------------------------------------------------------------
// Exclusive scan of the per-segment (nv, nt) counts, three phases.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    T u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}

// block-wide exclusive scan of (a, b) over kScanThreads threads; returns totals
__device__ void block_excl_scan2(long long& a, long long& b, long long* sa, long long* sb,
                                 long long& ta, long long& tb) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  long long ia = wave_incl_scan(a, lane), ib = wave_incl_scan(b, lane);
  if (lane == 63) { sa[wv] = ia; sb[wv] = ib; }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int nw = blockDim.x >> 6;
    long long xa = threadIdx.x < nw ? sa[threadIdx.x] : 0, xb = threadIdx.x < nw ? sb[threadIdx.x] : 0;
    long long ya = wave_incl_scan(xa, lane), yb = wave_incl_scan(xb, lane);
    if (threadIdx.x < nw) { sa[threadIdx.x] = ya - xa; sb[threadIdx.x] = yb - xb; }
    if (threadIdx.x == nw - 1) { sa[32] = ya; sb[32] = yb; }
  }
  __syncthreads();
  a = ia - a + sa[wv];
  b = ib - b + sb[wv];
  ta = sa[32];
  tb = sb[32];
  __syncthreads();
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const int4* __restrict__ seg_cnt, int64_t nseg,
                                                              longlong4* __restrict__ blk) {
  __shared__ long long sa[33], sb[33];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  long long a = 0, b = 0, c = 0;
  for (int q = 0; q < 4; ++q) {
    const int64_t j = base + (int64_t)threadIdx.x * 4 + q;
    if (j < nseg) { int4 v = seg_cnt[j]; a += v.x; b += v.y; c += v.z; }
  }
  long long ta, tb, tc, dummy;
  block_excl_scan2(a, b, sa, sb, ta, tb);
  long long z = 0;
  block_excl_scan2(c, z, sa, sb, tc, dummy);
  if (threadIdx.x == 0) blk[blockIdx.x] = make_longlong4(ta, tb, tc, 0);
}

__global__ void __launch_bounds__(kScanThreads) k_scan_blocks(longlong4* __restrict__ blk, int nblk,
                                                              long long* __restrict__ tot) {
  __shared__ long long sa[33], sb[33];
  long long ra = 0, rb = 0, rc = 0;
  for (int base = 0; base < nblk; base += kScanThreads) {
    const int j = base + threadIdx.x;
    longlong4 v = j < nblk ? blk[j] : make_longlong4(0, 0, 0, 0);
    long long a = v.x, b = v.y, ta, tb;
    block_excl_scan2(a, b, sa, sb, ta, tb);
    long long c = v.z, z = 0, tc, d;
    block_excl_scan2(c, z, sa, sb, tc, d);
    if (j < nblk) blk[j] = make_longlong4(ra + a, rb + b, rc + c, 0);
    ra += ta; rb += tb; rc += tc;
  }
  if (threadIdx.x == 0) { tot[0] = ra; tot[1] = rb; tot[2] = rc; }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const int4* __restrict__ seg_cnt, int64_t nseg,
                                                             const longlong4* __restrict__ blk,
                                                             longlong2* __restrict__ seg_off) {
  __shared__ long long sa[33], sb[33];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  int4 v[4];
  long long a = 0, b = 0;
  for (int q = 0; q < 4; ++q) {
    const int64_t j = base + (int64_t)threadIdx.x * 4 + q;
    v[q] = j < nseg ? seg_cnt[j] : make_int4(0, 0, 0, 0);
    a += v[q].x; b += v[q].y;
  }
  long long ta, tb;
  block_excl_scan2(a, b, sa, sb, ta, tb);
  const longlong4 bo = blk[blockIdx.x];
  a += bo.x; b += bo.y;
  for (int q = 0; q < 4; ++q) {
    const int64_t j = base + (int64_t)threadIdx.x * 4 + q;
    if (j < nseg) seg_off[j] = make_longlong2(a, b);
    a += v[q].x; b += v[q].y;
  }
}

// ---------------------------------------------------------------------------
// Emission.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Emission of a tile of kRB rows x kCB owners.
//   1. counts of the tile's owners plus a one-row / one-column halo; owners
//      with a non-uniform window are queued and classified densely, their
//      classification kept in LDS (up to kRec of them; later ones are
//      classified again at emission);
//   2. prefix sums of the counts of every row in LDS, plus the segment bases
//      from the plan, give each owner's first vertex and triangle id and its
//      neighbours' ids;
//   3. fast owners are emitted one per thread, then all slow owners densely.
// grid (NCB, ceil(NK / kRB)), kThreads threads.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_emit(Geo g, const uint32_t* __restrict__ bits_g,
                                                   const longlong2* __restrict__ seg_off,
                                                   const long long* __restrict__ tot, int64_t vcap, int64_t tcap,
                                                   double* __restrict__ verts, int32_t* __restrict__ tris,
                                                   uint8_t* __restrict__ codes) {
  constexpr int W = kCB + 2;  // columns c0-1 .. c0+CB
  __shared__ uint32_t info[kRB + 1][W];
  __shared__ int voff[kRB + 1][W];
  __shared__ int16_t toff[kRB][W];
  __shared__ uint32_t win[kWinRows * kWinWords];
  __shared__ uint16_t queue[(kRB + 1) * W];
  __shared__ uint16_t q1[(kRB + 1) * W];
  __shared__ SlowRec rec[kRec];
  __shared__ int qn, n1;
  __shared__ int rowR[kRB + 1];
  __shared__ long long tb[kRB];
  __shared__ int part[kRB + 1][2][kThreads / 64];
  __shared__ int trow[kRB];
  if (tot[0] > vcap || tot[1] > tcap || tot[3] != 0) return;  // does not fit / plan failed
  const int cb = blockIdx.x;
  const int k0 = blockIdx.y * kRB;
  const int c0 = cb * kCB;
  if (threadIdx.x <= kRB) rowR[threadIdx.x] = row_cell(k0 + threadIdx.x, g.h, g.s);
  if (threadIdx.x == 0) qn = n1 = 0;
  __syncthreads();
  const int klast = min(k0 + kRB + 1, g.NK) - 1;
  const Bits bw = stage_window(g, bits_g, win, rowR[0] + kRing, rowR[max(klast - k0, 0)] + 2 + kRing,
                               max(c0 - 1, 0), min(c0 + kCB + 1, g.NI) - 1);
  __syncthreads();
  // 1. counts: uniform windows one owner per thread, then the queued ones densely
  for (int idx = threadIdx.x; idx < (kRB + 1) * W; idx += kThreads) {
    const int rr = idx / W, col = idx - rr * W;
    const int k = k0 + rr, c = c0 - 1 + col;
    uint32_t fi = 0;
    if (k < g.NK && c >= 0 && c < g.NI) {
      const Frame f = owner_frame(g, bw, k, c, rowR[rr]);
      if (frame_uniform(f)) fi = fast_info(g, f);
      else q1[atomicAdd(&n1, 1)] = (uint16_t)idx;
    }
    info[rr][col] = fi;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < n1; q += kThreads) {
    const int idx = q1[q], rr = idx / W, col = idx - rr * W;
    const Frame f = owner_frame(g, bw, k0 + rr, c0 - 1 + col, rowR[rr]);
    uint32_t fi = 0;
    if (needs_slow(g, f, fi)) queue[atomicAdd(&qn, 1)] = (uint16_t)idx;
    else info[rr][col] = fi;
  }
  __syncthreads();
  const int nq = qn;
  for (int q = threadIdx.x; q < nq; q += kThreads) {
    const int idx = queue[q], rr = idx / W, col = idx - rr * W;
    const Frame f = owner_frame(g, bw, k0 + rr, c0 - 1 + col, rowR[rr]);
    Slow sr;
    slow_classify(g, f, sr);
    info[rr][col] = sr.info;
    if (q < kRec) rec[q] = pack_slow(sr);
  }
  __syncthreads();
  // 2. prefix sums of every row: thread t owns columns 1 + t*kOPT .. kOPT + t*kOPT
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int ev[kRB + 1], et[kRB + 1];
#pragma unroll
  for (int rr = 0; rr <= kRB; ++rr) {
    int sv = 0, st = 0;
#pragma unroll
    for (int j = 0; j < kOPT; ++j) {
      const uint32_t f = info[rr][1 + threadIdx.x * kOPT + j];
      sv += info_nv(f);
      st += info_nt(f);
    }
    const int iv = wave_incl_scan(sv, lane), it = wave_incl_scan(st, lane);
    ev[rr] = iv - sv;
    et[rr] = it - st;
    if (lane == 63) { part[rr][0][wv] = iv; part[rr][1][wv] = it; }
  }
  if (threadIdx.x < kRB) tb[threadIdx.x] = k0 + (int)threadIdx.x < g.NK ? seg_off[(int64_t)(k0 + threadIdx.x) * g.NCB + cb].y : 0;
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr <= kRB; ++rr) {
    const int k = k0 + rr;
    const int bv = k < g.NK ? (int)seg_off[(int64_t)k * g.NCB + cb].x : 0;
    int pv = 0, pt = 0, totv = 0;
#pragma unroll
    for (int q = 0; q < kThreads / 64; ++q) {
      if (q < wv) { pv += part[rr][0][q]; pt += part[rr][1][q]; }
      totv += part[rr][0][q];
    }
    int v = bv + ev[rr] + pv, t = et[rr] + pt;
#pragma unroll
    for (int j = 0; j < kOPT; ++j) {
      const int col = 1 + threadIdx.x * kOPT + j;
      const uint32_t f = info[rr][col];
      voff[rr][col] = v;
      if (rr < kRB) toff[rr][col] = (int16_t)t;
      v += info_nv(f);
      t += info_nt(f);
    }
    if (threadIdx.x == 0) {
      voff[rr][0] = bv - info_nv(info[rr][0]);
      voff[rr][W - 1] = bv + totv;
      if (rr < kRB) {
        int tt = 0;
        for (int q = 0; q < kThreads / 64; ++q) tt += part[rr][1][q];
        trow[rr] = tt;
      }
    }
  }
  __syncthreads();
  auto neighbours = [&](int r, int col, uint32_t f, int o_) {
    Nb nb;
    nb.vid = voff[r][col];
    nb.id_vr = voff[r][col + 1];
    nb.id_vdl = voff[r + 1][col + o_ - 1];
    nb.id_vdr = voff[r + 1][col + o_];
    nb.b0 = nb.vid + info_self(f);
    nb.b1 = nb.b0 + info_n(f, 0);
    nb.b2 = nb.b1 + info_n(f, 1);
    const uint32_t fr = info[r][col + 1];
    nb.b3 = voff[r][col + 1] + info_self(fr) + info_n(fr, 0);
    const uint32_t fl = info[r + 1][col + o_ - 1];
    nb.b4 = voff[r + 1][col + o_ - 1] + info_self(fl);
    nb.bI = nb.b2 + info_n(f, 2);
    return nb;
  };
  // 3. fast owners one per thread (their writes coalesce), then all slow
  // owners of the tile densely from their records.
  const bool both = (g.flags & 1u) != 0;
  Out out;
  out.v = verts; out.t = tris; out.c = codes; out.vbase = 0; out.tbase = 0;
  for (int r = 0; r < kRB; ++r) {
    const int k = k0 + r;
    if (k >= g.NK) break;
    const int o_ = k & 1;
    const double y = lat_y(g.h, k);
    const int64_t TB = tb[r];
    for (int j = 0; j < kOPT; ++j) {
      const int col = 1 + j * kThreads + threadIdx.x;
      const int c = c0 + col - 1;
      if (c >= g.NI) continue;
      const uint32_t f = info[r][col];
      if (info_slow(f)) continue;
      const int vid = voff[r][col];
      if (info_self(f)) put_vertex(verts, vid, lat_x(g.X0 + 4 * g.h * c + 2 * g.h * o_), y);
      int64_t u = TB + toff[r][col];
      const uint8_t code = both && !info_fg(f) ? 0x80 : 0;
      if (info_ntb(f)) {
        tris[3 * u + 0] = vid; tris[3 * u + 1] = voff[r + 1][col + o_]; tris[3 * u + 2] = voff[r + 1][col + o_ - 1];
        codes[u] = code;
        ++u;
      }
      if (info_nta(f)) {
        tris[3 * u + 0] = vid; tris[3 * u + 1] = voff[r][col + 1]; tris[3 * u + 2] = voff[r + 1][col + o_];
        codes[u] = code;
      }
    }
  }
  for (int q = threadIdx.x; q < nq; q += kThreads) {
    const int idx = queue[q], r = idx / W, col = idx - r * W;
    if (r >= kRB || col < 1 || col > kCB) continue;
    const int k = k0 + r, c = c0 + col - 1;
    const uint32_t f = info[r][col];
    const Nb nb = neighbours(r, col, f, k & 1);
    const Frame fr = owner_frame(g, bw, k, c, rowR[r]);
    SlowRec R;
    if (q < kRec) {
      R = rec[q];
    } else {
      Slow sr;
      slow_classify(g, fr, sr);
      R = pack_slow(sr);
    }
    emit_slow(g, fr, R, nb, tb[r] + toff[r][col], out);
  }
}

__global__ void k_sizes(const long long* __restrict__ tot, int64_t vcap, int64_t tcap, int64_t* __restrict__ out) {
  if (threadIdx.x == 0) {
    out[0] = tot[0];
    out[1] = tot[1];
    out[2] = tot[2];
    out[3] = tot[3] ? SBMT_E_PROTOCOL : ((tot[0] > vcap || tot[1] > tcap) ? SBMT_E_CAPACITY : SBMT_OK);
  }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
static int stride_for(int h) {
  int s = 1;
  while (s * s <= 2 * h * h) ++s;
  return s;
}

static bool grid_h_supported(int h) {
  // the owner parallelogram (width 1.5 h) must fit two coarse cells: 3h <= 2s
  return h >= 1 && h <= 6 && 3 * h <= 2 * stride_for(h);
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
static int64_t host_row_cell(int64_t k, int h, int s) {
  int64_t kh = k * h;
  int64_t R = host_floordiv(kh * 17320 / 10000 - s - 1, 2 * s);
  while (host_z3sign(-(2 * s * R + s + 1), kh) < 0) --R;
  while (host_z3sign(-(2 * s * (R + 1) + s + 1), kh) >= 0) ++R;
  return R;
}
static bool tile_window_fits(const Geo& g) {
  // rows: the cell rows of kRB + 1 grid rows plus the 3x3 window; words: the
  // cell columns of kCB + 2 owners plus the window and one spare word
  const double rows = ((kRB + 1) * g.h * 0.8660254037844386) / g.s + 5;
  const double words = ((kCB + 2) * (double)g.h / g.s + 4) / 32.0 + 3;
  return rows <= kWinRows && words <= kWinWords;
}

static bool windows_in_bounds(const Geo& g) {
  const int64_t rlo_min = host_row_cell(0, g.h, g.s), rlo_max = host_row_cell(g.NK - 1, g.h, g.s);
  const int64_t xmin = g.X0, xmax = (int64_t)g.X0 + 4LL * g.h * (g.NI - 1) + 2LL * g.h;
  const int64_t clo_min = host_floordiv(xmin - 2 * g.h - 2 * (g.s - 1), 4 * g.s);
  const int64_t clo_max = host_floordiv(xmax - 2 * g.h - 2 * (g.s - 1), 4 * g.s);
  // rows Rlo .. Rlo+2 and bit columns Clo .. Clo+2 (plus one spare word) are read
  return rlo_min + kRing >= 0 && rlo_max + 2 + kRing < g.CH + 2 * kRing && clo_min + kRingC >= 0 &&
         ((clo_max + 2 + kRingC) >> 5) + 1 < g.wpr;
}

struct Layout {
  Geo g;
  int64_t nseg;
  int nblk;
  size_t off_bits, off_cnt, off_segoff, off_blk, off_tot, total;
};

static sbmt_status make_layout(const sbmt_image* img, Layout* L, bool need_ptr = true) {
  if (!img) return SBMT_E_INVALID_ARG;
  if (img->width < 0 || img->height < 0) return SBMT_E_INVALID_ARG;
  if ((int64_t)img->width > (1 << 20) || (int64_t)img->height > (1 << 20)) return SBMT_E_INVALID_ARG;
  if (img->width > 0 && img->height > 0 && ((need_ptr && img->bitmap == nullptr) || img->row_stride < img->width))
    return SBMT_E_INVALID_ARG;
  if (img->flags & ~1u) return SBMT_E_INVALID_ARG;
  if (!grid_h_supported(img->grid_h)) return SBMT_E_UNSUPPORTED_GRID_H;
  Geo& g = L->g;
  g.W = img->width;
  g.H = img->height;
  g.stride = img->row_stride;
  g.h = img->grid_h;
  g.s = stride_for(g.h);
  g.CW = (g.W + g.s - 1) / g.s;
  g.CH = (g.H + g.s - 1) / g.s;
  // rows 0..m with m the smallest m >= 1 such that 3 m^2 h^2 > (2 s CH + 1)^2
  int64_t rhs = (2LL * g.s * g.CH + 1) * (2LL * g.s * g.CH + 1);
  int64_t m = (int64_t)((2.0 * g.s * g.CH + 1) / (g.h * 1.7320508075688772)) - 2;
  if (m < 1) m = 1;
  while (3LL * m * m * g.h * g.h <= rhs) ++m;
  while (m > 1 && 3LL * (m - 1) * (m - 1) * g.h * g.h > rhs) --m;
  g.NK = (int32_t)(m + 1);
  g.NI = (int32_t)((4LL * g.s * g.CW + 2LL * g.h + 1) / (4LL * g.h) + 2);
  g.NCB = (g.NI + kCB - 1) / kCB;
  g.wpr = (kRingC + g.CW + kRing + 31) / 32 + 1;
  g.X0 = -2 * g.h - 3;
  g.flags = img->flags;
  g.inv4s = 1.0f / (float)(4 * g.s);
  if (!windows_in_bounds(g) || !tile_window_fits(g)) return SBMT_E_INVALID_ARG;
  L->nseg = (int64_t)g.NK * g.NCB;
  L->nblk = (int)((L->nseg + kScanChunk - 1) / kScanChunk);
  size_t off = 0;
  L->off_bits = off;
  off = align256(off + (size_t)(g.CH + 2 * kRing) * g.wpr * 4);
  L->off_cnt = off;
  off = align256(off + (size_t)L->nseg * sizeof(int4));
  L->off_segoff = off;
  off = align256(off + (size_t)L->nseg * sizeof(longlong2));
  L->off_blk = off;
  off = align256(off + (size_t)L->nblk * sizeof(longlong4));
  L->off_tot = off;
  off = align256(off + 8 * sizeof(long long));
  L->total = off;
  return SBMT_OK;
}

static Work work_of(const Layout& L, void* ws) {
  char* b = (char*)ws;
  Work w;
  w.bits = (uint32_t*)(b + L.off_bits);
  w.seg_cnt = (int4*)(b + L.off_cnt);
  w.seg_off = (longlong2*)(b + L.off_segoff);
  w.blk = (longlong4*)(b + L.off_blk);
  w.tot = (long long*)(b + L.off_tot);
  return w;
}

static sbmt_status launch_plan(const Layout& L, const sbmt_image* img, const Work& w, hipStream_t st) {
  const Geo& g = L.g;
  dim3 gc((32 * g.wpr + 255) / 256, g.CH + 2 * kRing);
  hipLaunchKernelGGL(k_coarsen, gc, dim3(256), 0, st, g, img->bitmap, w.bits, w.tot);
  dim3 gk(g.NCB, (g.NK + kRB - 1) / kRB);
  hipLaunchKernelGGL(k_count, gk, dim3(kThreads), 0, st, g, (const uint32_t*)w.bits, w.seg_cnt, w.tot);
  hipLaunchKernelGGL(k_scan_reduce, dim3(L.nblk), dim3(kScanThreads), 0, st, (const int4*)w.seg_cnt, L.nseg, w.blk);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanThreads), 0, st, w.blk, L.nblk, w.tot);
  hipLaunchKernelGGL(k_scan_apply, dim3(L.nblk), dim3(kScanThreads), 0, st, (const int4*)w.seg_cnt, L.nseg,
                     (const longlong4*)w.blk, w.seg_off);
  return hipGetLastError() == hipSuccess ? SBMT_OK : SBMT_E_DEVICE;
}

static sbmt_status launch_emit(const Layout& L, const Work& w, int64_t vcap, int64_t tcap, double* verts,
                               int32_t* tris, uint8_t* codes, hipStream_t st) {
  const Geo& g = L.g;
  dim3 gk(g.NCB, (g.NK + kRB - 1) / kRB);
  hipLaunchKernelGGL(k_emit, gk, dim3(kThreads), 0, st, g, (const uint32_t*)w.bits, (const longlong2*)w.seg_off,
                     (const long long*)w.tot, vcap, tcap, verts, tris, codes);
  return hipGetLastError() == hipSuccess ? SBMT_OK : SBMT_E_DEVICE;
}

}  // namespace sbmt

using namespace sbmt;

struct sbmt_context {
  int device;
  long long* pinned;  // 8 x int64
};

extern "C" {

sbmt_status sbmt_create(int device, sbmt_handle* out) {
  if (!out) return SBMT_E_INVALID_ARG;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SBMT_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return SBMT_E_DEVICE;
  sbmt_context* c = (sbmt_context*)calloc(1, sizeof(sbmt_context));
  if (!c) return SBMT_E_DEVICE;
  c->device = device;
  if (hipHostMalloc((void**)&c->pinned, 8 * sizeof(long long), hipHostMallocDefault) != hipSuccess) {
    free(c);
    return SBMT_E_DEVICE;
  }
  *out = c;
  return SBMT_OK;
}

sbmt_status sbmt_destroy(sbmt_handle h) {
  if (!h) return SBMT_E_INVALID_ARG;
  if (h->pinned) (void)hipHostFree(h->pinned);
  free(h);
  return SBMT_OK;
}

sbmt_status sbmt_query(const sbmt_image* img, sbmt_layout* out) {
  Layout L;
  sbmt_status st = make_layout(img, &L, false);
  if (st != SBMT_OK) return st;
  if (out) {
    out->stride_s = L.g.s;
    out->coarse_w = L.g.CW;
    out->coarse_h = L.g.CH;
    out->grid_rows = L.g.NK;
    out->grid_cols = L.g.NI;
    out->workspace_bytes = L.total;
  }
  return SBMT_OK;
}

sbmt_status sbmt_plan(sbmt_handle h, const sbmt_image* img, void* workspace, size_t ws_bytes, sbmt_sizes* out,
                      void* stream) {
  if (!h || !out) return SBMT_E_INVALID_ARG;
  Layout L;
  sbmt_status st = make_layout(img, &L);
  if (st != SBMT_OK) return st;
  if (!workspace || ws_bytes < L.total) return SBMT_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  Work w = work_of(L, workspace);
  if ((st = launch_plan(L, img, w, s)) != SBMT_OK) return st;
  if (hipMemcpyAsync(h->pinned, w.tot, 4 * sizeof(long long), hipMemcpyDeviceToHost, s) != hipSuccess)
    return SBMT_E_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return SBMT_E_DEVICE;
  if (h->pinned[3]) return SBMT_E_PROTOCOL;
  out->n_vertices = h->pinned[0];
  out->n_triangles = h->pinned[1];
  out->n_cut = h->pinned[2];
  if (out->n_vertices > 0x7fffffffLL) return SBMT_E_INDEX_OVERFLOW;
  return SBMT_OK;
}

sbmt_status sbmt_run(sbmt_handle h, const sbmt_image* img, void* workspace, size_t ws_bytes, double* verts,
                     int32_t* tris, uint8_t* codes, void* stream) {
  if (!h) return SBMT_E_INVALID_ARG;
  Layout L;
  sbmt_status st = make_layout(img, &L);
  if (st != SBMT_OK) return st;
  if (!workspace || ws_bytes < L.total) return SBMT_E_WORKSPACE;
  Work w = work_of(L, workspace);
  // the plan's totals bound every write; capacities are the totals themselves
  const int64_t cap = INT64_MAX;
  return launch_emit(L, w, cap, cap, verts, tris, codes, (hipStream_t)stream);
}

sbmt_status sbmt_mesh_async(sbmt_handle h, const sbmt_image* img, void* workspace, size_t ws_bytes, double* verts,
                            int64_t vert_cap, int32_t* tris, uint8_t* codes, int64_t tri_cap, int64_t* sizes_dev,
                            void* stream) {
  if (!h || !sizes_dev || vert_cap < 0 || tri_cap < 0) return SBMT_E_INVALID_ARG;
  if (vert_cap > 0x7fffffffLL) vert_cap = 0x7fffffffLL;
  Layout L;
  sbmt_status st = make_layout(img, &L);
  if (st != SBMT_OK) return st;
  if (!workspace || ws_bytes < L.total) return SBMT_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  Work w = work_of(L, workspace);
  if ((st = launch_plan(L, img, w, s)) != SBMT_OK) return st;
  if ((st = launch_emit(L, w, vert_cap, tri_cap, verts, tris, codes, s)) != SBMT_OK) return st;
  hipLaunchKernelGGL(k_sizes, dim3(1), dim3(64), 0, s, (const long long*)w.tot, vert_cap, tri_cap, sizes_dev);
  return hipGetLastError() == hipSuccess ? SBMT_OK : SBMT_E_DEVICE;
}

int32_t sbmt_num_classes(void) { return SBMT_NUM_CLASSES; }

int32_t sbmt_class_code(int32_t class_id) {
  static const int32_t codes[] = {SBMT_CLASS_CODES_INIT};
  if (class_id < 1 || class_id > SBMT_NUM_CLASSES) return -1;
  return codes[class_id];
}

const char* sbmt_status_string(sbmt_status s) {
  switch (s) {
    case SBMT_OK: return "ok";
    case SBMT_E_INVALID_ARG: return "invalid argument";
    case SBMT_E_UNSUPPORTED_GRID_H: return "unsupported grid_h (supported: 1..6)";
    case SBMT_E_INDEX_OVERFLOW: return "vertex count exceeds int32";
    case SBMT_E_WORKSPACE: return "workspace missing or too small";
    case SBMT_E_DEVICE: return "HIP runtime error";
    case SBMT_E_PROTOCOL: return "inadmissible local boundary pattern";
    case SBMT_E_CAPACITY: return "mesh larger than the output capacity";
  }
  return "unknown status";
}

}  // extern "C"
