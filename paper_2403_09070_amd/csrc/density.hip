// Density map (Sec. IV-A, Eq. density-map-accum), its field-gather gradient and exact adjoint.
//
// Every instance is a cuboid [x -/+ w~/2] x [y -/+ h~/2] x [z -/+ d_z/4] clipped to the region,
// where w~ = max(w, sqrt2 w_b) is the local-smoothness stretch and omega = w h / (w~ h~) its
// weight; w, h follow the partition for cells (Eq. std-size-tech) and z linearly for macros
// (Eq. macro-size-tech).  rho_b = sum_i omega_i vol(D_i ∩ b) / vol(b).
//
// Work split (the adaptive scheme of Sec. IV-A, re-planned for LDS):
//   * the map is cut into T x T x Nz tiles, each owned by one workgroup that holds it in LDS;
//   * cells are bucketed by the tiles their footprint overlaps (a counting sort each call:
//     per-block tile histograms, a scan, a scatter of 32-byte entries), so a tile sweeps its
//     cells contiguously and accumulates with LDS atomics;
//   * large instances (movable macros, oversized cells) are swept bin-parallel by every tile
//     they overlap;
//   * each tile then writes its bins once (fixed-instance map + contributions), so the map is
//     written without global atomics, and reduces the per-die overflow on the way out.
// The field gather and the adjoint reuse the buckets: every (cell, tile) entry sums the bins of
// the tile it overlaps from an LDS copy of the maps, and a per-cell pass adds its <= 4 entries.
// Large instances take one workgroup each.  The constant map of fixed instances is built once.
//
// Planar extents are handled in coordinates local to the bin column holding the centre, so
// overlap lengths keep float32 precision relative to the bin size at any absolute coordinate.
#include "internal.h"

namespace p3d {
namespace {

struct Foot {
  int bx0, bx1, by0, by1, bz0, bz1;   // inclusive bin ranges of the clipped cuboid
  int cbx, cby;                       // bin column / row holding the centre (local origin)
  float lx0, lx1, ly0, ly1;           // clipped planar edges, local to (cbx*wb, cby*hb)
  float rx0, rx1, ry0, ry1;           // unclipped planar edges, local
  float z0, z1, rz0, rz1;             // clipped / unclipped z edges (absolute)
  float omega, w, h;
  float dw, dh;                       // macro size slope dw/dz, dh/dz inside the transition range
  float rx, ry, z, hw, hh;            // the local centre and stretched half extents it came from
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// A z within 2^-20 d_z of a bound of the movable range [d_z/4, 3 d_z/4] is on that bound (the
// clamp rounds the bounds to float32): -1 lower, +1 upper, 0 neither.
constexpr float kClampBand = 9.5367431640625e-07f;   // 2^-20
__device__ __forceinline__ int z_bound(const Geom& g, float z) {
  const float tol = kClampBand * g.dz;
  if (fabsf(z - 0.25f * g.dz) <= tol) return -1;
  if (fabsf(z - 0.75f * g.dz) <= tol) return 1;
  return 0;
}

// footprint from the centre in local coordinates (rx = x - cbx w_b) and the stretched half extents
__device__ __forceinline__ void foot_local(const Geom& g, Foot& f, int cbx, int cby, float rx, float ry, float z,
                                           float hw, float hh) {
  f.cbx = cbx;
  f.cby = cby;
  f.rx = rx; f.ry = ry; f.z = z; f.hw = hw; f.hh = hh;
  // the region's edges relative to the reference bin's origin
  const double ox = (double)cbx * g.wbd, oy = (double)cby * g.hbd;
  f.rx0 = rx - hw;
  f.rx1 = rx + hw;
  f.ry0 = ry - hh;
  f.ry1 = ry + hh;
  f.lx0 = fmaxf(f.rx0, (float)-ox);
  f.lx1 = fminf(f.rx1, (float)((double)g.dx - ox));
  f.ly0 = fmaxf(f.ry0, (float)-oy);
  f.ly1 = fminf(f.ry1, (float)((double)g.dy - oy));
  f.rz0 = z - 0.25f * g.dz;
  f.rz1 = z + 0.25f * g.dz;
  f.z0 = fmaxf(f.rz0, 0.f);
  f.z1 = fminf(f.rz1, g.dz);
  f.bx0 = clampi(cbx + (int)floorf(f.lx0 * g.inv_wb), 0, g.nx - 1);
  f.bx1 = clampi(cbx + (int)ceilf(f.lx1 * g.inv_wb) - 1, 0, g.nx - 1);
  f.by0 = clampi(cby + (int)floorf(f.ly0 * g.inv_hb), 0, g.ny - 1);
  f.by1 = clampi(cby + (int)ceilf(f.ly1 * g.inv_hb) - 1, 0, g.ny - 1);
  f.bz0 = clampi((int)floorf(f.z0 * g.inv_db), 0, g.nz - 1);
  f.bz1 = clampi((int)ceilf(f.z1 * g.inv_db) - 1, 0, g.nz - 1);
  f.bx1 = max(f.bx1, f.bx0);
  f.by1 = max(f.by1, f.by0);
  f.bz1 = max(f.bz1, f.bz0);
}

// an instance's inputs of the footprint, loaded together (so that callers can have the loads of
// several instances in flight before any arithmetic)
struct InstIn { float x, y, z, wbot, hbot, wtop, htop; uint8_t kind; };

__device__ __forceinline__ InstIn inst_in(const Geom& g, const float* __restrict__ xyz, const float* __restrict__ size,
                                          const uint8_t* __restrict__ kind, int i) {
  const int n = g.n;
  return {xyz[i], xyz[n + i], xyz[2 * n + i], size[i], size[n + i], size[2 * n + i], size[3 * n + i], kind[i]};
}

__device__ __forceinline__ Foot footprint_of(const Geom& g, const InstIn& in) {
  Foot f;
  const float x = in.x, y = in.y, z = in.z;
  const float wbot = in.wbot, hbot = in.hbot, wtop = in.wtop, htop = in.htop;
  const uint8_t kind = in.kind;
  float w, h;
  f.dw = 0.f;
  f.dh = 0.f;
  if (kind & PLACE3D_KIND_MACRO) {
    const float zl = 0.25f * g.dz, zh = 0.75f * g.dz;
    const float zc = fminf(fmaxf(z, zl), zh);
    const float t = 2.f * zc / g.dz;
    w = (t - 0.5f) * wtop + (1.5f - t) * wbot;
    h = (t - 0.5f) * htop + (1.5f - t) * hbot;
    // the size transition's slope, inside the movable range with its bounds (where the adjoint
    // takes the derivative into the range)
    if ((z > zl && z < zh) || z_bound(g, z) != 0) {
      f.dw = 2.f / g.dz * (wtop - wbot);
      f.dh = 2.f / g.dz * (htop - hbot);
    }
  } else {
    const bool top = z > g.half_dz;
    w = top ? wtop : wbot;
    h = top ? htop : hbot;
  }
  const float r2 = 1.41421356237309515f;
  const float wmin = r2 * g.wb, hmin = r2 * g.hb;
  f.w = w;
  f.h = h;
  f.omega = fminf(1.f, w / wmin) * fminf(1.f, h / hmin);
  const int cbx = clampi((int)floorf(x * g.inv_wb), 0, g.nx - 1);
  const int cby = clampi((int)floorf(y * g.inv_hb), 0, g.ny - 1);
  foot_local(g, f, cbx, cby, (float)((double)x - (double)cbx * g.wbd), (float)((double)y - (double)cby * g.hbd), z,
             0.5f * fmaxf(w, wmin),
             0.5f * fmaxf(h, hmin));
  return f;
}

__device__ __forceinline__ Foot footprint(const Geom& g, const float* __restrict__ xyz,
                                          const float* __restrict__ size, uint8_t kind, int i) {
  const int n = g.n;
  return footprint_of(g, {xyz[i], xyz[n + i], xyz[2 * n + i], size[i], size[n + i], size[2 * n + i], size[3 * n + i],
                          kind});
}

// bucket entry: (cbx | cby << 13 | q << 26 | filler << 28, rx, ry, z), (hw, hh, omega, cell index
// as int bits); q is the entry's ordinal among its cell's (at most four) tiles
__device__ __forceinline__ unsigned entry_word(int cbx, int cby, int q, bool filler) {
  return (unsigned)cbx | ((unsigned)cby << 13) | ((unsigned)q << 26) | ((filler ? 1u : 0u) << 28);
}
__device__ __forceinline__ int entry_q(float4 a) { return (int)((__float_as_uint(a.x) >> 26) & 3u); }
__device__ __forceinline__ bool entry_filler(float4 a) { return ((__float_as_uint(a.x) >> 28) & 1u) != 0u; }
__device__ __forceinline__ int entry_cell(float4 b) { return __float_as_int(b.w); }

__device__ __forceinline__ Foot foot_entry(const Geom& g, float4 a, float4 b) {
  Foot f;
  const unsigned packed = __float_as_uint(a.x);
  foot_local(g, f, (int)(packed & 0x1FFFu), (int)((packed >> 13) & 0x1FFFu), a.y, a.z, a.w, b.x, b.y);
  f.omega = b.z;
  f.w = f.h = 0.f;
  f.dw = f.dh = 0.f;
  return f;
}

// Large-instance record, computed once per call: [0] (cbx | cby << 16, rx, ry, z), [1] (hw, hh,
// omega, w), [2] (h, dw, dh, -), [3] (bx0, bx1, by0, by1) as integers.
__device__ __forceinline__ Foot foot_record(const Geom& g, const float4* __restrict__ rec, int j) {
  const float4 a = rec[4 * (size_t)j], b = rec[4 * (size_t)j + 1], c = rec[4 * (size_t)j + 2];
  Foot f;
  const unsigned packed = __float_as_uint(a.x);
  foot_local(g, f, (int)(packed & 0xFFFFu), (int)(packed >> 16), a.y, a.z, a.w, b.x, b.y);
  f.omega = b.z;
  f.w = b.w;
  f.h = c.x;
  f.dw = c.y;
  f.dh = c.z;
  return f;
}

// overlap lengths of the clipped cuboid with bin b along each axis, from the edges taken relative
// to the bin (a bin the cuboid covers gets exactly the bin size, whatever its distance from the
// footprint's reference bin)
__device__ __forceinline__ float len_x(const Geom& g, const Foot& f, int b) {
  const float lo = (float)(b - f.cbx) * g.wb;
  return fmaxf(0.f, fminf(f.lx1 - lo, g.wb) - fmaxf(f.lx0 - lo, 0.f));
}
__device__ __forceinline__ float len_y(const Geom& g, const Foot& f, int b) {
  const float lo = (float)(b - f.cby) * g.hb;
  return fmaxf(0.f, fminf(f.ly1 - lo, g.hb) - fmaxf(f.ly0 - lo, 0.f));
}
__device__ __forceinline__ float len_z(const Geom& g, const Foot& f, int b) {
  const float lo = (float)b * g.db;
  return fmaxf(0.f, fminf(f.z1 - lo, g.db) - fmaxf(f.z0 - lo, 0.f));
}

// One-sided derivatives of the overlap lengths (the adjoint).  The map is piecewise linear in each
// coordinate, with kinks where an edge meets a bin face or a face of the region.  Per axis the
// derivative is taken from above (the coordinate growing), or from below when the unclipped
// upper edge lies on or beyond the region's upper face; at the bounds of the movable range that
// is the direction the clamp allows (into the range).  Moving that way an edge at e changes the
// overlap of one bin: floor(e/s) from above if 0 <= e < L, ceil(e/s) - 1 from below if
// 0 < e <= L, none otherwise (the region holds the edge).
__device__ __forceinline__ int edge_bin(float e, float lo, float hi, float inv_step, bool down, int q0, int n) {
  if (down ? !(e > lo && e <= hi) : !(e >= lo && e < hi)) return -1;
  const float q = e * inv_step;
  return clampi(q0 + (down ? (int)ceilf(q) - 1 : (int)floorf(q)), 0, n - 1);
}

struct EdgeBins {
  int xl, xh, yl, yh, zl, zh;   // bins whose overlap each edge changes, -1 for none
  bool down_x, down_y, down_z;  // derivative from below along that axis
};

// the region's faces in the footprint's local planar coordinates (as foot_local clips them)
__device__ __forceinline__ float2 local_faces(float die, int cb, double step) {
  const double o = (double)cb * step;
  return make_float2((float)-o, (float)((double)die - o));
}

// A planar edge within 2^-20 of the region's extent of a region face is on that face for the
// one-sided decisions: the clamp holds an instance against a die side at a float32 position and
// the local coordinate rounds again, which leaves the edge a rounding away from the face on
// either side.  (The overlap lengths keep the edges as they are.)
__device__ __forceinline__ float snap_face(float e, float2 face, float band) {
  if (fabsf(e - face.x) <= band) return face.x;
  if (fabsf(e - face.y) <= band) return face.y;
  return e;
}

__device__ __forceinline__ EdgeBins edge_bins(const Geom& g, const Foot& f) {
  EdgeBins e;
  const float2 fx = local_faces(g.dx, f.cbx, g.wbd), fy = local_faces(g.dy, f.cby, g.hbd);
  const float bx = kClampBand * g.dx, by = kClampBand * g.dy;
  const float x0 = snap_face(f.rx0, fx, bx), x1 = snap_face(f.rx1, fx, bx);
  const float y0 = snap_face(f.ry0, fy, by), y1 = snap_face(f.ry1, fy, by);
  e.down_x = x1 >= fx.y;
  e.down_y = y1 >= fy.y;
  e.xl = edge_bin(x0, fx.x, fx.y, g.inv_wb, e.down_x, f.cbx, g.nx);
  e.xh = edge_bin(x1, fx.x, fx.y, g.inv_wb, e.down_x, f.cbx, g.nx);
  e.yl = edge_bin(y0, fy.x, fy.y, g.inv_hb, e.down_y, f.cby, g.ny);
  e.yh = edge_bin(y1, fy.x, fy.y, g.inv_hb, e.down_y, f.cby, g.ny);
  const int zb = z_bound(g, f.z);
  if (zb < 0) {            // on the lower bound: edges on the floor and the mid-plane, moving up
    e.down_z = false; e.zl = 0; e.zh = g.nz / 2;
  } else if (zb > 0) {     // on the upper bound: edges on the mid-plane and the ceiling, moving down
    e.down_z = true; e.zl = g.nz / 2 - 1; e.zh = g.nz - 1;
  } else {
    e.down_z = f.rz1 >= g.dz;
    e.zl = edge_bin(f.rz0, 0.f, g.dz, g.inv_db, e.down_z, 0, g.nz);
    e.zh = edge_bin(f.rz1, 0.f, g.dz, g.inv_db, e.down_z, 0, g.nz);
  }
  return e;
}

__device__ __forceinline__ size_t bin_index(const Geom& g, int bz, int by, int bx) {
  return ((size_t)bz * g.ny + by) * g.nx + bx;
}

template <int NQ>
__device__ __forceinline__ void block_partials(float (&v)[NQ], double* __restrict__ part, int stride, int slot0,
                                               int idx) {
  __shared__ double sh[NQ][1024 / kWave];
  __syncthreads();
  for (int q = 0; q < NQ; ++q) {
    double x = v[q];
    for (int m = kWave / 2; m > 0; m >>= 1) x += __shfl_xor(x, m);
    if ((threadIdx.x & (kWave - 1)) == 0) sh[q][threadIdx.x / kWave] = x;
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    double x = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) x += sh[threadIdx.x][w];
    part[(size_t)(slot0 + threadIdx.x) * stride + idx] = x;
  }
}

template <int NT>
__device__ __forceinline__ float block_sum(float v, float* sh) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  float r = 0.f;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / kWave; ++w) r += sh[w];
  return r;   // valid in thread 0
}

// ------------------------------------------------------------------ bucketing

// threads of a bucketing workgroup: its 2048 instances take two rounds, and 16 wavefronts per
// workgroup keep enough loads in flight at a few workgroups per compute unit
constexpr int kBucketThreads = 1024;
constexpr int kCellsPerThread = 2;      // cells a bucketing thread loads together per round

// number of entries (tiles) of a bucketed cell from its packed tile range, 0 for -1 (not bucketed)
__host__ __device__ inline int entry_count(int packed) {
  return packed < 0 ? 0 : (1 + ((packed >> 24) & 1)) * (1 + ((packed >> 25) & 1));
}

// tiles overlapped by a bucketed cell (at most 2 x 2 for the cells this path takes)
__device__ __forceinline__ void cell_tiles(const Foot& f, const TileGeom& t, int& tx0, int& tx1, int& ty0, int& ty1) {
  tx0 = f.bx0 >> t.lgT; tx1 = f.bx1 >> t.lgT;
  ty0 = f.by0 >> t.lgT; ty1 = f.by1 >> t.lgT;
}

// packed tile range of a bucketed cell: tx0 | ty0 << 12 | (tx1 - tx0) << 24 | (ty1 - ty0) << 25
__device__ __forceinline__ int pack_tiles(int tx0, int tx1, int ty0, int ty1) {
  return tx0 | (ty0 << 12) | ((tx1 - tx0) << 24) | ((ty1 - ty0) << 25);
}

// Counts entries per (tile, block) and records each cell's packed tile range in cell_entry[0][i],
// so that the scatter pass places a cell in exactly the tiles it was counted in.  Every
// instance's position is also written packed (x, y, z, 0) for the wirelength sweep.
__device__ __forceinline__ void large_record(const Geom& g, const float* __restrict__ xyz,
                                             const float* __restrict__ size, const uint8_t* __restrict__ kind,
                                             const int32_t* __restrict__ large, int j, float4* __restrict__ rec);

// Blocks [0, nblk) count; the blocks after them write the large-instance records.
__global__ __launch_bounds__(kBucketThreads) void k_bucket_count(Geom g, TileGeom t, const float* __restrict__ xyz,
                                                      const float* __restrict__ size, const uint8_t* __restrict__ kind,
                                                      const uint8_t* __restrict__ cls, int32_t* __restrict__ counts,
                                                      int32_t* __restrict__ tiles_of, float4* __restrict__ xyzp,
                                                      const int32_t* __restrict__ large, int nlarge,
                                                      float4* __restrict__ lrec) {
  extern __shared__ int hist[];
  if ((int)blockIdx.x >= t.nblk) {
    const int j = ((int)blockIdx.x - t.nblk) * blockDim.x + threadIdx.x;
    if (j < nlarge) large_record(g, xyz, size, kind, large, j, lrec);
    return;
  }
  for (int k = threadIdx.x; k < t.ntiles; k += blockDim.x) hist[k] = 0;
  __syncthreads();
  const int base = blockIdx.x * t.cpb;
  // kCellsPerThread cells per thread and round, every load of the round issued before any use
  for (int c0 = threadIdx.x; c0 < t.cpb; c0 += kCellsPerThread * blockDim.x) {
    InstIn in[kCellsPerThread];
    uint8_t cl[kCellsPerThread];
#pragma unroll
    for (int u = 0; u < kCellsPerThread; ++u) {
      const int c = c0 + u * (int)blockDim.x, i = min(base + c, g.n - 1);   // clamped: loads stay in bounds
      in[u] = inst_in(g, xyz, size, kind, i);
      cl[u] = cls[i];
    }
#pragma unroll
    for (int u = 0; u < kCellsPerThread; ++u) {
      const int c = c0 + u * (int)blockDim.x, i = base + c;
      if (c >= t.cpb || i >= g.n) continue;
      xyzp[i] = make_float4(in[u].x, in[u].y, in[u].z, 0.f);
      if (cl[u] != kClsCell) { tiles_of[i] = -1; continue; }
      const Foot f = footprint_of(g, in[u]);
      int tx0, tx1, ty0, ty1;
      cell_tiles(f, t, tx0, tx1, ty0, ty1);
      tx1 = min(tx1, tx0 + 1);           // bucketed cells span at most two tiles per axis
      ty1 = min(ty1, ty0 + 1);
      tiles_of[i] = pack_tiles(tx0, tx1, ty0, ty1);
      for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) atomicAdd(&hist[ty * t.ntx + tx], 1);
    }
  }
  __syncthreads();
  // block-major: this block's counts are one contiguous row
  for (int k = threadIdx.x; k < t.ntiles; k += blockDim.x) counts[(size_t)blockIdx.x * t.ntiles + k] = hist[k];
}

// Exclusive scan of every tile's counts over the bucket blocks (in place, counts block-major
// [nblk][ntiles]); the tile totals to totals.  A workgroup takes 64 adjacent tiles: lane l of
// wavefront q scans tile 64 g + l over the q-th of kScanParts ranges of blocks, so that a
// wavefront reads 64 adjacent counts (256 bytes) of one block row at a time; each range is then
// offset by the sums of the ranges before it.  A range of up to kScanHeld rows is loaded once into
// registers (all its loads in flight together) and written back from them; a longer range is
// read twice, kScanChunk rows at a time.
constexpr int kScanTiles = 64;
constexpr int kScanParts = 16;
constexpr int kScanHeld = 48;
constexpr int kScanChunk = 16;
__global__ __launch_bounds__(kScanTiles * kScanParts) void k_bucket_scan_cols(int nblk, int ntiles,
                                                                             int32_t* __restrict__ counts,
                                                                             int32_t* __restrict__ totals) {
  __shared__ int part[kScanParts][kScanTiles];
  const int l = threadIdx.x & (kScanTiles - 1), q = threadIdx.x / kScanTiles;
  const int tile = blockIdx.x * kScanTiles + l;
  const int per = (nblk + kScanParts - 1) / kScanParts;
  const int b0 = min(q * per, nblk), b1 = min(b0 + per, nblk);
  const bool held = per <= kScanHeld;
  int v[kScanHeld];
  int s = 0;
  if (tile < ntiles) {
    if (held) {
#pragma unroll
      for (int j = 0; j < kScanHeld; ++j) v[j] = b0 + j < b1 ? counts[(size_t)(b0 + j) * ntiles + tile] : 0;
#pragma unroll
      for (int j = 0; j < kScanHeld; ++j) s += v[j];
    } else {                    // longer ranges: kScanChunk rows at a time, each chunk's loads together
      for (int c0 = b0; c0 < b1; c0 += kScanChunk) {
#pragma unroll
        for (int j = 0; j < kScanChunk; ++j) v[j] = c0 + j < b1 ? counts[(size_t)(c0 + j) * ntiles + tile] : 0;
#pragma unroll
        for (int j = 0; j < kScanChunk; ++j) s += v[j];
      }
    }
  }
  part[q][l] = s;
  __syncthreads();
  int run = 0;
  for (int u = 0; u < q; ++u) run += part[u][l];
  if (tile < ntiles) {
    if (held) {
#pragma unroll
      for (int j = 0; j < kScanHeld; ++j)
        if (b0 + j < b1) {
          counts[(size_t)(b0 + j) * ntiles + tile] = run;
          run += v[j];
        }
    } else {
      for (int c0 = b0; c0 < b1; c0 += kScanChunk) {
#pragma unroll
        for (int j = 0; j < kScanChunk; ++j) v[j] = c0 + j < b1 ? counts[(size_t)(c0 + j) * ntiles + tile] : 0;
#pragma unroll
        for (int j = 0; j < kScanChunk; ++j)
          if (c0 + j < b1) {
            counts[(size_t)(c0 + j) * ntiles + tile] = run;
            run += v[j];
          }
      }
    }
    if (q == kScanParts - 1) totals[tile] = run;
  }
}

// Chunk plan of the current buckets, made by workgroup 0 of the scatter pass (every thread
// takes the tiles [k0, k1) of the tile scan): a tile of more than kChunkEntries entries is heavy;
// its chunks after the first are numbered after the tiles, in tile order, and it takes the next
// accumulator slot.  Layout of plan: [0] extra chunks, [1] heavy tiles, [2 + k] slot of tile k
// (-1 for a tile of one chunk), [2 + ntiles + e] tile of extra chunk e, [2 + ntiles + max_extra
// + e] its index within the tile.
__device__ void chunk_plan(const int32_t* __restrict__ totals, int k0, int k1, int ntiles, int max_extra,
                           int32_t* __restrict__ plan) {
  __shared__ int wx[kBucketThreads / kWave], wh[kBucketThreads / kWave];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  int ox = 0, oh = 0;
  for (int k = k0; k < k1; ++k) {
    const int v = totals[k];
    if (v > kChunkEntries) { ox += (v - 1) / kChunkEntries; ++oh; }
  }
  int ix = ox, ih = oh;                 // inclusive scans within the wavefront
  for (int o = 1; o < kWave; o <<= 1) {
    const int ux = __shfl_up(ix, o), uh = __shfl_up(ih, o);
    if (lane >= o) { ix += ux; ih += uh; }
  }
  if (lane == kWave - 1) { wx[wave] = ix; wh[wave] = ih; }
  __syncthreads();
  int ex = ix - ox, eh = ih - oh;       // exclusive prefixes of this thread's tiles
  for (int w = 0; w < wave; ++w) { ex += wx[w]; eh += wh[w]; }
  int32_t* extra = plan + 2 + ntiles;
  for (int k = k0; k < k1; ++k) {
    const int v = totals[k];
    if (v > kChunkEntries) {
      const int nx = (v - 1) / kChunkEntries;
      for (int j = 0; j < nx; ++j) {
        extra[ex + j] = k;
        extra[max_extra + ex + j] = j + 1;
      }
      ex += nx;
      plan[2 + k] = eh++;
    } else {
      plan[2 + k] = -1;
    }
  }
  // the last thread's tile range ends at the last tile: its running counts are the totals
  if (threadIdx.x == blockDim.x - 1) { plan[0] = ex; plan[1] = eh; }
}

__global__ __launch_bounds__(kBucketThreads) void k_bucket_scatter(Geom g, TileGeom t, const float* __restrict__ xyz,
                                                        const float* __restrict__ size, const uint8_t* __restrict__ kind,
                                                        const uint8_t* __restrict__ cls, const int32_t* __restrict__ counts,
                                                        const int32_t* __restrict__ totals,
                                                        int32_t* __restrict__ tile_start,
                                                        float4* __restrict__ entries, int32_t* __restrict__ cell_entry,
                                                        int max_extra, int32_t* __restrict__ plan) {
  // every workgroup scans the tile totals itself (exclusive prefix = tile_start) and workgroup 0
  // stores the result for the later passes; the cursor of tile k starts at tile_start[k] plus
  // this workgroup's offset within the tile
  extern __shared__ int cursor[];
  __shared__ int wsum[kBucketThreads / kWave];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int per = (t.ntiles + blockDim.x - 1) / blockDim.x;
  const int k0 = min((int)threadIdx.x * per, t.ntiles), k1 = min(k0 + per, t.ntiles);
  int own = 0;
  for (int k = k0; k < k1; ++k) { const int v = totals[k]; cursor[k] = v; own += v; }
  int incl = own;
  for (int o = 1; o < kWave; o <<= 1) {
    const int u = __shfl_up(incl, o);
    if (lane >= o) incl += u;
  }
  if (lane == kWave - 1) wsum[wave] = incl;
  __syncthreads();
  if (wave == 0) {
    const int nw = blockDim.x / kWave;
    const int wv = lane < nw ? wsum[lane] : 0;
    int wi = wv;
    for (int o = 1; o < kWave; o <<= 1) {
      const int u = __shfl_up(wi, o);
      if (lane >= o) wi += u;
    }
    if (lane < nw) wsum[lane] = wi - wv;
  }
  __syncthreads();
  int run = wsum[wave] + incl - own;
  for (int k = k0; k < k1; ++k) {
    const int v = cursor[k];
    if (blockIdx.x == 0) tile_start[k] = run;
    cursor[k] = run + counts[(size_t)blockIdx.x * t.ntiles + k];
    run += v;
  }
  if (blockIdx.x == 0 && k0 < k1 && k1 == t.ntiles) tile_start[t.ntiles] = run;
  __syncthreads();
  if (blockIdx.x == 0) chunk_plan(totals, k0, k1, t.ntiles, max_extra, plan);
  const int n = g.n;
  const int base = blockIdx.x * t.cpb;
  for (int c0 = threadIdx.x; c0 < t.cpb; c0 += kCellsPerThread * blockDim.x) {
    InstIn in[kCellsPerThread];
    int pk[kCellsPerThread];
#pragma unroll
    for (int u = 0; u < kCellsPerThread; ++u) {
      const int c = c0 + u * (int)blockDim.x, i = min(base + c, n - 1);     // clamped: loads stay in bounds
      in[u] = inst_in(g, xyz, size, kind, i);
      pk[u] = (c < t.cpb && base + c < n) ? cell_entry[i] : -1;         // tile range from the count pass
    }
#pragma unroll
    for (int u = 0; u < kCellsPerThread; ++u) {
      const int packed = pk[u];
      if (packed < 0) continue;
      const int i = base + c0 + u * (int)blockDim.x;
      const Foot f = footprint_of(g, in[u]);
      const int tx0 = packed & 0xFFF, ty0 = (packed >> 12) & 0xFFF;
      const int tx1 = tx0 + ((packed >> 24) & 1), ty1 = ty0 + ((packed >> 25) & 1);
      const bool filler = (in[u].kind & PLACE3D_KIND_FILLER) != 0;
      const float4 eb = make_float4(f.hw, f.hh, f.omega, __int_as_float(i));
      int q = 0;
      for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
          const int slot = atomicAdd(&cursor[ty * t.ntx + tx], 1);
          entries[2 * (size_t)slot] = make_float4(__uint_as_float(entry_word(f.cbx, f.cby, q++, filler)), f.rx, f.ry, f.z);
          entries[2 * (size_t)slot + 1] = eb;
        }
    }
  }
}

__device__ __forceinline__ void large_record(const Geom& g, const float* __restrict__ xyz,
                                             const float* __restrict__ size, const uint8_t* __restrict__ kind,
                                             const int32_t* __restrict__ large, int j, float4* __restrict__ rec) {
  const int i = large[j];
  const Foot f = footprint(g, xyz, size, kind[i], i);
  rec[4 * (size_t)j] = make_float4(__uint_as_float((unsigned)f.cbx | ((unsigned)f.cby << 16)), f.rx, f.ry, f.z);
  rec[4 * (size_t)j + 1] = make_float4(f.hw, f.hh, f.omega, f.w);
  rec[4 * (size_t)j + 2] = make_float4(f.h, f.dw, f.dh, 0.f);
  rec[4 * (size_t)j + 3] = make_float4(__int_as_float(f.bx0), __int_as_float(f.bx1), __int_as_float(f.by0),
                                       __int_as_float(f.by1));
}

// Compacts, in list order, the large instances whose records overlap the tile: chunks of the
// block size are tested in parallel; `hits` receives record indices, returns the count of the
// current chunk.  All threads must call it with the same chunk.
__device__ __forceinline__ int large_hits(const float4* __restrict__ rec, int nlarge, int chunk, int x0, int x1, int y0,
                                          int y1, int* hits, int* wave_cnt) {
  const int j = chunk + threadIdx.x;
  bool hit = false;
  if (j < nlarge) {
    const float4 b = rec[4 * (size_t)j + 3];
    hit = !(__float_as_int(b.y) < x0 || __float_as_int(b.x) > x1 || __float_as_int(b.w) < y0 || __float_as_int(b.z) > y1);
  }
  const unsigned long long mask = __ballot(hit);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) wave_cnt[wid] = __popcll(mask);
  __syncthreads();
  int base = 0, total = 0;
  for (int w = 0; w < (int)(blockDim.x / kWave); ++w) { if (w < wid) base += wave_cnt[w]; total += wave_cnt[w]; }
  if (hit) hits[base + __popcll(mask & ((1ull << lane) - 1ull))] = j;
  __syncthreads();
  return total;
}

// ------------------------------------------------------------------ tiled density map

struct TileBox { int x0, y0, wx, wy; };

// threads of a tile workgroup (density map, field gather, adjoint): eight wavefronts, so that the
// gathers of a tile's entries have more loads in flight than the LDS-bound occupancy allows
constexpr int kTileThreads = 512;

__device__ __forceinline__ TileBox tile_box(const Geom& g, const TileGeom& t, int tile) {
  TileBox b;
  const int tx = tile % t.ntx, ty = tile / t.ntx;
  b.x0 = tx * t.T;
  b.y0 = ty * t.T;
  b.wx = min(t.T, g.nx - b.x0);
  b.wy = min(t.T, g.ny - b.y0);
  return b;
}

__device__ __forceinline__ int lds_index(const TileGeom& t, int bz, int ly, int lx) { return (bz * t.T + ly) * t.T + lx; }

// The tile accumulates in 64-bit fixed point (2^-31 units): integer LDS atomics run at full rate
// where float LDS atomics serialise across lanes, and integer sums do not depend on the order in
// which cells arrive, so the map is reproducible bit for bit.  One instance adds at most one
// bin volume to a bin (a fraction <= 1), which converts through 32 bits; the fixed-instance map
// (any value) takes the full 64-bit conversion.
constexpr float kFix = 2147483648.f;          // 2^31
constexpr double kUnfix = 1.0 / 2147483648.0;

__device__ __forceinline__ unsigned long long to_fix(float v) { return __float2ull_rn(v * kFix); }
__device__ __forceinline__ unsigned long long to_fix_unit(float v) {   // 0 <= v < 2
  return (unsigned long long)__float2uint_rn(v * kFix);
}

// x bins of a bucketed entry whose overlap lengths are held in registers
constexpr int kSpanX = 4;

// A thread's entries of one tile (first, first + step, ... below last), read D entries ahead: the
// loads of the next D entries are in flight while the current one is processed, and the first D
// entries' are issued before the tile's maps are staged, so that their latency overlaps work
// already in hand (a thread holds ~2.5 entries of a tile at the 1.2M-cell workload, so D = 2
// issues nearly all of them at once).  D costs 8 VGPRs per entry held.
template <int D>
struct EntryStream {
  const float4* __restrict__ entries;
  int e, last, step;
  float4 na[D], nb[D];
  __device__ __forceinline__ void fetch(int k, int at) {
    if (at < last) { na[k] = entries[2 * (size_t)at]; nb[k] = entries[2 * (size_t)at + 1]; }
  }
  __device__ __forceinline__ EntryStream(const float4* __restrict__ en, int first, int last_, int step_)
      : entries(en), e(first), last(last_), step(step_) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      na[k] = nb[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      fetch(k, e + k * step);
    }
  }
  __device__ __forceinline__ bool next(float4& a, float4& b) {
    if (e >= last) return false;
    a = na[0];
    b = nb[0];
#pragma unroll
    for (int k = 0; k + 1 < D; ++k) { na[k] = na[k + 1]; nb[k] = nb[k + 1]; }
    e += step;
    fetch(D - 1, e + (D - 1) * step);
    return true;
  }
};

// The chunk plan of the current buckets, as the tile kernels take it.  Chunk q < ntiles is the
// first chunk of tile q; chunk ntiles + e is extra chunk e (its tile and its index >= 1 within the
// tile in the plan).  A launch of ntiles + max_extra workgroups gives workgroup q chunk q
// (straight-line code: a loop over chunks would hold more registers and cost the common
// one-chunk tiles occupancy).
struct Chunks {
  const int32_t* __restrict__ tile_start;   // [ntiles + 1] entry ranges of the tiles
  int32_t* plan;                            // the context's chunk plan (written by chunk_plan;
                                            // its layout is in the accessors below)
  int ntiles, max_extra;
  __device__ __forceinline__ int n_extra() const { return plan[0]; }
  __device__ __forceinline__ int slot(int tile) const { return plan[2 + tile]; }
  __device__ __forceinline__ int extra_tile(int e) const { return plan[2 + ntiles + e]; }
  __device__ __forceinline__ int extra_index(int e) const { return plan[2 + ntiles + max_extra + e]; }
  __device__ __forceinline__ int32_t* done(int slot) const { return plan + 2 + ntiles + 2 * max_extra + slot; }
};

struct ChunkRef {
  int tile, first, last;    // entries [first, last) of the chunk
  int nchunks;              // chunks of its tile
  bool chunk0;
};

// (q is the same in every lane: the values are moved to scalar registers, which the compiler
// cannot assume for loads through the struct's pointers)
__device__ __forceinline__ ChunkRef chunk_ref(const Chunks& ch, const TileGeom& t, int q) {
  ChunkRef ck;
  int kc = 0;
  if (q < t.ntiles) {
    ck.tile = q;
  } else {
    ck.tile = __builtin_amdgcn_readfirstlane(ch.extra_tile(q - t.ntiles));
    kc = __builtin_amdgcn_readfirstlane(ch.extra_index(q - t.ntiles));
  }
  const int ts = __builtin_amdgcn_readfirstlane(ch.tile_start[ck.tile]);
  const int te = __builtin_amdgcn_readfirstlane(ch.tile_start[ck.tile + 1]);
  ck.nchunks = te - ts > kChunkEntries ? (te - ts - 1) / kChunkEntries + 1 : 1;
  ck.chunk0 = kc == 0;
  ck.first = ts + kc * kChunkEntries;
  ck.last = min(ck.first + kChunkEntries, te);
  return ck;
}

// the finished tile into rho and its overflow partials; fix(k, real, filler) gives bin k's sums
template <class Fix>
__device__ __forceinline__ void write_tile(const Geom& g, const TileGeom& t, const TileBox& tb, int tile, float target,
                                           int fillers, Fix fix, float* __restrict__ rho, double* __restrict__ part,
                                           int stride) {
  const int tsz = t.T * t.T * g.nz;
  float ex[2] = {0.f, 0.f};
  const int half = g.nz / 2;
  // rows and tile width multiples of 4 bins: write 4 bins per store (aligned, as in the gather)
  const bool vec = (g.nx & 3) == 0 && (tb.wx & 3) == 0 && (reinterpret_cast<uintptr_t>(rho) & 15) == 0;
  for (int k = vec ? 4 * (int)threadIdx.x : tsz; k < tsz; k += 4 * (int)blockDim.x) {
    const int lx = k & (t.T - 1), ly = (k >> t.lgT) & (t.T - 1), bz = k >> (2 * t.lgT);
    if (lx < tb.wx && ly < tb.wy) {
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        unsigned long long real, fil;
        fix(k + j, real, fil);
        v[j] = (float)((double)(real + fil) * kUnfix);
        const float vr = fillers ? (float)((double)real * kUnfix) : v[j];
        ex[bz < half ? 0 : 1] += fmaxf(vr - target, 0.f) * g.vol_bin;
      }
      *reinterpret_cast<float4*>(rho + bin_index(g, bz, tb.y0 + ly, tb.x0 + lx)) = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
  for (int k = vec ? tsz : (int)threadIdx.x; k < tsz; k += blockDim.x) {
    const int lx = k & (t.T - 1), ly = (k >> t.lgT) & (t.T - 1), bz = k >> (2 * t.lgT);
    if (lx < tb.wx && ly < tb.wy) {
      unsigned long long real, fil;
      fix(k, real, fil);
      const float v = (float)((double)(real + fil) * kUnfix);
      const float vr = fillers ? (float)((double)real * kUnfix) : v;
      rho[bin_index(g, bz, tb.y0 + ly, tb.x0 + lx)] = v;
      ex[bz < half ? 0 : 1] += fmaxf(vr - target, 0.f) * g.vol_bin;
    }
  }
  block_partials<2>(ex, part, stride, R_EXCESS_BOT, tile);
}

// A chunk accumulates in LDS: its tile's fixed map and large-instance sweep with the first chunk,
// then its entries.  A tile of one chunk is written from LDS.  The chunks of a heavy tile add
// their LDS sums into the tile's accumulator slot (64-bit integer atomics, so the sum does not
// depend on their order) and count themselves done; the last one reads the slot back, clearing
// it, and writes the tile.
// (eight wavefronts per SIMD: the scalar registers its heavy-tile path needs would otherwise cost
// one; the excess goes to vector-register lanes)
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_density_tiles(Geom g, TileGeom t, const float4* __restrict__ entries,
                                                       Chunks ch, unsigned long long* __restrict__ heavy_acc,
                                                       const float* __restrict__ fixed_map,
                                                       const float4* __restrict__ lrec, int nlarge, float target,
                                                       int fillers, float* __restrict__ rho,
                                                       double* __restrict__ part, int stride) {
  extern __shared__ unsigned long long S64[];
  __shared__ int hits[kTileThreads];
  __shared__ int wave_cnt[kTileThreads / kWave];
  __shared__ int last_chunk;
  const int tsz = t.T * t.T * g.nz;
  const float inv_vol = 1.f / g.vol_bin;
  // with fillers, their share accumulates apart (SF) so that the overflow can leave them out;
  // the map written is the sum of both (exact: integer fixed point)
  unsigned long long* SF = fillers ? S64 + tsz : S64;
  // workgroup q takes chunk q; past the tile count, workgroups without an extra chunk leave
  const int qc = blockIdx.x;
  if (qc >= t.ntiles && qc >= t.ntiles + __builtin_amdgcn_readfirstlane(ch.n_extra())) return;
  {
    const ChunkRef ck = chunk_ref(ch, t, qc);
    const TileBox tb = tile_box(g, t, ck.tile);
    EntryStream<1> es(entries, ck.first + (int)threadIdx.x, ck.last, (int)blockDim.x);
    for (int k = threadIdx.x; k < tsz; k += blockDim.x) {
      const int lx = k & (t.T - 1), ly = (k >> t.lgT) & (t.T - 1), bz = k >> (2 * t.lgT);
      // fixed_map is null when the problem has no fixed instances (the map is then all zero)
      S64[k] = (ck.chunk0 && fixed_map && lx < tb.wx && ly < tb.wy)
                   ? to_fix(fixed_map[bin_index(g, bz, tb.y0 + ly, tb.x0 + lx)])
                   : 0ull;
      if (fillers) SF[k] = 0ull;
    }
    __syncthreads();
    // large instances: bin-parallel sweep of their part of this tile (first chunk)
    for (int chunk = 0; ck.chunk0 && chunk < nlarge; chunk += blockDim.x) {
      const int nh = large_hits(lrec, nlarge, chunk, tb.x0, tb.x0 + tb.wx - 1, tb.y0, tb.y0 + tb.wy - 1, hits, wave_cnt);
      for (int h_ = 0; h_ < nh; ++h_) {
        const Foot h = foot_record(g, lrec, hits[h_]);
        const int bx0 = max(h.bx0, tb.x0), bx1 = min(h.bx1, tb.x0 + tb.wx - 1);
        const int by0 = max(h.by0, tb.y0), by1 = min(h.by1, tb.y0 + tb.wy - 1);
        const float wgt = h.omega * inv_vol;
        // thread (column lx, row ry) of the tile takes the instance's bins of column bx0 + lx in
        // rows by0 + ry, by0 + ry + rows per pass, ... on every z layer: no index division, one
        // thread per bin within one instance
        const int lx = threadIdx.x & (t.T - 1), ry = threadIdx.x >> t.lgT, rstep = blockDim.x >> t.lgT;
        const int bx = bx0 + lx;
        if (bx <= bx1) {
          const float lxv = len_x(g, h, bx);
          for (int bz = h.bz0; bz <= h.bz1; ++bz) {
            const float lz = len_z(g, h, bz);
            for (int by = by0 + ry; by <= by1; by += rstep) {
              const float v = lxv * len_y(g, h, by) * lz * wgt;
              S64[lds_index(t, bz, by - tb.y0, bx - tb.x0)] += to_fix_unit(v);
            }
          }
        }
        __syncthreads();
      }
    }
    // bucketed cells
    float4 ea, eb;
    while (es.next(ea, eb)) {
      const Foot f = foot_entry(g, ea, eb);
      unsigned long long* acc = entry_filler(ea) ? SF : S64;
      const int bx0 = max(f.bx0, tb.x0), bx1 = min(f.bx1, tb.x0 + tb.wx - 1);
      const int by0 = max(f.by0, tb.y0), by1 = min(f.by1, tb.y0 + tb.wy - 1);
      const float wgt = f.omega * inv_vol;
      const int nbx = bx1 - bx0 + 1;
      if (nbx <= kSpanX) {
        float lxs[kSpanX];
#pragma unroll
        for (int j = 0; j < kSpanX; ++j) lxs[j] = j < nbx ? len_x(g, f, bx0 + j) : 0.f;
        for (int bz = f.bz0; bz <= f.bz1; ++bz) {
          const float lz = len_z(g, f, bz) * wgt;
          for (int by = by0; by <= by1; ++by) {
            const float lyz = len_y(g, f, by) * lz;
            unsigned long long* row = &acc[lds_index(t, bz, by - tb.y0, bx0 - tb.x0)];
#pragma unroll
            for (int j = 0; j < kSpanX; ++j)
              if (j < nbx) atomicAdd(row + j, to_fix_unit(lxs[j] * lyz));
          }
        }
      } else {
        for (int bz = f.bz0; bz <= f.bz1; ++bz) {
          const float lz = len_z(g, f, bz) * wgt;
          for (int by = by0; by <= by1; ++by) {
            const float lyz = len_y(g, f, by) * lz;
            for (int bx = bx0; bx <= bx1; ++bx)
              atomicAdd(&acc[lds_index(t, bz, by - tb.y0, bx - tb.x0)], to_fix_unit(len_x(g, f, bx) * lyz));
          }
        }
      }
    }
    __syncthreads();
    if (ck.nchunks == 1) {
      write_tile(g, t, tb, ck.tile, target, fillers,
                 [&](int k, unsigned long long& real, unsigned long long& fil) {
                   real = S64[k];
                   fil = fillers ? SF[k] : 0ull;
                 },
                 rho, part, stride);
    } else {
      const int slot = ch.slot(ck.tile);
      unsigned long long* acc = heavy_acc + (size_t)slot * 2 * tsz;
      for (int k = threadIdx.x; k < tsz; k += blockDim.x) {
        const unsigned long long a = S64[k];
        if (a) atomicAdd(acc + k, a);
        if (fillers) {
          const unsigned long long b = SF[k];
          if (b) atomicAdd(acc + tsz + k, b);
        }
      }
      __threadfence();          // this chunk's sums are in place before it counts itself done
      __syncthreads();
      if (threadIdx.x == 0) last_chunk = atomicAdd(ch.done(slot), 1) == ck.nchunks - 1;
      __syncthreads();
      if (last_chunk) {
        __threadfence();        // and the other chunks' sums before the last one reads them
        write_tile(g, t, tb, ck.tile, target, fillers,
                   [&](int k, unsigned long long& real, unsigned long long& fil) {
                     real = atomicExch(acc + k, 0ull);
                     fil = fillers ? atomicExch(acc + tsz + k, 0ull) : 0ull;
                   },
                   rho, part, stride);
        if (threadIdx.x == 0) atomicExch(ch.done(slot), 0);
      }
    }
  }
}

// fixed map: one workgroup per fixed instance, global atomics (built once)
__global__ void k_density_large(Geom g, const float* __restrict__ xyz, const float* __restrict__ size,
                                const uint8_t* __restrict__ kind, const int32_t* __restrict__ list,
                                float* __restrict__ rho) {
  const int i = list[blockIdx.x];
  const Foot f = footprint(g, xyz, size, kind[i], i);
  const int nbx = f.bx1 - f.bx0 + 1, nby = f.by1 - f.by0 + 1, nbz = f.bz1 - f.bz0 + 1;
  const long long total = (long long)nbx * nby * nbz;
  const float wgt = f.omega / g.vol_bin;
  for (long long q = threadIdx.x; q < total; q += blockDim.x) {
    const int bx = f.bx0 + (int)(q % nbx);
    const long long r = q / nbx;
    const int by = f.by0 + (int)(r % nby);
    const int bz = f.bz0 + (int)(r / nby);
    const float v = len_x(g, f, bx) * len_y(g, f, by) * len_z(g, f, bz) * wgt;
    if (v != 0.f) atomicAdd(rho + bin_index(g, bz, by, bx), v);
  }
}

// Instance-parallel scatter of the large instances (the baseline of Sec. IV-A, selected by
// PLACE3D_OPT_MACRO_INSTANCE): one thread per instance walks all its bins and adds its overlap
// with a global float atomic.  The tile kernel then runs without the large-instance sweep.
__global__ __launch_bounds__(64) void k_density_large_thread(Geom g, const float* __restrict__ xyz,
                                                             const float* __restrict__ size,
                                                             const uint8_t* __restrict__ kind,
                                                             const int32_t* __restrict__ list, int nlist,
                                                             float* __restrict__ rho) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nlist) return;
  const int i = list[j];
  const Foot f = footprint(g, xyz, size, kind[i], i);
  const float wgt = f.omega / g.vol_bin;
  for (int bz = f.bz0; bz <= f.bz1; ++bz) {
    const float lz = len_z(g, f, bz) * wgt;
    for (int by = f.by0; by <= f.by1; ++by) {
      const float lyz = len_y(g, f, by) * lz;
      for (int bx = f.bx0; bx <= f.bx1; ++bx) {
        const float v = len_x(g, f, bx) * lyz;
        if (v != 0.f) atomicAdd(rho + bin_index(g, bz, by, bx), v);
      }
    }
  }
}

// per-die overflow excess of a finished map, one partial per workgroup (the tile kernel's slots
// and partial count, so the same final reduction applies)
__global__ __launch_bounds__(256) void k_map_excess(Geom g, const float* __restrict__ rho, float target,
                                                    double* __restrict__ part, int stride) {
  const long long plane = (long long)g.nx * g.ny, total = plane * g.nz;
  const long long per = (total + gridDim.x - 1) / gridDim.x;
  const long long q0 = (long long)blockIdx.x * per, q1 = q0 + per < total ? q0 + per : total;
  const long long half = plane * (g.nz / 2);
  float ex[2] = {0.f, 0.f};
  for (long long q = q0 + threadIdx.x; q < q1; q += blockDim.x) ex[q < half ? 0 : 1] += fmaxf(rho[q] - target, 0.f);
  ex[0] *= g.vol_bin;
  ex[1] *= g.vol_bin;
  block_partials<2>(ex, part, stride, R_EXCESS_BOT, blockIdx.x);
}

__global__ void k_fill(float* __restrict__ p, long long n, float v) {
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
    p[q] = v;
}

__global__ void k_zero_f64(double* __restrict__ p, int n) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) p[q] = 0.0;
}

// out[q] = sum (or max) over b < nparts of part[(slot0 + q) * stride + b], in a fixed order
// Workgroups [0, nq0) reduce slots slot0.. over nparts0 partials into out0[]; workgroups from nq0
// on reduce slots slot1.. over nparts1 partials into out1[] (a second group in the same launch).
__global__ __launch_bounds__(256) void k_red_final(const double* __restrict__ part, int stride, int slot0, int nq0,
                                                   int nparts0, int is_max, double* __restrict__ out0, int slot1,
                                                   int nparts1, double* __restrict__ out1) {
  __shared__ double sh[256];
  const bool second = (int)blockIdx.x >= nq0;
  const int qi = second ? (int)blockIdx.x - nq0 : (int)blockIdx.x;
  const int q = (second ? slot1 : slot0) + qi;
  const int nparts = second ? nparts1 : nparts0;
  double* out = second ? out1 : out0;
  const double* row = part + (size_t)q * stride;
  // four independent accumulators keep four loads in flight per thread
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int b = threadIdx.x;
  for (; b + 768 < nparts; b += 1024) {
    const double v0 = row[b], v1 = row[b + 256], v2 = row[b + 512], v3 = row[b + 768];
    if (is_max) { a0 = fmax(a0, v0); a1 = fmax(a1, v1); a2 = fmax(a2, v2); a3 = fmax(a3, v3); }
    else { a0 += v0; a1 += v1; a2 += v2; a3 += v3; }
  }
  for (; b < nparts; b += 256) a0 = is_max ? fmax(a0, row[b]) : a0 + row[b];
  sh[threadIdx.x] = is_max ? fmax(fmax(a0, a1), fmax(a2, a3)) : (a0 + a1) + (a2 + a3);
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      sh[threadIdx.x] = is_max ? fmax(sh[threadIdx.x], sh[threadIdx.x + o]) : sh[threadIdx.x] + sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[qi] = sh[0];
}

// ------------------------------------------------------------------ field gather

// every (cell, tile) entry: sum over the tile's bins of overlap * map, for three maps; then, for
// every large instance overlapping the tile, its partial sums over the tile (to lpart[j][tile])
// Field maps stored as even / odd x halves (on = 1): column x < hx is E + O, column nx-1-x is
// sign (E - O), with E at column x and O at column hx + x of the stored map.
struct FoldX { int on, hx; float sx, sy, sz; };

__global__ __launch_bounds__(kTileThreads) void k_gather_tiles(Geom g, TileGeom t, const float4* __restrict__ entries,
                                                      Chunks ch,
                                                      const float* __restrict__ mx, const float* __restrict__ my,
                                                      const float* __restrict__ mz, FoldX fx, float4* __restrict__ out,
                                                      const float4* __restrict__ lrec, int nlarge,
                                                      float4* __restrict__ lpart) {
  extern __shared__ __align__(16) float S[];
  __shared__ int hits[kTileThreads];
  __shared__ int wave_cnt[kTileThreads / kWave];
  __shared__ float rsh[3][kTileThreads / kWave];
  const int tsz = t.T * t.T * g.nz;
  // workgroup q takes chunk q; past the tile count, workgroups without an extra chunk leave
  const int qc = blockIdx.x;
  if (qc >= t.ntiles && qc >= t.ntiles + __builtin_amdgcn_readfirstlane(ch.n_extra())) return;
  {
    const ChunkRef ck = chunk_ref(ch, t, qc);
    const int tile = ck.tile;
    const TileBox tb = tile_box(g, t, tile);
    EntryStream<2> es(entries, ck.first + (int)threadIdx.x, ck.last, (int)blockDim.x);
    // natural-order maps whose rows and tile width are multiples of 4 bins: stage 4 bins per load
    // (the row start tb.x0 + lx is then a multiple of 4, so the 16-byte loads are aligned)
    const bool vec = !fx.on && (g.nx & 3) == 0 && (tb.wx & 3) == 0 &&
                     ((reinterpret_cast<uintptr_t>(mx) | reinterpret_cast<uintptr_t>(my) |
                       reinterpret_cast<uintptr_t>(mz)) & 15) == 0;
    for (int k = vec ? 4 * (int)threadIdx.x : tsz; k < tsz; k += 4 * (int)blockDim.x) {
      const int lx = k & (t.T - 1), ly = (k >> t.lgT) & (t.T - 1), bz = k >> (2 * t.lgT);
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a, d = a;
      if (lx < tb.wx && ly < tb.wy) {
        const size_t q = bin_index(g, bz, tb.y0 + ly, tb.x0 + lx);
        a = *reinterpret_cast<const float4*>(mx + q);
        b = *reinterpret_cast<const float4*>(my + q);
        d = *reinterpret_cast<const float4*>(mz + q);
      }
      *reinterpret_cast<float4*>(S + k) = a;
      *reinterpret_cast<float4*>(S + tsz + k) = b;
      *reinterpret_cast<float4*>(S + 2 * tsz + k) = d;
    }
    for (int k = vec ? tsz : (int)threadIdx.x; k < tsz; k += blockDim.x) {
      const int lx = k & (t.T - 1), ly = (k >> t.lgT) & (t.T - 1), bz = k >> (2 * t.lgT);
      float a = 0.f, b = 0.f, d = 0.f;
      if (lx < tb.wx && ly < tb.wy) {
        const int gx = tb.x0 + lx;
        if (fx.on) {
          const bool up = gx >= fx.hx;
          const size_t e = bin_index(g, bz, tb.y0 + ly, up ? g.nx - 1 - gx : gx), o = e + fx.hx;
          a = up ? fx.sx * (mx[e] - mx[o]) : mx[e] + mx[o];
          b = up ? fx.sy * (my[e] - my[o]) : my[e] + my[o];
          d = up ? fx.sz * (mz[e] - mz[o]) : mz[e] + mz[o];
        } else {
          const size_t q = bin_index(g, bz, tb.y0 + ly, gx);
          a = mx[q];
          b = my[q];
          d = mz[q];
        }
      }
      S[k] = a;
      S[tsz + k] = b;
      S[2 * tsz + k] = d;
    }
    __syncthreads();
    float4 ea, eb;
    while (es.next(ea, eb)) {
      const Foot f = foot_entry(g, ea, eb);
      const size_t oi = (size_t)entry_q(ea) * g.n + entry_cell(eb);   // cell-major result slot
      const int bx0 = max(f.bx0, tb.x0), bx1 = min(f.bx1, tb.x0 + tb.wx - 1);
      const int by0 = max(f.by0, tb.y0), by1 = min(f.by1, tb.y0 + tb.wy - 1);
      float sx = 0.f, sy = 0.f, sz = 0.f;
      const int nbx = bx1 - bx0 + 1;
      if (nbx <= kSpanX) {
        float lxs[kSpanX];
  #pragma unroll
        for (int j = 0; j < kSpanX; ++j) lxs[j] = j < nbx ? len_x(g, f, bx0 + j) : 0.f;
        for (int bz = f.bz0; bz <= f.bz1; ++bz) {
          const float lz = len_z(g, f, bz);
          for (int by = by0; by <= by1; ++by) {
            const float lyz = len_y(g, f, by) * lz;
            const int k0 = lds_index(t, bz, by - tb.y0, bx0 - tb.x0);
  #pragma unroll
            for (int j = 0; j < kSpanX; ++j)
              if (j < nbx) {
                const float v = lxs[j] * lyz;
                sx += v * S[k0 + j];
                sy += v * S[tsz + k0 + j];
                sz += v * S[2 * tsz + k0 + j];
              }
          }
        }
      } else {
        for (int bz = f.bz0; bz <= f.bz1; ++bz) {
          const float lz = len_z(g, f, bz);
          for (int by = by0; by <= by1; ++by) {
            const float lyz = len_y(g, f, by) * lz;
            for (int bx = bx0; bx <= bx1; ++bx) {
              const float v = len_x(g, f, bx) * lyz;
              const int k = lds_index(t, bz, by - tb.y0, bx - tb.x0);
              sx += v * S[k];
              sy += v * S[tsz + k];
              sz += v * S[2 * tsz + k];
            }
          }
        }
      }
      out[oi] = make_float4(f.omega * sx, f.omega * sy, f.omega * sz, 0.f);
    }
    // large instances' partial sums over the tile (first chunk)
    if (lpart && ck.chunk0) {
      for (int chunk = 0; chunk < nlarge; chunk += blockDim.x) {
        const int nh = large_hits(lrec, nlarge, chunk, tb.x0, tb.x0 + tb.wx - 1, tb.y0, tb.y0 + tb.wy - 1, hits, wave_cnt);
        for (int r = 0; r < nh; ++r) {
          const int j = hits[r];
          const Foot h = foot_record(g, lrec, j);
          const int bx0 = max(h.bx0, tb.x0), bx1 = min(h.bx1, tb.x0 + tb.wx - 1);
          const int by0 = max(h.by0, tb.y0), by1 = min(h.by1, tb.y0 + tb.wy - 1);
          const int nbx = bx1 - bx0 + 1, nby = by1 - by0 + 1, nbz = h.bz1 - h.bz0 + 1;
          const int total_bins = nbx * nby * nbz;
          float sx = 0.f, sy = 0.f, sz = 0.f;
          for (int q = threadIdx.x; q < total_bins; q += blockDim.x) {
            const int bx = bx0 + q % nbx, by = by0 + (q / nbx) % nby, bz = h.bz0 + q / (nbx * nby);
            const float v = len_x(g, h, bx) * len_y(g, h, by) * len_z(g, h, bz);
            const int k = lds_index(t, bz, by - tb.y0, bx - tb.x0);
            sx += v * S[k];
            sy += v * S[tsz + k];
            sz += v * S[2 * tsz + k];
          }
          for (int o = kWave / 2; o > 0; o >>= 1) {
            sx += __shfl_xor(sx, o); sy += __shfl_xor(sy, o); sz += __shfl_xor(sz, o);
          }
          if ((threadIdx.x & (kWave - 1)) == 0) {
            rsh[0][threadIdx.x / kWave] = sx; rsh[1][threadIdx.x / kWave] = sy; rsh[2][threadIdx.x / kWave] = sz;
          }
          __syncthreads();
          if (threadIdx.x == 0) {
            float a = 0.f, b = 0.f, c = 0.f;
            for (int w = 0; w < (int)(blockDim.x / kWave); ++w) { a += rsh[0][w]; b += rsh[1][w]; c += rsh[2][w]; }
            lpart[(size_t)j * t.ntiles + tile] = make_float4(h.omega * a, h.omega * b, h.omega * c, 0.f);
          }
          __syncthreads();
        }
      }
    }
  }
}

// per large instance (one wavefront each): sum the partials of the tiles its record overlaps
__global__ void k_large_gather_finish(Geom g, TileGeom t, const int32_t* __restrict__ large, int nlarge,
                                      const float4* __restrict__ lrec, const float4* __restrict__ lpart, float scale,
                                      float* __restrict__ grad, int accumulate) {
  const int j = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (j >= nlarge) return;
  const float4 b = lrec[4 * (size_t)j + 3];
  const int tx0 = __float_as_int(b.x) >> t.lgT, tx1 = __float_as_int(b.y) >> t.lgT;
  const int ty0 = __float_as_int(b.z) >> t.lgT, ty1 = __float_as_int(b.w) >> t.lgT;
  const int ntx = tx1 - tx0 + 1, count = ntx * (ty1 - ty0 + 1);
  float sx = 0.f, sy = 0.f, sz = 0.f;
  for (int q = lane; q < count; q += kWave) {
    const float4 v = lpart[(size_t)j * t.ntiles + (ty0 + q / ntx) * t.ntx + tx0 + q % ntx];
    sx += v.x; sy += v.y; sz += v.z;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) { sx += __shfl_xor(sx, o); sy += __shfl_xor(sy, o); sz += __shfl_xor(sz, o); }
  if (lane == 0) {
    const int i = large[j], n = g.n;
    if (accumulate) { grad[i] += scale * sx; grad[n + i] += scale * sy; grad[2 * n + i] += scale * sz; }
    else { grad[i] = scale * sx; grad[n + i] = scale * sy; grad[2 * n + i] = scale * sz; }
  }
}

__device__ __forceinline__ void gather3(const Geom& g, const float* __restrict__ mx, const float* __restrict__ my,
                                        const float* __restrict__ mz, int bz, int by, int bx, float v, float& sx,
                                        float& sy, float& sz) {
  const size_t b = bin_index(g, bz, by, bx);
  sx += v * mx[b];
  sy += v * my[b];
  sz += v * mz[b];
}

// one workgroup per large instance: gather with a block reduction
__global__ void k_gather_large(Geom g, const float* __restrict__ xyz, const float* __restrict__ size,
                               const uint8_t* __restrict__ kind, const int32_t* __restrict__ list,
                               const float* __restrict__ mx, const float* __restrict__ my,
                               const float* __restrict__ mz, float scale, float* __restrict__ grad,
                               int accumulate) {
  __shared__ float sh[256 / kWave];
  const int i = list[blockIdx.x];
  const Foot f = footprint(g, xyz, size, kind[i], i);
  const int nbx = f.bx1 - f.bx0 + 1, nby = f.by1 - f.by0 + 1, nbz = f.bz1 - f.bz0 + 1;
  const long long total = (long long)nbx * nby * nbz;
  float sx = 0.f, sy = 0.f, sz = 0.f;
  for (long long q = threadIdx.x; q < total; q += blockDim.x) {
    const int bx = f.bx0 + (int)(q % nbx);
    const long long r = q / nbx;
    const int by = f.by0 + (int)(r % nby);
    const int bz = f.bz0 + (int)(r / nby);
    const float v = len_x(g, f, bx) * len_y(g, f, by) * len_z(g, f, bz);
    gather3(g, mx, my, mz, bz, by, bx, v, sx, sy, sz);
  }
  sx = block_sum<256>(sx, sh);
  sy = block_sum<256>(sy, sh);
  sz = block_sum<256>(sz, sh);
  if (threadIdx.x == 0) {
    const float s = scale * f.omega;
    const int n = g.n;
    if (accumulate) { grad[i] += s * sx; grad[n + i] += s * sy; grad[2 * n + i] += s * sz; }
    else { grad[i] = s * sx; grad[n + i] = s * sy; grad[2 * n + i] = s * sz; }
  }
}

// ------------------------------------------------------------------ exact adjoint

// Face sums of the map: the derivative of an overlap length with respect to an edge is +-1 on
// the bin holding that edge.  (gx, gy, gz) = face differences; for large instances also the sums
// the macro size-transition terms need.  Loops over the bins q = t0, t0 + tstep, ... of the box
// [bx0..bx1] x [by0..by1] x [bz0..bz1] (a sub-box of the footprint).
struct AdjSums { float gx, gy, gz, xs, ys, all; };

// widen [lo, hi] to an edge bin b (>= 0) lying inside the limits [l0, l1]
__device__ __forceinline__ void widen(int& lo, int& hi, int b, int l0, int l1) {
  if (b >= l0 && b <= l1) { lo = min(lo, b); hi = max(hi, b); }
}

// [bx0, bx1] x [by0, by1]: the footprint's bins inside the limits [xl0, xl1] x [yl0, yl1] (a
// tile, or the grid); the loop also visits the edge bins inside the limits that lie just off
// the footprint (an edge on a bin face).
template <class MapAt>
__device__ __forceinline__ AdjSums adjoint_sums(const Geom& g, const Foot& f, MapAt map_at, int bx0, int bx1,
                                                int by0, int by1, int xl0, int xl1, int yl0, int yl1, int t0,
                                                int tstep, bool with_size_terms) {
  const EdgeBins e = edge_bins(g, f);
  // the size transition moves the planar edges as z moves: an upper edge the way of dw/dz, a
  // lower edge the other way, each with its own one-sided bin
  int sxl = -1, sxh = -1, syl = -1, syh = -1;
  if (with_size_terms) {
    const float2 fx = local_faces(g.dx, f.cbx, g.wbd), fy = local_faces(g.dy, f.cby, g.hbd);
    const float bx = kClampBand * g.dx, by = kClampBand * g.dy;
    const bool hx = e.down_z != (f.dw < 0.f), hy = e.down_z != (f.dh < 0.f);   // upper edge moving down
    sxl = edge_bin(snap_face(f.rx0, fx, bx), fx.x, fx.y, g.inv_wb, !hx, f.cbx, g.nx);
    sxh = edge_bin(snap_face(f.rx1, fx, bx), fx.x, fx.y, g.inv_wb, hx, f.cbx, g.nx);
    syl = edge_bin(snap_face(f.ry0, fy, by), fy.x, fy.y, g.inv_hb, !hy, f.cby, g.ny);
    syh = edge_bin(snap_face(f.ry1, fy, by), fy.x, fy.y, g.inv_hb, hy, f.cby, g.ny);
  }
  int x0 = bx0, x1 = bx1, y0 = by0, y1 = by1, z0 = f.bz0, z1 = f.bz1;
  widen(x0, x1, e.xl, xl0, xl1); widen(x0, x1, e.xh, xl0, xl1);
  widen(x0, x1, sxl, xl0, xl1); widen(x0, x1, sxh, xl0, xl1);
  widen(y0, y1, e.yl, yl0, yl1); widen(y0, y1, e.yh, yl0, yl1);
  widen(y0, y1, syl, yl0, yl1); widen(y0, y1, syh, yl0, yl1);
  widen(z0, z1, e.zl, 0, g.nz - 1); widen(z0, z1, e.zh, 0, g.nz - 1);
  const int nbx = x1 - x0 + 1, nby = y1 - y0 + 1, nbz = z1 - z0 + 1;
  const int total = nbx * nby * nbz;
  AdjSums a = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int q = t0; q < total; q += tstep) {
    const int bx = x0 + q % nbx, by = y0 + (q / nbx) % nby, bz = z0 + q / (nbx * nby);
    const float mv = map_at(bz, by, bx);
    const float lx = len_x(g, f, bx), ly = len_y(g, f, by), lz = len_z(g, f, bz);
    const float fxh = (bx == e.xh) ? 1.f : 0.f, fxl = (bx == e.xl) ? 1.f : 0.f;
    const float fyh = (by == e.yh) ? 1.f : 0.f, fyl = (by == e.yl) ? 1.f : 0.f;
    const float fzh = (bz == e.zh) ? 1.f : 0.f, fzl = (bz == e.zl) ? 1.f : 0.f;
    a.gx += (fxh - fxl) * ly * lz * mv;
    a.gy += lx * (fyh - fyl) * lz * mv;
    a.gz += lx * ly * (fzh - fzl) * mv;
    if (with_size_terms) {
      const float sx = (bx == sxh ? 1.f : 0.f) + (bx == sxl ? 1.f : 0.f);
      const float sy = (by == syh ? 1.f : 0.f) + (by == syl ? 1.f : 0.f);
      a.xs += sx * ly * lz * mv;
      a.ys += lx * sy * lz * mv;
      a.all += lx * ly * lz * mv;
    }
  }
  return a;
}

// adjoint_sums of one bucketed cell (no size terms, one thread), as nested loops over z, y and x
// with the x overlaps and edge indicators held in registers: the same bins in the same order as
// the flat loop, so the same sums bit for bit, without its index divisions.  Boxes wider than
// kAdjSpan bins take the flat loop.
constexpr int kAdjSpan = 8;

template <class MapAt>
__device__ __forceinline__ AdjSums adjoint_sums_cell(const Geom& g, const Foot& f, MapAt map_at, int bx0, int bx1,
                                                     int by0, int by1, int xl0, int xl1, int yl0, int yl1) {
  const EdgeBins e = edge_bins(g, f);
  int x0 = bx0, x1 = bx1, y0 = by0, y1 = by1, z0 = f.bz0, z1 = f.bz1;
  widen(x0, x1, e.xl, xl0, xl1); widen(x0, x1, e.xh, xl0, xl1);
  widen(y0, y1, e.yl, yl0, yl1); widen(y0, y1, e.yh, yl0, yl1);
  widen(z0, z1, e.zl, 0, g.nz - 1); widen(z0, z1, e.zh, 0, g.nz - 1);
  const int nbx = x1 - x0 + 1;
  if (nbx > kAdjSpan) return adjoint_sums(g, f, map_at, bx0, bx1, by0, by1, xl0, xl1, yl0, yl1, 0, 1, false);
  float lxs[kAdjSpan], dxs[kAdjSpan];
#pragma unroll
  for (int j = 0; j < kAdjSpan; ++j) {
    const int bx = x0 + j;
    lxs[j] = j < nbx ? len_x(g, f, bx) : 0.f;
    dxs[j] = ((bx == e.xh) ? 1.f : 0.f) - ((bx == e.xl) ? 1.f : 0.f);
  }
  AdjSums a = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int bz = z0; bz <= z1; ++bz) {
    const float lz = len_z(g, f, bz);
    const float dz = ((bz == e.zh) ? 1.f : 0.f) - ((bz == e.zl) ? 1.f : 0.f);
    for (int by = y0; by <= y1; ++by) {
      const float ly = len_y(g, f, by);
      const float dy = ((by == e.yh) ? 1.f : 0.f) - ((by == e.yl) ? 1.f : 0.f);
#pragma unroll
      for (int j = 0; j < kAdjSpan; ++j)
        if (j < nbx) {
          const float mv = map_at(bz, by, x0 + j);
          a.gx += dxs[j] * ly * lz * mv;
          a.gy += lxs[j] * dy * lz * mv;
          a.gz += lxs[j] * ly * dz * mv;
        }
    }
  }
  return a;
}

__device__ __forceinline__ float3 adjoint_finish(const Geom& g, const Foot& f, const AdjSums& a) {
  float3 r = make_float3(f.omega * a.gx, f.omega * a.gy, f.omega * a.gz);
  if (f.dw != 0.f || f.dh != 0.f) {
    const float r2 = 1.41421356237309515f;
    const float wmin = r2 * g.wb, hmin = r2 * g.hb;
    const bool sw = f.w < wmin, sh = f.h < hmin;
    const float fw = fminf(1.f, f.w / wmin), fh = fminf(1.f, f.h / hmin);
    const float domega = (sw ? f.dw / wmin : 0.f) * fh + fw * (sh ? f.dh / hmin : 0.f);
    const float dwt = sw ? 0.f : f.dw, dht = sh ? 0.f : f.dh;
    r.z += domega * a.all + f.omega * 0.5f * (dwt * a.xs + dht * a.ys);
  }
  return r;
}

__global__ __launch_bounds__(kTileThreads) void k_adjoint_tiles(Geom g, TileGeom t, const float4* __restrict__ entries,
                                                       Chunks ch,
                                                       const float* __restrict__ m, float4* __restrict__ out,
                                                       const float4* __restrict__ lrec, int nlarge,
                                                       float4* __restrict__ lpart) {
  extern __shared__ __align__(16) float S[];
  __shared__ int hits[kTileThreads];
  __shared__ int wave_cnt[kTileThreads / kWave];
  __shared__ float rsh[6][kTileThreads / kWave];
  const int tsz = t.T * t.T * g.nz;
  // workgroup q takes chunk q; past the tile count, workgroups without an extra chunk leave
  const int qc = blockIdx.x;
  if (qc >= t.ntiles && qc >= t.ntiles + __builtin_amdgcn_readfirstlane(ch.n_extra())) return;
  {
    const ChunkRef ck = chunk_ref(ch, t, qc);
    const int tile = ck.tile;
    const TileBox tb = tile_box(g, t, tile);
    EntryStream<1> es(entries, ck.first + (int)threadIdx.x, ck.last, (int)blockDim.x);
    // rows and tile width multiples of 4 bins: stage 4 bins per load (aligned, as in the gather)
    const bool vec = (g.nx & 3) == 0 && (tb.wx & 3) == 0 && (reinterpret_cast<uintptr_t>(m) & 15) == 0;
    for (int k = vec ? 4 * (int)threadIdx.x : tsz; k < tsz; k += 4 * (int)blockDim.x) {
      const int lx = k & (t.T - 1), ly = (k >> t.lgT) & (t.T - 1), bz = k >> (2 * t.lgT);
      *reinterpret_cast<float4*>(S + k) =
          (lx < tb.wx && ly < tb.wy) ? *reinterpret_cast<const float4*>(m + bin_index(g, bz, tb.y0 + ly, tb.x0 + lx))
                                     : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    for (int k = vec ? tsz : (int)threadIdx.x; k < tsz; k += blockDim.x) {
      const int lx = k & (t.T - 1), ly = (k >> t.lgT) & (t.T - 1), bz = k >> (2 * t.lgT);
      S[k] = (lx < tb.wx && ly < tb.wy) ? m[bin_index(g, bz, tb.y0 + ly, tb.x0 + lx)] : 0.f;
    }
    __syncthreads();
    auto at = [&](int bz, int by, int bx) { return S[lds_index(t, bz, by - tb.y0, bx - tb.x0)]; };
    float4 ea, eb;
    while (es.next(ea, eb)) {
      const Foot f = foot_entry(g, ea, eb);
      const size_t oi = (size_t)entry_q(ea) * g.n + entry_cell(eb);   // cell-major result slot
      const int bx0 = max(f.bx0, tb.x0), bx1 = min(f.bx1, tb.x0 + tb.wx - 1);
      const int by0 = max(f.by0, tb.y0), by1 = min(f.by1, tb.y0 + tb.wy - 1);
      float3 r = make_float3(0.f, 0.f, 0.f);
      if (bx0 <= bx1 && by0 <= by1) {
        const AdjSums a = adjoint_sums_cell(g, f, at, bx0, bx1, by0, by1, tb.x0, tb.x0 + tb.wx - 1, tb.y0,
                                            tb.y0 + tb.wy - 1);
        r = adjoint_finish(g, f, a);
      }
      out[oi] = make_float4(r.x, r.y, r.z, 0.f);
    }
    // large instances' partial sums over the tile (first chunk)
    if (lpart && ck.chunk0) {
      for (int chunk = 0; chunk < nlarge; chunk += blockDim.x) {
        const int nh = large_hits(lrec, nlarge, chunk, tb.x0, tb.x0 + tb.wx - 1, tb.y0, tb.y0 + tb.wy - 1, hits, wave_cnt);
        for (int r = 0; r < nh; ++r) {
          const int j = hits[r];
          const Foot h = foot_record(g, lrec, j);
          const int bx0 = max(h.bx0, tb.x0), bx1 = min(h.bx1, tb.x0 + tb.wx - 1);
          const int by0 = max(h.by0, tb.y0), by1 = min(h.by1, tb.y0 + tb.wy - 1);
          AdjSums a = adjoint_sums(g, h, at, bx0, bx1, by0, by1, tb.x0, tb.x0 + tb.wx - 1, tb.y0, tb.y0 + tb.wy - 1,
                                   threadIdx.x, blockDim.x, true);
          float v[6] = {a.gx, a.gy, a.gz, a.xs, a.ys, a.all};
          for (int q = 0; q < 6; ++q) {
            for (int o = kWave / 2; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o);
            if ((threadIdx.x & (kWave - 1)) == 0) rsh[q][threadIdx.x / kWave] = v[q];
          }
          __syncthreads();
          if (threadIdx.x == 0) {
            float w[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            for (int q = 0; q < 6; ++q)
              for (int u = 0; u < (int)(blockDim.x / kWave); ++u) w[q] += rsh[q][u];
            lpart[2 * ((size_t)j * t.ntiles + tile)] = make_float4(w[0], w[1], w[2], 0.f);
            lpart[2 * ((size_t)j * t.ntiles + tile) + 1] = make_float4(w[3], w[4], w[5], 0.f);
          }
          __syncthreads();
        }
      }
    }
  }
}

__global__ void k_large_adjoint_finish(Geom g, TileGeom t, const int32_t* __restrict__ large, int nlarge,
                                       const float4* __restrict__ lrec, const float4* __restrict__ lpart, float scale,
                                       const double* __restrict__ dscale, float* __restrict__ grad, int accumulate) {
  const int j = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (j >= nlarge) return;
  const float4 b = lrec[4 * (size_t)j + 3];
  const int tx0 = __float_as_int(b.x) >> t.lgT, tx1 = __float_as_int(b.y) >> t.lgT;
  const int ty0 = __float_as_int(b.z) >> t.lgT, ty1 = __float_as_int(b.w) >> t.lgT;
  const int ntx = tx1 - tx0 + 1, count = ntx * (ty1 - ty0 + 1);
  AdjSums a = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int q = lane; q < count; q += kWave) {
    const size_t k = 2 * ((size_t)j * t.ntiles + (ty0 + q / ntx) * t.ntx + tx0 + q % ntx);
    const float4 u = lpart[k], w = lpart[k + 1];
    a.gx += u.x; a.gy += u.y; a.gz += u.z; a.xs += w.x; a.ys += w.y; a.all += w.z;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) {
    a.gx += __shfl_xor(a.gx, o); a.gy += __shfl_xor(a.gy, o); a.gz += __shfl_xor(a.gz, o);
    a.xs += __shfl_xor(a.xs, o); a.ys += __shfl_xor(a.ys, o); a.all += __shfl_xor(a.all, o);
  }
  if (lane == 0) {
    const Foot f = foot_record(g, lrec, j);
    const float3 r = adjoint_finish(g, f, a);
    const float s = scale / g.vol_bin * (dscale ? (float)dscale[0] : 1.f);
    const int i = large[j], n = g.n;
    if (accumulate) { grad[i] += s * r.x; grad[n + i] += s * r.y; grad[2 * n + i] += s * r.z; }
    else { grad[i] = s * r.x; grad[n + i] = s * r.y; grad[2 * n + i] = s * r.z; }
  }
}

__global__ void k_adjoint_large(Geom g, const float* __restrict__ xyz, const float* __restrict__ size,
                                const uint8_t* __restrict__ kind, const int32_t* __restrict__ list,
                                const float* __restrict__ m, float scale, const double* __restrict__ dscale,
                                float* __restrict__ grad, int accumulate) {
  __shared__ float sh[256 / kWave];
  const int i = list[blockIdx.x];
  const Foot f = footprint(g, xyz, size, kind[i], i);
  auto at = [&](int bz, int by, int bx) { return m[bin_index(g, bz, by, bx)]; };
  AdjSums a = adjoint_sums(g, f, at, f.bx0, f.bx1, f.by0, f.by1, 0, g.nx - 1, 0, g.ny - 1, threadIdx.x, blockDim.x,
                           true);
  a.gx = block_sum<256>(a.gx, sh);
  a.gy = block_sum<256>(a.gy, sh);
  a.gz = block_sum<256>(a.gz, sh);
  a.xs = block_sum<256>(a.xs, sh);
  a.ys = block_sum<256>(a.ys, sh);
  a.all = block_sum<256>(a.all, sh);
  if (threadIdx.x == 0) {
    const float3 r = adjoint_finish(g, f, a);
    const float s = scale / g.vol_bin * (dscale ? (float)dscale[0] : 1.f);
    const int n = g.n;
    if (accumulate) { grad[i] += s * r.x; grad[n + i] += s * r.y; grad[2 * n + i] += s * r.z; }
    else { grad[i] = s * r.x; grad[n + i] = s * r.y; grad[2 * n + i] = s * r.z; }
  }
}

// per instance: the sum of its (<= 4) entry results (cell-major, res[q][n]) for bucketed cells,
// zero for fixed instances; large instances are written by their own kernel
__global__ void k_cells_combine(int n, const uint8_t* __restrict__ cls, const int32_t* __restrict__ tiles_of,
                                const float4* __restrict__ res, float scale, const double* __restrict__ dscale,
                                float* __restrict__ grad, int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint8_t c = cls[i];
  if (c == kClsLarge) return;
  if (dscale) scale *= (float)dscale[0];
  float sx = 0.f, sy = 0.f, sz = 0.f;
  if (c == kClsCell) {
    const int cnt = entry_count(tiles_of[i]);
    for (int q = 0; q < cnt; ++q) { const float4 v = res[(size_t)q * n + i]; sx += v.x; sy += v.y; sz += v.z; }
    sx *= scale; sy *= scale; sz *= scale;
  }
  if (accumulate) { grad[i] += sx; grad[n + i] += sy; grad[2 * n + i] += sz; }
  else { grad[i] = sx; grad[n + i] = sy; grad[2 * n + i] = sz; }
}

size_t tile_lds(const place3d_ctx* c, int maps) { return sizeof(float) * (size_t)maps * c->tg.T * c->tg.T * c->g.nz; }

Chunks chunks_of(const place3d_ctx* c) { return Chunks{c->bk_tile_start, c->bk_plan, c->tg.ntiles, c->max_extra}; }

}  // namespace

// ------------------------------------------------------------------ launchers

int launch_zero_f64(place3d_ctx* c, double* p, int n, hipStream_t s) {
  ProfScope prof_(c, PLACE3D_STAGE_UPDATE, s);
  hipLaunchKernelGGL(k_zero_f64, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n);
  P3D_LAUNCH(c, "k_zero_f64");
  return PLACE3D_OK;
}

int launch_fill_f32(place3d_ctx* c, float* p, long long n, float v, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<long long>(blocks_for(n, 256), 4096);
  hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, s, p, n, v);
  P3D_LAUNCH(c, "k_fill");
  return PLACE3D_OK;
}

int reduce_final(place3d_ctx* c, int slot0, int nq, int nparts, bool is_max, double* out, hipStream_t s) {
  return reduce_final_in(c, c->part, c->part_stride, slot0, nq, nparts, is_max, out, s);
}

int reduce_final_in(place3d_ctx* c, const double* part, int stride, int slot0, int nq, int nparts, bool is_max,
                    double* out, hipStream_t s) {
  ProfScope prof_(c, PLACE3D_STAGE_UPDATE, s);
  hipLaunchKernelGGL(k_red_final, dim3(nq), dim3(256), 0, s, part, stride, slot0, nq, nparts, is_max ? 1 : 0, out,
                     0, 0, out);
  P3D_LAUNCH(c, "k_red_final");
  return PLACE3D_OK;
}

int reduce_final2(place3d_ctx* c, int slot0, int nq0, int nparts0, double* out0, int slot1, int nq1, int nparts1,
                  double* out1, hipStream_t s) {
  ProfScope prof_(c, PLACE3D_STAGE_UPDATE, s);
  hipLaunchKernelGGL(k_red_final, dim3(nq0 + nq1), dim3(256), 0, s, c->part, c->part_stride, slot0, nq0, nparts0, 0,
                     out0, slot1, nparts1, out1);
  P3D_LAUNCH(c, "k_red_final");
  return PLACE3D_OK;
}

int build_fixed_map(place3d_ctx* c, hipStream_t s) {
  const Geom& g = c->g;
  const long long map = (long long)g.nx * g.ny * g.nz;
  if (int rc = launch_fill_f32(c, c->fixed_map, map, 0.f, s)) return rc;
  if (c->n_fixed > 0) {
    hipLaunchKernelGGL(k_density_large, dim3(c->n_fixed), dim3(256), 0, s, g, c->prob.fixed_xyz,
                       c->prob.size, c->prob.kind, c->fixed_list, c->fixed_map);
    P3D_LAUNCH(c, "k_density_large(fixed)");
  }
  return PLACE3D_OK;
}

int bucket_cells(place3d_ctx* c, const float* xyz, hipStream_t s, int part) {
  const Geom& g = c->g;
  const TileGeom& t = c->tg;
  const place3d_problem& p = c->prob;
  ProfScope prof_(c, PLACE3D_STAGE_BUCKET, s);
  const size_t hist = sizeof(int) * t.ntiles;
  const int nrec = (c->n_large + kBucketThreads - 1) / kBucketThreads;
  if (part != 2) {
    hipLaunchKernelGGL(k_bucket_count, dim3(t.nblk + nrec), dim3(kBucketThreads), hist, s, g, t, xyz, p.size, p.kind,
                       c->cls, c->bk_counts, c->cell_entry, c->xyzp, c->large_list, c->n_large, c->large_rec);
    P3D_LAUNCH(c, "k_bucket_count");
  }
  if (part == 1) return PLACE3D_OK;
  hipLaunchKernelGGL(k_bucket_scan_cols, dim3((t.ntiles + kScanTiles - 1) / kScanTiles), dim3(kScanTiles * kScanParts), 0, s, t.nblk,
                     t.ntiles, c->bk_counts, c->bk_totals);
  P3D_LAUNCH(c, "k_bucket_scan_cols");
  hipLaunchKernelGGL(k_bucket_scatter, dim3(t.nblk), dim3(kBucketThreads), hist, s, g, t, xyz, p.size, p.kind, c->cls,
                     c->bk_counts, c->bk_totals, c->bk_tile_start, c->bk_entries, c->cell_entry, c->max_extra,
                     c->bk_plan);
  P3D_LAUNCH(c, "k_bucket_scatter");
  return PLACE3D_OK;
}

int density_tiles(place3d_ctx* c, const float* xyz, float* rho, double* red, hipStream_t s, bool reduce) {
  const Geom& g = c->g;
  const TileGeom& t = c->tg;
  const place3d_problem& p = c->prob;
  {
    ProfScope prof_(c, PLACE3D_STAGE_DENSITY, s);
    const int fillers = c->n_fillers > 0 ? 1 : 0;
    const bool inst = (p.options & PLACE3D_OPT_MACRO_INSTANCE) != 0;
    hipLaunchKernelGGL(k_density_tiles, dim3(t.ntiles + c->max_extra), dim3(kTileThreads), (2 + 2 * fillers) * tile_lds(c, 1), s, g,
                       t, c->bk_entries, chunks_of(c), c->heavy_acc,
                       c->n_fixed > 0 ? c->fixed_map : nullptr, c->large_rec,
                       inst ? 0 : c->n_large, (float)p.target_density, fillers, rho, c->part, c->part_stride);
    P3D_LAUNCH(c, "k_density_tiles");
    if (inst && c->n_large > 0) {
      hipLaunchKernelGGL(k_density_large_thread, dim3(blocks_for(c->n_large, 64)), dim3(64), 0, s, g, xyz, p.size,
                         p.kind, c->large_list, c->n_large, rho);
      P3D_LAUNCH(c, "k_density_large_thread");
      hipLaunchKernelGGL(k_map_excess, dim3(t.ntiles), dim3(256), 0, s, g, rho, (float)p.target_density, c->part,
                         c->part_stride);
      P3D_LAUNCH(c, "k_map_excess");
    }
  }
  if (!reduce) return PLACE3D_OK;
  return reduce_final(c, R_EXCESS_BOT, 2, t.ntiles, false, red + R_EXCESS_BOT, s);
}

int density_forward(place3d_ctx* c, const float* xyz, float* rho, hipStream_t s) {
  if (int rc = bucket_cells(c, xyz, s)) return rc;
  return density_tiles(c, xyz, rho, c->red2, s);
}

int gather_bucketed(place3d_ctx* c, const float* xyz, const float* ex, const float* ey, const float* ez, float scale,
                    float* grad, int accumulate, hipStream_t s, bool cells, bool xfold) {
  const Geom& g = c->g;
  const TileGeom& t = c->tg;
  const place3d_problem& p = c->prob;
  const bool tiled = large_in_tiles(c);
  ProfScope prof_(c, PLACE3D_STAGE_DGRAD, s);
  if (xfold && !tiled) return set_err(c, PLACE3D_ERR_ARG, "x-folded field maps need the tiled large-instance path");
  // Ex comes from the sine basis (unfold sign -1), Ey and Ez from the cosine basis (+1)
  const FoldX fx{xfold ? 1 : 0, g.nx / 2, -1.f, 1.f, 1.f};
  hipLaunchKernelGGL(k_gather_tiles, dim3(t.ntiles + c->max_extra), dim3(kTileThreads), tile_lds(c, 3), s, g, t, c->bk_entries,
                     chunks_of(c), ex, ey, ez, fx, c->entry_out, c->large_rec, c->n_large,
                     tiled && c->n_large > 0 ? c->lpart : nullptr);
  P3D_LAUNCH(c, "k_gather_tiles");
  if (c->n_large > 0 && tiled) {
    hipLaunchKernelGGL(k_large_gather_finish, dim3(blocks_for(c->n_large, 256 / kWave)), dim3(256), 0, s, g, t,
                       c->large_list, c->n_large, c->large_rec, c->lpart, scale, grad, accumulate);
    P3D_LAUNCH(c, "k_large_gather_finish");
  } else if (c->n_large > 0) {
    hipLaunchKernelGGL(k_gather_large, dim3(c->n_large), dim3(256), 0, s, g, xyz, p.size, p.kind, c->large_list, ex,
                       ey, ez, scale, grad, accumulate);
    P3D_LAUNCH(c, "k_gather_large");
  }
  c->cell_scale = scale;
  if (!cells) return PLACE3D_OK;
  hipLaunchKernelGGL(k_cells_combine, dim3(blocks_for(g.n, 256)), dim3(256), 0, s, g.n, c->cls, c->cell_entry,
                     c->entry_out, scale, (const double*)nullptr, grad, accumulate);
  P3D_LAUNCH(c, "k_cells_combine");
  return PLACE3D_OK;
}

int adjoint_bucketed(place3d_ctx* c, const float* xyz, const float* gmap, float scale, float* grad, int accumulate,
                     hipStream_t s, bool cells, const double* dscale) {
  const Geom& g = c->g;
  const TileGeom& t = c->tg;
  const place3d_problem& p = c->prob;
  const bool tiled = large_in_tiles(c);
  ProfScope prof_(c, PLACE3D_STAGE_DGRAD, s);
  hipLaunchKernelGGL(k_adjoint_tiles, dim3(t.ntiles + c->max_extra), dim3(kTileThreads), tile_lds(c, 1), s, g, t, c->bk_entries,
                     chunks_of(c), gmap, c->entry_out, c->large_rec, c->n_large,
                     tiled && c->n_large > 0 ? c->lpart : nullptr);
  P3D_LAUNCH(c, "k_adjoint_tiles");
  if (c->n_large > 0 && tiled) {
    hipLaunchKernelGGL(k_large_adjoint_finish, dim3(blocks_for(c->n_large, 256 / kWave)), dim3(256), 0, s, g, t,
                       c->large_list, c->n_large, c->large_rec, c->lpart, scale, dscale, grad, accumulate);
    P3D_LAUNCH(c, "k_large_adjoint_finish");
  } else if (c->n_large > 0) {
    hipLaunchKernelGGL(k_adjoint_large, dim3(c->n_large), dim3(256), 0, s, g, xyz, p.size, p.kind, c->large_list, gmap,
                       scale, dscale, grad, accumulate);
    P3D_LAUNCH(c, "k_adjoint_large");
  }
  c->cell_scale = scale / g.vol_bin;
  if (!cells) return PLACE3D_OK;
  hipLaunchKernelGGL(k_cells_combine, dim3(blocks_for(g.n, 256)), dim3(256), 0, s, g.n, c->cls, c->cell_entry,
                     c->entry_out, scale / g.vol_bin, dscale, grad, accumulate);
  P3D_LAUNCH(c, "k_cells_combine");
  return PLACE3D_OK;
}

int density_field_gather(place3d_ctx* c, const float* xyz, const float* ex, const float* ey, const float* ez,
                         float scale, float* grad, int accumulate, hipStream_t s) {
  if (int rc = bucket_cells(c, xyz, s)) return rc;
  return gather_bucketed(c, xyz, ex, ey, ez, scale, grad, accumulate, s);
}

int density_adjoint(place3d_ctx* c, const float* xyz, const float* gmap, float scale, float* grad, int accumulate,
                    hipStream_t s, const double* dscale) {
  if (int rc = bucket_cells(c, xyz, s)) return rc;
  return adjoint_bucketed(c, xyz, gmap, scale, grad, accumulate, s, true, dscale);
}

}  // namespace p3d
