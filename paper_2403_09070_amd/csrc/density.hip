// Density map (Sec. IV-A, Eq. density-map-accum), its field-gather gradient and exact adjoint.
//
// Every instance is a cuboid [x -/+ w~/2] x [y -/+ h~/2] x [z -/+ d_z/4] clipped to the region,
// where w~ = max(w, sqrt2 w_b) is the local-smoothness stretch and omega = w h / (w~ h~) its
// weight; w, h follow the partition for cells (Eq. std-size-tech) and z linearly for macros
// (Eq. macro-size-tech).  rho_b = sum_i omega_i vol(D_i ∩ b) / vol(b).
//
// Planar extents are handled in coordinates local to the bin column holding the centre, so
// that the overlap lengths keep float32 precision relative to the bin size even where the
// absolute coordinate is large.
//
// Work split: cells (small, many) take one thread per instance; macros (large, few) take one
// workgroup per instance sweeping its bins (the bin-parallel side of the paper's adaptive
// scheme).  Fixed instances form a constant map built once.
#include "internal.h"

namespace p3d {
namespace {

struct Foot {
  int bx0, bx1, by0, by1, bz0, bz1;   // inclusive bin ranges of the clipped cuboid
  int cbx, cby;                       // bin column / row holding the centre (local origin)
  float lx0, lx1, ly0, ly1;           // clipped planar edges, local to (cbx*wb, cby*hb)
  float rx0, rx1, ry0, ry1;           // unclipped planar edges, local
  float z0, z1, rz0, rz1;             // clipped / unclipped z edges (absolute)
  float omega, w, h, wt, ht;
  float dw, dh;                       // macro size slope dw/dz, dh/dz inside the transition range
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ Foot footprint(const Geom& g, const float* __restrict__ xyz,
                                          const float* __restrict__ size, uint8_t kind, int i) {
  Foot f;
  const int n = g.n;
  const float x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
  const float wbot = size[i], hbot = size[n + i], wtop = size[2 * n + i], htop = size[3 * n + i];
  float w, h;
  f.dw = 0.f;
  f.dh = 0.f;
  if (kind & PLACE3D_KIND_MACRO) {
    const float zl = 0.25f * g.dz, zh = 0.75f * g.dz;
    const float zc = fminf(fmaxf(z, zl), zh);
    const float t = 2.f * zc / g.dz;
    w = (t - 0.5f) * wtop + (1.5f - t) * wbot;
    h = (t - 0.5f) * htop + (1.5f - t) * hbot;
    if (z >= zl && z <= zh) {
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
  f.wt = fmaxf(w, wmin);
  f.ht = fmaxf(h, hmin);
  f.omega = fminf(1.f, w / wmin) * fminf(1.f, h / hmin);

  f.cbx = clampi((int)floorf(x * g.inv_wb), 0, g.nx - 1);
  f.cby = clampi((int)floorf(y * g.inv_hb), 0, g.ny - 1);
  const float ox = (float)f.cbx * g.wb, oy = (float)f.cby * g.hb;
  const float rx = x - ox, ry = y - oy;
  f.rx0 = rx - 0.5f * f.wt;
  f.rx1 = rx + 0.5f * f.wt;
  f.ry0 = ry - 0.5f * f.ht;
  f.ry1 = ry + 0.5f * f.ht;
  f.lx0 = fmaxf(f.rx0, -ox);
  f.lx1 = fminf(f.rx1, g.dx - ox);
  f.ly0 = fmaxf(f.ry0, -oy);
  f.ly1 = fminf(f.ry1, g.dy - oy);
  f.rz0 = z - 0.25f * g.dz;
  f.rz1 = z + 0.25f * g.dz;
  f.z0 = fmaxf(f.rz0, 0.f);
  f.z1 = fminf(f.rz1, g.dz);
  f.bx0 = clampi(f.cbx + (int)floorf(f.lx0 * g.inv_wb), 0, g.nx - 1);
  f.bx1 = clampi(f.cbx + (int)ceilf(f.lx1 * g.inv_wb) - 1, 0, g.nx - 1);
  f.by0 = clampi(f.cby + (int)floorf(f.ly0 * g.inv_hb), 0, g.ny - 1);
  f.by1 = clampi(f.cby + (int)ceilf(f.ly1 * g.inv_hb) - 1, 0, g.ny - 1);
  f.bz0 = clampi((int)floorf(f.z0 * g.inv_db), 0, g.nz - 1);
  f.bz1 = clampi((int)ceilf(f.z1 * g.inv_db) - 1, 0, g.nz - 1);
  f.bx1 = max(f.bx1, f.bx0);
  f.by1 = max(f.by1, f.by0);
  f.bz1 = max(f.bz1, f.bz0);
  return f;
}

// overlap lengths of the clipped cuboid with bin b along each axis
__device__ __forceinline__ float len_x(const Geom& g, const Foot& f, int b) {
  const float lo = (float)(b - f.cbx) * g.wb;
  return fmaxf(0.f, fminf(f.lx1, lo + g.wb) - fmaxf(f.lx0, lo));
}
__device__ __forceinline__ float len_y(const Geom& g, const Foot& f, int b) {
  const float lo = (float)(b - f.cby) * g.hb;
  return fmaxf(0.f, fminf(f.ly1, lo + g.hb) - fmaxf(f.ly0, lo));
}
__device__ __forceinline__ float len_z(const Geom& g, const Foot& f, int b) {
  const float lo = (float)b * g.db;
  return fmaxf(0.f, fminf(f.z1, lo + g.db) - fmaxf(f.z0, lo));
}

// bin holding an unclipped edge (or -1 when the region clips that edge)
__device__ __forceinline__ int edge_bin_x(const Geom& g, const Foot& f, float redge, int lo, int hi) {
  const float ox = (float)f.cbx * g.wb;
  if (!(redge > -ox && redge < g.dx - ox)) return -1;
  const int b = f.cbx + (int)floorf(redge * g.inv_wb);
  return (b >= lo && b <= hi) ? b : -1;
}
__device__ __forceinline__ int edge_bin_y(const Geom& g, const Foot& f, float redge, int lo, int hi) {
  const float oy = (float)f.cby * g.hb;
  if (!(redge > -oy && redge < g.dy - oy)) return -1;
  const int b = f.cby + (int)floorf(redge * g.inv_hb);
  return (b >= lo && b <= hi) ? b : -1;
}
__device__ __forceinline__ int edge_bin_z(const Geom& g, float zedge, int lo, int hi) {
  if (!(zedge > 0.f && zedge < g.dz)) return -1;
  const int b = (int)floorf(zedge * g.inv_db);
  return (b >= lo && b <= hi) ? b : -1;
}

__device__ __forceinline__ size_t bin_index(const Geom& g, int bz, int by, int bx) {
  return ((size_t)bz * g.ny + by) * g.nx + bx;
}

// ------------------------------------------------------------------ forward scatter

__global__ void k_density_cells(Geom g, const float* __restrict__ xyz, const float* __restrict__ size,
                                const uint8_t* __restrict__ kind, float* __restrict__ rho) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const uint8_t k = kind[i];
  if (k & (PLACE3D_KIND_MACRO | PLACE3D_KIND_FIXED)) return;
  const Foot f = footprint(g, xyz, size, k, i);
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

// one workgroup per listed instance, sweeping the bins of its cuboid
__global__ void k_density_large(Geom g, const float* __restrict__ xyz, const float* __restrict__ size,
                                const uint8_t* __restrict__ kind, const int32_t* __restrict__ list,
                                float* __restrict__ rho) {
  const int i = list[blockIdx.x];
  const Foot f = footprint(g, xyz, size, kind[i], i);
  const int nbx = f.bx1 - f.bx0 + 1, nby = f.by1 - f.by0 + 1, nbz = f.bz1 - f.bz0 + 1;
  const long long total = (long long)nbx * nby * nbz;
  const float wgt = f.omega / g.vol_bin;
  for (long long t = threadIdx.x; t < total; t += blockDim.x) {
    const int bx = f.bx0 + (int)(t % nbx);
    const long long r = t / nbx;
    const int by = f.by0 + (int)(r % nby);
    const int bz = f.bz0 + (int)(r / nby);
    const float v = len_x(g, f, bx) * len_y(g, f, by) * len_z(g, f, bz) * wgt;
    if (v != 0.f) atomicAdd(rho + bin_index(g, bz, by, bx), v);
  }
}

__global__ void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, long long n4) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n4; t += (long long)gridDim.x * blockDim.x)
    dst[t] = src[t];
}

__global__ void k_fill(float* __restrict__ p, long long n, float v) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
    p[t] = v;
}

__global__ void k_zero_f64(double* __restrict__ p, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0.0;
}

// ------------------------------------------------------------------ field gather

// out_a[i] (+)= scale * omega * sum_b vol(D_i ∩ b) M_a[b] for the three maps
__device__ __forceinline__ void gather3(const Geom& g, const Foot& f, const float* __restrict__ mx,
                                        const float* __restrict__ my, const float* __restrict__ mz,
                                        int bz, int by, int bx, float v, float& sx, float& sy, float& sz) {
  const size_t b = bin_index(g, bz, by, bx);
  sx += v * mx[b];
  sy += v * my[b];
  sz += v * mz[b];
}

__global__ void k_gather_cells(Geom g, const float* __restrict__ xyz, const float* __restrict__ size,
                               const uint8_t* __restrict__ kind, const float* __restrict__ mx,
                               const float* __restrict__ my, const float* __restrict__ mz, float scale,
                               float* __restrict__ grad, int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const uint8_t k = kind[i];
  if ((k & PLACE3D_KIND_MACRO) && !(k & PLACE3D_KIND_FIXED)) return;   // movable macros: k_gather_large
  float sx = 0.f, sy = 0.f, sz = 0.f;
  if (!(k & PLACE3D_KIND_FIXED)) {
    const Foot f = footprint(g, xyz, size, k, i);
    for (int bz = f.bz0; bz <= f.bz1; ++bz) {
      const float lz = len_z(g, f, bz);
      for (int by = f.by0; by <= f.by1; ++by) {
        const float lyz = len_y(g, f, by) * lz;
        for (int bx = f.bx0; bx <= f.bx1; ++bx) {
          const float v = len_x(g, f, bx) * lyz;
          if (v != 0.f) gather3(g, f, mx, my, mz, bz, by, bx, v, sx, sy, sz);
        }
      }
    }
    const float s = scale * f.omega;
    sx *= s; sy *= s; sz *= s;
  }
  const int n = g.n;
  if (accumulate) { grad[i] += sx; grad[n + i] += sy; grad[2 * n + i] += sz; }
  else { grad[i] = sx; grad[n + i] = sy; grad[2 * n + i] = sz; }
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

// one workgroup per macro: gather with a block reduction (fixed macros get 0)
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
  for (long long t = threadIdx.x; t < total; t += blockDim.x) {
    const int bx = f.bx0 + (int)(t % nbx);
    const long long r = t / nbx;
    const int by = f.by0 + (int)(r % nby);
    const int bz = f.bz0 + (int)(r / nby);
    const float v = len_x(g, f, bx) * len_y(g, f, by) * len_z(g, f, bz);
    gather3(g, f, mx, my, mz, bz, by, bx, v, sx, sy, sz);
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

// Face sums of the map for one instance: the derivative of each overlap length with respect to
// an edge is +-1 on the bin holding that edge.  Returns (sx_hi - sx_lo, ...) and, for macros,
// the size-transition terms, all times omega / vol(b).
struct AdjSums { float gx, gy, gz; };

__device__ __forceinline__ AdjSums adjoint_range(const Geom& g, const Foot& f, const float* __restrict__ m,
                                                 long long t0, long long tstep, bool is_macro) {
  // the flattened loop over (bz, by, bx) of the clipped box; each bin collects its own share
  const int ebx_lo = edge_bin_x(g, f, f.rx0, f.bx0, f.bx1), ebx_hi = edge_bin_x(g, f, f.rx1, f.bx0, f.bx1);
  const int eby_lo = edge_bin_y(g, f, f.ry0, f.by0, f.by1), eby_hi = edge_bin_y(g, f, f.ry1, f.by0, f.by1);
  const int ebz_lo = edge_bin_z(g, f.rz0, f.bz0, f.bz1), ebz_hi = edge_bin_z(g, f.rz1, f.bz0, f.bz1);
  const int nbx = f.bx1 - f.bx0 + 1, nby = f.by1 - f.by0 + 1, nbz = f.bz1 - f.bz0 + 1;
  const long long total = (long long)nbx * nby * nbz;
  float xd = 0.f, xs = 0.f, yd = 0.f, ys = 0.f, zd = 0.f, all = 0.f;
  for (long long t = t0; t < total; t += tstep) {
    const int bx = f.bx0 + (int)(t % nbx);
    const long long r = t / nbx;
    const int by = f.by0 + (int)(r % nby);
    const int bz = f.bz0 + (int)(r / nby);
    const float mv = m[bin_index(g, bz, by, bx)];
    const float lx = len_x(g, f, bx), ly = len_y(g, f, by), lz = len_z(g, f, bz);
    const float fxh = (bx == ebx_hi) ? 1.f : 0.f, fxl = (bx == ebx_lo) ? 1.f : 0.f;
    const float fyh = (by == eby_hi) ? 1.f : 0.f, fyl = (by == eby_lo) ? 1.f : 0.f;
    const float fzh = (bz == ebz_hi) ? 1.f : 0.f, fzl = (bz == ebz_lo) ? 1.f : 0.f;
    xd += (fxh - fxl) * ly * lz * mv;
    yd += lx * (fyh - fyl) * lz * mv;
    zd += lx * ly * (fzh - fzl) * mv;
    if (is_macro) {
      xs += (fxh + fxl) * ly * lz * mv;
      ys += lx * (fyh + fyl) * lz * mv;
      all += lx * ly * lz * mv;
    }
  }
  AdjSums a;
  a.gx = f.omega * xd;
  a.gy = f.omega * yd;
  a.gz = f.omega * zd;
  if (is_macro && (f.dw != 0.f || f.dh != 0.f)) {
    const float r2 = 1.41421356237309515f;
    const float wmin = r2 * g.wb, hmin = r2 * g.hb;
    const bool sw = f.w < wmin, sh = f.h < hmin;
    const float fw = fminf(1.f, f.w / wmin), fh = fminf(1.f, f.h / hmin);
    const float domega = (sw ? f.dw / wmin : 0.f) * fh + fw * (sh ? f.dh / hmin : 0.f);
    const float dwt = sw ? 0.f : f.dw, dht = sh ? 0.f : f.dh;
    a.gz += domega * all + f.omega * 0.5f * (dwt * xs + dht * ys);
  }
  return a;
}

__global__ void k_adjoint_cells(Geom g, const float* __restrict__ xyz, const float* __restrict__ size,
                                const uint8_t* __restrict__ kind, const float* __restrict__ m, float scale,
                                float* __restrict__ grad, int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const uint8_t k = kind[i];
  if ((k & PLACE3D_KIND_MACRO) && !(k & PLACE3D_KIND_FIXED)) return;   // movable macros: k_adjoint_large
  AdjSums a = {0.f, 0.f, 0.f};
  if (!(k & PLACE3D_KIND_FIXED)) {
    const Foot f = footprint(g, xyz, size, k, i);
    a = adjoint_range(g, f, m, 0, 1, false);
  }
  const float s = scale / g.vol_bin;
  const int n = g.n;
  if (accumulate) { grad[i] += s * a.gx; grad[n + i] += s * a.gy; grad[2 * n + i] += s * a.gz; }
  else { grad[i] = s * a.gx; grad[n + i] = s * a.gy; grad[2 * n + i] = s * a.gz; }
}

__global__ void k_adjoint_large(Geom g, const float* __restrict__ xyz, const float* __restrict__ size,
                                const uint8_t* __restrict__ kind, const int32_t* __restrict__ list,
                                const float* __restrict__ m, float scale, float* __restrict__ grad,
                                int accumulate) {
  __shared__ float sh[256 / kWave];
  const int i = list[blockIdx.x];
  const Foot f = footprint(g, xyz, size, kind[i], i);
  AdjSums a = adjoint_range(g, f, m, threadIdx.x, blockDim.x, true);
  a.gx = block_sum<256>(a.gx, sh);
  a.gy = block_sum<256>(a.gy, sh);
  a.gz = block_sum<256>(a.gz, sh);
  if (threadIdx.x == 0) {
    const float s = scale / g.vol_bin;
    const int n = g.n;
    if (accumulate) { grad[i] += s * a.gx; grad[n + i] += s * a.gy; grad[2 * n + i] += s * a.gz; }
    else { grad[i] = s * a.gx; grad[n + i] = s * a.gy; grad[2 * n + i] = s * a.gz; }
  }
}

// ------------------------------------------------------------------ overflow

__global__ void k_overflow(Geom g, const float* __restrict__ rho, float target, double* __restrict__ red) {
  __shared__ float sh[256 / kWave];
  const long long plane = (long long)g.nx * g.ny;
  const long long half = plane * (g.nz / 2), total = plane * g.nz;
  float bot = 0.f, top = 0.f;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const float e = fmaxf(rho[t] - target, 0.f);
    if (t < half) bot += e; else top += e;
  }
  bot = block_sum<256>(bot, sh);
  top = block_sum<256>(top, sh);
  if (threadIdx.x == 0) {
    atomicAdd(red + R_EXCESS_BOT, (double)bot * g.vol_bin);
    atomicAdd(red + R_EXCESS_TOP, (double)top * g.vol_bin);
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers

int launch_zero_f64(place3d_ctx* c, double* p, int n, hipStream_t s) {
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

int build_fixed_map(place3d_ctx* c, hipStream_t s) {
  const Geom& g = c->g;
  const long long map = (long long)g.nx * g.ny * g.nz;
  if (int rc = launch_fill_f32(c, c->fixed_map, map, 0.f, s)) return rc;
  if (c->n_fixed > 0) {
    hipLaunchKernelGGL(k_density_large, dim3(c->n_fixed), dim3(256), 0, s, g, c->prob.fixed_xyz,
                       c->prob.size, c->prob.kind, c->fixed_large, c->fixed_map);
    P3D_LAUNCH(c, "k_density_large(fixed)");
  }
  return PLACE3D_OK;
}

int density_forward(place3d_ctx* c, const float* xyz, float* rho, hipStream_t s) {
  const Geom& g = c->g;
  const long long map = (long long)g.nx * g.ny * g.nz;
  if (map % 4 == 0 && (reinterpret_cast<uintptr_t>(rho) & 15) == 0) {
    const unsigned nb = (unsigned)std::min<long long>(blocks_for(map / 4, 256), 8192);
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, s, reinterpret_cast<const float4*>(c->fixed_map),
                       reinterpret_cast<float4*>(rho), map / 4);
    P3D_LAUNCH(c, "k_copy");
  } else {
    P3D_HIP(c, hipMemcpyAsync(rho, c->fixed_map, sizeof(float) * map, hipMemcpyDeviceToDevice, s));
  }
  hipLaunchKernelGGL(k_density_cells, dim3(blocks_for(g.n, 256)), dim3(256), 0, s, g, xyz, c->prob.size,
                     c->prob.kind, rho);
  P3D_LAUNCH(c, "k_density_cells");
  if (c->n_movable_macros > 0) {
    hipLaunchKernelGGL(k_density_large, dim3(c->n_movable_macros), dim3(256), 0, s, g, xyz, c->prob.size,
                       c->prob.kind, c->movable_macros, rho);
    P3D_LAUNCH(c, "k_density_large");
  }
  return PLACE3D_OK;
}

int density_field_gather(place3d_ctx* c, const float* xyz, const float* ex, const float* ey,
                         const float* ez, float scale, float* grad, int accumulate, hipStream_t s) {
  const Geom& g = c->g;
  hipLaunchKernelGGL(k_gather_cells, dim3(blocks_for(g.n, 256)), dim3(256), 0, s, g, xyz, c->prob.size,
                     c->prob.kind, ex, ey, ez, scale, grad, accumulate);
  P3D_LAUNCH(c, "k_gather_cells");
  // macros (movable and fixed) are handled per workgroup; fixed ones get zero
  if (c->n_movable_macros > 0) {
    hipLaunchKernelGGL(k_gather_large, dim3(c->n_movable_macros), dim3(256), 0, s, g, xyz, c->prob.size,
                       c->prob.kind, c->movable_macros, ex, ey, ez, scale, grad, accumulate);
    P3D_LAUNCH(c, "k_gather_large");
  }
  return PLACE3D_OK;
}

int density_adjoint(place3d_ctx* c, const float* xyz, const float* gmap, float scale, float* grad,
                    int accumulate, hipStream_t s) {
  const Geom& g = c->g;
  hipLaunchKernelGGL(k_adjoint_cells, dim3(blocks_for(g.n, 256)), dim3(256), 0, s, g, xyz, c->prob.size,
                     c->prob.kind, gmap, scale, grad, accumulate);
  P3D_LAUNCH(c, "k_adjoint_cells");
  if (c->n_movable_macros > 0) {
    hipLaunchKernelGGL(k_adjoint_large, dim3(c->n_movable_macros), dim3(256), 0, s, g, xyz, c->prob.size,
                       c->prob.kind, c->movable_macros, gmap, scale, grad, accumulate);
    P3D_LAUNCH(c, "k_adjoint_large");
  }
  return PLACE3D_OK;
}

int overflow_reduce(place3d_ctx* c, const float* rho, double* red, hipStream_t s) {
  const Geom& g = c->g;
  const long long map = (long long)g.nx * g.ny * g.nz;
  const unsigned nb = (unsigned)std::min<long long>(blocks_for(map, 256), 2048);
  hipLaunchKernelGGL(k_overflow, dim3(nb), dim3(256), 0, s, g, rho, (float)c->prob.target_density, red);
  P3D_LAUNCH(c, "k_overflow");
  return PLACE3D_OK;
}

}  // namespace p3d
