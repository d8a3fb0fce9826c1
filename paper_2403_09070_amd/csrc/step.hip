// One global-placement iteration: objective gradient, mixed-size preconditioner
// (Eq. improved-precond; the ePlace and ePlace3D forms of Eq. general-precond as options), the
// Lipschitz step estimate and the Nesterov move, with the clamp to the movable region.
//
// The paper inherits its optimiser from ePlace/DREAMPlace without describing it.  The method
// implemented: a_0 = 1, a_{k+1} = (1 + sqrt(4 a_k^2 + 1)) / 2,
//   step = |v_k - v_{k-1}|_2 / |g_k - g_{k-1}|_2   (float64, movable coordinates),
//   u_{k+1} = clamp(v_k - step g_k),  v_{k+1} = clamp(u_{k+1} + (a_k - 1)/a_{k+1} (u_{k+1} - u_k)),
// with g the preconditioned gradient, lambda_0 = |grad W|_1 / |grad U|_1 at the start and
// lambda multiplied by a fixed ratio every step.  Clamp: z to [d_z/4, 3d_z/4], then x and y so
// that the instance, at the size its clamped z gives, stays inside the die.
#include <cmath>

#include "internal.h"

namespace p3d {
namespace {

// an instance's four sizes (bottom w, h, top w, h), loaded together
struct Sizes { float wbot, hbot, wtop, htop; };
__device__ __forceinline__ Sizes sizes_of(const float* __restrict__ size, int n, int i) {
  return {size[i], size[n + i], size[2 * n + i], size[3 * n + i]};
}

__device__ __forceinline__ void inst_wh(const Geom& g, const Sizes& sz, uint8_t kind, float z, float& w, float& h) {
  const float wbot = sz.wbot, hbot = sz.hbot, wtop = sz.wtop, htop = sz.htop;
  if (kind & PLACE3D_KIND_MACRO) {
    const float zc = fminf(fmaxf(z, 0.25f * g.dz), 0.75f * g.dz);
    const float t = 2.f * zc / g.dz;
    w = (t - 0.5f) * wtop + (1.5f - t) * wbot;
    h = (t - 0.5f) * htop + (1.5f - t) * hbot;
  } else {
    const bool top = z > g.half_dz;
    w = top ? wtop : wbot;
    h = top ? htop : hbot;
  }
}
__device__ __forceinline__ void inst_wh(const Geom& g, const float* __restrict__ size, uint8_t kind, int i, float z,
                                        float& w, float& h) {
  inst_wh(g, sizes_of(size, g.n, i), kind, z, w, h);
}

__device__ __forceinline__ void clamp_point(const Geom& g, const Sizes& sz, uint8_t kind, float& x, float& y,
                                            float& z) {
  z = fminf(fmaxf(z, 0.25f * g.dz), 0.75f * g.dz);
  float w, h;
  inst_wh(g, sz, kind, z, w, h);
  x = fminf(fmaxf(x, 0.5f * w), g.dx - 0.5f * w);
  y = fminf(fmaxf(y, 0.5f * h), g.dy - 0.5f * h);
}
__device__ __forceinline__ void clamp_point(const Geom& g, const float* __restrict__ size, uint8_t kind, int i,
                                            float& x, float& y, float& z) {
  clamp_point(g, sizes_of(size, g.n, i), kind, x, y, z);
}

// np: the instance's pin count (read only where the form uses it)
__device__ __forceinline__ float precond(const Geom& g, const Sizes& sz, float np, uint8_t kind, float z, double lam,
                                         int mode) {
  float w, h;
  inst_wh(g, sz, kind, z, w, h);
  const double lq = lam * (double)w * (double)h * (double)(0.5f * g.dz);
  double H;
  if (mode == PLACE3D_PRECOND_MIXED)
    H = (kind & PLACE3D_KIND_MACRO) ? fmax(1.0, (double)np + lq) : fmax(1.0, lq);
  else if (mode == PLACE3D_PRECOND_EPLACE)
    H = (double)np + lq;
  else
    H = lq;
  return (float)H;
}

// per-block partial sums: part[(slot0 + q) * stride + blockIdx.x]
template <int NQ>
__device__ __forceinline__ void block_partials(double (&v)[NQ], double* __restrict__ part, int stride, int slot0) {
  __shared__ double sh[NQ][256 / kWave];
  for (int q = 0; q < NQ; ++q) {
    double x = v[q];
    for (int m = kWave / 2; m > 0; m >>= 1) x += __shfl_xor(x, m);
    if ((threadIdx.x & (kWave - 1)) == 0) sh[q][threadIdx.x / kWave] = x;
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    double x = 0.0;
    for (int w = 0; w < 256 / kWave; ++w) x += sh[threadIdx.x][w];
    part[(size_t)(slot0 + threadIdx.x) * stride + blockIdx.x] = x;
  }
}

// u = v = clamp(xyz0)
__global__ void k_clamp_copy(Geom g, const float* __restrict__ size, const uint8_t* __restrict__ kind,
                             const float* __restrict__ src, float* __restrict__ u, float* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int n = g.n;
  float x = src[i], y = src[n + i], z = src[2 * n + i];
  if (!(kind[i] & PLACE3D_KIND_FIXED)) clamp_point(g, size, kind[i], i, x, y, z);
  u[i] = x; u[n + i] = y; u[2 * n + i] = z;
  if (v) { v[i] = x; v[n + i] = y; v[2 * n + i] = z; }
}

// L1 norms of the wirelength and density gradients over movable instances -> lambda_0 (the z
// components of z-held instances count as zero)
__global__ void k_l1_parts(Geom g, const uint8_t* __restrict__ kind, const float* __restrict__ gw,
                           const float* __restrict__ gd, double* __restrict__ part, int stride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = g.n;
  double v[2] = {0.0, 0.0};
  if (i < n && !(kind[i] & PLACE3D_KIND_FIXED)) {
    const int na = (kind[i] & PLACE3D_KIND_ZFIXED) ? 2 : 3;    // a held z has no gradient
    for (int a = 0; a < na; ++a) {
      v[0] += fabs((double)gw[a * n + i]);
      v[1] += fabs((double)gd[a * n + i]);
    }
  }
  block_partials<2>(v, part, stride, R_L1_WL);
}

// g = (gw + lambda gd) / H.  Mode 0 (init): write g to `gout` and track max|g|.  Mode 1 (step):
// accumulate |v - v_prev|^2 and |g - g_prev|^2, store g over g_prev, and the movable charge
// per die without fillers (overflow denominators).  A z-held instance's z-gradient is zero.
// Cell density gradients held as per-(cell, tile) shares (CellShares.entry != nullptr, cell-major
// [q][n], q < the cell's entry count read from its packed tile range) are summed here, in the
// order the separate combine pass uses, instead of being materialised first.
struct CellShares {
  const uint8_t* cls;
  const int32_t* cell_entry;
  const float4* entry;
  float scale;
};

// cls and packed: the instance's density class and packed tile range (loaded by the caller with
// its other operands); a cell's up to four shares are loaded together and summed in q order
__device__ __forceinline__ void density_grad_of(const CellShares& cs, const float* __restrict__ gd, int n, int i,
                                                uint8_t cls, int packed, float (&d)[3]) {
  if (!cs.entry || cls == kClsLarge) {
    for (int a = 0; a < 3; ++a) d[a] = gd[a * n + i];
    return;
  }
  float sx = 0.f, sy = 0.f, sz = 0.f;
  if (cls == kClsCell) {
    // the cell's entry count from its packed tile range; its shares are cell-major [q][n]
    // (a bucketed cell has 1, 2 or 4 entries: its tile range is 1 or 2 tiles per axis)
    const int cnt = packed < 0 ? 0 : (1 + ((packed >> 24) & 1)) * (1 + ((packed >> 25) & 1));
    // All four loads are issued together: an absent share's load re-reads share 0 (the same
    // cache line) and counts as zero, which leaves the sum in q order unchanged.
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const size_t i1 = cnt > 1 ? (size_t)n + i : (size_t)i;
    const size_t i2 = cnt > 2 ? 2 * (size_t)n + i : (size_t)i, i3 = cnt > 2 ? 3 * (size_t)n + i : (size_t)i;
    const float4 r0 = cs.entry[i], r1 = cs.entry[i1], r2 = cs.entry[i2], r3 = cs.entry[i3];
    const float4 v0 = r0, v1 = cnt > 1 ? r1 : z4, v2 = cnt > 2 ? r2 : z4, v3 = cnt > 2 ? r3 : z4;
    if (cnt > 0) {
      sx = ((v0.x + v1.x) + v2.x) + v3.x;
      sy = ((v0.y + v1.y) + v2.y) + v3.y;
      sz = ((v0.z + v1.z) + v2.z) + v3.z;
    }
    sx *= cs.scale; sy *= cs.scale; sz *= cs.scale;
  }
  d[0] = sx; d[1] = sy; d[2] = sz;
}

__global__ void k_combine(Geom g, const float* __restrict__ size, const uint8_t* __restrict__ kind,
                          const float* __restrict__ npins, const float* __restrict__ v,
                          const float* __restrict__ v_prev, const float* __restrict__ gw,
                          const float* __restrict__ gd, CellShares cs, const double* __restrict__ lam_ptr, int lam_slot,
                          int mode_pre, int mode, float* __restrict__ gout, double* __restrict__ part, int stride,
                          const double* __restrict__ a_src, double* __restrict__ a_copy) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = g.n;
  const double lam = lam_ptr[lam_slot];
  // the step's Nesterov coefficient a_k, copied where the move reads it, so that the move can
  // update the scalars while its other workgroups still run
  if (a_copy && i == 0) *a_copy = *a_src;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < n) {
    // the instance's operands are all loaded before any is used (one round of loads in flight,
    // then the cell's shares), whatever its kind
    const uint8_t k = kind[i];
    const Sizes sz = sizes_of(size, n, i);
    float wv[3], vv[3], vp[3] = {0.f, 0.f, 0.f}, go[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      wv[a] = gw[a * n + i];
      vv[a] = v[a * n + i];
    }
    if (mode == 1) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        vp[a] = v_prev[a * n + i];
        go[a] = gout[a * n + i];
      }
    }
    const uint8_t dcls = cs.entry ? cs.cls[i] : kClsLarge;
    const int packed = cs.entry ? cs.cell_entry[i] : -1;
    float gv[3] = {0.f, 0.f, 0.f};
    const float z = vv[2];
    if (!(k & PLACE3D_KIND_FIXED)) {
      const bool need_np = mode_pre == PLACE3D_PRECOND_EPLACE || (mode_pre == PLACE3D_PRECOND_MIXED && (k & PLACE3D_KIND_MACRO));
      const float H = precond(g, sz, need_np ? npins[i] : 0.f, k, z, lam, mode_pre);
      float d[3];
      density_grad_of(cs, gd, n, i, dcls, packed, d);
      for (int a = 0; a < 3; ++a)
        gv[a] = (float)(((double)wv[a] + lam * (double)d[a]) / (double)H);
      if (k & PLACE3D_KIND_ZFIXED) gv[2] = 0.f;               // z held (z-fixed fillers)
      if (mode == 1) {
        for (int a = 0; a < 3; ++a) {
          const double dv = (double)vv[a] - (double)vp[a];
          const double dg = (double)gv[a] - (double)go[a];
          acc[0] += dv * dv;
          acc[1] += dg * dg;
        }
        float w, h;
        inst_wh(g, sz, k, z, w, h);
        const double q = (k & PLACE3D_KIND_FILLER) ? 0.0 : (double)w * (double)h * (double)(0.5f * g.dz);
        if (z > g.half_dz) acc[3] += q; else acc[2] += q;
      } else {
        acc[0] = fmax(fmax(fabs((double)gv[0]), fabs((double)gv[1])), fabs((double)gv[2]));
      }
    }
    for (int a = 0; a < 3; ++a) gout[a * n + i] = gv[a];
  }
  if (mode == 1) {
    block_partials<4>(acc, part, stride, R_DV2);   // R_DV2, R_DG2, R_Q_BOT, R_Q_TOP
  } else {
    __shared__ double shm[256 / kWave];
    double m = acc[0];
    for (int o = kWave / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & (kWave - 1)) == 0) shm[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = 0.0;
      for (int w = 0; w < 256 / kWave; ++w) r = fmax(r, shm[w]);
      part[(size_t)R_GMAX * stride + blockIdx.x] = r;
    }
  }
}

// v_prev = clamp(v - 0.01 w_b g / max|g|)
__global__ void k_bootstrap(Geom g, const float* __restrict__ size, const uint8_t* __restrict__ kind,
                            const float* __restrict__ v, const float* __restrict__ g0, const double* __restrict__ red,
                            float* __restrict__ v_prev) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int n = g.n;
  const double gmax = red[R_GMAX];
  const float f = gmax > 0.0 ? (float)(0.01 * (double)g.wb / gmax) : 0.f;
  float x = v[i], y = v[n + i], z = v[2 * n + i];
  if (!(kind[i] & PLACE3D_KIND_FIXED)) {
    x -= f * g0[i]; y -= f * g0[n + i]; z -= f * g0[2 * n + i];
    clamp_point(g, size, kind[i], i, x, y, z);
  }
  v_prev[i] = x; v_prev[n + i] = y; v_prev[2 * n + i] = z;
}

__global__ void k_init_scalars(double* __restrict__ sc, const double* __restrict__ red) {
  if (threadIdx.x != 0) return;
  for (int q = 0; q < PLACE3D_NSCALARS; ++q) sc[q] = 0.0;
  sc[PLACE3D_S_A] = 1.0;
  sc[PLACE3D_S_LAMBDA] = red[R_L1_DEN] > 0.0 ? red[R_L1_WL] / red[R_L1_DEN] : 0.0;
  // the start's norms non-finite: flagged as iteration 0
  if (!isfinite(red[R_L1_WL]) || !isfinite(red[R_L1_DEN]) || !isfinite(sc[PLACE3D_S_LAMBDA]))
    sc[PLACE3D_S_NONFINITE] = 1.0;
}

// The step's scalars: step size, a_{k+1}, lambda ramp, iteration, overflow, energy, wirelength
// metrics and the non-finite flag, from the reductions (all complete before the move starts) and
// a = a_k.  Run by one thread of the move.
__device__ void finish_scalars(double* __restrict__ sc, const double* __restrict__ red, double ramp, double a) {
  const double dv2 = red[R_DV2], dg2 = red[R_DG2];
  sc[PLACE3D_S_STEP] = dg2 > 0.0 ? sqrt(dv2 / dg2) : 0.0;
  sc[PLACE3D_S_A] = 0.5 * (1.0 + sqrt(4.0 * a * a + 1.0));
  sc[PLACE3D_S_LAMBDA] *= ramp;
  sc[PLACE3D_S_ITER] += 1.0;
  sc[PLACE3D_S_OVFL_BOT] = red[R_Q_BOT] > 0.0 ? red[R_EXCESS_BOT] / red[R_Q_BOT] : 0.0;
  sc[PLACE3D_S_OVFL_TOP] = red[R_Q_TOP] > 0.0 ? red[R_EXCESS_TOP] / red[R_Q_TOP] : 0.0;
  sc[PLACE3D_S_ENERGY] = red[R_ENERGY];
  for (int q = 0; q <= PLACE3D_M_NORM_FDA; ++q) sc[PLACE3D_S_WL + q] = red[R_WA_BI + q];
  const double nf = red[R_NORM_FDA];
  sc[PLACE3D_S_WL + PLACE3D_M_FDA_SCALE] = nf > 0.0 ? (red[R_NORM_X] + red[R_NORM_Y]) / (2.0 * nf) : 0.0;
  // the step's float64 reductions: any NaN or infinity in a position, a gradient or a map shows in
  // one of them; the first iteration that saw one is kept (1 + its index)
  bool finite = isfinite(dv2) && isfinite(dg2) && isfinite(sc[PLACE3D_S_LAMBDA]) && isfinite(red[R_EXCESS_BOT]) &&
                isfinite(red[R_EXCESS_TOP]) && isfinite(red[R_ENERGY]);
  for (int q = R_WA_BI; q <= R_NORM_FDA; ++q) finite = finite && isfinite(red[q]);
  if (!finite && sc[PLACE3D_S_NONFINITE] == 0.0) sc[PLACE3D_S_NONFINITE] = sc[PLACE3D_S_ITER];
}

// the Nesterov move; g (the new preconditioned gradient) sits in g_prev
__global__ void k_nesterov(Geom g, const float* __restrict__ size, const uint8_t* __restrict__ kind,
                           double* __restrict__ sc, const double* __restrict__ red, double ramp,
                           float* __restrict__ u, float* __restrict__ v, float* __restrict__ v_prev,
                           const float* __restrict__ gk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  // a_k from the combine's copy: thread 0 writes a_{k+1} (and the other scalars) meanwhile
  const double a = red[R_A_PREV];
  if (i == 0) finish_scalars(sc, red, ramp, a);
  if (i >= g.n) return;
  const int n = g.n;
  const double dv2 = red[R_DV2], dg2 = red[R_DG2];
  const double step = dg2 > 0.0 ? sqrt(dv2 / dg2) : 0.0;
  const double a1 = 0.5 * (1.0 + sqrt(4.0 * a * a + 1.0));
  const float coef = (float)((a - 1.0) / a1);
  const float st = (float)step;
  // every operand loaded before any is used
  const uint8_t kd = kind[i];
  const float vx = v[i], vy = v[n + i], vz = v[2 * n + i];
  const float gx = gk[i], gy = gk[n + i], gz = gk[2 * n + i];
  const float ox = u[i], oy = u[n + i], oz = u[2 * n + i];
  const Sizes sz = sizes_of(size, n, i);
  // the move is computed for every instance (a fixed one's is not stored), so that no load waits
  // behind the branch
  float ux = vx - st * gx, uy = vy - st * gy, uz = vz - st * gz;
  clamp_point(g, sz, kd, ux, uy, uz);
  float nx = ux + coef * (ux - ox), ny = uy + coef * (uy - oy), nz = uz + coef * (uz - oz);
  clamp_point(g, sz, kd, nx, ny, nz);
  v_prev[i] = vx; v_prev[n + i] = vy; v_prev[2 * n + i] = vz;
  if (kd & PLACE3D_KIND_FIXED) return;
  u[i] = ux; u[n + i] = uy; u[2 * n + i] = uz;
  v[i] = nx; v[n + i] = ny; v[2 * n + i] = nz;
}


// wirelength and density gradients at xyz into gw and gd (both [3][n]); reductions into red.
// The cells are bucketed once and the buckets serve the density map and its gradient.
// cells_in_combine: leave the cells' density-gradient shares for k_combine to sum
// defer_excess: leave the overflow slots' partials for the caller's final reduction
int eval_parts(place3d_ctx* c, const float* xyz, float* gw, float* gd, double* red, hipStream_t s,
               bool cells_in_combine = false, bool defer_excess = false) {
  int rc;
  // every reduction slot read after an evaluation is written by it (the energy slot, read only
  // for the scalars, stays as gp_init zeroed it in the field-gather form)
  if ((rc = bucket_cells(c, xyz, s, 1))) return rc;  // the count pass packs xyz for the wirelength sweep
  // fork: the wirelength sweep (its own reduction slots, pin and instance scratch) runs on the
  // side stream while the bucketing, density, spectral and gather chain runs on s; joined below.
  // With the float32 contractions (2.6 times as long as the split ones) the sweep forks after
  // the scatter pass, which then runs alone, and overlaps the contractions; with the split ones
  // it forks right after the count pass, so that it is mostly done before they start.
  const bool fork_after_scatter = !c->sc.on;
  if (fork_after_scatter && (rc = bucket_cells(c, xyz, s, 2))) return rc;
  P3D_HIP(c, hipEventRecord(c->ev_fork, s));
  P3D_HIP(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
  if ((rc = wirelength_eval(c, xyz, gw, 0, red, nullptr, c->side, true))) return rc;
  P3D_HIP(c, hipEventRecord(c->ev_join, c->side));
  if (!fork_after_scatter && (rc = bucket_cells(c, xyz, s, 2))) return rc;
  if ((rc = density_tiles(c, xyz, c->rho, red, s, !defer_excess))) return rc;
  if (c->prob.dgrad == PLACE3D_DGRAD_FIELD) {
    // the float32 form's field stays x-folded for the gather, which unfolds it while staging its
    // tiles (the split-bf16 chain returns it unfolded)
    if ((rc = spectral_field(c, c->rho, nullptr, c->ex, c->ey, c->ez, nullptr, s, large_in_tiles(c)))) return rc;
    if ((rc = gather_bucketed(c, xyz, c->ex, c->ey, c->ez, -1.f, gd, 0, s, !cells_in_combine, c->field_xfold != 0)))
      return rc;
  } else {
    if ((rc = spectral_field(c, c->rho, c->phi, nullptr, nullptr, nullptr, red + R_ENERGY, s))) return rc;
    if ((rc = adjoint_bucketed(c, xyz, c->phi, c->g.vol_bin, gd, 0, s, !cells_in_combine))) return rc;
  }
  P3D_HIP(c, hipStreamWaitEvent(s, c->ev_join, 0));
  return PLACE3D_OK;
}

int check_state(place3d_ctx* c, const place3d_state* st) {
  if (!st || !st->u || !st->v || !st->v_prev || !st->g_prev || !st->scalars)
    return set_err(c, PLACE3D_ERR_ARG, "state has a NULL array");
  if ((reinterpret_cast<uintptr_t>(st->u) | reinterpret_cast<uintptr_t>(st->v) |
       reinterpret_cast<uintptr_t>(st->v_prev) | reinterpret_cast<uintptr_t>(st->g_prev)) & 3 ||
      (reinterpret_cast<uintptr_t>(st->scalars) & 7))
    return set_err(c, PLACE3D_ERR_ARG, "misaligned state array");
  return PLACE3D_OK;
}

}  // namespace
}  // namespace p3d

using namespace p3d;

extern "C" int32_t place3d_gp_init(place3d_ctx* c, place3d_state* st, const float* xyz0, void* stream) {
  if (!c) return PLACE3D_ERR_ARG;
  if (int rc = check_state(c, st)) return rc;
  if (!xyz0 || (reinterpret_cast<uintptr_t>(xyz0) & 3)) return set_err(c, PLACE3D_ERR_ARG, "xyz0 NULL or misaligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const Geom& g = c->g;
  const place3d_problem& p = c->prob;
  const unsigned nb = blocks_for(g.n, 256);
  int rc;
  {
    ProfScope prof_(c, PLACE3D_STAGE_UPDATE, s);
    hipLaunchKernelGGL(k_clamp_copy, dim3(nb), dim3(256), 0, s, g, p.size, p.kind, xyz0, st->u, st->v);
    P3D_LAUNCH(c, "k_clamp_copy");
  }
  // gradients at v0, lambda_0
  if ((rc = launch_zero_f64(c, c->red, R_COUNT, s))) return rc;
  if ((rc = eval_parts(c, st->v, c->gw, c->den_grad, c->red, s))) return rc;
  {
    ProfScope prof_(c, PLACE3D_STAGE_UPDATE, s);
    hipLaunchKernelGGL(k_l1_parts, dim3(nb), dim3(256), 0, s, g, p.kind, c->gw, c->den_grad, c->part, c->part_stride);
    P3D_LAUNCH(c, "k_l1_parts");
  }
  if ((rc = reduce_final(c, R_L1_WL, 2, (int)nb, false, c->red2 + R_L1_WL, s))) return rc;
  {
    ProfScope prof_(c, PLACE3D_STAGE_UPDATE, s);
    hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(64), 0, s, st->scalars, c->red2);
    P3D_LAUNCH(c, "k_init_scalars");
  }
  // g0 (into g_prev as scratch) and max|g0|
  {
    ProfScope prof_(c, PLACE3D_STAGE_UPDATE, s);
    hipLaunchKernelGGL(k_combine, dim3(nb), dim3(256), 0, s, g, p.size, p.kind, c->npins, st->v, st->v_prev,
                     c->gw, c->den_grad, CellShares{}, st->scalars, (int)PLACE3D_S_LAMBDA, p.precond, 0, st->g_prev,
                     c->part, c->part_stride, nullptr, nullptr);
    P3D_LAUNCH(c, "k_combine(init)");
  }
  if ((rc = reduce_final(c, R_GMAX, 1, (int)nb, true, c->red2 + R_GMAX, s))) return rc;
  {
    ProfScope prof_(c, PLACE3D_STAGE_UPDATE, s);
    hipLaunchKernelGGL(k_bootstrap, dim3(nb), dim3(256), 0, s, g, p.size, p.kind, st->v, st->g_prev, c->red2,
                     st->v_prev);
    P3D_LAUNCH(c, "k_bootstrap");
  }
  // preconditioned gradient at v_prev
  if ((rc = eval_parts(c, st->v_prev, c->gw, c->den_grad, c->red, s))) return rc;
  {
    ProfScope prof_(c, PLACE3D_STAGE_UPDATE, s);
    hipLaunchKernelGGL(k_combine, dim3(nb), dim3(256), 0, s, g, p.size, p.kind, c->npins, st->v_prev, st->v_prev,
                     c->gw, c->den_grad, CellShares{}, st->scalars, (int)PLACE3D_S_LAMBDA, p.precond, 0, st->g_prev,
                     c->part, c->part_stride, nullptr, nullptr);
    P3D_LAUNCH(c, "k_combine(init2)");
  }
  return PLACE3D_OK;
}

extern "C" int32_t place3d_step(place3d_ctx* c, place3d_state* st, void* stream) {
  if (!c) return PLACE3D_ERR_ARG;
  if (int rc = check_state(c, st)) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const Geom& g = c->g;
  const place3d_problem& p = c->prob;
  const unsigned nb = blocks_for(g.n, 256);
  int rc;
  if ((rc = eval_parts(c, st->v, c->gw, c->den_grad, c->red, s, true, true))) return rc;
  {
    ProfScope prof_(c, PLACE3D_STAGE_UPDATE, s);
    const CellShares cs{c->cls, c->cell_entry, c->entry_out, c->cell_scale};
    hipLaunchKernelGGL(k_combine, dim3(nb), dim3(256), 0, s, g, p.size, p.kind, c->npins, st->v, st->v_prev,
                     c->gw, c->den_grad, cs, st->scalars, (int)PLACE3D_S_LAMBDA, p.precond, 1, st->g_prev,
                     c->part, c->part_stride, st->scalars + PLACE3D_S_A, c->red + R_A_PREV);
    P3D_LAUNCH(c, "k_combine");
  }
  // the step's partials and the density pass's overflow partials, in one launch
  if ((rc = reduce_final2(c, R_DV2, 4, (int)nb, c->red + R_DV2, R_EXCESS_BOT, 2, c->tg.ntiles, c->red + R_EXCESS_BOT,
                          s)))
    return rc;
  {
    // the move, and the step's scalars from its first thread
    ProfScope prof_(c, PLACE3D_STAGE_UPDATE, s);
    hipLaunchKernelGGL(k_nesterov, dim3(nb), dim3(256), 0, s, g, p.size, p.kind, st->scalars, c->red, p.lambda_ramp,
                     st->u, st->v, st->v_prev, st->g_prev);
    P3D_LAUNCH(c, "k_nesterov");
  }
  return PLACE3D_OK;
}
