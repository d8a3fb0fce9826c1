// Bistratal weighted-average wirelength, its gradient and the FDA z-gradient
// (Sec. III-A: Eqs. wa-model-approx, optimal-region, wl-obj, wl-model, fda-grad, fda-normalize;
// Sec. IV-B: incremental evaluation from first and second extremes).
//
// Work split: nets are processed by lane groups of G = 2..64 lanes inside a wavefront (G the
// smallest power of two >= the degree, 64 for larger nets, which then loop).  A static schedule
// built at context creation orders nets by G, so a workgroup holds groups of one size.  Each lane
// takes the pins k = lane, lane + G, ...; per-group reductions are xor butterflies.
//
// Per net and axis the group reduces, for the top set e+ and the bottom set e-, the first and
// second largest and smallest pin coordinates (Sec. IV-B) and max-shifted exponential sums for
// the WA model.  Whole-net sums are the two partial sums rescaled to the whole-net shift.
//   p^_S = (M_S + t+_S/s+_S) - (m_S + t-_S/s-_S)  with t+ = sum (u - M) e^{(u - M)/gamma}
//   W^_u = max{p^_e, p^_e+ + p^_e-} for a net crossing the dies, else p^_e
//   W_u  = max{p_e, p_e+ + p_e-}  (exact, the FDA and HPWL metric)
// Each pin then writes its share of the gradient of the chosen branch, its WA z-gradient and
// (4/d_z)(W_Bi(owner on top) - W_Bi(owner on bottom)) evaluated in O(1) from the extremes: the
// pin leaves its set (the second extreme replaces it when it was the first) and joins the other
// set at its other-die offset.
//
// Pin coordinates x + o are carried as an exact float pair (hi, lo) so that differences between
// nearby pins keep full precision even at large absolute coordinates.
#include "internal.h"

namespace p3d {
namespace {

struct DF { float h, l; };   // exact value h + l

__device__ __forceinline__ DF two_sum(float a, float b) {
  const float s = a + b;
  const float bb = s - a;
  const float err = (a - (s - bb)) + (b - bb);
  return {s, err};
}
__device__ __forceinline__ float dsub(DF a, DF b) { return (a.h - b.h) + (a.l - b.l); }
__device__ __forceinline__ bool dgt(DF a, DF b) { return a.h > b.h || (a.h == b.h && a.l > b.l); }
__device__ __forceinline__ bool deq(DF a, DF b) { return a.h == b.h && a.l == b.l; }

constexpr float kNegInf = -__builtin_huge_valf();
constexpr float kPosInf = __builtin_huge_valf();

// first and second largest of a multiset (duplicates kept); "min" versions store the smallest
struct Top2 { DF a1, a2; };
__device__ __forceinline__ Top2 top2_empty_max() { return {{kNegInf, 0.f}, {kNegInf, 0.f}}; }
__device__ __forceinline__ Top2 top2_empty_min() { return {{kPosInf, 0.f}, {kPosInf, 0.f}}; }
__device__ __forceinline__ void top2_put_max(Top2& t, DF v) {
  if (dgt(v, t.a1)) { t.a2 = t.a1; t.a1 = v; }
  else if (dgt(v, t.a2)) { t.a2 = v; }
}
__device__ __forceinline__ void top2_put_min(Top2& t, DF v) {
  if (dgt(t.a1, v)) { t.a2 = t.a1; t.a1 = v; }
  else if (dgt(t.a2, v)) { t.a2 = v; }
}
__device__ __forceinline__ DF shfl(DF v, int m) { return {__shfl_xor(v.h, m), __shfl_xor(v.l, m)}; }
__device__ __forceinline__ void top2_merge_max(Top2& t, int m) {
  Top2 o = {shfl(t.a1, m), shfl(t.a2, m)};
  const DF hi = dgt(o.a1, t.a1) ? o.a1 : t.a1;
  const DF lo = dgt(o.a1, t.a1) ? t.a1 : o.a1;     // the smaller of the two firsts
  const DF s2 = dgt(o.a2, t.a2) ? o.a2 : t.a2;
  t.a1 = hi;
  t.a2 = dgt(lo, s2) ? lo : s2;
}
__device__ __forceinline__ void top2_merge_min(Top2& t, int m) {
  Top2 o = {shfl(t.a1, m), shfl(t.a2, m)};
  const DF lo = dgt(t.a1, o.a1) ? o.a1 : t.a1;
  const DF hi = dgt(t.a1, o.a1) ? t.a1 : o.a1;
  const DF s2 = dgt(t.a2, o.a2) ? o.a2 : t.a2;
  t.a1 = lo;
  t.a2 = dgt(s2, hi) ? hi : s2;
}

struct Ext {           // extremes of one set along one axis
  Top2 mx, mn;
};

struct SetSums {       // max/min-shifted exponential sums of one set along one axis
  float sp, tp, sm, tm;
};

struct PinData {
  DF ux, uy;           // position on the current die
  DF fx, fy;           // position on the other die
  float z;
  bool top;
  int node;
};

__device__ __forceinline__ PinData load_pin(const float* __restrict__ xyz, int n, const int32_t* __restrict__ pin_node,
                                            const float4* __restrict__ off, int slot, float half_dz) {
  PinData p;
  p.node = pin_node[slot];
  const float4 o = off[slot];
  const float x = xyz[p.node], y = xyz[n + p.node];
  p.z = xyz[2 * n + p.node];
  p.top = p.z > half_dz;
  p.ux = two_sum(x, p.top ? o.z : o.x);
  p.uy = two_sum(y, p.top ? o.w : o.y);
  p.fx = two_sum(x, p.top ? o.x : o.z);
  p.fy = two_sum(y, p.top ? o.y : o.w);
  return p;
}

// exact minimal D2D wirelength along one axis from the first extremes of the two sets
__device__ __forceinline__ float bistratal_exact(DF tmax, DF tmin, int ct, DF bmax, DF bmin, int cb) {
  const float pt = ct > 0 ? dsub(tmax, tmin) : 0.f;
  const float pb = cb > 0 ? dsub(bmax, bmin) : 0.f;
  DF wmax, wmin;
  if (ct > 0 && cb > 0) {
    wmax = dgt(tmax, bmax) ? tmax : bmax;
    wmin = dgt(tmin, bmin) ? bmin : tmin;
  } else if (ct > 0) { wmax = tmax; wmin = tmin; }
  else { wmax = bmax; wmin = bmin; }
  const float pe = (ct + cb) > 0 ? dsub(wmax, wmin) : 0.f;
  return fmaxf(pe, pt + pb);
}

// W along one axis with one pin moved from its set S to the other set O at position f
__device__ __forceinline__ float bistratal_flip(const Ext& S, int cs, const Ext& O, int co, DF u, DF f) {
  DF smax = S.mx.a1, smin = S.mn.a1;
  if (deq(u, smax)) smax = S.mx.a2;
  if (deq(u, smin)) smin = S.mn.a2;
  const int cs2 = cs - 1;
  DF omax = O.mx.a1, omin = O.mn.a1;
  if (co == 0) { omax = f; omin = f; }
  else {
    if (dgt(f, omax)) omax = f;
    if (dgt(omin, f)) omin = f;
  }
  return bistratal_exact(smax, smin, cs2, omax, omin, co + 1);
}

struct AxisWA {        // smoothed WA pieces along one axis, for the gradient of the chosen branch
  float Mt, At_p, st_p, mt, At_m, st_m;   // top set: shift and (A - shift) terms
  float Mb, Ab_p, sb_p, mb, Ab_m, sb_m;   // bottom set
  float Me, Ae_p, se_p, me, Ae_m, se_m;   // whole net
  bool split;
  float W;                                  // smoothed value
};

// Combine partial sums into the WA extents.  Shifts are the hi parts of the first extremes;
// A+_S = t+_S / s+_S is the weighted mean of (u - M_S) (<= 0).
__device__ __forceinline__ AxisWA axis_wa(const Ext& T, const SetSums& st, int ct, const Ext& B, const SetSums& sb,
                                          int cb, float inv_gamma) {
  AxisWA a;
  a.Mt = T.mx.a1.h; a.mt = T.mn.a1.h; a.Mb = B.mx.a1.h; a.mb = B.mn.a1.h;
  a.st_p = st.sp; a.st_m = st.sm; a.sb_p = sb.sp; a.sb_m = sb.sm;
  a.At_p = ct > 0 ? st.tp / st.sp : 0.f;
  a.At_m = ct > 0 ? st.tm / st.sm : 0.f;
  a.Ab_p = cb > 0 ? sb.tp / sb.sp : 0.f;
  a.Ab_m = cb > 0 ? sb.tm / sb.sm : 0.f;
  const float pt = ct > 0 ? (a.Mt - a.mt) + (a.At_p - a.At_m) : 0.f;
  const float pb = cb > 0 ? (a.Mb - a.mb) + (a.Ab_p - a.Ab_m) : 0.f;
  // whole net: rescale the partial sums to the whole-net shifts
  if (ct > 0 && cb > 0) {
    a.Me = fmaxf(a.Mt, a.Mb);
    a.me = fminf(a.mt, a.mb);
    const float dt = a.Mt - a.Me, db = a.Mb - a.Me;                 // <= 0
    const float rt = __expf(dt * inv_gamma), rb = __expf(db * inv_gamma);
    a.se_p = st.sp * rt + sb.sp * rb;
    const float te_p = rt * (st.tp + dt * st.sp) + rb * (sb.tp + db * sb.sp);
    const float dtm = a.mt - a.me, dbm = a.mb - a.me;              // >= 0
    const float qt = __expf(-dtm * inv_gamma), qb = __expf(-dbm * inv_gamma);
    a.se_m = st.sm * qt + sb.sm * qb;
    const float te_m = qt * (st.tm + dtm * st.sm) + qb * (sb.tm + dbm * sb.sm);
    a.Ae_p = te_p / a.se_p;
    a.Ae_m = te_m / a.se_m;
  } else if (ct > 0) {
    a.Me = a.Mt; a.me = a.mt; a.se_p = st.sp; a.se_m = st.sm; a.Ae_p = a.At_p; a.Ae_m = a.At_m;
  } else {
    a.Me = a.Mb; a.me = a.mb; a.se_p = sb.sp; a.se_m = sb.sm; a.Ae_p = a.Ab_p; a.Ae_m = a.Ab_m;
  }
  const float pe = (a.Me - a.me) + (a.Ae_p - a.Ae_m);
  a.split = (ct > 0 && cb > 0) && (pt + pb > pe);
  a.W = a.split ? pt + pb : pe;
  return a;
}

// d W^ / d u for one pin of the chosen branch
__device__ __forceinline__ float axis_grad(const AxisWA& a, DF u, bool top, float inv_gamma) {
  float M, Ap, sp, m, Am, sm;
  if (!a.split) { M = a.Me; Ap = a.Ae_p; sp = a.se_p; m = a.me; Am = a.Ae_m; sm = a.se_m; }
  else if (top) { M = a.Mt; Ap = a.At_p; sp = a.st_p; m = a.mt; Am = a.At_m; sm = a.st_m; }
  else { M = a.Mb; Ap = a.Ab_p; sp = a.sb_p; m = a.mb; Am = a.Ab_m; sm = a.sb_m; }
  const float du = (u.h - M) + u.l;       // u - M  (<= 0)
  const float dl = (u.h - m) + u.l;       // u - m  (>= 0)
  const float ep = __expf(du * inv_gamma), em = __expf(-dl * inv_gamma);
  return ep / sp * (1.f + (du - Ap) * inv_gamma) - em / sm * (1.f - (dl - Am) * inv_gamma);
}

__global__ __launch_bounds__(kWaBlock) void k_wl_nets(
    int n, float half_dz, float four_over_dz, float gamma, float alpha, const float* __restrict__ xyz,
    const int32_t* __restrict__ s_net_start, const int32_t* __restrict__ pin_node, const float4* __restrict__ off,
    float4* __restrict__ pin_out, ClassTab tab, double* __restrict__ part, int stride) {
  __shared__ double shred[5][kWaBlock / kWave];
  __shared__ int cls_s;
  if (threadIdx.x == 0) {
    int c = 0;
    while (c + 1 < kNumClasses && (int)blockIdx.x >= tab.block_begin[c + 1]) ++c;
    cls_s = c;
  }
  __syncthreads();
  const int cls = cls_s;
  const int G = 2 << cls;
  const int lane = threadIdx.x & (G - 1);
  const int group = threadIdx.x / G;
  const int net = tab.net_begin[cls] + ((int)blockIdx.x - tab.block_begin[cls]) * (kWaBlock / G) + group;
  const bool active = net < tab.net_begin[cls + 1];
  const float inv_gamma = 1.f / gamma;

  int s = 0, d = 0;
  if (active) { s = s_net_start[net]; d = s_net_start[net + 1] - s; }

  // ---- phase A: extremes per set and axis, z extremes, set sizes
  Ext tx = {top2_empty_max(), top2_empty_min()}, ty = tx, bx = tx, by = tx;
  float zmax = kNegInf, zmin = kPosInf;
  int ct = 0, cb = 0;
  for (int k = lane; k < d; k += G) {
    const PinData p = load_pin(xyz, n, pin_node, off, s + k, half_dz);
    if (p.top) {
      top2_put_max(tx.mx, p.ux); top2_put_min(tx.mn, p.ux);
      top2_put_max(ty.mx, p.uy); top2_put_min(ty.mn, p.uy);
      ++ct;
    } else {
      top2_put_max(bx.mx, p.ux); top2_put_min(bx.mn, p.ux);
      top2_put_max(by.mx, p.uy); top2_put_min(by.mn, p.uy);
      ++cb;
    }
    zmax = fmaxf(zmax, p.z); zmin = fminf(zmin, p.z);
  }
  for (int m = G >> 1; m > 0; m >>= 1) {
    top2_merge_max(tx.mx, m); top2_merge_min(tx.mn, m);
    top2_merge_max(ty.mx, m); top2_merge_min(ty.mn, m);
    top2_merge_max(bx.mx, m); top2_merge_min(bx.mn, m);
    top2_merge_max(by.mx, m); top2_merge_min(by.mn, m);
    zmax = fmaxf(zmax, __shfl_xor(zmax, m));
    zmin = fminf(zmin, __shfl_xor(zmin, m));
    ct += __shfl_xor(ct, m);
    cb += __shfl_xor(cb, m);
  }

  // ---- phase B: shifted exponential sums per set and axis, and for z over the whole net
  SetSums sxt = {0, 0, 0, 0}, sxb = sxt, syt = sxt, syb = sxt, sz = sxt;
  for (int k = lane; k < d; k += G) {
    const PinData p = load_pin(xyz, n, pin_node, off, s + k, half_dz);
    // shifts of the pin's own set; sums go to that set
    const float Mx = p.top ? tx.mx.a1.h : bx.mx.a1.h, mx = p.top ? tx.mn.a1.h : bx.mn.a1.h;
    const float My = p.top ? ty.mx.a1.h : by.mx.a1.h, my = p.top ? ty.mn.a1.h : by.mn.a1.h;
    const float dux = (p.ux.h - Mx) + p.ux.l, dlx = (p.ux.h - mx) + p.ux.l;
    const float duy = (p.uy.h - My) + p.uy.l, dly = (p.uy.h - my) + p.uy.l;
    const float epx = __expf(dux * inv_gamma), emx = __expf(-dlx * inv_gamma);
    const float epy = __expf(duy * inv_gamma), emy = __expf(-dly * inv_gamma);
    if (p.top) {
      sxt.sp += epx; sxt.tp += dux * epx; sxt.sm += emx; sxt.tm += dlx * emx;
      syt.sp += epy; syt.tp += duy * epy; syt.sm += emy; syt.tm += dly * emy;
    } else {
      sxb.sp += epx; sxb.tp += dux * epx; sxb.sm += emx; sxb.tm += dlx * emx;
      syb.sp += epy; syb.tp += duy * epy; syb.sm += emy; syb.tm += dly * emy;
    }
    {
      const float du = p.z - zmax, dl = p.z - zmin;
      const float ep = __expf(du * inv_gamma), em = __expf(-dl * inv_gamma);
      sz.sp += ep; sz.tp += du * ep; sz.sm += em; sz.tm += dl * em;
    }
  }
  for (int m = G >> 1; m > 0; m >>= 1) {
#define P3D_RED4(S) S.sp += __shfl_xor(S.sp, m); S.tp += __shfl_xor(S.tp, m); \
                    S.sm += __shfl_xor(S.sm, m); S.tm += __shfl_xor(S.tm, m);
    P3D_RED4(sxt) P3D_RED4(sxb) P3D_RED4(syt) P3D_RED4(syb) P3D_RED4(sz)
#undef P3D_RED4
  }

  const AxisWA wx = axis_wa(tx, sxt, ct, bx, sxb, cb, inv_gamma);
  const AxisWA wy = axis_wa(ty, syt, ct, by, syb, cb, inv_gamma);
  const float Azp = d > 0 ? sz.tp / sz.sp : 0.f, Azm = d > 0 ? sz.tm / sz.sm : 0.f;
  const float pz = d > 0 ? (zmax - zmin) + (Azp - Azm) : 0.f;
  const float Wx = bistratal_exact(tx.mx.a1, tx.mn.a1, ct, bx.mx.a1, bx.mn.a1, cb);
  const float Wy = bistratal_exact(ty.mx.a1, ty.mn.a1, ct, by.mx.a1, by.mn.a1, cb);

  // ---- phase C: per-pin gradient shares and FDA differences
  for (int k = lane; k < d; k += G) {
    const PinData p = load_pin(xyz, n, pin_node, off, s + k, half_dz);
    const float gx = axis_grad(wx, p.ux, p.top, inv_gamma);
    const float gy = axis_grad(wy, p.uy, p.top, inv_gamma);
    const float du = p.z - zmax, dl = p.z - zmin;
    const float ep = __expf(du * inv_gamma), em = __expf(-dl * inv_gamma);
    const float gz = alpha * (ep / sz.sp * (1.f + (du - Azp) * inv_gamma) - em / sz.sm * (1.f - (dl - Azm) * inv_gamma));
    float wfx, wfy;
    if (p.top) {
      wfx = bistratal_flip(tx, ct, bx, cb, p.ux, p.fx);
      wfy = bistratal_flip(ty, ct, by, cb, p.uy, p.fy);
    } else {
      wfx = bistratal_flip(bx, cb, tx, ct, p.ux, p.fx);
      wfy = bistratal_flip(by, cb, ty, ct, p.uy, p.fy);
    }
    // (4/d_z) (W with the owner on top - W with it on the bottom)
    const float dw = (wfx - Wx) + (wfy - Wy);
    const float fda = four_over_dz * (p.top ? -dw : dw);
    pin_out[s + k] = make_float4(gx, gy, gz, fda);
  }

  // ---- net totals: one contribution per group, block-reduced in float64
  double v[5] = {0, 0, 0, 0, 0};
  if (active && lane == 0 && d > 0) {
    DF xmax = tx.mx.a1, xmin = tx.mn.a1, ymax = ty.mx.a1, ymin = ty.mn.a1;
    if (cb > 0) {
      if (ct == 0 || dgt(bx.mx.a1, xmax)) xmax = bx.mx.a1;
      if (ct == 0 || dgt(xmin, bx.mn.a1)) xmin = bx.mn.a1;
      if (ct == 0 || dgt(by.mx.a1, ymax)) ymax = by.mx.a1;
      if (ct == 0 || dgt(ymin, by.mn.a1)) ymin = by.mn.a1;
    }
    v[0] = (double)wx.W + (double)wy.W;
    v[1] = (double)alpha * (double)pz;
    v[2] = (double)Wx + (double)Wy;
    v[3] = (double)dsub(xmax, xmin) + (double)dsub(ymax, ymin) + (double)alpha * (double)(zmax - zmin);
    v[4] = (ct > 0 && cb > 0) ? 1.0 : 0.0;
  }
  for (int q = 0; q < 5; ++q) {
    double x = v[q];
    for (int m = kWave / 2; m > 0; m >>= 1) x += __shfl_xor(x, m);
    if ((threadIdx.x & (kWave - 1)) == 0) shred[q][threadIdx.x / kWave] = x;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    double x = 0.0;
    for (int w = 0; w < kWaBlock / kWave; ++w) x += shred[threadIdx.x][w];
    part[(size_t)(R_WA_BI + threadIdx.x) * stride + blockIdx.x] = x;
  }
}

// per instance: sum the pin shares in slot order; L1 norms over movable instances
__global__ void k_wl_gather(int n, const uint8_t* __restrict__ kind, const int32_t* __restrict__ node_slot_start,
                            const int32_t* __restrict__ node_slots, const float4* __restrict__ pin_out,
                            float* __restrict__ grad, int accumulate, float* __restrict__ gz_wa,
                            float* __restrict__ fda, double* __restrict__ part, int stride) {
  __shared__ double sh[3][256 / kWave];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float gx = 0.f, gy = 0.f, gz = 0.f, gf = 0.f;
  if (i < n && !(kind[i] & PLACE3D_KIND_FIXED)) {
    for (int q = node_slot_start[i]; q < node_slot_start[i + 1]; ++q) {
      const float4 v = pin_out[node_slots[q]];
      gx += v.x; gy += v.y; gz += v.z; gf += v.w;
    }
  }
  if (i < n) {
    if (accumulate) { grad[i] += gx; grad[n + i] += gy; }
    else { grad[i] = gx; grad[n + i] = gy; }
    gz_wa[i] = gz;
    fda[i] = gf;
  }
  double a[3] = {fabs((double)gx), fabs((double)gy), fabs((double)gf)};
  for (int q = 0; q < 3; ++q) {
    double x = a[q];
    for (int m = kWave / 2; m > 0; m >>= 1) x += __shfl_xor(x, m);
    if ((threadIdx.x & (kWave - 1)) == 0) sh[q][threadIdx.x / kWave] = x;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double x = 0.0;
    for (int w = 0; w < 256 / kWave; ++w) x += sh[threadIdx.x][w];
    part[(size_t)(R_NORM_X + threadIdx.x) * stride + blockIdx.x] = x;
  }
}

__device__ __forceinline__ double fda_scale(const double* red) {
  const double nf = red[R_NORM_FDA];
  return nf > 0.0 ? (red[R_NORM_X] + red[R_NORM_Y]) / (2.0 * nf) : 0.0;
}

// grad_z (+)= scale * fda + gz_wa, scale = (|g_x|_1 + |g_y|_1) / (2 |fda|_1)
__global__ void k_wl_finish_z(int n, const float* __restrict__ gz_wa, const float* __restrict__ fda,
                              const double* __restrict__ red, float* __restrict__ grad, int accumulate,
                              double* __restrict__ metrics) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const float scale = (float)fda_scale(red);
  if (i < n) {
    const float v = scale * fda[i] + gz_wa[i];
    if (accumulate) grad[2 * n + i] += v; else grad[2 * n + i] = v;
  }
  if (metrics && i < PLACE3D_NMETRICS) {
    double v = 0.0;
    if (i <= PLACE3D_M_NORM_FDA) v = red[R_WA_BI + i];
    else if (i == PLACE3D_M_FDA_SCALE) v = fda_scale(red);
    metrics[i] = v;
  }
}

}  // namespace

int wirelength_eval(place3d_ctx* c, const float* xyz, float* grad, int accumulate, double* red,
                    double* metrics, hipStream_t s) {
  const Geom& g = c->g;
  const place3d_problem& p = c->prob;
  int rc;
  if (c->n_wa_blocks > 0) {
    ProfScope prof_(c, PLACE3D_STAGE_WL_NETS, s);
    hipLaunchKernelGGL(k_wl_nets, dim3(c->n_wa_blocks), dim3(kWaBlock), 0, s, g.n, g.half_dz, 4.f / g.dz,
                       (float)p.gamma, (float)p.alpha, xyz, c->s_net_start, c->s_pin_node, c->s_off, c->pin_out,
                       c->classes, c->part, c->part_stride);
    P3D_LAUNCH(c, "k_wl_nets");
  }
  if ((rc = reduce_final(c, R_WA_BI, 5, c->n_wa_blocks, false, red + R_WA_BI, s))) return rc;
  const unsigned nb = blocks_for(g.n, 256);
  {
    ProfScope prof_(c, PLACE3D_STAGE_WL_NODES, s);
    hipLaunchKernelGGL(k_wl_gather, dim3(nb), dim3(256), 0, s, g.n, p.kind, c->node_slot_start, c->node_slots,
                       c->pin_out, grad, accumulate, c->wl_gzwa, c->wl_fda, c->part, c->part_stride);
    P3D_LAUNCH(c, "k_wl_gather");
  }
  if ((rc = reduce_final(c, R_NORM_X, 3, (int)nb, false, red + R_NORM_X, s))) return rc;
  {
    ProfScope prof_(c, PLACE3D_STAGE_WL_NODES, s);
    hipLaunchKernelGGL(k_wl_finish_z, dim3(blocks_for(std::max(g.n, (int)PLACE3D_NMETRICS), 256)), dim3(256), 0, s,
                       g.n, c->wl_gzwa, c->wl_fda, red, grad, accumulate, metrics);
    P3D_LAUNCH(c, "k_wl_finish_z");
  }
  return PLACE3D_OK;
}

}  // namespace p3d
