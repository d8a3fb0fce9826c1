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
  float rt, rb, qt, qb;                   // e^{(M_S - M_e)/gamma}, e^{-(m_S - m_e)/gamma} per set
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
  a.rt = a.rb = a.qt = a.qb = 1.f;
  const float pt = ct > 0 ? (a.Mt - a.mt) + (a.At_p - a.At_m) : 0.f;
  const float pb = cb > 0 ? (a.Mb - a.mb) + (a.Ab_p - a.Ab_m) : 0.f;
  // whole net: rescale the partial sums to the whole-net shifts
  if (ct > 0 && cb > 0) {
    a.Me = fmaxf(a.Mt, a.Mb);
    a.me = fminf(a.mt, a.mb);
    const float dt = a.Mt - a.Me, db = a.Mb - a.Me;                 // <= 0
    a.rt = __expf(dt * inv_gamma);
    a.rb = __expf(db * inv_gamma);
    a.se_p = st.sp * a.rt + sb.sp * a.rb;
    const float te_p = a.rt * (st.tp + dt * st.sp) + a.rb * (sb.tp + db * sb.sp);
    const float dtm = a.mt - a.me, dbm = a.mb - a.me;              // >= 0
    a.qt = __expf(-dtm * inv_gamma);
    a.qb = __expf(-dbm * inv_gamma);
    a.se_m = st.sm * a.qt + sb.sm * a.qb;
    const float te_m = a.qt * (st.tm + dtm * st.sm) + a.qb * (sb.tm + dbm * sb.sm);
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

// a pin's offsets from its set's shifts and the shifted exponentials (phase B), kept for phase C
struct PinExp { float dux, dlx, epx, emx, duy, dly, epy, emy, duz, dlz, epz, emz; };

__device__ __forceinline__ PinExp pin_exps(const PinData& p, const Ext& tx, const Ext& bx, const Ext& ty,
                                           const Ext& by, float zmax, float zmin, float inv_gamma) {
  PinExp e;
  const float Mx = p.top ? tx.mx.a1.h : bx.mx.a1.h, mx = p.top ? tx.mn.a1.h : bx.mn.a1.h;
  const float My = p.top ? ty.mx.a1.h : by.mx.a1.h, my = p.top ? ty.mn.a1.h : by.mn.a1.h;
  e.dux = (p.ux.h - Mx) + p.ux.l; e.dlx = (p.ux.h - mx) + p.ux.l;
  e.duy = (p.uy.h - My) + p.uy.l; e.dly = (p.uy.h - my) + p.uy.l;
  e.duz = p.z - zmax; e.dlz = p.z - zmin;
  e.epx = __expf(e.dux * inv_gamma); e.emx = __expf(-e.dlx * inv_gamma);
  e.epy = __expf(e.duy * inv_gamma); e.emy = __expf(-e.dly * inv_gamma);
  e.epz = __expf(e.duz * inv_gamma); e.emz = __expf(-e.dlz * inv_gamma);
  return e;
}

__device__ __forceinline__ void add_sums(const PinExp& e, bool top, SetSums& sxt, SetSums& sxb, SetSums& syt,
                                         SetSums& syb, SetSums& sz) {
  if (top) {
    sxt.sp += e.epx; sxt.tp += e.dux * e.epx; sxt.sm += e.emx; sxt.tm += e.dlx * e.emx;
    syt.sp += e.epy; syt.tp += e.duy * e.epy; syt.sm += e.emy; syt.tm += e.dly * e.emy;
  } else {
    sxb.sp += e.epx; sxb.tp += e.dux * e.epx; sxb.sm += e.emx; sxb.tm += e.dlx * e.emx;
    syb.sp += e.epy; syb.tp += e.duy * e.epy; syb.sm += e.emy; syb.tm += e.dly * e.emy;
  }
  sz.sp += e.epz; sz.tp += e.duz * e.epz; sz.sm += e.emz; sz.tm += e.dlz * e.emz;
}

// d W^ / d u for one pin of the chosen branch, from its set-shifted offsets and exponentials.
// Every field is passed by value so that the branch choice is a select between values.
__device__ __forceinline__ float grad_branch(bool split, bool top, float du, float dl, float ep, float em,
                                             float inv_gamma, float Mt, float Mb, float Me, float mt, float mb,
                                             float me, float rt, float rb, float qt, float qb, float At_p, float Ab_p,
                                             float Ae_p, float st_p, float sb_p, float se_p, float At_m, float Ab_m,
                                             float Ae_m, float st_m, float sb_m, float se_m) {
  const float Ap_s = top ? At_p : Ab_p, sp_s = top ? st_p : sb_p;
  const float Am_s = top ? At_m : Ab_m, sm_s = top ? st_m : sb_m;
  // whole-net branch: move from the set's shifts to the whole-net shifts
  const float du_e = du + ((top ? Mt : Mb) - Me), dl_e = dl + ((top ? mt : mb) - me);
  const float ep_e = ep * (top ? rt : rb), em_e = em * (top ? qt : qb);
  const float Ap = split ? Ap_s : Ae_p, sp = split ? sp_s : se_p;
  const float Am = split ? Am_s : Ae_m, sm = split ? sm_s : se_m;
  const float u = split ? du : du_e, l = split ? dl : dl_e;
  const float p = split ? ep : ep_e, q = split ? em : em_e;
  return p / sp * (1.f + (u - Ap) * inv_gamma) - q / sm * (1.f - (l - Am) * inv_gamma);
}

#define P3D_AXIS_GRAD(a, top, du, dl, ep, em)                                                          \
  grad_branch((a).split, top, du, dl, ep, em, inv_gamma, (a).Mt, (a).Mb, (a).Me, (a).mt, (a).mb, (a).me, \
              (a).rt, (a).rb, (a).qt, (a).qb, (a).At_p, (a).Ab_p, (a).Ae_p, (a).st_p, (a).sb_p, (a).se_p, \
              (a).At_m, (a).Ab_m, (a).Ae_m, (a).st_m, (a).sb_m, (a).se_m)

__global__ __launch_bounds__(kWaBlock) void k_wl_nets(
    int n, float half_dz, float four_over_dz, float gamma, float alpha, const float* __restrict__ xyz,
    const int32_t* __restrict__ s_net_start, const int32_t* __restrict__ pin_node, const float4* __restrict__ off,
    const int32_t* __restrict__ slot_pos, float4* __restrict__ pin_out, ClassTab tab, double* __restrict__ part,
    int stride) {
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
  // the lane's first pin stays in registers through all phases; further pins (nets larger than
  // the group, only in the 64-lane class) are reloaded per phase
  const bool have0 = lane < d;
  PinData p0;
  if (have0) p0 = load_pin(xyz, n, pin_node, off, s + lane, half_dz);

  // ---- phase A: extremes per set and axis, z extremes, set sizes
  Ext tx = {top2_empty_max(), top2_empty_min()}, ty = tx, bx = tx, by = tx;
  float zmax = kNegInf, zmin = kPosInf;
  int ct = 0, cb = 0;
#define P3D_PUT(p)                                                          \
  do {                                                                      \
    if ((p).top) {                                                          \
      top2_put_max(tx.mx, (p).ux); top2_put_min(tx.mn, (p).ux);             \
      top2_put_max(ty.mx, (p).uy); top2_put_min(ty.mn, (p).uy);             \
      ++ct;                                                                 \
    } else {                                                                \
      top2_put_max(bx.mx, (p).ux); top2_put_min(bx.mn, (p).ux);             \
      top2_put_max(by.mx, (p).uy); top2_put_min(by.mn, (p).uy);             \
      ++cb;                                                                 \
    }                                                                       \
    zmax = fmaxf(zmax, (p).z); zmin = fminf(zmin, (p).z);                   \
  } while (0)
  if (have0) P3D_PUT(p0);
  for (int k = lane + G; k < d; k += G) {
    const PinData p = load_pin(xyz, n, pin_node, off, s + k, half_dz);
    P3D_PUT(p);
  }
#undef P3D_PUT
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
  PinExp e0 = {};
  if (have0) {
    e0 = pin_exps(p0, tx, bx, ty, by, zmax, zmin, inv_gamma);
    add_sums(e0, p0.top, sxt, sxb, syt, syb, sz);
  }
  for (int k = lane + G; k < d; k += G) {
    const PinData p = load_pin(xyz, n, pin_node, off, s + k, half_dz);
    add_sums(pin_exps(p, tx, bx, ty, by, zmax, zmin, inv_gamma), p.top, sxt, sxb, syt, syb, sz);
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
#define P3D_EMIT(p, e, slot)                                                                   \
  do {                                                                                         \
    const float gx_ = P3D_AXIS_GRAD(wx, (p).top, (e).dux, (e).dlx, (e).epx, (e).emx);          \
    const float gy_ = P3D_AXIS_GRAD(wy, (p).top, (e).duy, (e).dly, (e).epy, (e).emy);          \
    const float gz_ = alpha * ((e).epz / sz.sp * (1.f + ((e).duz - Azp) * inv_gamma) -         \
                               (e).emz / sz.sm * (1.f - ((e).dlz - Azm) * inv_gamma));         \
    float wfx_, wfy_;                                                                          \
    if ((p).top) {                                                                             \
      wfx_ = bistratal_flip(tx, ct, bx, cb, (p).ux, (p).fx);                                   \
      wfy_ = bistratal_flip(ty, ct, by, cb, (p).uy, (p).fy);                                   \
    } else {                                                                                   \
      wfx_ = bistratal_flip(bx, cb, tx, ct, (p).ux, (p).fx);                                   \
      wfy_ = bistratal_flip(by, cb, ty, ct, (p).uy, (p).fy);                                   \
    }                                                                                          \
    /* (4/d_z) (W with the owner on top - W with it on the bottom) */                          \
    const float dw_ = (wfx_ - Wx) + (wfy_ - Wy);                                               \
    pin_out[slot_pos[slot]] = make_float4(gx_, gy_, gz_, four_over_dz * ((p).top ? -dw_ : dw_)); \
  } while (0)
  if (have0) P3D_EMIT(p0, e0, s + lane);
  for (int k = lane + G; k < d; k += G) {
    const PinData p = load_pin(xyz, n, pin_node, off, s + k, half_dz);
    const PinExp e = pin_exps(p, tx, bx, ty, by, zmax, zmin, inv_gamma);
    P3D_EMIT(p, e, s + k);
  }
#undef P3D_EMIT

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

// per instance: sum its pin shares (contiguous, ascending slot order); L1 norms over movable instances
// per instance: sum its pin shares (contiguous, ascending slot order); L1 norms over movable
// instances.  Blocks [0, nlight) take one instance per thread; instances with more than
// kHeavyPins pins are left to the blocks after them, one wavefront per instance.
constexpr int kHeavyPins = 32;

__global__ void k_wl_gather(int n, int nlight, const int32_t* __restrict__ heavy, int nheavy,
                            const uint8_t* __restrict__ kind, const int32_t* __restrict__ node_slot_start,
                            const float4* __restrict__ pin_out, float* __restrict__ grad, int accumulate,
                            float* __restrict__ gz_wa, float* __restrict__ fda, double* __restrict__ part, int stride) {
  __shared__ double sh[3][256 / kWave];
  float gx = 0.f, gy = 0.f, gz = 0.f, gf = 0.f;
  int i = -1;
  bool writer = false;
  if ((int)blockIdx.x < nlight) {
    i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
      const int q0 = node_slot_start[i], q1 = node_slot_start[i + 1];
      writer = q1 - q0 <= kHeavyPins;
      if (writer && !(kind[i] & PLACE3D_KIND_FIXED))
        for (int q = q0; q < q1; ++q) {
          const float4 v = pin_out[q];
          gx += v.x; gy += v.y; gz += v.z; gf += v.w;
        }
    }
  } else {
    const int w = ((int)blockIdx.x - nlight) * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (w < nheavy) {
      i = heavy[w];
      if (!(kind[i] & PLACE3D_KIND_FIXED))
        for (int q = node_slot_start[i] + lane; q < node_slot_start[i + 1]; q += kWave) {
          const float4 v = pin_out[q];
          gx += v.x; gy += v.y; gz += v.z; gf += v.w;
        }
      for (int m = kWave / 2; m > 0; m >>= 1) {   // butterfly: lane sums, fixed order
        gx += __shfl_xor(gx, m); gy += __shfl_xor(gy, m);
        gz += __shfl_xor(gz, m); gf += __shfl_xor(gf, m);
      }
      writer = lane == 0;
    }
  }
  if (writer) {
    if (accumulate) { grad[i] += gx; grad[n + i] += gy; }
    else { grad[i] = gx; grad[n + i] = gy; }
    gz_wa[i] = gz;
    fda[i] = gf;
  } else {
    gx = gy = gz = gf = 0.f;
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
                       (float)p.gamma, (float)p.alpha, xyz, c->s_net_start, c->s_pin_node, c->s_off, c->slot_pos,
                       c->pin_out, c->classes, c->part, c->part_stride);
    P3D_LAUNCH(c, "k_wl_nets");
  }
  if ((rc = reduce_final(c, R_WA_BI, 5, c->n_wa_blocks, false, red + R_WA_BI, s))) return rc;
  const unsigned nlight = blocks_for(g.n, 256);
  const unsigned nb = nlight + (unsigned)((c->n_heavy + 3) / 4);
  {
    ProfScope prof_(c, PLACE3D_STAGE_WL_NODES, s);
    hipLaunchKernelGGL(k_wl_gather, dim3(nb), dim3(256), 0, s, g.n, (int)nlight, c->heavy_list, c->n_heavy, p.kind,
                       c->node_slot_start, c->pin_out, grad, accumulate, c->wl_gzwa, c->wl_fda, c->part,
                       c->part_stride);
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
