// Bistratal weighted-average wirelength, its gradient and the FDA z-gradient
// (Sec. III-A: Eqs. wa-model-approx, optimal-region, wl-obj, wl-model, fda-grad, fda-normalize;
// Sec. IV-B: incremental evaluation from first and second extremes).
//
// Work split: a net of degree d is taken by a group of G = 1, 2, 4, ..., 64 lanes, the smallest
// with d <= kPinsPerLane * G (64 lanes for larger nets, whose lanes then loop); most nets have
// few pins and are taken by a single lane.  Lane l of a group holds pins l, l + G, ... in
// registers and the group walks them three times: (A) first and second largest and smallest pin
// coordinate per die set and axis, z extremes, set sizes; (B) max-shifted exponential sums per
// set and axis, and over the whole net in z; (C) per pin: its share of the gradient of the
// chosen branch, its WA z-gradient and the FDA difference.  Group reductions after (A) and (B)
// are xor butterflies, symmetric, so every lane of a group holds the same net values.  A static
// schedule built at context creation lays out nets by class, widest groups first, so a workgroup
// holds groups of one size.
//
// Pin coordinates are taken relative to the x, y of the net's first pin's owner: the rounding of
// each relative coordinate is then bounded by the net's span, not by the die size, and every
// quantity computed here is invariant to that shift.
//
// Per net and axis:
//   p^_S = (M_S + t+_S/s+_S) - (m_S + t-_S/s-_S)  with t+ = sum (u - M) e^{(u - M)/gamma}
//   W^_u = max{p^_e, p^_e+ + p^_e-} for a net crossing the dies, else p^_e
//   W_u  = max{p_e, p_e+ + p_e-}  (exact, the FDA and HPWL metric)
// where the whole-net sums are the two set sums rescaled to the whole-net shifts.  The FDA of
// a pin is (4/d_z)(W(owner on top) - W(owner on bottom)) in O(1): the pin leaves its set (the
// second extreme replaces it when it was the first) and joins the other set at its other-die
// offset.
#include <mutex>

#include "internal.h"

namespace p3d {
namespace {

constexpr float kNegInf = -__builtin_huge_valf();
constexpr float kPosInf = __builtin_huge_valf();

// DPP lane exchange inside a row of 16 lanes
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Exchange with the partner lane of a butterfly step of width 2M.  Steps 1 and 2 are xor 1 and
// xor 2 (quad permutes); steps 4 and 8 use the half-row and row mirrors (xor 7, xor 15), which
// pair lanes inside the same aligned group of 2M lanes and, with the other steps, still reach
// every lane of a group; 16 and 32 use a cross-lane permute.  Every merge below is commutative,
// so both partners of an exchange compute the same value.
template <int M>
__device__ __forceinline__ float xchg(float v) {
  if constexpr (M == 1) return dpp<0xB1>(v);
  else if constexpr (M == 2) return dpp<0x4E>(v);
  else if constexpr (M == 4) return dpp<0x141>(v);
  else if constexpr (M == 8) return dpp<0x140>(v);
  else return __shfl_xor(v, M);
}
template <int M>
__device__ __forceinline__ int xchg(int v) {
  return __float_as_int(xchg<M>(__int_as_float(v)));
}

struct PinRel {        // one pin, relative to the net anchor
  float ux, uy;        // on its owner's current die
  float fx, fy;        // on the other die
  float z;
  bool top;
};

__device__ __forceinline__ PinRel load_pin(const float4* __restrict__ xyzp, const int32_t* __restrict__ pin_node,
                                           const float4* __restrict__ off, int slot, float half_dz, float xa, float ya) {
  const float4 q = xyzp[pin_node[slot]];
  const float4 o = off[slot];
  const float dx = q.x - xa, dy = q.y - ya;
  PinRel p;
  p.z = q.z;
  p.top = p.z > half_dz;
  p.ux = dx + (p.top ? o.z : o.x);
  p.uy = dy + (p.top ? o.w : o.y);
  p.fx = dx + (p.top ? o.x : o.z);
  p.fy = dy + (p.top ? o.y : o.w);
  return p;
}

// first and second largest and smallest of a multiset (duplicates kept)
struct Ext2 { float max1, max2, min1, min2; };

__device__ __forceinline__ Ext2 ext_empty() { return {kNegInf, kNegInf, kPosInf, kPosInf}; }
// vmax / vmin: the value, or the -inf / +inf sentinel for a pin outside the set
__device__ __forceinline__ void ext_put(Ext2& e, float vmax, float vmin) {
  e.max2 = fmaxf(e.max2, fminf(e.max1, vmax));
  e.max1 = fmaxf(e.max1, vmax);
  e.min2 = fminf(e.min2, fmaxf(e.min1, vmin));
  e.min1 = fminf(e.min1, vmin);
}
__device__ __forceinline__ Ext2 ext_sel(bool c, const Ext2& a, const Ext2& b) {
  return {c ? a.max1 : b.max1, c ? a.max2 : b.max2, c ? a.min1 : b.min1, c ? a.min2 : b.min2};
}

struct NetExt {
  Ext2 tx, ty, bx, by;        // top / bottom set, x / y
  float zmax, zmin;
  int ct, cb;
};

// every set is updated with values or sentinels (no branch on the die): a branch would let
// the compiler select between the sets' addresses and move them to scratch memory
__device__ __forceinline__ void ext_add(NetExt& a, const PinRel& p) {
  const float tx_hi = p.top ? p.ux : kNegInf, tx_lo = p.top ? p.ux : kPosInf;
  const float bx_hi = p.top ? kNegInf : p.ux, bx_lo = p.top ? kPosInf : p.ux;
  const float ty_hi = p.top ? p.uy : kNegInf, ty_lo = p.top ? p.uy : kPosInf;
  const float by_hi = p.top ? kNegInf : p.uy, by_lo = p.top ? kPosInf : p.uy;
  ext_put(a.tx, tx_hi, tx_lo);
  ext_put(a.bx, bx_hi, bx_lo);
  ext_put(a.ty, ty_hi, ty_lo);
  ext_put(a.by, by_hi, by_lo);
  a.ct += p.top ? 1 : 0;
  a.cb += p.top ? 0 : 1;
  a.zmax = fmaxf(a.zmax, p.z);
  a.zmin = fminf(a.zmin, p.z);
}

template <int M>
__device__ __forceinline__ void ext_merge(Ext2& e) {
  const float a1 = xchg<M>(e.max1), a2 = xchg<M>(e.max2);
  const float b1 = xchg<M>(e.min1), b2 = xchg<M>(e.min2);
  e.max2 = fmaxf(fmaxf(e.max2, a2), fminf(e.max1, a1));
  e.max1 = fmaxf(e.max1, a1);
  e.min2 = fminf(fminf(e.min2, b2), fmaxf(e.min1, b1));
  e.min1 = fminf(e.min1, b1);
}

// A float32 sum, compensated when C (the rounding error of every addition is kept in c and added
// back at the end), plain otherwise.  add_small: for a term no larger in magnitude than the
// running sum, whose rounding error is then x - (t - s) exactly (Dekker's Fast2Sum); a lane's
// exponential sums use it by starting from an offset of their terms' sign at least as large as
// any term (so the running sum never falls below a term) and taking the offset off, exactly,
// before they are merged or read.  merge<M> adds the partner lane's sum with Neumaier's variant
// of Kahan summation (terms of any size); it is commutative, so both partners of a butterfly hold
// the same sum.
template <bool C>
struct Acc {
  float s, c;
  __device__ __forceinline__ void add_small(float x) {
    if constexpr (C) {
      const float t = s + x;
      c += x - (t - s);
      s = t;
    } else {
      s += x;
    }
  }
  template <int M>
  __device__ __forceinline__ void merge() {
    const float o = xchg<M>(s);
    if constexpr (C) {
      const float oc = xchg<M>(c);
      const float t = s + o;
      const float e = fabsf(s) >= fabsf(o) ? (s - t) + o : (o - t) + s;
      c = (c + oc) + e;
      s = t;
    } else {
      s += o;
    }
  }
  __device__ __forceinline__ float value() const { return C ? s + c : s; }
};

// shifted exponential sums of one set along one axis: s+ = sum e^{(u-M)/g}, t+ = sum (u-M) e^{(u-M)/g},
// s- = sum e^{-(u-m)/g}, t- = sum (u-m) e^{-(u-m)/g}
template <bool C>
struct Sums4 { Acc<C> sp, tp, sm, tm; };
struct Sums4v { float sp, tp, sm, tm; };

template <bool C>
__device__ __forceinline__ Sums4v val(const Sums4<C>& s) { return {s.sp.value(), s.tp.value(), s.sm.value(), s.tm.value()}; }

template <int M, bool C>
__device__ __forceinline__ void sums_merge(Sums4<C>& s) {
  s.sp.template merge<M>(); s.tp.template merge<M>();
  s.sm.template merge<M>(); s.tm.template merge<M>();
}

// the sums of one axis: the top set, the bottom set
template <bool C>
struct AxisSums { Sums4<C> t, b; };

// Starting values of a lane's four sums and their removal.  The terms e^{(u-M)/g} and e^{-(u-m)/g}
// lie in (0, 1] and (u-M) e^{(u-M)/g} in [-g/e, 0], (u-m) e^{-(u-m)/g} in [0, g/e]; with big a
// power of two above gamma, the offsets 1, -big, 1, big bound every term, and s - offset is exact
// (both are multiples of the sum's ulp and the difference is no larger than the sum).
template <bool C>
__device__ __forceinline__ Sums4<C> sums_start(float big) {
  if constexpr (C) return {{1.f, 0.f}, {-big, 0.f}, {1.f, 0.f}, {big, 0.f}};
  else return {};
}
template <bool C>
__device__ __forceinline__ void sums_settle(Sums4<C>& s, float big) {
  if constexpr (C) {
    s.sp.s -= 1.f; s.tp.s += big; s.sm.s -= 1.f; s.tm.s -= big;
  }
}

template <bool C>
__device__ __forceinline__ void sums_add(Sums4<C>& s, bool in, float du, float dl, float ep, float em) {
  s.sp.add_small(in ? ep : 0.f);
  s.tp.add_small(in ? du * ep : 0.f);
  s.sm.add_small(in ? em : 0.f);
  s.tm.add_small(in ? dl * em : 0.f);
}

// one pin's terms along one axis: u its coordinate, (M, m) the extremes of its own set
template <bool C>
__device__ __forceinline__ void sums_axis(AxisSums<C>& S, bool top, float u, float M, float m, float ig) {
  const float du = u - M, dl = u - m;
  const float ep = __expf(du * ig), em = __expf(-dl * ig);
  sums_add(S.t, top, du, dl, ep, em);
  sums_add(S.b, !top, du, dl, ep, em);
}
template <bool C>
__device__ __forceinline__ void sums_z(Sums4<C>& S, const NetExt& a, const PinRel& p, float ig) {
  const float duz = p.z - a.zmax, dlz = p.z - a.zmin;
  sums_add(S, true, duz, dlz, __expf(duz * ig), __expf(-dlz * ig));
}

// gradient coefficients of one set along one axis for the chosen branch:
//   dW^/du = e^{(u-M)/g} ap (1 + (u - M - bp)/g) - e^{-(u-m)/g} am (1 - (u - m - bm)/g)
struct SetCoef { float M, m, ap, bp, am, bm; };

struct AxisCoef {
  SetCoef t, b;
  float W;                    // smoothed bistratal value
};

// 1 / x by the hardware reciprocal (1 ulp); the sums it divides by are >= 1 (each holds its
// set's extreme term e^0) or are not used
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ AxisCoef axis_coef(const Ext2& T, const Sums4v& st, int ct, const Ext2& B, const Sums4v& sb,
                                              int cb, float ig) {
  const float Mt = T.max1, mt = T.min1, Mb = B.max1, mb = B.min1;
  const float rt_p = ct > 0 ? rcp(st.sp) : 0.f, rt_m = ct > 0 ? rcp(st.sm) : 0.f;
  const float rb_p = cb > 0 ? rcp(sb.sp) : 0.f, rb_m = cb > 0 ? rcp(sb.sm) : 0.f;
  const float At_p = st.tp * rt_p, At_m = st.tm * rt_m;
  const float Ab_p = sb.tp * rb_p, Ab_m = sb.tm * rb_m;
  const float pt = ct > 0 ? (Mt - mt) + (At_p - At_m) : 0.f;
  const float pb = cb > 0 ? (Mb - mb) + (Ab_p - Ab_m) : 0.f;
  AxisCoef c;
  if (ct > 0 && cb > 0) {
    // whole net: both set sums rescaled to the whole-net shifts
    const float Me = fmaxf(Mt, Mb), me = fminf(mt, mb);
    const float dt = Mt - Me, db = Mb - Me;          // <= 0
    const float rt = __expf(dt * ig), rb = __expf(db * ig);
    const float ie_p = rcp(st.sp * rt + sb.sp * rb);
    const float Ae_p = (rt * (st.tp + dt * st.sp) + rb * (sb.tp + db * sb.sp)) * ie_p;
    const float dtm = mt - me, dbm = mb - me;         // >= 0
    const float qt = __expf(-dtm * ig), qb = __expf(-dbm * ig);
    const float ie_m = rcp(st.sm * qt + sb.sm * qb);
    const float Ae_m = (qt * (st.tm + dtm * st.sm) + qb * (sb.tm + dbm * sb.sm)) * ie_m;
    const float pe = (Me - me) + (Ae_p - Ae_m);
    const bool split = pt + pb > pe;
    c.W = split ? pt + pb : pe;
    if (split) {
      c.t = {Mt, mt, rt_p, At_p, rt_m, At_m};
      c.b = {Mb, mb, rb_p, Ab_p, rb_m, Ab_m};
    } else {
      c.t = {Mt, mt, rt * ie_p, Ae_p - dt, qt * ie_m, Ae_m - dtm};
      c.b = {Mb, mb, rb * ie_p, Ae_p - db, qb * ie_m, Ae_m - dbm};
    }
  } else {
    // one set only: the whole net is that set
    c.W = ct > 0 ? pt : pb;
    c.t = {Mt, mt, rt_p, At_p, rt_m, At_m};
    c.b = {Mb, mb, rb_p, Ab_p, rb_m, Ab_m};
  }
  return c;
}

__device__ __forceinline__ float axis_grad(const AxisCoef& c, bool top, float u, float ig) {
  const float M = top ? c.t.M : c.b.M, m = top ? c.t.m : c.b.m;
  const float ap = top ? c.t.ap : c.b.ap, bp = top ? c.t.bp : c.b.bp;
  const float am = top ? c.t.am : c.b.am, bm = top ? c.t.bm : c.b.bm;
  const float du = u - M, dl = u - m;
  return __expf(du * ig) * ap * (1.f + (du - bp) * ig) - __expf(-dl * ig) * am * (1.f - (dl - bm) * ig);
}

// exact bistratal extent along one axis from the first extremes of the two sets (empty sets
// hold the -inf / +inf sentinels)
__device__ __forceinline__ float w_exact(float tmax, float tmin, int ct, float bmax, float bmin, int cb) {
  const float pt = ct > 0 ? tmax - tmin : 0.f;
  const float pb = cb > 0 ? bmax - bmin : 0.f;
  const float pe = (ct + cb) > 0 ? fmaxf(tmax, bmax) - fminf(tmin, bmin) : 0.f;
  return fmaxf(pe, pt + pb);
}

// the same with one pin (at u in set S) moved to the other set O at f
__device__ __forceinline__ float w_flip(Ext2 S, int cs, Ext2 O, int co, float u, float f) {
  const float smax = u == S.max1 ? S.max2 : S.max1;
  const float smin = u == S.min1 ? S.min2 : S.min1;
  return w_exact(smax, smin, cs - 1, fmaxf(O.max1, f), fminf(O.min1, f), co + 1);
}

struct NetCoef {
  AxisCoef x, y;
  float zmax, zmin, az_p, Az_p, az_m, Az_m;
  float Wx, Wy;
};

// per pin: (dW^/dx, dW^/dy, alpha dW^z/dz, FDA difference)
__device__ __forceinline__ float4 pin_result(const PinRel& p, const NetExt& a, const NetCoef& c, float ig, float alpha,
                                             float four_over_dz) {
  const float gx = axis_grad(c.x, p.top, p.ux, ig);
  const float gy = axis_grad(c.y, p.top, p.uy, ig);
  const float duz = p.z - c.zmax, dlz = p.z - c.zmin;
  const float gz = alpha * (__expf(duz * ig) * c.az_p * (1.f + (duz - c.Az_p) * ig) -
                            __expf(-dlz * ig) * c.az_m * (1.f - (dlz - c.Az_m) * ig));
  const int cs = p.top ? a.ct : a.cb, co = p.top ? a.cb : a.ct;
  const float wfx = w_flip(ext_sel(p.top, a.tx, a.bx), cs, ext_sel(p.top, a.bx, a.tx), co, p.ux, p.fx);
  const float wfy = w_flip(ext_sel(p.top, a.ty, a.by), cs, ext_sel(p.top, a.by, a.ty), co, p.uy, p.fy);
  // (4/d_z) (W with the owner on top - W with it on the bottom)
  const float dw = (wfx - c.Wx) + (wfy - c.Wy);
  return make_float4(gx, gy, gz, four_over_dz * (p.top ? -dw : dw));
}

template <int M>
__device__ __forceinline__ void merge_step(NetExt& a) {
  ext_merge<M>(a.tx); ext_merge<M>(a.bx); ext_merge<M>(a.ty); ext_merge<M>(a.by);
  a.zmax = fmaxf(a.zmax, xchg<M>(a.zmax));
  a.zmin = fminf(a.zmin, xchg<M>(a.zmin));
  a.ct += xchg<M>(a.ct);
  a.cb += xchg<M>(a.cb);
}
template <int M, bool C>
__device__ __forceinline__ void merge_step(AxisSums<C>& S) {
  sums_merge<M>(S.t); sums_merge<M>(S.b);
}
template <int M, bool C>
__device__ __forceinline__ void merge_step(Sums4<C>& S) {
  sums_merge<M>(S);
}
// reduce over a group of G lanes, widest step first
template <int G, class T>
__device__ __forceinline__ void group_merge(T& v) {
  if constexpr (G >= 64) merge_step<32>(v);
  if constexpr (G >= 32) merge_step<16>(v);
  if constexpr (G >= 16) merge_step<8>(v);
  if constexpr (G >= 8) merge_step<4>(v);
  if constexpr (G >= 4) merge_step<2>(v);
  if constexpr (G >= 2) merge_step<1>(v);
}

struct NetTotals { float wa_bi, wa_z, hpwl, hpwl3d, ncut; };

template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the wavefront in a fixed order: quad, half-row and row sums by DPP exchanges
// (xor 1, xor 2, mirror 8, mirror 16), then the four row sums; in float64 when C (at least as
// accurate as a compensated float32 sum of these 64 values, and fewer instructions).
template <bool C>
__device__ __forceinline__ double wave_sum(float v) {
  if constexpr (!C) {
    float a = v;
    a += dpp<0xB1>(a);       // quad_perm(1, 0, 3, 2)
    a += dpp<0x4E>(a);       // quad_perm(2, 3, 0, 1)
    a += dpp<0x141>(a);      // row_half_mirror
    a += dpp<0x140>(a);      // row_mirror
    return (double)((lane_value(a, 0) + lane_value(a, 16)) + (lane_value(a, 32) + lane_value(a, 48)));
  } else {
    double a = (double)v;
    a += dpp<0xB1>(a);
    a += dpp<0x4E>(a);
    a += dpp<0x141>(a);
    a += dpp<0x140>(a);
    return (lane_value(a, 0) + lane_value(a, 16)) + (lane_value(a, 32) + lane_value(a, 48));
  }
}

// one net per group of G lanes; lane lg of the group holds pins lg + G j.  kGrad: also write the
// per-pin results (phase C); else only the net totals.  C: compensated exponential sums.
template <int G, bool kGrad, bool C>
__device__ __forceinline__ NetTotals wl_group(int net, int lg, float half_dz, float four_over_dz, float ig, float big,
                                              float alpha, const float4* __restrict__ xyzp,
                                              const int32_t* __restrict__ s_net_start,
                                              const int32_t* __restrict__ pin_node, const float4* __restrict__ off,
                                              const int32_t* __restrict__ slot_pos, float4* __restrict__ pin_out) {
  const int s = s_net_start[net], d = s_net_start[net + 1] - s;
  const float4 q0 = xyzp[pin_node[s]];
  const float xa = q0.x, ya = q0.y;
  PinRel pc[kPinsPerLane];

  // ---- phase A: extremes
  NetExt a = {ext_empty(), ext_empty(), ext_empty(), ext_empty(), kNegInf, kPosInf, 0, 0};
#pragma unroll
  for (int j = 0; j < kPinsPerLane; ++j)
    if (lg + G * j < d) {
      pc[j] = load_pin(xyzp, pin_node, off, s + lg + G * j, half_dz, xa, ya);
      ext_add(a, pc[j]);
    }
  for (int k = lg + G * kPinsPerLane; k < d; k += G) ext_add(a, load_pin(xyzp, pin_node, off, s + k, half_dz, xa, ya));
  group_merge<G>(a);

  // ---- phase B: shifted exponential sums, one axis at a time, each reduced to its gradient
  // coefficients before the next axis starts (one axis's sums live at a time: compensated sums
  // hold two floats each)
  NetCoef c;
  {
    AxisSums<C> S = {sums_start<C>(big), sums_start<C>(big)};
#pragma unroll
    for (int j = 0; j < kPinsPerLane; ++j)
      if (lg + G * j < d)
        sums_axis(S, pc[j].top, pc[j].ux, pc[j].top ? a.tx.max1 : a.bx.max1, pc[j].top ? a.tx.min1 : a.bx.min1, ig);
    for (int k = lg + G * kPinsPerLane; k < d; k += G) {
      const PinRel p = load_pin(xyzp, pin_node, off, s + k, half_dz, xa, ya);
      sums_axis(S, p.top, p.ux, p.top ? a.tx.max1 : a.bx.max1, p.top ? a.tx.min1 : a.bx.min1, ig);
    }
    sums_settle(S.t, big); sums_settle(S.b, big);
    group_merge<G>(S);
    c.x = axis_coef(a.tx, val(S.t), a.ct, a.bx, val(S.b), a.cb, ig);
  }
  {
    AxisSums<C> S = {sums_start<C>(big), sums_start<C>(big)};
#pragma unroll
    for (int j = 0; j < kPinsPerLane; ++j)
      if (lg + G * j < d)
        sums_axis(S, pc[j].top, pc[j].uy, pc[j].top ? a.ty.max1 : a.by.max1, pc[j].top ? a.ty.min1 : a.by.min1, ig);
    for (int k = lg + G * kPinsPerLane; k < d; k += G) {
      const PinRel p = load_pin(xyzp, pin_node, off, s + k, half_dz, xa, ya);
      sums_axis(S, p.top, p.uy, p.top ? a.ty.max1 : a.by.max1, p.top ? a.ty.min1 : a.by.min1, ig);
    }
    sums_settle(S.t, big); sums_settle(S.b, big);
    group_merge<G>(S);
    c.y = axis_coef(a.ty, val(S.t), a.ct, a.by, val(S.b), a.cb, ig);
  }
  {
    Sums4<C> S = sums_start<C>(big);
#pragma unroll
    for (int j = 0; j < kPinsPerLane; ++j)
      if (lg + G * j < d) sums_z(S, a, pc[j], ig);
    for (int k = lg + G * kPinsPerLane; k < d; k += G) sums_z(S, a, load_pin(xyzp, pin_node, off, s + k, half_dz, xa, ya), ig);
    sums_settle(S, big);
    group_merge<G>(S);
    const Sums4v sz = val(S);
    c.az_p = rcp(sz.sp); c.Az_p = sz.tp * c.az_p;
    c.az_m = rcp(sz.sm); c.Az_m = sz.tm * c.az_m;
  }
  c.zmax = a.zmax; c.zmin = a.zmin;
  c.Wx = w_exact(a.tx.max1, a.tx.min1, a.ct, a.bx.max1, a.bx.min1, a.cb);
  c.Wy = w_exact(a.ty.max1, a.ty.min1, a.ct, a.by.max1, a.by.min1, a.cb);

  // ---- phase C: per-pin results, written at the pin's node-ordered position
  if constexpr (kGrad) {
#pragma unroll
    for (int j = 0; j < kPinsPerLane; ++j)
      if (lg + G * j < d) pin_out[slot_pos[s + lg + G * j]] = pin_result(pc[j], a, c, ig, alpha, four_over_dz);
    for (int k = lg + G * kPinsPerLane; k < d; k += G)
      pin_out[slot_pos[s + k]] =
          pin_result(load_pin(xyzp, pin_node, off, s + k, half_dz, xa, ya), a, c, ig, alpha, four_over_dz);
  }

  // ---- net totals, from the group's first lane
  NetTotals t = {0.f, 0.f, 0.f, 0.f, 0.f};
  if (lg == 0) {
    t.wa_bi = c.x.W + c.y.W;
    t.wa_z = alpha * ((a.zmax - a.zmin) + (c.Az_p - c.Az_m));
    t.hpwl = c.Wx + c.Wy;
    t.hpwl3d = (fmaxf(a.tx.max1, a.bx.max1) - fminf(a.tx.min1, a.bx.min1)) +
               (fmaxf(a.ty.max1, a.by.max1) - fminf(a.ty.min1, a.by.min1)) + alpha * (a.zmax - a.zmin);
    t.ncut = (a.ct > 0 && a.cb > 0) ? 1.f : 0.f;
  }
  return t;
}

// tanh(x/2) for x >= 0: below x = 1/2 its Taylor series to the y^9 term (y = x/2; the first term
// left out is under 1e-8 of the value there), else (1 - e^{-x}) / (1 + e^{-x}), which no longer
// cancels badly
__device__ __forceinline__ float tanh_half(float x) {
  const float y = 0.5f * x, y2 = y * y;
  const float ser = y * (1.f + y2 * (-1.f / 3.f + y2 * (2.f / 15.f + y2 * (-17.f / 315.f + y2 * (62.f / 2835.f)))));
  const float e = __expf(-x);
  return x < 0.5f ? ser : (1.f - e) * rcp(1.f + e);
}

// A two-pin net in closed form.  With D = u_p - u_q, a = |D| and x = a/gamma every exponential sum
// above is 1 + e^{-x}, so the smoothed extent is W = a tanh(x/2) and dW/du_p = sign(D) (tanh(x/2) +
// x (1 - tanh^2(x/2)) / 2) = -dW/du_q.  A crossing two-pin net has one pin per set, each set's
// extent is 0, and W^ is the whole-net W, as for a net on one die; moving either pin to the other
// die gives the exact extent |f - u_other| in both cases.
struct PairAxis { float W, g; };
__device__ __forceinline__ PairAxis pair_axis(float D, float ig) {
  const float a = fabsf(D), x = a * ig, th = tanh_half(x);
  const float g = th + 0.5f * x * (1.f - th * th);
  return {a * th, D >= 0.f ? g : -g};
}

template <bool kGrad>
__device__ __forceinline__ NetTotals wl_pair(int s, float half_dz, float four_over_dz, float ig, float alpha,
                                             const float4* __restrict__ xyzp, const int32_t* __restrict__ pin_node,
                                             const float4* __restrict__ off, const int32_t* __restrict__ slot_pos,
                                             float4* __restrict__ pin_out) {
  const float4 q0 = xyzp[pin_node[s]];
  const PinRel p = load_pin(xyzp, pin_node, off, s, half_dz, q0.x, q0.y);
  const PinRel q = load_pin(xyzp, pin_node, off, s + 1, half_dz, q0.x, q0.y);
  const float dx = p.ux - q.ux, dy = p.uy - q.uy, dz = p.z - q.z;
  const PairAxis ax = pair_axis(dx, ig), ay = pair_axis(dy, ig), az = pair_axis(dz, ig);
  const float hx = fabsf(dx), hy = fabsf(dy);
  if constexpr (kGrad) {
    const float dwp = (fabsf(p.fx - q.ux) - hx) + (fabsf(p.fy - q.uy) - hy);
    const float dwq = (fabsf(q.fx - p.ux) - hx) + (fabsf(q.fy - p.uy) - hy);
    pin_out[slot_pos[s]] = make_float4(ax.g, ay.g, alpha * az.g, four_over_dz * (p.top ? -dwp : dwp));
    pin_out[slot_pos[s + 1]] = make_float4(-ax.g, -ay.g, -(alpha * az.g), four_over_dz * (q.top ? -dwq : dwq));
  }
  NetTotals t;
  t.wa_bi = ax.W + ay.W;
  t.wa_z = alpha * az.W;
  t.hpwl = hx + hy;
  t.hpwl3d = (hx + hy) + alpha * fabsf(dz);
  t.ncut = p.top != q.top ? 1.f : 0.f;
  return t;
}

template <bool kGrad, bool C>
__global__ __launch_bounds__(kWaBlock) void k_wl_nets(
    float half_dz, float four_over_dz, float gamma, float alpha, const float4* __restrict__ xyzp,
    const int32_t* __restrict__ s_net_start, const int32_t* __restrict__ pin_node, const float4* __restrict__ off,
    const int32_t* __restrict__ slot_pos, float4* __restrict__ pin_out, ClassTab tab,
    const int32_t* __restrict__ block_order, double* __restrict__ part, int stride) {
  __shared__ double shred[5][kWaBlock / kWave];
  // workgroups run in netlist order of their first net; each die takes a contiguous range
  const int blk = block_order[xcd_swizzle((int)blockIdx.x, (int)gridDim.x)];
  int pos = 0;                                     // layout position of this block's class
  while (pos + 1 < kNumClasses && blk >= tab.block_begin[pos + 1]) ++pos;
  const int lg2 = pos < kNumGroups ? kNumGroups - 1 - pos : 0;   // log2 of the group width
  const int net = tab.net_begin[pos] + (blk - tab.block_begin[pos]) * (kWaBlock >> lg2) + ((int)threadIdx.x >> lg2);
  const int lg = threadIdx.x & ((1 << lg2) - 1);
  const float ig = 1.f / gamma;
  int ge;
  (void)frexpf(gamma, &ge);
  const float big = ldexpf(1.f, ge);               // a power of two above gamma
  NetTotals t = {0.f, 0.f, 0.f, 0.f, 0.f};
  if (net < tab.net_begin[pos + 1]) {
#define P3D_GROUP(G) \
  wl_group<G, kGrad, C>(net, lg, half_dz, four_over_dz, ig, big, alpha, xyzp, s_net_start, pin_node, off, slot_pos, pin_out)
    if (pos == kNumClasses - 1) {
      // the class's slots are consecutive, two per net: the first pin's slot follows from the
      // class's first slot (one uniform load) without a per-net load
      const int c0 = tab.net_begin[pos];
      const int s = __builtin_amdgcn_readfirstlane(s_net_start[c0]) + 2 * (net - c0);
      t = wl_pair<kGrad>(s, half_dz, four_over_dz, ig, alpha, xyzp, pin_node, off, slot_pos, pin_out);
    } else switch (lg2) {
      case 0: t = P3D_GROUP(1); break;
      case 1: t = P3D_GROUP(2); break;
      case 2: t = P3D_GROUP(4); break;
      case 3: t = P3D_GROUP(8); break;
      case 4: t = P3D_GROUP(16); break;
      case 5: t = P3D_GROUP(32); break;
      default: t = P3D_GROUP(64); break;
    }
#undef P3D_GROUP
  }
  // net totals: summed over the wavefront (at most 64 nets; in float64 when compensated), float64
  // across wavefronts
  const float v[5] = {t.wa_bi, t.wa_z, t.hpwl, t.hpwl3d, t.ncut};
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const double x = wave_sum<C>(v[q]);
    if ((threadIdx.x & (kWave - 1)) == 0) shred[q][threadIdx.x / kWave] = x;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    double x = 0.0;
    for (int w = 0; w < kWaBlock / kWave; ++w) x += shred[threadIdx.x][w];
    part[(size_t)(R_WA_BI + threadIdx.x) * stride + blk] = x;
  }
}

__global__ void k_pack_xyz(int n, const float* __restrict__ xyz, float4* __restrict__ xyzp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) xyzp[i] = make_float4(xyz[i], xyz[n + i], xyz[2 * n + i], 0.f);
}

// per instance: sum its pin shares (contiguous, ascending slot order); L1 norms over movable
// instances.  Blocks [0, nlight) take one instance per thread; instances with more than
// kHeavyPins pins are left to the blocks after them, one wavefront per instance.
constexpr int kHeavyPins = 32;

__global__ void k_wl_gather(int n, int nlight, const int32_t* __restrict__ heavy, int nheavy,
                            const uint8_t* __restrict__ kind, const int32_t* __restrict__ node_slot_start,
                            const float4* __restrict__ pin_out, float* __restrict__ grad, int accumulate,
                            const double* __restrict__ dscale, float* __restrict__ gz_wa, float* __restrict__ fda,
                            double* __restrict__ part, int stride) {
  __shared__ double sh[3][256 / kWave];
  float gx = 0.f, gy = 0.f, gz = 0.f, gf = 0.f;
  int i = -1;
  bool writer = false;
  if ((int)blockIdx.x < nlight) {
    i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
      // the kind with the slot range, and the shares four at a time, so that loads overlap
      const int q0 = node_slot_start[i], q1 = node_slot_start[i + 1];
      const uint8_t kd = kind[i];
      writer = q1 - q0 <= kHeavyPins;
      if (writer & !(kd & PLACE3D_KIND_FIXED))
        for (int q = q0; q < q1; q += 4) {
          float4 v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = q + u < q1 ? pin_out[q + u] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (q + u < q1) { gx += v[u].x; gy += v[u].y; gz += v[u].z; gf += v[u].w; }
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
    const float sc = dscale ? (float)dscale[0] : 1.f;     // the caller's factor (a vjp's incoming gradient)
    if (accumulate) { grad[i] += sc * gx; grad[n + i] += sc * gy; }
    else { grad[i] = sc * gx; grad[n + i] = sc * gy; }
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

// grad_z (+)= sc (scale * fda + gz_wa), scale = (|g_x|_1 + |g_y|_1) / (2 |fda|_1); without the FDA
// term (with_fda == 0) grad_z (+)= sc gz_wa, the derivative of the model's value
__global__ void k_wl_finish_z(int n, const float* __restrict__ gz_wa, const float* __restrict__ fda,
                              const double* __restrict__ red, int with_fda, const double* __restrict__ dscale,
                              float* __restrict__ grad, int accumulate, double* __restrict__ metrics) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const float scale = (float)fda_scale(red);
  if (i < n) {
    const float sc = dscale ? (float)dscale[0] : 1.f;
    const float v = sc * (with_fda ? scale * fda[i] + gz_wa[i] : gz_wa[i]);
    if (accumulate) grad[2 * n + i] += v; else grad[2 * n + i] = v;
  }
  if (metrics && i < PLACE3D_NMETRICS) {
    double v = 0.0;
    if (i <= PLACE3D_M_NORM_FDA) v = red[R_WA_BI + i];
    else if (i == PLACE3D_M_FDA_SCALE) v = fda_scale(red);
    metrics[i] = v;
  }
}

__device__ __forceinline__ void set_put(float& mx, float& mn, float u) {
  mx = fmaxf(mx, u);
  mn = fminf(mn, u);
}

// The FDA difference of the instance owning slot s on its net (slots [b, e)), re-evaluated from
// all the net's pins: the exact bistratal wirelength with every pin of that instance on the top
// die minus that with every one on the bottom die, times 4/d_z (Eq. fda-grad is per instance).
// 0 when an earlier slot of the net has the same owner: the instance counts once per net.
// Coordinates are relative to the net's first owner, as in k_wl_nets.
__device__ float fda_owner(int s, int b, int e, float half_dz, float four_over_dz, const float4* __restrict__ xyzp,
                           const int32_t* __restrict__ pin_node, const float4* __restrict__ off) {
  const int own = pin_node[s];
  for (int q = b; q < s; ++q)
    if (pin_node[q] == own) return 0.f;
  const float4 q0 = xyzp[pin_node[b]];
  const float xa = q0.x, ya = q0.y;
  float txM = kNegInf, txm = kPosInf, tyM = kNegInf, tym = kPosInf;   // other owners' pins, on
  float bxM = kNegInf, bxm = kPosInf, byM = kNegInf, bym = kPosInf;   // their own dies
  float otxM = kNegInf, otxm = kPosInf, otyM = kNegInf, otym = kPosInf;   // the owner's pins on top
  float obxM = kNegInf, obxm = kPosInf, obyM = kNegInf, obym = kPosInf;   // and on the bottom
  int ct = 0, cb = 0, co = 0;
  for (int q = b; q < e; ++q) {
    const PinRel p = load_pin(xyzp, pin_node, off, q, half_dz, xa, ya);
    if (pin_node[q] == own) {
      set_put(otxM, otxm, p.top ? p.ux : p.fx); set_put(otyM, otym, p.top ? p.uy : p.fy);
      set_put(obxM, obxm, p.top ? p.fx : p.ux); set_put(obyM, obym, p.top ? p.fy : p.uy);
      ++co;
    } else if (p.top) {
      set_put(txM, txm, p.ux); set_put(tyM, tym, p.uy); ++ct;
    } else {
      set_put(bxM, bxm, p.ux); set_put(byM, bym, p.uy); ++cb;
    }
  }
  const float wx_top = w_exact(fmaxf(txM, otxM), fminf(txm, otxm), ct + co, bxM, bxm, cb);
  const float wy_top = w_exact(fmaxf(tyM, otyM), fminf(tym, otym), ct + co, byM, bym, cb);
  const float wx_bot = w_exact(txM, txm, ct, fmaxf(bxM, obxM), fminf(bxm, obxm), cb + co);
  const float wy_bot = w_exact(tyM, tym, ct, fmaxf(byM, obyM), fminf(bym, obym), cb + co);
  return four_over_dz * ((wx_top - wx_bot) + (wy_top - wy_bot));
}

// Vanilla FDA (the O(|P_e|^2) baseline of Sec. IV-B, selected by PLACE3D_OPT_FDA_VANILLA): one
// thread per pin slot re-evaluates its owner's difference from all |P_e| pins (fda_owner) and
// overwrites the FDA value k_wl_nets stored for the slot.
__global__ __launch_bounds__(256) void k_fda_vanilla(int nslots, int nnets, float half_dz, float four_over_dz,
                                                     const float4* __restrict__ xyzp,
                                                     const int32_t* __restrict__ s_net_start,
                                                     const int32_t* __restrict__ pin_node,
                                                     const float4* __restrict__ off,
                                                     const int32_t* __restrict__ slot_pos,
                                                     float4* __restrict__ pin_out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  int lo = 0, hi = nnets - 1;                    // the net holding slot s: last e with start <= s
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_net_start[mid] <= s) lo = mid; else hi = mid - 1;
  }
  pin_out[slot_pos[s]].w =
      fda_owner(s, s_net_start[lo], s_net_start[lo + 1], half_dz, four_over_dz, xyzp, pin_node, off);
}

// Nets holding an instance on more than one pin (listed at create, in schedule numbering): the
// incremental FDA of k_wl_nets flips one pin at a time, so these nets' FDA values are redone per
// instance, one wavefront per net.
__global__ __launch_bounds__(256) void k_fda_shared(const int32_t* __restrict__ nets, int nnets, float half_dz,
                                                    float four_over_dz, const float4* __restrict__ xyzp,
                                                    const int32_t* __restrict__ s_net_start,
                                                    const int32_t* __restrict__ pin_node,
                                                    const float4* __restrict__ off,
                                                    const int32_t* __restrict__ slot_pos,
                                                    float4* __restrict__ pin_out) {
  const int w = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (w >= nnets) return;
  const int k = nets[w], b = s_net_start[k], e = s_net_start[k + 1];
  for (int s = b + (int)(threadIdx.x & (kWave - 1)); s < e; s += kWave)
    pin_out[slot_pos[s]].w = fda_owner(s, b, e, half_dz, four_over_dz, xyzp, pin_node, off);
}

}  // namespace

int wirelength_eval(place3d_ctx* c, const float* xyz, float* grad, int accumulate, double* red,
                    double* metrics, hipStream_t s, bool packed, const double* dscale, bool with_fda) {
  const Geom& g = c->g;
  const place3d_problem& p = c->prob;
  const bool comp = p.precision == PLACE3D_BF16X3;      // the precision form compensates the sums
  int rc;
  if (c->n_wa_blocks > 0) {
    if (!packed) {
      ProfScope prof_(c, PLACE3D_STAGE_WL_NODES, s);
      hipLaunchKernelGGL(k_pack_xyz, dim3(blocks_for(g.n, 256)), dim3(256), 0, s, g.n, xyz, c->xyzp);
      P3D_LAUNCH(c, "k_pack_xyz");
    }
    ProfScope prof_(c, PLACE3D_STAGE_WL_NETS, s);
    auto kern = comp ? k_wl_nets<true, true> : k_wl_nets<true, false>;
    hipLaunchKernelGGL(kern, dim3(c->n_wa_blocks), dim3(kWaBlock), 0, s, g.half_dz, 4.f / g.dz, (float)p.gamma,
                       (float)p.alpha, c->xyzp, c->s_net_start, c->s_pin_node, c->s_off, c->slot_pos, c->pin_out,
                       c->classes, c->wa_block_order, c->part, c->part_stride);
    P3D_LAUNCH(c, "k_wl_nets");
    if (p.options & PLACE3D_OPT_FDA_VANILLA) {
      const int nslots = p.n_pins, nnets = c->classes.net_begin[kNumClasses];
      hipLaunchKernelGGL(k_fda_vanilla, dim3(blocks_for(nslots, 256)), dim3(256), 0, s, nslots, nnets, g.half_dz,
                         4.f / g.dz, c->xyzp, c->s_net_start, c->s_pin_node, c->s_off, c->slot_pos, c->pin_out);
      P3D_LAUNCH(c, "k_fda_vanilla");
    } else if (c->n_shared_nets > 0) {
      hipLaunchKernelGGL(k_fda_shared, dim3(blocks_for(c->n_shared_nets, 256 / kWave)), dim3(256), 0, s,
                         c->shared_nets, c->n_shared_nets, g.half_dz, 4.f / g.dz, c->xyzp, c->s_net_start,
                         c->s_pin_node, c->s_off, c->slot_pos, c->pin_out);
      P3D_LAUNCH(c, "k_fda_shared");
    }
  }
  if ((rc = reduce_final(c, R_WA_BI, 5, c->n_wa_blocks, false, red + R_WA_BI, s))) return rc;
  const unsigned nlight = blocks_for(g.n, 256);
  const unsigned nb = nlight + (unsigned)((c->n_heavy + 3) / 4);
  {
    ProfScope prof_(c, PLACE3D_STAGE_WL_NODES, s);
    hipLaunchKernelGGL(k_wl_gather, dim3(nb), dim3(256), 0, s, g.n, (int)nlight, c->heavy_list, c->n_heavy, p.kind,
                       c->node_slot_start, c->pin_out, grad, accumulate, dscale, c->wl_gzwa, c->wl_fda, c->part,
                       c->part_stride);
    P3D_LAUNCH(c, "k_wl_gather");
  }
  if ((rc = reduce_final(c, R_NORM_X, 3, (int)nb, false, red + R_NORM_X, s))) return rc;
  {
    ProfScope prof_(c, PLACE3D_STAGE_WL_NODES, s);
    hipLaunchKernelGGL(k_wl_finish_z, dim3(blocks_for(std::max(g.n, (int)PLACE3D_NMETRICS), 256)), dim3(256), 0, s,
                       g.n, c->wl_gzwa, c->wl_fda, red, with_fda ? 1 : 0, dscale, grad, accumulate, metrics);
    P3D_LAUNCH(c, "k_wl_finish_z");
  }
  return PLACE3D_OK;
}

int wirelength_value(place3d_ctx* c, const float* xyz, double* metrics, hipStream_t s, float4* xyzp, double* part,
                     int stride) {
  const Geom& g = c->g;
  const place3d_problem& p = c->prob;
  const bool comp = p.precision == PLACE3D_BF16X3;
  if (!xyzp) { xyzp = c->xyzp; part = c->part; stride = c->part_stride; }
  int rc;
  if (c->n_wa_blocks > 0) {
    {
      ProfScope prof_(c, PLACE3D_STAGE_WL_NODES, s);
      hipLaunchKernelGGL(k_pack_xyz, dim3(blocks_for(g.n, 256)), dim3(256), 0, s, g.n, xyz, xyzp);
      P3D_LAUNCH(c, "k_pack_xyz");
    }
    ProfScope prof_(c, PLACE3D_STAGE_WL_NETS, s);
    auto kern = comp ? k_wl_nets<false, true> : k_wl_nets<false, false>;
    hipLaunchKernelGGL(kern, dim3(c->n_wa_blocks), dim3(kWaBlock), 0, s, g.half_dz, 4.f / g.dz, (float)p.gamma,
                       (float)p.alpha, xyzp, c->s_net_start, c->s_pin_node, c->s_off, c->slot_pos, c->pin_out,
                       c->classes, c->wa_block_order, part, stride);
    P3D_LAUNCH(c, "k_wl_nets(value)");
  }
  // the five net totals straight into the metrics; the gradient norms are not computed here
  if ((rc = launch_zero_f64(c, metrics, PLACE3D_NMETRICS, s))) return rc;
  return reduce_final_in(c, part, stride, R_WA_BI, 5, c->n_wa_blocks, false, metrics + PLACE3D_M_WA_BI, s);
}

// ---- the value call without workspace scratch (place3d_wl_value_static)
//
// Its per-call scratch lives in this array instead of the context's workspace: the packed
// positions (16 B per instance) and one float64 partial per wirelength workgroup for each of the
// five net totals.  Every GPU the library runs on holds its own copy until the process ends.
// Host code never passes the array's name to a kernel (on the host it is only a stand-in): the
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kStaticPosBytes = size_t(kStaticMaxInst) * sizeof(float4);
constexpr size_t kStaticPartBytes = size_t(5 + R_WA_BI) * kStaticMaxBlocks * sizeof(double);
static __device__ __align__(256) unsigned char scratch[kStaticPosBytes + kStaticPartBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int static_scratch_setup(place3d_ctx* c, void** out) {
  int dev = -1;
  P3D_HIP(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_err(c, PLACE3D_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    P3D_HIP(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255))
      return set_err(c, PLACE3D_ERR_HIP, "static scratch: no 256-byte aligned device address");
    g_scratch_ptr[dev] = ptr;
  }
  if (out) *out = g_scratch_ptr[dev];
  return PLACE3D_OK;
}

int wirelength_value_static(place3d_ctx* c, const float* xyz, double* metrics, hipStream_t s) {
  if (c->g.n > kStaticMaxInst)
    return set_err(c, PLACE3D_ERR_SIZE, "place3d_wl_value_static: more than " + std::to_string(kStaticMaxInst) +
                                            " instances (its static scratch holds that many positions)");
  if (c->n_wa_blocks > kStaticMaxBlocks)
    return set_err(c, PLACE3D_ERR_SIZE, "place3d_wl_value_static: more than " + std::to_string(kStaticMaxBlocks) +
                                            " wirelength workgroups (its static scratch holds that many partials)");
  void* base = nullptr;
  if (int rc = static_scratch_setup(c, &base)) return rc;
  // every word of the scratch that is read is written first by the same call (positions by the
  // pack pass, one partial per workgroup and total by the net pass), so nothing is cleared
  float4* xyzp = reinterpret_cast<float4*>(base);
  double* part = reinterpret_cast<double*>(reinterpret_cast<char*>(base) + kStaticPosBytes);
  return wirelength_value(c, xyz, metrics, s, xyzp, part, kStaticMaxBlocks);
}

}  // namespace p3d
