// Split-bfloat16 chain of the folded spectral Poisson solve (Sec. III-A, Eqs. density-coef,
// poisson-sol-potential, possion-sol-force): the contractions of the float32 path, with every
// operand held in HBM as bfloat16 hi / lo planes (hi = RNE(v), lo = RNE(v - hi)) and each
// product taken as hi.hi + hi.lo + lo.hi with float32 accumulation.
//
// Each contraction is C[m][n] = sum_k A[m][k] B[n][k] over two plane pairs with k padded to a
// multiple of 32 with zeros and blocked by 32: element (row, k) of a plane of R rows sits at
// ((k / 32) R + row) 32 + k % 32, so that one k step of consecutive rows is one contiguous run
// and an epilogue's rows are written as contiguous runs.  Operand tiles go from HBM straight into LDS
// (global_load_lds_dwordx4, no register staging, no conversion) through a ring of kStages
// stages, so that loads run several k steps ahead of the matrix cores.  What the float32 path
// does in separate passes happens in the epilogues, from the accumulators:
//   pre-pass  rho -> x-folded sum / difference planes (split)
//   x forward  T = S . Fx_even, D . Fx_odd; epilogue folds T about the y middle and writes the
//              y-folded planes transposed, [z][x frequency][y]
//   y forward  A = Fy_even . T_sum, Fy_odd . T_diff per (z, x frequency); epilogue mixes z
//              (Fz), divides by |omega|^2 and writes the coefficients [l][x frequency][y frequency]
//   y inverse  V = Gy . b, Hy . b (even and odd frequency halves into two accumulators);
//              epilogue unfolds y and writes V transposed, [z frequency][y][x frequency]
//   x inverse  E = V . Gx_even, O = V . Gx_odd (two accumulators); epilogue unfolds x and mixes
//              z (Gz or Hz), which commutes with the x contraction
// Rows of a tile are chosen so that everything an epilogue combines sits in one lane's
// accumulator registers or in the lane 32 apart: the y fold pairs a row with its mirror across
// lane halves, the z mixing keeps the layers of a point in one lane (x inverse, layers in the
// register quads) or in one group of adjacent lanes (y forward, exchanged by DPP).
#include <cmath>

#include "internal.h"

namespace p3d {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

constexpr int kTile = 128;          // output tile is 128 x 128, four 64 x 64 wavefront tiles
constexpr int kStep = 32;           // k per stage

enum Kind { XF = 0, YF = 1, YI = 2, XI = 3 };

// two values to packed bfloat16 {hi, lo} (hardware round to nearest even)
__device__ __forceinline__ u32x2 split2(float a, float b) {
  const f32x2 x = {a, b};
  const unsigned hp = __builtin_bit_cast(unsigned, __builtin_convertvector(x, bf16x2v));
  const f32x2 back = {__uint_as_float(hp << 16), __uint_as_float(hp & 0xffff0000u)};
  return (u32x2){hp, __builtin_bit_cast(unsigned, __builtin_convertvector(x - back, bf16x2v))};
}

__device__ __forceinline__ unsigned short rne16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

struct SJob {
  const uint16_t *ah, *al, *bh, *bl;   // operand planes
  int koa, kob;                        // k offsets into the rows of A and B
  int sel;                             // which half / basis the job computes (per kind)
  uint16_t *oh0, *ol0, *oh1, *ol1;     // split outputs
  float* of;                           // float32 output (x inverse)
  float sg;                            // x inverse: parity sign of the basis (-1 sine, +1 cosine)
};

constexpr int kMaxJobs = 8;

struct SArgs {
  int ntm, ntn, ksteps;
  int ra, rb, ro;                      // rows of the A, B and split output planes
  int nx, ny, nz, hx, hy, rx, ry;
  float px, py, pz;                    // pi / length per axis
  const float* zmat;
  SJob job[kMaxJobs];
};

// ------------------------------------------------------------------ tile rows

// global row of A for local row r of m tile tm
template <int KIND, int NZ>
__device__ __forceinline__ int a_row(const SArgs& g, int tm, int r) {
  if constexpr (KIND == XF) {
    // 64 mirror pairs of one layer: 32-row group t holds y' = yp0 + 16 t + (r & 3 | (r >> 3) << 2)
    // on bit 2 clear and its mirror ny - 1 - y' on bit 2 set
    const int nyt = (g.hy + 63) / 64, z = tm / nyt, yp0 = (tm % nyt) * 64;
    const int t = r >> 5, b = r & 31;
    int yp = yp0 + 16 * t + ((b & 3) | ((b >> 3) << 2));
    yp = yp < g.hy ? yp : g.hy - 1;
    const int y = ((b >> 2) & 1) ? g.ny - 1 - yp : yp;
    return z * g.ny + y;
  } else if constexpr (KIND == YF) {
    const int k = tm * kTile + r;
    return k < g.hy ? k : g.hy - 1;
  } else if constexpr (KIND == YI) {
    // 32-row group t: bits 3-4 of the row = register quad = layer (and, for NZ < 4, the high x
    // bits), bits 0-2 = x frequency
    const int t = r >> 5, b = r & 31, q = b >> 3;
    const int l = q % NZ, kx0 = tm * (kTile / NZ) + t * (32 / NZ);
    int kx = kx0 + ((b & 7) | ((q / NZ) << 3));
    kx = kx < g.nx ? kx : g.nx - 1;
    return kx * NZ + l;
  } else {
    // the same layout over (z frequency, y): the layers of a point in one lane's register quads
    const int t = r >> 5, b = r & 31, q = b >> 3;
    const int l = q % NZ, y0 = tm * (kTile / NZ) + t * (32 / NZ);
    int y = y0 + ((b & 7) | ((q / NZ) << 3));
    y = y < g.ny ? y : g.ny - 1;
    return l * g.ny + y;
  }
}

// global row of B for local column c of n tile tn
template <int KIND, int NZ>
__device__ __forceinline__ int b_row(const SArgs& g, int tn, int c) {
  if constexpr (KIND == YF) {
    // layers of one x frequency in adjacent columns
    int kx = tn * (kTile / NZ) + c / NZ;
    kx = kx < g.nx ? kx : g.nx - 1;
    return (c % NZ) * g.nx + kx;
  } else {
    const int lim = KIND == YI ? g.hy : g.hx;
    const int n = tn * kTile + c;
    return n < lim ? n : lim - 1;
  }
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// value of lane (group base + z) of a group of NZ adjacent lanes
template <int NZ, int Z>
__device__ __forceinline__ float group_lane(float v) {
  if constexpr (NZ == 2) return dpp<Z == 0 ? 0xA0 : 0xF5>(v);   // quad_perm (0,0,2,2) / (1,1,3,3)
  else return dpp<Z * 0x55>(v);                                 // quad_perm (Z,Z,Z,Z)
}

// 16 bytes per lane from global memory into LDS: lane i fills bytes [16 i, 16 i + 16) of the
// wavefront's 1 KiB at dst (the LDS address is wavefront-uniform)
__device__ __forceinline__ void lds_load16(const uint16_t* src, unsigned short* dst) {
  __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
}

// 1 / |omega|^2 by the hardware reciprocal (1 ulp, far below the split products' rounding); the
// (0,0,0) mode is dropped
__device__ __forceinline__ float inv_w2(const SArgs& g, int j, int k, int l) {
  const float wx = g.px * (float)j, wy = g.py * (float)k, wz = g.pz * (float)l;
  const float w2 = wx * wx + wy * wy + wz * wz;
  return w2 > 0.f ? __builtin_amdgcn_rcpf(w2) : 0.f;
}

// the value of lane l ^ 32 (the other half of the wavefront), by one lane-half swap
__device__ __forceinline__ float other_half(float v, bool upper) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(upper ? r[0] : r[1]);
}

__device__ __forceinline__ int xfreq(int pos, int h) { return pos < h ? 2 * pos : 2 * (pos - h) + 1; }

// ------------------------------------------------------------------ contraction

// kStages: LDS ring depth (32 KiB per stage)
template <int KIND, int NZ, int kStages>
__global__ __launch_bounds__(256) void k_sgemm(SArgs g) {
  constexpr bool DUAL = KIND == YI || KIND == XI;
  // stage s: [0] A hi, [1] A lo, [2] B hi, [3] B lo, each 128 rows of 32 bfloat16 (four 16-byte
  // units); unit u of row r sits at position u ^ ((r >> 1) & 3), so that the MFMA fragment reads
  // (8 consecutive rows, one unit) touch distinct banks
  __shared__ __attribute__((aligned(16))) unsigned short L[kStages][4][kTile][kStep];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wm = w >> 1, wn = w & 1;
  int tm, tn, jb;
  {
    const int x = xcd_swizzle((int)blockIdx.x, (int)gridDim.x);
    if constexpr (KIND == YF) {   // m tiles fastest: they share the data tile of B
      tm = x % g.ntm; tn = (x / g.ntm) % g.ntn; jb = x / (g.ntm * g.ntn);
    } else {                      // n tiles fastest: they share the data tile of A
      tn = x % g.ntn; tm = (x / g.ntn) % g.ntm; jb = x / (g.ntm * g.ntn);
    }
  }
  const SJob J = g.job[jb];
  const int KT = g.ksteps;

  // each wavefront streams rows [32 w, 32 w + 32) of the four arrays, 16 rows (1 KiB) per
  // instruction: lane i fills row 32 w + 16 j + i / 4 at position i % 4
  const int lr = w * 32 + (lane >> 2);
  const int unit = (lane & 3) ^ ((lr >> 1) & 3);   // the same for row lr + 16
  const size_t sa = (size_t)g.ra * kStep, sb = (size_t)g.rb * kStep;   // one k block of A, of B
  const size_t oa0 = (J.koa / kStep) * sa + (size_t)a_row<KIND, NZ>(g, tm, lr) * kStep + 8 * unit;
  const size_t oa1 = (J.koa / kStep) * sa + (size_t)a_row<KIND, NZ>(g, tm, lr + 16) * kStep + 8 * unit;
  const size_t ob0 = (J.kob / kStep) * sb + (size_t)b_row<KIND, NZ>(g, tn, lr) * kStep + 8 * unit;
  const size_t ob1 = (J.kob / kStep) * sb + (size_t)b_row<KIND, NZ>(g, tn, lr + 16) * kStep + 8 * unit;
  auto issue = [&](int kt) {
    const int st = kt % kStages;
    const size_t ka = kt * sa, kb = kt * sb;
    unsigned short* d = &L[st][0][w * 32][0];   // [0] A hi; the arrays are kTile * kStep apart
    constexpr int ARR = kTile * kStep;
    lds_load16(J.ah + oa0 + ka, d);
    lds_load16(J.ah + oa1 + ka, d + 16 * kStep);
    lds_load16(J.al + oa0 + ka, d + ARR);
    lds_load16(J.al + oa1 + ka, d + ARR + 16 * kStep);
    lds_load16(J.bh + ob0 + kb, d + 2 * ARR);
    lds_load16(J.bh + ob1 + kb, d + 2 * ARR + 16 * kStep);
    lds_load16(J.bl + ob0 + kb, d + 3 * ARR);
    lds_load16(J.bl + ob1 + kb, d + 3 * ARR + 16 * kStep);
  };
  constexpr int kLoadsPerStage = 8;

  f32x16 acc[2][2][2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[h][a][b] = (f32x16)(0.f);

  auto mma = [&](int st, f32x16 (&C)[2][2]) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const int u = 2 * kk + (lane >> 5);
      bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int ar = wm * 64 + t * 32 + (lane & 31), br = wn * 64 + t * 32 + (lane & 31);
        const int pa = 8 * (u ^ ((ar >> 1) & 3)), pb = 8 * (u ^ ((br >> 1) & 3));
        ah[t] = *reinterpret_cast<const bf16x8*>(&L[st][0][ar][pa]);
        al[t] = *reinterpret_cast<const bf16x8*>(&L[st][1][ar][pa]);
        bh[t] = *reinterpret_cast<const bf16x8*>(&L[st][2][br][pb]);
        bl[t] = *reinterpret_cast<const bf16x8*>(&L[st][3][br][pb]);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          C[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], C[a][b], 0, 0, 0);
          C[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], C[a][b], 0, 0, 0);
          C[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], C[a][b], 0, 0, 0);
        }
    }
  };
  // Stage kt is waited for by count: the loads of the kStages - 2 later stages may still be in
  // flight.  The barrier carries no memory fence (which would wait for every load into LDS);
  // reads of a stage all feed MFMAs before the wavefront reaches the barrier that lets the
  // stage be refilled.
  auto sync_stage = [&](int kt) {
    if (kt + kStages - 2 < KT) {
      constexpr int n = kLoadsPerStage * (kStages - 2);
      __builtin_amdgcn_s_waitcnt((n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14));
    } else {
      __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));
    }
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };

#pragma unroll
  for (int s = 0; s < kStages - 1; ++s)
    if (s < KT) issue(s);
  const int KH = DUAL ? KT / 2 : KT;
  for (int kt = 0; kt < KH; ++kt) {
    sync_stage(kt);
    if (kt + kStages - 1 < KT) issue(kt + kStages - 1);
    mma(kt % kStages, acc[0]);
  }
  if constexpr (DUAL) {
    for (int kt = KH; kt < KT; ++kt) {
      sync_stage(kt);
      if (kt + kStages - 1 < KT) issue(kt + kStages - 1);
      mma(kt % kStages, acc[1]);
    }
  }

  // ---------------------------------------------------------------- epilogues
  if constexpr (KIND == XF) {
    // lane < 32 holds rows y' = yb + r of column n, lane + 32 the mirrors; lane < 32 writes the
    // sum, lane + 32 the difference: the 32 y' of one k block (a = 0, 1) of row (z, x frequency)
    const int nyt = (g.hy + 63) / 64, z = tm / nyt, yp0 = (tm % nyt) * 64;
    const bool upper = lane >= 32;
    uint16_t* oh = upper ? J.oh1 : J.oh0;
    uint16_t* ol = upper ? J.ol1 : J.ol0;
    const int yk = yp0 + 32 * wm;   // first y' of the k block (ry and yk are multiples of 32)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int n = tn * kTile + wn * 64 + b * 32 + (lane & 31);
      u32x4 hv[4], lv[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        float v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float own = acc[0][a][b][r], oth = other_half(own, upper);
          const float sv = upper ? oth - own : own + oth;
          v[r] = yk + 16 * a + r < g.hy ? sv : 0.f;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const u32x2 t_ = split2(v[2 * e], v[2 * e + 1]);
          hv[2 * a + e / 4][e % 4] = t_[0];
          lv[2 * a + e / 4][e % 4] = t_[1];
        }
      }
      if (n < g.hx && yk < g.ry) {
        const size_t o = ((size_t)(yk / kStep) * g.ro + (size_t)(z * g.nx + J.sel * g.hx + n)) * kStep;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          *reinterpret_cast<u32x4*>(oh + o + 8 * q) = hv[q];
          *reinterpret_cast<u32x4*>(ol + o + 8 * q) = lv[q];
        }
      }
    }
  } else if constexpr (KIND == YF) {
    // column c = (x frequency kx, layer z = c % NZ); the lane's output layer is its own z:
    // b[l] = inv_w2 * sum_z Fz[z][l] A[z]; rows ky = 4 consecutive per register quad
    const int lz = lane % NZ;
    float fz[NZ];
#pragma unroll
    for (int z = 0; z < NZ; ++z) fz[z] = g.zmat[z * kMaxNz + lz];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int c = wn * 64 + b * 32 + (lane & 31);
        const int kx = tn * (kTile / NZ) + c / NZ;
        const int j = xfreq(kx, g.hx);
        float o[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float v = acc[0][a][b][r];
          float s = fz[0] * group_lane<NZ, 0>(v);
          if constexpr (NZ > 1) s += fz[1] * group_lane<NZ, 1>(v);
          if constexpr (NZ > 2) {
            s += fz[2] * group_lane<NZ, 2>(v);
            s += fz[3] * group_lane<NZ, 3>(v);
          }
          o[r] = s;
        }
        if (kx < g.nx) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int ky0 = tm * kTile + wm * 64 + a * 32 + 8 * q + 4 * (lane >> 5);
            if (ky0 >= g.ry) continue;
            float v4[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int ky = ky0 + e;
              v4[e] = ky < g.hy ? o[4 * q + e] * inv_w2(g, j, 2 * ky + J.sel, lz) : 0.f;
            }
            u32x2 hh, ll;
            { const u32x2 t_ = split2(v4[0], v4[1]); hh[0] = t_[0]; ll[0] = t_[1]; }
            { const u32x2 t_ = split2(v4[2], v4[3]); hh[1] = t_[0]; ll[1] = t_[1]; }
            const int kcol = J.sel * g.ry + ky0;
            const size_t off = ((size_t)(kcol / kStep) * g.ro + (size_t)(kx * NZ + lz)) * kStep + kcol % kStep;
            *reinterpret_cast<u32x2*>(J.oh0 + off) = hh;
            *reinterpret_cast<u32x2*>(J.ol0 + off) = ll;
          }
        }
      }
  } else if constexpr (KIND == YI) {
    // rows: register quad q -> layer q % NZ and x bits (q / NZ) << 3, register r % 4 and lane
    // half -> x bits 0-2; column = y'.  V(y') = E + O, V(ny-1-y') = E - O (cosine, sel 0) or
    // O - E (sine, sel 1).  Each side is staged in LDS as [layer][y'][x frequency] and written
    // out as whole rows (layer, y) of the blocked output.
    const bool cosine = J.sel == 0;
    constexpr int KXT = kTile / NZ;          // x frequencies of the tile
    constexpr int SR = KXT + 8;              // staged row stride (bfloat16), 16-byte multiple
    constexpr int PL = NZ * kTile * SR;      // one staged hi or lo plane
    constexpr int CH = KXT / 8;              // 16-byte chunks per staged row
    static_assert(2 * PL * 2 <= (int)sizeof(L), "staging does not fit");
    unsigned short* S = &L[0][0][0][0];
    __syncthreads();
#pragma unroll
    for (int side = 0; side < 2; ++side) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int yl = wn * 64 + b * 32 + (lane & 31);
#pragma unroll
          for (int gq = 0; gq < 4 / NZ; ++gq) {
            const int kxl = (wm * 2 + a) * (32 / NZ) + (gq << 3) + ((lane >> 5) << 2);
#pragma unroll
            for (int l = 0; l < NZ; ++l) {
              float o[4];
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const float E = acc[0][a][b][4 * (gq * NZ + l) + e], O = acc[1][a][b][4 * (gq * NZ + l) + e];
                o[e] = side == 0 ? E + O : (cosine ? E - O : O - E);
              }
              const u32x2 t0 = split2(o[0], o[1]), t1 = split2(o[2], o[3]);
              const int at = (l * kTile + yl) * SR + kxl;
              *reinterpret_cast<u32x2*>(S + at) = (u32x2){t0[0], t1[0]};
              *reinterpret_cast<u32x2*>(S + PL + at) = (u32x2){t0[1], t1[1]};
            }
          }
        }
      __syncthreads();
      // copy out: consecutive threads take consecutive 16-byte chunks of consecutive rows
      for (int idx = tid; idx < 2 * NZ * kTile * CH; idx += 256) {
        const int hl = idx / (NZ * kTile * CH), rem = idx % (NZ * kTile * CH);
        const int c = rem % CH, rl = rem / CH, l = rl / kTile, yl = rl % kTile;
        const int yp = tn * kTile + yl;
        if (yp >= g.hy) continue;
        const int y = side ? g.ny - 1 - yp : yp;
        const size_t grow = (size_t)(l * g.ny + y);
        uint16_t* dst = hl ? J.ol0 : J.oh0;
        const unsigned short* src = S + hl * PL + rl * SR + 8 * c;
        const int kx0 = tm * KXT + 8 * c;
        if (kx0 + 8 <= g.hx || (kx0 >= g.hx && kx0 + 8 <= g.nx && (g.hx & 7) == 0)) {
          const int col = kx0 < g.hx ? kx0 : g.rx + kx0 - g.hx;
          *reinterpret_cast<u32x4*>(dst + ((size_t)(col / kStep) * g.ro + grow) * kStep + col % kStep) =
              *reinterpret_cast<const u32x4*>(src);
        } else {
          for (int e = 0; e < 8; ++e) {
            const int kx = kx0 + e;
            if (kx >= g.nx) break;
            const int col = kx < g.hx ? kx : g.rx + kx - g.hx;
            dst[((size_t)(col / kStep) * g.ro + grow) * kStep + col % kStep] = src[e];
          }
        }
      }
      __syncthreads();
    }
  } else {
    // x inverse: E (even x frequencies) and O (odd) of column x' < nx/2 for the layers of a point
    // (register quads, as in the y inverse); the output rows (z, y) get Z^T (E + O) at x' and
    // sg Z^T (E - O) at the mirror nx-1-x', Z = Gz or Hz
    const float* Z = g.zmat + (J.sel ? 2 : 1) * kMaxNz * kMaxNz;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int xp = tn * kTile + wn * 64 + b * 32 + (lane & 31);
        if (xp >= g.hx) continue;
#pragma unroll
        for (int gq = 0; gq < 4 / NZ; ++gq)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int y = tm * (kTile / NZ) + (wm * 2 + a) * (32 / NZ) + (gq << 3) + ((lane >> 5) << 2) + e;
            if (y >= g.ny) continue;
            float u[NZ], v[NZ];
#pragma unroll
            for (int l = 0; l < NZ; ++l) {
              const float E = acc[0][a][b][4 * (gq * NZ + l) + e], O = acc[1][a][b][4 * (gq * NZ + l) + e];
              u[l] = E + O;
              v[l] = E - O;
            }
#pragma unroll
            for (int z = 0; z < NZ; ++z) {
              float pu = 0.f, pv = 0.f;
#pragma unroll
              for (int l = 0; l < NZ; ++l) {
                pu += Z[l * kMaxNz + z] * u[l];
                pv += Z[l * kMaxNz + z] * v[l];
              }
              float* row = J.of + (size_t)(z * g.ny + y) * g.nx;
              row[xp] = pu;
              row[g.nx - 1 - xp] = J.sg * pv;
            }
          }
      }
  }
}

// ------------------------------------------------------------------ pre-pass and bases

// rho [Nz Ny][Nx] -> x-folded sum and difference planes (rows Nz Ny, k = x' < rx, blocked),
// split; one thread per 8 consecutive x' of a row, consecutive threads on consecutive outputs
__global__ __launch_bounds__(256) void k_fold_split_x(const float* __restrict__ rho, int rows, int nx, int hx, int rx,
                                                      uint16_t* __restrict__ sh, uint16_t* __restrict__ sl,
                                                      uint16_t* __restrict__ dh, uint16_t* __restrict__ dl) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)rows * (rx / 8)) return;
  const int per_block = rows * 4;
  const int kb = (int)(t / per_block), rem = (int)(t % per_block);
  const int row = rem >> 2, x0 = kb * 32 + (rem & 3) * 8;
  const float* src = rho + (size_t)row * nx;
  float a[8], b[8];
  if (x0 + 8 <= hx && (nx & 3) == 0) {
    const float4 a0 = *reinterpret_cast<const float4*>(src + x0);
    const float4 a1 = *reinterpret_cast<const float4*>(src + x0 + 4);
    const float4 m0 = *reinterpret_cast<const float4*>(src + nx - 8 - x0);   // mirrors of x0+7..x0+4
    const float4 m1 = *reinterpret_cast<const float4*>(src + nx - 4 - x0);   // mirrors of x0+3..x0
    a[0] = a0.x; a[1] = a0.y; a[2] = a0.z; a[3] = a0.w; a[4] = a1.x; a[5] = a1.y; a[6] = a1.z; a[7] = a1.w;
    b[0] = m1.w; b[1] = m1.z; b[2] = m1.y; b[3] = m1.x; b[4] = m0.w; b[5] = m0.z; b[6] = m0.y; b[7] = m0.x;
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int x = x0 + e;
      a[e] = x < hx ? src[x] : 0.f;
      b[e] = x < hx ? src[nx - 1 - x] : 0.f;
    }
  }
  u32x4 h, l, h2, l2;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const u32x2 ts = split2(a[2 * e] + b[2 * e], a[2 * e + 1] + b[2 * e + 1]);
    const u32x2 td = split2(a[2 * e] - b[2 * e], a[2 * e + 1] - b[2 * e + 1]);
    h[e] = ts[0]; l[e] = ts[1];
    h2[e] = td[0]; l2[e] = td[1];
  }
  const size_t o = (size_t)t * 8;
  *reinterpret_cast<u32x4*>(sh + o) = h;
  *reinterpret_cast<u32x4*>(sl + o) = l;
  *reinterpret_cast<u32x4*>(dh + o) = h2;
  *reinterpret_cast<u32x4*>(dl + o) = l2;
}

// panel (rows x width, blocked) from a float32 basis: logical k index kk = k (k < h), or for a
// dual panel kk = h + k - rp on the second half (rp <= k < rp + h); zero elsewhere.  The source
// element is src[kk][r + noff] (trans) or src[r + noff][kk].
__global__ void k_panel(const float* __restrict__ src, int ld, int trans, int rows, int noff, int h, int rp, int dual,
                        int width, uint16_t* __restrict__ hi, uint16_t* __restrict__ lo) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)rows * width) return;
  const int kb = (int)(t / ((long long)rows * 32)), rem = (int)(t % ((long long)rows * 32));
  const int r = rem / 32, k = kb * 32 + rem % 32;
  int kk = k;
  bool ok = k < h;
  if (dual && k >= rp) {
    kk = h + (k - rp);
    ok = (k - rp) < h;
  }
  float v = 0.f;
  if (ok) v = trans ? src[(size_t)kk * ld + r + noff] : src[(size_t)(r + noff) * ld + kk];
  const unsigned short hv = rne16(v);
  hi[t] = hv;
  lo[t] = rne16(v - __uint_as_float((unsigned)hv << 16));
}

// the caller brackets its consecutive launches with one profiler scope and counts them in `made`
template <int KIND>
int launch(place3d_ctx* c, SArgs& a, int njobs, hipStream_t s, int& made) {
  const long long tiles = (long long)a.ntm * a.ntn * njobs;
  if (tiles <= 0) return PLACE3D_OK;
  if (tiles > 0x7fffffffLL) return set_err(c, PLACE3D_ERR_SIZE, "contraction grid too large");
  for (int i = njobs; i < kMaxJobs; ++i) a.job[i] = a.job[0];
  ++made;
  const dim3 grid((unsigned)tiles), block(256);
  // three stages for the launches of one workgroup per compute unit, two for the x inverse,
  // whose 768 workgroups then run two per compute unit
  constexpr int ST = KIND == XI ? 2 : 3;
  if (a.nz == 2) hipLaunchKernelGGL((k_sgemm<KIND, 2, ST>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_sgemm<KIND, 4, ST>), grid, block, 0, s, a);
  P3D_LAUNCH(c, "k_sgemm");
  return PLACE3D_OK;
}

}  // namespace

int build_split_chain(place3d_ctx* c, hipStream_t s) {
  SplitChain& q = c->sc;
  if (!q.on) return PLACE3D_OK;
  const DctBases& d = c->dct;
  const Geom& g = c->g;
  const int nx = g.nx, ny = g.ny;
  auto panel = [&](const float* src, int ld, int trans, int rows, int noff, int h, int rp, int dual, int width,
                   const HL& out) {
    const long long n = (long long)rows * width;
    hipLaunchKernelGGL(k_panel, dim3(blocks_for(n, 256)), dim3(256), 0, s, src, ld, trans, rows, noff, h, rp, dual,
                       width, out.h, out.l);
  };
  panel(d.Fx, nx, 1, q.hx, 0, q.hx, 0, 0, q.rx, q.fx[0]);
  panel(d.Fx, nx, 1, q.hx, q.hx, q.hx, 0, 0, q.rx, q.fx[1]);
  panel(d.FyT, ny, 0, q.hy, 0, q.hy, 0, 0, q.ry, q.fy[0]);
  panel(d.FyT, ny, 0, q.hy, q.hy, q.hy, 0, 0, q.ry, q.fy[1]);
  panel(d.Gy, ny, 0, q.hy, 0, q.hy, q.ry, 1, 2 * q.ry, q.gy);
  panel(d.Hy, ny, 0, q.hy, 0, q.hy, q.ry, 1, 2 * q.ry, q.hy_s);
  panel(d.Gx, nx, 1, q.hx, 0, q.hx, q.rx, 1, 2 * q.rx, q.gx);
  panel(d.Hx, nx, 1, q.hx, 0, q.hx, q.rx, 1, 2 * q.rx, q.hx_s);
  P3D_LAUNCH(c, "k_panel");
  // the pad columns of the inverse-y outputs are never written: clear them once
  const size_t px = (size_t)g.nz * ny * 2 * q.rx * sizeof(uint16_t);
  for (const HL* h : {&q.vg, &q.vh}) {
    P3D_HIP(c, hipMemsetAsync(h->h, 0, px, s));
    P3D_HIP(c, hipMemsetAsync(h->l, 0, px, s));
  }
  return PLACE3D_OK;
}

int field_split(place3d_ctx* c, const float* rho, float* phi, float* ex, float* ey, float* ez, hipStream_t s) {
  const SplitChain& q = c->sc;
  const Geom& g = c->g;
  const place3d_problem& p = c->prob;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  int rc;
  SArgs a{};
  a.nx = nx; a.ny = ny; a.nz = nz; a.hx = q.hx; a.hy = q.hy; a.rx = q.rx; a.ry = q.ry;
  {
    const double wb = p.die_x / p.nx, hb = p.die_y / p.ny, dz = p.nz * 0.5 * (wb + hb);
    a.px = (float)(M_PI / p.die_x); a.py = (float)(M_PI / p.die_y); a.pz = (float)(M_PI / dz);
  }
  a.zmat = c->dct.zmat;
  const int mt = kTile / nz;   // x frequencies per tile of the z-mixing kinds

  {
    ProfScope prof_(c, PLACE3D_STAGE_ZMIX, s);
    const long long work = (long long)nz * ny * (q.rx / 8);
    hipLaunchKernelGGL(k_fold_split_x, dim3(blocks_for(work, 256)), dim3(256), 0, s, rho, nz * ny, nx, q.hx, q.rx,
                       q.xs[0].h, q.xs[0].l, q.xs[1].h, q.xs[1].l);
    P3D_LAUNCH(c, "k_fold_split_x");
  }
  // the four contractions run back to back on s: one profiler scope for all of them
  ProfScope gemm_(c, PLACE3D_STAGE_GEMM, s);
  gemm_.launches = 0;
  // x forward
  {
    a.ntm = nz * ((q.hy + 63) / 64); a.ntn = (q.hx + kTile - 1) / kTile; a.ksteps = q.rx / kStep;
    a.ra = nz * ny; a.rb = q.hx; a.ro = nz * nx;
    for (int i = 0; i < 2; ++i)
      a.job[i] = SJob{q.xs[i].h, q.xs[i].l, q.fx[i].h, q.fx[i].l, 0, 0, i,
                      q.ys[0].h, q.ys[0].l, q.ys[1].h, q.ys[1].l, nullptr, 1.f};
    if ((rc = launch<XF>(c, a, 2, s, gemm_.launches))) return rc;
  }
  // y forward and the z mixing of the coefficients
  {
    a.ntm = (q.hy + kTile - 1) / kTile; a.ntn = (nx + mt - 1) / mt; a.ksteps = q.ry / kStep;
    a.ra = q.hy; a.rb = nz * nx; a.ro = nz * nx;
    for (int i = 0; i < 2; ++i)
      a.job[i] = SJob{q.fy[i].h, q.fy[i].l, q.ys[i].h, q.ys[i].l, 0, 0, i, q.bb.h, q.bb.l, nullptr, nullptr, nullptr, 1.f};
    if ((rc = launch<YF>(c, a, 2, s, gemm_.launches))) return rc;
  }
  // y inverse and unfold
  const bool need_g = phi || ex || ez, need_h = ey != nullptr;
  {
    a.ntm = (nx + mt - 1) / mt; a.ntn = (q.hy + kTile - 1) / kTile; a.ksteps = 2 * q.ry / kStep;
    a.ra = nz * nx; a.rb = q.hy; a.ro = nz * ny;
    int nj = 0;
    if (need_g) a.job[nj++] = SJob{q.bb.h, q.bb.l, q.gy.h, q.gy.l, 0, 0, 0, q.vg.h, q.vg.l, nullptr, nullptr, nullptr, 1.f};
    if (need_h) a.job[nj++] = SJob{q.bb.h, q.bb.l, q.hy_s.h, q.hy_s.l, 0, 0, 1, q.vh.h, q.vh.l, nullptr, nullptr, nullptr, 1.f};
    if ((rc = launch<YI>(c, a, nj, s, gemm_.launches))) return rc;
  }
  // x inverse, even and odd frequency halves into two accumulators; unfold and z mixing in the
  // epilogue (Ex = Gz^T Vg Hx, Ey = Gz^T Vh Gx, Ez = Hz^T Vg Gx, phi = Gz^T Vg Gx)
  {
    a.ntm = (ny + mt - 1) / mt; a.ntn = (q.hx + kTile - 1) / kTile; a.ksteps = 2 * q.rx / kStep;
    a.ra = nz * ny; a.rb = q.hx; a.ro = 0;
    struct Out { const HL* in; const HL* basis; int zsin; float* out; float sg; };
    Out o[4];
    int no = 0;
    if (ex) o[no++] = {&q.vg, &q.hx_s, 0, ex, -1.f};
    if (ey) o[no++] = {&q.vh, &q.gx, 0, ey, 1.f};
    if (ez) o[no++] = {&q.vg, &q.gx, 1, ez, 1.f};
    if (phi) o[no++] = {&q.vg, &q.gx, 0, phi, 1.f};
    int nj = 0;
    for (int i = 0; i < no; ++i)
      a.job[nj++] = SJob{o[i].in->h, o[i].in->l, o[i].basis->h, o[i].basis->l, 0, 0, o[i].zsin,
                         nullptr, nullptr, nullptr, nullptr, o[i].out, o[i].sg};
    if ((rc = launch<XI>(c, a, nj, s, gemm_.launches))) return rc;
  }
  return PLACE3D_OK;
}

}  // namespace p3d
