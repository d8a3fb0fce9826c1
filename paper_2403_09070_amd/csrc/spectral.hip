// Spectral Neumann Poisson solve (Sec. III-A, Eqs. density-coef, poisson-sol-potential,
// possion-sol-force) as dense separable contractions on MFMA.
//
// Map layout [z][y][x].  Sampling at bin centres x_i = (i + 1/2) w_b, omega_j = j pi / d_x.  The
// coefficients carry (2 - [j = 0]) / N per axis so that the cosine series reproduces the map
// (the normalisation under which the potential solves the Poisson equation), the (0,0,0) mode is
// dropped, and
//   phi = sum b cos cos cos,  E_x = sum b omega_j sin cos cos, ...,  b = a / |omega|^2.
//
// Matrices (row-major, float32):
//   Fx[x][j]  = c_j cos(pi j (x+1/2)/Nx)   forward along x, used as the right operand
//   Gx[j][x]  = cos(pi j (x+1/2)/Nx)       inverse cosine along x
//   Hx[j][x]  = omega_j sin(pi j (x+1/2)/Nx)  inverse sine along x, derivative factor folded in
//   FyT[k][y] = c_k cos(pi k (y+1/2)/Ny)   forward along y, used as the left operand
//   Gy[y][k], Hy[y][k]                      inverse along y
//   z (Nz <= 16) is mixed by small matrices on the vector ALUs.
//
// Pipeline of place3d_field:
//   T   = rho . Fx                   (x pass, M = Nz Ny, N = K = Nx)
//   A   = FyT . T[z]  per z          (y pass)
//   b   = zmix_fwd(A) / |omega|^2    (elementwise over (k, j), 16 x 16 at most)
//   Vg  = Gy . b[l], Vh = Hy . b[l]  (inverse y)
//   Pc, Ps, Qc = zmix_inv(Vg, Vh)    (cos / sin*omega_l along z)
//   Ex = Pc . Hx, phi = Pc . Gx, Ey = Qc . Gx, Ez = Ps . Gx   (inverse x)
// Every contraction is one launch of k_gemm: NN row-major, batched, with the float32 or the
// split-bfloat16 (hi.hi + hi.lo + lo.hi, float32 accumulation) MFMA path.
#include <cmath>

#include "internal.h"

namespace p3d {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------------ bases

__global__ void k_basis_x(int n, double length, float* Fx, float* Gx, float* Hx) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  const int r = (int)(t / n), c = (int)(t % n);
  {  // Fx[x = r][j = c]
    const double arg = M_PI * c * (r + 0.5) / n;
    Fx[t] = (float)((c == 0 ? 1.0 : 2.0) / n * cos(arg));
  }
  {  // Gx[j = r][x = c], Hx[j = r][x = c]
    const double arg = M_PI * r * (c + 0.5) / n;
    Gx[t] = (float)cos(arg);
    Hx[t] = (float)(M_PI * r / length * sin(arg));
  }
}

__global__ void k_basis_y(int n, double length, float* FyT, float* Gy, float* Hy) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  const int r = (int)(t / n), c = (int)(t % n);
  {  // FyT[k = r][y = c]
    const double arg = M_PI * r * (c + 0.5) / n;
    FyT[t] = (float)((r == 0 ? 1.0 : 2.0) / n * cos(arg));
  }
  {  // Gy[y = r][k = c], Hy[y = r][k = c]
    const double arg = M_PI * c * (r + 0.5) / n;
    Gy[t] = (float)cos(arg);
    Hy[t] = (float)(M_PI * c / length * sin(arg));
  }
}

// zmat: [0] Fz[z][l], [1] Gz[l][z], [2] Hz[l][z], each kMaxNz x kMaxNz
__global__ void k_basis_z(int n, double length, float* zmat) {
  const int t = threadIdx.x;
  if (t >= kMaxNz * kMaxNz) return;
  const int r = t / kMaxNz, c = t % kMaxNz;
  float f = 0.f, gz = 0.f, hz = 0.f;
  if (r < n && c < n) {
    f = (float)((c == 0 ? 1.0 : 2.0) / n * cos(M_PI * c * (r + 0.5) / n));   // Fz[z=r][l=c]
    const double arg = M_PI * r * (c + 0.5) / n;                               // Gz[l=r][z=c]
    gz = (float)cos(arg);
    hz = (float)(M_PI * r / length * sin(arg));
  }
  zmat[t] = f;
  zmat[kMaxNz * kMaxNz + t] = gz;
  zmat[2 * kMaxNz * kMaxNz + t] = hz;
}

__global__ void k_inv_w2(int nx, int ny, int nz, double dx, double dy, double dz, float* out) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long total = (long long)nx * ny * nz;
  if (t >= total) return;
  const int j = (int)(t % nx);
  const int k = (int)((t / nx) % ny);
  const int l = (int)(t / ((long long)nx * ny));
  const double wx = M_PI * j / dx, wy = M_PI * k / dy, wz = M_PI * l / dz;
  const double w2 = wx * wx + wy * wy + wz * wz;
  out[t] = w2 > 0.0 ? (float)(1.0 / w2) : 0.f;
}

// ------------------------------------------------------------------ GEMM

struct GemmProb {
  const float* A;
  const float* B;
  float* C;
  long long sA, sB, sC;   // batch strides in elements (0 = shared operand)
};

struct GemmArgs {
  int M, N, K, nbatch;    // every problem of a launch has the same shape and batch count
  GemmProb p[4];
};

constexpr int BM = 128, BN = 128;

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// C[M][N] = A[M][K] . B[K][N] on float32 MFMA (32x32x2): 4 waves, each a 64 x 64 sub-tile.
__global__ __launch_bounds__(256) void k_gemm_f32(GemmArgs args) {
  constexpr int BK = 16, PAD = 4;
  __shared__ float As[2][BK][BM + PAD];
  __shared__ float Bs[2][BK][BN + PAD];
  const int M = args.M, N = args.N, K = args.K;
  const int prob = blockIdx.z / args.nbatch, bat = blockIdx.z % args.nbatch;
  const GemmProb P = args.p[prob];
  const float* __restrict__ A = P.A + bat * P.sA;
  const float* __restrict__ B = P.B + bat * P.sB;
  float* __restrict__ C = P.C + bat * P.sC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const bool vec = ((K & 3) == 0) && ((N & 3) == 0) &&
                   ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0;

  float ra[8], rb[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int f = tid + 256 * q;
      const int ar = f >> 2, ak = (f & 3) * 4;          // A: 128 rows x 4 float4
      const int gm = m0 + ar, gk = k0 + ak;
      if (vec && gm < M && gk + 3 < K) {
        const float4 v = *reinterpret_cast<const float4*>(A + (size_t)gm * K + gk);
        ra[4 * q] = v.x; ra[4 * q + 1] = v.y; ra[4 * q + 2] = v.z; ra[4 * q + 3] = v.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[4 * q + e] = (gm < M && gk + e < K) ? A[(size_t)gm * K + gk + e] : 0.f;
      }
      const int br = f >> 5, bn = (f & 31) * 4;         // B: 16 rows x 32 float4
      const int gkb = k0 + br, gn = n0 + bn;
      if (vec && gkb < K && gn + 3 < N) {
        const float4 v = *reinterpret_cast<const float4*>(B + (size_t)gkb * N + gn);
        rb[4 * q] = v.x; rb[4 * q + 1] = v.y; rb[4 * q + 2] = v.z; rb[4 * q + 3] = v.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) rb[4 * q + e] = (gkb < K && gn + e < N) ? B[(size_t)gkb * N + gn + e] : 0.f;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int f = tid + 256 * q;
      const int ar = f >> 2, ak = (f & 3) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) As[buf][ak + e][ar] = ra[4 * q + e];
      const int br = f >> 5, bn = (f & 31) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) Bs[buf][br][bn + e] = rb[4 * q + e];
    }
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  const int KT = (K + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < KT) load((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const int kr = kk + (lane >> 5);
      const float a0 = As[cur][kr][wm * 64 + (lane & 31)];
      const float a1 = As[cur][kr][wm * 64 + 32 + (lane & 31)];
      const float b0 = Bs[cur][kr][wn * 64 + (lane & 31)];
      const float b1 = Bs[cur][kr][wn * 64 + 32 + (lane & 31)];
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (kt + 1 < KT) store(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = n0 + wn * 64 + b * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 64 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row < M && col < N) C[(size_t)row * N + col] = acc[a][b][r];
      }
    }
}

// Same contraction with each float32 operand split into bfloat16 hi + lo (round to nearest
// even) and three products hi.hi + hi.lo + lo.hi accumulated in float32 (32x32x16 bf16 MFMA).
// One operand is a DCT basis, split once at context creation and stored with k contiguous
// ([rows][K] for a left basis, transposed [N][K] for a right basis); the other is a map,
// loaded as float32 and split on the way into LDS.  LDS holds both operands k-contiguous,
// double-buffered, one barrier per 32-wide k step.
struct GemmSplitProb {
  const float* data;                 // map operand, float32 row-major
  const uint16_t* bhi;               // basis hi, k contiguous
  const uint16_t* blo;               // basis lo
  float* C;
  long long s_data, s_C;             // batch strides (elements)
};

struct GemmSplitArgs {
  int M, N, K, nbatch;
  GemmSplitProb p[4];
};

template <bool LEFT_BASIS>
__global__ __launch_bounds__(256) void k_gemm_bf16x3(GemmSplitArgs args) {
  constexpr int BK = 32, LDK = BK + 8;
  __shared__ unsigned short Ah[2][BM][LDK], Al[2][BM][LDK];
  __shared__ unsigned short Bh[2][BN][LDK], Bl[2][BN][LDK];
  const int M = args.M, N = args.N, K = args.K;
  const int prob = blockIdx.z / args.nbatch, bat = blockIdx.z % args.nbatch;
  const GemmSplitProb P = args.p[prob];
  const float* __restrict__ D = P.data + bat * P.s_data;
  const uint16_t* __restrict__ Bh_g = P.bhi;
  const uint16_t* __restrict__ Bl_g = P.blo;
  float* __restrict__ C = P.C + bat * P.s_C;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const bool full = (m0 + BM <= M) && (n0 + BN <= N) && (K % BK == 0) && (N % 4 == 0) && (K % 8 == 0);

  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  // staging registers: 16 data floats, 2 x 2 basis groups of 8 bf16
  float rd[16];
  u16x8 rbh[2], rbl[2];

  // basis tile: rows [r0, r0 + 128) of a k-contiguous [rows][K] array; thread takes row f >> 2,
  // k group (f & 3) * 8 for f = tid, tid + 256
  auto load_basis = [&](int k0, int r0, int rows) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int f = tid + 256 * q;
      const int r = f >> 2, kg = (f & 3) * 8;
      const int gr = r0 + r, gk = k0 + kg;
      if (full) {
        rbh[q] = *reinterpret_cast<const u16x8*>(Bh_g + (size_t)gr * K + gk);
        rbl[q] = *reinterpret_cast<const u16x8*>(Bl_g + (size_t)gr * K + gk);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const bool ok = gr < rows && gk + e < K;
          rbh[q][e] = ok ? Bh_g[(size_t)gr * K + gk + e] : (unsigned short)0;
          rbl[q][e] = ok ? Bl_g[(size_t)gr * K + gk + e] : (unsigned short)0;
        }
      }
    }
  };
  auto store_basis = [&](unsigned short (*H)[LDK], unsigned short (*L)[LDK]) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int f = tid + 256 * q;
      const int r = f >> 2, kg = (f & 3) * 8;
      *reinterpret_cast<u16x8*>(&H[r][kg]) = rbh[q];
      *reinterpret_cast<u16x8*>(&L[r][kg]) = rbl[q];
    }
  };
  // hi = RNE(v), lo = RNE(v - hi), two values per hardware conversion
  auto split_store = [&](unsigned short* h, unsigned short* l, const float* v) {
    u32x4 hh, ll;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const f32x2 x = {v[2 * e], v[2 * e + 1]};
      const unsigned hp = __builtin_bit_cast(unsigned, __builtin_convertvector(x, bf16x2v));
      const f32x2 back = {__uint_as_float(hp << 16), __uint_as_float(hp & 0xffff0000u)};
      hh[e] = hp;
      ll[e] = __builtin_bit_cast(unsigned, __builtin_convertvector(x - back, bf16x2v));
    }
    *reinterpret_cast<u32x4*>(h) = hh;
    *reinterpret_cast<u32x4*>(l) = ll;
  };
  // left data operand (map as A [M][K]): thread takes row f >> 2, k group (f & 3) * 8
  auto load_left_data = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int f = tid + 256 * q;
      const int r = f >> 2, kg = (f & 3) * 8;
      const int gm = m0 + r, gk = k0 + kg;
      if (full) {
        const float4 v0 = *reinterpret_cast<const float4*>(D + (size_t)gm * K + gk);
        const float4 v1 = *reinterpret_cast<const float4*>(D + (size_t)gm * K + gk + 4);
        rd[8 * q + 0] = v0.x; rd[8 * q + 1] = v0.y; rd[8 * q + 2] = v0.z; rd[8 * q + 3] = v0.w;
        rd[8 * q + 4] = v1.x; rd[8 * q + 5] = v1.y; rd[8 * q + 6] = v1.z; rd[8 * q + 7] = v1.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) rd[8 * q + e] = (gm < M && gk + e < K) ? D[(size_t)gm * K + gk + e] : 0.f;
      }
    }
  };
  auto store_left_data = [&](unsigned short (*H)[LDK], unsigned short (*L)[LDK]) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int f = tid + 256 * q;
      const int r = f >> 2, kg = (f & 3) * 8;
      split_store(&H[r][kg], &L[r][kg], rd + 8 * q);
    }
  };
  // right data operand (map as B [K][N]): thread takes columns 2 (tid & 63) + {0, 1} and k group
  // (tid >> 6) * 8, loading 8 rows of 2 consecutive columns and transposing them in registers
  auto load_right_data = [&](int k0) {
    const int cn = 2 * (tid & 63), kg = (tid >> 6) * 8;
    const int gn = n0 + cn;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int gk = k0 + kg + e;
      if (full) {
        const float2 v = *reinterpret_cast<const float2*>(D + (size_t)gk * N + gn);
        rd[e] = v.x;
        rd[8 + e] = v.y;
      } else {
        rd[e] = (gk < K && gn < N) ? D[(size_t)gk * N + gn] : 0.f;
        rd[8 + e] = (gk < K && gn + 1 < N) ? D[(size_t)gk * N + gn + 1] : 0.f;
      }
    }
  };
  auto store_right_data = [&](unsigned short (*H)[LDK], unsigned short (*L)[LDK]) {
    const int cn = 2 * (tid & 63), kg = (tid >> 6) * 8;
    split_store(&H[cn][kg], &L[cn][kg], rd);
    split_store(&H[cn + 1][kg], &L[cn + 1][kg], rd + 8);
  };
  auto load = [&](int k0) {
    if (LEFT_BASIS) { load_basis(k0, m0, M); load_right_data(k0); }
    else { load_left_data(k0); load_basis(k0, n0, N); }
  };
  auto store = [&](int buf) {
    if (LEFT_BASIS) { store_basis(Ah[buf], Al[buf]); store_right_data(Bh[buf], Bl[buf]); }
    else { store_left_data(Ah[buf], Al[buf]); store_basis(Bh[buf], Bl[buf]); }
  };

  const int KT = (K + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < KT) load((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const int ko = kk + 8 * (lane >> 5);
      bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int ar = wm * 64 + t * 32 + (lane & 31);
        const int bc = wn * 64 + t * 32 + (lane & 31);
        ah[t] = *reinterpret_cast<const bf16x8*>(&Ah[cur][ar][ko]);
        al[t] = *reinterpret_cast<const bf16x8*>(&Al[cur][ar][ko]);
        bh[t] = *reinterpret_cast<const bf16x8*>(&Bh[cur][bc][ko]);
        bl[t] = *reinterpret_cast<const bf16x8*>(&Bl[cur][bc][ko]);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
        }
    }
    if (kt + 1 < KT) store(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = n0 + wn * 64 + b * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 64 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row < M && col < N) C[(size_t)row * N + col] = acc[a][b][r];
      }
    }
}

// hi/lo bfloat16 split of a float32 matrix src[rows][cols]; with `transpose` the outputs are
// [cols][rows] (so that a right-hand basis becomes k-contiguous)
__global__ void k_split_bf16(const float* __restrict__ src, int rows, int cols, int transpose,
                             uint16_t* __restrict__ hi, uint16_t* __restrict__ lo) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)rows * cols) return;
  const int r = (int)(t / cols), c = (int)(t % cols);
  const float v = src[t];
  const unsigned short h = bf16_rne(v);
  const size_t o = transpose ? (size_t)c * rows + r : (size_t)t;
  hi[o] = h;
  lo[o] = bf16_rne(v - bf16_to_f32(h));
}

// ------------------------------------------------------------------ z mixing

// b[l][k][j] = inv_w2[l][k][j] * sum_z Fz[z][l] A[z][k][j]   (in place)
__global__ void k_zmix_fwd(int plane, int nz, const float* __restrict__ zmat, const float* __restrict__ inv_w2,
                           float* __restrict__ a) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= plane) return;
  float v[kMaxNz], o[kMaxNz];
  for (int z = 0; z < nz; ++z) v[z] = a[z * (long long)plane + t];
  for (int l = 0; l < nz; ++l) {
    float s = 0.f;
    for (int z = 0; z < nz; ++z) s += zmat[z * kMaxNz + l] * v[z];
    o[l] = s * inv_w2[l * (long long)plane + t];
  }
  for (int l = 0; l < nz; ++l) a[l * (long long)plane + t] = o[l];
}

// pc[z] = sum_l Gz[l][z] vg[l], ps[z] = sum_l Hz[l][z] vg[l], qc[z] = sum_l Gz[l][z] vh[l]
__global__ void k_zmix_inv(int plane, int nz, const float* __restrict__ zmat, const float* __restrict__ vg,
                           const float* __restrict__ vh, float* __restrict__ pc, float* __restrict__ ps,
                           float* __restrict__ qc) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= plane) return;
  const float* Gz = zmat + kMaxNz * kMaxNz;
  const float* Hz = zmat + 2 * kMaxNz * kMaxNz;
  float g[kMaxNz], h[kMaxNz];
  if (vg) for (int l = 0; l < nz; ++l) g[l] = vg[l * (long long)plane + t];
  if (vh) for (int l = 0; l < nz; ++l) h[l] = vh[l * (long long)plane + t];
  for (int z = 0; z < nz; ++z) {
    if (pc) { float s = 0.f; for (int l = 0; l < nz; ++l) s += Gz[l * kMaxNz + z] * g[l]; pc[z * (long long)plane + t] = s; }
    if (ps) { float s = 0.f; for (int l = 0; l < nz; ++l) s += Hz[l * kMaxNz + z] * g[l]; ps[z * (long long)plane + t] = s; }
    if (qc) { float s = 0.f; for (int l = 0; l < nz; ++l) s += Gz[l * kMaxNz + z] * h[l]; qc[z * (long long)plane + t] = s; }
  }
}

// partials of 1/2 vol(b) sum rho phi, one per block
__global__ void k_energy(long long total, const float* __restrict__ rho, const float* __restrict__ phi, float half_vol,
                         double* __restrict__ part) {
  __shared__ double sh[256 / kWave];
  double s = 0.0;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x)
    s += (double)rho[t] * (double)phi[t];
  for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
  const int wid = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) sh[wid] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < 256 / kWave; ++w) r += sh[w];
    part[blockIdx.x] = r * (double)half_vol;
  }
}

// A basis operand of a contraction: its float32 matrix and its k-contiguous bfloat16 split
struct Basis { const float* f32; const uint16_t* hi; const uint16_t* lo; };

// batched C = A . B where exactly one of A (left_basis) or B is a DCT basis shared by the batch
int gemm(place3d_ctx* c, int M, int N, int K, int nbatch, bool left_basis, const float* const* data,
         long long s_data, const Basis* basis, float* const* out, long long s_out, int nprob, hipStream_t s) {
  if (nprob <= 0) return PLACE3D_OK;
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, nbatch * nprob);
  ProfScope prof_(c, PLACE3D_STAGE_GEMM, s);
  if (c->prob.precision == PLACE3D_BF16X3) {
    GemmSplitArgs a;
    a.M = M; a.N = N; a.K = K; a.nbatch = nbatch;
    for (int i = 0; i < 4; ++i) {
      const int j = i < nprob ? i : 0;
      a.p[i] = {data[j], basis[j].hi, basis[j].lo, out[j], s_data, s_out};
    }
    if (left_basis) hipLaunchKernelGGL(k_gemm_bf16x3<true>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_gemm_bf16x3<false>, grid, dim3(256), 0, s, a);
  } else {
    GemmArgs a;
    a.M = M; a.N = N; a.K = K; a.nbatch = nbatch;
    for (int i = 0; i < 4; ++i) {
      const int j = i < nprob ? i : 0;
      a.p[i] = left_basis ? GemmProb{basis[j].f32, data[j], out[j], 0, s_data, s_out}
                          : GemmProb{data[j], basis[j].f32, out[j], s_data, 0, s_out};
    }
    hipLaunchKernelGGL(k_gemm_f32, grid, dim3(256), 0, s, a);
  }
  P3D_LAUNCH(c, "k_gemm");
  return PLACE3D_OK;
}

}  // namespace

int build_dct_bases(place3d_ctx* c, hipStream_t s) {
  const Geom& g = c->g;
  const place3d_problem& p = c->prob;
  const double wb = p.die_x / p.nx, hb = p.die_y / p.ny, dz = p.nz * 0.5 * (wb + hb);
  hipLaunchKernelGGL(k_basis_x, dim3(blocks_for((long long)g.nx * g.nx, 256)), dim3(256), 0, s, g.nx, p.die_x,
                     c->dct.Fx, c->dct.Gx, c->dct.Hx);
  P3D_LAUNCH(c, "k_basis_x");
  hipLaunchKernelGGL(k_basis_y, dim3(blocks_for((long long)g.ny * g.ny, 256)), dim3(256), 0, s, g.ny, p.die_y,
                     c->dct.FyT, c->dct.Gy, c->dct.Hy);
  P3D_LAUNCH(c, "k_basis_y");
  {
    const DctBases& d = c->dct;
    const unsigned bx = blocks_for((long long)g.nx * g.nx, 256), by = blocks_for((long long)g.ny * g.ny, 256);
    hipLaunchKernelGGL(k_split_bf16, dim3(bx), dim3(256), 0, s, d.Fx, g.nx, g.nx, 1, d.Fx_h, d.Fx_l);
    hipLaunchKernelGGL(k_split_bf16, dim3(bx), dim3(256), 0, s, d.Gx, g.nx, g.nx, 1, d.Gx_h, d.Gx_l);
    hipLaunchKernelGGL(k_split_bf16, dim3(bx), dim3(256), 0, s, d.Hx, g.nx, g.nx, 1, d.Hx_h, d.Hx_l);
    hipLaunchKernelGGL(k_split_bf16, dim3(by), dim3(256), 0, s, d.FyT, g.ny, g.ny, 0, d.FyT_h, d.FyT_l);
    hipLaunchKernelGGL(k_split_bf16, dim3(by), dim3(256), 0, s, d.Gy, g.ny, g.ny, 0, d.Gy_h, d.Gy_l);
    hipLaunchKernelGGL(k_split_bf16, dim3(by), dim3(256), 0, s, d.Hy, g.ny, g.ny, 0, d.Hy_h, d.Hy_l);
    P3D_LAUNCH(c, "k_split_bf16");
  }
  hipLaunchKernelGGL(k_basis_z, dim3(1), dim3(kMaxNz * kMaxNz), 0, s, g.nz, dz, c->dct.zmat);
  P3D_LAUNCH(c, "k_basis_z");
  const long long map = (long long)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL(k_inv_w2, dim3(blocks_for(map, 256)), dim3(256), 0, s, g.nx, g.ny, g.nz, p.die_x, p.die_y, dz,
                     c->dct.inv_w2);
  P3D_LAUNCH(c, "k_inv_w2");
  return PLACE3D_OK;
}

int spectral_field(place3d_ctx* c, const float* rho, float* phi, float* ex, float* ey, float* ez,
                   double* energy, hipStream_t s) {
  const Geom& g = c->g;
  const DctBases& d = c->dct;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long long plane = (long long)nx * ny;
  int rc;
  const Basis Fx{d.Fx, d.Fx_h, d.Fx_l}, Gx{d.Gx, d.Gx_h, d.Gx_l}, Hx{d.Hx, d.Hx_h, d.Hx_l};
  const Basis FyT{d.FyT, d.FyT_h, d.FyT_l}, Gy{d.Gy, d.Gy_h, d.Gy_l}, Hy{d.Hy, d.Hy_h, d.Hy_l};
  // forward x: T = rho . Fx;  forward y: A[z] = FyT . T[z]
  {
    const float* in[1] = {rho};
    float* out[1] = {c->map_t};
    if ((rc = gemm(c, nz * ny, nx, nx, 1, false, in, 0, &Fx, out, 0, 1, s))) return rc;
  }
  {
    const float* in[1] = {c->map_t};
    float* out[1] = {c->map_a};
    if ((rc = gemm(c, ny, nx, ny, nz, true, in, plane, &FyT, out, plane, 1, s))) return rc;
  }
  {
    ProfScope prof_(c, PLACE3D_STAGE_ZMIX, s);
    hipLaunchKernelGGL(k_zmix_fwd, dim3(blocks_for(plane, 256)), dim3(256), 0, s, (int)plane, nz, d.zmat, d.inv_w2,
                       c->map_a);
    P3D_LAUNCH(c, "k_zmix_fwd");
  }
  // inverse y: Vg = Gy . b[l], Vh = Hy . b[l]
  const bool need_g = phi || ex || ez, need_h = ey != nullptr;
  {
    const float* in[2] = {c->map_a, c->map_a};
    Basis bs[2];
    float* out[2];
    int np = 0;
    if (need_g) { bs[np] = Gy; out[np++] = c->map_vg; }
    if (need_h) { bs[np] = Hy; out[np++] = c->map_vh; }
    if ((rc = gemm(c, ny, nx, ny, nz, true, in, plane, bs, out, plane, np, s))) return rc;
  }
  float* pc = (phi || ex) ? c->map_pc : nullptr;
  float* ps = ez ? c->map_ps : nullptr;
  float* qc = ey ? c->map_qc : nullptr;
  if (pc || ps || qc) {
    {
      ProfScope prof_(c, PLACE3D_STAGE_ZMIX, s);
      hipLaunchKernelGGL(k_zmix_inv, dim3(blocks_for(plane, 256)), dim3(256), 0, s, (int)plane, nz, d.zmat,
                       need_g ? c->map_vg : nullptr, need_h ? c->map_vh : nullptr, pc, ps, qc);
      P3D_LAUNCH(c, "k_zmix_inv");
    }
  }
  // inverse x: Ex = Pc . Hx, Ey = Qc . Gx, Ez = Ps . Gx, phi = Pc . Gx
  {
    const float* in[4];
    Basis bs[4];
    float* out[4];
    int np = 0;
    if (ex) { in[np] = c->map_pc; bs[np] = Hx; out[np++] = ex; }
    if (ey) { in[np] = c->map_qc; bs[np] = Gx; out[np++] = ey; }
    if (ez) { in[np] = c->map_ps; bs[np] = Gx; out[np++] = ez; }
    if (phi) { in[np] = c->map_pc; bs[np] = Gx; out[np++] = phi; }
    if ((rc = gemm(c, nz * ny, nx, nx, 1, false, in, 0, bs, out, 0, np, s))) return rc;
  }
  if (energy) {
    const long long map = plane * nz;
    const unsigned nb = (unsigned)std::min<long long>(blocks_for(map, 256), 1024);
    {
      ProfScope prof_(c, PLACE3D_STAGE_ZMIX, s);
      hipLaunchKernelGGL(k_energy, dim3(nb), dim3(256), 0, s, map, rho, phi, 0.5f * g.vol_bin,
                         c->part + (size_t)R_ENERGY * c->part_stride);
      P3D_LAUNCH(c, "k_energy");
    }
    if ((rc = reduce_final(c, R_ENERGY, 1, (int)nb, false, energy, s))) return rc;
  }
  return PLACE3D_OK;
}

}  // namespace p3d
