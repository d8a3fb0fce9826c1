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
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------------ bases

// Spectral index order.  With an even axis length the DCT bases obey
//   B[n-1-x][k] = (-1)^k B[x][k] (cosine),  (-1)^(k+1) B[x][k] (sine),
// so every contraction splits into an even-frequency and an odd-frequency half of half the
// size, on the data folded about the axis middle (x[i] +- x[n-1-i]).  Spectral arrays then hold
// the even frequencies first: position p < n/2 is frequency 2p, position n/2 + p is 2p + 1.
// Odd lengths keep the natural order and the dense contractions.
__host__ __device__ inline int freq_of(int p, int n, int fold) {
  if (!fold) return p;
  const int h = n / 2;
  return p < h ? 2 * p : 2 * (p - h) + 1;
}

__global__ void k_basis_x(int n, int fold, double length, float* Fx, float* Gx, float* Hx) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  const int r = (int)(t / n), c = (int)(t % n);
  {  // Fx[x = r][position c]
    const int j = freq_of(c, n, fold);
    const double arg = M_PI * j * (r + 0.5) / n;
    Fx[t] = (float)((j == 0 ? 1.0 : 2.0) / n * cos(arg));
  }
  {  // Gx[position r][x = c], Hx[position r][x = c]
    const int j = freq_of(r, n, fold);
    const double arg = M_PI * j * (c + 0.5) / n;
    Gx[t] = (float)cos(arg);
    Hx[t] = (float)(M_PI * j / length * sin(arg));
  }
}

__global__ void k_basis_y(int n, int fold, double length, float* FyT, float* Gy, float* Hy) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  const int r = (int)(t / n), c = (int)(t % n);
  {  // FyT[position r][y = c]
    const int k = freq_of(r, n, fold);
    const double arg = M_PI * k * (c + 0.5) / n;
    FyT[t] = (float)((k == 0 ? 1.0 : 2.0) / n * cos(arg));
  }
  {  // Gy[y = r][position c], Hy[y = r][position c]
    const int k = freq_of(c, n, fold);
    const double arg = M_PI * k * (r + 0.5) / n;
    Gy[t] = (float)cos(arg);
    Hy[t] = (float)(M_PI * k / length * sin(arg));
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

__global__ void k_inv_w2(int nx, int ny, int nz, int fold, double dx, double dy, double dz, float* out) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long total = (long long)nx * ny * nz;
  if (t >= total) return;
  const int j = freq_of((int)(t % nx), nx, fold);
  const int k = freq_of((int)((t / nx) % ny), ny, fold);
  const int l = (int)(t / ((long long)nx * ny));
  const double wx = M_PI * j / dx, wy = M_PI * k / dy, wz = M_PI * l / dz;
  const double w2 = wx * wx + wy * wy + wz * wz;
  out[t] = w2 > 0.0 ? (float)(1.0 / w2) : 0.f;
}

// ------------------------------------------------------------------ GEMM

constexpr int kMaxProb = 8;

// One contraction C = A . B of a launch: A is M x K, B is K x N, C is M x N, with the leading
// dimensions of the launch.  One operand is a map (the data operand); with fold != 0 it is
// folded along k about the middle of an axis of length fold_n: X(k) + fold * X(fold_n - 1 - k).
struct GemmProb {
  const float* A;
  const float* B;
  float* C;
  long long sA, sB, sC;   // batch strides in elements (0 = shared operand)
  float fold;
};

struct GemmArgs {
  int M, N, K, nbatch;    // every problem of a launch has the same shape and batch count
  int lda, ldb, ldc;
  int fold_n;
  int fold_a;             // 1: A is the data operand, 0: B
  GemmProb p[kMaxProb];
};

constexpr int BM = 128, BN = 128;

__device__ __forceinline__ bool al16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Output tile of a workgroup.  The launch is one-dimensional over (n tile, m tile, problem x
// batch), n fastest, and the XCD-aware order gives each die a contiguous run of tiles: the n
// tiles of one m block (which share its rows of the data operand) then stay on one die's L2.
struct TileIdx { int n, m, z; };
template <int BMT = BM>
__device__ __forceinline__ TileIdx tile_of(int M, int N) {
  const int ntn = (N + BN - 1) / BN, ntm = (M + BMT - 1) / BMT;
  const int w = xcd_swizzle((int)blockIdx.x, (int)gridDim.x);
  return {w % ntn, (w / ntn) % ntm, w / (ntn * ntm)};
}

// C[M][N] = A[M][K] . B[K][N] on float32 MFMA (32x32x2): 4 waves, each a 64 x 64 sub-tile.
__global__ __launch_bounds__(256) void k_gemm_f32(GemmArgs args) {
  constexpr int BK = 16, PAD = 4;
  __shared__ float As[2][BK][BM + PAD];
  __shared__ float Bs[2][BK][BN + PAD];
  const int M = args.M, N = args.N, K = args.K, lda = args.lda, ldb = args.ldb, ldc = args.ldc, fn = args.fold_n;
  const TileIdx ti = tile_of(M, N);
  const int prob = ti.z / args.nbatch, bat = ti.z % args.nbatch;
  const GemmProb P = args.p[prob];
  const float* __restrict__ A = P.A + bat * P.sA;
  const float* __restrict__ B = P.B + bat * P.sB;
  float* __restrict__ C = P.C + bat * P.sC;
  const float fa = args.fold_a ? P.fold : 0.f, fb = args.fold_a ? 0.f : P.fold;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = ti.m * BM, n0 = ti.n * BN;
  const bool vec = ((K & 3) == 0) && ((N & 3) == 0) && ((lda & 3) == 0) && ((ldb & 3) == 0) && ((fn & 3) == 0) &&
                   al16(A) && al16(B);

  // staged operands; wa / wb hold the scaled mirrored values of a fold (zero otherwise)
  float ra[8], rb[8], wa[8], wb[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) wa[e] = wb[e] = 0.f;
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int f = tid + 256 * q;
      const int ar = f >> 2, ak = (f & 3) * 4;          // A: 128 rows x 4 float4
      const int gm = m0 + ar, gk = k0 + ak;
      if (vec && gm < M && gk + 3 < K) {
        const float4 v = *reinterpret_cast<const float4*>(A + (size_t)gm * lda + gk);
        ra[4 * q] = v.x; ra[4 * q + 1] = v.y; ra[4 * q + 2] = v.z; ra[4 * q + 3] = v.w;
        if (fa != 0.f) {   // mirrored group, added when the stage is stored
          const float4 w = *reinterpret_cast<const float4*>(A + (size_t)gm * lda + fn - 4 - gk);
          wa[4 * q] = fa * w.w; wa[4 * q + 1] = fa * w.z; wa[4 * q + 2] = fa * w.y; wa[4 * q + 3] = fa * w.x;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float v = 0.f, w = 0.f;
          if (gm < M && gk + e < K) {
            v = A[(size_t)gm * lda + gk + e];
            if (fa != 0.f) w = fa * A[(size_t)gm * lda + fn - 1 - gk - e];
          }
          ra[4 * q + e] = v;
          wa[4 * q + e] = w;
        }
      }
      const int br = f >> 5, bn = (f & 31) * 4;         // B: 16 rows x 32 float4
      const int gkb = k0 + br, gn = n0 + bn;
      if (vec && gkb < K && gn + 3 < N) {
        const float4 v = *reinterpret_cast<const float4*>(B + (size_t)gkb * ldb + gn);
        rb[4 * q] = v.x; rb[4 * q + 1] = v.y; rb[4 * q + 2] = v.z; rb[4 * q + 3] = v.w;
        if (fb != 0.f) {
          const float4 w = *reinterpret_cast<const float4*>(B + (size_t)(fn - 1 - gkb) * ldb + gn);
          wb[4 * q] = fb * w.x; wb[4 * q + 1] = fb * w.y; wb[4 * q + 2] = fb * w.z; wb[4 * q + 3] = fb * w.w;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float v = 0.f, w = 0.f;
          if (gkb < K && gn + e < N) {
            v = B[(size_t)gkb * ldb + gn + e];
            if (fb != 0.f) w = fb * B[(size_t)(fn - 1 - gkb) * ldb + gn + e];
          }
          rb[4 * q + e] = v;
          wb[4 * q + e] = w;
        }
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int f = tid + 256 * q;
      const int ar = f >> 2, ak = (f & 3) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) As[buf][ak + e][ar] = ra[4 * q + e] + wa[4 * q + e];
      const int br = f >> 5, bn = (f & 31) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) Bs[buf][br][bn + e] = rb[4 * q + e] + wb[4 * q + e];
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
        if (row < M && col < N) C[(size_t)row * ldc + col] = acc[a][b][r];
      }
    }
}

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// Same contraction with each float32 operand split into bfloat16 hi + lo (round to nearest
// even) and three products hi.hi + hi.lo + lo.hi accumulated in float32 (32x32x16 bf16 MFMA).
// One operand is a DCT basis, split once at context creation and stored with k contiguous
// ([rows][ldb] for a left basis, transposed to [N][ldb] for a right basis); the other is a map,
// loaded as float32 (folded if asked) and split on the way into LDS.  LDS holds both operands
// k-contiguous, double-buffered, one barrier per 32-wide k step.
struct GemmSplitProb {
  const float* data;                 // map operand, float32 row-major
  const uint16_t* bhi;               // basis hi, k contiguous
  const uint16_t* blo;               // basis lo
  float* C;
  long long s_data, s_C;             // batch strides (elements)
  float fold;
};

struct GemmSplitArgs {
  int M, N, K, nbatch;
  int ldd, ldb, ldc;                 // leading dimensions: data, basis (split), output
  int fold_n;
  GemmSplitProb p[kMaxProb];
};

// BMT: block rows, 128 or 64 (64 doubles the workgroups of a launch that would otherwise not
// fill the chip); each of the 2 x 2 wavefronts computes BMT/2 x 64 of the block's BMT x 128.
template <bool LEFT_BASIS, int BMT>
__global__ __launch_bounds__(256) void k_gemm_bf16x3(GemmSplitArgs args) {
  constexpr int QA = BMT / 64;       // 256-thread passes over the A tile (BMT rows x 4 units)
  constexpr int TA = BMT / 64;       // 32-row MFMA tiles per wavefront
  // LDS rows of 32 bf16 (four 16-byte units), unit u of row r stored at u ^ ((r >> 1) & 3): the
  // MFMA fragment reads (8 consecutive rows, one unit) and the staging writes (2 rows x 4 units,
  // or 8 consecutive rows x 1 unit) then touch distinct banks
  constexpr int BK = 32, LDK = BK;
  __shared__ unsigned short Ah[2][BMT][LDK], Al[2][BMT][LDK];
  __shared__ unsigned short Bh[2][BN][LDK], Bl[2][BN][LDK];
  auto sw = [](int r, int unit) { return 8 * (unit ^ ((r >> 1) & 3)); };
  const int M = args.M, N = args.N, K = args.K, ldd = args.ldd, ldb = args.ldb, ldc = args.ldc, fn = args.fold_n;
  const TileIdx ti = tile_of<BMT>(M, N);
  const int prob = ti.z / args.nbatch, bat = ti.z % args.nbatch;
  const GemmSplitProb P = args.p[prob];
  const float* __restrict__ D = P.data + bat * P.s_data;
  const uint16_t* __restrict__ Bh_g = P.bhi;
  const uint16_t* __restrict__ Bl_g = P.blo;
  float* __restrict__ C = P.C + bat * P.s_C;
  const float fold = P.fold;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = ti.m * BMT, n0 = ti.n * BN;
  const bool full = (m0 + BMT <= M) && (n0 + BN <= N) && (K % BK == 0) && (ldd % 8 == 0) && (ldb % 8 == 0) &&
                    (fn % 8 == 0) && al16(D) && al16(Bh_g) && al16(Bl_g);

  f32x16 acc[TA][2];
#pragma unroll
  for (int a = 0; a < TA; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  // staging registers: two groups of 8 data floats (and, on the full path, the scaled mirrored
  // values of a fold, added when the stage is stored so that no load of the next stage is
  // waited for before the MFMAs), 2 x 2 basis groups of 8 bf16
  f32x8 rd[2], rw[2];
  u16x8 rbh[2], rbl[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) rw[q] = (f32x8)(0.f);

  // basis tile: rows [r0, r0 + 64 nq) of a k-contiguous array; thread takes row f >> 2, k group
  // (f & 3) * 8 for f = tid + 256 q, q < nq
  auto load_basis = [&](int k0, int r0, int rows, int nq) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (q >= nq) break;
      const int f = tid + 256 * q;
      const int r = f >> 2, kg = (f & 3) * 8;
      const int gr = r0 + r, gk = k0 + kg;
      if (full) {
        rbh[q] = *reinterpret_cast<const u16x8*>(Bh_g + (size_t)gr * ldb + gk);
        rbl[q] = *reinterpret_cast<const u16x8*>(Bl_g + (size_t)gr * ldb + gk);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const bool ok = gr < rows && gk + e < K;
          rbh[q][e] = ok ? Bh_g[(size_t)gr * ldb + gk + e] : (unsigned short)0;
          rbl[q][e] = ok ? Bl_g[(size_t)gr * ldb + gk + e] : (unsigned short)0;
        }
      }
    }
  };
  auto store_basis = [&](unsigned short (*H)[LDK], unsigned short (*L)[LDK], int nq) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (q >= nq) break;
      const int f = tid + 256 * q;
      const int r = f >> 2, kg = (f & 3) * 8;
      *reinterpret_cast<u16x8*>(&H[r][sw(r, kg >> 3)]) = rbh[q];
      *reinterpret_cast<u16x8*>(&L[r][sw(r, kg >> 3)]) = rbl[q];
    }
  };
  // hi = RNE(v), lo = RNE(v - hi), two values per hardware conversion
  auto split_store = [&](unsigned short* h, unsigned short* l, f32x8 v) {
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
  // left data operand (map as A [M][K]): thread takes row f >> 2, k group (f & 3) * 8; a fold
  // reads the mirrored group as two float4 and reverses it
  auto load_left_data = [&](int k0) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int f = tid + 256 * q;
      const int r = f >> 2, kg = (f & 3) * 8;
      const int gm = m0 + r, gk = k0 + kg;
      float v[8], w[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) w[e] = 0.f;
      if (full) {
        const float* row = D + (size_t)gm * ldd;
        const float4 v0 = *reinterpret_cast<const float4*>(row + gk);
        const float4 v1 = *reinterpret_cast<const float4*>(row + gk + 4);
        v[0] = v0.x; v[1] = v0.y; v[2] = v0.z; v[3] = v0.w;
        v[4] = v1.x; v[5] = v1.y; v[6] = v1.z; v[7] = v1.w;
        if (fold != 0.f) {
          const float4 w0 = *reinterpret_cast<const float4*>(row + fn - 8 - gk);   // mirror of gk+7..gk+4
          const float4 w1 = *reinterpret_cast<const float4*>(row + fn - 4 - gk);   // mirror of gk+3..gk
          w[0] = fold * w1.w; w[1] = fold * w1.z; w[2] = fold * w1.y; w[3] = fold * w1.x;
          w[4] = fold * w0.w; w[5] = fold * w0.z; w[6] = fold * w0.y; w[7] = fold * w0.x;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          float a = 0.f;
          if (gm < M && gk + e < K) {
            a = D[(size_t)gm * ldd + gk + e];
            if (fold != 0.f) a += fold * D[(size_t)gm * ldd + fn - 1 - gk - e];
          }
          v[e] = a;
        }
      }
      rd[q] = (f32x8){v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
      rw[q] = (f32x8){w[0], w[1], w[2], w[3], w[4], w[5], w[6], w[7]};
    }
  };
  auto store_left_data = [&](unsigned short (*H)[LDK], unsigned short (*L)[LDK]) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int f = tid + 256 * q;
      const int r = f >> 2, kg = (f & 3) * 8;
      split_store(&H[r][sw(r, kg >> 3)], &L[r][sw(r, kg >> 3)], rd[q] + rw[q]);
    }
  };
  // right data operand (map as B [K][N]): thread takes columns c0 = tid & 63 and c0 + 64 and k
  // group (tid >> 6) * 8, loading 8 rows of each column (coalesced across the wavefront) and
  // transposing them in registers (rd[0] column c0, rd[1] column c0 + 64); a fold adds the
  // mirrored rows
  auto load_right_data = [&](int k0) {
    const int c0 = tid & 63, kg = (tid >> 6) * 8;
    const int gn0 = n0 + c0, gn1 = gn0 + 64;
    float v0[8], v1[8], w0[8], w1[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) w0[e] = w1[e] = 0.f;
    if (full) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float* row = D + (size_t)(k0 + kg + e) * ldd;
        v0[e] = row[gn0];
        v1[e] = row[gn1];
      }
      if (fold != 0.f) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float* row = D + (size_t)(fn - 1 - (k0 + kg + e)) * ldd;
          w0[e] = fold * row[gn0];
          w1[e] = fold * row[gn1];
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int gk = k0 + kg + e;
        float a = 0.f, b = 0.f;
        if (gk < K) {
          if (gn0 < N) {
            a = D[(size_t)gk * ldd + gn0];
            if (fold != 0.f) a += fold * D[(size_t)(fn - 1 - gk) * ldd + gn0];
          }
          if (gn1 < N) {
            b = D[(size_t)gk * ldd + gn1];
            if (fold != 0.f) b += fold * D[(size_t)(fn - 1 - gk) * ldd + gn1];
          }
        }
        v0[e] = a;
        v1[e] = b;
      }
    }
    // one assignment of the staging vectors after both paths (no store is sunk into a choice
    // between the arrays, which would move them to scratch memory)
    rd[0] = (f32x8){v0[0], v0[1], v0[2], v0[3], v0[4], v0[5], v0[6], v0[7]};
    rd[1] = (f32x8){v1[0], v1[1], v1[2], v1[3], v1[4], v1[5], v1[6], v1[7]};
    rw[0] = (f32x8){w0[0], w0[1], w0[2], w0[3], w0[4], w0[5], w0[6], w0[7]};
    rw[1] = (f32x8){w1[0], w1[1], w1[2], w1[3], w1[4], w1[5], w1[6], w1[7]};
  };
  auto store_right_data = [&](unsigned short (*H)[LDK], unsigned short (*L)[LDK]) {
    const int c0 = tid & 63, c1 = c0 + 64, u = tid >> 6;
    split_store(&H[c0][sw(c0, u)], &L[c0][sw(c0, u)], rd[0] + rw[0]);
    split_store(&H[c1][sw(c1, u)], &L[c1][sw(c1, u)], rd[1] + rw[1]);
  };
  auto load = [&](int k0) {
    if constexpr (LEFT_BASIS) { load_basis(k0, m0, M, QA); load_right_data(k0); }
    else { load_left_data(k0); load_basis(k0, n0, N, 2); }
  };
  auto store = [&](int buf) {
    if constexpr (LEFT_BASIS) { store_basis(Ah[buf], Al[buf], QA); store_right_data(Bh[buf], Bl[buf]); }
    else { store_left_data(Ah[buf], Al[buf]); store_basis(Bh[buf], Bl[buf], 2); }
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
      bf16x8 ah[TA], al[TA], bh[2], bl[2];
#pragma unroll
      for (int t = 0; t < TA; ++t) {
        const int ar = wm * (BMT / 2) + t * 32 + (lane & 31);
        ah[t] = *reinterpret_cast<const bf16x8*>(&Ah[cur][ar][sw(ar, ko >> 3)]);
        al[t] = *reinterpret_cast<const bf16x8*>(&Al[cur][ar][sw(ar, ko >> 3)]);
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int bc = wn * 64 + t * 32 + (lane & 31);
        bh[t] = *reinterpret_cast<const bf16x8*>(&Bh[cur][bc][sw(bc, ko >> 3)]);
        bl[t] = *reinterpret_cast<const bf16x8*>(&Bl[cur][bc][sw(bc, ko >> 3)]);
      }
#pragma unroll
      for (int a = 0; a < TA; ++a)
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
  for (int a = 0; a < TA; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = n0 + wn * 64 + b * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * (BMT / 2) + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row < M && col < N) C[(size_t)row * ldc + col] = acc[a][b][r];
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

// Folded y axis: rows [0, h) of vg / vh hold the even-frequency half E and rows [h, ny) the
// odd half O of the inverse-y contraction; row y is E + O and row ny-1-y is E - O for the
// cosine basis, O - E for the sine basis.  One thread per (y < h, x) writes both rows.
__global__ void k_zmix_inv_fold(int nx, int ny, int nz, const float* __restrict__ zmat, const float* __restrict__ vg,
                                const float* __restrict__ vh, float* __restrict__ pc, float* __restrict__ ps,
                                float* __restrict__ qc) {
  const int h = ny / 2;
  const long long plane = (long long)nx * ny;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)h * nx) return;
  const int y = (int)(t / nx), x = (int)(t % nx);
  const long long lo = (long long)y * nx + x, hi = (long long)(h + y) * nx + x, mir = (long long)(ny - 1 - y) * nx + x;
  const float* Gz = zmat + kMaxNz * kMaxNz;
  const float* Hz = zmat + 2 * kMaxNz * kMaxNz;
  float g0[kMaxNz], g1[kMaxNz], h0[kMaxNz], h1[kMaxNz];
  if (vg)
    for (int l = 0; l < nz; ++l) {
      const float e = vg[l * plane + lo], o = vg[l * plane + hi];
      g0[l] = e + o;
      g1[l] = e - o;
    }
  if (vh)
    for (int l = 0; l < nz; ++l) {
      const float e = vh[l * plane + lo], o = vh[l * plane + hi];
      h0[l] = e + o;
      h1[l] = o - e;
    }
  for (int z = 0; z < nz; ++z) {
    if (pc) {
      float a = 0.f, b = 0.f;
      for (int l = 0; l < nz; ++l) { a += Gz[l * kMaxNz + z] * g0[l]; b += Gz[l * kMaxNz + z] * g1[l]; }
      pc[z * plane + lo] = a; pc[z * plane + mir] = b;
    }
    if (ps) {
      float a = 0.f, b = 0.f;
      for (int l = 0; l < nz; ++l) { a += Hz[l * kMaxNz + z] * g0[l]; b += Hz[l * kMaxNz + z] * g1[l]; }
      ps[z * plane + lo] = a; ps[z * plane + mir] = b;
    }
    if (qc) {
      float a = 0.f, b = 0.f;
      for (int l = 0; l < nz; ++l) { a += Gz[l * kMaxNz + z] * h0[l]; b += Gz[l * kMaxNz + z] * h1[l]; }
      qc[z * plane + lo] = a; qc[z * plane + mir] = b;
    }
  }
}

// Folded x axis, in place: columns [0, h) of each row hold E, columns [h, nx) hold O; column x
// becomes E + O and column nx-1-x becomes sign (E - O).  A thread takes the column pair
// (x, h-1-x), whose four positions {x, h-1-x, h+x, nx-1-x} it alone reads and writes.
struct Unfold { float* out[4]; float sign[4]; };

__global__ void k_unfold_x(int rows, int nx, Unfold u) {
  const int h = nx / 2, hp = (h + 1) / 2;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)rows * hp) return;
  const int r = (int)(t / hp), x = (int)(t % hp), x2 = h - 1 - x;
  float* row = u.out[blockIdx.y] + (size_t)r * nx;
  const float sg = u.sign[blockIdx.y];
  const float e1 = row[x], o1 = row[h + x];
  const float e2 = row[x2], o2 = row[h + x2];
  row[x] = e1 + o1;
  row[nx - 1 - x] = sg * (e1 - o1);
  if (x2 != x) {
    row[x2] = e2 + o2;
    row[nx - 1 - x2] = sg * (e2 - o2);
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

// A basis operand of a contraction, possibly a sub-block of an n x n basis: its float32 view
// and its k-contiguous bfloat16 split (leading dimension n for both)
struct Basis { const float* f32; const uint16_t* hi; const uint16_t* lo; };

// sub-block at row r, column c of the float32 basis (a right basis, K x N, is stored split
// transposed, so the split offset swaps the roles of r and c)
Basis sub(const Basis& b, int n, bool right, int r, int c) {
  const size_t of = (size_t)r * n + c, os = right ? (size_t)c * n + r : of;
  return {b.f32 + of, b.hi + os, b.lo + os};
}

struct GemmJob { const float* data; Basis basis; float* out; float fold; };

// batched C = A . B where exactly one of A (left_basis) or B is a DCT basis shared by the batch
int gemm(place3d_ctx* c, int M, int N, int K, int nbatch, bool left_basis, int ld_data, int ld_basis, int ldc,
         int fold_n, long long s_data, long long s_out, const GemmJob* jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return PLACE3D_OK;
  if (njobs > kMaxProb) return set_err(c, PLACE3D_ERR_ARG, "too many contractions in one launch");
  const long long tiles = (long long)((N + BN - 1) / BN) * ((M + BM - 1) / BM) * nbatch * njobs;
  if (tiles > 0x7fffffffLL) return set_err(c, PLACE3D_ERR_SIZE, "contraction grid too large");
  const dim3 grid((unsigned)tiles);
  ProfScope prof_(c, PLACE3D_STAGE_GEMM, s);
  if (c->prob.precision == PLACE3D_BF16X3) {
    // 64-row blocks when 128-row ones would leave the chip with fewer than two per compute unit
    const bool half = tiles < 512 && M > 64;
    const long long tiles64 = (long long)((N + BN - 1) / BN) * ((M + 63) / 64) * nbatch * njobs;
    const dim3 grid_s(half ? (unsigned)tiles64 : (unsigned)tiles);
    GemmSplitArgs a;
    a.M = M; a.N = N; a.K = K; a.nbatch = nbatch;
    a.ldd = ld_data; a.ldb = ld_basis; a.ldc = ldc; a.fold_n = fold_n;
    for (int i = 0; i < kMaxProb; ++i) {
      const GemmJob& jb = jobs[i < njobs ? i : 0];
      a.p[i] = {jb.data, jb.basis.hi, jb.basis.lo, jb.out, s_data, s_out, jb.fold};
    }
    if (left_basis) {
      if (half) hipLaunchKernelGGL((k_gemm_bf16x3<true, 64>), grid_s, dim3(256), 0, s, a);
      else hipLaunchKernelGGL((k_gemm_bf16x3<true, 128>), grid_s, dim3(256), 0, s, a);
    } else {
      if (half) hipLaunchKernelGGL((k_gemm_bf16x3<false, 64>), grid_s, dim3(256), 0, s, a);
      else hipLaunchKernelGGL((k_gemm_bf16x3<false, 128>), grid_s, dim3(256), 0, s, a);
    }
  } else {
    GemmArgs a;
    a.M = M; a.N = N; a.K = K; a.nbatch = nbatch;
    a.lda = left_basis ? ld_basis : ld_data;
    a.ldb = left_basis ? ld_data : ld_basis;
    a.ldc = ldc; a.fold_n = fold_n; a.fold_a = left_basis ? 0 : 1;
    for (int i = 0; i < kMaxProb; ++i) {
      const GemmJob& jb = jobs[i < njobs ? i : 0];
      a.p[i] = left_basis ? GemmProb{jb.basis.f32, jb.data, jb.out, 0, s_data, s_out, jb.fold}
                          : GemmProb{jb.data, jb.basis.f32, jb.out, s_data, 0, s_out, jb.fold};
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
  c->dct.fold = (g.nx % 2 == 0 && g.ny % 2 == 0) ? 1 : 0;
  hipLaunchKernelGGL(k_basis_x, dim3(blocks_for((long long)g.nx * g.nx, 256)), dim3(256), 0, s, g.nx, c->dct.fold,
                     p.die_x, c->dct.Fx, c->dct.Gx, c->dct.Hx);
  P3D_LAUNCH(c, "k_basis_x");
  hipLaunchKernelGGL(k_basis_y, dim3(blocks_for((long long)g.ny * g.ny, 256)), dim3(256), 0, s, g.ny, c->dct.fold,
                     p.die_y, c->dct.FyT, c->dct.Gy, c->dct.Hy);
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
  hipLaunchKernelGGL(k_inv_w2, dim3(blocks_for(map, 256)), dim3(256), 0, s, g.nx, g.ny, g.nz, c->dct.fold, p.die_x,
                     p.die_y, dz, c->dct.inv_w2);
  P3D_LAUNCH(c, "k_inv_w2");
  return build_split_chain(c, s);
}

int spectral_field(place3d_ctx* c, const float* rho, float* phi, float* ex, float* ey, float* ez,
                   double* energy, hipStream_t s, bool x_folded_out) {
  const Geom& g = c->g;
  const DctBases& d = c->dct;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long long plane = (long long)nx * ny;
  int rc;
  const Basis Fx{d.Fx, d.Fx_h, d.Fx_l}, Gx{d.Gx, d.Gx_h, d.Gx_l}, Hx{d.Hx, d.Hx_h, d.Hx_l};
  const Basis FyT{d.FyT, d.FyT_h, d.FyT_l}, Gy{d.Gy, d.Gy_h, d.Gy_l}, Hy{d.Hy, d.Hy_h, d.Hy_l};
  const bool need_g = phi || ex || ez, need_h = ey != nullptr;
  float* pc = (phi || ex) ? c->map_pc : nullptr;
  float* ps = ez ? c->map_ps : nullptr;
  float* qc = ey ? c->map_qc : nullptr;
  // the x-inverse outputs: Ex = Pc . Hx, Ey = Qc . Gx, Ez = Ps . Gx, phi = Pc . Gx
  struct XOut { const float* in; Basis b; float* out; float sign; };
  XOut xo[4];
  int nxo = 0;
  if (ex) xo[nxo++] = {c->map_pc, Hx, ex, -1.f};
  if (ey) xo[nxo++] = {c->map_qc, Gx, ey, 1.f};
  if (ez) xo[nxo++] = {c->map_ps, Gx, ez, 1.f};
  if (phi) xo[nxo++] = {c->map_pc, Gx, phi, 1.f};

  if (d.fold) {
    const int hx = nx / 2, hy = ny / 2;
    if (c->sc.on) {
      if ((rc = field_split(c, rho, phi, ex, ey, ez, s))) return rc;
    } else {
    // forward x: T[:, even half] = S . Fx_even, T[:, odd half] = D . Fx_odd with S, D the rows
    // of rho folded about the x middle (+, -)
    {
      const GemmJob j[2] = {{rho, sub(Fx, nx, true, 0, 0), c->map_t, 1.f},
                            {rho, sub(Fx, nx, true, 0, hx), c->map_t + hx, -1.f}};
      if ((rc = gemm(c, nz * ny, hx, hx, 1, false, nx, nx, nx, nx, 0, 0, j, 2, s))) return rc;
    }
    // forward y, per layer: A[even half] = FyT_even . (T folded +), A[odd half] = FyT_odd . (T folded -)
    {
      const GemmJob j[2] = {{c->map_t, sub(FyT, ny, false, 0, 0), c->map_a, 1.f},
                            {c->map_t, sub(FyT, ny, false, hy, 0), c->map_a + (size_t)hy * nx, -1.f}};
      if ((rc = gemm(c, hy, nx, hy, nz, true, nx, ny, nx, ny, plane, plane, j, 2, s))) return rc;
    }
    {
      ProfScope prof_(c, PLACE3D_STAGE_ZMIX, s);
      hipLaunchKernelGGL(k_zmix_fwd, dim3(blocks_for(plane, 256)), dim3(256), 0, s, (int)plane, nz, d.zmat,
                         d.inv_w2, c->map_a);
      P3D_LAUNCH(c, "k_zmix_fwd");
    }
    // inverse y, per layer: E = Gy[:, even half] . b[even half], O = Gy[:, odd half] . b[odd half]
    // into rows [0, hy) and [hy, ny) of vg (and the same with Hy into vh)
    {
      GemmJob j[4];
      int nj = 0;
      if (need_g) {
        j[nj++] = {c->map_a, sub(Gy, ny, false, 0, 0), c->map_vg, 0.f};
        j[nj++] = {c->map_a + (size_t)hy * nx, sub(Gy, ny, false, 0, hy), c->map_vg + (size_t)hy * nx, 0.f};
      }
      if (need_h) {
        j[nj++] = {c->map_a, sub(Hy, ny, false, 0, 0), c->map_vh, 0.f};
        j[nj++] = {c->map_a + (size_t)hy * nx, sub(Hy, ny, false, 0, hy), c->map_vh + (size_t)hy * nx, 0.f};
      }
      if ((rc = gemm(c, hy, nx, hy, nz, true, nx, ny, nx, 0, plane, plane, j, nj, s))) return rc;
    }
    if (pc || ps || qc) {
      ProfScope prof_(c, PLACE3D_STAGE_ZMIX, s);
      hipLaunchKernelGGL(k_zmix_inv_fold, dim3(blocks_for((long long)hy * nx, 256)), dim3(256), 0, s, nx, ny, nz,
                         d.zmat, need_g ? c->map_vg : nullptr, need_h ? c->map_vh : nullptr, pc, ps, qc);
      P3D_LAUNCH(c, "k_zmix_inv_fold");
    }
    // inverse x: E = P[:, even half] . Gx[even half] into columns [0, hx), O likewise into
    // [hx, nx); then each row is unfolded in place
    {
      GemmJob j[8];
      int nj = 0;
      for (int q = 0; q < nxo; ++q) {
        j[nj++] = {xo[q].in, sub(xo[q].b, nx, true, 0, 0), xo[q].out, 0.f};
        j[nj++] = {xo[q].in + hx, sub(xo[q].b, nx, true, hx, 0), xo[q].out + hx, 0.f};
      }
      if ((rc = gemm(c, nz * ny, hx, hx, 1, false, nx, nx, nx, 0, 0, 0, j, nj, s))) return rc;
    }
    }
    // the split chain unfolds x in its last contraction
    c->field_xfold = x_folded_out && !phi && !energy && !c->sc.on;
    if (nxo > 0 && !c->field_xfold && !c->sc.on) {
      ProfScope prof_(c, PLACE3D_STAGE_ZMIX, s);
      Unfold u;
      for (int q = 0; q < 4; ++q) {
        u.out[q] = xo[q < nxo ? q : 0].out;
        u.sign[q] = xo[q < nxo ? q : 0].sign;
      }
      const long long work = (long long)nz * ny * ((hx + 1) / 2);
      hipLaunchKernelGGL(k_unfold_x, dim3(blocks_for(work, 256), nxo), dim3(256), 0, s, nz * ny, nx, u);
      P3D_LAUNCH(c, "k_unfold_x");
    }
  } else {
    c->field_xfold = 0;
    // dense contractions in natural frequency order
    {
      const GemmJob j[1] = {{rho, Fx, c->map_t, 0.f}};
      if ((rc = gemm(c, nz * ny, nx, nx, 1, false, nx, nx, nx, 0, 0, 0, j, 1, s))) return rc;
    }
    {
      const GemmJob j[1] = {{c->map_t, FyT, c->map_a, 0.f}};
      if ((rc = gemm(c, ny, nx, ny, nz, true, nx, ny, nx, 0, plane, plane, j, 1, s))) return rc;
    }
    {
      ProfScope prof_(c, PLACE3D_STAGE_ZMIX, s);
      hipLaunchKernelGGL(k_zmix_fwd, dim3(blocks_for(plane, 256)), dim3(256), 0, s, (int)plane, nz, d.zmat,
                         d.inv_w2, c->map_a);
      P3D_LAUNCH(c, "k_zmix_fwd");
    }
    {
      GemmJob j[2];
      int nj = 0;
      if (need_g) j[nj++] = {c->map_a, Gy, c->map_vg, 0.f};
      if (need_h) j[nj++] = {c->map_a, Hy, c->map_vh, 0.f};
      if ((rc = gemm(c, ny, nx, ny, nz, true, nx, ny, nx, 0, plane, plane, j, nj, s))) return rc;
    }
    if (pc || ps || qc) {
      ProfScope prof_(c, PLACE3D_STAGE_ZMIX, s);
      hipLaunchKernelGGL(k_zmix_inv, dim3(blocks_for(plane, 256)), dim3(256), 0, s, (int)plane, nz, d.zmat,
                         need_g ? c->map_vg : nullptr, need_h ? c->map_vh : nullptr, pc, ps, qc);
      P3D_LAUNCH(c, "k_zmix_inv");
    }
    {
      GemmJob j[4];
      for (int q = 0; q < nxo; ++q) j[q] = {xo[q].in, xo[q].b, xo[q].out, 0.f};
      if ((rc = gemm(c, nz * ny, nx, nx, 1, false, nx, nx, nx, 0, 0, 0, j, nxo, s))) return rc;
    }
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
