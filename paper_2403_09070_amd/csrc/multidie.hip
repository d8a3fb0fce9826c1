// Multi-die 2D global placement (Sec. III-C, Eq. 2d-place) on the library's 3D machinery.
//
// The three 2D systems (bottom die, top die, HBT layer) each run as a context of their own over
// the layer's nodes, on the same planar grid with two z bins and every node at the mid-plane
// z = d_z/2 at equal bottom and top sizes.  Its cuboid [z - d_z/4, z + d_z/4] then covers half of
// each z bin, so the map is uniform in z, rho_3 = rho / 2, the cosine solve keeps only its l = 0
// modes (the 2D solve), phi_3 = phi / 2, E_3 = E / 2 with E_z = 0, and exactly
//     field gather: grad_3 = (d_z/4) grad       energy: U_3 = (d_z/4) U
//     overflow excess with target rho_t/2:  excess_3 = (d_z/2) excess,
// the 2D quantities of the layer scaled by constants.  A fourth context holds every node at the
// mid-plane with the partial nets, alpha = 0 and both dies' offsets equal: every net then lies on
// one die, its bistratal model is the plain WA of the partial net in x and y (Eq. wa-model-approx)
// and its exact value the partial net's HPWL.  The step kernels here combine the parts with each
// node's layer weight and take the optimiser's move in x and y.
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

using namespace p3d;

namespace {

enum MdSlot {   // float64 reduction slots of the multi-die context
  M_DV2 = 0, M_DG2, M_GMAX, M_L1W, M_L1D = M_L1W + 3, M_COUNT = M_L1D + 3
};

}  // namespace

struct place3d_md2d_ctx {
  place3d_md2d_problem prob;
  std::string err;
  place3d_ctx* wl = nullptr;
  place3d_ctx* lay[3] = {nullptr, nullptr, nullptr};
  int n_of[3] = {0, 0, 0};
  double area[3] = {0, 0, 0};   // movable non-filler area of each layer
  float zmid = 0.f;             // the nodes' z in the sub-problems
  float dz = 0.f;               // d_z of the two-bin grid
  // device, in the workspace
  float *wl_size = nullptr, *wl_off = nullptr, *wl_fixed = nullptr;
  uint8_t* wl_kind = nullptr;
  float *l_size[3] = {}, *l_fixed[3] = {};
  uint8_t* l_kind[3] = {};
  int32_t* l_start[3] = {};
  int32_t* node_local = nullptr;     // [n] index of a node in its layer's sub-problem
  float* xyz_wl = nullptr;           // [3][n]
  float* g_wl = nullptr;             // [3][n]
  float* xyz_l[3] = {};              // [3][n_L]
  float* g_l[3] = {};                // [3][n_L]
  double* red = nullptr;             // [M_COUNT]
  double* part = nullptr;
  int part_stride = 0;
  char* sub_ws[4] = {};
  size_t sub_bytes[4] = {};
  // an evaluation forks the wirelength and the three layers onto the sub-contexts' side streams
  hipEvent_t ev_fork = nullptr, ev_done[4] = {};
  ~place3d_md2d_ctx() {
    place3d_destroy(wl);
    for (auto* c : lay) place3d_destroy(c);
    if (ev_fork) hipEventDestroy(ev_fork);
    for (auto& ev : ev_done)
      if (ev) hipEventDestroy(ev);
  }
};

namespace {

thread_local std::string g_md_err;

int md_err(place3d_md2d_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg; else g_md_err = msg;
  return code;
}

// ------------------------------------------------------------------ kernels

// positions of the sub-problems: every node at (x, y, zmid) in the wirelength context and in its
// layer's context
__global__ void k_md_pack(int n, const float* __restrict__ xy, const uint8_t* __restrict__ layer,
                          const int32_t* __restrict__ local, float zmid, float* __restrict__ xyz_wl, float* l0,
                          float* l1, float* l2, int n0, int n1, int n2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = xy[i], y = xy[n + i];
  xyz_wl[i] = x; xyz_wl[n + i] = y; xyz_wl[2 * n + i] = zmid;
  const int L = layer[i], j = local[i];
  float* d = L == 0 ? l0 : (L == 1 ? l1 : l2);
  const int m = L == 0 ? n0 : (L == 1 ? n1 : n2);
  d[j] = x; d[m + j] = y; d[2 * m + j] = zmid;
}

struct LayerGrads {
  const float* g[3];
  int n[3];
};

__device__ __forceinline__ void den_grad(const LayerGrads& lg, const uint8_t* __restrict__ layer,
                                         const int32_t* __restrict__ local, int i, float& gx, float& gy) {
  const int L = layer[i], j = local[i];
  const float* g = L == 0 ? lg.g[0] : (L == 1 ? lg.g[1] : lg.g[2]);
  const int m = L == 0 ? lg.n[0] : (L == 1 ? lg.n[1] : lg.n[2]);
  gx = g[j];
  gy = g[m + j];
}

// the two objective parts per node (grad_wl: x, y of the wirelength context's gradient)
__global__ void k_md_parts(int n, const uint8_t* __restrict__ layer, const int32_t* __restrict__ local,
                           const float* __restrict__ g_wl, LayerGrads lg, float* __restrict__ gw,
                           float* __restrict__ gd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  gw[i] = g_wl[i];
  gw[n + i] = g_wl[n + i];
  float x, y;
  den_grad(lg, layer, local, i, x, y);
  gd[i] = x;
  gd[n + i] = y;
}

// layer L's map rho = rho_3[z = 0] + rho_3[z = 1] (each holds half)
__global__ void k_md_map(long long plane, const float* __restrict__ r3, float* __restrict__ out) {
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < plane; q += (long long)gridDim.x * blockDim.x)
    out[q] = r3[q] + r3[plane + q];
}

template <int NQ>
__device__ __forceinline__ void md_partials(double (&v)[NQ], double* __restrict__ part, int stride, int slot0) {
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

__device__ __forceinline__ void clamp2(const float* __restrict__ size, int n, int i, float& x, float& y, float dx,
                                       float dy) {
  const float w = size[i], h = size[n + i];
  x = fminf(fmaxf(x, 0.5f * w), dx - 0.5f * w);
  y = fminf(fmaxf(y, 0.5f * h), dy - 0.5f * h);
}

// u = v = clamp(xy0)
__global__ void k_md_clamp_copy(int n, const float* __restrict__ size, const uint8_t* __restrict__ kind, float dx,
                                float dy, const float* __restrict__ src, float* __restrict__ u, float* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float x = src[i], y = src[n + i];
  if (!(kind[i] & PLACE3D_KIND_FIXED)) clamp2(size, n, i, x, y, dx, dy);
  u[i] = x; u[n + i] = y;
  v[i] = x; v[n + i] = y;
}

// |grad W|_1 and |grad U_L|_1 over each layer's movable nodes
__global__ void k_md_l1(int n, const uint8_t* __restrict__ kind, const uint8_t* __restrict__ layer,
                        const int32_t* __restrict__ local, const float* __restrict__ g_wl, LayerGrads lg,
                        double* __restrict__ part, int stride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double v[6] = {0, 0, 0, 0, 0, 0};
  if (i < n && !(kind[i] & PLACE3D_KIND_FIXED)) {
    const int L = layer[i];
    float x, y;
    den_grad(lg, layer, local, i, x, y);
    const double w = fabs((double)g_wl[i]) + fabs((double)g_wl[n + i]), d = fabs((double)x) + fabs((double)y);
#pragma unroll
    for (int q = 0; q < 3; ++q) {      // selects, not a runtime index into the register array
      v[q] = L == q ? w : 0.0;
      v[3 + q] = L == q ? d : 0.0;
    }
  }
  md_partials<6>(v, part, stride, M_L1W);
}

// g = (grad W + lambda_L grad U_L) / H, H of Eq. improved-precond with q = w h and the node's layer
// weight.  Mode 0: g to gout and max|g| partials; mode 1: |v - v_prev|^2 and |g - g_prev|^2
// partials, g over g_prev.
__global__ void k_md_combine(int n, const float* __restrict__ size, const uint8_t* __restrict__ kind,
                             const uint8_t* __restrict__ layer, const int32_t* __restrict__ local,
                             const float* __restrict__ npins, const float* __restrict__ v,
                             const float* __restrict__ v_prev, const float* __restrict__ g_wl, LayerGrads lg,
                             const double* __restrict__ sc, int mode, float* __restrict__ gout,
                             double* __restrict__ part, int stride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double acc[2] = {0.0, 0.0};
  if (i < n) {
    const uint8_t k = kind[i];
    float gv[2] = {0.f, 0.f};
    if (!(k & PLACE3D_KIND_FIXED)) {
      const int L = layer[i];
      const double lam = sc[PLACE3D_MS_LAMBDA + L];
      const double lq = lam * (double)size[i] * (double)size[n + i];
      const double H = (k & PLACE3D_KIND_MACRO) ? fmax(1.0, (double)npins[i] + lq) : fmax(1.0, lq);
      float d[2];
      den_grad(lg, layer, local, i, d[0], d[1]);
      for (int a = 0; a < 2; ++a) gv[a] = (float)(((double)g_wl[a * n + i] + lam * (double)d[a]) / H);
      if (mode == 1) {
        for (int a = 0; a < 2; ++a) {
          const double dv = (double)v[a * n + i] - (double)v_prev[a * n + i];
          const double dg = (double)gv[a] - (double)gout[a * n + i];
          acc[0] += dv * dv;
          acc[1] += dg * dg;
        }
      } else {
        acc[0] = fmax(fabs((double)gv[0]), fabs((double)gv[1]));
      }
    }
    gout[i] = gv[0];
    gout[n + i] = gv[1];
  }
  if (mode == 1) {
    md_partials<2>(acc, part, stride, M_DV2);
  } else {
    __shared__ double shm[256 / kWave];
    double m = acc[0];
    for (int o = kWave / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & (kWave - 1)) == 0) shm[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = 0.0;
      for (int w = 0; w < 256 / kWave; ++w) r = fmax(r, shm[w]);
      part[(size_t)M_GMAX * stride + blockIdx.x] = r;
    }
  }
}

__global__ void k_md_init_scalars(double* __restrict__ sc, const double* __restrict__ red) {
  if (threadIdx.x != 0) return;
  for (int q = 0; q < PLACE3D_NSCALARS; ++q) sc[q] = 0.0;
  sc[PLACE3D_MS_A] = 1.0;
  bool finite = true;
  for (int L = 0; L < 3; ++L) {
    const double w = red[M_L1W + L], d = red[M_L1D + L];
    sc[PLACE3D_MS_LAMBDA + L] = d > 0.0 ? w / d : 0.0;
    finite = finite && isfinite(w) && isfinite(d) && isfinite(sc[PLACE3D_MS_LAMBDA + L]);
  }
  if (!finite) sc[PLACE3D_MS_NONFINITE] = 1.0;
}

// v_prev = clamp(v - 0.01 w_b g / max|g|)
__global__ void k_md_bootstrap(int n, const float* __restrict__ size, const uint8_t* __restrict__ kind, float dx,
                               float dy, float wb, const float* __restrict__ v, const float* __restrict__ g0,
                               const double* __restrict__ red, float* __restrict__ v_prev) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double gmax = red[M_GMAX];
  const float f = gmax > 0.0 ? (float)(0.01 * (double)wb / gmax) : 0.f;
  float x = v[i], y = v[n + i];
  if (!(kind[i] & PLACE3D_KIND_FIXED)) {
    x -= f * g0[i];
    y -= f * g0[n + i];
    clamp2(size, n, i, x, y, dx, dy);
  }
  v_prev[i] = x;
  v_prev[n + i] = y;
}

__global__ void k_md_nesterov(int n, const float* __restrict__ size, const uint8_t* __restrict__ kind, float dx,
                              float dy, const double* __restrict__ sc, const double* __restrict__ red,
                              float* __restrict__ u, float* __restrict__ v, float* __restrict__ v_prev,
                              const float* __restrict__ gk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double dv2 = red[M_DV2], dg2 = red[M_DG2];
  const float st = (float)(dg2 > 0.0 ? sqrt(dv2 / dg2) : 0.0);
  const double a = sc[PLACE3D_MS_A];
  const double a1 = 0.5 * (1.0 + sqrt(4.0 * a * a + 1.0));
  const float coef = (float)((a - 1.0) / a1);
  const float vx = v[i], vy = v[n + i];
  v_prev[i] = vx;
  v_prev[n + i] = vy;
  if (kind[i] & PLACE3D_KIND_FIXED) return;
  float ux = vx - st * gk[i], uy = vy - st * gk[n + i];
  clamp2(size, n, i, ux, uy, dx, dy);
  float nx = ux + coef * (ux - u[i]), ny = uy + coef * (uy - u[n + i]);
  clamp2(size, n, i, nx, ny, dx, dy);
  u[i] = ux; u[n + i] = uy;
  v[i] = nx; v[n + i] = ny;
}

struct LayerRed { const double* r[3]; double scale[3]; };   // excess slots and (2/d_z)/area per layer

// wirelength totals and the layers' overflow at the evaluation point (slots 0..4 of out)
__device__ __forceinline__ void md_metrics(const double* __restrict__ wl_red, const LayerRed& lr, double* out) {
  out[PLACE3D_MD_WA] = wl_red[R_WA_BI];
  out[PLACE3D_MD_HPWL] = wl_red[R_HPWL];
  for (int L = 0; L < 3; ++L)
    out[PLACE3D_MD_OVFL + L] = (lr.r[L][R_EXCESS_BOT] + lr.r[L][R_EXCESS_TOP]) * lr.scale[L];
}

__global__ void k_md_step_finish(double* __restrict__ sc, const double* __restrict__ red,
                                 const double* __restrict__ wl_red, LayerRed lr, double ramp) {
  if (threadIdx.x != 0) return;
  const double dv2 = red[M_DV2], dg2 = red[M_DG2];
  const double a = sc[PLACE3D_MS_A];
  sc[PLACE3D_MS_STEP] = dg2 > 0.0 ? sqrt(dv2 / dg2) : 0.0;
  sc[PLACE3D_MS_A] = 0.5 * (1.0 + sqrt(4.0 * a * a + 1.0));
  for (int L = 0; L < 3; ++L) sc[PLACE3D_MS_LAMBDA + L] *= ramp;
  sc[PLACE3D_MS_ITER] += 1.0;
  md_metrics(wl_red, lr, sc + PLACE3D_MS_METRICS);
  bool finite = isfinite(dv2) && isfinite(dg2);
  for (int q = 0; q < 5; ++q) finite = finite && isfinite(sc[PLACE3D_MS_METRICS + q]);
  for (int L = 0; L < 3; ++L) finite = finite && isfinite(sc[PLACE3D_MS_LAMBDA + L]);
  if (!finite && sc[PLACE3D_MS_NONFINITE] == 0.0) sc[PLACE3D_MS_NONFINITE] = sc[PLACE3D_MS_ITER];
}

__global__ void k_md_eval_metrics(const double* __restrict__ wl_red, LayerRed lr, const double* __restrict__ en,
                                  double energy_scale, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  for (int q = 0; q < PLACE3D_NMETRICS; ++q) out[q] = 0.0;
  md_metrics(wl_red, lr, out);
  for (int L = 0; L < 3; ++L) out[PLACE3D_MD_ENERGY + L] = en ? en[L] * energy_scale : 0.0;
}

// ------------------------------------------------------------------ host side

struct Carve {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// the sub-problems (device pointers filled in by the caller of this function)
place3d_problem wl_problem(const place3d_md2d_problem& p) {
  place3d_problem q = {};
  q.n_inst = p.n_nodes; q.n_pins = p.n_pins; q.n_nets = p.n_nets;
  q.nx = p.nx; q.ny = p.ny; q.nz = 2;
  q.die_x = p.die_x; q.die_y = p.die_y;
  q.gamma = p.gamma; q.alpha = 0.0; q.target_density = p.target_density; q.lambda_ramp = 1.0;
  q.precision = p.precision; q.dgrad = PLACE3D_DGRAD_FIELD; q.precond = PLACE3D_PRECOND_MIXED; q.options = 0;
  return q;
}

place3d_problem layer_problem(const place3d_md2d_problem& p, int n_l) {
  place3d_problem q = {};
  q.n_inst = n_l; q.n_pins = 0; q.n_nets = 0;
  q.nx = p.nx; q.ny = p.ny; q.nz = 2;
  q.die_x = p.die_x; q.die_y = p.die_y;
  q.gamma = p.gamma; q.alpha = 0.0;
  q.target_density = 0.5 * p.target_density;     // the layer's map holds half the 2D density per z bin
  q.lambda_ramp = 1.0;
  q.precision = p.precision; q.dgrad = PLACE3D_DGRAD_FIELD; q.precond = PLACE3D_PRECOND_MIXED; q.options = 0;
  return q;
}

// placeholder device pointers for sizing a sub-problem (never dereferenced)
void fake_arrays(place3d_problem& q) {
  static const float f = 0.f;
  static const uint8_t b = 0;
  static const int32_t i = 0;
  q.size = &f; q.kind = &b; q.net_start = &i; q.fixed_xyz = &f;
  if (q.n_pins > 0) { q.pin2node = &i; q.pin_off = &f; }
}

int check_md(const place3d_md2d_problem* p, std::string& why) {
  if (!p) { why = "problem is NULL"; return PLACE3D_ERR_ARG; }
  if (p->n_nodes < 3 || p->n_pins < 0 || p->n_nets < 0) { why = "n_nodes < 3 or negative pin/net count"; return PLACE3D_ERR_SIZE; }
  for (int L = 0; L < 3; ++L)
    if (p->n_layer[L] < 1) { why = "every layer needs a node"; return PLACE3D_ERR_SIZE; }
  if ((long long)p->n_layer[0] + p->n_layer[1] + p->n_layer[2] != p->n_nodes) {
    why = "n_layer does not add up to n_nodes";
    return PLACE3D_ERR_SIZE;
  }
  if (!p->size || !p->kind || !p->layer || !p->net_start || !p->fixed_xy) { why = "null device array"; return PLACE3D_ERR_ARG; }
  if (p->n_pins > 0 && (!p->pin2node || !p->pin_off)) { why = "null pin arrays"; return PLACE3D_ERR_ARG; }
  if ((reinterpret_cast<uintptr_t>(p->size) | reinterpret_cast<uintptr_t>(p->fixed_xy) |
       reinterpret_cast<uintptr_t>(p->pin_off) | reinterpret_cast<uintptr_t>(p->net_start) |
       reinterpret_cast<uintptr_t>(p->pin2node)) & 3) { why = "misaligned device array"; return PLACE3D_ERR_ARG; }
  return PLACE3D_OK;
}

// carve the multi-die workspace: the four sub-workspaces, then the arrays of this context
int md_layout(place3d_md2d_ctx* c, const place3d_md2d_problem& p, char* base, size_t& total, std::string& why) {
  Carve w{base};
  place3d_problem sub[4] = {wl_problem(p), layer_problem(p, p.n_layer[0]), layer_problem(p, p.n_layer[1]),
                            layer_problem(p, p.n_layer[2])};
  for (int k = 0; k < 4; ++k) {
    fake_arrays(sub[k]);
    size_t b = 0;
    const int rc = place3d_workspace_size(&sub[k], &b);
    if (rc != PLACE3D_OK) { why = std::string("sub-problem: ") + place3d_last_error(nullptr); return rc; }
    c->sub_bytes[k] = b;
    c->sub_ws[k] = w.take<char>(b);
  }
  const size_t n = p.n_nodes, P = p.n_pins;
  c->wl_size = w.take<float>(4 * n);
  c->wl_kind = w.take<uint8_t>(n);
  c->wl_off = w.take<float>(4 * P + 1);
  c->wl_fixed = w.take<float>(3 * n);
  c->node_local = w.take<int32_t>(n);
  c->xyz_wl = w.take<float>(3 * n);
  c->g_wl = w.take<float>(3 * n);
  for (int L = 0; L < 3; ++L) {
    const size_t m = p.n_layer[L];
    c->l_size[L] = w.take<float>(4 * m);
    c->l_kind[L] = w.take<uint8_t>(m);
    c->l_fixed[L] = w.take<float>(3 * m);
    c->l_start[L] = w.take<int32_t>(1);
    c->xyz_l[L] = w.take<float>(3 * m);
    c->g_l[L] = w.take<float>(3 * m);
  }
  c->red = w.take<double>(M_COUNT);
  c->part_stride = (int)blocks_for(p.n_nodes, 256);
  c->part = w.take<double>((size_t)M_COUNT * c->part_stride);
  total = (w.off + 255) & ~size_t(255);
  return PLACE3D_OK;
}

LayerGrads layer_grads(const place3d_md2d_ctx* c) {
  LayerGrads lg;
  for (int L = 0; L < 3; ++L) { lg.g[L] = c->g_l[L]; lg.n[L] = c->n_of[L]; }
  return lg;
}

LayerRed layer_red(const place3d_md2d_ctx* c) {
  LayerRed lr;
  for (int L = 0; L < 3; ++L) {
    lr.r[L] = c->lay[L]->red2;
    lr.scale[L] = c->area[L] > 0.0 ? 2.0 / (double)c->dz / c->area[L] : 0.0;
  }
  return lr;
}

#define MD_HIP(c, call)                                                                     \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return md_err((c), PLACE3D_ERR_HIP, std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_)); \
  } while (0)

#define MD_SUB(c, sub, call)                                                                \
  do {                                                                                      \
    const int rc_ = (call);                                                                 \
    if (rc_ != PLACE3D_OK) return md_err((c), rc_, std::string(place3d_last_error(sub)));   \
  } while (0)

// both objective parts at xy: the wirelength context's gradient into g_wl, each layer's 2D
// field-gather gradient into g_l; with energy, also phi and U_3 of each layer into en[3]
// The partial nets' wirelength and the three layers' density chains share nothing but the packed
// positions: after the pack on s they run concurrently, each on its sub-context's side stream
// (default priority), and s waits for all four before anything reads their results.
int md_evaluate(place3d_md2d_ctx* c, const float* xy, hipStream_t s, double* en = nullptr) {
  const place3d_md2d_problem& p = c->prob;
  const int n = p.n_nodes;
  hipLaunchKernelGGL(k_md_pack, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, xy, p.layer, c->node_local, c->zmid,
                     c->xyz_wl, c->xyz_l[0], c->xyz_l[1], c->xyz_l[2], c->n_of[0], c->n_of[1], c->n_of[2]);
  MD_HIP(c, hipGetLastError());
  MD_HIP(c, hipEventRecord(c->ev_fork, s));
  hipStream_t ws = c->wl->side;
  MD_HIP(c, hipStreamWaitEvent(ws, c->ev_fork, 0));
  MD_SUB(c, c->wl, wirelength_eval(c->wl, c->xyz_wl, c->g_wl, 0, c->wl->red, nullptr, ws, false, nullptr, false));
  MD_HIP(c, hipEventRecord(c->ev_done[0], ws));
  for (int L = 0; L < 3; ++L) {
    place3d_ctx* lc = c->lay[L];
    hipStream_t ls = lc->side;
    MD_HIP(c, hipStreamWaitEvent(ls, c->ev_fork, 0));
    MD_SUB(c, lc, density_forward(lc, c->xyz_l[L], lc->rho, ls));
    MD_SUB(c, lc, spectral_field(lc, lc->rho, en ? lc->phi : nullptr, lc->ex, lc->ey, nullptr, en ? en + L : nullptr, ls));
    // grad = (4/d_z) grad_3: the layer's 2D field-gather gradient; E_z is read from a zero map
    MD_SUB(c, lc, gather_bucketed(lc, c->xyz_l[L], lc->ex, lc->ey, lc->ez, -4.f / c->dz, c->g_l[L], 0, ls));
    MD_HIP(c, hipEventRecord(c->ev_done[1 + L], ls));
  }
  for (auto& ev : c->ev_done) MD_HIP(c, hipStreamWaitEvent(s, ev, 0));
  return PLACE3D_OK;
}

int md_reduce(place3d_md2d_ctx* c, int slot0, int nq, bool is_max, hipStream_t s) {
  MD_SUB(c, c->wl, reduce_final_in(c->wl, c->part, c->part_stride, slot0, nq, (int)blocks_for(c->prob.n_nodes, 256),
                                   is_max, c->red + slot0, s));
  return PLACE3D_OK;
}

int check_state(place3d_md2d_ctx* c, const place3d_md2d_state* st) {
  if (!st || !st->u || !st->v || !st->v_prev || !st->g_prev || !st->scalars)
    return md_err(c, PLACE3D_ERR_ARG, "state has a NULL array");
  if ((reinterpret_cast<uintptr_t>(st->u) | reinterpret_cast<uintptr_t>(st->v) |
       reinterpret_cast<uintptr_t>(st->v_prev) | reinterpret_cast<uintptr_t>(st->g_prev)) & 3 ||
      (reinterpret_cast<uintptr_t>(st->scalars) & 7))
    return md_err(c, PLACE3D_ERR_ARG, "misaligned state array");
  return PLACE3D_OK;
}

}  // namespace

extern "C" {

int32_t place3d_md2d_workspace_size(const place3d_md2d_problem* prob, size_t* bytes) {
  std::string why;
  int rc = check_md(prob, why);
  if (rc != PLACE3D_OK) { g_md_err = why; return rc; }
  if (!bytes) { g_md_err = "bytes is NULL"; return PLACE3D_ERR_ARG; }
  place3d_md2d_ctx tmp;
  size_t total = 0;
  rc = md_layout(&tmp, *prob, nullptr, total, why);
  if (rc != PLACE3D_OK) { g_md_err = why; return rc; }
  *bytes = total;
  return PLACE3D_OK;
}

const char* place3d_md2d_last_error(const place3d_md2d_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_md_err.c_str();
}

int32_t place3d_md2d_create(const place3d_md2d_problem* prob, void* d_workspace, size_t bytes, void* stream,
                            place3d_md2d_ctx** out) {
  std::string why;
  int rc = check_md(prob, why);
  if (rc != PLACE3D_OK) { g_md_err = why; return rc; }
  if (!out) { g_md_err = "out is NULL"; return PLACE3D_ERR_ARG; }
  *out = nullptr;
  if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255)) {
    g_md_err = "workspace NULL or not 256-byte aligned";
    return PLACE3D_ERR_ARG;
  }
  place3d_md2d_ctx* c = new (std::nothrow) place3d_md2d_ctx();
  if (!c) { g_md_err = "out of host memory"; return PLACE3D_ERR_ARG; }
  c->prob = *prob;
  const place3d_md2d_problem& p = c->prob;
  size_t need = 0;
  rc = md_layout(c, p, reinterpret_cast<char*>(d_workspace), need, why);
  if (rc == PLACE3D_OK && bytes < need) { why = "workspace too small: need " + std::to_string(need) + " bytes"; rc = PLACE3D_ERR_SIZE; }
  if (rc != PLACE3D_OK) { g_md_err = why; delete c; return rc; }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t n = p.n_nodes, P = p.n_pins;
  // the node arrays, read back once
  std::vector<float> size(2 * n), fxy(2 * n), off(2 * P);
  std::vector<uint8_t> kind(n), layer(n);
  auto fail = [&](int code, const std::string& msg) { g_md_err = msg; delete c; return code; };
  hipError_t e = hipMemcpyAsync(size.data(), p.size, sizeof(float) * 2 * n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(fxy.data(), p.fixed_xy, sizeof(float) * 2 * n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(kind.data(), p.kind, n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(layer.data(), p.layer, n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && P > 0) e = hipMemcpyAsync(off.data(), p.pin_off, sizeof(float) * 2 * P, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(PLACE3D_ERR_HIP, std::string("reading the problem back: ") + hipGetErrorString(e));
  // the sub-problems' arrays
  const double wb = p.die_x / p.nx, hb = p.die_y / p.ny;
  c->dz = (float)(2.0 * 0.5 * (wb + hb));            // d_z of the two-bin grid
  c->zmid = 0.5f * c->dz;
  std::vector<int32_t> local(n);
  std::vector<float> wl_size(4 * n), wl_fixed(3 * n), wl_off(4 * P + 1, 0.f);
  std::vector<uint8_t> wl_kind(n);
  std::vector<float> l_size[3], l_fixed[3];
  std::vector<uint8_t> l_kind[3];
  int cnt[3] = {0, 0, 0};
  for (size_t i = 0; i < n; ++i) {
    const int L = layer[i];
    if (L > 2) return fail(PLACE3D_ERR_ARG, "layer value beyond PLACE3D_LAYER_HBT");
    if (kind[i] & ~(PLACE3D_KIND_MACRO | PLACE3D_KIND_FIXED | PLACE3D_KIND_FILLER))
      return fail(PLACE3D_ERR_ARG, "node kind beyond MACRO, FIXED, FILLER");
    local[i] = cnt[L]++;
  }
  for (int L = 0; L < 3; ++L) {
    if (cnt[L] != p.n_layer[L]) return fail(PLACE3D_ERR_SIZE, "n_layer does not match the layer array");
    c->n_of[L] = cnt[L];
    l_size[L].resize(4 * (size_t)cnt[L]);
    l_fixed[L].resize(3 * (size_t)cnt[L]);
    l_kind[L].resize(cnt[L]);
  }
  for (size_t i = 0; i < n; ++i) {
    const float w = size[i], h = size[n + i];
    if (!(w > 0.f) || !(h > 0.f) || !std::isfinite(w) || !std::isfinite(h)) return fail(PLACE3D_ERR_ARG, "node size not positive");
    const int L = layer[i];
    const size_t j = local[i], m = cnt[L];
    for (int q = 0; q < 2; ++q) { wl_size[2 * q * n + i] = w; wl_size[(2 * q + 1) * n + i] = h; }
    wl_fixed[i] = fxy[i]; wl_fixed[n + i] = fxy[n + i]; wl_fixed[2 * n + i] = c->zmid;
    wl_kind[i] = kind[i];
    for (int q = 0; q < 2; ++q) { l_size[L][2 * q * m + j] = w; l_size[L][(2 * q + 1) * m + j] = h; }
    l_fixed[L][j] = fxy[i]; l_fixed[L][m + j] = fxy[n + i]; l_fixed[L][2 * m + j] = c->zmid;
    l_kind[L][j] = kind[i];
    if (!(kind[i] & (PLACE3D_KIND_FIXED | PLACE3D_KIND_FILLER))) c->area[L] += (double)w * (double)h;
  }
  for (size_t k = 0; k < P; ++k)
    for (int q = 0; q < 2; ++q) { wl_off[2 * q * P + k] = off[k]; wl_off[(2 * q + 1) * P + k] = off[P + k]; }
  const int32_t zero = 0;
  e = hipMemcpyAsync(c->node_local, local.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->wl_size, wl_size.data(), sizeof(float) * 4 * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->wl_fixed, wl_fixed.data(), sizeof(float) * 3 * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->wl_kind, wl_kind.data(), n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->wl_off, wl_off.data(), sizeof(float) * (4 * P + 1), hipMemcpyHostToDevice, s);
  for (int L = 0; L < 3 && e == hipSuccess; ++L) {
    const size_t m = cnt[L];
    e = hipMemcpyAsync(c->l_size[L], l_size[L].data(), sizeof(float) * 4 * m, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->l_fixed[L], l_fixed[L].data(), sizeof(float) * 3 * m, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->l_kind[L], l_kind[L].data(), m, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->l_start[L], &zero, sizeof(int32_t), hipMemcpyHostToDevice, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(PLACE3D_ERR_HIP, std::string("uploading the sub-problems: ") + hipGetErrorString(e));
  // the four contexts
  place3d_problem q = wl_problem(p);
  q.size = c->wl_size; q.kind = c->wl_kind; q.net_start = p.net_start; q.pin2node = p.pin2node;
  q.pin_off = c->wl_off; q.fixed_xyz = c->wl_fixed;
  rc = place3d_create(&q, c->sub_ws[0], c->sub_bytes[0], stream, &c->wl);
  if (rc != PLACE3D_OK) return fail(rc, std::string("wirelength context: ") + place3d_last_error(nullptr));
  for (int L = 0; L < 3; ++L) {
    place3d_problem r = layer_problem(p, cnt[L]);
    r.size = c->l_size[L]; r.kind = c->l_kind[L]; r.net_start = c->l_start[L]; r.fixed_xyz = c->l_fixed[L];
    rc = place3d_create(&r, c->sub_ws[1 + L], c->sub_bytes[1 + L], stream, &c->lay[L]);
    if (rc != PLACE3D_OK) return fail(rc, "layer " + std::to_string(L) + " context: " + place3d_last_error(nullptr));
    // E_z of a z-uniform map is zero: the gather reads it from a zero map
    const long long map = (long long)p.nx * p.ny * 2;
    rc = launch_fill_f32(c->lay[L], c->lay[L]->ez, map, 0.f, s);
    if (rc != PLACE3D_OK) return fail(rc, place3d_last_error(c->lay[L]));
  }
  e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
  for (auto& ev : c->ev_done)
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(PLACE3D_ERR_HIP, std::string("create: ") + hipGetErrorString(e));
  *out = c;
  return PLACE3D_OK;
}

int32_t place3d_md2d_destroy(place3d_md2d_ctx* ctx) {
  delete ctx;
  return PLACE3D_OK;
}

int32_t place3d_md2d_eval(place3d_md2d_ctx* c, const float* xy, float* grad_wl, float* grad_den, float* rho,
                          double* metrics, void* stream) {
  if (!c) { g_md_err = "ctx is NULL"; return PLACE3D_ERR_ARG; }
  auto bad = [](const void* q) { return !q || (reinterpret_cast<uintptr_t>(q) & 3); };
  if (bad(xy) || bad(grad_wl) || bad(grad_den)) return md_err(c, PLACE3D_ERR_ARG, "NULL or misaligned array");
  if ((rho && (reinterpret_cast<uintptr_t>(rho) & 3)) || (metrics && (reinterpret_cast<uintptr_t>(metrics) & 7)))
    return md_err(c, PLACE3D_ERR_ARG, "misaligned output");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const place3d_md2d_problem& p = c->prob;
  const int n = p.n_nodes;
  double* en = c->red + M_COUNT - 3;       // three scratch slots for the layers' U_3 (the L1 slots)
  if (int rc = md_evaluate(c, xy, s, metrics ? en : nullptr)) return rc;
  hipLaunchKernelGGL(k_md_parts, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, p.layer, c->node_local, c->g_wl,
                     layer_grads(c), grad_wl, grad_den);
  MD_HIP(c, hipGetLastError());
  if (rho) {
    const long long plane = (long long)p.nx * p.ny;
    for (int L = 0; L < 3; ++L) {
      hipLaunchKernelGGL(k_md_map, dim3((unsigned)std::min<long long>(blocks_for(plane, 256), 2048)), dim3(256), 0, s,
                         plane, c->lay[L]->rho, rho + L * plane);
      MD_HIP(c, hipGetLastError());
    }
  }
  if (metrics) {
    hipLaunchKernelGGL(k_md_eval_metrics, dim3(1), dim3(64), 0, s, c->wl->red, layer_red(c), en,
                       4.0 / (double)c->dz, metrics);
    MD_HIP(c, hipGetLastError());
  }
  return PLACE3D_OK;
}

int32_t place3d_md2d_gp_init(place3d_md2d_ctx* c, place3d_md2d_state* st, const float* xy0, void* stream) {
  if (!c) { g_md_err = "ctx is NULL"; return PLACE3D_ERR_ARG; }
  if (int rc = check_state(c, st)) return rc;
  if (!xy0 || (reinterpret_cast<uintptr_t>(xy0) & 3)) return md_err(c, PLACE3D_ERR_ARG, "xy0 NULL or misaligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const place3d_md2d_problem& p = c->prob;
  const int n = p.n_nodes;
  const unsigned nb = blocks_for(n, 256);
  const float dx = (float)p.die_x, dy = (float)p.die_y, wb = (float)(p.die_x / p.nx);
  hipLaunchKernelGGL(k_md_clamp_copy, dim3(nb), dim3(256), 0, s, n, p.size, p.kind, dx, dy, xy0, st->u, st->v);
  MD_HIP(c, hipGetLastError());
  if (int rc = md_evaluate(c, st->v, s)) return rc;
  hipLaunchKernelGGL(k_md_l1, dim3(nb), dim3(256), 0, s, n, p.kind, p.layer, c->node_local, c->g_wl, layer_grads(c),
                     c->part, c->part_stride);
  MD_HIP(c, hipGetLastError());
  if (int rc = md_reduce(c, M_L1W, 6, false, s)) return rc;
  hipLaunchKernelGGL(k_md_init_scalars, dim3(1), dim3(64), 0, s, st->scalars, c->red);
  MD_HIP(c, hipGetLastError());
  hipLaunchKernelGGL(k_md_combine, dim3(nb), dim3(256), 0, s, n, p.size, p.kind, p.layer, c->node_local,
                     c->wl->npins, st->v, st->v_prev, c->g_wl, layer_grads(c), st->scalars, 0, st->g_prev, c->part,
                     c->part_stride);
  MD_HIP(c, hipGetLastError());
  if (int rc = md_reduce(c, M_GMAX, 1, true, s)) return rc;
  hipLaunchKernelGGL(k_md_bootstrap, dim3(nb), dim3(256), 0, s, n, p.size, p.kind, dx, dy, wb, st->v, st->g_prev,
                     c->red, st->v_prev);
  MD_HIP(c, hipGetLastError());
  if (int rc = md_evaluate(c, st->v_prev, s)) return rc;
  hipLaunchKernelGGL(k_md_combine, dim3(nb), dim3(256), 0, s, n, p.size, p.kind, p.layer, c->node_local,
                     c->wl->npins, st->v_prev, st->v_prev, c->g_wl, layer_grads(c), st->scalars, 0, st->g_prev,
                     c->part, c->part_stride);
  MD_HIP(c, hipGetLastError());
  return PLACE3D_OK;
}

int32_t place3d_md2d_step(place3d_md2d_ctx* c, place3d_md2d_state* st, void* stream) {
  if (!c) { g_md_err = "ctx is NULL"; return PLACE3D_ERR_ARG; }
  if (int rc = check_state(c, st)) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const place3d_md2d_problem& p = c->prob;
  const int n = p.n_nodes;
  const unsigned nb = blocks_for(n, 256);
  const float dx = (float)p.die_x, dy = (float)p.die_y;
  if (int rc = md_evaluate(c, st->v, s)) return rc;
  hipLaunchKernelGGL(k_md_combine, dim3(nb), dim3(256), 0, s, n, p.size, p.kind, p.layer, c->node_local,
                     c->wl->npins, st->v, st->v_prev, c->g_wl, layer_grads(c), st->scalars, 1, st->g_prev, c->part,
                     c->part_stride);
  MD_HIP(c, hipGetLastError());
  if (int rc = md_reduce(c, M_DV2, 2, false, s)) return rc;
  hipLaunchKernelGGL(k_md_nesterov, dim3(nb), dim3(256), 0, s, n, p.size, p.kind, dx, dy, st->scalars, c->red, st->u,
                     st->v, st->v_prev, st->g_prev);
  MD_HIP(c, hipGetLastError());
  hipLaunchKernelGGL(k_md_step_finish, dim3(1), dim3(64), 0, s, st->scalars, c->red, c->wl->red, layer_red(c),
                     p.lambda_ramp);
  MD_HIP(c, hipGetLastError());
  return PLACE3D_OK;
}

}  // extern "C"
