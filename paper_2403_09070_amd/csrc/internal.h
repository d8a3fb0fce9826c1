// Internal declarations shared by the HIP sources of libplace3d (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/place3d.h"

namespace p3d {

constexpr int kWave = 64;
constexpr int kMaxNz = 16;
constexpr int kNumXcd = 8;              // accelerator dies; workgroups go to them round-robin
constexpr int kWaBlock = 256;           // threads per wirelength block
constexpr int kPinsPerLane = 4;         // net pins a wirelength lane keeps in registers
constexpr int kNumGroups = 7;           // nets by lane group: 1, 2, 4, ..., 64 lanes
constexpr int kNumClasses = kNumGroups + 1;   // the groups, then two-pin nets (one lane each)
constexpr int kChunkEntries = 16384;    // (cell, tile) entries one tile workgroup takes at a time

// Reduction slots (float64, device) inside the workspace.
enum RedSlot {
  R_WA_BI = 0, R_WA_Z, R_HPWL, R_HPWL3D, R_NCUT, R_NORM_X, R_NORM_Y, R_NORM_FDA,
  R_DV2, R_DG2, R_Q_BOT, R_Q_TOP, R_EXCESS_BOT, R_EXCESS_TOP, R_ENERGY,
  R_L1_WL, R_L1_DEN, R_GMAX, R_NONFINITE, R_A_PREV,
  R_COUNT = 32
};


struct ClassTab {       // net schedule in layout order: position i < kNumGroups holds groups of
                        // 2^(kNumGroups-1-i) lanes, the last position the two-pin nets
  int32_t net_begin[kNumClasses + 1];
  int32_t block_begin[kNumClasses + 1];
};

// instance classes for the density path
constexpr uint8_t kClsCell = 0;    // movable cell bucketed by tile
constexpr uint8_t kClsLarge = 1;   // movable macro or oversized cell: swept bin-parallel
constexpr uint8_t kClsFixed = 2;   // fixed: part of the constant map

struct TileGeom {       // map tiles owned by one workgroup each, and the bucketing partition
  int T, lgT, ntx, nty, ntiles;   // T = 2^lgT bins per tile side
  int cpb, nblk;        // cells per bucket block, bucket blocks
};

struct Geom {
  int n, nx, ny, nz;
  float dx, dy, dz, wb, hb, db, inv_wb, inv_hb, inv_db, half_dz, vol_bin;
  double wbd, hbd;      // bin sizes in float64: bin origins b * size are formed in float64, so
                        // that a size that float32 cannot hold does not shift far bins' edges
};

struct DctBases {
  // float32 [N][N] row-major, see spectral.hip for the definition of each matrix
  float *Fx, *Gx, *Hx;      // x: forward (sample, freq), inverse cos (freq, sample), inverse sin*omega
  float *FyT, *Gy, *Hy;     // y: forward^T (freq, sample), inverse cos (sample, freq), inverse sin*omega
  // bfloat16 hi/lo splits, k contiguous: x bases transposed to [N][K], y bases as stored
  uint16_t *Fx_h, *Fx_l, *Gx_h, *Gx_l, *Hx_h, *Hx_l;
  uint16_t *FyT_h, *FyT_l, *Gy_h, *Gy_l, *Hy_h, *Hy_l;
  float* zmat;              // small z matrices, see spectral.hip
  int fold = 0;             // even x and y: folded contractions, spectra in even-first order
  float* inv_w2;            // [Nz][Ny][Nx] 1/|omega|^2 with the (0,0,0) entry 0
};

// hi / lo bfloat16 planes of one split operand
struct HL { uint16_t* h = nullptr; uint16_t* l = nullptr; };

// Split-bfloat16 chain of the folded solve (even x and y, Nz of 2 or 4): every contraction
// operand lives in HBM as hi / lo planes whose rows are k-contiguous, padded with zeros to a
// multiple of 32, so that the contractions stream both operands straight into LDS.  hx, hy are
// the axis halves, rx, ry their padded widths.
struct SplitChain {
  int on = 0;
  int hx = 0, hy = 0, rx = 0, ry = 0;
  HL fx[2];              // forward x, even / odd frequencies: [hx][rx], row = frequency, k = x
  HL fy[2];              // forward y: [hy][ry], row = frequency, k = y
  HL gy, hy_s;           // inverse y (cosine, sine): [hy][2 ry], row = y, k = even then odd frequencies
  HL gx, hx_s;           // inverse x: [hx][2 rx], row = x, k = even then odd frequencies
  HL xs[2];              // x-folded map (sum, difference): [Nz Ny][rx]
  HL ys[2];              // y-folded x spectra (sum, difference): [Nz Nx][ry], row = (z, x frequency)
  HL bb;                 // potential coefficients: [Nx Nz][2 ry], row = x frequency * Nz + z frequency
  HL vg, vh;             // inverse-y results (cosine, sine basis): [Nz Ny][2 rx], row = (z frequency, y)
};

}  // namespace p3d

namespace p3d {
struct ProfRec { int stage; hipEvent_t a, b; int launches; };
}

struct place3d_ctx {
  place3d_problem prob;
  // optional per-stage event profiler
  uint32_t prof_mask = 0;              // stages whose launches are bracketed by events
  std::vector<p3d::ProfRec> prof_pending;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_free;
  double prof_ms[PLACE3D_NSTAGES] = {0};
  long long prof_count[PLACE3D_NSTAGES] = {0};
  // side stream (default priority) on which the wirelength sweep of a step runs concurrently with
  // the density / spectral chain, and the events that fork it from and join it to the caller's stream
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  ~place3d_ctx();
  p3d::Geom g;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::string err;
  // spectral
  p3d::DctBases dct;
  p3d::SplitChain sc;
  float *map_t = nullptr, *map_a = nullptr, *map_vg = nullptr, *map_vh = nullptr;
  float *map_pc = nullptr, *map_ps = nullptr, *map_qc = nullptr;
  // step scratch maps (rho, phi, ex, ey, ez)
  float *rho = nullptr, *phi = nullptr, *ex = nullptr, *ey = nullptr, *ez = nullptr;
  float* fixed_map = nullptr;
  // instances
  uint8_t* cls = nullptr;              // [n] kClsCell / kClsLarge / kClsFixed
  int32_t* large_list = nullptr;       // movable macros and oversized cells
  int32_t n_large = 0;
  float4* large_rec = nullptr;         // [4 * n_large] per-call footprint records of large instances
  float4* lpart = nullptr;             // [2 * lpart_cap] per (large instance, tile) partial sums
  long long lpart_cap = 0;
  int32_t* fixed_list = nullptr;       // fixed instances (their map is built once)
  int32_t n_fixed = 0;
  int32_t n_fillers = 0;               // instances of kind FILLER (bucketed cells)
  // tiles and per-call buckets
  p3d::TileGeom tg = {};
  int32_t* bk_counts = nullptr;        // [nblk][ntiles] counts, then exclusive offsets
  int32_t* bk_totals = nullptr;        // [ntiles]
  int32_t* bk_tile_start = nullptr;    // [ntiles + 1]
  float4* bk_entries = nullptr;        // [2 * 4n] (cell, tile) entries
  // tiles holding more than kChunkEntries entries are split into chunks of that many: chunk 0 is
  // taken by the tile's own workgroup, the extra chunks by the workgroups that loop past the
  // tile count; their density sums meet in a fixed-point accumulator per heavy tile
  int32_t max_extra = 0, max_heavy = 0;   // bounds: 4n / kChunkEntries (+1)
  // chunk plan, one array (the tile kernels take one pointer): [0] extra chunks and [1] heavy
  // tiles of the current buckets, then per tile its accumulator slot (-1: one chunk), per extra
  // chunk its tile and its index within the tile, and per slot the chunks finished (zero
  // between calls)
  int32_t* bk_plan = nullptr;          // [2 + ntiles + 2 max_extra + max_heavy]
  unsigned long long* heavy_acc = nullptr;   // [max_heavy][2][T * T * nz] zero between calls
  int32_t* cell_entry = nullptr;       // [n] packed tile range of each bucketed cell, -1 if none
  float4* entry_out = nullptr;         // [4][n] per-(cell, tile) gather / adjoint results, cell-major
  // two-stage reductions: part[slot * part_stride + block]
  double* part = nullptr;
  int32_t part_stride = 0;
  float* npins = nullptr;              // |E_i| as float [n]
  // wirelength schedule (nets ordered by lane-group class)
  int32_t* s_net_start = nullptr;      // [n_sched_nets + 1] slot ranges
  int32_t* s_pin_node = nullptr;       // [n_pins] owner per slot
  float4* s_off = nullptr;             // [n_pins] (ox_bot, oy_bot, ox_top, oy_top) per slot
  float4* pin_out = nullptr;           // [n_pins] (gx, gy, gz_wa, fda) in node order
  int32_t* node_slot_start = nullptr;  // [n+1] node -> range of pin_out
  int32_t* slot_pos = nullptr;         // [n_pins] slot -> position in node order
  int32_t* shared_nets = nullptr;      // [n_shared_nets] schedule nets holding an instance on
  int32_t n_shared_nets = 0;           // more than one pin (their FDA is redone per instance)
  int32_t* heavy_list = nullptr;       // instances with more than 32 pins (summed per wavefront)
  int32_t n_heavy = 0;
  p3d::ClassTab classes = {};
  int field_xfold = 0;                 // the last spectral_field left its field maps x-folded
  float cell_scale = 0.f;              // factor of the per-(cell, tile) gradient shares of the last gather
  int32_t* wa_block_order = nullptr;   // [n_wa_blocks] schedule blocks in order of their first net
  int32_t n_wa_blocks = 0;
  // per-instance scratch
  float4* xyzp = nullptr;              // [n] (x, y, z, 0) per instance, the net kernel's gather source
  float* wl_gzwa = nullptr;            // [n] alpha d p^(z)/dz per instance
  float* wl_fda = nullptr;             // [n] FDA z-gradient before normalisation
  float* gw = nullptr;                 // [3][n] wirelength gradient inside the GP step
  float* den_grad = nullptr;           // [3][n] density-penalty gradient inside the GP step
  double* red = nullptr;               // [R_COUNT] reductions
  double* red2 = nullptr;              // [R_COUNT] second set (init)
};

namespace p3d {

inline int set_err(place3d_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}
int hip_fail(place3d_ctx* c, hipError_t e, const char* where);

#define P3D_HIP(ctx, call)                                                     \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) return p3d::hip_fail((ctx), e_, #call);              \
  } while (0)

#define P3D_LAUNCH(ctx, what)                                                  \
  do {                                                                         \
    hipError_t e_ = hipGetLastError();                                         \
    if (e_ != hipSuccess) return p3d::hip_fail((ctx), e_, what);               \
  } while (0)

// large instances go through the density tiles when their per-tile partials fit the workspace
inline bool large_in_tiles(const place3d_ctx* c) {
  return (long long)c->n_large * c->tg.ntiles <= c->lpart_cap;
}

inline unsigned blocks_for(long long n, int threads) {
  long long b = (n + threads - 1) / threads;
  return (unsigned)(b < 1 ? 1 : b);
}

// Workgroup b of a launch of nb runs on die b % kNumXcd.  This bijection hands die x the
// contiguous work range [x q + min(x, r), ...) (q = nb / kNumXcd, r = nb % kNumXcd), so that
// neighbouring work items, which read neighbouring data, share one die's L2.
__host__ __device__ inline int xcd_swizzle(int b, int nb) {
  const int q = nb / kNumXcd, r = nb % kNumXcd, x = b % kNumXcd, i = b / kNumXcd;
  return x * q + (x < r ? x : r) + i;
}

// Profiler brackets (no-ops unless profiling is on).  prof_end records on the same stream.
int prof_begin(place3d_ctx* c, int stage, hipStream_t s);
int prof_end(place3d_ctx* c, hipStream_t s, int launches);

// One event pair per scope; `launches` is how many kernel launches the scope holds (a scope
// around several consecutive launches of one stage perturbs the stream less than one per launch)
struct ProfScope {
  place3d_ctx* c;
  hipStream_t s;
  bool on;
  int launches = 1;
  ProfScope(place3d_ctx* c_, int stage, hipStream_t s_) : c(c_), s(s_), on((c_->prof_mask >> stage) & 1u) {
    if (on) prof_begin(c, stage, s);
  }
  ~ProfScope() { if (on) prof_end(c, s, launches); }
};

// ---- launchers implemented in the .hip sources (all enqueue only) ----
int launch_zero_f64(place3d_ctx* c, double* p, int n, hipStream_t s);
int launch_fill_f32(place3d_ctx* c, float* p, long long n, float v, hipStream_t s);

int build_dct_bases(place3d_ctx* c, hipStream_t s);
// x_folded_out: with folded contractions, leave ex / ey / ez as even and odd x halves (columns
// [0, nx/2) and [nx/2, nx)) for a consumer that unfolds them on load; ctx->field_xfold says
// whether that happened
int spectral_field(place3d_ctx* c, const float* rho, float* phi, float* ex, float* ey, float* ez,
                   double* energy, hipStream_t s, bool x_folded_out = false);
// the split chain's bases (at creation) and its contractions; outputs in natural x order
int build_split_chain(place3d_ctx* c, hipStream_t s);
int field_split(place3d_ctx* c, const float* rho, float* phi, float* ex, float* ey, float* ez, hipStream_t s);

// out[0..nq) = sums (max if is_max) of partial slots slot0.. over nparts blocks, fixed order
int reduce_final(place3d_ctx* c, int slot0, int nq, int nparts, bool is_max, double* out, hipStream_t s);
// the same over the partials in `part` (stride per slot) instead of the workspace's
int reduce_final_in(place3d_ctx* c, const double* part, int stride, int slot0, int nq, int nparts, bool is_max,
                    double* out, hipStream_t s);
// two sum reductions in one launch: slots slot0.. (nq0 of them, nparts0 partials) into out0[] and
// slots slot1.. (nq1, nparts1) into out1[]
int reduce_final2(place3d_ctx* c, int slot0, int nq0, int nparts0, double* out0, int slot1, int nq1, int nparts1,
                  double* out1, hipStream_t s);

int build_fixed_map(place3d_ctx* c, hipStream_t s);
// part 0: the whole bucketing; 1: only the count pass (which also packs xyzp); 2: the rest
int bucket_cells(place3d_ctx* c, const float* xyz, hipStream_t s, int part = 0);
// reduce: finish the overflow reduction here (else the caller reduces the R_EXCESS slots later)
int density_tiles(place3d_ctx* c, const float* xyz, float* rho, double* red, hipStream_t s, bool reduce = true);
int gather_bucketed(place3d_ctx* c, const float* xyz, const float* ex, const float* ey, const float* ez, float scale,
                    float* grad, int accumulate, hipStream_t s, bool cells = true,
                    bool xfold = false);
// dscale: a device float64 factor multiplying scale (NULL: 1)
int adjoint_bucketed(place3d_ctx* c, const float* xyz, const float* gmap, float scale, float* grad, int accumulate,
                     hipStream_t s, bool cells = true, const double* dscale = nullptr);
int density_forward(place3d_ctx* c, const float* xyz, float* rho, hipStream_t s);
int density_field_gather(place3d_ctx* c, const float* xyz, const float* ex, const float* ey,
                         const float* ez, float scale, float* grad, int accumulate, hipStream_t s);
int density_adjoint(place3d_ctx* c, const float* xyz, const float* gmap, float scale, float* grad,
                    int accumulate, hipStream_t s, const double* dscale = nullptr);

// packed: c->xyzp already holds xyz (the bucket pass of the same positions wrote it); dscale: a
// device float64 factor of the gradient (NULL: 1); with_fda: the z-gradient carries the normalised
// FDA term, else only the derivative of alpha p^(z)
int wirelength_eval(place3d_ctx* c, const float* xyz, float* grad, int accumulate, double* red,
                    double* metrics, hipStream_t s, bool packed = false, const double* dscale = nullptr,
                    bool with_fda = true);
// the model's net totals only (no gradient, nothing per pin) into metrics[PLACE3D_NMETRICS]; the
// packed positions and the per-workgroup partials go to xyzp / part (stride per slot) when given,
// else to the workspace's
int wirelength_value(place3d_ctx* c, const float* xyz, double* metrics, hipStream_t s, float4* xyzp = nullptr,
                     double* part = nullptr, int stride = 0);
// the same with the scratch in the library's static device array (place3d_wl_value_static)
constexpr int kStaticMaxInst = 1 << 21;      // instances whose positions the static scratch holds
constexpr int kStaticMaxBlocks = 1 << 18;    // wirelength workgroups whose partials it holds
int wirelength_value_static(place3d_ctx* c, const float* xyz, double* metrics, hipStream_t s);
// device address of the static scratch on the current device, looked up once per device
int static_scratch_setup(place3d_ctx* c, void** out);

}  // namespace p3d
