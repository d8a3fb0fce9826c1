// Context creation, workspace layout, argument checks and the public C entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using p3d::set_err;

namespace {

thread_local std::string g_create_err;

struct Carver {
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

int check_grid_fits(const place3d_problem& p, std::string& why);

int check_problem(const place3d_problem* p, std::string& why) {
  if (!p) { why = "problem is NULL"; return PLACE3D_ERR_ARG; }
  if (p->n_inst < 1 || p->n_pins < 0 || p->n_nets < 0) { why = "n_inst < 1 or negative pin/net count"; return PLACE3D_ERR_SIZE; }
  // the kernels index arrays of four rows per instance or pin ([4][n] sizes, offsets and
  // per-(cell, tile) shares) with 32-bit integers
  constexpr int32_t kMaxCount = 1 << 28;
  if (p->n_inst > kMaxCount || p->n_pins > kMaxCount || p->n_nets > kMaxCount) {
    why = "n_inst, n_pins and n_nets must not exceed 2^28";
    return PLACE3D_ERR_SIZE;
  }
  if (p->nx < 2 || p->ny < 2 || p->nx > 8192 || p->ny > 8192) { why = "nx, ny must lie in [2, 8192]"; return PLACE3D_ERR_SIZE; }
  if (p->nz < 2 || p->nz > p3d::kMaxNz || (p->nz & 1)) { why = "nz must be even and in [2, 16]"; return PLACE3D_ERR_SIZE; }
  if (!(p->die_x > 0) || !(p->die_y > 0) || !std::isfinite(p->die_x) || !std::isfinite(p->die_y)) { why = "die extent must be positive"; return PLACE3D_ERR_ARG; }
  if (!(p->gamma > 0) || !std::isfinite(p->gamma)) { why = "gamma must be positive"; return PLACE3D_ERR_ARG; }
  if (!(p->alpha >= 0) || !std::isfinite(p->alpha)) { why = "alpha must be >= 0"; return PLACE3D_ERR_ARG; }
  if (!std::isfinite(p->target_density) || !std::isfinite(p->lambda_ramp)) { why = "non-finite target density or ramp"; return PLACE3D_ERR_ARG; }
  if (p->precision != PLACE3D_FP32 && p->precision != PLACE3D_BF16X3) { why = "bad precision"; return PLACE3D_ERR_ARG; }
  if (p->dgrad != PLACE3D_DGRAD_FIELD && p->dgrad != PLACE3D_DGRAD_ADJOINT) { why = "bad dgrad"; return PLACE3D_ERR_ARG; }
  if (p->precond < PLACE3D_PRECOND_MIXED || p->precond > PLACE3D_PRECOND_EPLACE3D) { why = "bad precond"; return PLACE3D_ERR_ARG; }
  if (p->options & ~(PLACE3D_OPT_MACRO_INSTANCE | PLACE3D_OPT_FDA_VANILLA)) { why = "unknown option bits"; return PLACE3D_ERR_ARG; }
  if (!p->size || !p->kind || !p->net_start || !p->fixed_xyz) { why = "null device array in problem"; return PLACE3D_ERR_ARG; }
  if (p->n_pins > 0 && (!p->pin2node || !p->pin_off)) { why = "null pin arrays"; return PLACE3D_ERR_ARG; }
  if ((reinterpret_cast<uintptr_t>(p->size) | reinterpret_cast<uintptr_t>(p->pin_off) |
       reinterpret_cast<uintptr_t>(p->fixed_xyz) | reinterpret_cast<uintptr_t>(p->net_start) |
       reinterpret_cast<uintptr_t>(p->pin2node)) & 3) { why = "misaligned device array"; return PLACE3D_ERR_ARG; }
  return check_grid_fits(*p, why);
}

p3d::TileGeom tile_geom(const place3d_problem& p);

// the bucketing passes keep one int per density tile in LDS (a workgroup may use up to 160 KiB on
// gfx950; 1 KiB is left for the passes' other LDS)
constexpr size_t kBucketLdsBudget = 159 * 1024;

int check_grid_fits(const place3d_problem& p, std::string& why) {
  const p3d::TileGeom t = tile_geom(p);
  if (sizeof(int32_t) * (size_t)t.ntiles > kBucketLdsBudget) {
    why = "grid too large: " + std::to_string(t.ntiles) + " density tiles of " + std::to_string(t.T) + "x" +
          std::to_string(t.T) + " bins exceed the bucketing pass's LDS histogram";
    return PLACE3D_ERR_SIZE;
  }
  return PLACE3D_OK;
}

p3d::TileGeom tile_geom(const place3d_problem& p) {
  p3d::TileGeom t;
  int T = 32;
  while (T > 4 && (3 * T * T * p.nz * 4 > 60 * 1024 || T > p.nx || T > p.ny)) T >>= 1;
  t.T = T;
  t.lgT = 0;
  while ((1 << t.lgT) < T) ++t.lgT;
  t.ntx = (p.nx + T - 1) / T;
  t.nty = (p.ny + T - 1) / T;
  t.ntiles = t.ntx * t.nty;
  t.cpb = 2048;
  t.nblk = (p.n_inst + t.cpb - 1) / t.cpb;
  return t;
}

int parts_bound(const place3d_problem& p, const p3d::TileGeom& t) {
  int b = std::max(p.n_nets / 4 + 16, p.n_inst / 256 + p.n_pins / 128 + 8);
  b = std::max(b, t.ntiles);
  b = std::max(b, t.nblk);
  return std::max(b, 1024);
}

size_t layout(place3d_ctx* c, const place3d_problem& p, char* base) {
  Carver w{base};
  c->tg = tile_geom(p);
  c->part_stride = parts_bound(p, c->tg);
  const size_t nx = p.nx, ny = p.ny, nz = p.nz, n = p.n_inst, P = p.n_pins, m = p.n_nets;
  const size_t map = nx * ny * nz;
  auto& d = c->dct;
  d.Fx = w.take<float>(nx * nx); d.Gx = w.take<float>(nx * nx); d.Hx = w.take<float>(nx * nx);
  d.FyT = w.take<float>(ny * ny); d.Gy = w.take<float>(ny * ny); d.Hy = w.take<float>(ny * ny);
  for (uint16_t** q : {&d.Fx_h, &d.Fx_l, &d.Gx_h, &d.Gx_l, &d.Hx_h, &d.Hx_l}) *q = w.take<uint16_t>(nx * nx);
  for (uint16_t** q : {&d.FyT_h, &d.FyT_l, &d.Gy_h, &d.Gy_l, &d.Hy_h, &d.Hy_l}) *q = w.take<uint16_t>(ny * ny);
  d.zmat = w.take<float>(4 * p3d::kMaxNz * p3d::kMaxNz);
  {
    auto& q = c->sc;
    q = p3d::SplitChain{};
    q.on = p.precision == PLACE3D_BF16X3 && nx % 2 == 0 && ny % 2 == 0 && (nz == 2 || nz == 4);
    if (q.on) {
      const size_t hx = nx / 2, hy = ny / 2, rx = (hx + 31) / 32 * 32, ry = (hy + 31) / 32 * 32;
      q.hx = (int)hx; q.hy = (int)hy; q.rx = (int)rx; q.ry = (int)ry;
      auto hl = [&](p3d::HL& x, size_t count) { x.h = w.take<uint16_t>(count); x.l = w.take<uint16_t>(count); };
      for (int i = 0; i < 2; ++i) { hl(q.fx[i], hx * rx); hl(q.fy[i], hy * ry); }
      hl(q.gy, hy * 2 * ry); hl(q.hy_s, hy * 2 * ry); hl(q.gx, hx * 2 * rx); hl(q.hx_s, hx * 2 * rx);
      for (int i = 0; i < 2; ++i) { hl(q.xs[i], nz * ny * rx); hl(q.ys[i], nz * nx * ry); }
      hl(q.bb, nz * nx * 2 * ry);
      hl(q.vg, nz * ny * 2 * rx); hl(q.vh, nz * ny * 2 * rx);
    }
  }
  d.inv_w2 = w.take<float>(map);
  c->map_t = w.take<float>(map); c->map_a = w.take<float>(map);
  c->map_vg = w.take<float>(map); c->map_vh = w.take<float>(map);
  c->map_pc = w.take<float>(map); c->map_ps = w.take<float>(map); c->map_qc = w.take<float>(map);
  c->rho = w.take<float>(map); c->phi = w.take<float>(map);
  c->ex = w.take<float>(map); c->ey = w.take<float>(map); c->ez = w.take<float>(map);
  c->fixed_map = w.take<float>(map);
  c->cls = w.take<uint8_t>(n);
  c->large_list = w.take<int32_t>(n);
  c->large_rec = w.take<float4>(4 * n);
  c->lpart_cap = std::min<long long>((long long)n * c->tg.ntiles, 1ll << 22);
  c->lpart = w.take<float4>(2 * (size_t)c->lpart_cap);
  c->fixed_list = w.take<int32_t>(n);
  c->bk_counts = w.take<int32_t>((size_t)c->tg.ntiles * c->tg.nblk);
  c->bk_totals = w.take<int32_t>(c->tg.ntiles);
  c->bk_tile_start = w.take<int32_t>(c->tg.ntiles + 1);
  c->bk_entries = w.take<float4>(8 * n);
  c->max_extra = (int32_t)(4 * n / p3d::kChunkEntries + 1);
  c->max_heavy = std::min(c->max_extra, c->tg.ntiles);
  c->bk_plan = w.take<int32_t>(2 + (size_t)c->tg.ntiles + 2 * (size_t)c->max_extra + c->max_heavy);
  c->heavy_acc = w.take<unsigned long long>((size_t)c->max_heavy * 2 * c->tg.T * c->tg.T * p.nz);
  c->cell_entry = w.take<int32_t>(n);
  c->entry_out = w.take<float4>(4 * n);
  c->part = w.take<double>((size_t)p3d::R_COUNT * c->part_stride);
  c->npins = w.take<float>(n);
  c->s_net_start = w.take<int32_t>(m + 1);
  c->wa_block_order = w.take<int32_t>(m / 256 + P / 512 + 16);
  c->s_pin_node = w.take<int32_t>(P + 1);
  c->s_off = w.take<float4>(P + 1);
  c->pin_out = w.take<float4>(P + 1);
  c->node_slot_start = w.take<int32_t>(n + 1);
  c->slot_pos = w.take<int32_t>(P + 1);
  c->heavy_list = w.take<int32_t>(n);
  c->shared_nets = w.take<int32_t>(m);
  c->wl_gzwa = w.take<float>(n);
  c->xyzp = w.take<float4>(n);
  c->gw = w.take<float>(3 * n);
  c->wl_fda = w.take<float>(n);
  c->den_grad = w.take<float>(3 * n);
  c->red = w.take<double>(p3d::R_COUNT);
  c->red2 = w.take<double>(p3d::R_COUNT);
  return (w.off + 255) & ~size_t(255);
}

void fill_geom(place3d_ctx* c) {
  const place3d_problem& p = c->prob;
  auto& g = c->g;
  g.n = p.n_inst; g.nx = p.nx; g.ny = p.ny; g.nz = p.nz;
  const double wb = p.die_x / p.nx, hb = p.die_y / p.ny, db = 0.5 * (wb + hb);
  const double dz = p.nz * db;
  g.dx = (float)p.die_x; g.dy = (float)p.die_y; g.dz = (float)dz;
  g.wb = (float)wb; g.hb = (float)hb; g.db = (float)db;
  g.wbd = wb; g.hbd = hb;
  g.inv_wb = (float)(1.0 / wb); g.inv_hb = (float)(1.0 / hb); g.inv_db = (float)(1.0 / db);
  g.half_dz = (float)(0.5 * dz);
  g.vol_bin = (float)(wb * hb * db);
}

int build_schedule(place3d_ctx* c, hipStream_t s) {
  const place3d_problem& p = c->prob;
  const int n = p.n_inst, P = p.n_pins, m = p.n_nets;
  std::vector<int32_t> ns(m + 1), p2n(P);
  std::vector<float> off(4 * (size_t)P);
  std::vector<uint8_t> kind(n);
  std::vector<float> size(4 * (size_t)n);
  P3D_HIP(c, hipMemcpyAsync(ns.data(), p.net_start, sizeof(int32_t) * (m + 1), hipMemcpyDeviceToHost, s));
  if (P > 0) {
    P3D_HIP(c, hipMemcpyAsync(p2n.data(), p.pin2node, sizeof(int32_t) * P, hipMemcpyDeviceToHost, s));
    P3D_HIP(c, hipMemcpyAsync(off.data(), p.pin_off, sizeof(float) * 4 * (size_t)P, hipMemcpyDeviceToHost, s));
  }
  P3D_HIP(c, hipMemcpyAsync(kind.data(), p.kind, n, hipMemcpyDeviceToHost, s));
  P3D_HIP(c, hipMemcpyAsync(size.data(), p.size, sizeof(float) * 4 * (size_t)n, hipMemcpyDeviceToHost, s));
  P3D_HIP(c, hipStreamSynchronize(s));

  if (ns[0] != 0 || ns[m] != P) return set_err(c, PLACE3D_ERR_NETLIST, "net_start[0] must be 0 and net_start[n_nets] == n_pins");
  for (int e = 0; e < m; ++e)
    if (ns[e + 1] < ns[e]) return set_err(c, PLACE3D_ERR_NETLIST, "net_start is not monotone at net " + std::to_string(e));
  for (int q = 0; q < P; ++q)
    if (p2n[q] < 0 || p2n[q] >= n) return set_err(c, PLACE3D_ERR_NETLIST, "pin2node out of range at pin " + std::to_string(q));
  // nets holding an instance on more than one pin (allowed; their FDA is redone per instance)
  std::vector<char> shared(m, 0);
  {
    std::vector<int32_t> tmp;
    for (int e = 0; e < m; ++e) {
      tmp.assign(p2n.begin() + ns[e], p2n.begin() + ns[e + 1]);
      std::sort(tmp.begin(), tmp.end());
      shared[e] = std::adjacent_find(tmp.begin(), tmp.end()) != tmp.end();
    }
  }

  // nets by lane-group class: a net of degree d takes G = 2^c lanes, the smallest with
  // d <= kPinsPerLane * G (64 lanes for larger nets, which then loop), except that two-pin nets
  // form a class of their own (one lane each, in closed form), so that no wavefront mixes them
  // with the general single-lane nets.  Classes are laid out from the widest groups down, then
  // the two-pin nets, nets in netlist order within a class; empty nets are dropped.  The
  // workgroups of all classes then run in the order of their first net (block_order), so the
  // whole sweep walks the netlist once and the owners it gathers stay cache-resident.
  auto net_pos = [](int d) {          // layout position of a net of degree d
    if (d == 2) return p3d::kNumClasses - 1;
    int cl = 0;
    while (p3d::kPinsPerLane * (1 << cl) < d && cl < p3d::kNumGroups - 1) ++cl;
    return p3d::kNumGroups - 1 - cl;
  };
  auto pos_lanes_log2 = [](int i) { return i < p3d::kNumGroups ? p3d::kNumGroups - 1 - i : 0; };
  std::vector<int32_t> order;
  order.reserve(m);
  for (int e = 0; e < m; ++e)
    if (ns[e + 1] > ns[e]) order.push_back(e);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return net_pos(ns[a + 1] - ns[a]) < net_pos(ns[b + 1] - ns[b]);
  });
  {
    int nb = 0;
    size_t k = 0;
    for (int i = 0; i < p3d::kNumClasses; ++i) {
      c->classes.net_begin[i] = (int32_t)k;
      c->classes.block_begin[i] = nb;
      size_t k1 = k;
      while (k1 < order.size() && net_pos(ns[order[k1] + 1] - ns[order[k1]]) == i) ++k1;
      const int per_block = p3d::kWaBlock >> pos_lanes_log2(i);
      nb += (int)((k1 - k + per_block - 1) / per_block);
      k = k1;
    }
    c->classes.net_begin[p3d::kNumClasses] = (int32_t)order.size();
    c->classes.block_begin[p3d::kNumClasses] = nb;
    c->n_wa_blocks = nb;
  }
  if ((size_t)c->n_wa_blocks > (size_t)m / 256 + (size_t)P / 512 + 16)
    return set_err(c, PLACE3D_ERR_NETLIST, "net schedule exceeds its workgroup bound");
  std::vector<int32_t> block_order(c->n_wa_blocks);
  {
    std::vector<int32_t> first(c->n_wa_blocks);
    for (int i = 0; i < p3d::kNumClasses; ++i) {
      const int per_block = p3d::kWaBlock >> pos_lanes_log2(i);
      for (int b = c->classes.block_begin[i]; b < c->classes.block_begin[i + 1]; ++b)
        first[b] = order[c->classes.net_begin[i] + (size_t)(b - c->classes.block_begin[i]) * per_block];
    }
    for (int b = 0; b < c->n_wa_blocks; ++b) block_order[b] = b;
    std::stable_sort(block_order.begin(), block_order.end(), [&](int32_t a, int32_t b) { return first[a] < first[b]; });
  }

  const int ms = (int)order.size();
  std::vector<int32_t> sns(ms + 1), spn(P > 0 ? P : 1), slot_of_pin(P > 0 ? P : 1);
  std::vector<float> soff(4 * (size_t)(P > 0 ? P : 1));
  int slot = 0;
  for (int k = 0; k < ms; ++k) {
    const int e = order[k];
    sns[k] = slot;
    for (int q = ns[e]; q < ns[e + 1]; ++q, ++slot) {
      spn[slot] = p2n[q];
      slot_of_pin[q] = slot;
      soff[4 * (size_t)slot + 0] = off[q];
      soff[4 * (size_t)slot + 1] = off[(size_t)P + q];
      soff[4 * (size_t)slot + 2] = off[2 * (size_t)P + q];
      soff[4 * (size_t)slot + 3] = off[3 * (size_t)P + q];
    }
  }
  sns[ms] = slot;
  {
    std::vector<int32_t> sh;
    for (int k = 0; k < ms; ++k)
      if (shared[order[k]]) sh.push_back(k);
    c->n_shared_nets = (int32_t)sh.size();
    if (!sh.empty())
      P3D_HIP(c, hipMemcpyAsync(c->shared_nets, sh.data(), sizeof(int32_t) * sh.size(), hipMemcpyHostToDevice, s));
  }

  // node -> slot CSR, slots ascending per node (fixed summation order)
  std::vector<int32_t> nss(n + 1, 0), nsl(P > 0 ? P : 1);
  for (int q = 0; q < P; ++q) nss[p2n[q] + 1]++;
  for (int i = 0; i < n; ++i) nss[i + 1] += nss[i];
  {
    // position of every slot in node order (slots ascending per node): the net kernel writes a
    // pin's results there, so each node's shares are contiguous for the node-side sum
    std::vector<int32_t> fill(nss.begin(), nss.end() - 1);
    for (int sl = 0; sl < slot; ++sl) nsl[sl] = fill[spn[sl]]++;
  }
  std::vector<float> npins(n);
  std::vector<int32_t> heavy;
  for (int i = 0; i < n; ++i) {
    npins[i] = (float)(nss[i + 1] - nss[i]);
    if (nss[i + 1] - nss[i] > 32) heavy.push_back(i);
  }
  c->n_heavy = (int32_t)heavy.size();
  if (!heavy.empty())
    P3D_HIP(c, hipMemcpyAsync(c->heavy_list, heavy.data(), sizeof(int32_t) * heavy.size(), hipMemcpyHostToDevice, s));

  // density classes: bucketed cells must span at most two tiles per axis on either die
  std::vector<int32_t> large, fixed;
  std::vector<uint8_t> cls(n);
  int32_t n_fill = 0;
  {
    const double wb = p.die_x / p.nx, hb = p.die_y / p.ny;
    const double wlim = (c->tg.T - 1) * wb, hlim = (c->tg.T - 1) * hb;
    for (int i = 0; i < n; ++i) {
      const bool filler = (kind[i] & PLACE3D_KIND_FILLER) != 0;
      if (filler && (kind[i] & (PLACE3D_KIND_MACRO | PLACE3D_KIND_FIXED)))
        return set_err(c, PLACE3D_ERR_ARG, "filler " + std::to_string(i) + " is also a macro or fixed");
      if (filler && nss[i + 1] > nss[i])
        return set_err(c, PLACE3D_ERR_NETLIST, "filler " + std::to_string(i) + " has a pin");
      n_fill += filler;
      if (kind[i] & PLACE3D_KIND_FIXED) { cls[i] = p3d::kClsFixed; fixed.push_back(i); continue; }
      const double w = std::max(size[i], size[2 * (size_t)n + i]);
      const double h = std::max(size[(size_t)n + i], size[3 * (size_t)n + i]);
      if ((kind[i] & PLACE3D_KIND_MACRO) || w > wlim || h > hlim) {
        if (filler) return set_err(c, PLACE3D_ERR_ARG, "filler " + std::to_string(i) + " is wider than a density tile");
        cls[i] = p3d::kClsLarge;
        large.push_back(i);
      } else {
        cls[i] = p3d::kClsCell;
      }
    }
  }
  c->n_fillers = n_fill;
  if (n_fill > 0 && (p.options & PLACE3D_OPT_MACRO_INSTANCE))
    return set_err(c, PLACE3D_ERR_UNSUPPORTED, "the instance-parallel macro scatter cannot leave fillers out of the overflow");
  c->n_large = (int32_t)large.size();
  c->n_fixed = (int32_t)fixed.size();
  P3D_HIP(c, hipMemcpyAsync(c->cls, cls.data(), n, hipMemcpyHostToDevice, s));

  P3D_HIP(c, hipMemcpyAsync(c->s_net_start, sns.data(), sizeof(int32_t) * (ms + 1), hipMemcpyHostToDevice, s));
  if (P > 0) {
    P3D_HIP(c, hipMemcpyAsync(c->s_pin_node, spn.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice, s));
    P3D_HIP(c, hipMemcpyAsync(c->s_off, soff.data(), sizeof(float) * 4 * (size_t)P, hipMemcpyHostToDevice, s));
    P3D_HIP(c, hipMemcpyAsync(c->slot_pos, nsl.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice, s));
  }
  P3D_HIP(c, hipMemcpyAsync(c->node_slot_start, nss.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, s));
  if (c->n_wa_blocks > 0)
    P3D_HIP(c, hipMemcpyAsync(c->wa_block_order, block_order.data(), sizeof(int32_t) * c->n_wa_blocks,
                              hipMemcpyHostToDevice, s));
  P3D_HIP(c, hipMemcpyAsync(c->npins, npins.data(), sizeof(float) * n, hipMemcpyHostToDevice, s));
  if (!large.empty())
    P3D_HIP(c, hipMemcpyAsync(c->large_list, large.data(), sizeof(int32_t) * large.size(), hipMemcpyHostToDevice, s));
  if (!fixed.empty())
    P3D_HIP(c, hipMemcpyAsync(c->fixed_list, fixed.data(), sizeof(int32_t) * fixed.size(), hipMemcpyHostToDevice, s));
  P3D_HIP(c, hipStreamSynchronize(s));   // host vectors die at return
  return PLACE3D_OK;
}

}  // namespace

place3d_ctx::~place3d_ctx() {
  if (side) hipStreamDestroy(side);
  if (ev_fork) hipEventDestroy(ev_fork);
  if (ev_join) hipEventDestroy(ev_join);
  for (auto& r : prof_pending) { hipEventDestroy(r.a); hipEventDestroy(r.b); }
  for (auto& e : prof_free) { hipEventDestroy(e.first); hipEventDestroy(e.second); }
}

namespace p3d {
int prof_begin(place3d_ctx* c, int stage, hipStream_t s) {
  std::pair<hipEvent_t, hipEvent_t> ev;
  if (!c->prof_free.empty()) {
    ev = c->prof_free.back();
    c->prof_free.pop_back();
  } else {
    if (hipEventCreate(&ev.first) != hipSuccess) return PLACE3D_ERR_HIP;
    if (hipEventCreate(&ev.second) != hipSuccess) { hipEventDestroy(ev.first); return PLACE3D_ERR_HIP; }
  }
  c->prof_pending.push_back({stage, ev.first, ev.second, 1});
  return hipEventRecord(ev.first, s) == hipSuccess ? PLACE3D_OK : PLACE3D_ERR_HIP;
}
int prof_end(place3d_ctx* c, hipStream_t s, int launches) {
  if (c->prof_pending.empty()) return PLACE3D_OK;
  c->prof_pending.back().launches = launches;
  return hipEventRecord(c->prof_pending.back().b, s) == hipSuccess ? PLACE3D_OK : PLACE3D_ERR_HIP;
}
int hip_fail(place3d_ctx* c, hipError_t e, const char* where) {
  std::string msg = std::string("HIP error ") + std::to_string((int)e) + " (" + hipGetErrorString(e) + ") in " + where;
  if (c) c->err = msg; else g_create_err = msg;
  return PLACE3D_ERR_HIP;
}
}  // namespace p3d

extern "C" {

int32_t place3d_abi_version(void) { return PLACE3D_ABI_VERSION; }

const char* place3d_last_error(const place3d_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int32_t place3d_workspace_size(const place3d_problem* prob, size_t* bytes) {
  std::string why;
  int rc = check_problem(prob, why);
  if (rc != PLACE3D_OK) { g_create_err = why; return rc; }
  if (!bytes) { g_create_err = "bytes is NULL"; return PLACE3D_ERR_ARG; }
  place3d_ctx tmp;
  *bytes = layout(&tmp, *prob, nullptr);
  return PLACE3D_OK;
}

int32_t place3d_create(const place3d_problem* prob, void* d_workspace, size_t bytes, void* stream,
                       place3d_ctx** out) {
  std::string why;
  int rc = check_problem(prob, why);
  if (rc != PLACE3D_OK) { g_create_err = why; return rc; }
  if (!out) { g_create_err = "out is NULL"; return PLACE3D_ERR_ARG; }
  *out = nullptr;
  if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255)) { g_create_err = "workspace NULL or not 256-byte aligned"; return PLACE3D_ERR_ARG; }
  place3d_ctx* c = new (std::nothrow) place3d_ctx();
  if (!c) { g_create_err = "out of host memory"; return PLACE3D_ERR_ARG; }
  c->prob = *prob;
  size_t need = layout(c, *prob, reinterpret_cast<char*>(d_workspace));
  if (bytes < need) {
    g_create_err = "workspace too small: need " + std::to_string(need) + " bytes";
    delete c;
    return PLACE3D_ERR_SIZE;
  }
  c->ws = reinterpret_cast<char*>(d_workspace);
  c->ws_bytes = bytes;
  fill_geom(c);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  {
    hipError_t e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
    if (e != hipSuccess) {
      g_create_err = std::string("side stream / events: ") + hipGetErrorString(e);
      delete c;
      return PLACE3D_ERR_HIP;
    }
  }
  rc = build_schedule(c, s);
  // the device address of the static scratch of place3d_wl_value_static, once per device
  if (rc == PLACE3D_OK) rc = p3d::static_scratch_setup(c, nullptr);
  if (rc == PLACE3D_OK) {
    hipError_t e = hipMemsetAsync(c->red, 0, sizeof(double) * p3d::R_COUNT, s);
    // the heavy tiles' accumulators and chunk counters start at zero; every call leaves them so
    const size_t acc = sizeof(unsigned long long) * (size_t)c->max_heavy * 2 * c->tg.T * c->tg.T * prob->nz;
    if (e == hipSuccess) e = hipMemsetAsync(c->heavy_acc, 0, acc, s);
    int32_t* done = c->bk_plan + 2 + c->tg.ntiles + 2 * (size_t)c->max_extra;
    if (e == hipSuccess) e = hipMemsetAsync(done, 0, sizeof(int32_t) * c->max_heavy, s);
    if (e != hipSuccess) rc = p3d::hip_fail(c, e, "hipMemsetAsync(create)");
  }
  if (rc == PLACE3D_OK) rc = p3d::build_dct_bases(c, s);
  if (rc == PLACE3D_OK) rc = p3d::build_fixed_map(c, s);
  if (rc == PLACE3D_OK) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = p3d::hip_fail(c, e, "hipStreamSynchronize(create)");
  }
  if (rc != PLACE3D_OK) {
    g_create_err = c->err;
    delete c;
    return rc;
  }
  *out = c;
  return PLACE3D_OK;
}

int32_t place3d_destroy(place3d_ctx* ctx) {
  delete ctx;
  return PLACE3D_OK;
}

int32_t place3d_profile_enable(place3d_ctx* ctx, int32_t on) {
  if (!ctx) return PLACE3D_ERR_ARG;
  ctx->prof_mask = (uint32_t)on & ((1u << PLACE3D_NSTAGES) - 1u);
  return PLACE3D_OK;
}

int32_t place3d_profile_read(place3d_ctx* ctx, int32_t stage, double* ms, int64_t* launches, int32_t reset) {
  if (!ctx) return PLACE3D_ERR_ARG;
  if (stage < 0 || stage >= PLACE3D_NSTAGES) return set_err(ctx, PLACE3D_ERR_ARG, "bad stage");
  for (auto& r : ctx->prof_pending) {
    P3D_HIP(ctx, hipEventSynchronize(r.b));
    float t = 0.f;
    P3D_HIP(ctx, hipEventElapsedTime(&t, r.a, r.b));
    ctx->prof_ms[r.stage] += t;
    ctx->prof_count[r.stage] += r.launches;
    ctx->prof_free.push_back({r.a, r.b});
  }
  ctx->prof_pending.clear();
  if (ms) *ms = ctx->prof_ms[stage];
  if (launches) *launches = ctx->prof_count[stage];
  if (reset)
    for (int k = 0; k < PLACE3D_NSTAGES; ++k) { ctx->prof_ms[k] = 0.0; ctx->prof_count[k] = 0; }
  return PLACE3D_OK;
}

static int check_ctx(place3d_ctx* ctx) {
  if (!ctx) { g_create_err = "ctx is NULL"; return PLACE3D_ERR_ARG; }
  return PLACE3D_OK;
}

static bool bad_ptr(const void* p) { return !p || (reinterpret_cast<uintptr_t>(p) & 3); }

int32_t place3d_density(place3d_ctx* ctx, const float* xyz, float* rho, void* stream) {
  if (int rc = check_ctx(ctx)) return rc;
  if (bad_ptr(xyz) || bad_ptr(rho)) return set_err(ctx, PLACE3D_ERR_ARG, "xyz/rho NULL or misaligned");
  return p3d::density_forward(ctx, xyz, rho, reinterpret_cast<hipStream_t>(stream));
}

int32_t place3d_field(place3d_ctx* ctx, const float* rho, float* phi, float* ex, float* ey, float* ez,
                      double* energy, void* stream) {
  if (int rc = check_ctx(ctx)) return rc;
  if (bad_ptr(rho)) return set_err(ctx, PLACE3D_ERR_ARG, "rho NULL or misaligned");
  if (energy && !phi) return set_err(ctx, PLACE3D_ERR_ARG, "energy needs phi");
  for (const void* q : {(const void*)phi, (const void*)ex, (const void*)ey, (const void*)ez})
    if (q && (reinterpret_cast<uintptr_t>(q) & 3)) return set_err(ctx, PLACE3D_ERR_ARG, "misaligned output map");
  return p3d::spectral_field(ctx, rho, phi, ex, ey, ez, energy, reinterpret_cast<hipStream_t>(stream));
}

int32_t place3d_field_force(place3d_ctx* ctx, const float* xyz, const float* ex, const float* ey,
                            const float* ez, float lambda, float* grad_xyz, int32_t accumulate, void* stream) {
  if (int rc = check_ctx(ctx)) return rc;
  if (bad_ptr(xyz) || bad_ptr(ex) || bad_ptr(ey) || bad_ptr(ez) || bad_ptr(grad_xyz))
    return set_err(ctx, PLACE3D_ERR_ARG, "NULL or misaligned array");
  if (!std::isfinite(lambda)) return set_err(ctx, PLACE3D_ERR_ARG, "lambda not finite");
  return p3d::density_field_gather(ctx, xyz, ex, ey, ez, -lambda, grad_xyz, accumulate != 0,
                                   reinterpret_cast<hipStream_t>(stream));
}

int32_t place3d_density_vjp(place3d_ctx* ctx, const float* xyz, const float* g_rho, float scale,
                            const double* d_scale, float* grad_xyz, int32_t accumulate, void* stream) {
  if (int rc = check_ctx(ctx)) return rc;
  if (bad_ptr(xyz) || bad_ptr(g_rho) || bad_ptr(grad_xyz)) return set_err(ctx, PLACE3D_ERR_ARG, "NULL or misaligned array");
  if (d_scale && (reinterpret_cast<uintptr_t>(d_scale) & 7)) return set_err(ctx, PLACE3D_ERR_ARG, "misaligned d_scale");
  if (!std::isfinite(scale)) return set_err(ctx, PLACE3D_ERR_ARG, "scale not finite");
  return p3d::density_adjoint(ctx, xyz, g_rho, scale, grad_xyz, accumulate != 0, reinterpret_cast<hipStream_t>(stream),
                              d_scale);
}

int32_t place3d_wl_grad(place3d_ctx* ctx, const float* xyz, float* grad_xyz, double* metrics,
                        int32_t accumulate, void* stream) {
  if (int rc = check_ctx(ctx)) return rc;
  if (bad_ptr(xyz) || bad_ptr(grad_xyz)) return set_err(ctx, PLACE3D_ERR_ARG, "NULL or misaligned array");
  if (metrics && (reinterpret_cast<uintptr_t>(metrics) & 7)) return set_err(ctx, PLACE3D_ERR_ARG, "misaligned metrics");
  return p3d::wirelength_eval(ctx, xyz, grad_xyz, accumulate != 0, ctx->red, metrics,
                              reinterpret_cast<hipStream_t>(stream));
}

int32_t place3d_wl_value(place3d_ctx* ctx, const float* xyz, double* metrics, void* stream) {
  if (int rc = check_ctx(ctx)) return rc;
  if (bad_ptr(xyz)) return set_err(ctx, PLACE3D_ERR_ARG, "xyz NULL or misaligned");
  if (!metrics || (reinterpret_cast<uintptr_t>(metrics) & 7)) return set_err(ctx, PLACE3D_ERR_ARG, "metrics NULL or misaligned");
  return p3d::wirelength_value(ctx, xyz, metrics, reinterpret_cast<hipStream_t>(stream));
}

int32_t place3d_wl_value_static(place3d_ctx* ctx, const float* xyz, double* metrics, void* stream) {
  if (int rc = check_ctx(ctx)) return rc;
  if (bad_ptr(xyz)) return set_err(ctx, PLACE3D_ERR_ARG, "xyz NULL or misaligned");
  if (!metrics || (reinterpret_cast<uintptr_t>(metrics) & 7)) return set_err(ctx, PLACE3D_ERR_ARG, "metrics NULL or misaligned");
  return p3d::wirelength_value_static(ctx, xyz, metrics, reinterpret_cast<hipStream_t>(stream));
}

int32_t place3d_wl_vjp(place3d_ctx* ctx, const float* xyz, const double* d_scale, int32_t z_mode, float* grad_xyz,
                       int32_t accumulate, void* stream) {
  if (int rc = check_ctx(ctx)) return rc;
  if (bad_ptr(xyz) || bad_ptr(grad_xyz)) return set_err(ctx, PLACE3D_ERR_ARG, "NULL or misaligned array");
  if (d_scale && (reinterpret_cast<uintptr_t>(d_scale) & 7)) return set_err(ctx, PLACE3D_ERR_ARG, "misaligned d_scale");
  if (z_mode != PLACE3D_WLZ_FDA && z_mode != PLACE3D_WLZ_VALUE) return set_err(ctx, PLACE3D_ERR_ARG, "bad z_mode");
  return p3d::wirelength_eval(ctx, xyz, grad_xyz, accumulate != 0, ctx->red, nullptr,
                              reinterpret_cast<hipStream_t>(stream), false, d_scale, z_mode == PLACE3D_WLZ_FDA);
}

int32_t place3d_read_scalars(place3d_ctx* ctx, const place3d_state* state, double* host_scalars, void* stream) {
  if (int rc = check_ctx(ctx)) return rc;
  if (!state || !state->scalars || !host_scalars) return set_err(ctx, PLACE3D_ERR_ARG, "NULL state or output");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  P3D_HIP(ctx, hipMemcpyAsync(host_scalars, state->scalars, sizeof(double) * PLACE3D_NSCALARS, hipMemcpyDeviceToHost, s));
  P3D_HIP(ctx, hipStreamSynchronize(s));
  const double flag = host_scalars[PLACE3D_S_NONFINITE];
  if (flag != 0.0)
    return set_err(ctx, PLACE3D_ERR_NONFINITE,
                   "a non-finite value at GP iteration " + std::to_string((long long)flag - 1) +
                       " (step size, gradient change, wirelength, overflow, norm or lambda)");
  return PLACE3D_OK;
}

PLACE3D_API int32_t place3d_plan_fillers(int32_t n_inst, const float* size, const uint8_t* kind, const float* z0,
                                         double die_x, double die_y, int32_t nx, int32_t ny, int32_t nz,
                                         double u_top, double u_bot, place3d_filler_plan* out) {
  if (!size || !kind || !z0 || !out) return PLACE3D_ERR_ARG;
  if (n_inst < 1 || nx < 2 || ny < 2 || nz < 2 || (nz & 1)) return PLACE3D_ERR_SIZE;
  if (!(die_x > 0) || !(die_y > 0) || !std::isfinite(die_x) || !std::isfinite(die_y)) return PLACE3D_ERR_ARG;
  if (!(u_top >= 0 && u_top <= 1) || !(u_bot >= 0 && u_bot <= 1)) return PLACE3D_ERR_ARG;
  const size_t n = (size_t)n_inst;
  const double dz = nz * 0.5 * (die_x / nx + die_y / ny);
  // mean footprint area of the movable standard cells on each die's size
  double a_bot = 0.0, a_top = 0.0;
  long long cells = 0;
  for (size_t i = 0; i < n; ++i) {
    if (kind[i] & (PLACE3D_KIND_MACRO | PLACE3D_KIND_FIXED | PLACE3D_KIND_FILLER)) continue;
    a_bot += (double)size[i] * (double)size[n + i];
    a_top += (double)size[2 * n + i] * (double)size[3 * n + i];
    ++cells;
  }
  if (cells == 0) return PLACE3D_ERR_ARG;
  a_bot /= (double)cells;
  a_top /= (double)cells;
  const double a_free = 0.5 * (a_top + a_bot);
  // vol_a: every instance at the size its initial z gives (cells by partition, macros by the
  // linear transition over the clamped z)
  double vol_a = 0.0;
  for (size_t i = 0; i < n; ++i) {
    const double wb = size[i], hb = size[n + i], wt = size[2 * n + i], ht = size[3 * n + i];
    const double z = z0[i];
    double w, h;
    if (kind[i] & PLACE3D_KIND_MACRO) {
      const double zc = std::min(std::max(z, 0.25 * dz), 0.75 * dz);
      const double t = 2.0 * zc / dz;
      w = (t - 0.5) * wt + (1.5 - t) * wb;
      h = (t - 0.5) * ht + (1.5 - t) * hb;
    } else {
      const bool top = z > 0.5 * dz;
      w = top ? wt : wb;
      h = top ? ht : hb;
    }
    vol_a += w * h * 0.5 * dz;
  }
  const double total = die_x * die_y * dz;
  out->vol_top = 0.5 * total * (1.0 - u_top);
  out->vol_bot = 0.5 * total * (1.0 - u_bot);
  out->vol_free = std::max(total - (out->vol_top + out->vol_bot + vol_a), 0.0);
  out->vol_a = vol_a;
  out->side_top = std::sqrt(a_top);
  out->side_bot = std::sqrt(a_bot);
  out->side_free = std::sqrt(a_free);
  auto count = [&](double vol, double area) { return (int64_t)std::floor(vol / (area * 0.5 * dz) + 0.5); };
  out->n_top = count(out->vol_top, a_top);
  out->n_bot = count(out->vol_bot, a_bot);
  out->n_free = count(out->vol_free, a_free);
  return PLACE3D_OK;
}

}  // extern "C"
