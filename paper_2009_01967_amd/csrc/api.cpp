// C ABI entry points: argument validation, host-to-device staging of the
// structure and force constants, and dispatch to the device stages.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <sstream>
#include <tuple>

#include "common.h"
#include "internal.h"
#include "tune.h"

namespace kaldo {

kaldo_status fail(kaldo_ctx ctx, kaldo_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

thread_local Arena* g_arena = nullptr;

// Step-B and GEMM-1 output per partner batch of a crystal in the persistent
// batch kernel (one pool shared by the crystals, which run one after the
// other): larger rounds than an eager call's (256 MB), so that each GEMM phase
// has many block tiles per resident workgroup and the rounds, with their two
// grid barriers each, are few.  32 GB (on the 32-crystal batch, 1/16 of the
// points: 4 GB 13.63 s, 8 GB 13.35 s, 16 GB 13.27 s; later 16 GB 12.92 s,
// 32 GB 12.85 s), at most a quarter of the device memory free at planning
// time, at least 1 GB.
// (KALDO_BATCH_XY_MB in the environment overrides it, for tuning.)
static size_t batch_xy_budget() {
  const char* e = std::getenv("KALDO_BATCH_XY_MB");
  const long v = e ? std::atol(e) : 0;
  if (v > 0) return (size_t)v << 20;
  size_t budget = (size_t)32 << 30;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) budget = std::min(budget, free_b / 4);
  return std::max(budget, (size_t)1 << 30);
}

kaldo_status hip_fail(kaldo_ctx ctx, hipError_t e, const char* what) {
  std::ostringstream os;
  os << what << ": " << hipGetErrorString(e);
  if (e == hipErrorOutOfMemory && g_arena && g_arena->short_by)
    os << " (the workspace is " << g_arena->short_by << " bytes short)";
  return fail(ctx, e == hipErrorOutOfMemory ? KALDO_ENOMEM : KALDO_EDEVICE, os.str());
}

void prof_begin(kaldo_ctx ctx) {
  if (!ctx->prof || ctx->mode != kRun) return;
  if (hipEventCreate(&ctx->prof_open) != hipSuccess) {
    ctx->prof_open = nullptr;
    return;
  }
  (void)hipEventRecord(ctx->prof_open, ctx->stream);
}

void prof_end(kaldo_ctx ctx, const char* name) {
  if (!ctx->prof || !ctx->prof_open || ctx->mode != kRun) return;
  hipEvent_t stop;
  if (hipEventCreate(&stop) != hipSuccess) return;
  (void)hipEventRecord(stop, ctx->stream);
  ctx->prof_tab[name].pending.emplace_back(ctx->prof_open, stop);
  ctx->prof_open = nullptr;
}

static void prof_collect(kaldo_ctx ctx) {
  for (auto& kv : ctx->prof_tab) {
    for (auto& ev : kv.second.pending) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ev.first, ev.second) == hipSuccess) {
        kv.second.total_ms += ms;
        kv.second.launches += 1;
      }
      (void)hipEventDestroy(ev.first);
      (void)hipEventDestroy(ev.second);
    }
    kv.second.pending.clear();
  }
}

void prof_clear(kaldo_ctx ctx) {
  (void)hipStreamSynchronize(ctx->stream);
  prof_collect(ctx);
  ctx->prof_tab.clear();
  ctx->prof_dense = 0.0;
  ctx->prof_batch_executed = 0.0;
}

int autotune(kaldo_ctx ctx, const std::string& key, int nv, int fallback, const std::function<void(int)>& launch) {
  kaldo_ctx owner = ctx->tune_owner ? ctx->tune_owner : ctx;
  if (owner->tuning >= KALDO_TUNE_SHAPE0) {
    const int v = owner->tuning - KALDO_TUNE_SHAPE0;
    return v < nv ? v : fallback;
  }
  if (owner->tuning != KALDO_TUNE_AUTO || nv <= 1) return fallback;
  auto it = owner->tuned.find(key);
  if (it != owner->tuned.end()) return it->second;
  if (ctx->mode == kCapture) return fallback;  // no timing inside a capture
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fallback;
  }
  int best = fallback;
  float best_ms = 0.0f;
  for (int v = 0; v < nv; ++v) {
    launch(v);
    (void)hipEventRecord(e0, ctx->stream);
    launch(v);
    (void)hipEventRecord(e1, ctx->stream);
    float ms = 0.0f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) continue;
    if (v == 0 || ms < best_ms) {
      best = v;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  owner->tuned[key] = best;
  return best;
}

std::vector<int> linewidth_points(const kaldo_ctx_s* c) {
  std::vector<char> take(c->nk, 0);
  for (int k = k_lo(c); k < k_hi(c); ++k) take[std::min(k, k_mirror(k, c->grid[0], c->grid[1], c->grid[2]))] = 1;
  std::vector<int> out;
  for (int k = 0; k < c->nk; ++k)
    if (take[k]) out.push_back(k);
  return out;
}

kaldo_status upload_linewidth_points(kaldo_ctx ctx, int* npts) {
  std::vector<int> pts = linewidth_points(ctx);
  *npts = (int)pts.size();
  if (ctx->mode == kCapture) {
    if (pts != ctx->klist_host) return fail(ctx, KALDO_ESTATE, "first-mode points changed after planning");
    return KALDO_OK;
  }
  KALDO_HIP(ctx, ctx->d_klist.ensure(pts.size() * sizeof(int)));
  ctx->klist_host = std::move(pts);
  KALDO_HIP(ctx, hipMemcpyAsync(ctx->d_klist.p, ctx->klist_host.data(), ctx->klist_host.size() * sizeof(int),
                                hipMemcpyHostToDevice, ctx->stream));
  return KALDO_OK;
}

kaldo_status copy_out(kaldo_ctx ctx, void* dst, const void* src, size_t bytes) {
  if (!dst || bytes == 0) return KALDO_OK;
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  bool device = false;
  hipError_t e = hipPointerGetAttributes(&attr, dst);
  if (e == hipSuccess) {
    device = attr.type == hipMemoryTypeDevice;
  } else {
    (void)hipGetLastError();
  }
  if (device) {
    KALDO_HIP(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  } else {
    KALDO_HIP(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->stream));
    KALDO_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  return KALDO_OK;
}

// src: host memory or device memory of the context's GPU; complete on the
// context's stream in order (a host source is copied before the call returns)
kaldo_status copy_in(kaldo_ctx ctx, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return KALDO_OK;
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  bool device = false;
  hipError_t e = hipPointerGetAttributes(&attr, src);
  if (e == hipSuccess) {
    device = attr.type == hipMemoryTypeDevice;
  } else {
    (void)hipGetLastError();
  }
  if (device) {
    KALDO_HIP(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  } else {
    KALDO_HIP(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
    KALDO_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  return KALDO_OK;
}

template <typename T>
static kaldo_status upload(kaldo_ctx ctx, DevBuf& buf, const T* src, size_t count) {
  KALDO_HIP(ctx, buf.ensure(count * sizeof(T)));
  if (count) KALDO_HIP(ctx, hipMemcpy(buf.p, src, count * sizeof(T), hipMemcpyHostToDevice));
  return KALDO_OK;
}

static bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

static kaldo_status load_structure(kaldo_ctx ctx, const kaldo_structure* s) {
  if (!s->positions || !s->masses) return fail(ctx, KALDO_EINVAL, "structure: NULL positions or masses");
  if (s->n_atoms < 1 || s->n_atoms > 100000) return fail(ctx, KALDO_EINVAL, "structure: n_atoms out of range");
  const int N = s->n_atoms;
  if (!finite_all(s->cell, 9) || !finite_all(s->positions, 3 * (size_t)N))
    return fail(ctx, KALDO_EINVAL, "structure: non-finite cell or positions");
  const double* c = s->cell;
  double det = c[0] * (c[4] * c[8] - c[5] * c[7]) - c[1] * (c[3] * c[8] - c[5] * c[6]) +
               c[2] * (c[3] * c[7] - c[4] * c[6]);
  if (!(std::fabs(det) > 1e-6)) return fail(ctx, KALDO_EINVAL, "structure: singular cell");
  for (int a = 0; a < N; ++a)
    if (!(s->masses[a] > 0.0) || !std::isfinite(s->masses[a]))
      return fail(ctx, KALDO_EINVAL, "structure: masses must be positive");
  ctx->n_atoms = N;
  std::memcpy(ctx->cell, s->cell, sizeof(ctx->cell));
  ctx->positions.assign(s->positions, s->positions + 3 * N);
  ctx->masses.assign(s->masses, s->masses + N);
  kaldo_status st;
  if ((st = upload(ctx, ctx->d_positions, s->positions, 3 * (size_t)N)) != KALDO_OK) return st;
  if ((st = upload(ctx, ctx->d_masses, s->masses, (size_t)N)) != KALDO_OK) return st;
  ctx->have_structure = true;
  // force constants refer to atom indices of the previous structure
  ctx->have_fc2 = ctx->have_fc3 = ctx->have_phonons = ctx->have_gamma = false;
  return KALDO_OK;
}

static kaldo_status load_fc2(kaldo_ctx ctx, const kaldo_fc2* f) {
  const int N = ctx->n_atoms;
  const int64_t nb = f->n_blocks;
  if (nb < 1 || !f->i || !f->j || !f->R || !f->blocks) return fail(ctx, KALDO_EINVAL, "fc2: empty or NULL arrays");
  for (int64_t b = 0; b < nb; ++b) {
    if (f->i[b] < 0 || f->i[b] >= N || f->j[b] < 0 || f->j[b] >= N)
      return fail(ctx, KALDO_EINVAL, "fc2: atom index out of range at block " + std::to_string(b));
    for (int c = 0; c < 3; ++c)
      if (std::abs(f->R[3 * b + c]) > 15) return fail(ctx, KALDO_EINVAL, "fc2: |R| > 15 at block " + std::to_string(b));
  }
  if (!finite_all(f->blocks, 9 * (size_t)nb)) return fail(ctx, KALDO_EINVAL, "fc2: non-finite values");
  std::vector<int64_t> order(nb);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    return std::make_pair(f->i[x], f->j[x]) < std::make_pair(f->i[y], f->j[y]);
  });
  std::vector<int> pair(2 * (size_t)N * N, 0), R(3 * nb), bi(nb), bj(nb);
  std::vector<double> val(9 * nb);
  for (int64_t q = 0; q < nb; ++q) {
    int64_t b = order[q];
    bi[q] = f->i[b];
    bj[q] = f->j[b];
    for (int c = 0; c < 3; ++c) R[3 * q + c] = f->R[3 * b + c];
    for (int c = 0; c < 9; ++c) val[9 * q + c] = f->blocks[9 * b + c];
  }
  for (int64_t q = 0; q < nb; ++q) {
    size_t p = (size_t)bi[q] * N + bj[q];
    if (pair[2 * p + 1] == 0) pair[2 * p] = (int)q;
    pair[2 * p + 1] = (int)q + 1;
  }
  // the coupled atom pairs row by row (i, j, first block, end): the sparse
  // displacement Hessian of the QHGK velocities has one 3 x 3 block per pair
  std::vector<int> rows((size_t)N + 1, 0), plist;
  for (int64_t q = 0; q < nb;) {
    int64_t e = q;
    while (e < nb && bi[e] == bi[q] && bj[e] == bj[q]) ++e;
    plist.insert(plist.end(), {bi[q], bj[q], (int)q, (int)e});
    rows[(size_t)bi[q] + 1] += 1;
    q = e;
  }
  for (int i = 0; i < N; ++i) rows[(size_t)i + 1] += rows[i];
  kaldo_status st;
  if ((st = upload(ctx, ctx->d_fc2_rows, rows.data(), rows.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, ctx->d_fc2_plist, plist.data(), plist.size())) != KALDO_OK) return st;
  ctx->n_fc2_pairs = (int)(plist.size() / 4);
  if ((st = upload(ctx, ctx->d_fc2_pair, pair.data(), pair.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, ctx->d_fc2_R, R.data(), R.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, ctx->d_fc2_val, val.data(), val.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, ctx->d_fc2_i, bi.data(), bi.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, ctx->d_fc2_j, bj.data(), bj.size())) != KALDO_OK) return st;
  ctx->nb2 = nb;
  ctx->have_fc2 = true;
  ctx->have_phonons = ctx->have_gamma = false;
  return KALDO_OK;
}

static kaldo_status load_fc3(kaldo_ctx ctx, const kaldo_fc3* f) {
  const int N = ctx->n_atoms;
  const int64_t nb = f->n_blocks;
  if (nb < 0 || (nb > 0 && (!f->i || !f->j || !f->l || !f->R1 || !f->R2 || !f->blocks)))
    return fail(ctx, KALDO_EINVAL, "fc3: NULL arrays");
  if (nb > (int64_t)1 << 30) return fail(ctx, KALDO_EINVAL, "fc3: too many blocks");
  for (int64_t b = 0; b < nb; ++b) {
    if (f->i[b] < 0 || f->i[b] >= N || f->j[b] < 0 || f->j[b] >= N || f->l[b] < 0 || f->l[b] >= N)
      return fail(ctx, KALDO_EINVAL, "fc3: atom index out of range at block " + std::to_string(b));
    for (int c = 0; c < 3; ++c)
      if (std::abs(f->R1[3 * b + c]) > 7 || std::abs(f->R2[3 * b + c]) > 7)
        return fail(ctx, KALDO_EINVAL, "fc3: |R| > 7 at block " + std::to_string(b));
  }
  if (nb && !finite_all(f->blocks, 27 * (size_t)nb)) return fail(ctx, KALDO_EINVAL, "fc3: non-finite values");
  // distinct Delta = R2 - R1
  std::map<std::tuple<int, int, int>, int> dmap;
  std::vector<int> didx(nb);
  for (int64_t b = 0; b < nb; ++b) {
    auto key = std::make_tuple(f->R2[3 * b] - f->R1[3 * b], f->R2[3 * b + 1] - f->R1[3 * b + 1],
                               f->R2[3 * b + 2] - f->R1[3 * b + 2]);
    dmap.emplace(key, -1);
  }
  Fc3Layout& L = ctx->fc3;
  L.delta.clear();
  // Slot order: pairs (Delta, -Delta), Delta != 0, in adjacent slots 2m, 2m + 1
  // first, then every Delta whose negative is absent, and Delta = 0.  The
  // few-branch projection sums each pair with one real phase multiply per part.
  int nd = 0;
  auto put = [&](std::map<std::tuple<int, int, int>, int>::iterator it) {
    it->second = nd++;
    L.delta.push_back(std::get<0>(it->first));
    L.delta.push_back(std::get<1>(it->first));
    L.delta.push_back(std::get<2>(it->first));
  };
  const auto zero = std::make_tuple(0, 0, 0);
  for (auto it = dmap.begin(); it != dmap.end(); ++it) {
    if (!(zero < it->first)) continue;
    auto neg = dmap.find(std::make_tuple(-std::get<0>(it->first), -std::get<1>(it->first), -std::get<2>(it->first)));
    if (neg == dmap.end()) continue;
    put(it);
    put(neg);
  }
  L.n_dpair = nd / 2;
  for (auto it = dmap.begin(); it != dmap.end(); ++it)
    if (it->second < 0) put(it);
  for (int64_t b = 0; b < nb; ++b) {
    auto key = std::make_tuple(f->R2[3 * b] - f->R1[3 * b], f->R2[3 * b + 1] - f->R1[3 * b + 1],
                               f->R2[3 * b + 2] - f->R1[3 * b + 2]);
    didx[b] = dmap[key];
  }
  std::vector<int64_t> order(nb);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    return std::make_tuple(didx[x], f->j[x], f->l[x]) < std::make_tuple(didx[y], f->j[y], f->l[y]);
  });
  const size_t ngroup = (size_t)std::max(nd, 1) * N * N;
  std::vector<int> group(2 * ngroup, 0), bi(std::max<int64_t>(nb, 1)), bj(std::max<int64_t>(nb, 1)),
      bl(std::max<int64_t>(nb, 1)), R2(3 * std::max<int64_t>(nb, 1));
  std::vector<double> val(27 * std::max<int64_t>(nb, 1), 0.0);
  for (int64_t q = 0; q < nb; ++q) {
    const int64_t b = order[q];
    bi[q] = f->i[b];
    bj[q] = f->j[b];
    bl[q] = f->l[b];
    for (int c = 0; c < 3; ++c) R2[3 * q + c] = f->R2[3 * b + c];
    const double s = 1.0 / std::sqrt(ctx->masses[bi[q]] * ctx->masses[bj[q]] * ctx->masses[bl[q]]);
    for (int c = 0; c < 27; ++c) val[27 * q + c] = f->blocks[27 * b + c] * s;
    const size_t g = ((size_t)didx[b] * N + bj[q]) * N + bl[q];
    if (group[2 * g + 1] == 0) group[2 * g] = (int)q;
    group[2 * g + 1] = (int)q + 1;
  }
  if (nd == 0) {
    L.delta.assign(3, 0);
    nd = 1;
  }
  // crystal layout: non-empty (Delta, j, l) groups and their per-pair lists
  std::vector<int> cg_block, cg_delta, cg_j, cg_l;
  for (int d = 0; d < nd; ++d)
    for (int j = 0; j < N; ++j)
      for (int l = 0; l < N; ++l) {
        const size_t g = ((size_t)d * N + j) * N + l;
        if (group[2 * g + 1] > group[2 * g]) {
          cg_block.push_back(group[2 * g]);
          cg_block.push_back(group[2 * g + 1]);
          cg_delta.push_back(d);
          cg_j.push_back(j);
          cg_l.push_back(l);
        }
      }
  const int ng = (int)cg_delta.size();
  std::vector<int> cg_order(ng);
  std::iota(cg_order.begin(), cg_order.end(), 0);
  std::stable_sort(cg_order.begin(), cg_order.end(), [&](int x, int y) {
    return std::make_tuple(cg_j[x], cg_l[x], cg_delta[x]) < std::make_tuple(cg_j[y], cg_l[y], cg_delta[y]);
  });
  std::vector<int> cpair;  // (j, l, first, last+1)
  for (int q = 0; q < ng; ++q) {
    const int g = cg_order[q];
    if (q == 0 || cg_j[g] != cg_j[cg_order[q - 1]] || cg_l[g] != cg_l[cg_order[q - 1]]) {
      cpair.insert(cpair.end(), {cg_j[g], cg_l[g], q, q + 1});
    } else {
      cpair.back() = q + 1;
    }
  }
  const int ncp = (int)cpair.size() / 4;
  if (ng == 0) {
    cg_block.assign(2, 0);
    cg_delta.assign(1, 0);
    cg_order.assign(1, 0);
  }
  std::vector<int> cpairmap((size_t)N * N, -1);
  for (int c = 0; c < ncp; ++c) cpairmap[(size_t)cpair[4 * c] * N + cpair[4 * c + 1]] = c;
  if (ncp == 0) cpair.assign(4, 0);
  // Gamma-point layout: blocks grouped by atom pair (j, l), all cells merged
  std::vector<int64_t> gorder(nb);
  std::iota(gorder.begin(), gorder.end(), 0);
  std::stable_sort(gorder.begin(), gorder.end(), [&](int64_t x, int64_t y) {
    return std::make_pair(f->j[x], f->l[x]) < std::make_pair(f->j[y], f->l[y]);
  });
  std::vector<int> gpstart, gpl, grow(N + 1, 0), gbi(std::max<int64_t>(nb, 1));
  std::vector<double> gval(27 * std::max<int64_t>(nb, 1), 0.0);
  for (int64_t q = 0; q < nb; ++q) {
    const int64_t b = gorder[q];
    const bool fresh = q == 0 || f->j[b] != f->j[gorder[q - 1]] || f->l[b] != f->l[gorder[q - 1]];
    if (fresh) {
      gpstart.push_back((int)q);
      gpl.push_back(f->l[b]);
      grow[f->j[b] + 1] += 1;
    }
    gbi[q] = f->i[b];
    const double s = 1.0 / std::sqrt(ctx->masses[f->i[b]] * ctx->masses[f->j[b]] * ctx->masses[f->l[b]]);
    for (int c = 0; c < 27; ++c) gval[27 * q + c] = f->blocks[27 * b + c] * s;
  }
  const int npairs = (int)gpl.size();
  gpstart.push_back((int)nb);
  for (int a = 0; a < N; ++a) grow[a + 1] += grow[a];
  if (gpl.empty()) gpl.push_back(0);
  kaldo_status st;
  if ((st = upload(ctx, L.d_group, group.data(), group.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, L.d_blk_i, bi.data(), bi.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, L.d_blk_j, bj.data(), bj.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, L.d_blk_l, bl.data(), bl.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, L.d_blk_R2, R2.data(), R2.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, L.d_blk_val, val.data(), val.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, L.d_delta, L.delta.data(), L.delta.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, L.d_gpair_start, gpstart.data(), gpstart.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, L.d_gpair_l, gpl.data(), gpl.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, L.d_grow_start, grow.data(), grow.size())) != KALDO_OK) return st;
  L.grow_start = grow;
  if ((st = upload(ctx, L.d_gblk_i, gbi.data(), gbi.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, L.d_gblk_val, gval.data(), gval.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, L.d_cg_block, cg_block.data(), cg_block.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, L.d_cg_delta, cg_delta.data(), cg_delta.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, L.d_cg_order, cg_order.data(), cg_order.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, L.d_cpair, cpair.data(), cpair.size())) != KALDO_OK) return st;
  if ((st = upload(ctx, L.d_cpairmap, cpairmap.data(), cpairmap.size())) != KALDO_OK) return st;
  L.n_cgroups = ng;
  L.n_cpairs = ncp;
  L.n_pairs = npairs;
  L.n_blocks = nb;
  L.n_delta = nd;
  ctx->have_fc3 = true;
  ctx->have_gamma = false;
  return KALDO_OK;
}

}  // namespace kaldo

using namespace kaldo;

extern "C" {

kaldo_status kaldo_create(kaldo_ctx* out, int device, void* hip_stream) {
  if (!out) return KALDO_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return KALDO_EDEVICE;
  if (device < 0 || device >= ndev) return KALDO_EINVAL;
  kaldo_ctx ctx = new (std::nothrow) kaldo_ctx_s();
  if (!ctx) return KALDO_ENOMEM;
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return KALDO_EDEVICE;
  }
  if (hip_stream) {
    ctx->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreate(&ctx->stream) != hipSuccess) {
      delete ctx;
      return KALDO_EDEVICE;
    }
    ctx->own_stream = true;
  }
  if (rocblas_create_handle(&ctx->blas) != rocblas_status_success) {
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return KALDO_EDEVICE;
  }
  rocblas_set_stream(ctx->blas, ctx->stream);
  // device address of the allocation-free entry point's scratch array (its
  // failure only disables kaldo_kappa_rta_noalloc, which then reports it)
  (void)noalloc_setup(device);
  *out = ctx;
  return KALDO_OK;
}

// Destroy the captured batch graph once the stream has drained (a launch of it
// may still be in flight).
static void batch_drop_graph(kaldo_ctx ctx) {
  if (ctx->batch_exec) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipGraphExecDestroy(ctx->batch_exec);
  }
  ctx->batch_exec = nullptr;
  ctx->batch_key.clear();
}

static void batch_release(kaldo_ctx ctx) {
  batch_drop_graph(ctx);
  ctx->batch_key.clear();
  for (kaldo_ctx sub : ctx->batch) kaldo_destroy(sub);
  ctx->batch.clear();
}

void kaldo_destroy(kaldo_ctx ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  batch_release(ctx);
  prof_clear(ctx);
  if (ctx->blas) rocblas_destroy_handle(ctx->blas);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

const char* kaldo_last_error(kaldo_ctx ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

kaldo_status kaldo_phonons(kaldo_ctx ctx, const kaldo_structure* structure, const kaldo_fc2* fc2,
                           const int32_t grid[3], double* nu_out, double* vel_out) {
  if (!ctx) return KALDO_EINVAL;
  ArenaScope arena_scope(&ctx->arena);
  ctx->err.clear();
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  if (!grid) return fail(ctx, KALDO_EINVAL, "grid is NULL");
  int64_t nk = 1;
  for (int c = 0; c < 3; ++c) {
    if (grid[c] < 1 || grid[c] > 4096) return fail(ctx, KALDO_EINVAL, "grid entries must be in [1, 4096]");
    nk *= grid[c];
  }
  if (nk > (1 << 22)) return fail(ctx, KALDO_EINVAL, "grid too large");
  kaldo_status st;
  if (structure) {
    if ((st = load_structure(ctx, structure)) != KALDO_OK) return st;
  } else if (!ctx->have_structure) {
    return fail(ctx, KALDO_ESTATE, "no structure resident: pass one");
  }
  if (fc2) {
    if ((st = load_fc2(ctx, fc2)) != KALDO_OK) return st;
  } else if (!ctx->have_fc2) {
    return fail(ctx, KALDO_ESTATE, "no fc2 resident: pass one");
  }
  for (int c = 0; c < 3; ++c) ctx->grid[c] = grid[c];
  ctx->nk = (int)nk;
  ctx->nm = 3 * ctx->n_atoms;
  ctx->have_phonons = false;
  ctx->have_gamma = false;
  const bool want_vel = nk > 1;
  if ((st = run_phonons(ctx, want_vel)) != KALDO_OK) return st;
  ctx->have_phonons = true;
  const size_t nmode = (size_t)ctx->nk * ctx->nm;
  if (nu_out) {
    // nu = omega / 2 pi is computed on the device into the scratch buffer
    if ((st = copy_out(ctx, nu_out, ctx->d_work.p, nmode * sizeof(double))) != KALDO_OK) return st;
  }
  if (vel_out) {
    if (!want_vel) {
      KALDO_HIP(ctx, ctx->d_vel.ensure(nmode * 3 * sizeof(double)));
      KALDO_HIP(ctx, hipMemsetAsync(ctx->d_vel.p, 0, nmode * 3 * sizeof(double), ctx->stream));
    }
    if ((st = copy_out(ctx, vel_out, ctx->d_vel.p, nmode * 3 * sizeof(double))) != KALDO_OK) return st;
  }
  return KALDO_OK;
}

static kaldo_status check_linewidth_args(kaldo_ctx ctx, const double* T, int32_t nT, double sigma_thz,
                                         kaldo_delta delta, kaldo_stats stats, kaldo_precision precision) {
  if (!T || nT < 1 || nT > KALDO_MAX_T) return fail(ctx, KALDO_EINVAL, "need 1 <= nT <= KALDO_MAX_T temperatures");
  if (delta != KALDO_DELTA_GAUSS && delta != KALDO_DELTA_LORENTZ && delta != KALDO_DELTA_TRIANGLE)
    return fail(ctx, KALDO_EINVAL, "unknown delta kind");
  if (stats != KALDO_QUANTUM && stats != KALDO_CLASSICAL) return fail(ctx, KALDO_EINVAL, "bad statistics");
  if (precision != KALDO_FP64 && precision != KALDO_FP32 && precision != KALDO_BF16X3)
    return fail(ctx, KALDO_EINVAL, "bad precision");
  if (!(sigma_thz > 0.0) || !std::isfinite(sigma_thz)) return fail(ctx, KALDO_EINVAL, "sigma must be > 0");
  for (int t = 0; t < nT; ++t) {
    if (!std::isfinite(T[t]) || T[t] < 0.0 || (T[t] == 0.0 && stats == KALDO_CLASSICAL))
      return fail(ctx, KALDO_EINVAL, "temperatures must be finite, >= 0 (> 0 for classical)");
  }
  return KALDO_OK;
}

kaldo_status kaldo_linewidths(kaldo_ctx ctx, const kaldo_fc3* fc3, const double* T, int32_t nT,
                              double sigma_thz, kaldo_delta delta, kaldo_stats stats,
                              kaldo_precision precision, double* gamma_out) {
  if (!ctx) return KALDO_EINVAL;
  ArenaScope arena_scope(&ctx->arena);
  ctx->err.clear();
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  if (!ctx->have_phonons) return fail(ctx, KALDO_ESTATE, "kaldo_linewidths before kaldo_phonons");
  kaldo_status st;
  if ((st = check_linewidth_args(ctx, T, nT, sigma_thz, delta, stats, precision)) != KALDO_OK) return st;
  if (fc3) {
    if ((st = load_fc3(ctx, fc3)) != KALDO_OK) return st;
  } else if (!ctx->have_fc3) {
    return fail(ctx, KALDO_ESTATE, "no fc3 resident: pass one");
  }
  if (k_lo(ctx) >= k_hi(ctx)) return fail(ctx, KALDO_EINVAL, "the k range holds no grid point");
  if (ctx->adaptive_scale > 0.0 && (delta != KALDO_DELTA_GAUSS || ctx->nk == 1))
    return fail(ctx, KALDO_EINVAL, "adaptive widths need the Gaussian delta and a grid other than {1,1,1}");
  ctx->nT = nT;
  for (int t = 0; t < nT; ++t) ctx->T[t] = T[t];
  ctx->stats = stats;
  ctx->delta = delta;
  ctx->sigma_thz = sigma_thz;
  ctx->have_gamma = false;
  ctx->gamma_external = false;
  ctx->gamma_adaptive = ctx->adaptive_scale > 0.0;
  if ((st = run_linewidths(ctx, sigma_thz, precision)) != KALDO_OK) return st;
  ctx->g_lo = k_lo(ctx);
  ctx->g_hi = k_hi(ctx);
  ctx->have_gamma = true;
  if (gamma_out) {
    const size_t bytes = (size_t)nT * ctx->nk * ctx->nm * sizeof(double);
    if ((st = copy_out(ctx, gamma_out, ctx->d_gamma.p, bytes)) != KALDO_OK) return st;
  }
  return KALDO_OK;
}

kaldo_status kaldo_phase_space(kaldo_ctx ctx, const double* T, int32_t nT, double sigma_thz, kaldo_delta delta,
                               kaldo_stats stats, double* g_out) {
  if (!ctx) return KALDO_EINVAL;
  ArenaScope arena_scope(&ctx->arena);
  ctx->err.clear();
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  if (!ctx->have_phonons) return fail(ctx, KALDO_ESTATE, "kaldo_phase_space before kaldo_phonons");
  kaldo_status st;
  if ((st = check_linewidth_args(ctx, T, nT, sigma_thz, delta, stats, KALDO_FP64)) != KALDO_OK) return st;
  if (!g_out) return fail(ctx, KALDO_EINVAL, "g_out is required");
  double* g = nullptr;
  if ((st = run_phase_space(ctx, T, nT, sigma_thz, delta, stats, &g)) != KALDO_OK) return st;
  return copy_out(ctx, g_out, g, (size_t)nT * ctx->nk * ctx->nm * sizeof(double));
}

kaldo_status kaldo_kappa_rta(kaldo_ctx ctx, double* kappa_out) {
  if (!ctx) return KALDO_EINVAL;
  ArenaScope arena_scope(&ctx->arena);
  ctx->err.clear();
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  if (!ctx->have_gamma) return fail(ctx, KALDO_ESTATE, "kaldo_kappa_rta before kaldo_linewidths");
  if (ctx->nk == 1) return fail(ctx, KALDO_EINVAL, "kaldo_kappa_rta needs a grid other than {1,1,1}");
  kaldo_status st;
  if ((st = run_kappa_rta(ctx)) != KALDO_OK) return st;
  if (kappa_out) return copy_out(ctx, kappa_out, ctx->d_kappa.p, (size_t)ctx->nT * 9 * sizeof(double));
  return KALDO_OK;
}

kaldo_status kaldo_kappa_bte(kaldo_ctx ctx, kaldo_bte_method method, int32_t max_terms, double tol,
                             double* kappa_out, int32_t* terms_out) {
  if (!ctx) return KALDO_EINVAL;
  ArenaScope arena_scope(&ctx->arena);
  ctx->err.clear();
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  if (terms_out) *terms_out = 0;
  if (!ctx->have_gamma || !ctx->have_fc3 || ctx->gamma_external)
    return fail(ctx, KALDO_ESTATE, "kaldo_kappa_bte before kaldo_linewidths");
  if (ctx->gamma_adaptive)
    return fail(ctx, KALDO_EINVAL, "kaldo_kappa_bte: the scattering operator takes the fixed width, not adaptive ones");
  if (method != KALDO_BTE_INVERSE && method != KALDO_BTE_SELF_CONSISTENT)
    return fail(ctx, KALDO_EINVAL, "kaldo_kappa_bte: unknown method");
  if (method == KALDO_BTE_SELF_CONSISTENT && (max_terms < 1 || !(tol > 0.0) || !std::isfinite(tol)))
    return fail(ctx, KALDO_EINVAL, "kaldo_kappa_bte: need max_terms >= 1 and tol > 0");
  if (!kappa_out) return fail(ctx, KALDO_EINVAL, "kaldo_kappa_bte: kappa_out is required");
  if (ctx->nk == 1) return fail(ctx, KALDO_EINVAL, "kaldo_kappa_bte needs a grid other than {1,1,1}");
  if (ctx->nm != 3 && ctx->nm != 6)
    return fail(ctx, KALDO_EINVAL, "kaldo_kappa_bte: implemented for cells of 1 or 2 atoms");
  if (k_partial(ctx)) return fail(ctx, KALDO_EINVAL, "kaldo_kappa_bte: needs the whole grid (no k range)");
  int terms = 0;
  const kaldo_status st = run_kappa_bte(ctx, method, max_terms, tol, kappa_out, &terms);
  if (terms_out) *terms_out = terms;
  return st;
}

kaldo_status kaldo_kappa_rta_noalloc(kaldo_ctx ctx, double* kappa_out) {
  if (!ctx) return KALDO_EINVAL;
  ctx->err.clear();
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  if (!ctx->have_gamma) return fail(ctx, KALDO_ESTATE, "kaldo_kappa_rta_noalloc before kaldo_linewidths");
  if (ctx->nk == 1) return fail(ctx, KALDO_EINVAL, "kaldo_kappa_rta_noalloc needs a grid other than {1,1,1}");
  if (!kappa_out) return fail(ctx, KALDO_EINVAL, "kaldo_kappa_rta_noalloc: kappa_out is required");
  return run_kappa_rta_noalloc(ctx, kappa_out);
}

kaldo_status kaldo_kappa_qhgk(kaldo_ctx ctx, double* kappa_out) {
  if (!ctx) return KALDO_EINVAL;
  ArenaScope arena_scope(&ctx->arena);
  ctx->err.clear();
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  if (!ctx->have_gamma) return fail(ctx, KALDO_ESTATE, "kaldo_kappa_qhgk before kaldo_linewidths");
  if (ctx->nk != 1) return fail(ctx, KALDO_EINVAL, "kaldo_kappa_qhgk needs grid {1,1,1}");
  kaldo_status st;
  if ((st = run_kappa_qhgk(ctx)) != KALDO_OK) return st;
  if (kappa_out) return copy_out(ctx, kappa_out, ctx->d_kappa.p, (size_t)ctx->nT * 9 * sizeof(double));
  return KALDO_OK;
}

kaldo_status kaldo_mode_diffusivity(kaldo_ctx ctx, double* d_out) {
  if (!ctx) return KALDO_EINVAL;
  ArenaScope arena_scope(&ctx->arena);
  ctx->err.clear();
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  if (!ctx->have_gamma) return fail(ctx, KALDO_ESTATE, "kaldo_mode_diffusivity before kaldo_linewidths");
  if (ctx->nk != 1) return fail(ctx, KALDO_EINVAL, "kaldo_mode_diffusivity needs grid {1,1,1}");
  if (!d_out) return fail(ctx, KALDO_EINVAL, "kaldo_mode_diffusivity: d_out is required");
  kaldo_status st;
  if ((st = run_mode_diffusivity(ctx)) != KALDO_OK) return st;
  return copy_out(ctx, d_out, ctx->d_diff.p, (size_t)ctx->nT * ctx->nm * 3 * sizeof(double));
}

kaldo_status kaldo_adaptive_width(kaldo_ctx ctx, double scale) {
  if (!ctx) return KALDO_EINVAL;
  ctx->err.clear();
  if (!std::isfinite(scale) || scale < 0.0)
    return fail(ctx, KALDO_EINVAL, "kaldo_adaptive_width: scale must be finite and >= 0");
  ctx->adaptive_scale = scale;
  return KALDO_OK;
}

kaldo_status kaldo_qhgk_options(kaldo_ctx ctx, double bandwidth, double threshold) {
  if (!ctx) return KALDO_EINVAL;
  ctx->err.clear();
  if (!std::isfinite(bandwidth) || bandwidth < 0.0)
    return fail(ctx, KALDO_EINVAL, "kaldo_qhgk_options: bandwidth must be finite and >= 0");
  if (std::isnan(threshold) || threshold < 0.0)
    return fail(ctx, KALDO_EINVAL, "kaldo_qhgk_options: threshold must be >= 0");
  ctx->qhgk_bandwidth = bandwidth;
  ctx->qhgk_threshold = std::isinf(threshold) ? 0.0 : threshold;
  return KALDO_OK;
}

static kaldo_status check_temperatures(kaldo_ctx ctx, const double* T, int32_t nT, kaldo_stats stats) {
  if (!T || nT < 1 || nT > KALDO_MAX_T) return fail(ctx, KALDO_EINVAL, "need 1 <= nT <= KALDO_MAX_T temperatures");
  if (stats != KALDO_QUANTUM && stats != KALDO_CLASSICAL) return fail(ctx, KALDO_EINVAL, "bad statistics");
  for (int t = 0; t < nT; ++t) {
    if (!std::isfinite(T[t]) || T[t] < 0.0 || (T[t] == 0.0 && stats == KALDO_CLASSICAL))
      return fail(ctx, KALDO_EINVAL, "temperatures must be finite, >= 0 (> 0 for classical)");
  }
  return KALDO_OK;
}

// the temperatures and statistics of an installed gamma; the gamma itself follows
static void install_gamma_state(kaldo_ctx ctx, const double* T, int32_t nT, kaldo_stats stats) {
  ctx->nT = nT;
  for (int t = 0; t < nT; ++t) ctx->T[t] = T[t];
  ctx->stats = stats;
  ctx->g_lo = 0;
  ctx->g_hi = ctx->nk;
}

kaldo_status kaldo_set_gamma(kaldo_ctx ctx, const double* T, int32_t nT, kaldo_stats stats, const double* gamma) {
  if (!ctx) return KALDO_EINVAL;
  ArenaScope arena_scope(&ctx->arena);
  ctx->err.clear();
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  if (!ctx->have_phonons) return fail(ctx, KALDO_ESTATE, "kaldo_set_gamma before kaldo_phonons");
  kaldo_status st;
  if ((st = check_temperatures(ctx, T, nT, stats)) != KALDO_OK) return st;
  const size_t count = (size_t)nT * ctx->nk * ctx->nm;
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  bool device = false;
  if (gamma) {
    if (hipPointerGetAttributes(&attr, gamma) == hipSuccess)
      device = attr.type == hipMemoryTypeDevice;
    else
      (void)hipGetLastError();
    if (!device) {
      for (size_t i = 0; i < count; ++i)
        if (!std::isfinite(gamma[i]) || gamma[i] < 0.0)
          return fail(ctx, KALDO_EINVAL, "kaldo_set_gamma: linewidths must be finite and >= 0");
    }
  }
  ctx->have_gamma = false;
  KALDO_HIP(ctx, ctx->d_gamma.ensure(count * sizeof(double)));
  if (gamma) {
    if ((st = copy_in(ctx, ctx->d_gamma.p, gamma, count * sizeof(double))) != KALDO_OK) return st;
  } else if ((st = fill_zero(ctx, ctx->d_gamma.p, count * sizeof(double))) != KALDO_OK) {
    return st;
  }
  install_gamma_state(ctx, T, nT, stats);
  ctx->gamma_external = true;
  ctx->have_gamma = true;
  return KALDO_OK;
}

kaldo_status kaldo_gamma_interpolate(kaldo_ctx ctx, const double* T, int32_t nT, kaldo_stats stats,
                                     const double* omega_src, const double* gamma_src, int64_t n_src,
                                     int32_t n_bins, double* gamma_out) {
  if (!ctx) return KALDO_EINVAL;
  ArenaScope arena_scope(&ctx->arena);
  ctx->err.clear();
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  if (!ctx->have_phonons) return fail(ctx, KALDO_ESTATE, "kaldo_gamma_interpolate before kaldo_phonons");
  kaldo_status st;
  if ((st = check_temperatures(ctx, T, nT, stats)) != KALDO_OK) return st;
  if (!omega_src || !gamma_src || n_src < 1 || n_src > ((int64_t)1 << 31))
    return fail(ctx, KALDO_EINVAL, "kaldo_gamma_interpolate: need source arrays of 1 .. 2^31 modes");
  if (n_bins < 1 || n_bins > 4096) return fail(ctx, KALDO_EINVAL, "kaldo_gamma_interpolate: n_bins in 1 .. 4096");
  ctx->have_gamma = false;
  const int keep_nT = ctx->nT;
  ctx->nT = nT;
  st = run_gamma_interpolate(ctx, omega_src, gamma_src, n_src, n_bins);
  if (st != KALDO_OK) {
    ctx->nT = keep_nT;
    return st;
  }
  install_gamma_state(ctx, T, nT, stats);
  ctx->gamma_external = true;
  ctx->have_gamma = true;
  return copy_out(ctx, gamma_out, ctx->d_gamma.p, (size_t)nT * ctx->nk * ctx->nm * sizeof(double));
}

kaldo_status kaldo_batch_add(kaldo_ctx ctx, const kaldo_structure* structure, const kaldo_fc2* fc2,
                             const kaldo_fc3* fc3, const int32_t grid[3], int32_t* handle) {
  if (!ctx) return KALDO_EINVAL;
  ArenaScope arena_scope(&ctx->arena);
  ctx->err.clear();
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  if (!structure || !fc2 || !fc3 || !grid || !handle)
    return fail(ctx, KALDO_EINVAL, "kaldo_batch_add: structure, fc2, fc3, grid and handle are required");
  if (ctx->batch.size() >= 4096) return fail(ctx, KALDO_EINVAL, "kaldo_batch_add: at most 4096 crystals");
  kaldo_ctx sub = nullptr;
  kaldo_status st = kaldo_create(&sub, ctx->device, ctx->stream);
  if (st != KALDO_OK) return fail(ctx, st, "kaldo_batch_add: cannot create a crystal context");
  sub->tune_owner = ctx;
  if ((st = kaldo_phonons(sub, structure, fc2, grid, nullptr, nullptr)) != KALDO_OK ||
      (st = load_fc3(sub, fc3)) != KALDO_OK) {
    const std::string msg = "kaldo_batch_add: " + sub->err;
    kaldo_destroy(sub);
    return fail(ctx, st, msg);
  }
  batch_drop_graph(ctx);
  ctx->batch.push_back(sub);
  *handle = (int32_t)ctx->batch.size() - 1;
  return KALDO_OK;
}

kaldo_status kaldo_batch_clear(kaldo_ctx ctx) {
  if (!ctx) return KALDO_EINVAL;
  ctx->err.clear();
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  KALDO_HIP(ctx, hipStreamSynchronize(ctx->stream));
  batch_release(ctx);
  return KALDO_OK;
}

// Capture the linewidths of every crystal of the batch into one graph: the
// many-branch crystals as one persistent kernel over a cost-sorted table of
// rounds (crystal, k, partner range), the few-branch crystals as their own
// per-chunk kernels.
static kaldo_status batch_capture(kaldo_ctx ctx, double sigma_thz, int precision) {
  kaldo_status st = KALDO_OK;
  // plan: size every buffer, build the static operands and record each
  // many-branch crystal's plan, outside the capture
  std::vector<kaldo_ctx> pers, eager;
  for (kaldo_ctx sub : ctx->batch) {
    sub->mode = kPlan;
    sub->cplan.valid = 0;
    sub->xy_budget = batch_xy_budget();
    sub->xy_shared = true;
    st = run_linewidths(sub, sigma_thz, precision);
    sub->xy_shared = false;
    sub->mode = kRun;
    if (st != KALDO_OK) return fail(ctx, st, "kaldo_batch_run (plan): " + sub->err);
    if (sub->cplan.valid && sub->cplan.precision == precision) pers.push_back(sub);
    else eager.push_back(sub);
  }
  if ((st = batch_persistent_prepare(ctx, pers, precision)) != KALDO_OK) return st;
  KALDO_HIP(ctx, hipStreamSynchronize(ctx->stream));
  KALDO_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  for (kaldo_ctx sub : eager) {
    sub->mode = kCapture;
    st = run_linewidths(sub, sigma_thz, precision);
    sub->mode = kRun;
    if (st != KALDO_OK) {
      st = fail(ctx, st, "kaldo_batch_run (capture): " + sub->err);
      break;
    }
  }
  if (st == KALDO_OK) st = batch_persistent_launch(ctx);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->stream, &graph);
  if (st == KALDO_OK && e != hipSuccess) st = hip_fail(ctx, e, "hipStreamEndCapture");
  if (st == KALDO_OK) {
    const hipError_t ei = hipGraphInstantiate(&ctx->batch_exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      ctx->batch_exec = nullptr;
      st = hip_fail(ctx, ei, "hipGraphInstantiate");
    }
  }
  if (graph) (void)hipGraphDestroy(graph);
  return st;
}

// Plan and capture the batch graph for these arguments unless it exists.
static kaldo_status batch_prepare(kaldo_ctx ctx, const double* T, int32_t nT, double sigma_thz, kaldo_stats stats,
                                  kaldo_precision precision) {
  if (ctx->batch.empty()) return fail(ctx, KALDO_ESTATE, "kaldo_batch_run: the batch is empty");
  kaldo_status st;
  if ((st = check_linewidth_args(ctx, T, nT, sigma_thz, KALDO_DELTA_GAUSS, stats, precision)) != KALDO_OK) return st;
  std::vector<double> key = {sigma_thz, (double)stats, (double)precision, (double)nT};
  for (int t = 0; t < nT; ++t) key.push_back(T[t]);
  for (kaldo_ctx sub : ctx->batch) {
    sub->nT = nT;
    for (int t = 0; t < nT; ++t) sub->T[t] = T[t];
    sub->stats = stats;
    sub->delta = KALDO_DELTA_GAUSS;
    sub->sigma_thz = sigma_thz;
    sub->have_gamma = false;
  }
  if (ctx->batch_exec && key != ctx->batch_key)
    return fail(ctx, KALDO_ESTATE,
                "kaldo_batch_run: the batch holds a graph captured with other arguments; re-capturing on the same "
                "context is not supported (kaldo_batch_clear, or a new context, for other arguments)");
  if (!ctx->batch_exec) {
    if ((st = batch_capture(ctx, sigma_thz, precision)) != KALDO_OK) return st;
    ctx->batch_key = key;
  }
  return KALDO_OK;
}

kaldo_status kaldo_batch_plan(kaldo_ctx ctx, const double* T, int32_t nT, double sigma_thz, kaldo_stats stats,
                              kaldo_precision precision) {
  if (!ctx) return KALDO_EINVAL;
  ArenaScope arena_scope(&ctx->arena);
  ctx->err.clear();
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  return batch_prepare(ctx, T, nT, sigma_thz, stats, precision);
}

kaldo_status kaldo_batch_run(kaldo_ctx ctx, const double* T, int32_t nT, double sigma_thz, kaldo_stats stats,
                             kaldo_precision precision, double* const* gamma_out) {
  if (!ctx) return KALDO_EINVAL;
  ArenaScope arena_scope(&ctx->arena);
  ctx->err.clear();
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  kaldo_status st;
  if ((st = batch_prepare(ctx, T, nT, sigma_thz, stats, precision)) != KALDO_OK) return st;
  prof_begin(ctx);
  KALDO_HIP(ctx, hipGraphLaunch(ctx->batch_exec, ctx->stream));
  prof_end(ctx, "batch_graph");
  if ((st = batch_persistent_check(ctx)) != KALDO_OK) return st;
  for (size_t i = 0; i < ctx->batch.size(); ++i) {
    kaldo_ctx sub = ctx->batch[i];
    sub->g_lo = k_lo(sub);
    sub->g_hi = k_hi(sub);
    sub->have_gamma = true;
    if (gamma_out && gamma_out[i]) {
      const size_t bytes = (size_t)nT * sub->nk * sub->nm * sizeof(double);
      if ((st = copy_out(ctx, gamma_out[i], sub->d_gamma.p, bytes)) != KALDO_OK) return st;
    }
  }
  return KALDO_OK;
}

kaldo_status kaldo_set_workspace(kaldo_ctx ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return KALDO_EINVAL;
  ctx->err.clear();
  if (ctx->have_phonons || ctx->have_fc3 || !ctx->batch.empty())
    return fail(ctx, KALDO_ESTATE, "kaldo_set_workspace: only on a context that holds no data yet");
  if (!dev_ptr || bytes == 0) {
    if (dev_ptr || bytes) return fail(ctx, KALDO_EINVAL, "kaldo_set_workspace: pointer and size go together");
    ctx->arena = Arena{};
    return KALDO_OK;
  }
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  if (hipPointerGetAttributes(&attr, dev_ptr) != hipSuccess || attr.type != hipMemoryTypeDevice ||
      attr.device != ctx->device) {
    (void)hipGetLastError();
    return fail(ctx, KALDO_EINVAL, "kaldo_set_workspace: not device memory of the context's device");
  }
  ctx->arena = Arena{static_cast<char*>(dev_ptr), bytes, 0, 0};
  return KALDO_OK;
}

kaldo_status kaldo_set_k_range(kaldo_ctx ctx, int32_t k_begin, int32_t k_end) {
  if (!ctx) return KALDO_EINVAL;
  ctx->err.clear();
  if (k_begin < 0 || k_end <= k_begin) return fail(ctx, KALDO_EINVAL, "kaldo_set_k_range: need 0 <= k_begin < k_end");
  ctx->k_begin = k_begin;
  ctx->k_end = k_end;
  return KALDO_OK;
}

kaldo_status kaldo_batch_set_k_range(kaldo_ctx ctx, int32_t handle, int32_t k_begin, int32_t k_end) {
  if (!ctx) return KALDO_EINVAL;
  ctx->err.clear();
  if (handle < 0 || handle >= (int32_t)ctx->batch.size())
    return fail(ctx, KALDO_EINVAL, "kaldo_batch_set_k_range: no such crystal");
  kaldo_ctx sub = ctx->batch[handle];
  if (k_begin < 0 || k_end <= k_begin || k_begin >= sub->nk)
    return fail(ctx, KALDO_EINVAL, "kaldo_batch_set_k_range: need 0 <= k_begin < min(k_end, N_k)");
  sub->k_begin = k_begin;
  sub->k_end = k_end;
  batch_drop_graph(ctx);  // the captured launches change
  return KALDO_OK;
}

kaldo_status kaldo_set_tuning(kaldo_ctx ctx, kaldo_tuning mode) {
  if (!ctx) return KALDO_EINVAL;
  if (mode != KALDO_TUNE_AUTO && mode != KALDO_TUNE_FIXED && !(mode >= KALDO_TUNE_SHAPE0 && mode < KALDO_TUNE_SHAPE0 + 16))
    return fail(ctx, KALDO_EINVAL, "kaldo_set_tuning: unknown mode");
  ctx->tuning = mode;
  ctx->tuned.clear();
  return KALDO_OK;
}

kaldo_status kaldo_profile_enable(kaldo_ctx ctx, int enable) {
  if (!ctx) return KALDO_EINVAL;
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  prof_clear(ctx);
  ctx->prof = enable != 0;
  if (ctx->prof) KALDO_HIP(ctx, ctx->d_prof_flops.ensure(sizeof(unsigned long long)));
  if (ctx->d_prof_flops.p) {
    KALDO_HIP(ctx, hipMemsetAsync(ctx->d_prof_flops.p, 0, sizeof(unsigned long long), ctx->stream));
    KALDO_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  return KALDO_OK;
}

kaldo_status kaldo_profile_read(kaldo_ctx ctx, const char* kernel, double* total_ms, int64_t* launches) {
  if (!ctx || !kernel) return KALDO_EINVAL;
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  KALDO_HIP(ctx, hipStreamSynchronize(ctx->stream));
  prof_collect(ctx);
  auto it = ctx->prof_tab.find(kernel);
  if (total_ms) *total_ms = it == ctx->prof_tab.end() ? 0.0 : it->second.total_ms;
  if (launches) *launches = it == ctx->prof_tab.end() ? 0 : it->second.launches;
  return KALDO_OK;
}

kaldo_status kaldo_profile_flops(kaldo_ctx ctx, double* executed, double* dense) {
  if (!ctx) return KALDO_EINVAL;
  KALDO_HIP(ctx, hipSetDevice(ctx->device));
  unsigned long long run = 0;
  if (ctx->d_prof_flops.p) {
    KALDO_HIP(ctx, hipMemcpyAsync(&run, ctx->d_prof_flops.p, sizeof(run), hipMemcpyDeviceToHost, ctx->stream));
    KALDO_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  if (executed) *executed = (double)run + ctx->prof_batch_executed;
  if (dense) *dense = ctx->prof_dense;
  return KALDO_OK;
}

}  // extern "C"
