// Kernel configuration and the autotuner.
//
// Every Wilson apply asks choose_cfg() which kernel to run: a configuration
// forced by the caller (tests, experiments), else the autotuner's measured
// best for the same (kind, lattice, nrhs, precision, layout), else the
// default.  lqcd_autotune() times the candidate kernels (one work item per
// site, time-streaming pencils with and without LDS-staged links, several
// tile shapes and segment counts, with and without non-temporal output
// stores) on the caller's buffers with HIP events and records the fastest.
// For the odd-even operator it also times the whole Schur apply, two hop
// passes against the fused kernel, and records that choice separately.
// The table can be saved to and loaded from a text file.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "batch.h"
#include "kernels.h"

namespace lq {

int fail(int code, const char* fmt, ...);
int check_lattice(const lqcd_lattice* lat);
int check_block(int nrhs, int layout, int prec);
int hip_status(hipError_t e, const char* what);

typedef std::tuple<int, int, int, int, int, int, int, int> tkey;  // kind, dims[4], nrhs, prec, layout

static std::mutex g_mu;
static std::map<tkey, std::pair<kcfg, double>> g_table;
static kcfg g_forced = {0, 0, 0, 0, 0, 0};
static const kcfg kDefault = {2, 0, 0, 0, 1, 0};

static tkey key_of(int kind, const lqcd_lattice* lat, int nrhs, int prec, int layout) {
  return tkey(kind, lat->dims[0], lat->dims[1], lat->dims[2], lat->dims[3], nrhs, prec, layout);
}

void set_variant(int v, const int* pencil) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_forced.variant = v;
  g_forced.ty = pencil ? pencil[0] : 0;
  g_forced.tz = pencil ? pencil[1] : 0;
  g_forced.nseg = pencil ? pencil[2] : 0;
  g_forced.nt = 0;
  g_forced.occ = 0;
}

static void set_forced(const kcfg& c) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_forced = c;
}

kcfg choose_cfg(int kind, const lqcd_lattice* lat, int nrhs, int prec, int layout) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_forced.variant != 0) return g_forced;
  auto it = g_table.find(key_of(kind, lat, nrhs, prec, layout));
  if (it != g_table.end()) return it->second.first;
  return kDefault;
}

bool tuned_time(int kind, const lqcd_lattice* lat, int nrhs, int prec, int layout, double* ms) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(key_of(kind, lat, nrhs, prec, layout));
  if (it == g_table.end() || !(it->second.second > 0.0)) return false;
  *ms = it->second.second;
  return true;
}

static const int kTiles[][2] = {{0, 0}, {2, 1}, {2, 2}, {4, 2}, {4, 4}, {8, 2}, {8, 4}};
// interior tiles of the fused Schur kernel (tile_y, tile_z)
static const int kSchurTiles[][2] = {{4, 4}, {4, 2}, {2, 4}, {2, 2}, {2, 1}, {1, 1}};

static bool tile_ok(const lqcd_lattice* lat, const int* t, int sg) {
  return !((t[0] && lat->dims[2] % t[0]) || (t[1] && lat->dims[1] % t[1]) || (sg && lat->dims[0] % sg));
}

// First pass: every kernel, tile, segment count and store kind, without a
// residency cap.
static std::vector<kcfg> candidates(const lqcd_lattice* lat, int layout, int prec, int nrhs, bool eo) {
  std::vector<kcfg> out;
  out.push_back({1, 0, 0, 0, 0, 0});
  for (int nt = 0; nt <= 1; ++nt)
    for (auto& t : kTiles)
      for (int sg : {0, 1, 2}) {
        if (!tile_ok(lat, t, sg)) continue;
        out.push_back({2, t[0], t[1], sg, nt, 0});
        if (layout != LQCD_RHS_OUTER && t[0] == 0 && sg == 0) out.push_back({3, 0, 0, 0, nt, 0});
        if (nr_supported(prec, layout, nrhs)) out.push_back({4, t[0], t[1], sg, nt, 0});
        if (!eo && dma_supported(prec, layout, nrhs)) out.push_back({5, t[0], t[1], sg, nt, 0});
        if (bc_supported(layout, nrhs)) {
          out.push_back({6, t[0], t[1], sg, nt, 0});
          out.push_back({7, t[0], t[1], sg, nt, 0});
        }
      }
  return out;
}

// Second pass: every pencil kernel again with capped residency (1 or 2
// workgroups per compute unit), so that the columns one XCD works on at a
// time stay few enough for its L2 to serve their spatial neighbours; with
// one wavefront per SIMD the kernels are latency-bound on L2 misses rather
// than short of wavefronts.  Keeps the first pass's store kind.
static std::vector<kcfg> capped_candidates(const lqcd_lattice* lat, int layout, int prec, int nrhs, const kcfg& w) {
  std::vector<kcfg> out;
  for (int occ = 1; occ <= 2; ++occ)
    for (auto& t : kTiles)
      for (int sg : {1, 2}) {
        if (!tile_ok(lat, t, sg)) continue;
        out.push_back({2, t[0], t[1], sg, w.nt, occ});
        if (layout != LQCD_RHS_OUTER) out.push_back({3, t[0], t[1], sg, w.nt, occ});
        if (nr_supported(prec, layout, nrhs)) out.push_back({4, t[0], t[1], sg, w.nt, occ});
        if (bc_supported(layout, nrhs)) {
          out.push_back({6, t[0], t[1], sg, w.nt, occ});
          out.push_back({7, t[0], t[1], sg, w.nt, occ});
        }
      }
  return out;
}

}  // namespace lq

using namespace lq;

extern "C" {

int lqcd_set_kernel_variant(int variant, const int32_t* pencil) {
  if (variant < 0 || variant > 8) return fail(LQCD_ERR_ARG, "unknown kernel variant %d", variant);
  int p[3] = {0, 0, 0};
  if (pencil)
    for (int i = 0; i < 3; ++i) {
      if (pencil[i] < 0) return fail(LQCD_ERR_ARG, "negative pencil parameter");
      p[i] = pencil[i];
    }
  set_variant(variant, pencil ? p : nullptr);
  return LQCD_OK;
}

int lqcd_set_kernel_config(const lqcd_kernel_config* c) {
  if (!c) {
    set_forced(kcfg{0, 0, 0, 0, 0, 0});
    return LQCD_OK;
  }
  if (c->variant < 0 || c->variant > 8) return fail(LQCD_ERR_ARG, "unknown kernel variant %d", c->variant);
  if (c->tile_y < 0 || c->tile_z < 0 || c->segments < 0 || c->wg_per_cu < 0 || c->wg_per_cu > 8)
    return fail(LQCD_ERR_ARG, "kernel parameter out of range");
  set_forced(kcfg{c->variant, c->tile_y, c->tile_z, c->segments, c->nontemporal ? 1 : 0, c->wg_per_cu});
  return LQCD_OK;
}

int lqcd_autotune(const lqcd_lattice* lat, const void* U, const void* psi, void* eta, int nrhs, int prec,
                  int layout, int eo, int reps, lqcd_kernel_config* best, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if ((rc = check_block(nrhs, layout, prec))) return rc;
  if (!U || !psi || !eta) return fail(LQCD_ERR_ARG, "lqcd_autotune: null array pointer");
  if (reps < 1) reps = 3;
  hipStream_t s = (hipStream_t)stream;
  const int kind = eo ? KIND_EO : KIND_FULL;
  kcfg saved;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    saved = g_forced;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(LQCD_ERR_HIP, "lqcd_autotune: event creation failed");
  double best_ms = 1e300;
  kcfg best_c = kDefault;
  // one hop pass of the Schur operator (the kernel a Schur apply runs twice)
  std::function<hipError_t()> run = [&]() -> hipError_t {
    if (eo) return wilson_eo(lat, U, psi, nullptr, eta, 1, nrhs, 0.0, 1.0, layout, prec, false, nullptr, s);
    return wilson_full(lat, U, psi, eta, nrhs, 3.95, -0.5, layout, prec, false, s);
  };
  auto time_all = [&](const std::vector<kcfg>& cands) -> int {
    for (const kcfg& c : cands) {
      set_forced(c);
      hipError_t e = run();  // warm-up
      if (e != hipSuccess && c.occ > 0) {  // launch refused: residency cap not expressible on this device
        (void)hipGetLastError();
        continue;
      }
      if (e != hipSuccess) return hip_status(e, "lqcd_autotune: candidate launch");
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps; ++r) (void)run();
      (void)hipEventRecord(e1, s);
      if ((e = hipEventSynchronize(e1)) != hipSuccess) return hip_status(e, "lqcd_autotune: timing");
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double per = ms / reps;
      if (per < best_ms) {
        best_ms = per;
        best_c = c;
      }
    }
    return LQCD_OK;
  };
  int err = time_all(candidates(lat, layout, prec, nrhs, eo != 0));
  if (!err) err = time_all(capped_candidates(lat, layout, prec, nrhs, best_c));
  const kcfg hop_c = best_c;
  const double hop_ms = best_ms;
  // odd-even: the whole Schur apply, two hop passes with the configuration
  // just chosen against the fused kernel's candidates
  if (!err && eo) {
    const size_t V = (size_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
    const size_t esz = prec == LQCD_F64 ? 16 : prec == LQCD_F32 ? 8 : 4;
    void* tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, V / 2 * 12 * (size_t)nrhs * esz);
    if (e != hipSuccess) {
      err = hip_status(e, "lqcd_autotune: odd temporary");
    } else {
      run = [&]() -> hipError_t {
        return schur_apply(lat, U, psi, eta, tmp, nrhs, 4.0, layout, prec, false, nullptr, s);
      };
      best_ms = 1e300;
      err = time_all({hop_c});
      std::vector<kcfg> fused;
      for (auto& t : kSchurTiles)
        for (int occ = 1; occ <= 2; ++occ)
          for (int nt = 0; nt <= 1; ++nt) {
            const kcfg c{8, t[0], t[1], 0, nt, occ};
            if (schur_fused_supported(lat, nrhs, prec, c)) fused.push_back(c);
          }
      if (!err) err = time_all(fused);
      (void)hipFree(tmp);
      if (!err) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table[key_of(KIND_SCHUR, lat, nrhs, prec, layout)] = std::make_pair(best_c, best_ms);
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  set_forced(saved);
  if (err) return err;
  best_c = hop_c;
  best_ms = hop_ms;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[key_of(kind, lat, nrhs, prec, layout)] = std::make_pair(best_c, best_ms);
  }
  if (best) {
    best->variant = best_c.variant;
    best->tile_y = best_c.ty;
    best->tile_z = best_c.tz;
    best->segments = best_c.nseg;
    best->nontemporal = best_c.nt;
    best->wg_per_cu = best_c.occ;
    best->ms = best_ms;
  }
  return LQCD_OK;
}

int lqcd_tune_save(const char* path) {
  if (!path) return fail(LQCD_ERR_ARG, "lqcd_tune_save: null path");
  FILE* f = fopen(path, "w");
  if (!f) return fail(LQCD_ERR_ARG, "lqcd_tune_save: cannot open %s", path);
  std::lock_guard<std::mutex> lk(g_mu);
  fprintf(f, "# kind N0 N1 N2 N3 nrhs prec layout : variant tile_y tile_z segments nontemporal wg_per_cu ms\n");
  for (auto& kv : g_table) {
    const tkey& k = kv.first;
    const kcfg& c = kv.second.first;
    fprintf(f, "%d %d %d %d %d %d %d %d : %d %d %d %d %d %d %.6f\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
            std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k), std::get<7>(k), c.variant, c.ty, c.tz,
            c.nseg, c.nt, c.occ, kv.second.second);
  }
  fclose(f);
  return LQCD_OK;
}

int lqcd_tune_load(const char* path) {
  if (!path) return fail(LQCD_ERR_ARG, "lqcd_tune_load: null path");
  FILE* f = fopen(path, "r");
  if (!f) return fail(LQCD_ERR_ARG, "lqcd_tune_load: cannot open %s", path);
  char line[512];
  int n = 0;
  std::lock_guard<std::mutex> lk(g_mu);
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    // "k0 .. k7 : v ty tz seg nt [wg_per_cu] ms" (older lines lack wg_per_cu)
    int k[8], c[6] = {0, 0, 0, 0, 0, 0};
    double val[8];
    const char* colon = strchr(line, ':');
    if (!colon || sscanf(line, "%d %d %d %d %d %d %d %d", &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &k[6], &k[7]) != 8)
      continue;
    int nv = 0;
    const char* q = colon + 1;
    char* end = nullptr;
    while (nv < 8) {
      val[nv] = strtod(q, &end);
      if (end == q) break;
      ++nv;
      q = end;
    }
    if (nv != 6 && nv != 7) continue;
    bool ints = true;
    for (int i = 0; i < nv - 1; ++i) {
      if (!(val[i] > -1e6 && val[i] < 1e6)) {
        ints = false;
        break;
      }
      c[i] = (int)val[i];
      if ((double)c[i] != val[i]) ints = false;
    }
    if (!ints) continue;
    if (nv == 6) c[5] = 0;
    const double ms = val[nv - 1];
    if (c[0] < 1 || c[0] > 8 || c[5] < 0 || c[5] > 8) continue;
    g_table[tkey(k[0], k[1], k[2], k[3], k[4], k[5], k[6], k[7])] =
        std::make_pair(kcfg{c[0], c[1], c[2], c[3], c[4], c[5]}, ms);
    ++n;
  }
  fclose(f);
  return n;
}

void lqcd_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
}

// ---------------------------------------------------- persistent batch grid
int lqcd_autotune_batch(int nprob, const lqcd_problem* probs, int prec, int reps, int* best_kernel, int* best_grid,
                        void* stream) {
  if (reps < 1) reps = 3;
  int dev = 0, ncu = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(LQCD_ERR_HIP, "lqcd_autotune_batch: event creation failed");
  double best_ms = 1e300;
  int best = 0, bestk = 0, besto = 0;
  int rc = LQCD_OK;
  for (int kind : {1, 2}) {
    if ((rc = lqcd_set_batch_kernel(kind))) break;
    for (int occ : {0, 1, 2}) {  // residency cap of the pencil launch
      if (kind == 1 && occ) continue;
      set_batch_occupancy(occ);
      for (int per_cu : {0, 1, 2, 4, 8, 16}) {  // 0: default grid of the kernel
        if ((rc = lqcd_set_batch_grid(per_cu * ncu))) break;
        if ((rc = dirac_apply_batch(nprob, probs, prec, 0, stream))) break;
        (void)hipEventRecord(e0, (hipStream_t)stream);
        for (int r = 0; r < reps; ++r) (void)dirac_apply_batch(nprob, probs, prec, 0, stream);
        (void)hipEventRecord(e1, (hipStream_t)stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms / reps < best_ms) {
          best_ms = ms / reps;
          best = per_cu * ncu;
          bestk = kind;
          besto = occ;
        }
      }
      if (rc) break;
    }
    if (rc) break;
  }
  set_batch_occupancy(besto);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  // the kernel choice applies to full-lattice batches; the solver's odd-even
  // passes keep the automatic choice
  (void)lqcd_set_batch_kernel(0);
  (void)lqcd_set_batch_grid(best);
  if (bestk == 1) (void)lqcd_set_batch_kernel(1);
  if (best_kernel) *best_kernel = bestk;
  if (best_grid) *best_grid = best;
  return LQCD_OK;
}

}  // extern "C"
