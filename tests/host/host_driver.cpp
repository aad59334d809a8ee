// Random sequences of calls through the C ABI against the emulated runtime
// of fake_hip.cpp, built with the address sanitizer: the serving pool
// (admission, advances, polls, promotions, early and late retirement, arena
// reuse, pool re-creation), the single-solve API (create, step, solve, field
// access, checkpoints) and the allocation-free solve.  Every buffer handed to
// the library has exactly the size the ABI documents, so an access past it
// is reported.  Exits 0 when every sequence completes.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#include "../../include/maxflow.h"

extern "C" long long fake_hip_graph_launches();
extern "C" void fake_hip_stop_every(long long n);

namespace {

uint64_t g_rng = 88172645463325252ull;
uint64_t rnd() {
  g_rng ^= g_rng << 13;
  g_rng ^= g_rng >> 7;
  g_rng ^= g_rng << 17;
  return g_rng;
}
int rint_(int lo, int hi) { return lo + (int)(rnd() % (uint64_t)(hi - lo + 1)); }

void fail(const char* what) {
  std::fprintf(stderr, "host_driver: %s (last error: %s)\n", what, maxflow_last_error());
  std::exit(2);
}

struct Prob {
  mf_params p;
  long long npix;
  int L, ncap;
};

Prob random_problem(bool pool) {
  Prob r;
  std::memset(&r.p, 0, sizeof(r.p));
  mf_params& p = r.p;
  const bool d3 = rint_(0, 9) == 0;
  p.ndim = d3 ? 3 : 2;
  if (d3) {
    p.shape[0] = rint_(1, 20);
    p.shape[1] = rint_(1, 40);
    p.shape[2] = rint_(1, 90);
  } else {
    p.shape[0] = rint_(1, 150);
    p.shape[1] = rint_(1, 260);
  }
  const int nl[] = {2, 2, 3, 4, 8};
  const int n = nl[rint_(0, 4)];
  p.model = (n == 2 && rint_(0, 2) != 0) || d3 ? MF_TWO_LABEL : MF_POTTS;
  p.nlabels = n;
  if (p.model == MF_TWO_LABEL) p.nlabels = 2;
  p.method = pool ? rint_(0, 1) : rint_(0, 4);
  p.tv = rint_(0, 1);
  p.storage = rint_(0, 1);
  p.variant = pool ? MF_FUSED : rint_(0, 1);
  p.alpha = 0.3;
  p.max_iter = pool ? 10 * rint_(1, 30) : rint_(0, 200);
  p.tol = rint_(0, 3) ? 1e-4 : 0.0;
  p.check_every = 10;
  if (!pool) {
    if (p.method <= 1 && p.model == MF_TWO_LABEL && p.ndim == 2 && p.variant == MF_FUSED) p.depth = rint_(0, 2);
    if (p.method == MF_RPDRQ) p.gs_sweeps = rint_(1, 5);
    p.tile_rows = (const int[]){0, 8, 16, 32}[rint_(0, 3)];
    if (p.method == MF_RPADMM_EB && rint_(0, 3) == 0) {
      p.relax = 1.9;
      p.relax0 = 1.0;
      p.relax_ramp = rint_(1, 40);
    }
  }
  if (pool && p.storage == MF_BF16 && rint_(0, 1)) p.promote_iter = 10 * rint_(1, 10);
  r.npix = p.shape[0] * p.shape[1] * (d3 ? p.shape[2] : 1);
  r.L = p.model == MF_TWO_LABEL ? 1 : p.nlabels;
  r.ncap = p.model == MF_TWO_LABEL ? 2 : p.nlabels;
  return r;
}

float* make_caps(const Prob& r) {
  const size_t n = (size_t)r.ncap * r.npix;
  float* c = (float*)std::malloc(n * sizeof(float));
  for (size_t i = 0; i < n; i++) c[i] = (float)(rnd() % 1000) * 1e-3f;
  return c;
}

// ---------------------------------------------------------------- the pool
void pool_sequences(int rounds) {
  for (int round = 0; round < rounds; round++) {
    const int max_slots = rint_(1, 24), max_tiles = rint_(64, 3000);
    const size_t tb = mf_pool_table_bytes(max_slots, max_tiles);
    const size_t arena_bytes = tb + (size_t)rint_(1, 64) * (1u << 20);
    void* arena = std::aligned_alloc(256, (arena_bytes + 255) / 256 * 256);
    void* stream = (void*)0x1;
    mf_pool* P = nullptr;
    if (mf_pool_create(arena, arena_bytes, max_slots, max_tiles, 10, rint_(0, 2), stream, &P) != MF_OK)
      fail("pool create");
    std::map<int64_t, Prob> live;
    std::vector<int64_t> ids(max_slots);
    std::vector<mf_gap> gaps(max_slots);
    const int steps = rint_(50, 400);
    for (int it = 0; it < steps; it++) {
      // admissions until the pool refuses
      for (int a = rint_(0, 4); a > 0; a--) {
        Prob r = random_problem(true);
        float* caps = make_caps(r);
        int64_t sid = -1;
        const mf_status st = mf_pool_admit(P, &r.p, caps, &sid);
        std::free(caps);   // the pool copied it
        if (st == MF_OK) live[sid] = r;
        else if (st != MF_ENOMEM && st != MF_EINVAL) fail("admit");
      }
      if (live.empty()) continue;
      if (mf_pool_advance(P) != MF_OK) fail("advance");
      int nd = 0;
      const int cap = rint_(1, max_slots);
      if (mf_pool_poll(P, ids.data(), gaps.data(), cap, &nd) != MF_OK) fail("poll");
      if (nd > cap) fail("poll overflow");
      for (int i = 0; i < nd; i++) {
        auto f = live.find(ids[i]);
        if (f == live.end()) fail("poll reported an unknown solve");
        const Prob& r = f->second;
        float* u = rint_(0, 1) ? (float*)std::malloc(sizeof(float) * r.L * r.npix) : nullptr;
        int32_t* lab = rint_(0, 3) ? (int32_t*)std::malloc(sizeof(int32_t) * r.npix) : nullptr;
        if (mf_pool_retire(P, ids[i], u, lab) != MF_OK) fail("retire");
        std::free(u);
        std::free(lab);
        live.erase(f);
      }
      // now and then retire a solve before any poll reported it
      if (!live.empty() && rint_(0, 9) == 0) {
        auto f = live.begin();
        std::advance(f, rint_(0, (int)live.size() - 1));
        const Prob& r = f->second;
        float* u = (float*)std::malloc(sizeof(float) * r.L * r.npix);
        int32_t* lab = (int32_t*)std::malloc(sizeof(int32_t) * r.npix);
        if (mf_pool_retire(P, f->first, u, lab) != MF_OK) fail("early retire");
        std::free(u);
        std::free(lab);
        live.erase(f);
      }
      int32_t active = 0;
      size_t used = 0, largest = 0;
      if (mf_pool_stats(P, &active, &used, &largest) != MF_OK) fail("stats");
      if (active != (int32_t)live.size()) fail("active count");
      size_t want = 0;
      for (auto& kv : live) {
        mf_params q = kv.second.p;
        want += mf_pool_footprint(&q);
      }
      // promoted solves occupy their FP32 footprint
      if (used < want && mf_pool_promotions(P) == 0) fail("bytes in use");
    }
    for (auto& kv : live)
      if (mf_pool_retire(P, kv.first, nullptr, nullptr) != MF_OK) fail("final retire");
    int32_t active = -1;
    size_t used = 1, largest = 0;
    mf_pool_stats(P, &active, &used, &largest);
    if (active != 0 || used != 0) fail("pool not empty after retiring everything");
    if (largest != arena_bytes - tb) fail("free list did not coalesce back to one block");
    mf_pool_destroy(P);
    std::free(arena);
  }
}

// ---------------------------------------------------------------- single solves
void solver_sequences(int n) {
  for (int i = 0; i < n; i++) {
    Prob r = random_problem(false);
    const size_t ws = maxflow_workspace_bytes(&r.p);
    if (!ws) continue;   // invalid combination
    void* w = std::aligned_alloc(256, (ws + 255) / 256 * 256);
    float* caps = make_caps(r);
    mf_solver* s = nullptr;
    if (maxflow_create(&r.p, caps, w, ws, nullptr, &s) != MF_OK) fail("create");
    std::free(caps);
    fake_hip_stop_every(rint_(1, 9));
    maxflow_step(s, rint_(0, 37));
    mf_gap g;
    const mf_status st = maxflow_solve(s, &g);
    if (st != MF_OK && st != MF_ENOTCONV) fail("solve");
    if (g.iter != maxflow_iter(s)) fail("solve iterate");
    const long long np = r.npix;
    const int nq = r.L * r.p.ndim;
    const int planes[] = {r.L, nq, 1, r.L, nq, 1, r.L};
    for (int f = 0; f < (r.p.method == MF_RPDRQ ? 7 : 4); f++) {
      float* buf = (float*)std::malloc(sizeof(float) * planes[f] * np);
      if (maxflow_read_field(s, f, buf) != MF_OK) fail("read_field");
      if (f < 4 && maxflow_write_field(s, f, buf) != MF_OK) fail("write_field");
      std::free(buf);
    }
    int32_t* lab = (int32_t*)std::malloc(sizeof(int32_t) * np);
    if (maxflow_labels(s, lab) != MF_OK) fail("labels");
    std::free(lab);
    const size_t sb = maxflow_state_bytes(s);
    void* blob = std::malloc(sb);
    if (maxflow_export_state(s, blob) != MF_OK || maxflow_import_state(s, blob, rint_(0, 50)) != MF_OK)
      fail("checkpoint");
    std::free(blob);
    if (maxflow_gap(s, &g) != MF_OK) fail("gap");
    maxflow_destroy(s);
    std::free(w);
  }
}

void static_sequences(int n) {
  for (int i = 0; i < n; i++) {
    Prob r = random_problem(false);
    if (!maxflow_workspace_bytes(&r.p)) continue;
    float* caps = make_caps(r);
    float* u = (float*)std::malloc(sizeof(float) * r.L * r.npix);
    int32_t* lab = (int32_t*)std::malloc(sizeof(int32_t) * r.npix);
    fake_hip_stop_every(rint_(1, 9));
    mf_gap g;
    const mf_status st = maxflow_solve_static(&r.p, caps, rint_(0, 3) ? u : nullptr, rint_(0, 3) ? lab : nullptr,
                                              &g, nullptr);
    if (st != MF_OK && st != MF_ENOTCONV) fail("solve_static");
    std::free(caps);
    std::free(u);
    std::free(lab);
  }
}

}  // namespace

int main(int argc, char** argv) {
  const int scale = argc > 1 ? std::atoi(argv[1]) : 1;
  if (argc > 2) g_rng = std::strtoull(argv[2], nullptr, 10) | 1;
  pool_sequences(20 * scale);
  solver_sequences(300 * scale);
  static_sequences(100 * scale);
  std::printf("host_driver ok: %lld graph launches\n", fake_hip_graph_launches());
  return 0;
}
