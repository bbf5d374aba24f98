// Grouped multi-problem ETD2RKds steps ("batch plans").
//
// Many independent problems of different grid sizes, dimensions, models and
// step sizes advance together: each phase of the step (stage 1, the d mode
// products of each Tucker operator, stage 2, ...) is ONE launch over all of
// them, driven by per-phase job tables that live in device memory.  The tables
// are built once per plan, so a whole step can be captured in a hipGraph and
// replayed.  Tile shapes of the grouped mode products are chosen per phase by
// timing the candidates on the plan's own data (cached per phase signature).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "adr.h"
#include "common.h"
#include "host_common.h"

using namespace adr;
using namespace adr::host;

namespace {

constexpr int kMaxMu = 3;

struct ModePhase {
  // one job table per tile configuration (tile offsets depend on the tile shape)
  TileJob* jobs[kNumTileCfgs] = {};
  LowpJob* ljobs = nullptr;
  bool lvec = true;              // all FP32 jobs allow vectorised loads
  int njobs = 0;
  long long ntiles[kNumTileCfgs] = {};
  long long ltiles = 0;
  bool kfast = false;
  TileCfg cfg = TileCfg::I128X128;
  std::string signature;
};

// Device memory of plan tables is pooled: destroying a plan returns its block
// here instead of calling hipFree (which waits for the whole device), so plans
// can be rebuilt while other work runs.  Blocks live until the process ends.
std::mutex g_pool_mu;
std::multimap<size_t, char*> g_pool;  // capacity -> free block
std::map<char*, size_t> g_cap;        // every block -> its capacity

char* pool_take(size_t bytes) {
  {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    auto it = g_pool.lower_bound(bytes);
    if (it != g_pool.end() && it->first <= 4 * bytes + 65536) {
      char* p = it->second;
      g_pool.erase(it);
      return p;
    }
  }
  // round up so that blocks are reusable by plans of similar size
  size_t cap = 65536;
  while (cap < bytes) cap *= 2;
  char* p = nullptr;
  if (hipMalloc(&p, cap) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(g_pool_mu);
  g_cap[p] = cap;
  return p;
}

void pool_give(char* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lock(g_pool_mu);
  g_pool.emplace(g_cap[p], p);
}

// autotune cache: phase signature -> chosen configuration
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;

void tune_cache_load() {
  static bool loaded = false;
  if (loaded) return;
  loaded = true;
  const char* path = std::getenv("ADR_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char key[4096];
  int val;
  while (std::fscanf(f, "%4095s %d", key, &val) == 2) g_tune[key] = val;
  std::fclose(f);
}

void tune_cache_store(const std::string& key, int val) {
  g_tune[key] = val;
  const char* path = std::getenv("ADR_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d\n", key.c_str(), val);
  std::fclose(f);
}

}  // namespace

struct adr_batch {
  int count = 0;
  int precision = ADR_F64;
  int d_max = 0;
  std::vector<adr_problem> probs;
  std::vector<Geometry> geoms;
  std::vector<Carve> carves;
  std::vector<double*> U, V;
  char* dev = nullptr;           // all device job tables
  StageJob* stage1 = nullptr;    // point-kernel jobs first, then tiled-kernel jobs
  int n_stage = 0;
  int n_stage1[2] = {0, 0};       // jobs per stage-1 variant (point, tile)
  long long stage1_blocks[2] = {0, 0};
  PointJob* stage2 = nullptr;
  PointJob* finalize = nullptr;  // reduced precision only
  long long point_blocks = 0;
  ModePhase mode[2][kMaxMu];     // [Tucker operator][mu]
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  bool autotuned = false;
  // one event per stream that adr_batch_run used, recorded after its last
  // enqueued step: destroy waits for them before the tables go back to the pool
  std::vector<std::pair<hipStream_t, hipEvent_t>> runs;
};

namespace {

hipError_t launch_mode_phase(const adr_batch& b, const ModePhase& m, hipStream_t s) {
  if (m.njobs == 0) return hipSuccess;
  if (b.precision == ADR_F64)
    return launch_mode_grouped_f64(m.cfg, m.kfast, m.jobs[(int)m.cfg], m.njobs,
                                   m.ntiles[(int)m.cfg], s);
  return launch_tgemm_lowp_grouped(b.precision, m.ljobs, m.njobs, m.ltiles, m.lvec, s);
}

// One ETD2RKds step of every problem of the plan (timed launch by launch when
// kernel timing is on and the stream is not being captured).
hipError_t batch_step(const adr_batch& b, hipStream_t s, bool capturing) {
  const bool lowp = b.precision != ADR_F64;
  auto run = [&](int kind, auto&& f) { return capturing ? f() : timed(kind, s, f); };
  hipError_t e = hipSuccess;
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    if (b.n_stage1[k] == 0) continue;
    const StageJob* jobs = b.stage1 + (k == 0 ? 0 : b.n_stage1[0]);
    const int kind = k == 0 ? kStage1Point : kStage1Tile;
    e = run(kKindStage, [&] {
      return launch_stage1_grouped(jobs, b.n_stage1[k], b.stage1_blocks[k], kind, lowp ? 1 : 0, s);
    });
  }
  for (int mu = 0; mu < b.d_max && e == hipSuccess; ++mu)
    e = run(kKindMode, [&] { return launch_mode_phase(b, b.mode[0][mu], s); });
  if (e == hipSuccess)
    e = run(kKindStage, [&] {
      return launch_pointwise_grouped(b.stage2, b.n_stage, b.point_blocks, lowp ? 1 : 0, s);
    });
  for (int mu = 0; mu < b.d_max && e == hipSuccess; ++mu)
    e = run(kKindMode, [&] { return launch_mode_phase(b, b.mode[1][mu], s); });
  if (lowp && e == hipSuccess)
    e = run(kKindStage, [&] {
      return launch_pointwise_grouped(b.finalize, b.n_stage, b.point_blocks, 1, s);
    });
  return e;
}

// Buffers of the Tucker chain of problem i, component c, for Tucker operator t:
// input, ping (T) and pong (R, the clobbered input), output and addend.
struct Chain {
  const void* in;
  void* t1;
  void* t2;
  void* out;
  const double* Y;
};

Chain chain_of(const adr_batch& b, int i, int c, int t) {
  const Carve& cv = b.carves[i];
  const int d = b.geoms[i].d;
  const bool lowp = b.precision != ADR_F64;
  Chain ch;
  ch.in = cv.R[c];
  ch.t1 = cv.T[c];
  ch.t2 = cv.R[c];
  if (!lowp) {
    ch.out = t == 0 ? (c == 0 ? cv.U2 : cv.V2) : (c == 0 ? b.U[i] : b.V[i]);
    ch.Y = t == 0 ? (c == 0 ? b.U[i] : b.V[i]) : (c == 0 ? cv.U2 : cv.V2);
  } else {
    ch.out = t == 0 ? static_cast<void*>(cv.D[c]) : (d == 2 ? cv.R[c] : cv.T[c]);
    ch.Y = nullptr;
  }
  return ch;
}

// Autotune key of a mode-product phase: precision, direction, largest n_mu,
// number of products, and the phase's multiply-adds rounded to a power of two.
// Plans with similar mixes (as a serving loop builds them) share a decision.
std::string phase_signature(const adr_batch& b, int mu) {
  int nmax = 0, jobs = 0;
  double macs = 0.0;
  for (int i = 0; i < b.count; ++i) {
    const Geometry& g = b.geoms[i];
    if (mu >= g.d) continue;
    nmax = std::max(nmax, g.n[mu]);
    jobs += 2;
    macs += 2.0 * (double)g.n[mu] * (double)g.N;
  }
  std::ostringstream os;
  os << "p" << b.precision << "_mu" << mu << "_n" << nmax << "_j" << jobs << "_m"
     << (macs > 0 ? (int)std::lround(std::log2(macs)) : 0);
  return os.str();
}

int validate(int count, const adr_problem* probs, double* const* U, double* const* V,
             void* const* work, const size_t* work_bytes, std::vector<Geometry>& geoms) {
  if (count < 1 || count > 4096 || !probs || !U || !V || !work || !work_bytes) return ADR_EINVAL;
  geoms.resize(count);
  for (int i = 0; i < count; ++i) {
    const adr_problem* p = &probs[i];
    const int st = check_problem(p, geoms[i]);
    if (st != ADR_OK) return st;
    if (p->scheme != ADR_ETD2RKDS) return ADR_ENOTSUP;
    if (p->precision != probs[0].precision || (p->precision != ADR_F64 && p->precision != ADR_F32)) return ADR_ENOTSUP;
    for (int c = 0; c < 2; ++c)
      for (int mu = 0; mu < p->d; ++mu)
        if (!p->band[c][mu]) return ADR_ENOTSUP;
    if (!U[i] || !V[i] || !work[i]) return ADR_EINVAL;
    if (reinterpret_cast<uintptr_t>(work[i]) % kAlign != 0) return ADR_EINVAL;
    if (work_bytes[i] < carve(p, geoms[i], nullptr).bytes) return ADR_ENOMEM;
  }
  return ADR_OK;
}

hipError_t time_phase(const adr_batch& b, const ModePhase& m, hipStream_t s, float& ms) {
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch_mode_phase(b, m, s);  // warm
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int r = 0; r < 2 && e == hipSuccess; ++r) e = launch_mode_phase(b, m, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

// Without autotuning: 128x128 tiles when the phase has work for several of them
// per CU, else 64x64 (four times the tiles, and four workgroups per CU), which
// the tuner picks for mixes of grids up to 512^2.
TileCfg default_cfg(const adr_batch& b, int mu) {
  long long tiles128 = 0;
  for (int i = 0; i < b.count; ++i) {
    const Geometry& g = b.geoms[i];
    if (mu >= g.d) continue;
    const long long X = g.N / g.n[mu];
    tiles128 += 2LL * ((g.n[mu] + 127) / 128) * ((X + 127) / 128);
  }
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  return tiles128 >= 8LL * cus ? TileCfg::I128X128 : TileCfg::I64X64;
}

void destroy(adr_batch* b) {
  if (!b) return;
  // kernels of runs still queued read the job tables and may replay the graph:
  // wait for them (a host wait on this plan's work only) before releasing either
  for (auto& r : b->runs) {
    (void)hipEventSynchronize(r.second);
    (void)hipEventDestroy(r.second);
  }
  b->runs.clear();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  pool_give(b->dev);
  delete b;
}

}  // namespace

extern "C" {

int adr_batch_create(int count, const adr_problem* problems, double* const* U, double* const* V,
                     void* const* work, const size_t* work_bytes, int flags, void* stream,
                     adr_batch** plan) {
  if (!plan) return ADR_EINVAL;
  *plan = nullptr;
  const int forced = (flags >> 8) & 0xff;   // 0: none, else tile configuration + 1
  if ((flags & ~(ADR_BATCH_AUTOTUNE | ADR_BATCH_GRAPH | ADR_BATCH_PREPARED | (0xff << 8))) ||
      forced > kNumTileCfgs)
    return ADR_EINVAL;
  std::vector<Geometry> geoms;
  int st = validate(count, problems, U, V, work, work_bytes, geoms);
  if (st != ADR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  adr_batch* b = new adr_batch();
  b->count = count;
  b->precision = problems[0].precision;
  b->probs.assign(problems, problems + count);
  b->geoms = geoms;
  b->U.assign(U, U + count);
  b->V.assign(V, V + count);
  for (int i = 0; i < count; ++i) {
    b->carves.push_back(carve(&b->probs[i], geoms[i], static_cast<char*>(work[i])));
    b->d_max = std::max(b->d_max, geoms[i].d);
  }
  const bool lowp = b->precision != ADR_F64;

  // ---- host job tables
  std::vector<StageJob> s1(count);
  std::vector<PointJob> s2(count), fin(count);
  long long pblocks = 0;
  for (int i = 0; i < count; ++i) {
    const adr_problem* p = &b->probs[i];
    const Geometry& g = geoms[i];
    StageJob& j = s1[i];
    j.g.d = g.d;
    j.g.N = g.N;
    for (int mu = 0; mu < 3; ++mu) j.g.n[mu] = g.n[mu];
    for (int c = 0; c < 2; ++c)
      for (int mu = 0; mu < 3; ++mu) j.g.band[c][mu] = mu < g.d ? p->band[c][mu] : nullptr;
    j.r = reaction_of(p);
    j.U = U[i];
    j.V = V[i];
    j.R[0] = b->carves[i].R[0];
    j.R[1] = b->carves[i].R[1];
    int gz;
    const int nb = stage1_plan(j.g, j.kind, j.gx, j.gy, gz);
    j.block_begin = nb;   // block count for now; offsets once the jobs are ordered
    PointJob& q = s2[i];
    q = PointJob{};
    q.kind = lowp ? 1 : 0;
    q.r = j.r;
    q.N = g.N;
    q.U = U[i];
    q.V = V[i];
    q.A = lowp ? static_cast<const void*>(b->carves[i].D[0]) : b->carves[i].U2;
    q.B = lowp ? static_cast<const void*>(b->carves[i].D[1]) : b->carves[i].V2;
    q.R[0] = b->carves[i].R[0];
    q.R[1] = b->carves[i].R[1];
    q.block_begin = pblocks;
    PointJob& f = fin[i];
    f = PointJob{};
    f.kind = 2;
    f.N = g.N;
    f.U = U[i];
    f.V = V[i];
    f.A = b->carves[i].D[0];
    f.B = b->carves[i].D[1];
    f.C2 = chain_of(*b, i, 0, 1).out;
    f.D2 = chain_of(*b, i, 1, 1).out;
    f.block_begin = pblocks;
    pblocks += (g.N + 255) / 256;
  }
  b->n_stage = count;
  b->point_blocks = pblocks;
  // stage-1 table: point-kernel jobs, then tiled-kernel jobs, offsets per segment
  std::stable_sort(s1.begin(), s1.end(),
                   [](const StageJob& x, const StageJob& y) { return x.kind < y.kind; });
  for (StageJob& j : s1) {
    const int k = j.kind == kStage1Tile ? 1 : 0;
    const long long nb = j.block_begin;
    j.block_begin = b->stage1_blocks[k];
    b->stage1_blocks[k] += nb;
    ++b->n_stage1[k];
  }

  // mode phases: for Tucker t and direction mu, two jobs (u, v) per problem with d > mu
  std::vector<TileJob> tj[2][kMaxMu][kNumTileCfgs];
  std::vector<LowpJob> lj[2][kMaxMu];
  for (int t = 0; t < 2; ++t)
    for (int mu = 0; mu < b->d_max; ++mu) {
      ModePhase& m = b->mode[t][mu];
      m.kfast = (mu == 0);
      m.signature = phase_signature(*b, mu);
      for (int i = 0; i < count; ++i) {
        const Geometry& g = geoms[i];
        if (mu >= g.d) continue;
        const adr_problem* p = &b->probs[i];
        const bool last = (mu == g.d - 1);
        long long L, R;
        mode_geometry(g, mu, L, R);
        const double alpha = t == 0 ? p->tau : std::ldexp(p->tau, g.d - 1);
        const Carve& cv = b->carves[i];
        for (int c = 0; c < 2; ++c) {
          const Chain ch = chain_of(*b, i, c, t);
          const void* W = (mu == 0) ? ch.in : ((mu % 2 == 1) ? ch.t1 : ch.t2);
          void* out = last ? ch.out : ((mu % 2 == 0) ? ch.t1 : ch.t2);
          if (!lowp) {
            for (int k = 0; k < kNumTileCfgs; ++k) {
              int BI, BX;
              tile_cfg_dims((TileCfg)k, BI, BX);
              TileJob j{};
              j.W = static_cast<const double*>(W);
              j.M = p->phi[c][t + 1][mu];
              j.out = static_cast<double*>(out);
              j.Y = last ? ch.Y : nullptr;
              j.Z = nullptr;
              j.alpha = last ? alpha : 1.0;
              j.beta = last ? 1.0 : 0.0;
              j.gamma = 0.0;
              j.L = L;
              j.X = L * R;
              j.n = g.n[mu];
              j.n_itiles = (g.n[mu] + BI - 1) / BI;
              j.tile_begin = m.ntiles[k];
              m.ntiles[k] += (long long)j.n_itiles * ((j.X + BX - 1) / BX);
              tj[t][mu][k].push_back(j);
            }
          } else {
            LowpJob j{};
            j.W = static_cast<const float*>(W);
            j.M = cv.phi32[c][t + 1][mu];
            j.out = out;
            j.alpha = last ? alpha : 1.0;
            j.n = g.n[mu];
            j.X = g.N / g.n[mu];
            j.out_f64 = 0;
            j.n_itiles = (g.n[mu] + 127) / 128;
            j.tile_begin = m.ltiles;
            m.ltiles += (long long)j.n_itiles * ((j.X + 127) / 128);
            m.lvec = m.lvec && j.n % 4 == 0 && reinterpret_cast<uintptr_t>(j.W) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(j.M) % 16 == 0;
            lj[t][mu].push_back(j);
          }
        }
      }
      // largest contractions first (work per tile grows with n): the long tiles
      // start early and the short ones fill the end of the launch.  Each tile's
      // arithmetic does not depend on its position, so results are unchanged.
      for (int k = 0; k < kNumTileCfgs; ++k) {
        auto& v = tj[t][mu][k];
        std::stable_sort(v.begin(), v.end(), [](const TileJob& x, const TileJob& y) { return x.n > y.n; });
        long long off = 0;
        for (TileJob& j : v) {
          int BI, BX;
          tile_cfg_dims((TileCfg)k, BI, BX);
          j.tile_begin = off;
          off += (long long)j.n_itiles * ((j.X + BX - 1) / BX);
        }
      }
      {
        auto& v = lj[t][mu];
        std::stable_sort(v.begin(), v.end(), [](const LowpJob& x, const LowpJob& y) { return x.n > y.n; });
        long long off = 0;
        for (LowpJob& j : v) {
          j.tile_begin = off;
          off += (long long)j.n_itiles * ((j.X + 127) / 128);
        }
      }
      m.njobs = lowp ? (int)lj[t][mu].size() : (int)tj[t][mu][0].size();
      m.cfg = forced ? (TileCfg)(forced - 1) : default_cfg(*b, mu);
    }

  // every buffer a launch will touch must exist
  for (int t = 0; t < 2; ++t)
    for (int mu = 0; mu < b->d_max; ++mu) {
      for (const TileJob& j : tj[t][mu][0])
        if (!j.W || !j.M || !j.out) { destroy(b); return ADR_EINVAL; }
      for (const LowpJob& j : lj[t][mu])
        if (!j.W || !j.M || !j.out) { destroy(b); return ADR_EINVAL; }
    }
  for (int i = 0; i < count; ++i) {
    if (!s1[i].R[0] || !s1[i].R[1] || !s2[i].A || !s2[i].B) { destroy(b); return ADR_EINVAL; }
    if (lowp && (!fin[i].A || !fin[i].B || !fin[i].C2 || !fin[i].D2)) { destroy(b); return ADR_EINVAL; }
  }

  // ---- device copies of the tables (one allocation)
  size_t bytes = 0;
  auto reserve = [&](size_t sz) { size_t off = bytes; bytes += align_up(sz); return off; };
  const size_t o_s1 = reserve(sizeof(StageJob) * count);
  const size_t o_s2 = reserve(sizeof(PointJob) * count);
  const size_t o_fin = reserve(sizeof(PointJob) * count);
  size_t o_mode[2][kMaxMu][kNumTileCfgs] = {};
  size_t o_low[2][kMaxMu] = {};
  for (int t = 0; t < 2; ++t)
    for (int mu = 0; mu < b->d_max; ++mu) {
      for (int k = 0; k < kNumTileCfgs; ++k) o_mode[t][mu][k] = reserve(sizeof(TileJob) * tj[t][mu][k].size() + 1);
      o_low[t][mu] = reserve(sizeof(LowpJob) * lj[t][mu].size() + 1);
    }
  b->dev = pool_take(bytes);
  if (!b->dev) {
    destroy(b);
    return ADR_ENOMEM;
  }
  std::vector<char> host(bytes, 0);
  std::memcpy(host.data() + o_s1, s1.data(), sizeof(StageJob) * count);
  std::memcpy(host.data() + o_s2, s2.data(), sizeof(PointJob) * count);
  std::memcpy(host.data() + o_fin, fin.data(), sizeof(PointJob) * count);
  b->stage1 = reinterpret_cast<StageJob*>(b->dev + o_s1);
  b->stage2 = reinterpret_cast<PointJob*>(b->dev + o_s2);
  b->finalize = reinterpret_cast<PointJob*>(b->dev + o_fin);
  for (int t = 0; t < 2; ++t)
    for (int mu = 0; mu < b->d_max; ++mu) {
      ModePhase& m = b->mode[t][mu];
      for (int k = 0; k < kNumTileCfgs; ++k) {
        if (!tj[t][mu][k].empty())
          std::memcpy(host.data() + o_mode[t][mu][k], tj[t][mu][k].data(), sizeof(TileJob) * tj[t][mu][k].size());
        m.jobs[k] = reinterpret_cast<TileJob*>(b->dev + o_mode[t][mu][k]);
      }
      if (!lj[t][mu].empty())
        std::memcpy(host.data() + o_low[t][mu], lj[t][mu].data(), sizeof(LowpJob) * lj[t][mu].size());
      m.ljobs = reinterpret_cast<LowpJob*>(b->dev + o_low[t][mu]);
    }
  if (hipMemcpyAsync(b->dev, host.data(), bytes, hipMemcpyHostToDevice, s) != hipSuccess) {
    destroy(b);
    return ADR_EDEVICE;
  }
  // reduced precision: FP32 copies of the small matrices (they do not change)
  for (int i = 0; i < count && lowp && !(flags & ADR_BATCH_PREPARED); ++i)
    if (prepare_lowp(&b->probs[i], geoms[i], b->carves[i], s) != hipSuccess) {
      destroy(b);
      return ADR_EDEVICE;
    }

  // ---- autotune the tile shape of every FP64 mode phase (timed on phase 0's
  // buffers, whose outputs are workspace; phase 1 has the same shapes)
  if ((flags & ADR_BATCH_AUTOTUNE) && !lowp && !forced) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_cache_load();
    for (int mu = 0; mu < b->d_max; ++mu) {
      ModePhase& m0 = b->mode[0][mu];
      auto it = g_tune.find(m0.signature);
      int best = (int)m0.cfg;
      if (it != g_tune.end()) {
        best = it->second;
      } else {
        float best_ms = 1e30f;
        for (int k = 0; k < kNumTileCfgs; ++k) {
          m0.cfg = (TileCfg)k;
          float ms = 0.f;
          if (time_phase(*b, m0, s, ms) != hipSuccess) {
            destroy(b);
            return ADR_EDEVICE;
          }
          if (ms < best_ms) {
            best_ms = ms;
            best = k;
          }
        }
        tune_cache_store(m0.signature, best);
      }
      m0.cfg = (TileCfg)best;
      b->mode[1][mu].cfg = (TileCfg)best;
    }
    b->autotuned = true;
  }

  // the tables (from a host vector) and the matrix copies are complete on return
  if (hipStreamSynchronize(s) != hipSuccess) {
    destroy(b);
    return ADR_EDEVICE;
  }

  // ---- capture one step in a graph
  if (flags & ADR_BATCH_GRAPH) {
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
      destroy(b);
      return ADR_EDEVICE;
    }
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const hipError_t e1 = batch_step(*b, b->cap, true);
      e = hipStreamEndCapture(b->cap, &b->graph);
      if (e1 != hipSuccess) e = e1;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      destroy(b);
      return ADR_EDEVICE;
    }
  }
  *plan = b;
  return ADR_OK;
}

int adr_batch_run(adr_batch* plan, int nsteps, void* stream) {
  if (!plan || nsteps < 0) return ADR_EINVAL;
  if (nsteps == 0) return ADR_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t* done = nullptr;
  for (auto& r : plan->runs)
    if (r.first == s) done = &r.second;
  if (!done) {
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return ADR_EDEVICE;
    plan->runs.emplace_back(s, ev);
    done = &plan->runs.back().second;
  }
  for (int it = 0; it < nsteps; ++it) {
    const hipError_t e = plan->exec ? hipGraphLaunch(plan->exec, s) : batch_step(*plan, s, false);
    if (e != hipSuccess) {
      (void)hipEventRecord(*done, s);
      return ADR_EDEVICE;
    }
  }
  return hipEventRecord(*done, s) == hipSuccess ? ADR_OK : ADR_EDEVICE;
}

int adr_batch_info(const adr_batch* plan, int* tile_cfg, int max_phases, int* graph_captured) {
  if (!plan || (max_phases > 0 && !tile_cfg)) return ADR_EINVAL;
  for (int mu = 0; mu < max_phases; ++mu)
    tile_cfg[mu] = (mu < plan->d_max && plan->precision == ADR_F64) ? (int)plan->mode[0][mu].cfg : -1;
  if (graph_captured) *graph_captured = plan->exec ? 1 : 0;
  return ADR_OK;
}

int adr_batch_destroy(adr_batch* plan) {
  if (!plan) return ADR_EINVAL;
  destroy(plan);
  return ADR_OK;
}

}  // extern "C"
