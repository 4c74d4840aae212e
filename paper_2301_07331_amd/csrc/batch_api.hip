// batch_api.hip -- the batched form: many independent jobs in one pass
// (job plan, device tables, autotuned zone-height factor, graph capture).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "host.hpp"
#include "tune_cache.hpp"

namespace hlc {
namespace {

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------
struct BatchPlan {
  int tile = BATCH_TILE;  // sources per partition tile
  int32_t njobs = 0, lb_bits = 31;
  uint64_t NA = 0, NB = 0;
  uint32_t ztotal = 0;
  std::vector<BatchJob> jobs;
  std::vector<BatchTile> tA, tB;
};

// 64-bit hash of a byte range, eight bytes per step (multiply and xor-shift
// mixing of each word into the state).
uint64_t hash_words(const void* p, size_t n, uint64_t h = 0x9e3779b97f4a7c15ull) {
  const unsigned char* c = (const unsigned char*)p;
  size_t i = 0;
  for (; i + 8 <= n; i += 8) {
    uint64_t w;
    std::memcpy(&w, c + i, 8);
    h ^= w;
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
  }
  uint64_t w = 0;
  std::memcpy(&w, c + i, n - i);
  h ^= w ^ (uint64_t)n;
  h *= 0xc4ceb9fe1a85ec53ull;
  h ^= h >> 29;
  return h;
}

uint64_t fnv(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

int build_plan(const hlc_job* jobs, int32_t njobs, int tile, BatchPlan& P) {
  if (njobs < 0 || njobs > 65536) return HLC_E_INVAL;
  if (njobs > 0 && !jobs) return HLC_E_INVAL;
  if (!batch_tile_ok(tile)) return HLC_E_INVAL;
  P.tile = tile;
  P.njobs = njobs;
  P.lb_bits = 32 - std::max(1, ceil_log2((uint64_t)std::max(njobs, 1)));
  P.jobs.resize(njobs);
  uint64_t ea = 0, eb = 0, zo = 0;
  const uint32_t zmax = 1u << (P.lb_bits - 8);
  for (int32_t j = 0; j < njobs; ++j) {
    const hlc_job& J = jobs[j];
    if (J.a_off < 0 || J.na < 0 || J.b_off < 0 || J.nb < 0) return HLC_E_INVAL;
    if (!(J.r_arcsec > 0.0) || !(J.r_arcsec <= 3600.0)) return HLC_E_INVAL;
    if (J.a_off + J.na >= (int64_t(1) << 31) || J.b_off + J.nb >= (int64_t(1) << 31)) return HLC_E_INVAL;
    BatchJob& B = P.jobs[j];
    B.a_off = J.a_off;
    B.na = J.na;
    B.b_off = J.b_off;
    B.nb = J.nb;
    B.r_arcsec = J.r_arcsec;
    const double sh = std::sin(0.5 * (J.r_arcsec / 3600.0) * (M_PI / 180.0));
    B.H_lo = sh * sh * (1.0 - EPS_BAND);
    B.H_hi = sh * sh * (1.0 + EPS_BAND);
    B.a_entry = (uint32_t)ea;
    B.b_entry = (uint32_t)eb;
    // zone budget: enough zones for about 16 sources per zone row, at most 2^(LB-8)
    B.zcap = (uint32_t)std::min<uint64_t>(zmax, 4 + (uint64_t)(J.na + J.nb) / 16);
    B.zoff = (uint32_t)zo;
    zo += B.zcap + 1;
    for (int64_t t = 0; t < J.na; t += tile)
      P.tA.push_back({(uint32_t)j, (uint32_t)(ea + t), (uint32_t)(J.a_off + t),
                      (uint32_t)std::min<int64_t>(tile, J.na - t)});
    for (int64_t t = 0; t < J.nb; t += tile)
      P.tB.push_back({(uint32_t)j, (uint32_t)(eb + t), (uint32_t)(J.b_off + t),
                      (uint32_t)std::min<int64_t>(tile, J.nb - t)});
    ea += J.na;
    eb += J.nb;
    if (ea >= (uint64_t(1) << 30) || eb >= (uint64_t(1) << 30) || zo >= (uint64_t(1) << 31))
      return HLC_E_INVAL;
  }
  P.NA = ea;
  P.NB = eb;
  P.ztotal = (uint32_t)zo;
  return HLC_OK;
}

struct BatchState {  // per device
  void* tables = nullptr;
  size_t tables_bytes = 0;
  uint64_t tables_hash = 0;
  BatchJob* d_jobs = nullptr;
  BatchTile *d_tA = nullptr, *d_tB = nullptr;
  hipStream_t st = nullptr;
  hipStream_t st2 = nullptr;  // A's chain, beside B's
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
  hipEvent_t ev_fork[2] = {nullptr, nullptr}, ev_join[2] = {nullptr, nullptr};
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  uint64_t graph_key = 0;
  int ncu = 256;
  // the last batch's plan, reused while the caller's job table repeats
  BatchPlan plan;
  uint64_t plan_hash = 0;
  std::vector<hlc_job> plan_jobs;  // the job table the plan was built from
  uint64_t plan_gen = 0;           // bumped whenever the plan is rebuilt
  bool plan_ok = false;
};
BatchState g_bstate[MAX_DEVICES];

void drop_graph(BatchState& B) {
  if (B.exec) (void)hipGraphExecDestroy(B.exec);
  if (B.graph) (void)hipGraphDestroy(B.graph);
  B.exec = nullptr;
  B.graph = nullptr;
  B.graph_key = 0;
}

struct BatchBufs {
  unsigned long long* bounds;
  JobGeom* geo;
  uint32_t *kA, *vA, *kB, *vB, *lb, *msplit, *zstart, *ckey, *cval;
  int32_t* zmarg;
  GroupRanges* ranges;
  Rec64 *rA64, *rB64;
  Rec32 *rA32, *rB32;
  double2 *radecA, *radecB;
  uint2* band;
  uint32_t* band_job;
  uint64_t band_cap;
  Regions reg;
  unsigned long long* jcount;
  SortScratch sc, scA;
};

void carve_batch(Carve& c, BatchBufs& b, const BatchPlan& P, bool fp32, const Caps& caps, bool own_jcount) {
  const uint64_t band_cap = caps.band;
  const uint32_t NA = std::max<uint32_t>((uint32_t)P.NA, 1), NB2 = std::max<uint32_t>(2 * (uint32_t)P.NB, 1);
  const uint32_t ng = (NA + GROUP - 1) / GROUP;
  b.bounds = c.take<unsigned long long>(4 * (size_t)std::max(P.njobs, 1));
  b.geo = c.take<JobGeom>(std::max(P.njobs, 1));
  b.kA = c.take<uint32_t>(NA);
  b.vA = c.take<uint32_t>(NA);
  b.kB = c.take<uint32_t>(NB2);
  b.vB = c.take<uint32_t>(NB2);
  carve_sort(c, b.sc, std::max(NB2, ng));
  carve_sort(c, b.scA, NA);
  if (fp32) {
    b.rA32 = c.take<Rec32>(NA);
    b.rB32 = c.take<Rec32>(NB2);
    b.radecA = c.take<double2>(NA);
    b.radecB = c.take<double2>(NB2);
    b.rA64 = b.rB64 = nullptr;
  } else {
    b.rA64 = c.take<Rec64>(NA);
    b.rB64 = c.take<Rec64>(NB2);
    b.rA32 = b.rB32 = nullptr;
    b.radecA = b.radecB = nullptr;
  }
  b.lb = c.take<uint32_t>(NA);
  b.msplit = c.take<uint32_t>(merge_splits_len(NA, NB2));
  b.ranges = c.take<GroupRanges>(ng);
  b.ckey = c.take<uint32_t>(ng);
  b.cval = c.take<uint32_t>(ng);
  b.zmarg = c.take<int32_t>(std::max<uint32_t>(P.ztotal, 1));
  b.zstart = c.take<uint32_t>(std::max<uint32_t>(P.ztotal, 1));
  b.band = c.take<uint2>(band_cap);
  b.band_job = c.take<uint32_t>(band_cap);
  b.band_cap = band_cap;
  carve_regions(c, b.reg, caps, true);
  b.jcount = own_jcount ? c.take<unsigned long long>(std::max(P.njobs, 1)) : nullptr;
}

// The batched form's tuned launch parameters: the zone-height factor of each
// job's frame, the partition tile (sources per block of the bounds and keygen
// kernels) and the persistent match grid (blocks per compute unit).
struct BatchConfig {
  double factor;
  int tile;
  int bpc;
};
constexpr BatchConfig DEFAULT_CONFIG{1.0, BATCH_TILE, 4};
// the candidates the autotuner times, one knob after the other
constexpr double FACTORS[] = {0.35, 0.5, 0.7, 1.0, 1.4, 2.0, 2.8};
constexpr int BPCS[] = {1, 2, 4, 8};
constexpr int TILES[] = {256, 512, 1024, 2048};

// Every launch of one batched call on stream s, A's chain forked to BS.st2
// and joined back (no host synchronisation, so the sequence can be captured
// into a graph with two branches).
void batch_enqueue(Device& dev, BatchState& BS, const BatchPlan& P, const BatchBufs& b, const double* a_ra,
                   const double* a_dec, const double* b_ra, const double* b_dec, hlc_pair* out_pairs,
                   double* out_sep, uint64_t cap, unsigned long long* jcount, const BatchConfig& cfg, bool fp32,
                   hipStream_t s) {
  const uint32_t NA = (uint32_t)P.NA, NB = (uint32_t)P.NB;
  hipStream_t s2 = BS.st2;
  auto fork = [&](int k) {
    (void)hipEventRecord(BS.ev_fork[k], s);
    (void)hipStreamWaitEvent(s2, BS.ev_fork[k], 0);
  };
  auto join = [&](int k) {
    (void)hipEventRecord(BS.ev_join[k], s2);
    (void)hipStreamWaitEvent(s, BS.ev_join[k], 0);
  };
  launch_zero_counters(dev.cnt, s);
  launch_zero_u64(jcount, (uint32_t)P.njobs, s);
  launch_job_bounds_init(b.bounds, P.njobs, s);
  fork(0);
  launch_job_bounds(BS.d_tA, (uint32_t)P.tA.size(), P.tile, BS.d_jobs, a_ra, b_ra, a_ra, a_dec, false, b.bounds,
                    dev.cnt, s2);
  launch_job_bounds(BS.d_tB, (uint32_t)P.tB.size(), P.tile, BS.d_jobs, a_ra, b_ra, b_ra, b_dec, true, b.bounds,
                    dev.cnt, s);
  join(0);
  launch_job_frames(BS.d_jobs, P.njobs, a_ra, b_ra, b.bounds, P.lb_bits, cfg.factor, b.geo, s);
  const DevCount cA{NA, NA, nullptr};
  const DevCount cB{NB, 2 * NB, &dev.cnt->n_halo};
  fork(1);
  launch_batch_keygen(BS.d_tA, (uint32_t)P.tA.size(), P.tile, b.geo, a_ra, a_dec, P.lb_bits, false, NA, b.kA, b.vA,
                      dev.cnt, s2);
  radix_sort(b.kA, b.vA, cA, 32, b.scA, s2);
  if (fp32) launch_batch_layout32(b.kA, b.vA, cA, a_ra, a_dec, b.geo, P.lb_bits, b.rA32, b.radecA, s2);
  else launch_layout64(b.vA, cA, a_ra, a_dec, b.rA64, s2);
  launch_batch_keygen(BS.d_tB, (uint32_t)P.tB.size(), P.tile, b.geo, b_ra, b_dec, P.lb_bits, true, NB, b.kB, b.vB,
                      dev.cnt, s);
  radix_sort(b.kB, b.vB, cB, 32, b.sc, s);
  if (fp32) launch_batch_layout32(b.kB, b.vB, cB, b_ra, b_dec, b.geo, P.lb_bits, b.rB32, b.radecB, s);
  else launch_layout64(b.vB, cB, b_ra, b_dec, b.rB64, s);
  launch_batch_zone_tables(b.geo, P.njobs, BS.d_jobs, P.ztotal, P.lb_bits, b.kB, cB, b.zmarg, b.zstart, s);
  join(1);
  launch_merge_lb(b.kA, cA, b.kB, cB, b.msplit, b.lb, s);
  launch_batch_ranges(b.kA, cA, b.lb, b.kB, b.geo, P.lb_bits, b.zmarg, b.zstart, b.ranges, b.ckey, b.cval, s);
  const uint32_t ng = (NA + GROUP - 1) / GROUP;
  radix_sort(b.ckey, b.cval, DevCount{ng, ng, nullptr}, 32, b.sc, s);
  BatchMatchArgs ma{};
  ma.ranges = b.ranges;
  ma.order = b.cval;
  ma.queue = &dev.cnt->queue;
  ma.na = cA;
  ma.keysA = b.kA;
  ma.keysB = b.kB;
  ma.recA64 = b.rA64;
  ma.recB64 = b.rB64;
  ma.recA32 = b.rA32;
  ma.recB32 = b.rB32;
  ma.radecA = b.radecA;
  ma.radecB = b.radecB;
  ma.geo = b.geo;
  ma.lb_bits = P.lb_bits;
  ma.job_count = jcount;
  OutArgs oa = out_args(out_pairs, out_sep, cap, b.band, b.band_cap, b.reg, dev.cnt);
  oa.band_job = b.band_job;
  launch_regions_reset(oa, s);
  // persistent grid: cfg.bpc 256-thread blocks per CU, at most one wave per
  // item of four groups
  const uint32_t nblocks =
      std::max<uint32_t>(1, std::min<uint32_t>((uint32_t)cfg.bpc * (uint32_t)BS.ncu, (ng + 15) / 16));
  launch_batch_match(ma, oa, fp32, nblocks, s);
  launch_batch_certify(a_ra, a_dec, b_ra, b_dec, BS.d_jobs, oa, jcount, s);
  launch_compact(oa, s);
}

// The plan for (jobs, tile): kept while the caller passes the same job table
// again (the hash rejects a changed table quickly; a full comparison
// confirms a repeated one) and the tile is the same.
int ensure_plan(BatchState& BS, const hlc_job* jobs, int32_t njobs, int tile) {
  const size_t jbytes = sizeof(hlc_job) * (size_t)njobs;
  const uint64_t jh = hash_words(jobs, jbytes, (uint64_t)njobs);
  const bool same = BS.plan_ok && BS.plan.tile == tile && BS.plan_hash == jh &&
                    BS.plan_jobs.size() == (size_t)njobs &&
                    (njobs == 0 || std::memcmp(BS.plan_jobs.data(), jobs, jbytes) == 0);
  if (same) return HLC_OK;
  BS.plan_ok = false;
  BS.plan = BatchPlan();
  HLC_CHECK(build_plan(jobs, njobs, tile, BS.plan));
  BS.plan_jobs.assign(jobs, jobs + njobs);
  BS.plan_hash = jh;
  ++BS.plan_gen;
  BS.plan_ok = true;
  return HLC_OK;
}

// Device copies of the plan's job and tile tables (uploaded again whenever
// the plan was rebuilt; its generation identifies them).
int ensure_tables(BatchState& BS, hipStream_t s) {
  const BatchPlan& P = BS.plan;
  if (BS.plan_gen == BS.tables_hash && BS.tables) return HLC_OK;
  drop_graph(BS);
  Carve sz{nullptr};
  sz.take<BatchJob>(P.jobs.size());
  sz.take<BatchTile>(std::max<size_t>(P.tA.size(), 1));
  sz.take<BatchTile>(std::max<size_t>(P.tB.size(), 1));
  if (sz.off + 256 > BS.tables_bytes) {
    if (BS.tables) {
      (void)hipDeviceSynchronize();
      (void)hipFree(BS.tables);
      BS.tables = nullptr;
      BS.tables_bytes = 0;
    }
    HLC_CHECK(dev_alloc(&BS.tables, sz.off + 256));
    BS.tables_bytes = sz.off + 256;
  }
  Carve c{(char*)BS.tables};
  BS.d_jobs = c.take<BatchJob>(P.jobs.size());
  BS.d_tA = c.take<BatchTile>(std::max<size_t>(P.tA.size(), 1));
  BS.d_tB = c.take<BatchTile>(std::max<size_t>(P.tB.size(), 1));
  HLC_TRY(hipMemcpyAsync(BS.d_jobs, P.jobs.data(), P.jobs.size() * sizeof(BatchJob), hipMemcpyHostToDevice, s));
  HLC_TRY(hipMemcpyAsync(BS.d_tA, P.tA.data(), P.tA.size() * sizeof(BatchTile), hipMemcpyHostToDevice, s));
  HLC_TRY(hipMemcpyAsync(BS.d_tB, P.tB.data(), P.tB.size() * sizeof(BatchTile), hipMemcpyHostToDevice, s));
  HLC_TRY(hipStreamSynchronize(s));
  BS.tables_hash = BS.plan_gen;
  return HLC_OK;
}

int batch_impl(const hlc_job* jobs, int32_t njobs, const double* a_ra, const double* a_dec,
               const double* b_ra, const double* b_dec, hlc_pair* out_pairs, double* out_sep,
               int64_t* job_pair_count, const hlc_opts* o) {
  if (njobs < 0 || njobs > 65536 || (njobs > 0 && !jobs)) return HLC_E_INVAL;
  const hlc_tuning* tu = o->tuning;
  if (tu && ((tu->batch_tile != 0 && !batch_tile_ok(tu->batch_tile)) || tu->batch_blocks_per_cu < 0 ||
             tu->batch_blocks_per_cu > 8 || tu->zone_height_factor < 0))
    return HLC_E_INVAL;
  int dev_id = 0;
  Device* dev = nullptr;
  HLC_CHECK(get_device(&dev, &dev_id));
  BatchState& BS = g_bstate[dev_id];
  // given knobs, else the cached ones, else the defaults (tuned below)
  BatchConfig cfg = DEFAULT_CONFIG;
  const bool g_factor = tu && tu->zone_height_factor > 0, g_tile = tu && tu->batch_tile > 0,
             g_bpc = tu && tu->batch_blocks_per_cu > 0;
  if (g_factor) cfg.factor = tu->zone_height_factor;
  if (g_tile) cfg.tile = tu->batch_tile;
  if (g_bpc) cfg.bpc = tu->batch_blocks_per_cu;
  const bool fp32 = o->precision == HLC_FP32_RECHECK;
  // the cache bucket: precision, device, size class (from the job totals, so
  // that the plan is built once, for the tile the call will use)
  int64_t tot_a = 0, tot_b = 0;
  for (int32_t j = 0; j < njobs; ++j) {
    tot_a += std::max<int64_t>(jobs[j].na, 0);
    tot_b += std::max<int64_t>(jobs[j].nb, 0);
  }
  char size_class[96];
  std::snprintf(size_class, sizeof size_class, "|j%d|a%d|b%d", ceil_log2((uint64_t)njobs),
                ceil_log2((uint64_t)tot_a), ceil_log2((uint64_t)tot_b));
  const std::string bucket = std::string("batch|") + (fp32 ? "fp32|" : "fp64|") + tune_device_tag() + size_class;
  bool tune = !(g_factor && g_tile && g_bpc);
  if (tune) {
    std::vector<double> v;
    if (tune_lookup(bucket, &v) && v.size() >= 3 && v[0] > 0 && batch_tile_ok((int)v[1]) && v[2] >= 1 &&
        v[2] <= 8) {
      if (!g_factor) cfg.factor = v[0];
      if (!g_tile) cfg.tile = (int)v[1];
      if (!g_bpc) cfg.bpc = (int)v[2];
      tune = false;
    }
  }
  HLC_CHECK(ensure_plan(BS, jobs, njobs, cfg.tile));
  const BatchPlan& P0 = BS.plan;
  if ((P0.NA > 0 && (!a_ra || !a_dec)) || (P0.NB > 0 && (!b_ra || !b_dec))) return HLC_E_INVAL;
  std::memset(&g_stats, 0, sizeof(g_stats));
  if (P0.NA == 0 || P0.NB == 0) {
    // nothing can match; still reject invalid coordinates
    if (job_pair_count && njobs > 0)
      HLC_TRY(hipMemsetAsync(job_pair_count, 0, sizeof(int64_t) * njobs, (hipStream_t)o->stream));
    for (const hlc_job* J = jobs; J < jobs + njobs; ++J) {
      if (J->na > 0) HLC_CHECK(validate_only(a_ra + J->a_off, a_dec + J->a_off, J->na, nullptr, nullptr, 0, J->r_arcsec, o));
      if (J->nb > 0) HLC_CHECK(validate_only(nullptr, nullptr, 0, b_ra + J->b_off, b_dec + J->b_off, J->nb, J->r_arcsec, o));
    }
    *o->n_pairs = 0;
    return HLC_OK;
  }
  if (!BS.st) {
    HLC_TRY(hipStreamCreate(&BS.st));
    HLC_TRY(hipStreamCreateWithFlags(&BS.st2, hipStreamNonBlocking));
    for (int k = 0; k < 2; ++k) {
      HLC_TRY(hipEventCreateWithFlags(&BS.ev_fork[k], hipEventDisableTiming));
      HLC_TRY(hipEventCreateWithFlags(&BS.ev_join[k], hipEventDisableTiming));
    }
    HLC_TRY(hipEventCreateWithFlags(&BS.ev_in, hipEventDisableTiming));
    HLC_TRY(hipEventCreateWithFlags(&BS.ev_out, hipEventDisableTiming));
    HLC_TRY(hipEventCreate(&BS.ev_t0));
    HLC_TRY(hipEventCreate(&BS.ev_t1));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev_id) == hipSuccess && prop.multiProcessorCount > 0)
      BS.ncu = prop.multiProcessorCount;
  }
  hipStream_t us = (hipStream_t)o->stream;
  HLC_TRY(hipEventRecord(BS.ev_in, us));
  HLC_TRY(hipStreamWaitEvent(BS.st, BS.ev_in, 0));
  hipStream_t s = BS.st;

  unsigned long long* jcount = reinterpret_cast<unsigned long long*>(job_pair_count);
  const uint64_t cap = (uint64_t)o->capacity;
  Caps caps = initial_caps(*dev, (uint64_t)(P0.NA + P0.NB), cap, false, true);
  double* sep = (o->flags & HLC_NO_SEP) ? nullptr : out_sep;

  for (int attempt = 0; attempt < 3; ++attempt) {
    BatchBufs b;
    Carve sz{nullptr};
    carve_batch(sz, b, BS.plan, fp32, caps, jcount == nullptr);
    HLC_CHECK(ensure_ws(*dev, sz.off + 256));
    Carve c{(char*)dev->ws};
    carve_batch(c, b, BS.plan, fp32, caps, jcount == nullptr);
    unsigned long long* jc = jcount ? jcount : b.jcount;
    if (tune) {
      // autotune on this batch: each knob not given is timed over its
      // candidates with the others fixed, in the order factor, grid, tile
      // (the tile changes the plan and its tables). Each candidate runs as
      // the call itself does, as a captured graph: one untimed replay, then
      // the best of two timed ones
      drop_graph(BS);
      auto timed = [&](const BatchConfig& k, double* ms_out) -> int {
        HLC_CHECK(ensure_plan(BS, jobs, njobs, k.tile));
        HLC_CHECK(ensure_tables(BS, s));
        hipGraph_t gr = nullptr;
        hipGraphExec_t ex = nullptr;
        HLC_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        batch_enqueue(*dev, BS, BS.plan, b, a_ra, a_dec, b_ra, b_dec, out_pairs, sep, cap, jc, k, fp32, s);
        HLC_TRY(hipStreamEndCapture(s, &gr));
        hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        double best = 1e30;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
          if ((e = hipEventRecord(BS.ev_t0, s)) != hipSuccess) break;
          if ((e = hipGraphLaunch(ex, s)) != hipSuccess) break;
          if ((e = hipEventRecord(BS.ev_t1, s)) != hipSuccess) break;
          if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
          float ms = 0.f;
          if ((e = hipEventElapsedTime(&ms, BS.ev_t0, BS.ev_t1)) != hipSuccess) break;
          if (rep > 0) best = std::min(best, (double)ms);
        }
        if (ex) (void)hipGraphExecDestroy(ex);
        (void)hipGraphDestroy(gr);
        HLC_TRY(e);
        *ms_out = best;
        return HLC_OK;
      };
      double t = 0.0;
      if (!g_factor) {
        double best_t = 1e30;
        BatchConfig k = cfg;
        for (double f : FACTORS) {
          k.factor = f;
          HLC_CHECK(timed(k, &t));
          if (t < best_t) { best_t = t; cfg.factor = f; }
        }
      }
      if (!g_bpc) {
        double best_t = 1e30;
        BatchConfig k = cfg;
        for (int v : BPCS) {
          k.bpc = v;
          HLC_CHECK(timed(k, &t));
          if (t < best_t) { best_t = t; cfg.bpc = v; }
        }
      }
      if (!g_tile) {
        double best_t = 1e30;
        BatchConfig k = cfg;
        for (int v : TILES) {
          k.tile = v;
          HLC_CHECK(timed(k, &t));
          if (t < best_t) { best_t = t; cfg.tile = v; }
        }
      }
      tune_store(bucket, {cfg.factor, (double)cfg.tile, (double)cfg.bpc});
      tune = false;
    }
    HLC_CHECK(ensure_plan(BS, jobs, njobs, cfg.tile));
    HLC_CHECK(ensure_tables(BS, s));
    const BatchPlan& P = BS.plan;
    const bool prof = (o->flags & HLC_PROFILE) != 0;
    const uint64_t th = BS.plan_gen;
    uint64_t gk = fnv(&th, sizeof th);
    const void* keyp[] = {a_ra, a_dec, b_ra, b_dec, out_pairs, sep, jc, dev->ws, dev->cnt};
    gk = fnv(keyp, sizeof keyp, gk);
    const double keyd[] = {cfg.factor, (double)cfg.tile, (double)cfg.bpc, (double)cap, (double)caps.band,
                           (double)caps.stage, (double)fp32, (double)dev->ws_bytes};
    gk = fnv(keyd, sizeof keyd, gk);
    if (BS.exec == nullptr || BS.graph_key != gk) {
      drop_graph(BS);
      HLC_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      batch_enqueue(*dev, BS, P, b, a_ra, a_dec, b_ra, b_dec, out_pairs, sep, cap, jc, cfg, fp32, s);
      hipError_t e = hipStreamEndCapture(s, &BS.graph);
      if (e != hipSuccess) {
        BS.graph = nullptr;
        return map_err(e);
      }
      e = hipGraphInstantiate(&BS.exec, BS.graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        drop_graph(BS);
        return map_err(e);
      }
      BS.graph_key = gk;
    }
    if (prof) HLC_TRY(hipEventRecord(BS.ev_t0, s));
    HLC_TRY(hipGraphLaunch(BS.exec, s));
    if (prof) HLC_TRY(hipEventRecord(BS.ev_t1, s));
    HLC_TRY(hipMemcpyAsync(dev->cnt_host, dev->cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HLC_TRY(hipStreamSynchronize(s));
    HLC_TRY(hipEventRecord(BS.ev_out, s));
    HLC_TRY(hipStreamWaitEvent(us, BS.ev_out, 0));
    const Counters& h = *dev->cnt_host;
    if (h.err) {
      *o->n_pairs = 0;
      return HLC_E_INVAL;
    }
    if (regrow(*dev, h, cap, caps)) {
      drop_graph(BS);
      continue;
    }
    g_stats.na = (int64_t)P.NA;
    g_stats.nb = (int64_t)P.NB;
    g_stats.nb_halo = (int64_t)(P.NB + h.n_halo);
    g_stats.n_pairs = (int64_t)h.n_pairs;
    g_stats.n_candidates = (int64_t)h.n_cand;
    g_stats.n_band = (int64_t)h.n_band;
    g_stats.n_ties = (int64_t)h.n_ties;
    g_stats.n_zones = (int32_t)P.ztotal;
    g_stats.zone_height_arcsec = cfg.factor;  // batched form: the zone-height factor used
    g_stats.batch_tile = cfg.tile;
    g_stats.batch_blocks_per_cu = cfg.bpc;
    if (prof) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, BS.ev_t0, BS.ev_t1);
      g_stats.t_total_ms = ms;
    }
    *o->n_pairs = (int64_t)h.n_pairs;
    return h.n_pairs > cap ? HLC_E_OVERFLOW : HLC_OK;
  }
  return HLC_E_NOMEM;
}

}  // namespace

void batch_release_all() {
  for (auto& B : g_bstate) {
    drop_graph(B);
    if (B.tables) (void)hipFree(B.tables);
    if (B.st) (void)hipStreamDestroy(B.st);
    if (B.st2) (void)hipStreamDestroy(B.st2);
    for (hipEvent_t e : {B.ev_in, B.ev_out, B.ev_t0, B.ev_t1, B.ev_fork[0], B.ev_fork[1], B.ev_join[0],
                         B.ev_join[1]})
      if (e) (void)hipEventDestroy(e);
    B = BatchState();
  }
}

}  // namespace hlc

using namespace hlc;

extern "C" {

int hlc_xmatch_batch(const hlc_job* jobs, int32_t njobs, const double* a_ra, const double* a_dec,
                     const double* b_ra, const double* b_dec, hlc_pair* out_pairs, double* out_sep_arcsec,
                     int64_t* job_pair_count, const hlc_opts* opts) {
  HLC_CHECK(check_opts(opts));
  if (opts->flags & HLC_SELF) return HLC_E_UNSUPPORTED;
  if (opts->capacity > 0 && (!out_pairs || (!(opts->flags & HLC_NO_SEP) && !out_sep_arcsec)))
    return HLC_E_INVAL;
  try {
    return sort_output(
        batch_impl(jobs, njobs, a_ra, a_dec, b_ra, b_dec, out_pairs, out_sep_arcsec, job_pair_count, opts),
        out_pairs, out_sep_arcsec, opts, int64_t(1) << 31, int64_t(1) << 31);
  } catch (const std::bad_alloc&) {
    return HLC_E_NOMEM;
  } catch (...) {
    return HLC_E_DEVICE;
  }
}

}  // extern "C"
