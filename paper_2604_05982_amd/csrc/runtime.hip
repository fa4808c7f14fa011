// runtime.hip -- host side of the C ABI declared in include/gtap.h.
//
// gtap_init lays out one device workspace (frame pools, deques, depot, job
// table, control block), gtap_submit packs root-task arguments into job
// slots, gtap_run resets the scheduler state with a small kernel and launches
// the persistent scheduler kernel once for every pending job on the caller's
// stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>

#include "../../include/gtap.h"
#include "fmm.h"
#include "fmm_eval.h"
#include "kclique_bits.h"
#include "layout.h"
#include "probes.h"
#include "sched_block.h"
#include "sched_thread.h"

using namespace gtap;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

struct Layout {
  size_t ctl, jobs, dq, rings, bins_s, store_s, bins_b, store_b, frames_s, frames_b, cq, cring, total;
  uint32_t bincap_s, bincap_b, stride_b, ccap;
};

// Centralised-queue variant: one ring for the grid, as many slots as all the
// wavefronts' deques together (a power of two, at most 2^26), and at least
// 256 per wavefront (a reservation keeps 64 per wavefront clear of claims
// that may still be reading).
uint32_t central_capacity(const gtap_config &c, uint32_t nwaves) {
  if (!(c.flags & GTAP_FLAG_SCHED_CENTRAL)) return 0;
  uint64_t want = static_cast<uint64_t>(c.deque_capacity) * nwaves;
  if (want > (1ull << 26)) want = 1ull << 26;
  uint32_t cap = 1u << 16;
  while (static_cast<uint64_t>(cap) * 2 <= want || cap < 256ull * nwaves) cap *= 2;
  return cap;
}

Layout make_layout(const gtap_config &c, uint32_t nwaves) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const size_t nd = static_cast<size_t>(nwaves) * c.num_queues;
  L.stride_b = align_up(kFrameWords + c.big_frame_ints, 16);  // 64-byte multiples
  // Depot capacity covers every frame of the pool plus one chunk per bin.
  L.bincap_s = static_cast<uint32_t>(align_up((c.small_frames + kDepotBins - 1) / kDepotBins + kChunkSmall, kChunkSmall));
  L.bincap_b = static_cast<uint32_t>(align_up((c.big_frames + kDepotBins - 1) / kDepotBins + kChunkBig, kChunkBig));
  L.ctl = take(sizeof(Control));
  L.jobs = take(sizeof(JobSlot) * static_cast<size_t>(c.max_jobs));
  L.dq = take(sizeof(DequeMeta) * nd);
  L.rings = take(sizeof(uint32_t) * nd * c.deque_capacity);
  L.bins_s = take(sizeof(DepotBin) * kDepotBins);
  L.store_s = take(sizeof(uint32_t) * static_cast<size_t>(kDepotBins) * L.bincap_s);
  L.bins_b = take(sizeof(DepotBin) * kDepotBins);
  L.store_b = take(sizeof(uint32_t) * static_cast<size_t>(kDepotBins) * L.bincap_b);
  L.frames_s = take(sizeof(uint32_t) * kFrameWords * static_cast<size_t>(c.small_frames));
  L.frames_b = take(sizeof(uint32_t) * static_cast<size_t>(L.stride_b) * c.big_frames);
  L.ccap = central_capacity(c, nwaves);
  L.cq = take(L.ccap ? sizeof(CentralQueue) : 0);
  L.cring = take(sizeof(uint64_t) * static_cast<size_t>(L.ccap));
  L.total = off;
  return L;
}

template <int WPB>
int occupancy_blocks(int *blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, thread_sched_kernel<WPB>, 64 * WPB, 0) ==
                 hipSuccess
             ? 0
             : -1;
}

template <int NT>
int occupancy_block_mode(int *blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, block_sched_kernel<NT>, NT, 0) == hipSuccess
             ? 0
             : -1;
}

int max_resident_waves(int mode, int wpb, uint32_t *out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GTAP_E_HIP;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return GTAP_E_HIP;
  int bpc = 0, rc = -1;
  if (mode == GTAP_MODE_BLOCK) {
    switch (wpb) {
      case 1: rc = occupancy_block_mode<64>(&bpc); break;
      case 2: rc = occupancy_block_mode<128>(&bpc); break;
      case 4: rc = occupancy_block_mode<256>(&bpc); break;
      default: return GTAP_E_INVAL;
    }
  } else {
    switch (wpb) {
      case 1: rc = occupancy_blocks<1>(&bpc); break;
      case 2: rc = occupancy_blocks<2>(&bpc); break;
      case 4: rc = occupancy_blocks<4>(&bpc); break;
      case 8: rc = occupancy_blocks<8>(&bpc); break;
      default: return GTAP_E_INVAL;
    }
  }
  if (rc != 0 || bpc <= 0 || ncu <= 0) return GTAP_E_HIP;
  *out = static_cast<uint32_t>(bpc) * static_cast<uint32_t>(ncu) * static_cast<uint32_t>(wpb);
  return GTAP_OK;
}

bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

int validate(const gtap_config &c) {
  if (c.mode != GTAP_MODE_THREAD && c.mode != GTAP_MODE_BLOCK) return GTAP_E_INVAL;
  if (c.waves_per_group != 1 && c.waves_per_group != 2 && c.waves_per_group != 4 && c.waves_per_group != 8)
    return GTAP_E_INVAL;
  if (c.mode == GTAP_MODE_BLOCK && (c.waves_per_group > 4 || c.num_queues != 1)) return GTAP_E_INVAL;
  if (c.num_waves < 0 || c.num_queues < 1 || c.num_queues > static_cast<int32_t>(kMaxQueues)) return GTAP_E_INVAL;
  if (c.daq_policy < GTAP_DAQ_NONE || c.daq_policy > GTAP_DAQ_CILKSORT) return GTAP_E_INVAL;
  if (!is_pow2(c.deque_capacity) || c.deque_capacity < 128 || c.deque_capacity > (1u << 28)) return GTAP_E_INVAL;
  if (c.steal_below < 1 || c.steal_below > 64) return GTAP_E_INVAL;
  if (c.steal_probes < 1 || c.steal_probes > 64 || c.steal_div < 1 || c.steal_div > 64) return GTAP_E_INVAL;
  if (c.small_frames < 1024 || c.small_frames >= (1ull << 31)) return GTAP_E_INVAL;
  if (c.big_frames >= (1ull << 31)) return GTAP_E_INVAL;
  if (c.big_frame_ints > (1u << 24)) return GTAP_E_INVAL;
  if (c.max_jobs < 1 || c.max_jobs > (1u << 24)) return GTAP_E_INVAL;
  const uint32_t known = GTAP_FLAG_NO_PRIVATE_STACK | GTAP_FLAG_SCHED_SINGLE | GTAP_FLAG_SCHED_CENTRAL;
  if (c.flags & ~known) return GTAP_E_INVAL;
  // the comparison variants are built for four wavefronts per group only
  if (c.flags && (c.mode != GTAP_MODE_THREAD || c.num_queues != 1 || c.waves_per_group != 4)) return GTAP_E_INVAL;
  if ((c.flags & GTAP_FLAG_SCHED_SINGLE) && (c.flags & GTAP_FLAG_SCHED_CENTRAL)) return GTAP_E_INVAL;
  return GTAP_OK;
}

uint32_t reset_blocks(uint32_t ndeques, uint32_t ccap) {
  const uint32_t n = std::max(ndeques, ccap);
  return std::min<uint32_t>(std::max<uint32_t>((n + 255) / 256, 1), 4096);
}

__global__ void reset_kernel(Params p, uint32_t ndeques) {
  const size_t i0 = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t d = i0; d < ndeques; d += stride) {
    p.dq[d].count = 0;
    p.dq[d].head = 0;
    p.dq[d].lock = 0;
    p.dq[d].pad[0] = 0;  // block mode reads the line as {int64 top, int64 bottom}
  }
  for (size_t b = i0; b < kDepotBins; b += stride) {
    p.bins_s[b].lock = 0;
    p.bins_s[b].nchunks = 0;
    p.bins_b[b].lock = 0;
    p.bins_b[b].nchunks = 0;
  }
  // centralised queue: positions restart at 0, so no slot may carry a tag
  // from an earlier run
  for (size_t s = i0; s < p.ccap; s += stride) p.cring[s] = ~0ull;
  if (i0 == 0 && p.ccap) {
    p.cq->tail = 0;
    p.cq->count = 0;
    p.cq->head = 0;
  }
  if (i0 == 0) {
    Control *c = p.ctl;
    c->jobs_remaining = static_cast<int32_t>(p.njobs);
    c->error = 0;
    c->err_pool = 0;
    c->err_wave = -1;
    c->err_job = -1;
    c->err_capacity = 0;
    c->err_requested = 0;
    c->bump_small = 0;
    c->bump_big = 0;
    c->admitted = 0;
    c->live_small = 0;
    c->live_big = 0;
    c->hungry = 0;
    for (int s = 0; s < static_cast<int>(ST_COUNT); ++s) c->stats[s] = 0;
  }
}

// Kernel parameters of a batch run whose workspace starts at `ws` and is
// laid out by L; returns the device wall-clock rate (kHz) the watchdog uses.
int fill_params(const gtap_config &cfg, uint32_t nw, const Layout &L, char *ws, Params &p) {
  p = Params{};
  p.ctl = reinterpret_cast<Control *>(ws + L.ctl);
  p.jobs = reinterpret_cast<JobSlot *>(ws + L.jobs);
  p.njobs = 0;
  p.nwaves = nw;
  p.dq = reinterpret_cast<DequeMeta *>(ws + L.dq);
  p.rings = reinterpret_cast<uint32_t *>(ws + L.rings);
  p.cap = cfg.deque_capacity;
  p.Q = static_cast<uint32_t>(cfg.num_queues);
  p.frames_s = reinterpret_cast<uint32_t *>(ws + L.frames_s);
  p.nframes_s = static_cast<uint32_t>(cfg.small_frames);
  p.frames_b = reinterpret_cast<uint32_t *>(ws + L.frames_b);
  p.nframes_b = static_cast<uint32_t>(cfg.big_frames);
  p.stride_b = L.stride_b;
  p.big_ints = cfg.big_frame_ints;
  p.bins_s = reinterpret_cast<DepotBin *>(ws + L.bins_s);
  p.store_s = reinterpret_cast<uint32_t *>(ws + L.store_s);
  p.bincap_s = L.bincap_s;
  p.bins_b = reinterpret_cast<DepotBin *>(ws + L.bins_b);
  p.store_b = reinterpret_cast<uint32_t *>(ws + L.store_b);
  p.bincap_b = L.bincap_b;
  p.steal_below = cfg.steal_below;
  p.steal_probes = cfg.steal_probes;
  p.steal_div = cfg.steal_div;
  p.daq_policy = static_cast<uint32_t>(cfg.daq_policy);
  for (uint32_t i = 0; i < kMaxQueues - 1; ++i) p.daq_bounds[i] = cfg.daq_bounds[i];
  const uint32_t fl = cfg.flags;
  p.sched = (fl & GTAP_FLAG_SCHED_CENTRAL)       ? kSchedCentral
            : (fl & GTAP_FLAG_SCHED_SINGLE)      ? kSchedSingle
            : (fl & GTAP_FLAG_NO_PRIVATE_STACK) ? kSchedBatchedNoLocal
                                                 : kSchedBatched;
  p.ccap = L.ccap;
  p.cq = p.ccap ? reinterpret_cast<CentralQueue *>(ws + L.cq) : nullptr;
  p.cring = p.ccap ? reinterpret_cast<uint64_t *>(ws + L.cring) : nullptr;
  int dev = 0, rate_khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || rate_khz <= 0)
    rate_khz = 100000;  // gfx9 constant clock: 100 MHz
  const uint32_t tmo = cfg.timeout_ms ? cfg.timeout_ms : 120000;
  p.timeout_ticks = static_cast<uint64_t>(tmo) * static_cast<uint64_t>(rate_khz);
  return rate_khz;
}

}  // namespace

struct gtap_ctx {
  gtap_config cfg;
  hipStream_t stream = nullptr;
  uint32_t nwaves = 0;
  Layout lay{};
  char *ws = nullptr;
  bool owns_ws = false;
  Params params{};
  std::vector<JobSlot> pending;
  std::vector<JobSlot> done_jobs;
  uint64_t next_job_id = 0;
  uint64_t pending_first = 0;
  uint64_t done_first = 0;
  bool have_done = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  uint32_t clock_khz = 100000;
  // serving
  bool serving = false;
  JobSlot *ring = nullptr;          // pinned host memory
  uint64_t *ring_seq = nullptr;     // pinned host memory
  HostCompletion *done_host = nullptr;
  int32_t *stop_host = nullptr;
  uint64_t next_ticket = 0;
  // FMM jobs: arguments by pending position, results by run position
  std::vector<gtap_fmm_args> pending_fmm;
  std::vector<gtap_fmm_result> done_fmm;
  // split k-clique jobs: per pending job, each vertex's offset (in 64-bit
  // words) into the job's bit-matrix buffer, n+1 entries (empty: no matrices)
  std::vector<std::vector<uint64_t>> pending_ks;
  gtap_stats stats{};
  gtap_error_report err{};
};

extern "C" {

void gtap_config_default(gtap_config *cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->mode = GTAP_MODE_THREAD;
  cfg->num_waves = 0;
  cfg->waves_per_group = 4;
  cfg->num_queues = 1;
  cfg->daq_policy = GTAP_DAQ_NONE;
  const int32_t bounds[7] = {8, 32, 128, 1 << 30, 1 << 30, 1 << 30, 1 << 30};
  std::memcpy(cfg->daq_bounds, bounds, sizeof(bounds));
  cfg->deque_capacity = 1u << 15;
  cfg->steal_below = 64;
  cfg->steal_probes = 16;
  cfg->steal_div = 2;
  cfg->small_frames = 1ull << 24;
  cfg->big_frames = 1ull << 16;
  cfg->big_frame_ints = 512;
  cfg->max_jobs = 1u << 15;
  cfg->timeout_ms = 120000;
}

int gtap_workspace_size(const gtap_config *cfg, uint64_t *bytes) {
  if (!cfg || !bytes) return GTAP_E_INVAL;
  int rc = validate(*cfg);
  if (rc) return rc;
  uint32_t maxw = 0;
  rc = max_resident_waves(cfg->mode, cfg->waves_per_group, &maxw);
  if (rc) return rc;
  uint32_t nw = cfg->num_waves ? std::min<uint32_t>(cfg->num_waves, maxw) : maxw;
  nw = std::max<uint32_t>(nw / cfg->waves_per_group, 1) * cfg->waves_per_group;
  *bytes = make_layout(*cfg, nw).total;
  return GTAP_OK;
}

int gtap_init(const gtap_config *cfg, gtap_ctx **out) {
  if (!cfg || !out) return GTAP_E_INVAL;
  *out = nullptr;
  int rc = validate(*cfg);
  if (rc) return rc;
  uint32_t maxw = 0;
  rc = max_resident_waves(cfg->mode, cfg->waves_per_group, &maxw);
  if (rc) return rc;
  gtap_ctx *c = new (std::nothrow) gtap_ctx();
  if (!c) return GTAP_E_NOMEM;
  c->cfg = *cfg;
  if (c->cfg.timeout_ms == 0) c->cfg.timeout_ms = 120000;
  c->stream = static_cast<hipStream_t>(cfg->stream);
  uint32_t nw = cfg->num_waves ? std::min<uint32_t>(cfg->num_waves, maxw) : maxw;
  nw = std::max<uint32_t>(nw / cfg->waves_per_group, 1) * cfg->waves_per_group;
  c->nwaves = nw;
  c->lay = make_layout(c->cfg, nw);
  if (cfg->workspace_dev) {
    if (cfg->workspace_bytes < c->lay.total || (reinterpret_cast<uintptr_t>(cfg->workspace_dev) % kAlign)) {
      delete c;
      return GTAP_E_NOMEM;
    }
    c->ws = static_cast<char *>(cfg->workspace_dev);
  } else {
    if (hipMalloc(&c->ws, c->lay.total) != hipSuccess) {
      delete c;
      return GTAP_E_NOMEM;
    }
    c->owns_ws = true;
  }
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    gtap_finalize(c);
    return GTAP_E_HIP;
  }
  const int rate_khz = fill_params(c->cfg, nw, c->lay, c->ws, c->params);
  c->clock_khz = static_cast<uint32_t>(rate_khz);
  c->stats.num_waves = static_cast<int32_t>(nw);
  c->stats.waves_per_group = c->cfg.waves_per_group;
  c->stats.num_queues = c->cfg.num_queues;
  *out = c;
  return GTAP_OK;
}

}  // extern "C"

extern "C" int32_t gtap_kclique_split_buffer_ints(int32_t max_outdeg) {
  if (max_outdeg < 0 || max_outdeg > static_cast<int32_t>(kcs::kMaxW * 64)) return 0;
  return static_cast<int32_t>(kcs::buffer_ints(static_cast<uint32_t>(max_outdeg)));
}

// Validate a root task's arguments and pack them into a job slot.
static int pack_job(const gtap_config &cfg, hipStream_t stream, int32_t kind, const void *args,
                    size_t args_bytes, JobSlot &J, std::vector<uint64_t> *ks_off = nullptr) {
  if (!args) return GTAP_E_INVAL;
  std::memset(&J, 0, sizeof(J));
  J.kind = static_cast<uint32_t>(kind);
  const bool block = cfg.mode == GTAP_MODE_BLOCK;
  if (block && kind != GTAP_KIND_FIB && kind != GTAP_KIND_UTS && kind != GTAP_KIND_FMM) return GTAP_E_INVAL;
  switch (kind) {
    case GTAP_KIND_FIB: {
      if (args_bytes != sizeof(gtap_fib_args)) return GTAP_E_INVAL;
      gtap_fib_args a;
      std::memcpy(&a, args, sizeof(a));
      if (a.n < 0 || a.n > 92) return GTAP_E_INVAL;
      J.a[0] = static_cast<uint64_t>(a.n);
      return GTAP_OK;
    }
    case GTAP_KIND_NQUEENS: {
      if (args_bytes != sizeof(gtap_nqueens_args)) return GTAP_E_INVAL;
      gtap_nqueens_args a;
      std::memcpy(&a, args, sizeof(a));
      if (a.n < 1 || a.n > 31) return GTAP_E_INVAL;
      J.a[0] = static_cast<uint64_t>(a.n);
      J.a[1] = (1ull << a.n) - 1ull;
      return GTAP_OK;
    }
    case GTAP_KIND_UTS: {
      if (args_bytes != sizeof(gtap_uts_args)) return GTAP_E_INVAL;
      gtap_uts_args a;
      std::memcpy(&a, args, sizeof(a));
      if (a.max_depth < 0 || a.max_depth > 255) return GTAP_E_INVAL;
      J.a[0] = a.seed;
      J.a[1] = a.threshold;
      J.a[2] = static_cast<uint64_t>(a.max_depth);
      return GTAP_OK;
    }
    case GTAP_KIND_KCLIQUE: {
      if (args_bytes != sizeof(gtap_kclique_args)) return GTAP_E_INVAL;
      gtap_kclique_args a;
      std::memcpy(&a, args, sizeof(a));
      if (a.n < 0 || a.k < 1 || a.range_leaf < 1 || a.max_outdeg < 0) return GTAP_E_INVAL;
      // a task forks at most range_leaf or max_outdeg children (join-word count field)
      if (static_cast<uint32_t>(a.range_leaf) > kMaxChildren || static_cast<uint32_t>(a.max_outdeg) > kMaxChildren)
        return GTAP_E_INVAL;
      if (a.n > 0 && (!a.row_ptr_dev || !a.col_dev)) return GTAP_E_INVAL;
      // candidate tasks at level >= 2 keep C' in a big frame (k >= 4)
      if (a.k >= 4 && static_cast<uint32_t>(a.max_outdeg) > cfg.big_frame_ints) return GTAP_E_INVAL;
      if (a.k >= 4 && cfg.big_frames == 0) return GTAP_E_INVAL;
      J.a[0] = reinterpret_cast<uint64_t>(a.row_ptr_dev);
      J.a[1] = reinterpret_cast<uint64_t>(a.col_dev);
      J.a[2] = static_cast<uint64_t>(a.n);
      J.a[3] = static_cast<uint64_t>(a.k);
      J.a[4] = static_cast<uint64_t>(a.range_leaf);
      J.a[5] = static_cast<uint64_t>(a.max_outdeg);
      return GTAP_OK;
    }
    case GTAP_KIND_KCLIQUE_SPLIT: {
      if (args_bytes != sizeof(gtap_kclique_split_args)) return GTAP_E_INVAL;
      gtap_kclique_split_args a;
      std::memcpy(&a, args, sizeof(a));
      if (block || cfg.waves_per_group != 4 || cfg.flags != 0) return GTAP_E_INVAL;
      if (a.n < 0 || a.k < 1 || a.k > static_cast<int32_t>(kcs::kMaxK) || a.range_leaf < 1 ||
          static_cast<uint32_t>(a.range_leaf) > kMaxChildren || a.max_outdeg < 0 ||
          a.max_outdeg > static_cast<int32_t>(kcs::kMaxW * 64) || a.threshold < 0 ||
          a.threshold > static_cast<int32_t>(kcs::kMaxThr) ||
          (a.algorithm != GTAP_KCLIQUE_ORIENT && a.algorithm != GTAP_KCLIQUE_PIVOT))
        return GTAP_E_INVAL;
      if (a.n > 0 && (!a.row_ptr_dev || !a.col_dev)) return GTAP_E_INVAL;
      if (a.k >= 4 && (cfg.big_frames == 0 ||
                       kcs::buffer_ints(static_cast<uint32_t>(a.max_outdeg)) > cfg.big_frame_ints))
        return GTAP_E_INVAL;
      // the frame buffers are sized from max_outdeg: check it against the graph
      if (a.n > 0) {
        std::vector<int32_t> rp(static_cast<size_t>(a.n) + 1);
        if (hipMemcpyAsync(rp.data(), a.row_ptr_dev, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                           stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
          return GTAP_E_HIP;
        for (int32_t v = 0; v < a.n; ++v)
          if (rp[v + 1] < rp[v] || rp[v + 1] - rp[v] > a.max_outdeg) return GTAP_E_INVAL;
        // k >= 4: a vertex that forks row tasks (at least k-1 and more than
        // threshold out-neighbours; smaller ones count in place) gets its
        // d x W bit matrix (two of them for pivoting) in the job's buffer
        if (ks_off && a.k >= 4) {
          ks_off->assign(static_cast<size_t>(a.n) + 1, 0);
          const uint64_t mats = a.algorithm == GTAP_KCLIQUE_PIVOT ? 2 : 1;
          for (int32_t v = 0; v < a.n; ++v) {
            const uint64_t d = static_cast<uint64_t>(rp[v + 1] - rp[v]);
            const bool forks = d >= static_cast<uint64_t>(a.k - 1) && d > static_cast<uint64_t>(a.threshold);
            (*ks_off)[v + 1] = (*ks_off)[v] + (forks ? mats * d * ((d + 63) / 64) : 0);
          }
        }
      }
      J.a[0] = reinterpret_cast<uint64_t>(a.row_ptr_dev);
      J.a[1] = reinterpret_cast<uint64_t>(a.col_dev);
      J.a[2] = static_cast<uint64_t>(a.n);
      J.a[3] = static_cast<uint64_t>(a.k);
      J.a[4] = static_cast<uint64_t>(a.range_leaf);
      J.a[5] = static_cast<uint64_t>(a.max_outdeg);
      J.a[6] = static_cast<uint64_t>(a.threshold) | (static_cast<uint64_t>(a.algorithm) << 8);
      return GTAP_OK;
    }
    case GTAP_KIND_CILKSORT: {
      if (args_bytes != sizeof(gtap_cilksort_args)) return GTAP_E_INVAL;
      gtap_cilksort_args a;
      std::memcpy(&a, args, sizeof(a));
      if (block || cfg.waves_per_group != 4 || cfg.flags != 0) return GTAP_E_INVAL;
      if (a.n < 0 || a.n >= (1ll << 29) || a.sort_cutoff < 1 || a.sort_cutoff > 64 || a.merge_cutoff < 2 ||
          a.merge_cutoff > (1 << 20) || (a.n > 0 && (!a.keys_dev || !a.tmp_dev)))
        return GTAP_E_INVAL;
      J.a[0] = reinterpret_cast<uint64_t>(a.keys_dev);
      J.a[1] = reinterpret_cast<uint64_t>(a.tmp_dev);
      J.a[2] = static_cast<uint64_t>(a.n);
      J.a[3] = static_cast<uint64_t>(a.sort_cutoff) | (static_cast<uint64_t>(a.merge_cutoff) << 32);
      return GTAP_OK;
    }
    case GTAP_KIND_FMM: {
      if (args_bytes != sizeof(gtap_fmm_args)) return GTAP_E_INVAL;
      gtap_fmm_args a;
      std::memcpy(&a, args, sizeof(a));
      if (a.n < 1 || !a.x_dev || !a.y_dev || !a.z_dev || !a.q_dev || !a.phi_dev) return GTAP_E_INVAL;
      if (a.leaf_max < 1 || a.leaf_max > 64 || a.order != fmm::kP) return GTAP_E_INVAL;
      if (a.theta_num < 0 || a.theta_den < 1 || a.theta_den > 64 || a.theta_num > a.theta_den) return GTAP_E_INVAL;
      // traversal with the work inside the tasks: block mode; list-building
      // traversals: thread mode (its FMM kernel is built for four wavefronts
      // per group, without the comparison variants)
      if (block ? a.traversal != GTAP_FMM_TASKS
                : (a.traversal != GTAP_FMM_LISTS && a.traversal != GTAP_FMM_WORKLIST) ||
                      cfg.waves_per_group != 4 || cfg.flags != 0)
        return GTAP_E_INVAL;
      return GTAP_OK;  // the device descriptor is built by gtap_run
    }
    default:
      return GTAP_E_INVAL;
  }
}

extern "C" int gtap_submit(gtap_ctx *c, int32_t kind, const void *args, size_t args_bytes, uint64_t *job_id) {
  if (!c || !args) return GTAP_E_INVAL;
  if (c->serving) return GTAP_E_STATE;
  if (c->pending.size() >= c->cfg.max_jobs) return GTAP_E_FULL;
  JobSlot J;
  std::vector<uint64_t> ks_off;
  const int rc = pack_job(c->cfg, c->stream, kind, args, args_bytes, J, &ks_off);
  if (rc) return rc;
  if (c->pending.empty()) {
    c->pending_first = c->next_job_id;
    c->pending_fmm.clear();
    c->pending_ks.clear();
  }
  c->pending.push_back(J);
  gtap_fmm_args fa{};
  if (kind == GTAP_KIND_FMM) std::memcpy(&fa, args, sizeof(fa));
  c->pending_fmm.push_back(fa);
  c->pending_ks.push_back(std::move(ks_off));
  if (job_id) *job_id = c->next_job_id;
  c->next_job_id++;
  return GTAP_OK;
}

extern "C" {

// Copy a finished run's statistics and error report into the context.
static int record_run(gtap_ctx *c, const Control &ctl, float ms) {
  gtap_stats &s = c->stats;
  s.tasks = ctl.stats[ST_TASKS];
  s.conts = ctl.stats[ST_CONTS];
  s.spawns = ctl.stats[ST_SPAWNS];
  s.pushed = ctl.stats[ST_PUSHED];
  s.push_batches = ctl.stats[ST_PUSH_BATCHES];
  s.popped = ctl.stats[ST_POPPED];
  s.pop_batches = ctl.stats[ST_POP_BATCHES];
  s.stolen = ctl.stats[ST_STOLEN];
  s.steal_batches = ctl.stats[ST_STEAL_BATCHES];
  s.steal_attempts = ctl.stats[ST_STEAL_ATTEMPTS];
  s.iterations = ctl.stats[ST_ITERS];
  s.idle_iterations = ctl.stats[ST_IDLE];
  s.small_frames_touched = ctl.bump_small;
  s.big_frames_touched = ctl.bump_big;
  s.depot_spills = ctl.stats[ST_SPILLS];
  s.depot_refills = ctl.stats[ST_REFILLS];
  s.busy_cycles = ctl.stats[ST_BUSY_CYCLES];
  s.idle_cycles = ctl.stats[ST_IDLE_CYCLES];
  s.admitted = ctl.stats[ST_ADMITTED];
  s.local_pushed = ctl.stats[ST_LOCAL];
  s.atomics = ctl.stats[ST_RMW];
  s.data_bytes = 4 * ctl.stats[ST_DATA_WORDS];
  s.kernel_ms = ms;
  if (ctl.error != 0) {
    c->err.code = ctl.error;
    c->err.pool = ctl.err_pool;
    c->err.capacity = ctl.err_capacity;
    c->err.requested = ctl.err_requested;
    c->err.wave = ctl.err_wave;
    c->err.job = ctl.err_job;
    return ctl.error;
  }
  return GTAP_OK;
}

static int launch_sched(gtap_ctx *c, uint32_t ext = 0) {
  const uint32_t wpb = static_cast<uint32_t>(c->cfg.waves_per_group);
  const dim3 grid(c->nwaves / wpb), block(64 * wpb);
  if (c->cfg.mode == GTAP_MODE_BLOCK) {
    switch (wpb) {
      case 1: hipLaunchKernelGGL(block_sched_kernel<64>, grid, block, 0, c->stream, c->params); break;
      case 2: hipLaunchKernelGGL(block_sched_kernel<128>, grid, block, 0, c->stream, c->params); break;
      case 4: hipLaunchKernelGGL(block_sched_kernel<256>, grid, block, 0, c->stream, c->params); break;
      default: return GTAP_E_INVAL;
    }
    return hipGetLastError() == hipSuccess ? GTAP_OK : GTAP_E_HIP;
  }
  switch (wpb) {
    case 1: hipLaunchKernelGGL(thread_sched_kernel<1>, grid, block, 0, c->stream, c->params); break;
    case 2: hipLaunchKernelGGL(thread_sched_kernel<2>, grid, block, 0, c->stream, c->params); break;
    case 4:
      switch (c->params.sched) {
        case kSchedSingle:
          hipLaunchKernelGGL((thread_sched_kernel<4, kSchedSingle>), grid, block, 0, c->stream, c->params);
          break;
        case kSchedCentral:
          hipLaunchKernelGGL((thread_sched_kernel<4, kSchedCentral>), grid, block, 0, c->stream, c->params);
          break;
        case kSchedBatchedNoLocal:
          hipLaunchKernelGGL((thread_sched_kernel<4, kSchedBatchedNoLocal>), grid, block, 0, c->stream, c->params);
          break;
        default:
          if (ext == kExtLists)  // FMM list traversal, Cilksort
            hipLaunchKernelGGL((thread_sched_kernel<4, kSchedBatched, kExtLists>), grid, block, 0, c->stream, c->params);
          else if (ext != 0)  // and split k-clique
            hipLaunchKernelGGL((thread_sched_kernel<4, kSchedBatched, kExtAll>), grid, block, 0, c->stream, c->params);
          else
            hipLaunchKernelGGL(thread_sched_kernel<4>, grid, block, 0, c->stream, c->params);
          break;
      }
      break;
    case 8: hipLaunchKernelGGL(thread_sched_kernel<8>, grid, block, 0, c->stream, c->params); break;
    default: return GTAP_E_INVAL;
  }
  return hipGetLastError() == hipSuccess ? GTAP_OK : GTAP_E_HIP;
}

}  // extern "C"

// ---- FMM jobs: passes around the block-mode traversal -----------------------
namespace {

struct FmmJobMem {
  uint64_t *keys = nullptr, *keys_sorted = nullptr;
  int32_t *idx = nullptr, *perm = nullptr;
  void *sort_tmp = nullptr;
  double *pts = nullptr;  // px | py | pz | pq | phi, n each
  int32_t *cell = nullptr, *parent = nullptr;
  int64_t cell_cap = 0;
  int32_t *scratch = nullptr;  // nch | off | bnd | flags
  double *Q = nullptr, *L = nullptr;
  fmm::FmmDesc *desc = nullptr;
  std::vector<std::pair<int32_t, int32_t>> levels;
  int32_t ncells = 0;
  hipEvent_t ev[6] = {};
  // list-building traversals
  uint64_t *m2l = nullptr, *p2p = nullptr;
  uint64_t m2l_cap = 0, p2p_cap = 0;
  uint64_t *front = nullptr;   // two frontiers of front_cap pairs, then the counter
  uint64_t front_cap = 0;
  int64_t rounds = 0, retries = 0;
  float worklist_ms = 0.f;
  hipEvent_t lev[8] = {};
  fmm::FmmDesc hdesc{};        // host copy of the descriptor (lists, capacities)
  uint64_t *seg = nullptr, *sorted = nullptr;
  void *lsort_tmp = nullptr;
};

void fmm_free(FmmJobMem &m) {
  void *ptrs[] = {m.keys, m.keys_sorted, m.idx, m.perm, m.sort_tmp, m.pts, m.cell, m.parent, m.scratch,
                  m.Q, m.L, m.desc, m.m2l, m.p2p, m.front, m.seg, m.sorted, m.lsort_tmp};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  for (hipEvent_t &e : m.ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t &e : m.lev)
    if (e) (void)hipEventDestroy(e);
  m = FmmJobMem{};
}

template <typename T>
bool dev_alloc(T **p, size_t count) {
  return hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * (count ? count : 1)) == hipSuccess;
}

unsigned nblk(int64_t n, unsigned b) { return static_cast<unsigned>(std::max<int64_t>((n + b - 1) / b, 1)); }

// Interaction-list capacities: the caller's, else an estimate from the number
// of cells and theta (100 M2L and 30 P2P pairs per cell at theta = 1, growing
// as theta^-3: above what uniform points need, below clustered ones, whose
// lists then grow once; every leaf pair when theta = 0).
void fmm_list_caps(const gtap_fmm_args &a, int32_t ncells, uint64_t &m2l, uint64_t &p2p) {
  const double nc = static_cast<double>(ncells);
  double em = 0.0, ep = nc * nc;
  if (a.theta_num > 0) {
    const double s = static_cast<double>(a.theta_den) / a.theta_num;
    em = nc * 100.0 * s * s * s;
    ep = nc * 30.0 * s * s * s;
  }
  em = std::min(std::max(em, 65536.0), 4.0e9);
  ep = std::min(std::max(ep, 65536.0), 4.0e9);
  m2l = a.m2l_capacity ? a.m2l_capacity : static_cast<uint64_t>(em);
  p2p = a.p2p_capacity ? a.p2p_capacity : static_cast<uint64_t>(ep);
}

// Sort, octree, P2M and M2M of one FMM job; fills the device descriptor.
int fmm_prepare(gtap_ctx *c, const gtap_fmm_args &a, FmmJobMem &m) {
  hipStream_t st = c->stream;
  const int32_t n = a.n;
  for (hipEvent_t &e : m.ev)
    if (hipEventCreate(&e) != hipSuccess) return GTAP_E_HIP;
  if (!dev_alloc(&m.keys, n) || !dev_alloc(&m.keys_sorted, n) || !dev_alloc(&m.idx, n) ||
      !dev_alloc(&m.perm, n) || !dev_alloc(&m.pts, 5 * static_cast<size_t>(n)) ||
      !dev_alloc(&m.scratch, 11 * (static_cast<size_t>(n) + 1) + 2))
    return GTAP_E_NOMEM;
  int32_t *nch = m.scratch, *off = nch + (n + 1), *bnd = off + (n + 1), *flags = bnd + 9 * (static_cast<size_t>(n) + 1);
  double *px = m.pts, *py = px + n, *pz = py + n, *pq = pz + n, *phi = pq + n;
  if (hipEventRecord(m.ev[0], st) != hipSuccess) return GTAP_E_HIP;
  if (hipMemsetAsync(flags, 0, 2 * sizeof(int32_t), st) != hipSuccess) return GTAP_E_HIP;
  hipLaunchKernelGGL(fmm::k_keys, dim3(nblk(n, 256)), dim3(256), 0, st, n, a.x_dev, a.y_dev, a.z_dev, m.keys,
                     m.idx, flags + 1);
  size_t tmp_bytes = 0;
  if (rocprim::radix_sort_pairs(nullptr, tmp_bytes, m.keys, m.keys_sorted, m.idx, m.perm,
                                static_cast<size_t>(n), 0, 63, st) != hipSuccess)
    return GTAP_E_HIP;
  if (hipMalloc(&m.sort_tmp, tmp_bytes ? tmp_bytes : 1) != hipSuccess) return GTAP_E_NOMEM;
  if (rocprim::radix_sort_pairs(m.sort_tmp, tmp_bytes, m.keys, m.keys_sorted, m.idx, m.perm,
                                static_cast<size_t>(n), 0, 63, st) != hipSuccess)
    return GTAP_E_HIP;
  hipLaunchKernelGGL(fmm::k_gather, dim3(nblk(n, 256)), dim3(256), 0, st, n, m.perm, a.x_dev, a.y_dev, a.z_dev,
                     a.q_dev, px, py, pz, pq, phi);
  // octree, one level at a time (the host learns each level's size)
  m.cell_cap = 2 * static_cast<int64_t>(n) + 64;
  if (!dev_alloc(&m.cell, static_cast<size_t>(m.cell_cap) * fmm::kCellInts) ||
      !dev_alloc(&m.parent, static_cast<size_t>(m.cell_cap)))
    return GTAP_E_NOMEM;
  hipLaunchKernelGGL(fmm::k_root, dim3(1), dim3(64), 0, st, m.cell, m.parent, n);
  int32_t lo = 0, hi = 1;
  m.levels.clear();
  m.levels.emplace_back(lo, hi);
  for (;;) {
    const int32_t w = hi - lo;
    hipLaunchKernelGGL(fmm::k_level_count, dim3(nblk(w, 256)), dim3(256), 0, st, m.cell, lo, hi, m.keys_sorted,
                       a.leaf_max, nch, bnd);
    hipLaunchKernelGGL(fmm::k_scan, dim3(1), dim3(1024), 0, st, nch, off, w, flags);
    int32_t hf[2] = {0, 0};
    if (hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return GTAP_E_HIP;
    if (hf[1] != 0) return GTAP_E_INVAL;  // a point outside the root cube
    const int32_t total = hf[0];
    if (total == 0) break;
    if (hi + static_cast<int64_t>(total) > m.cell_cap) {
      const int64_t cap2 = std::max<int64_t>(2 * m.cell_cap, hi + static_cast<int64_t>(total) + 64);
      int32_t *c2 = nullptr, *p2 = nullptr;
      if (!dev_alloc(&c2, static_cast<size_t>(cap2) * fmm::kCellInts) || !dev_alloc(&p2, static_cast<size_t>(cap2)))
        return GTAP_E_NOMEM;
      if (hipMemcpyAsync(c2, m.cell, sizeof(int32_t) * fmm::kCellInts * hi, hipMemcpyDeviceToDevice, st) !=
              hipSuccess ||
          hipMemcpyAsync(p2, m.parent, sizeof(int32_t) * hi, hipMemcpyDeviceToDevice, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return GTAP_E_HIP;
      (void)hipFree(m.cell);
      (void)hipFree(m.parent);
      m.cell = c2;
      m.parent = p2;
      m.cell_cap = cap2;
    }
    hipLaunchKernelGGL(fmm::k_level_write, dim3(nblk(w, 256)), dim3(256), 0, st, m.cell, m.parent, lo, hi, nch,
                       off, bnd);
    lo = hi;
    hi += total;
    m.levels.emplace_back(lo, hi);
  }
  m.ncells = hi;
  if (hipEventRecord(m.ev[1], st) != hipSuccess) return GTAP_E_HIP;
  if (!dev_alloc(&m.Q, static_cast<size_t>(m.ncells) * fmm::kNc) ||
      !dev_alloc(&m.L, static_cast<size_t>(m.ncells) * fmm::kNc))
    return GTAP_E_NOMEM;
  if (hipMemsetAsync(m.L, 0, sizeof(double) * fmm::kNc * m.ncells, st) != hipSuccess) return GTAP_E_HIP;
  hipLaunchKernelGGL(fmm::k_p2m, dim3(m.ncells), dim3(128), 0, st, m.cell, 0, m.ncells, px, py, pz, pq, m.Q);
  for (size_t l = m.levels.size(); l-- > 0;) {
    const auto [l0, l1] = m.levels[l];
    hipLaunchKernelGGL(fmm::k_m2m, dim3(l1 - l0), dim3(128), 0, st, m.cell, l0, l1, m.Q);
  }
  if (hipEventRecord(m.ev[2], st) != hipSuccess) return GTAP_E_HIP;
  fmm::FmmDesc d{};
  d.cell = m.cell;
  d.Q = m.Q;
  d.L = m.L;
  d.px = px;
  d.py = py;
  d.pz = pz;
  d.pq = pq;
  d.phi = phi;
  d.ta = a.theta_num;
  d.tb = a.theta_den;
  d.ncells = static_cast<uint32_t>(m.ncells);
  if (a.traversal != GTAP_FMM_TASKS) {
    fmm_list_caps(a, m.ncells, m.m2l_cap, m.p2p_cap);
    if (a.traversal == GTAP_FMM_LISTS && !a.m2l_capacity && !a.p2p_capacity) {
      // every wavefront may hold a partly filled chunk of each list
      m.m2l_cap += static_cast<uint64_t>(c->nwaves) * fmm::kListChunk;
      m.p2p_cap += static_cast<uint64_t>(c->nwaves) * fmm::kListChunk;
    }
    if (!dev_alloc(&m.m2l, m.m2l_cap) || !dev_alloc(&m.p2p, m.p2p_cap)) return GTAP_E_NOMEM;
    d.m2l_list = m.m2l;
    d.p2p_list = m.p2p;
    d.m2l_cap = m.m2l_cap;
    d.p2p_cap = m.p2p_cap;
  }
  m.hdesc = d;
  if (!dev_alloc(&m.desc, 1)) return GTAP_E_NOMEM;
  if (hipMemcpyAsync(m.desc, &d, sizeof(d), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return GTAP_E_HIP;
  return hipGetLastError() == hipSuccess ? GTAP_OK : GTAP_E_HIP;
}

// Give the lists room for need_m2l / need_p2p pairs (plus a quarter), clear
// their counters and the descriptor's statistics.
int fmm_grow_lists(gtap_ctx *c, FmmJobMem &m, uint64_t need_m2l, uint64_t need_p2p) {
  if (need_m2l > m.m2l_cap) {
    (void)hipFree(m.m2l);
    m.m2l = nullptr;
    m.m2l_cap = need_m2l + need_m2l / 4 + 1024;
    if (!dev_alloc(&m.m2l, m.m2l_cap)) return GTAP_E_NOMEM;
  }
  if (need_p2p > m.p2p_cap) {
    (void)hipFree(m.p2p);
    m.p2p = nullptr;
    m.p2p_cap = need_p2p + need_p2p / 4 + 1024;
    if (!dev_alloc(&m.p2p, m.p2p_cap)) return GTAP_E_NOMEM;
  }
  fmm::FmmDesc &d = m.hdesc;
  d.m2l_list = m.m2l;
  d.p2p_list = m.p2p;
  d.m2l_cap = m.m2l_cap;
  d.p2p_cap = m.p2p_cap;
  d.m2l_n = d.p2p_n = 0;
  d.m2l_pairs = d.p2p_pairs = d.m2l_hash = d.p2p_hash = d.p2p_inter = d.coincident = 0;
  if (hipMemcpyAsync(m.desc, &d, sizeof(d), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return GTAP_E_HIP;
  return GTAP_OK;
}

// The list counters after a traversal (they count past the capacities).
int fmm_list_counts(gtap_ctx *c, const FmmJobMem &m, uint64_t &n_m2l, uint64_t &n_p2p) {
  uint64_t v[2] = {0, 0};
  static_assert(offsetof(fmm::FmmDesc, p2p_n) == offsetof(fmm::FmmDesc, m2l_n) + sizeof(uint64_t), "counters");
  if (hipMemcpyAsync(v, &m.desc->m2l_n, sizeof(v), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return GTAP_E_HIP;
  n_m2l = v[0];
  n_p2p = v[1];
  return GTAP_OK;
}

// Level-synchronous worklist traversal (the GPU baseline of Sec. 6.4.1): one
// launch per frontier, the host reads the next frontier's size after each.
// A frontier or list overflow re-runs it with room to spare.
int fmm_worklist(gtap_ctx *c, FmmJobMem &m) {
  hipStream_t st = c->stream;
  for (hipEvent_t &e : m.lev)
    if (!e && hipEventCreate(&e) != hipSuccess) return GTAP_E_HIP;
  if (!m.front) {
    // a frontier holds the pairs of one level (grown and re-run if not)
    m.front_cap = std::max<uint64_t>(1u << 20, (m.m2l_cap + m.p2p_cap) / 2);
    if (!dev_alloc(&m.front, 2 * m.front_cap + 1)) return GTAP_E_NOMEM;
  }
  for (int attempt = 0; attempt < 4; ++attempt) {
    if (hipEventRecord(m.lev[0], st) != hipSuccess) return GTAP_E_HIP;
    if (hipMemsetAsync(m.front, 0, sizeof(uint64_t), st) != hipSuccess) return GTAP_E_HIP;  // pair (root, root)
    uint64_t nin = 1, nout = 0;
    int64_t rounds = 0;
    bool over = false;
    while (nin > 0) {
      uint64_t *fin = m.front + (rounds & 1) * m.front_cap, *fout = m.front + ((rounds + 1) & 1) * m.front_cap;
      uint64_t *cnt = m.front + 2 * m.front_cap;
      if (hipMemsetAsync(cnt, 0, sizeof(uint64_t), st) != hipSuccess) return GTAP_E_HIP;
      hipLaunchKernelGGL(fmm::k_dtt_frontier,
                         dim3(static_cast<unsigned>((nin + fmm::kFrontierThreads - 1) / fmm::kFrontierThreads)),
                         dim3(fmm::kFrontierThreads), 0, st, m.desc, fin, nin, fout, cnt, m.front_cap);
      if (hipMemcpyAsync(&nout, cnt, sizeof(nout), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return GTAP_E_HIP;
      ++rounds;
      if (nout > m.front_cap) {
        over = true;
        break;
      }
      nin = nout;
    }
    if (hipEventRecord(m.lev[1], st) != hipSuccess) return GTAP_E_HIP;
    uint64_t n_m2l = 0, n_p2p = 0;
    int rc = fmm_list_counts(c, m, n_m2l, n_p2p);
    if (rc) return rc;
    m.rounds = rounds;
    if (!over && n_m2l <= m.m2l_cap && n_p2p <= m.p2p_cap) {
      (void)hipEventElapsedTime(&m.worklist_ms, m.lev[0], m.lev[1]);
      return GTAP_OK;
    }
    ++m.retries;
    if (over) {
      (void)hipFree(m.front);
      m.front = nullptr;
      m.front_cap = 2 * nout;
      if (!dev_alloc(&m.front, 2 * m.front_cap + 1)) return GTAP_E_NOMEM;
    }
    rc = fmm_grow_lists(c, m, over ? 0 : n_m2l, over ? 0 : n_p2p);
    if (rc) return rc;
  }
  return GTAP_E_CAPACITY;
}

// Sort both lists by target, find each target's segment and evaluate: M2L into
// the local expansions, P2P into the sorted-order potentials; the pair counts,
// hashes, interactions and coincident pairs go to the descriptor.
int fmm_eval_lists(gtap_ctx *c, FmmJobMem &m, uint64_t n_m2l, uint64_t n_p2p, gtap_fmm_result &r) {
  hipStream_t st = c->stream;
  for (hipEvent_t &e : m.lev)
    if (!e && hipEventCreate(&e) != hipSuccess) return GTAP_E_HIP;
  const uint64_t nmax = std::max<uint64_t>(std::max(n_m2l, n_p2p), 1);
  unsigned end_bit = 32;
  while (end_bit < 64 && (static_cast<uint64_t>(m.ncells) >> (end_bit - 32)) != 0) ++end_bit;
  size_t tmp_bytes = 0;
  if (rocprim::radix_sort_keys(nullptr, tmp_bytes, m.m2l, m.m2l, static_cast<size_t>(nmax), 32, end_bit, st) !=
      hipSuccess)
    return GTAP_E_HIP;
  // segments of targets 0..ncells (ncells: the gaps of chunked appends)
  const size_t nseg = static_cast<size_t>(m.ncells) + 1;
  if (!dev_alloc(&m.sorted, nmax) || !dev_alloc(&m.seg, 2 * nseg) ||
      hipMalloc(&m.lsort_tmp, tmp_bytes ? tmp_bytes : 1) != hipSuccess)
    return GTAP_E_NOMEM;
  uint64_t *lo = m.seg, *hi = m.seg + nseg;
  fmm::FmmDesc *D = m.desc;
  auto prepare = [&](uint64_t *list, uint64_t cnt, uint64_t *hash, uint64_t *pairs) -> int {
    if (hipMemsetAsync(m.seg, 0, sizeof(uint64_t) * 2 * nseg, st) != hipSuccess) return GTAP_E_HIP;
    if (cnt == 0) return GTAP_OK;
    size_t tb = tmp_bytes;
    if (rocprim::radix_sort_keys(m.lsort_tmp, tb, list, m.sorted, static_cast<size_t>(cnt), 32, end_bit, st) !=
        hipSuccess)
      return GTAP_E_HIP;
    hipLaunchKernelGGL(fmm::k_list_segments, dim3(nblk(static_cast<int64_t>(cnt), 256)), dim3(256), 0, st, m.sorted,
                       cnt, lo, hi);
    hipLaunchKernelGGL(fmm::k_list_hash, dim3(1024), dim3(256), 0, st, m.sorted, cnt,
                       static_cast<uint32_t>(m.ncells), hash, pairs);
    return GTAP_OK;
  };
  int rc = GTAP_OK;
  if (hipEventRecord(m.lev[2], st) != hipSuccess) return GTAP_E_HIP;
  if ((rc = prepare(m.m2l, n_m2l, &D->m2l_hash, &D->m2l_pairs))) return rc;
  if (hipEventRecord(m.lev[3], st) != hipSuccess) return GTAP_E_HIP;
  hipLaunchKernelGGL(fmm::k_scale_moments, dim3(nblk(static_cast<int64_t>(m.ncells) * fmm::kNc, 256)), dim3(256), 0,
                     st, m.Q, static_cast<int64_t>(m.ncells));
  hipLaunchKernelGGL(fmm::k_m2l_list, dim3(m.ncells), dim3(fmm::kM2LThreads), 0, st, m.hdesc.cell, m.hdesc.Q,
                     m.hdesc.L, m.sorted, lo, hi);
  if (hipEventRecord(m.lev[4], st) != hipSuccess) return GTAP_E_HIP;
  if ((rc = prepare(m.p2p, n_p2p, &D->p2p_hash, &D->p2p_pairs))) return rc;
  if (hipEventRecord(m.lev[5], st) != hipSuccess) return GTAP_E_HIP;
  hipLaunchKernelGGL(fmm::k_p2p_list, dim3(nblk(static_cast<int64_t>((n_p2p + kWave - 1) / kWave), fmm::kP2PThreads / kWave)),
                     dim3(fmm::kP2PThreads), 0, st, m.hdesc.cell, m.hdesc.px, m.hdesc.py, m.hdesc.pz, m.hdesc.pq,
                     m.hdesc.phi, m.sorted, n_p2p, static_cast<uint32_t>(m.ncells), &D->p2p_inter, &D->coincident);
  if (hipEventRecord(m.lev[6], st) != hipSuccess) return GTAP_E_HIP;
  if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) return GTAP_E_HIP;
  float s1 = 0.f, mm = 0.f, s2 = 0.f, pp = 0.f;
  (void)hipEventElapsedTime(&s1, m.lev[2], m.lev[3]);
  (void)hipEventElapsedTime(&mm, m.lev[3], m.lev[4]);
  (void)hipEventElapsedTime(&s2, m.lev[4], m.lev[5]);
  (void)hipEventElapsedTime(&pp, m.lev[5], m.lev[6]);
  r.sort_ms = s1 + s2;
  r.m2l_ms = mm;
  r.p2p_ms = pp;
  return GTAP_OK;
}

// L2L, L2P and the scatter to the caller's order; statistics into r.
int fmm_finish(gtap_ctx *c, const gtap_fmm_args &a, FmmJobMem &m, float traversal_ms, gtap_fmm_result &r) {
  hipStream_t st = c->stream;
  const int32_t n = a.n;
  double *px = m.pts, *py = px + n, *pz = py + n, *phi = pz + 2 * static_cast<size_t>(n);
  if (hipEventRecord(m.ev[3], st) != hipSuccess) return GTAP_E_HIP;
  for (size_t l = 1; l < m.levels.size(); ++l) {
    const auto [l0, l1] = m.levels[l];
    hipLaunchKernelGGL(fmm::k_l2l, dim3(l1 - l0), dim3(128), 0, st, m.cell, m.parent, l0, l1, m.L);
  }
  hipLaunchKernelGGL(fmm::k_l2p, dim3(m.ncells), dim3(128), 0, st, m.cell, 0, m.ncells, m.L, px, py, pz, phi);
  hipLaunchKernelGGL(fmm::k_scatter, dim3(nblk(n, 256)), dim3(256), 0, st, n, m.perm, phi, a.phi_dev);
  if (hipEventRecord(m.ev[4], st) != hipSuccess) return GTAP_E_HIP;
  fmm::FmmDesc d{};
  std::vector<int32_t> cells(static_cast<size_t>(m.ncells) * fmm::kCellInts);
  if (hipMemcpyAsync(&d, m.desc, sizeof(d), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(cells.data(), m.cell, sizeof(int32_t) * cells.size(), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return GTAP_E_HIP;
  r = gtap_fmm_result{};
  r.n_cells = m.ncells;
  for (int32_t i = 0; i < m.ncells; ++i) r.n_leaves += cells[static_cast<size_t>(i) * fmm::kCellInts + 7] == 0;
  r.max_level = static_cast<int64_t>(m.levels.size()) - 1;
  r.m2l_pairs = static_cast<int64_t>(d.m2l_pairs);
  r.p2p_pairs = static_cast<int64_t>(d.p2p_pairs);
  r.m2l_hash = d.m2l_hash;
  r.p2p_hash = d.p2p_hash;
  r.p2p_interactions = static_cast<int64_t>(d.p2p_inter);
  r.coincident = static_cast<int64_t>(d.coincident);
  float t0 = 0.f, t1 = 0.f, t2 = 0.f;
  (void)hipEventElapsedTime(&t0, m.ev[0], m.ev[1]);
  (void)hipEventElapsedTime(&t1, m.ev[1], m.ev[2]);
  (void)hipEventElapsedTime(&t2, m.ev[3], m.ev[4]);
  r.tree_ms = t0;
  r.upward_ms = t1;
  r.traversal_ms = traversal_ms;
  r.downward_ms = t2;
  return hipGetLastError() == hipSuccess ? GTAP_OK : GTAP_E_HIP;
}

}  // namespace

extern "C" {

int gtap_run(gtap_ctx *c) {
  if (!c) return GTAP_E_INVAL;
  if (c->serving) return GTAP_E_STATE;
  const size_t nj = c->pending.size();
  c->err = gtap_error_report{};
  if (nj == 0) return GTAP_OK;
  Params &p = c->params;
  p.njobs = static_cast<uint32_t>(nj);
  p.serving = 0;
  const bool block = c->cfg.mode == GTAP_MODE_BLOCK;
  // FMM jobs: tree and upward pass before the launch; the worklist traversal
  // runs here too (its root task in the launch is empty)
  std::vector<FmmJobMem> fm;
  bool any_fmm = false;
  uint32_t ext = 0;  // extension task sets the batch needs
  for (size_t j = 0; j < nj; ++j) {
    any_fmm |= c->pending[j].kind == GTAP_KIND_FMM;
    if (c->pending[j].kind == GTAP_KIND_FMM || c->pending[j].kind == GTAP_KIND_CILKSORT) ext |= kExtLists;
    if (c->pending[j].kind == GTAP_KIND_KCLIQUE_SPLIT) ext |= kExtSplit;
  }
  std::vector<void *> ks_mem;
  auto drop_pending = [&]() {
    for (FmmJobMem &m : fm) fmm_free(m);
    for (void *q : ks_mem) (void)hipFree(q);
    c->pending.clear();
    c->pending_fmm.clear();
    c->pending_ks.clear();
  };
  // split k-clique jobs: offsets and bit matrices in one device buffer
  for (size_t j = 0; j < nj; ++j) {
    const std::vector<uint64_t> &off = c->pending_ks[j];
    if (c->pending[j].kind != GTAP_KIND_KCLIQUE_SPLIT || off.empty()) continue;
    void *q = nullptr;
    const size_t words = off.size() + off.back();
    if (hipMalloc(&q, words * sizeof(uint64_t)) != hipSuccess) {
      drop_pending();
      return GTAP_E_NOMEM;
    }
    ks_mem.push_back(q);
    if (hipMemcpyAsync(q, off.data(), off.size() * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream) !=
        hipSuccess) {
      drop_pending();
      return GTAP_E_HIP;
    }
    c->pending[j].a[7] = reinterpret_cast<uint64_t>(q);
  }
  if (any_fmm) {
    fm.resize(nj);
    for (size_t j = 0; j < nj; ++j) {
      if (c->pending[j].kind != GTAP_KIND_FMM) continue;
      const gtap_fmm_args &a = c->pending_fmm[j];
      int rc = fmm_prepare(c, a, fm[j]);
      if (rc == GTAP_OK && a.traversal == GTAP_FMM_WORKLIST) rc = fmm_worklist(c, fm[j]);
      if (rc != GTAP_OK) {
        drop_pending();
        return rc;
      }
      c->pending[j].a[0] = reinterpret_cast<uint64_t>(fm[j].desc);
      if (block) {
        c->pending[j].pending = 1;  // the root cell pair
      } else {
        c->pending[j].a[1] = static_cast<uint64_t>(a.traversal);
        c->pending[j].a[2] = static_cast<uint64_t>(a.theta_num) | (static_cast<uint64_t>(a.theta_den) << 8);
      }
    }
  }
  // one launch; a list-building traversal whose lists overflowed is re-run
  // with lists that fit (every job of the batch runs again)
  Control ctl;
  float ms = 0.f;
  int rc = GTAP_OK;
  for (int attempt = 0;; ++attempt) {
    if (hipMemcpyAsync(p.jobs, c->pending.data(), nj * sizeof(JobSlot), hipMemcpyHostToDevice, c->stream) !=
        hipSuccess) {
      drop_pending();
      return GTAP_E_HIP;
    }
    const uint32_t ndq = c->nwaves * p.Q;
    hipLaunchKernelGGL(reset_kernel, dim3(reset_blocks(ndq, p.ccap)), dim3(256), 0, c->stream, p, ndq);
    if (hipGetLastError() != hipSuccess || hipEventRecord(c->ev0, c->stream) != hipSuccess) rc = GTAP_E_HIP;
    if (rc == GTAP_OK) rc = launch_sched(c, block ? 0u : ext);
    if (rc == GTAP_OK && hipEventRecord(c->ev1, c->stream) != hipSuccess) rc = GTAP_E_HIP;
    if (rc != GTAP_OK) {
      (void)hipStreamSynchronize(c->stream);
      drop_pending();
      return rc;
    }
    c->done_jobs.resize(nj);
    if (hipMemcpyAsync(c->done_jobs.data(), p.jobs, nj * sizeof(JobSlot), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipMemcpyAsync(&ctl, p.ctl, sizeof(Control), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
      drop_pending();
      return GTAP_E_HIP;
    }
    (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
    bool again = false;
    if (ctl.error == 0 && any_fmm && !block) {
      std::vector<std::pair<uint64_t, uint64_t>> counts(nj, {0, 0});
      for (size_t j = 0; j < nj && rc == GTAP_OK; ++j) {
        if (c->pending[j].kind != GTAP_KIND_FMM || c->pending_fmm[j].traversal != GTAP_FMM_LISTS) continue;
        rc = fmm_list_counts(c, fm[j], counts[j].first, counts[j].second);
        if (counts[j].first > fm[j].m2l_cap || counts[j].second > fm[j].p2p_cap) again = true;
      }
      if (rc == GTAP_OK && again && attempt >= 2) rc = GTAP_E_CAPACITY;
      // every list-building job runs again: its lists grow if needed, its
      // counters restart
      for (size_t j = 0; j < nj && rc == GTAP_OK && again; ++j) {
        if (c->pending[j].kind != GTAP_KIND_FMM || c->pending_fmm[j].traversal != GTAP_FMM_LISTS) continue;
        rc = fmm_grow_lists(c, fm[j], counts[j].first, counts[j].second);
        ++fm[j].retries;
      }
    }
    if (rc != GTAP_OK) {
      drop_pending();
      return rc;
    }
    if (!again) break;
  }
  c->done_first = c->pending_first;
  c->have_done = true;

  const int rc_run = record_run(c, ctl, ms);
  for (size_t j = 0; rc_run == GTAP_OK && j < nj; ++j)
    if (c->done_jobs[j].done != 1) rc = GTAP_E_STATE;
  if (rc_run == GTAP_OK && rc == GTAP_OK && any_fmm) {
    c->done_fmm.assign(nj, gtap_fmm_result{});
    for (size_t j = 0; j < nj && rc == GTAP_OK; ++j) {
      if (c->pending[j].kind != GTAP_KIND_FMM) continue;
      const gtap_fmm_args &a = c->pending_fmm[j];
      FmmJobMem &m = fm[j];
      gtap_fmm_result ev{};
      if (a.traversal != GTAP_FMM_TASKS) {
        uint64_t n_m2l = 0, n_p2p = 0;
        rc = fmm_list_counts(c, m, n_m2l, n_p2p);
        if (rc == GTAP_OK) rc = fmm_eval_lists(c, m, n_m2l, n_p2p, ev);
      }
      const float trav = a.traversal == GTAP_FMM_WORKLIST ? m.worklist_ms : ms;
      if (rc == GTAP_OK) rc = fmm_finish(c, a, m, trav, c->done_fmm[j]);
      gtap_fmm_result &r = c->done_fmm[j];
      r.sort_ms = ev.sort_ms;
      r.m2l_ms = ev.m2l_ms;
      r.p2p_ms = ev.p2p_ms;
      r.dtt_rounds = m.rounds;
      r.list_retries = m.retries;
    }
  }
  drop_pending();
  if (rc_run != GTAP_OK || rc != GTAP_OK) {
    c->have_done = false;
    return rc_run != GTAP_OK ? rc_run : rc;
  }
  return GTAP_OK;
}

// ---- serving -------------------------------------------------------------
static double host_seconds() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

int gtap_serve_start(gtap_ctx *c, uint32_t max_inflight, uint32_t headroom_small, uint32_t headroom_big) {
  if (!c) return GTAP_E_INVAL;
  if (c->serving || !c->pending.empty()) return GTAP_E_STATE;
  if (c->cfg.mode != GTAP_MODE_THREAD || c->cfg.flags != 0) return GTAP_E_INVAL;
  if (max_inflight == 0 || max_inflight > c->cfg.max_jobs) return GTAP_E_INVAL;
  const size_t R = c->cfg.max_jobs;
  if (!c->ring) {
    const unsigned fl = hipHostMallocCoherent | hipHostMallocMapped;
    if (hipHostMalloc(reinterpret_cast<void **>(&c->ring), R * sizeof(JobSlot), fl) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&c->ring_seq), R * sizeof(uint64_t), fl) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&c->done_host), R * sizeof(HostCompletion), fl) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&c->stop_host), 64, fl) != hipSuccess)
      return GTAP_E_NOMEM;
  }
  std::memset(c->ring, 0, R * sizeof(JobSlot));
  std::memset(c->ring_seq, 0, R * sizeof(uint64_t));
  std::memset(c->done_host, 0, R * sizeof(HostCompletion));
  __atomic_store_n(c->stop_host, 0, __ATOMIC_RELEASE);
  c->next_ticket = 0;
  c->err = gtap_error_report{};
  Params &p = c->params;
  p.njobs = 0;
  p.serving = 1;
  p.ring_cap = static_cast<uint32_t>(R);
  p.ring = c->ring;
  p.ring_seq = c->ring_seq;
  p.done_host = c->done_host;
  p.stop_host = c->stop_host;
  p.max_inflight = max_inflight;
  p.admit_headroom_small = headroom_small;
  p.admit_headroom_big = headroom_big;
  const uint32_t ndq = c->nwaves * p.Q;
  hipLaunchKernelGGL(reset_kernel, dim3(reset_blocks(ndq, p.ccap)), dim3(256), 0, c->stream, p, ndq);
  if (hipGetLastError() != hipSuccess) return GTAP_E_HIP;
  if (hipEventRecord(c->ev0, c->stream) != hipSuccess) return GTAP_E_HIP;
  const int rc = launch_sched(c);
  if (rc) return rc;
  if (hipEventRecord(c->ev1, c->stream) != hipSuccess) return GTAP_E_HIP;
  c->serving = true;
  c->have_done = false;
  return GTAP_OK;
}

int gtap_serve_submit(gtap_ctx *c, int32_t kind, const void *args, size_t args_bytes, uint64_t *ticket) {
  if (!c || !ticket) return GTAP_E_INVAL;
  if (!c->serving) return GTAP_E_STATE;
  // the serving kernel runs the scheduler as designed: no FMM, no Cilksort,
  // no split k-clique search
  if (kind == GTAP_KIND_FMM || kind == GTAP_KIND_CILKSORT || kind == GTAP_KIND_KCLIQUE_SPLIT) return GTAP_E_INVAL;
  JobSlot J;
  const int rc = pack_job(c->cfg, c->stream, kind, args, args_bytes, J);
  if (rc) return rc;
  const uint64_t t = c->next_ticket;
  const uint64_t R = c->params.ring_cap;
  const uint64_t slot = t % R;
  // the slot's previous job (ticket t - R) must have completed
  if (t >= R && __atomic_load_n(&c->done_host[slot].done, __ATOMIC_ACQUIRE) != t - R + 1) return GTAP_E_FULL;
  std::memcpy(&c->ring[slot], &J, sizeof(J));
  __atomic_store_n(&c->ring_seq[slot], t + 1, __ATOMIC_RELEASE);
  c->next_ticket = t + 1;
  *ticket = t;
  return GTAP_OK;
}

int gtap_serve_poll(gtap_ctx *c, uint64_t ticket, int64_t *result, uint64_t *done_ticks) {
  if (!c || !c->done_host) return GTAP_E_INVAL;
  if (ticket >= c->next_ticket) return GTAP_E_NOJOB;
  const HostCompletion &h = c->done_host[ticket % c->params.ring_cap];
  if (__atomic_load_n(&h.done, __ATOMIC_ACQUIRE) != ticket + 1) return GTAP_E_PENDING;
  if (result) *result = __atomic_load_n(&h.result, __ATOMIC_RELAXED);
  if (done_ticks) *done_ticks = __atomic_load_n(&h.t_done, __ATOMIC_RELAXED);
  return GTAP_OK;
}

// True once the serving kernel has exited (it only exits early on an abort).
static bool serving_kernel_ended(gtap_ctx *c) { return hipStreamQuery(c->stream) == hipSuccess; }

int gtap_serve_stop(gtap_ctx *c, uint32_t wait_ms) {
  if (!c) return GTAP_E_INVAL;
  if (!c->serving) return GTAP_E_STATE;
  int rc = GTAP_OK;
  const double deadline = host_seconds() + wait_ms / 1000.0;
  double next_query = host_seconds() + 1e-3;
  const uint64_t R = c->params.ring_cap;
  bool ended = false;
  for (uint64_t t = (c->next_ticket > R ? c->next_ticket - R : 0); t < c->next_ticket && !ended; ++t) {
    while (__atomic_load_n(&c->done_host[t % R].done, __ATOMIC_ACQUIRE) != t + 1) {
      const double now = host_seconds();
      if (now > deadline) {
        rc = GTAP_E_TIMEOUT;
        break;
      }
      if (now > next_query) {
        next_query = now + 1e-3;
        if (serving_kernel_ended(c)) {
          ended = true;  // aborted: the device's error code is returned below
          break;
        }
      }
      std::this_thread::yield();
    }
    if (rc) break;
  }
  __atomic_store_n(c->stop_host, 1, __ATOMIC_RELEASE);
  Control ctl;
  if (hipMemcpyAsync(&ctl, c->params.ctl, sizeof(Control), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    c->serving = false;
    return GTAP_E_HIP;
  }
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
  c->serving = false;
  c->params.serving = 0;
  const int rr = record_run(c, ctl, ms);
  return rr != GTAP_OK ? rr : rc;
}

int gtap_trace_run(gtap_ctx *c, const gtap_trace_job *jobs, size_t n, gtap_trace_result *out, uint32_t timeout_ms) {
  if (!c || (n && (!jobs || !out))) return GTAP_E_INVAL;
  if (!c->serving) return GTAP_E_STATE;
  std::vector<uint64_t> ticket(n, 0);
  std::vector<size_t> open;
  open.reserve(n);
  const double t0 = host_seconds();
  const double deadline = t0 + timeout_ms / 1000.0;
  size_t next = 0, done = 0;
  double next_query = 1e-3;
  for (size_t i = 0; i < n; ++i) out[i] = gtap_trace_result{0, -1.0, -1.0, GTAP_E_PENDING, 0};
  while (done < n) {
    double now = host_seconds() - t0;
    if (now > next_query) {
      next_query = now + 1e-3;
      // the kernel exited early: it aborted; end the session and report why
      if (serving_kernel_ended(c)) {
        const int rc = gtap_serve_stop(c, 0);
        return rc != GTAP_OK ? rc : GTAP_E_STATE;
      }
    }
    while (next < n && jobs[next].arrival_s <= now) {
      const gtap_trace_job &J = jobs[next];
      if (J.args_bytes > sizeof(J.args)) return GTAP_E_INVAL;
      const int rc = gtap_serve_submit(c, J.kind, J.args, J.args_bytes, &ticket[next]);
      if (rc == GTAP_E_FULL) break;  // retry once a slot frees up
      if (rc != GTAP_OK) {
        out[next].status = rc;
        return rc;
      }
      out[next].submit_s = now;
      open.push_back(next);
      ++next;
    }
    size_t w = 0;
    for (size_t k = 0; k < open.size(); ++k) {
      const size_t i = open[k];
      int64_t r = 0;
      if (gtap_serve_poll(c, ticket[i], &r, nullptr) == GTAP_OK) {
        out[i].result = r;
        out[i].done_s = host_seconds() - t0;
        out[i].status = GTAP_OK;
        ++done;
      } else {
        open[w++] = i;
      }
    }
    open.resize(w);
    if (host_seconds() > deadline) return GTAP_E_TIMEOUT;
    if (open.empty() && next < n) {
      // nothing in flight: sleep until shortly before the next arrival
      const double gap = jobs[next].arrival_s - (host_seconds() - t0);
      if (gap > 2e-4) std::this_thread::sleep_for(std::chrono::duration<double>(gap - 1e-4));
    }
  }
  return GTAP_OK;
}

int gtap_trace_run_plain(gtap_ctx *c, const gtap_trace_job *jobs, size_t n, gtap_trace_result *out) {
  if (!c || (n && (!jobs || !out))) return GTAP_E_INVAL;
  if (c->serving || !c->pending.empty()) return GTAP_E_STATE;
  const double t0 = host_seconds();
  for (size_t i = 0; i < n; ++i) {
    const gtap_trace_job &J = jobs[i];
    while (host_seconds() - t0 < J.arrival_s) {
    }
    out[i].submit_s = host_seconds() - t0;
    uint64_t id = 0;
    int rc = gtap_submit(c, J.kind, J.args, J.args_bytes, &id);
    if (rc == GTAP_OK) rc = gtap_run(c);
    int64_t r = 0;
    if (rc == GTAP_OK) rc = gtap_result(c, id, &r, sizeof(r));
    out[i].result = r;
    out[i].done_s = host_seconds() - t0;
    out[i].status = rc;
    if (rc != GTAP_OK) return rc;
  }
  return GTAP_OK;
}

// ---- autotuner ------------------------------------------------------------------
// Best wall time (ms) of `repeats` timed batches of the calibration jobs under
// cfg; pools grow on exhaustion.  Returns GTAP_OK or the last failure.
static int tune_candidate(gtap_config &cfg, const gtap_trace_job *jobs, size_t n, uint32_t repeats,
                          double *best_ms, gtap_stats *st) {
  int rc = GTAP_OK;
  for (int attempt = 0; attempt < 4; ++attempt) {
    gtap_ctx *c = nullptr;
    rc = gtap_init(&cfg, &c);
    if (rc != GTAP_OK) return rc;
    double best = 1e300;
    for (uint32_t r = 0; r <= repeats && rc == GTAP_OK; ++r) {
      for (size_t i = 0; i < n && rc == GTAP_OK; ++i) {
        uint64_t id = 0;
        rc = gtap_submit(c, jobs[i].kind, jobs[i].args, jobs[i].args_bytes, &id);
      }
      if (rc != GTAP_OK) break;
      const double t0 = host_seconds();
      rc = gtap_run(c);
      const double t1 = host_seconds();
      if (rc == GTAP_OK && r > 0) best = std::min(best, 1e3 * (t1 - t0));
    }
    const gtap_error_report err = c->err;
    if (st) *st = c->stats;
    gtap_finalize(c);
    if (rc == GTAP_OK) {
      *best_ms = best;
      return GTAP_OK;
    }
    if (rc != GTAP_E_CAPACITY || (err.pool != 0 && err.pool != 1)) return rc;
    if (err.pool == 0) cfg.small_frames = std::min<uint64_t>(cfg.small_frames * 2, (1ull << 31) - 1);
    else cfg.big_frames = std::min<uint64_t>(std::max<uint64_t>(cfg.big_frames * 2, 1024), (1ull << 31) - 1);
  }
  return rc;
}

int gtap_autotune(const gtap_config *base, const gtap_trace_job *calib, size_t n, const gtap_tune_space *space,
                  gtap_config *best, gtap_tune_report *report) {
  if (!base || !calib || !space || !best || n == 0 || n > base->max_jobs) return GTAP_E_INVAL;
  for (size_t i = 0; i < n; ++i)
    if (calib[i].args_bytes > sizeof(calib[i].args)) return GTAP_E_INVAL;
  const uint32_t repeats = std::max<uint32_t>(space->repeats, 1);
  gtap_tune_report rep{};
  gtap_config b = *base;
  b.workspace_dev = nullptr;
  b.workspace_bytes = 0;
  gtap_stats st{};
  double base_ms = 0.0;
  int rc = tune_candidate(b, calib, n, repeats, &base_ms, &st);
  if (rc != GTAP_OK) return rc;
  rep.candidates = 1;
  rep.base_ms = base_ms;
  gtap_config win = b;
  double win_ms = base_ms;
  gtap_stats win_st = st;
  auto list = [](const int32_t *v, int32_t dflt) {
    std::vector<int32_t> out;
    for (int i = 0; i < 4 && v[i] != 0; ++i) out.push_back(v[i]);
    if (out.empty()) out.push_back(dflt);
    return out;
  };
  for (int32_t q : list(space->num_queues, b.num_queues)) {
    const std::vector<int32_t> pols =
        q > 1 ? list(space->daq_policies, GTAP_DAQ_BY_KIND) : std::vector<int32_t>{GTAP_DAQ_NONE};
    for (int32_t pol : pols) {
      const bool by_bounds = q > 1 && pol == GTAP_DAQ_KCLIQUE && space->bounds_sets > 0;
      const int nb = by_bounds ? std::min(space->bounds_sets, 4) : 1;
      for (int bi = 0; bi < nb; ++bi)
        for (int32_t wpg : list(space->waves_per_group, b.waves_per_group))
          for (int32_t nw : list(space->num_waves, b.num_waves)) {
            gtap_config cand = b;
            cand.num_queues = q;
            cand.daq_policy = pol;
            if (by_bounds) std::memcpy(cand.daq_bounds, space->bounds[bi], sizeof(cand.daq_bounds));
            cand.waves_per_group = wpg;
            cand.num_waves = nw < 0 ? 0 : nw;
            double ms = 0.0;
            ++rep.candidates;
            if (validate(cand) != GTAP_OK ||
                tune_candidate(cand, calib, n, repeats, &ms, &st) != GTAP_OK) {
              ++rep.failed;
              continue;
            }
            if (ms < win_ms) {
              win_ms = ms;
              win = cand;
              win_st = st;
            }
          }
    }
  }
  // frame pools: four times what the best run touched, at least 2^20, at most the base sizes
  auto size_pool = [](uint64_t touched, uint64_t cap) {
    uint64_t v = std::max<uint64_t>(4 * touched, 1ull << 20);
    uint64_t p2 = 1;
    while (p2 < v) p2 <<= 1;
    return std::min<uint64_t>(p2, cap);
  };
  win.small_frames = size_pool(win_st.small_frames_touched, std::max(win.small_frames, b.small_frames));
  if (win.big_frames > 0) win.big_frames = size_pool(win_st.big_frames_touched, std::max(win.big_frames, b.big_frames));
  win.workspace_dev = base->workspace_dev;
  win.workspace_bytes = base->workspace_bytes;
  win.stream = base->stream;
  rep.best_ms = win_ms;
  rep.small_frames_touched = win_st.small_frames_touched;
  rep.big_frames_touched = win_st.big_frames_touched;
  *best = win;
  if (report) *report = rep;
  return GTAP_OK;
}

int gtap_result(gtap_ctx *c, uint64_t job_id, void *out, size_t out_bytes) {
  if (!c || !out || out_bytes < sizeof(int64_t)) return GTAP_E_INVAL;
  if (c->have_done && job_id >= c->done_first && job_id < c->done_first + c->done_jobs.size()) {
    const size_t j = job_id - c->done_first;
    const JobSlot &J = c->done_jobs[j];
    if (J.kind == GTAP_KIND_FMM) {
      if (out_bytes < sizeof(gtap_fmm_result) || j >= c->done_fmm.size()) return GTAP_E_INVAL;
      std::memcpy(out, &c->done_fmm[j], sizeof(gtap_fmm_result));
      return GTAP_OK;
    }
    std::memcpy(out, &J.result, sizeof(int64_t));
    return GTAP_OK;
  }
  if (!c->pending.empty() && job_id >= c->pending_first && job_id < c->pending_first + c->pending.size())
    return GTAP_E_PENDING;
  if (job_id < c->next_job_id) return GTAP_E_PENDING;
  return GTAP_E_NOJOB;
}

int gtap_finalize(gtap_ctx *c) {
  if (!c) return GTAP_E_INVAL;
  // a serving kernel still running stops once its admitted jobs drain (or
  // its watchdog fires); the pinned buffers it reads are freed only after
  if (c->serving && c->stop_host) __atomic_store_n(c->stop_host, 1, __ATOMIC_RELEASE);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->owns_ws && c->ws) (void)hipFree(c->ws);
  if (c->ring) (void)hipHostFree(c->ring);
  if (c->ring_seq) (void)hipHostFree(c->ring_seq);
  if (c->done_host) (void)hipHostFree(c->done_host);
  if (c->stop_host) (void)hipHostFree(c->stop_host);
  delete c;
  return GTAP_OK;
}

int gtap_stats_get(gtap_ctx *c, gtap_stats *out) {
  if (!c || !out) return GTAP_E_INVAL;
  *out = c->stats;
  return GTAP_OK;
}

int gtap_last_error(gtap_ctx *c, gtap_error_report *out) {
  if (!c || !out) return GTAP_E_INVAL;
  *out = c->err;
  return GTAP_OK;
}

const char *gtap_status_string(int32_t s) {
  switch (s) {
    case GTAP_OK: return "ok";
    case GTAP_E_INVAL: return "invalid argument";
    case GTAP_E_NOMEM: return "out of device memory or workspace too small";
    case GTAP_E_HIP: return "HIP runtime error";
    case GTAP_E_STATE: return "invalid state";
    case GTAP_E_FULL: return "too many pending jobs";
    case GTAP_E_CAPACITY: return "frame pool or deque capacity exhausted";
    case GTAP_E_PENDING: return "job not completed";
    case GTAP_E_TIMEOUT: return "device watchdog expired";
    case GTAP_E_NOJOB: return "unknown job";
    default: return "unknown status";
  }
}

}  // extern "C"

// ---- platform probes ----------------------------------------------------------
namespace {

struct ProbeEvents {
  hipEvent_t a = nullptr, b = nullptr;
  ~ProbeEvents() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  bool make() { return hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess; }
};

}  // namespace

extern "C" int gtap_probe_atomics(int32_t mode, uint32_t blocks, uint32_t iters, uint64_t *words_dev,
                                  uint64_t words, void *stream_v, double *rmw_per_s, double *ms_out) {
  if (!words_dev || !rmw_per_s || blocks < 1 || blocks > 65536 || iters < 1 || iters > 65536) return GTAP_E_INVAL;
  const uint64_t need = mode == GTAP_PROBE_DISTINCT   ? static_cast<uint64_t>(blocks) * 256 * 8
                        : mode == GTAP_PROBE_PER_WAVE ? static_cast<uint64_t>(blocks) * 4 * 16
                        : mode == GTAP_PROBE_ONE_WORD ? 1
                                                      : 0;
  if (need == 0 || words < need + 1) return GTAP_E_INVAL;  // one more word: the sink
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  ProbeEvents ev;
  if (!ev.make()) return GTAP_E_HIP;
  if (hipMemsetAsync(words_dev, 0, (need + 1) * sizeof(uint64_t), stream) != hipSuccess) return GTAP_E_HIP;
  if (hipEventRecord(ev.a, stream) != hipSuccess) return GTAP_E_HIP;
  hipLaunchKernelGGL(probe::atomic_probe_kernel, dim3(blocks), dim3(256), 0, stream, words_dev,
                     static_cast<uint32_t>(mode), iters, words_dev + need);
  if (hipGetLastError() != hipSuccess || hipEventRecord(ev.b, stream) != hipSuccess ||
      hipEventSynchronize(ev.b) != hipSuccess)
    return GTAP_E_HIP;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, ev.a, ev.b) != hipSuccess || ms <= 0.f) return GTAP_E_HIP;
  const double lanes = mode == GTAP_PROBE_DISTINCT ? 256.0 * blocks : 4.0 * blocks;
  *rmw_per_s = lanes * iters / (ms * 1e-3);
  if (ms_out) *ms_out = ms;
  return GTAP_OK;
}

extern "C" int gtap_litmus(int32_t test, int32_t ordered, uint32_t pairs, uint32_t rounds, void *buf_dev,
                           uint64_t buf_bytes, void *stream_v, gtap_litmus_result *out) {
  if ((test != 0 && test != 1) || pairs < 1 || pairs > 1024 || rounds < 1 || rounds > 65536 || !buf_dev || !out)
    return GTAP_E_INVAL;
  const uint64_t inst = static_cast<uint64_t>(pairs) * kWave;
  const uint64_t need = static_cast<uint64_t>(pairs) * (16384 + 512ull * rounds) + 16384;
  if (buf_bytes < need) return GTAP_E_NOMEM;
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  char *b = static_cast<char *>(buf_dev);
  uint32_t *cells = reinterpret_cast<uint32_t *>(b);                       // inst * 256 B
  uint32_t *xcc = reinterpret_cast<uint32_t *>(b + inst * 256);            // 2 * pairs words
  unsigned long long *counts = reinterpret_cast<unsigned long long *>(b + inst * 256 + 8192);
  uint32_t *res = reinterpret_cast<uint32_t *>(b + inst * 256 + 8192 + 64);  // MP: 2 * inst; SB: 2 * inst * rounds
  const size_t clear = static_cast<size_t>(inst * 256 + 8192 + 64);
  if (hipMemsetAsync(b, 0, clear, stream) != hipSuccess) return GTAP_E_HIP;
  std::memset(out, 0, sizeof(*out));
  out->instances = inst;
  out->pairs = static_cast<int32_t>(pairs);
  const uint32_t reads = rounds * 4;
  if (test == 0) {
    uint32_t *stale = res, *mid = res + inst;
    if (ordered)
      hipLaunchKernelGGL(probe::litmus_mp_kernel<true>, dim3(2 * pairs), dim3(64), 0, stream, cells, rounds, reads,
                         stale, mid, xcc);
    else
      hipLaunchKernelGGL(probe::litmus_mp_kernel<false>, dim3(2 * pairs), dim3(64), 0, stream, cells, rounds, reads,
                         stale, mid, xcc);
    if (hipGetLastError() != hipSuccess) return GTAP_E_HIP;
    std::vector<uint32_t> h(2 * inst);
    if (hipMemcpyAsync(h.data(), res, h.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, stream) != hipSuccess)
      return GTAP_E_HIP;
    std::vector<uint32_t> hx(2 * pairs);
    if (hipMemcpyAsync(hx.data(), xcc, hx.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return GTAP_E_HIP;
    for (uint64_t i = 0; i < inst; ++i) {
      out->mp_stale += h[i];
      out->mp_overlap += h[inst + i];
    }
    out->mp_reads = inst * reads;
    for (uint32_t q = 0; q < pairs; ++q) out->pairs_on_distinct_xcds += (hx[2 * q] & 15u) != (hx[2 * q + 1] & 15u);
    return GTAP_OK;
  }
  if (ordered)
    hipLaunchKernelGGL(probe::litmus_sb_kernel<true>, dim3(2 * pairs), dim3(64), 0, stream, cells, rounds, res, xcc);
  else
    hipLaunchKernelGGL(probe::litmus_sb_kernel<false>, dim3(2 * pairs), dim3(64), 0, stream, cells, rounds, res, xcc);
  if (hipGetLastError() != hipSuccess) return GTAP_E_HIP;
  const uint64_t total = inst * rounds;
  hipLaunchKernelGGL(probe::litmus_sb_count_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0,
                     stream, res, rounds, static_cast<uint32_t>(inst), counts);
  if (hipGetLastError() != hipSuccess) return GTAP_E_HIP;
  unsigned long long hc[4] = {0, 0, 0, 0};
  std::vector<uint32_t> hx(2 * pairs);
  if (hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipMemcpyAsync(hx.data(), xcc, hx.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return GTAP_E_HIP;
  out->sb_rounds = total;
  out->sb_both_new = hc[0];
  out->sb_a_new_only = hc[1];
  out->sb_b_new_only = hc[2];
  out->sb_both_old = hc[3];
  for (uint32_t q = 0; q < pairs; ++q) out->pairs_on_distinct_xcds += (hx[2 * q] & 15u) != (hx[2 * q + 1] & 15u);
  return GTAP_OK;
}

// ---- allocation-free batch run --------------------------------------------
// The runtime's workspace (control block, job table, deques, depots, frame
// pools) lives in a static device array instead of a hipMalloc'd buffer.  In
// host code `scratch` names a host-side stand-in, never the device memory:
// its device address is looked up once per device and used from then on.
static __device__ __align__(256) char scratch[GTAP_STATIC_SCRATCH_BYTES];

namespace {

constexpr size_t kStaticScratchBytes = static_cast<size_t>(GTAP_STATIC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_dev[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on the first call
// on the device, with that device current).
int static_scratch(char **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GTAP_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GTAP_E_HIP;
    g_scratch_dev[dev] = static_cast<char *>(ptr);
  }
  *out = g_scratch_dev[dev];
  return GTAP_OK;
}

constexpr size_t kStaticChunk = 32;  // job slots staged per copy (4 KB on the stack)

}  // namespace

extern "C" int gtap_run_static(const gtap_config *cfg_in, const gtap_trace_job *jobs, size_t n, int64_t *results,
                               gtap_error_report *report) {
  if (report) *report = gtap_error_report{};
  if (!cfg_in || (n > 0 && (!jobs || !results))) return GTAP_E_INVAL;
  if (n > GTAP_STATIC_MAX_JOBS) return GTAP_E_INVAL;
  if (n == 0) return GTAP_OK;
  for (size_t i = 0; i < n; ++i) {
    const int32_t k = jobs[i].kind;
    if (k != GTAP_KIND_FIB && k != GTAP_KIND_NQUEENS && k != GTAP_KIND_UTS && k != GTAP_KIND_KCLIQUE)
      return GTAP_E_INVAL;
    if (jobs[i].args_bytes > sizeof(jobs[i].args)) return GTAP_E_INVAL;
  }
  gtap_config cfg = *cfg_in;
  cfg.max_jobs = static_cast<uint32_t>(n);
  cfg.workspace_dev = nullptr;
  cfg.workspace_bytes = 0;
  if (cfg.timeout_ms == 0) cfg.timeout_ms = 120000;
  int rc = validate(cfg);
  if (rc) return rc;
  uint32_t maxw = 0;
  rc = max_resident_waves(cfg.mode, cfg.waves_per_group, &maxw);
  if (rc) return rc;
  uint32_t nw = cfg.num_waves ? std::min<uint32_t>(cfg.num_waves, maxw) : maxw;
  nw = std::max<uint32_t>(nw / cfg.waves_per_group, 1) * cfg.waves_per_group;
  const Layout L = make_layout(cfg, nw);
  if (L.total > kStaticScratchBytes) return GTAP_E_NOMEM;
  char *ws = nullptr;
  rc = static_scratch(&ws);
  if (rc) return rc;

  // a context on the stack: the launch helpers read its configuration,
  // grid, stream and kernel parameters (its containers stay empty)
  gtap_ctx c;
  c.cfg = cfg;
  c.stream = static_cast<hipStream_t>(cfg.stream);
  c.nwaves = nw;
  c.lay = L;
  c.ws = ws;
  fill_params(cfg, nw, L, ws, c.params);
  Params &p = c.params;
  p.njobs = static_cast<uint32_t>(n);
  p.serving = 0;

  JobSlot buf[kStaticChunk];
  for (size_t i0 = 0; i0 < n; i0 += kStaticChunk) {
    const size_t m = std::min(kStaticChunk, n - i0);
    for (size_t i = 0; i < m; ++i) {
      rc = pack_job(cfg, c.stream, jobs[i0 + i].kind, jobs[i0 + i].args, jobs[i0 + i].args_bytes, buf[i]);
      if (rc) return rc;
    }
    if (hipMemcpyAsync(p.jobs + i0, buf, m * sizeof(JobSlot), hipMemcpyHostToDevice, c.stream) != hipSuccess ||
        hipStreamSynchronize(c.stream) != hipSuccess)
      return GTAP_E_HIP;
  }
  const uint32_t ndq = nw * p.Q;
  hipLaunchKernelGGL(reset_kernel, dim3(reset_blocks(ndq, p.ccap)), dim3(256), 0, c.stream, p, ndq);
  if (hipGetLastError() != hipSuccess) return GTAP_E_HIP;
  rc = launch_sched(&c);
  if (rc) {
    (void)hipStreamSynchronize(c.stream);
    return rc;
  }
  Control ctl;
  if (hipMemcpyAsync(&ctl, p.ctl, sizeof(Control), hipMemcpyDeviceToHost, c.stream) != hipSuccess ||
      hipStreamSynchronize(c.stream) != hipSuccess)
    return GTAP_E_HIP;
  if (ctl.error != 0) {
    if (report) {
      report->code = ctl.error;
      report->pool = ctl.err_pool;
      report->capacity = ctl.err_capacity;
      report->requested = ctl.err_requested;
      report->wave = ctl.err_wave;
      report->job = ctl.err_job;
    }
    return ctl.error;
  }
  for (size_t i0 = 0; i0 < n; i0 += kStaticChunk) {
    const size_t m = std::min(kStaticChunk, n - i0);
    if (hipMemcpyAsync(buf, p.jobs + i0, m * sizeof(JobSlot), hipMemcpyDeviceToHost, c.stream) != hipSuccess ||
        hipStreamSynchronize(c.stream) != hipSuccess)
      return GTAP_E_HIP;
    for (size_t i = 0; i < m; ++i) {
      if (buf[i].done != 1) return GTAP_E_STATE;
      results[i0 + i] = buf[i].result;
    }
  }
  return GTAP_OK;
}
