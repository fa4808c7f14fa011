// layout.h -- device memory layout shared by the host library and the kernels.
//
// Everything the runtime touches lives in one device workspace, carved into:
//   control block   (counters, error report, statistics)
//   job table       (one 128-byte slot per root task)
//   deque metadata  (one 128-byte line per deque: count, head, lock)
//   deque rings     (u32 task IDs, `cap` per deque, waves x queues deques)
//   depot bins      (free-frame chunks shared between wavefronts, per pool)
//   frame pools     (small: 64-byte frames; big: 64-byte header + int32 buffer)
// Task IDs are frame indices (GTaP Sec. 5.1.1: a task ID indexes the storage
// holding its record); bit 31 selects the big pool.
#pragma once
#include <stdint.h>

namespace gtap {

constexpr uint32_t kNone = 0xFFFFFFFFu;        // "no task" / "no parent"
constexpr uint32_t kBigBit = 0x80000000u;      // task ID of a big-pool frame
constexpr uint32_t kFrameWords = 16;           // 64-byte frame header+payload
constexpr uint32_t kWave = 64;                 // CDNA wavefront width
constexpr uint32_t kMaxQueues = 8;             // DAQ deques per wavefront
constexpr uint32_t kDepotBins = 256;           // depot bins per pool

// Per-wave LDS free-stack capacities and depot chunk sizes (IDs).
constexpr uint32_t kStackSmall = 1024;
constexpr uint32_t kStackBig = 128;
constexpr uint32_t kChunkSmall = 256;
constexpr uint32_t kChunkBig = 64;

// Frame word map (u32 words).  A spawn writes words 0..7 as four 64-bit
// device-coherent stores; a fork writes the state word, the join counter and
// the accumulator.  Big frames carry an int32 buffer from word 16 on.
enum FrameWord : uint32_t {
  FW_PARENT = 0,   // parent task ID, kNone for a job's root
  FW_JOB = 1,      // job slot
  FW_STATE = 2,    // kind | resume point << 8 | queue class << 16
  FW_P0 = 3,       // payload words 3..7 (p0..p4)
  FW_JOIN = 8,     // join word (words 8,9): children's results << 20 | waiting children
  FW_BIGACC = 10,  // int64 accumulator for results too large for the join word
  FW_BUF = 16,     // big frames: candidate buffer
};
constexpr uint32_t kPayloadWords = 5;

// Join word: one 64-bit RMW per completing child both adds its result and
// decrements the waiting-child count, so no ordering is needed between the
// two.  The low kJoinBits bits hold the count; the rest a signed sum of
// results.  A delivery whose value has magnitude >= 2^kSmallValueBits goes to
// the separate 64-bit accumulator first, which bounds the packed sum by
// 2^(kSmallValueBits + kJoinBits) < 2^43.
constexpr uint32_t kJoinBits = 20;
constexpr uint64_t kJoinMask = (1ull << kJoinBits) - 1;
constexpr uint32_t kMaxChildren = (1u << kJoinBits) - 1;
constexpr uint32_t kSmallValueBits = 23;

// Task kinds of the thread-mode state machines.
enum TaskKind : uint32_t {
  TK_FIB = 1,
  TK_NQ = 2,
  TK_UTS = 3,
  TK_KC_RANGE = 4,
  TK_KC_VERTEX = 5,
  TK_KC_CAND = 6,
  TK_FMM = 7,       // block mode: FMM cell pair (A, B)
  TK_DTT = 8,       // thread mode: FMM cell pair (A, B) that only builds the interaction lists
  TK_SORT = 9,      // Cilksort: sort a range into a buffer
  TK_MERGE = 10,    // Cilksort: merge two sorted ranges
  TK_KS_RANGE = 11,   // k-clique with splitting: vertex range
  TK_KS_VERTEX = 12,  //   vertex: one edge task per out-neighbour
  TK_KS_EDGE = 13,    //   edge (u, v): candidates N+(u) /\ N+(v), counted in place if few
  TK_KS_HEAVY = 14,   //   edge with many candidates: their bit matrix, the search's root
  TK_KS_NODE = 15,    //   branch of a node that split
  TK_KS_ROW = 16,     //   one row of a vertex's bit matrix
};

// Extension task sets of the thread-mode kernel, each compiled in only where
// a launch needs it: the split k-clique bodies alone add private memory and
// registers to every task of the kernel.
constexpr uint32_t kExtLists = 1;  // FMM list-building cell pairs, Cilksort sorts and merges
constexpr uint32_t kExtSplit = 2;  // k-clique with bitset candidate subgraphs (TK_KS_*)
constexpr uint32_t kExtAll = kExtLists | kExtSplit;

struct alignas(128) DequeMeta {
  int32_t count;   // unclaimed entries (every claim is a CAS on this word)
  uint32_t head;   // steal end, advanced by the lock holder after loading
  int32_t lock;    // serialises thieves
  int32_t pad[29];
};
static_assert(sizeof(DequeMeta) == 128, "deque metadata must fill one line");

struct alignas(128) DepotBin {
  int32_t lock;
  int32_t nchunks;
  int32_t pad[30];
};
static_assert(sizeof(DepotBin) == 128, "depot bin must fill one line");

// One job (root task).  Written by the host before a run, results by the
// device.  128 bytes.
struct alignas(128) JobSlot {
  uint32_t kind;       // gtap_kind
  uint32_t done;       // 1 once the root task completed
  int64_t result;      // root task's return value
  uint64_t a[8];       // kind arguments (see runtime.hip: pack_args)
  uint64_t t_done;     // device wall clock at completion
  uint64_t ticket;     // serving: the job's ticket (set by the admitting wave)
  int64_t pending;     // block-mode FMM: outstanding cell-pair tasks (see sched_block.h)
  uint64_t pad[2];
};
static_assert(sizeof(JobSlot) == 128, "job slot is one 128-byte line");

enum StatIdx : uint32_t {
  ST_TASKS = 0, ST_CONTS, ST_SPAWNS, ST_PUSHED, ST_PUSH_BATCHES, ST_POPPED,
  ST_POP_BATCHES, ST_STOLEN, ST_STEAL_BATCHES, ST_STEAL_ATTEMPTS, ST_ITERS,
  ST_IDLE, ST_SPILLS, ST_REFILLS, ST_BUSY_CYCLES, ST_IDLE_CYCLES, ST_ADMITTED, ST_LOCAL,
  ST_RMW,  // device-scope read-modify-writes issued by the scheduler (one per lane)
  ST_DATA_WORDS,  // 4-byte words of task data (input lists, candidate buffers) task bodies moved
  ST_COUNT
};

// Serving: the host appends jobs to a ring in pinned host memory and the
// running kernel admits them.  Slot t % ring_cap holds ticket t once
// ring_seq[t % ring_cap] == t + 1.
struct alignas(16) HostCompletion {
  int64_t result;
  uint64_t done;      // ticket + 1 once the job's root completed
  uint64_t t_done;    // device wall clock at completion
  uint64_t pad;
};
static_assert(sizeof(HostCompletion) == 32, "completion record");
constexpr uint32_t kAdmitWaves = 8;       // waves that poll the admission ring

// Control block: first 4 KB of the workspace.
struct alignas(128) Control {
  int32_t jobs_remaining;   // root tasks not yet completed
  int32_t error;            // first error wins (CAS from 0)
  int32_t err_pool;
  int32_t err_wave;
  int32_t err_job;
  int32_t pad0[3];
  uint64_t err_capacity;
  uint64_t err_requested;
  uint64_t pad1[12];
  uint64_t bump_small;      // 128-byte aligned: fresh-frame bump pointers
  uint64_t pad2[15];
  uint64_t bump_big;
  uint64_t pad3[15];
  uint64_t admitted;        // serving: next ticket to admit (128-byte aligned)
  uint64_t pad4[15];
  int64_t live_small;       // serving: frames handed out and not yet returned
  int64_t live_big;
  uint64_t pad5[14];
  int32_t hungry;           // thread mode: wavefronts that found no work (a hint for exposure)
  int32_t pad6[31];
  uint64_t stats[ST_COUNT];
};

// Kernel parameters (passed by value).
// Centralised queue (scheduler comparison): positions are 32-bit counters
// that wrap; a slot holds (position << 32 | task ID), so a reader waits for
// the writer of its own position.  Each word on its own line.
struct alignas(128) CentralQueue {
  uint32_t tail;      // next position to reserve (pushes)
  uint32_t pad0[31];
  int32_t count;      // published, unclaimed entries (claims CAS on it)
  uint32_t pad1[31];
  uint32_t head;      // next position to claim (pops)
  uint32_t pad2[31];
};
constexpr uint32_t kSchedBatched = 0, kSchedSingle = 1, kSchedCentral = 2, kSchedBatchedNoLocal = 3;

struct Params {
  Control *ctl;
  JobSlot *jobs;
  uint32_t njobs;
  uint32_t nwaves;          // persistent wavefronts in the grid
  DequeMeta *dq;            // [wave * Q + q]
  uint32_t *rings;          // [(wave * Q + q) * cap + slot]
  uint32_t cap;             // deque capacity (power of two)
  uint32_t Q;               // queues per wave
  uint32_t *frames_s;       // small frames, 16 words each
  uint32_t nframes_s;
  uint32_t *frames_b;       // big frames, stride_b words each
  uint32_t nframes_b;
  uint32_t stride_b;        // words per big frame (16 + buffer ints)
  uint32_t big_ints;        // buffer capacity of a big frame
  DepotBin *bins_s;
  uint32_t *store_s;        // [bin * bincap_s + i]
  uint32_t bincap_s;        // IDs per small bin
  DepotBin *bins_b;
  uint32_t *store_b;
  uint32_t bincap_b;
  uint32_t steal_below;
  uint32_t steal_probes;    // victims probed per steal attempt (1..64)
  uint32_t steal_div;       // claim ceil(count / steal_div), at most 64 - cnt
  uint32_t daq_policy;
  int32_t daq_bounds[kMaxQueues - 1];
  uint64_t timeout_ticks;   // watchdog, device wall-clock ticks
  // serving mode (serving == 0: a batch run over jobs[0, njobs))
  uint32_t serving;
  uint32_t ring_cap;        // admission ring slots == job table slots
  const JobSlot *ring;      // pinned host memory
  const uint64_t *ring_seq; // pinned host memory
  HostCompletion *done_host;  // pinned host memory, [ring_cap]
  const int32_t *stop_host;   // pinned host memory
  uint32_t max_inflight;    // admitted and not completed
  uint32_t admit_headroom_small;  // frames that must stay free after admitting a job
  uint32_t admit_headroom_big;
  // scheduler variant (kSched*; the kernel is instantiated per variant)
  uint32_t sched;
  CentralQueue *cq;         // kSchedCentral only
  uint64_t *cring;          // [ccap] tagged slots
  uint32_t ccap;            // power of two, 0 unless kSchedCentral
};

}  // namespace gtap
