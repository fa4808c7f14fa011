/*
 * gtap.h -- C ABI of the MI355X (gfx950) fork-join task runtime.
 *
 * The runtime executes fine-grained fork-join task trees inside one persistent
 * kernel (GTaP, Sec. 5.1.1 "Overview"): every wavefront of the grid runs a
 * scheduler loop that acquires runnable task IDs from its own work-stealing
 * deque or steals them from another wavefront's, executes them, and publishes
 * the tasks they make runnable.  A task that forks suspends at its join with
 * a waiting-child counter and a saved resume point and is re-executed in
 * place when the last child completes (Sec. 5.1.2 "Implementation of
 * Fork-Join").  Thread mode runs one task per lane of a 64-lane wavefront;
 * block mode runs one task per workgroup (Sec. 4.2, Sec. 4.3).
 *
 * The paper's host API is initialize(config) / launch(kernel, args) /
 * finalize() with a configuration giving launch geometry, preallocated task
 * capacity and the number of DAQ queues, and capacity overflow reported as a
 * structured error (Sec. 4, "Programming Model", opening paragraphs).  This ABI
 * splits launch into submit (one root task per job, arguments copied at submit
 * time like a task's firstprivate arguments, Sec. 4.1) and run (one persistent
 * launch for every submitted job).
 *
 * Conventions for every entry point:
 *   - returns GTAP_OK (0) on success or a negative gtap_status; no exception
 *     or abort crosses the ABI;
 *   - pointers named *_dev are device pointers (hipMalloc or a PyTorch CUDA
 *     tensor's data_ptr()); all other pointers are host pointers;
 *   - a gtap_ctx is not thread-safe: one host thread drives one context.
 */
#ifndef GTAP_H
#define GTAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
enum gtap_status {
    GTAP_OK = 0,
    GTAP_E_INVAL = -1,     /* bad argument or configuration                   */
    GTAP_E_NOMEM = -2,     /* device allocation failed / workspace too small   */
    GTAP_E_HIP = -3,       /* a HIP runtime call failed                        */
    GTAP_E_STATE = -4,     /* call not valid in the context's current state   */
    GTAP_E_FULL = -5,      /* max_jobs pending jobs already submitted          */
    GTAP_E_CAPACITY = -6,  /* frame pool or deque exhausted on the device:
                              the run was aborted, see gtap_last_error        */
    GTAP_E_PENDING = -7,   /* job has not completed                           */
    GTAP_E_TIMEOUT = -8,   /* device watchdog expired: the run was aborted    */
    GTAP_E_NOJOB = -9      /* unknown job id                                  */
};

/* ---- execution modes and task kinds -------------------------------------- */
enum gtap_mode { GTAP_MODE_THREAD = 0, GTAP_MODE_BLOCK = 1 };

enum gtap_kind {
    GTAP_KIND_FIB = 1,      /* gtap_fib_args                                   */
    GTAP_KIND_NQUEENS = 2,  /* gtap_nqueens_args                               */
    GTAP_KIND_UTS = 3,      /* gtap_uts_args                                   */
    GTAP_KIND_KCLIQUE = 4,  /* gtap_kclique_args                               */
    GTAP_KIND_FMM = 5,      /* gtap_fmm_args (traversal TASKS: block mode;
                               LISTS, WORKLIST: thread mode)                  */
    GTAP_KIND_CILKSORT = 6, /* gtap_cilksort_args (thread mode)                */
    GTAP_KIND_KCLIQUE_SPLIT = 7  /* gtap_kclique_split_args (thread mode)      */
};

/* Fibonacci with a task at every call (Sec. 6.3, microbenchmarks): result is
 * fib(n), 0 <= n <= 92. */
typedef struct { int32_t n; int32_t reserved; } gtap_fib_args;

/* N-Queens solution count by bitmask backtracking, one child task per legal
 * column (Sec. 6.3): 1 <= n <= 31. */
typedef struct { int32_t n; int32_t reserved; } gtap_nqueens_args;

/* Unbalanced tree search: node count of the tree rooted at mix64(seed).  A
 * node at depth < max_depth has as many children as leading splitmix64 draws
 * below `threshold` (geometric, mean T/(2^64-T)); child i of node id has id
 * split(id, i).  0 <= max_depth <= 255. */
typedef struct { uint64_t seed; uint64_t threshold; int32_t max_depth; int32_t reserved; } gtap_uts_args;

/* k-clique count on an oriented graph (Sec. 6.4.2, orientation algorithm).
 * row_ptr_dev: int32[n+1], col_dev: int32[row_ptr[n]]: sorted out-lists of an
 * acyclic orientation, device-resident and borrowed: the caller keeps them
 * alive and unchanged until gtap_run returns.  max_outdeg must be >= every
 * out-degree and <= the context's big_frame_ints.  Vertex ranges larger than
 * range_leaf are split in halves; smaller ones fork one task per vertex.
 * range_leaf and max_outdeg are at most 2^20 - 1 (children per fork). */
typedef struct {
    const int32_t *row_ptr_dev;
    const int32_t *col_dev;
    int32_t n;
    int32_t k;
    int32_t range_leaf;
    int32_t max_outdeg;
} gtap_kclique_args;

/* k-clique count with bitset-encoded candidate subgraphs and cost-threshold
 * task splitting (Sec. 6.4.2: the orientation and the pivoting algorithms).
 * The vertex range splits as for GTAP_KIND_KCLIQUE.  For k >= 4 a vertex u
 * with at least k-1 out-neighbours encodes the subgraph induced on N+(u) as a
 * bit matrix (one row task per out-neighbour), then forks one edge task per
 * out-neighbour v: the edge's candidates N+(u) /\ N+(v) are row v, and it
 * counts the (k-2)-cliques among them (k = 3: the size of the intersection).
 * A vertex with at most `threshold` out-neighbours counts all its edges in
 * place instead.  gtap_run allocates the job's matrices for the run: sum over
 * the vertices that fork of d * ceil(d/64) * 8 bytes (twice that for
 * pivoting), d = out-degree.
 * A search node whose candidate set has more than
 * `threshold` members splits into one child task per branch -- per candidate
 * for the orientation algorithm; the pivot and each of its non-neighbours for
 * pivoting -- and every child applies the same test; smaller nodes are
 * counted in place by one lane.  Same graph contract as gtap_kclique_args
 * (row_ptr_dev/col_dev borrowed until gtap_run returns, sorted acyclic
 * out-lists); the library reads row_ptr once at submit and rejects a graph
 * whose largest out-degree exceeds max_outdeg or 1024.  Needs thread mode,
 * waves_per_group 4, flags 0, 1 <= k <= 32, 0 <= threshold <= 64 and, for
 * k >= 4, big frames of at least gtap_kclique_split_buffer_ints(max_outdeg)
 * ints.  The result is the number of k-cliques. */
typedef struct {
    const int32_t *row_ptr_dev;
    const int32_t *col_dev;
    int32_t n;
    int32_t k;
    int32_t range_leaf;
    int32_t max_outdeg;
    int32_t threshold;      /* split when a node has more candidates than this */
    int32_t algorithm;      /* gtap_kclique_algorithm                          */
} gtap_kclique_split_args;

enum gtap_kclique_algorithm { GTAP_KCLIQUE_ORIENT = 0, GTAP_KCLIQUE_PIVOT = 1 };

/* Big-frame buffer ints a GTAP_KIND_KCLIQUE_SPLIT job needs for out-degrees up
 * to max_outdeg (0 if max_outdeg is negative or above 1024). */
int32_t gtap_kclique_split_buffer_ints(int32_t max_outdeg);

/* 3D Laplace FMM whose interaction phase is a dual-tree traversal run as
 * block-mode tasks (Sec. 6.4.1, "FMM Dual-Tree Traversal").  The library builds
 * an octree over the n points (root cube [-128, 128)^3; a cell with more than
 * leaf_max points below level 21 splits into its non-empty octants), computes
 * multipole moments (P2M, M2M), runs the traversal from the (root, root) cell
 * pair -- each task accepts its pair by the integer MAC with
 * theta = theta_num / theta_den and adds an M2L contribution, runs a
 * workgroup-wide P2P on a pair of leaves, or forks the child pairs of the
 * wider cell -- and finishes with L2L and L2P.  Expansions are Cartesian
 * Taylor series of total degree `order` (must be 6).  phi_dev[i] receives
 * sum over j != i of q_j / |x_i - x_j| approximated by the FMM (coincident
 * distinct points skipped).  All pointers are fp64 device arrays of n entries,
 * borrowed until gtap_run returns.  Requires 1 <= n < 2^31, every coordinate
 * in [-128, 128), 1 <= leaf_max <= 64, 0 <= theta_num and 1 <= theta_den <= 64
 * with theta_num <= theta_den. */
typedef struct {
    const double *x_dev;
    const double *y_dev;
    const double *z_dev;
    const double *q_dev;
    double *phi_dev;
    int32_t n;
    int32_t leaf_max;
    int32_t theta_num;
    int32_t theta_den;
    int32_t order;
    int32_t traversal;       /* gtap_fmm_traversal                            */
    uint64_t m2l_capacity;   /* LISTS / WORKLIST: list capacities in pairs     */
    uint64_t p2p_capacity;   /*   (0 = estimated from the tree and theta)      */
} gtap_fmm_args;

/* How an FMM job's dual-tree traversal runs.
 *   GTAP_FMM_TASKS     block mode: every cell-pair task does its M2L or
 *                      workgroup-wide P2P itself (the description above)
 *   GTAP_FMM_LISTS     thread mode, as in the paper's FMM pipeline: the
 *                      cell-pair tasks only append accepted pairs to an M2L
 *                      list and leaf pairs to a P2P list (fixed-capacity
 *                      arrays, one atomic add per wavefront and list); the
 *                      lists are then sorted by target and evaluated by
 *                      data-parallel M2L and P2P kernels
 *   GTAP_FMM_WORKLIST  thread mode, the level-synchronous GPU worklist
 *                      baseline of the same section: ping-pong frontiers of
 *                      cell pairs, one kernel launch and one host
 *                      synchronisation per frontier, the same lists and
 *                      evaluation kernels (its root task is empty)
 * Lists that overflow their capacity are counted to the end; the library then
 * re-runs the traversal once with capacities that fit (list_retries). */
enum gtap_fmm_traversal { GTAP_FMM_TASKS = 0, GTAP_FMM_LISTS = 1, GTAP_FMM_WORKLIST = 2 };

/* What gtap_result returns for an FMM job (out_bytes >= its size).  The pair
 * hashes are wrapping sums of splitmix64((A << 32) | B) over the (target cell,
 * source cell) pairs of each list, independent of the traversal's order. */
typedef struct {
    int64_t n_cells;
    int64_t n_leaves;
    int64_t max_level;
    int64_t m2l_pairs;
    int64_t p2p_pairs;
    uint64_t m2l_hash;
    uint64_t p2p_hash;
    int64_t p2p_interactions;  /* (i, j != i) pairs evaluated by P2P          */
    int64_t coincident;        /* of those, distinct points at the same place */
    double tree_ms;            /* sort and octree construction               */
    double upward_ms;          /* P2M and M2M                                */
    double traversal_ms;       /* TASKS, LISTS: the scheduler launch (shared by
                                  the run's jobs); WORKLIST: its kernels and
                                  host loop                                   */
    double downward_ms;        /* L2L, L2P and the scatter to phi_dev        */
    double sort_ms;            /* LISTS, WORKLIST: sorting the lists by target */
    double m2l_ms;             /*   M2L list evaluation                      */
    double p2p_ms;             /*   P2P list evaluation                      */
    int64_t dtt_rounds;        /* WORKLIST: frontier launches                */
    int64_t list_retries;      /* traversals re-run after a list overflowed   */
} gtap_fmm_result;

/* Cilksort (Sec. 6.3, microbenchmarks): sorts keys_dev[0, n) in place with a
 * parallel mergesort whose merges are split in parallel too.  sort(lo, n)
 * sorts ranges of at most sort_cutoff keys serially (a 64-wide sorting network
 * on one lane), otherwise sorts both halves into the other buffer and merges
 * them back; a merge of more than merge_cutoff keys splits the longer range at
 * its middle key and the other by binary search into two independent merges.
 * tmp_dev is a scratch buffer of n keys.  Both are device arrays borrowed
 * until gtap_run returns.  Thread mode with four wavefronts per group; the
 * result is n.  Requires 0 <= n < 2^29, 1 <= sort_cutoff <= 64,
 * 2 <= merge_cutoff <= 2^20.  With num_queues >= 3 and GTAP_DAQ_CILKSORT,
 * recursive tasks, serial sorts and serial merges wait in separate queues. */
typedef struct {
    uint32_t *keys_dev;
    uint32_t *tmp_dev;
    int64_t n;
    int32_t sort_cutoff;
    int32_t merge_cutoff;
} gtap_cilksort_args;

/* ---- configuration -------------------------------------------------------- */
enum gtap_daq_policy {
    GTAP_DAQ_NONE = 0,      /* every task in queue 0                            */
    GTAP_DAQ_BY_KIND = 1,   /* queue = task kind (mod num_queues)               */
    GTAP_DAQ_KCLIQUE = 2,   /* k-clique: queue = bucket of the candidate-set
                               bound, buckets split at daq_bounds[]            */
    GTAP_DAQ_CILKSORT = 3   /* Cilksort: queue 0 recursive sorts and merges,
                               1 serial sorts, 2 serial merges (mod num_queues) */
};

typedef struct gtap_config {
    int32_t mode;             /* gtap_mode.  Thread mode runs every kind but
                                 FMM; block mode runs FIB, UTS and FMM, one
                                 task per workgroup, one Chase-Lev deque per
                                 workgroup (num_queues must be 1)            */
    int32_t num_waves;        /* persistent wavefronts; 0 = every wavefront the
                                 device can keep resident                      */
    int32_t waves_per_group;  /* wavefronts per workgroup: 1, 2, 4 or 8 (block
                                 mode: 1, 2 or 4, i.e. 64..256 threads)       */
    int32_t num_queues;       /* DAQ deques per wavefront, 1..8 (1 = DAQ off)  */
    int32_t daq_policy;       /* gtap_daq_policy                               */
    int32_t daq_bounds[7];    /* ascending class boundaries (GTAP_DAQ_KCLIQUE) */
    uint32_t deque_capacity;  /* slots per deque, power of two >= 128          */
    uint32_t steal_below;     /* steal when fewer lanes than this hold a task
                                 after the local pop (1..64)                   */
    uint32_t steal_probes;    /* victims whose deque size one steal attempt
                                 reads at once, the fullest is robbed (1..64) */
    uint32_t steal_div;       /* a steal claims ceil(count / steal_div)
                                 entries, at most the free lanes (1..64)      */
    uint64_t small_frames;    /* frames in the 64-byte frame pool              */
    uint64_t big_frames;      /* frames in the candidate-buffer pool           */
    uint32_t big_frame_ints;  /* int32 capacity of a big frame's buffer        */
    uint32_t max_jobs;        /* jobs per run                                  */
    uint32_t timeout_ms;      /* device watchdog per run (0 = 120000)          */
    uint32_t flags;           /* gtap_flags (thread mode); 0 = the scheduler
                                 as designed                                  */
    void *stream;             /* hipStream_t to launch on (NULL = default)     */
    void *workspace_dev;      /* optional caller-owned device memory of
                                 workspace_bytes (>= gtap_workspace_size);
                                 NULL = the library allocates and frees it    */
    uint64_t workspace_bytes;
} gtap_config;

/* Scheduler variants for the comparison of thread-mode schedulers (Sec. 6.5,
 * "GPU-Side Scheduler Comparison"): all share the runtime and differ only in
 * queue management.  Thread mode, one queue, four wavefronts per group, batch
 * runs only (serving and block mode reject them); each variant is its own
 * kernel instantiation, so flags == 0 runs the scheduler unchanged.
 *   GTAP_FLAG_NO_PRIVATE_STACK  children beyond the 64 lanes go to the
 *                               wavefront's deque at once (no LDS stack), as
 *                               in the paper's Algorithm 1
 *   GTAP_FLAG_SCHED_SINGLE      non-batched work stealing: every pop and every
 *                               steal claims one task; a wavefront issues up
 *                               to 64 of them per iteration (implies no
 *                               private stack)
 *   GTAP_FLAG_SCHED_CENTRAL     one FIFO queue for the whole grid instead of
 *                               per-wavefront deques: batched pushes reserve
 *                               ring positions with one atomic, pops claim
 *                               by CAS on its count; no stealing (implies no
 *                               private stack)
 * SINGLE and CENTRAL are exclusive. */
enum gtap_flags {
    GTAP_FLAG_NO_PRIVATE_STACK = 1,
    GTAP_FLAG_SCHED_SINGLE = 2,
    GTAP_FLAG_SCHED_CENTRAL = 4
};

/* Fill *cfg with defaults (thread mode, occupancy-sized grid, one queue). */
void gtap_config_default(gtap_config *cfg);

/* Device bytes a context with this configuration needs (for workspace_dev).
 * Needs a current HIP device (the grid size depends on it). */
int gtap_workspace_size(const gtap_config *cfg, uint64_t *bytes);

/* ---- lifecycle ------------------------------------------------------------ */
typedef struct gtap_ctx gtap_ctx;

/* Validate cfg, size the grid, lay out (and unless cfg->workspace_dev is set,
 * allocate) frame pools, deques and job tables on the current HIP device.
 * *out receives a context owned by the caller until gtap_finalize.
 * Errors: GTAP_E_INVAL, GTAP_E_NOMEM, GTAP_E_HIP. */
int gtap_init(const gtap_config *cfg, gtap_ctx **out);

/* Queue one root task.  args points to the kind's argument struct (host
 * memory, args_bytes == sizeof of it); it is copied before the call returns.
 * *job_id receives the job's id.  Errors: GTAP_E_INVAL (kind, size or value),
 * GTAP_E_FULL (max_jobs already pending), GTAP_E_STATE. */
int gtap_submit(gtap_ctx *ctx, int32_t kind, const void *args, size_t args_bytes,
                uint64_t *job_id);

/* Launch one persistent kernel for every pending job on cfg->stream and wait
 * for it.  Jobs' results become readable with gtap_result.  FMM jobs also run
 * their tree construction and upward pass before, and their downward pass
 * after, that launch (device memory for them is allocated and freed inside
 * this call).  Returns GTAP_E_CAPACITY or GTAP_E_TIMEOUT when the device
 * aborted the run (results of that run are then invalid; the context stays
 * usable), GTAP_E_INVAL when an FMM job's points leave the root cube,
 * GTAP_E_NOMEM, GTAP_E_HIP on a HIP failure. */
int gtap_run(gtap_ctx *ctx);

/* Copy job job_id's result into host memory out: an int64 count
 * (out_bytes >= 8), or for an FMM job a gtap_fmm_result (out_bytes >= its
 * size; the potentials are in the job's phi_dev).  Valid for the jobs of the
 * most recent gtap_run.  Errors: GTAP_E_NOJOB, GTAP_E_PENDING (not part of a
 * completed run), GTAP_E_INVAL. */
int gtap_result(gtap_ctx *ctx, uint64_t job_id, void *out, size_t out_bytes);

/* Release the context and any memory the library allocated for it. */
int gtap_finalize(gtap_ctx *ctx);

/* ---- diagnostics ---------------------------------------------------------- */
typedef struct gtap_stats {
    uint64_t tasks;          /* first executions of a task (resume point 0)    */
    uint64_t conts;          /* re-executions after a join                    */
    uint64_t spawns;         /* child tasks created                           */
    uint64_t pushed;         /* task IDs published to a deque                 */
    uint64_t push_batches;   /* deque publications (one fence + one atomic)   */
    uint64_t popped;         /* task IDs claimed from the owner's deque       */
    uint64_t pop_batches;
    uint64_t stolen;         /* task IDs claimed from another wave's deque    */
    uint64_t steal_batches;  /* successful steals                             */
    uint64_t steal_attempts;
    uint64_t iterations;     /* scheduler loop iterations that ran tasks      */
    uint64_t idle_iterations;
    uint64_t small_frames_touched; /* high-water mark of the small pool       */
    uint64_t big_frames_touched;
    uint64_t depot_spills;
    uint64_t depot_refills;
    uint64_t busy_cycles;    /* shader-clock cycles in iterations that ran tasks */
    uint64_t idle_cycles;    /* shader-clock cycles in iterations that found none */
    uint64_t admitted;       /* serving: jobs admitted from the ring           */
    uint64_t local_pushed;   /* children kept in a wavefront's LDS stack       */
    uint64_t atomics;        /* thread mode: device-scope read-modify-writes the
                                scheduler issued (join updates, deque counts,
                                claims and thieves' locks; one per lane)      */
    uint64_t data_bytes;     /* thread mode: bytes of task data the k-clique task
                                bodies read or wrote (row bounds, candidate
                                lists, neighbour lists, new candidate lists;
                                split jobs: bit-matrix rows and node states),
                                each list or row counted once at full length */
    double kernel_ms;        /* device time of the last run's persistent kernel */
    int32_t num_waves;
    int32_t waves_per_group;
    int32_t num_queues;
    int32_t reserved;
} gtap_stats;

typedef struct gtap_error_report {
    int32_t code;       /* gtap_status of the abort, GTAP_OK if none           */
    int32_t pool;       /* 0 small frames, 1 big frames, 2 deque, 3 watchdog   */
    uint64_t capacity;  /* capacity of the exhausted resource                  */
    uint64_t requested; /* amount requested when it ran out                    */
    int32_t wave;       /* wavefront that detected it                          */
    int32_t job;        /* job slot being served, -1 if unknown                */
} gtap_error_report;

/* ---- serving: continuous admission into a running kernel ------------------ */
/* Not in the paper (its launch runs one root to completion); this is the
 * serving extension of the same runtime.  The host appends jobs to an
 * admission ring in pinned host memory while the persistent kernel runs; a
 * few wavefronts poll the ring and admit jobs while fewer than max_inflight
 * are in flight and the frame pools keep headroom_small / headroom_big
 * frames free after admission (admission by free frame-pool memory).
 * Results are written to pinned host memory as roots complete.  Job slots
 * (max_jobs of them) are reused: ticket t uses slot t mod max_jobs, and a
 * slot is free again once its previous ticket completed.  k-clique CSR
 * buffers are borrowed until the job completes. */

/* Reset the scheduler state and launch the persistent kernel in serving mode
 * on cfg->stream (asynchronous).  cfg->timeout_ms bounds the whole serving
 * session.  Errors: GTAP_E_STATE (jobs pending or already serving),
 * GTAP_E_NOMEM (pinned memory), GTAP_E_HIP. */
int gtap_serve_start(gtap_ctx *ctx, uint32_t max_inflight, uint32_t headroom_small,
                     uint32_t headroom_big);

/* Append one job to the admission ring; *ticket identifies it.  Arguments as
 * for gtap_submit.  GTAP_E_FULL when the job's slot still holds an
 * unfinished job. */
int gtap_serve_submit(gtap_ctx *ctx, int32_t kind, const void *args, size_t args_bytes,
                      uint64_t *ticket);

/* Non-blocking: GTAP_OK and *result once ticket completed, else
 * GTAP_E_PENDING.  *done_ticks (optional) receives the device wall clock at
 * completion. */
int gtap_serve_poll(gtap_ctx *ctx, uint64_t ticket, int64_t *result, uint64_t *done_ticks);

/* Wait (up to wait_ms) for every submitted job, then stop the kernel and
 * wait for it.  Returns the device's abort code if it aborted, GTAP_E_TIMEOUT
 * if jobs were still pending after wait_ms (the kernel is stopped anyway once
 * they drain or its watchdog fires). */
int gtap_serve_stop(gtap_ctx *ctx, uint32_t wait_ms);

/* One job of a request trace: kind, argument struct (as for gtap_submit,
 * args_bytes <= 32) and its arrival time in seconds from the trace start. */
typedef struct gtap_trace_job {
    int32_t kind;
    uint32_t args_bytes;
    double arrival_s;
    uint64_t args[4];
} gtap_trace_job;

typedef struct gtap_trace_result {
    int64_t result;
    double submit_s;   /* host time the job entered the system               */
    double done_s;     /* host time its completion was observed              */
    int32_t status;    /* GTAP_OK, or the error that stopped the trace       */
    int32_t reserved;
} gtap_trace_result;

/* Host request loop against a serving kernel (gtap_serve_start first): submit
 * each job at its arrival time (open loop; a full ring delays it), poll
 * completions, record host times.  Returns when every job completed, on a
 * device error, or after timeout_ms. */
int gtap_trace_run(gtap_ctx *ctx, const gtap_trace_job *jobs, size_t n, gtap_trace_result *out,
                   uint32_t timeout_ms);

/* Baseline for the same trace: one persistent launch per job, in arrival
 * order on the context's stream (a job that arrives while another runs
 * waits).  Not valid while serving. */
int gtap_trace_run_plain(gtap_ctx *ctx, const gtap_trace_job *jobs, size_t n,
                         gtap_trace_result *out);

int gtap_stats_get(gtap_ctx *ctx, gtap_stats *out);
int gtap_last_error(gtap_ctx *ctx, gtap_error_report *out);
const char *gtap_status_string(int32_t status);

/* ---- batching: configuration autotuner ---------------------------------------- */
/* Not in the paper (its configuration is chosen by hand).  Candidate values,
 * each list terminated by 0 (or by its length).  Every combination of
 * num_queues x (for num_queues > 1: DAQ class function x, for
 * GTAP_DAQ_KCLIQUE, daq_bounds sets) x waves_per_group x num_waves is tried
 * on the calibration jobs. */
typedef struct {
    int32_t num_queues[4];       /* 1 = DAQ off                                 */
    int32_t daq_policies[4];     /* class functions tried when num_queues > 1
                                    (gtap_daq_policy; an empty list means
                                    GTAP_DAQ_BY_KIND)                          */
    int32_t waves_per_group[4];
    int32_t num_waves[4];        /* a negative entry means 0 (occupancy maximum) */
    int32_t bounds_sets;         /* daq_bounds candidates in bounds[] (0..4)    */
    int32_t bounds[4][7];
    uint32_t repeats;            /* timed runs per candidate, the best counts (>= 1) */
    uint32_t reserved;
} gtap_tune_space;

typedef struct {
    int32_t candidates;          /* configurations tried                        */
    int32_t failed;              /* of those, aborted after pool growth         */
    double best_ms;              /* best wall time of the calibration batch     */
    double base_ms;              /* the same for the base configuration         */
    uint64_t small_frames_touched;  /* frame high-water of the best run        */
    uint64_t big_frames_touched;
} gtap_tune_report;

/* Run the calibration jobs (one batch, one gtap_run per timed repeat after an
 * untimed warm-up) under every candidate configuration derived from *base and
 * write the fastest to *best.  A candidate that exhausts a frame pool is
 * retried with that pool doubled, up to three times.  The chosen
 * configuration's frame pools are then sized to max(4 x the frames the best
 * run touched, 2^20), capped at the base sizes.  Contexts are created and
 * finalized internally (library-owned workspaces; base->workspace_dev is
 * ignored).  n <= base->max_jobs.  k-clique job buffers are borrowed for the
 * duration of the call.  Errors: GTAP_E_INVAL, or the base configuration's
 * own failure. */
int gtap_autotune(const gtap_config *base, const gtap_trace_job *calib, size_t n,
                  const gtap_tune_space *space, gtap_config *best, gtap_tune_report *report);

/* ---- allocation-free batch run --------------------------------------------------- */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): the same batch
 * as gtap_init + one gtap_submit per job + gtap_run + gtap_result +
 * gtap_finalize, but the runtime's workspace (control block, job table,
 * deques, frame pools) is a static device array of GTAP_STATIC_SCRATCH_BYTES
 * inside the library, one per device, held from the first call on that device
 * until the process ends.  The call performs no hipMalloc, hipFree, host
 * pinned allocation or event creation; it launches on cfg->stream and waits
 * for it.
 *   cfg:     as for gtap_init; max_jobs, workspace_dev and workspace_bytes are
 *            ignored (the job table holds exactly n jobs);
 *   jobs:    host array of n jobs (kind and argument struct as for
 *            gtap_submit, arrival_s ignored); kinds GTAP_KIND_FIB, _NQUEENS,
 *            _UTS and _KCLIQUE only (the other kinds allocate per-job buffers);
 *            device pointers inside the arguments are borrowed until return;
 *   results: host array receiving job i's result at index i;
 *   report:  NULL, or receives the structured report of a device abort
 *            (as gtap_last_error would), zeroed otherwise.
 * n <= GTAP_STATIC_MAX_JOBS.  Errors: GTAP_E_INVAL (arguments, kinds,
 * configuration), GTAP_E_NOMEM (the configuration's workspace, as reported by
 * gtap_workspace_size for max_jobs = n, exceeds GTAP_STATIC_SCRATCH_BYTES:
 * shrink the frame pools or deques), GTAP_E_CAPACITY / GTAP_E_TIMEOUT (the
 * device run aborted: see *report), GTAP_E_HIP.  Every call on a device
 * uses that device's one array: calls that overlap on one device (from two
 * host threads, or on two streams) race and must not be made; each call
 * clears the state it needs first, so back-to-back calls are independent. */
#define GTAP_STATIC_SCRATCH_BYTES (256u << 20)
#define GTAP_STATIC_MAX_JOBS 4096u
int gtap_run_static(const gtap_config *cfg, const gtap_trace_job *jobs, size_t n, int64_t *results,
                    gtap_error_report *report);

/* ---- platform probes ------------------------------------------------------------ */
/* Not in the paper: measurements of the two platform properties the runtime's
 * design rests on (its hand-offs use relaxed device-scope accesses ordered by
 * waiting for completion instead of release/acquire fences, Sec. 5.1.3's
 * publication fence and count update).  Both launch on `stream` (NULL = the
 * default stream), wait for it, and use only the caller's device buffer. */

/* Device-scope 64-bit fetch-add throughput.  `blocks` workgroups of 256
 * threads; every issuing lane performs `iters` RMWs with return:
 *   GTAP_PROBE_DISTINCT  every lane on its own 64-byte line (like the join
 *                        words of different frames); words >= blocks*256*8
 *   GTAP_PROBE_PER_WAVE  lane 0 of each wavefront on that wavefront's word
 *                        (like a deque count); words >= blocks*4*16
 *   GTAP_PROBE_ONE_WORD  lane 0 of every wavefront on one word; words >= 1
 * words_dev: caller-owned uint64 device array of `words` entries (contents
 * overwritten).  *rmw_per_s receives RMWs / kernel time, *ms the kernel time.
 * Errors: GTAP_E_INVAL (mode, sizes, iters outside 1..65536, blocks outside
 * 1..65536), GTAP_E_HIP. */
enum gtap_probe_mode { GTAP_PROBE_DISTINCT = 0, GTAP_PROBE_PER_WAVE = 1, GTAP_PROBE_ONE_WORD = 2 };
int gtap_probe_atomics(int32_t mode, uint32_t blocks, uint32_t iters, uint64_t *words_dev, uint64_t words,
                       void *stream, double *rmw_per_s, double *ms);

/* Litmus tests between the two one-wavefront workgroups of each of `pairs`
 * pairs (workgroups 2p and 2p+1, which the dispatcher places on different
 * XCDs; the XCC ids read by each workgroup are checked), 64 lane instances
 * per pair, each on its own 128-byte lines, with relaxed device-scope stores
 * and loads and, when `ordered`, a wait for completion between the two
 * accesses of each thread:
 *   test 0, message passing: the writer stores data = k then flag = k for
 *     k = 1..rounds; the reader, 4*rounds times, loads flag then data and
 *     counts data < flag (stale: forbidden when ordered);
 *   test 1, store buffering: in round r = 1..rounds, A stores x = r then
 *     loads y, B stores y = r then loads x; both loads seeing a value below r
 *     is forbidden when ordered.
 * buf_dev: caller-owned device memory of at least
 * pairs * (16384 + 512 * rounds) + 16384 bytes.  No wait in the
 * kernels depends on the other workgroup: every run ends.
 * Errors: GTAP_E_INVAL (test, pairs outside 1..1024, rounds outside
 * 1..65536, null pointers), GTAP_E_NOMEM (buffer too small), GTAP_E_HIP. */
typedef struct {
    uint64_t instances;       /* lane pairs tested (64 per workgroup pair)     */
    uint64_t mp_reads;        /* message passing: flag-then-data reads         */
    uint64_t mp_stale;        /*   of those, data older than the flag          */
    uint64_t mp_overlap;      /*   of those, a flag strictly inside (0, rounds):
                                   reader and writer ran at the same time     */
    uint64_t sb_rounds;       /* store buffering: rounds over all instances     */
    uint64_t sb_both_new;     /*   both loads saw the other's round-r store     */
    uint64_t sb_a_new_only;
    uint64_t sb_b_new_only;
    uint64_t sb_both_old;     /*   neither did (forbidden when ordered)         */
    int32_t pairs;
    int32_t pairs_on_distinct_xcds;
} gtap_litmus_result;
int gtap_litmus(int32_t test, int32_t ordered, uint32_t pairs, uint32_t rounds, void *buf_dev, uint64_t buf_bytes,
                void *stream, gtap_litmus_result *out);

#ifdef __cplusplus
}
#endif
#endif /* GTAP_H */
