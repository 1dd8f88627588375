/*
 * simplexmap.h -- C ABI of the MI355X (gfx950) block-space thread maps for
 * discrete orthogonal m-simplex domains.
 *
 * Domain (Section 1, Eq. 1):
 *     Delta_n^m = { x in Z_+^m : 0 <= x_i <= n, x_1 + ... + x_m <= n },
 * with C(n+m, m) elements, m in {2, 3, 4}.
 *
 * Data layout of every buffer: the (n+1)^m bounding box, row-major, x_1
 * fastest; element x is at index i(x) = sum_k x_k (n+1)^(k-1).  Buffers are
 * device pointers owned by the caller; the library never allocates, frees
 * or retains them.  Elements outside the simplex are never written, and
 * input elements outside it are never used as data (they may hold anything).
 *
 * Work decomposition: the box is cut into tiles of rho^m elements.  The
 * tiles that meet the simplex form the block simplex
 *     { b in Z_+^m : b_1 + ... + b_m <= floor(n / rho) },
 * and one workgroup (the paper's "block", Section 4.1, Theorem 1) processes
 * one tile.  The H launch maps a reduced workgroup grid onto the block
 * simplex (Section 4.1: Theorem 1 and eq_map2d for m = 2; Section 4.3: the
 * 3-D theorem, eq_3simplex_map and its hinge for m = 3; Section 6: the
 * self-similar set with scale r and replication beta, eq_generic-m, for
 * m = 4; general n by a native power-of-two part plus shell layers, in the
 * spirit of Section 4.2's trapezoids).  The BB launch
 * covers the whole box of tiles and discards tiles outside the simplex
 * (Section 2, the bounding-box map f(x) = x).
 *
 * Operations (Section 5.1, Table tab:tests, plus a hit counter and a hash):
 *   SMAP_OP_MAP   mapping only; reads and writes nothing.      in, out: unused
 *   SMAP_OP_ACCUM out[i] = in[i] + 1 (uint32, mod 2^32).        in, out: uint32
 *                 in == out (in place) is allowed.
 *   SMAP_OP_HITS  out[i] += 1 (atomic, uint32): coverage probe. out: uint32
 *   SMAP_OP_HASH  out[i] = hash32(x): FNV-1a over the 32-bit words x_1..x_m
 *                 (basis 0x811C9DC5, prime 0x01000193) then MurmurHash3's
 *                 fmix32 finaliser.  Project-defined.          out: uint32
 *   SMAP_OP_CA2   one Life step, B3/S23 over the Moore 8-neighbourhood,
 *                 m = 2 only.                                   in, out: uint8
 *   SMAP_OP_CA3   one step of rule B6/S567 over the 26-neighbourhood,
 *                 m = 3 only.                                   in, out: uint8
 *   SMAP_OP_EDM   Euclidean distance matrix (Section 5.1, test 3), m = 2
 *                 only: out[x] = float32 distance between points i = x_1
 *                 and j = n - x_2 (x_1 + x_2 <= n is i <= j, the diagonal
 *                 i = j being x_1 + x_2 = n), computed in float32 as
 *                 sqrtf(dx^2 + dy^2 + dz^2).  in: n+1 points in R^3 as
 *                 float32 (x, y, z) triples, 16-byte aligned; out: float32
 *                 (n+1)^2 box.
 *   For CA ops the cells in the simplex must hold 0 or 1 (1 = alive);
 *   neighbours outside the simplex count as dead; in and out must not
 *   overlap (ping-pong between two buffers across steps).
 *
 * Streams and errors: every launch call enqueues on `stream` (a hipStream_t;
 * NULL = the null stream) and returns without synchronising.  Arguments are
 * checked before anything is enqueued; on error nothing is launched and a
 * negative status is returned.  A launch failure reported by the runtime
 * returns SMAP_EHIP.  Faults inside a kernel surface at the caller's next
 * synchronisation.  No call aborts or prints.  All calls are thread-safe.
 */
#ifndef SIMPLEXMAP_H
#define SIMPLEXMAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SMAP_OK            0
#define SMAP_EINVAL       (-1) /* bad m, n, op, pointer or buffer overlap       */
#define SMAP_EUNSUPPORTED (-2) /* valid but unsupported (r, beta) or tile       */
#define SMAP_ERANGE       (-3) /* sizes overflow the supported index ranges     */
#define SMAP_EHIP         (-4) /* the HIP runtime reported a launch error       */

/* operations */
#define SMAP_OP_MAP   0
#define SMAP_OP_ACCUM 1
#define SMAP_OP_HITS  2
#define SMAP_OP_HASH  3
#define SMAP_OP_CA2   4
#define SMAP_OP_CA3   5
#define SMAP_OP_EDM   6

/* Description of one launch plan (filled by simplex_plan_info). */
struct simplex_plan_info {
    int32_t  m;
    int32_t  use_bb;          /* 1: bounding-box launch, 0: H launch            */
    int64_t  n;
    int32_t  r;               /* 1/r, the reciprocal of the scale (H only)       */
    int32_t  beta;            /* replication factor (H only)                     */
    int32_t  rho;             /* tile side in elements                           */
    int32_t  wg_threads;      /* threads per workgroup                           */
    int32_t  tile_side_k;     /* K = floor(n/rho) + 1, side of the block simplex */
    int32_t  native_n;        /* N = 2^j: the native part covers sum(b) <= N-2   */
    int32_t  shell_layers;    /* L = K - (N-1)                                   */
    int32_t  n_pieces;        /* pieces of the fused H launch (native + shell)   */
    int32_t  wgs_per_tile;    /* workgroups per tile (row sub-blocks), >= 1      */
    uint64_t useful_elements; /* C(n+m, m)                                       */
    uint64_t useful_tiles;    /* tiles meeting the simplex: C(K-1+m, m)          */
    uint64_t launched_tiles;  /* tiles (map units) in the launch grid            */
    uint64_t launched_wgs;    /* workgroups: launched_tiles * wgs_per_tile       */
    uint64_t native_wgs;      /* tiles in the native piece (H only)              */
    uint64_t full_tiles;      /* tiles lying entirely inside the simplex         */
    int32_t  tiles_per_wg;    /* map units per workgroup (pointwise ops), >= 1;
                                 above 1, launched_wgs is ceil(launched_tiles /
                                 tiles_per_wg) for H, ceil(kbox / tiles_per_wg)
                                 workgroups per row of the tile grid for BB   */
};

/*
 * H launch: run `op` over Delta_n^m with the block-space map H.
 *   m      2, 3 or 4 (m = 1 needs no map, Section 4).
 *   n      >= 0.
 *   r      1/r as an integer: 2 is the paper's r = 1/2; 0 selects the default.
 *   beta   replication factor; 0 selects the default.  Supported (r, beta):
 *          m = 2: (2, 2); m = 3: (2, 2) with the hinge fold; m = 4: (2, 3)
 *          with the fold (default) or (2, 4) without it.  Others return
 *          SMAP_EUNSUPPORTED.
 *   op     SMAP_OP_*; CA2 needs m = 2 and CA3 needs m = 3.
 *   buf_in, buf_out   device pointers to (n+1)^m-element boxes (see above);
 *          unused pointers may be NULL.
 *   stream hipStream_t to enqueue on.
 * Returns SMAP_OK or a negative status.
 */
int simplex_map_launch(int m, int64_t n, int r, int beta, int op,
                       const void *buf_in, void *buf_out, void *stream);

/*
 * BB launch (the baseline): same operation and buffers as simplex_map_launch,
 * launched over the whole box of tiles; tiles outside the simplex exit at
 * once and partial tiles filter their elements (Section 2).  The grid is
 * 2-D (m = 2), 3-D (m = 3), or 3-D with z = b_3 + kbox * b_4 (m = 4), where
 * kbox = ceil((n+1)/rho); a y or z extent above 65535 returns SMAP_ERANGE.
 */
int simplex_bb_launch(int m, int64_t n, int op,
                      const void *buf_in, void *buf_out, void *stream);

/* *out = C(n+m, m), the number of elements of Delta_n^m (Eq. 1).
 * SMAP_ERANGE if it does not fit in 64 bits, SMAP_EINVAL for bad m, n, out. */
int simplex_count(int m, int64_t n, uint64_t *out);

/* Fill *out with the plan that the corresponding launch would use (no GPU
 * work).  use_bb selects simplex_bb_launch's plan (r, beta ignored). */
int simplex_plan_info(int m, int64_t n, int r, int beta, int op, int use_bb,
                      struct simplex_plan_info *out);

/*
 * Host-side decode of every workgroup of a plan, in launch order (no GPU
 * work; the same decode functions the kernels run).  For workgroup w,
 * tiles[5w] = 1 if it maps onto a tile and 0 if it is discarded, and
 * tiles[5w+1 .. 5w+m] = its tile coordinates b_1..b_m (unused entries 0).
 * At most `cap` entries are written; *written receives the number of
 * launched tiles of the plan (the map's units; a tile may be processed by
 * several workgroups).  tiles may be NULL to only query the count.
 */
int simplex_plan_tiles(int m, int64_t n, int r, int beta, int op, int use_bb,
                       int32_t *tiles, uint64_t cap, uint64_t *written);

/*
 * Select the tile side rho and workgroup size for (m, op) in later calls of
 * this process (both launch kinds).  rho = 0 restores the default.  Only
 * the compiled combinations are accepted (others: SMAP_EUNSUPPORTED):
 *   MAP/ACCUM/HITS/HASH  m=2: rho 32 (256 threads), 16 (64), 64 (256), 128 (256)
 *                        m=3: rho 16 (256), 8 (128), 32 (256)
 *                        m=4: rho 8 (256; two tiles per workgroup), 4 (64), 16 (256)
 *                        (the first listed rho of each m is the default; more
 *                        shapes through simplex_set_shape)
 *   CA2 (m=2): rho 1024 (64 threads; 128 or 256), 512 (512), 256 (256),
 *              128 (128), 2048 (128 or 256), 4096 (256).  From 2048 on
 *              the waves of a workgroup stand side by side along x, each
 *              on a 1024-byte column of the tile.
 *   Large tiles are split into sub-blocks of rows (and planes), one
 *   workgroup each (wgs_per_tile in the plan info).
 *   CA3 (m=3): rho 256 (256 threads, the default from n = 768 on; or 128
 *              or 512), 128 (256, the default below n = 768; or 128 or
 *              512), 64 (128 or 256), 32 (64).
 * wg_threads = 0 picks the first listed size; any other value must be one
 * of the listed sizes.
 */
int simplex_set_tile(int m, int op, int rho, int wg_threads);

/*
 * simplex_set_tile with the number of tiles per workgroup as well, for the
 * pointwise ops (MAP, ACCUM, HITS, HASH): a workgroup then takes
 * tiles_per_wg consecutive map units -- which the H map places
 * x_1-adjacent wherever a cube of the map runs along x_1 -- with its lanes
 * side by side across their rows, so one store of a wave covers
 * tiles_per_wg tile rows of contiguous memory (for BB: tiles_per_wg
 * x_1-adjacent box tiles).  Compiled shapes beyond simplex_set_tile's:
 *   m=4: rho 8 (256 threads: 2, 4 or 8 tiles; 128 threads: 2 or 4 tiles;
 *        64 threads: 1, 2 or 4 tiles), rho 4 (256 threads: 8 or 16 tiles)
 *   m=3: rho 16 (256 threads: 2 tiles; 64 threads: 1 or 2 tiles),
 *        rho 8 (256 threads: 4 tiles)
 *   m=2: rho 32 (64 threads: 1 or 2 tiles)
 * tiles_per_wg = 0 takes the first listed grouping of (rho, wg_threads)
 * (simplex_set_tile's choice; 1 for the shapes simplex_set_tile lists), 1
 * asks for one tile per workgroup.  The automata accept 0 or 1 only.
 * Returns SMAP_EUNSUPPORTED for a combination that is not compiled,
 * SMAP_EINVAL for a negative wg_threads or tiles_per_wg.
 */
int simplex_set_shape(int m, int op, int rho, int wg_threads, int tiles_per_wg);

/*
 * Layout of the native part of the 3-D H map for later launches of this
 * process (H launches, plans and plan info; BB is not affected):
 *   SMAP_LAYOUT_AUTO (default): LEVELS for one-job CA3 launches (one step
 *     or several generations, their plans and plan info), PACKED for the
 *     per-element ops and for the batched and work-queue launches;
 *   SMAP_LAYOUT_PACKED: the packed grid (N/2) x (N/2) x (N/2 + N/4)
 *     of Section 4.3, one launch, 1/8 of its workgroups discarded
 *     (launched / useful tiles of the native part -> 9/8);
 *   SMAP_LAYOUT_LEVELS: the fully efficient variant of Section 4.3 (one
 *     parallel space per level of the recursion), realised as the levels'
 *     ranges concatenated into one launch; level l holds 2^l cubes of side
 *     N/2^(l+1), every workgroup lands on a tile (launched = useful).
 * Only m = 3 is accepted (others: SMAP_EINVAL); an unknown layout gives
 * SMAP_EINVAL.
 */
#define SMAP_LAYOUT_AUTO (-1)
#define SMAP_LAYOUT_PACKED 0
#define SMAP_LAYOUT_LEVELS 1
int simplex_set_layout(int m, int layout);

/*
 * How an H launch (simplex_map_launch) runs the pieces of its plan when n is
 * not of the native form (the native map plus the shell pieces, which play
 * the role of the concurrent trapezoids of Section 4.2), in later calls of
 * this process:
 *   SMAP_GENERAL_FUSED (default): all pieces in one launch; a workgroup
 *     finds its piece from the piece table.
 *   SMAP_GENERAL_STREAMS: one launch per piece, each on a stream of its own
 *     so the pieces run concurrently.  The streams (default priority) and
 *     their events are created on the first such launch on a device and kept
 *     until the process ends; the pieces start after the work already
 *     enqueued on the caller's stream, and later work on that stream waits
 *     for all of them.  Results are identical to the fused launch.
 * Errors: SMAP_EINVAL for an unknown strategy.
 */
#define SMAP_GENERAL_FUSED 0
#define SMAP_GENERAL_STREAMS 1
int simplex_set_general(int strategy);

/* ---- autotuning and graphs ------------------------------------------------
 *
 * Theorem 3 (Section 6) frames the choice of the scale and replication
 * parameters as an optimisation; here the choice of (beta, rho, workgroup
 * size) for one (m, n, op) is made by measurement.
 */
struct simplex_tune_result {
    int32_t rho;
    int32_t wg_threads;
    int32_t beta;
    float us;             /* mean duration of one H launch, microseconds */
    int32_t tiles_per_wg; /* map units per workgroup of the chosen shape */
};

/*
 * Times every compiled shape (rho, workgroup size, tiles per workgroup) of
 * (m, op) -- and beta 3 and 4 for m = 4 -- with `reps` H launches each (after 2 warm-up launches) on
 * `stream`, picks the fastest, and installs it for later H launches of this
 * (m, n, op class) in this process (the tile of simplex_set_tile still
 * applies to other n, and to BB).  A later simplex_map_launch with beta = 0
 * uses the tuned beta.  Buffers as for simplex_map_launch; for the automata
 * every timed launch steps buf_in into buf_out (so buf_out ends with one
 * step of buf_in); ACCUM must not run in place here (buf_in != buf_out).
 * Synchronises `stream`.
 *
 * cache_path (may be NULL): a text file of earlier results, one line per
 * (device, m, n, op) ("smap-tune-v2 <device> m n op rho threads
 * tiles_per_wg beta us"; lines of other formats are ignored).  If it holds
 * this key, that result is installed and returned with no timing;
 * otherwise the new result is appended.
 *
 * Errors as for simplex_map_launch; reps < 1 gives SMAP_EINVAL; a cache
 * file that cannot be written gives SMAP_EINVAL after installing the result.
 */
int simplex_autotune(int m, int64_t n, int op, const void *buf_in, void *buf_out, int32_t reps,
                     const char *cache_path, void *stream, struct simplex_tune_result *best);

/*
 * Drops every tuned entry (simplex_autotune) of this process.
 */
int simplex_autotune_reset(void);

/*
 * Captures `steps` launches of op over (m, n) -- H, or BB when use_bb is
 * non-zero (r and beta are then ignored) -- into a HIP graph (an
 * executable graph instance, *graph).  Pointwise ops repeat the same launch
 * (ACCUM in place adds `steps` per replay); the automata alternate
 * buf_in -> buf_out, buf_out -> buf_in, ... (an even `steps` leaves the
 * result in buf_in).  The capture uses the tile and plan current at
 * creation.  Nothing runs until simplex_graph_launch.  No memset nodes are
 * recorded.  Errors as for simplex_map_launch; steps < 1 or a NULL graph
 * gives SMAP_EINVAL; a capture or instantiation failure gives SMAP_EHIP.
 */
int simplex_graph_create(int m, int64_t n, int r, int beta, int op, int use_bb, const void *buf_in,
                         void *buf_out, int32_t steps, void **graph);

/* Enqueues one replay of the graph on `stream`. */
int simplex_graph_launch(void *graph, void *stream);

/* Frees the graph (after its replays have finished). NULL is a no-op. */
int simplex_graph_destroy(void *graph);

/* Static, human-readable text for a status code. */
const char *simplex_strerror(int status);

/*
 * Measurement probe (no operation of the paper): copies the simplex cells of
 * a uint8 (n+1)^m box, m = 2 or 3, from buf_in to buf_out, row by row (the
 * cells x_1 = 0 .. n - (x_2 + ... + x_m) of each row are contiguous), with
 * no tiles, no halo and no map.  It moves exactly the bytes of one automaton
 * step (Section 5.1: one read and one write per simplex cell), so its time
 * is the floor that the bounding-box layout puts on one pass over the
 * simplex.  Cells outside the simplex are neither read nor written.
 *   buf_in, buf_out: device pointers to (n+1)^m bytes, not overlapping.
 * Enqueues on `stream` and returns without synchronising.  Errors:
 * SMAP_EINVAL for m not in {2, 3}, n < 0, a NULL or overlapping buffer;
 * SMAP_ERANGE for boxes beyond the index range; SMAP_EHIP for a launch
 * failure.
 */
int simplex_copy_launch(int m, int64_t n, const void *buf_in, void *buf_out, void *stream);

/* ---- several generations per launch -------------------------------------
 *
 * `steps` generations of the automaton (Section 5.1 runs a fixed number of
 * steps) with temporal blocking: each pass loads a tile plus a halo into
 * LDS and advances it as many generations as the halo is wide, so HBM is
 * read and written once per pass instead of once per generation.
 * Supported (others: SMAP_EUNSUPPORTED):
 *   m = 2, SMAP_OP_CA2: 256 x 256 tiles, halo 32: up to G = 32 per pass;
 *   m = 3, SMAP_OP_CA3: 64^3 tiles, halo 16: up to G = 16 per pass.
 *
 * buf_out receives the state after `steps` generations of buf_in (layout
 * and rules as for simplex_map_launch; the buffers must not overlap).
 * With steps <= G one pass runs and buf_in is left unchanged; with more,
 * passes alternate between the two buffers (an odd number of passes, the
 * last one writing buf_out) and buf_in's simplex cells are overwritten
 * with intermediate states.  Cells outside the simplex are never written.
 * steps < 1 gives SMAP_EINVAL; other errors as for simplex_map_launch.
 */
int simplex_map_launch_steps(int m, int64_t n, int r, int beta, int op, int32_t steps, void *buf_in,
                             void *buf_out, void *stream);

/* The same passes with the bounding-box map (the baseline). */
int simplex_bb_launch_steps(int m, int64_t n, int op, int32_t steps, void *buf_in, void *buf_out,
                            void *stream);

/* ---- batched launch ---------------------------------------------------
 *
 * One job of a batched launch: one automaton step over Delta_n^m with the
 * job's own buffers (layout and rules as for simplex_map_launch).
 *   m = 2 with op SMAP_OP_CA2, or m = 3 with op SMAP_OP_CA3; n >= 0.
 *   buf_in, buf_out: device pointers to (n+1)^m uint8 cells, not
 *   overlapping each other.  Different jobs may share an input buffer but
 *   no job's output may overlap any buffer of another job in the batch.
 */
struct simplex_job {
    int32_t m;
    int32_t op;
    int64_t n;
    const void *buf_in;
    void *buf_out;
};

/*
 * Steps every job of `jobs[0..njobs)` with the H map in as few launches as
 * possible: the H-mapped tile ranges of all jobs of one op class are
 * concatenated into one grid, and a device-side table of the jobs'
 * workgroup prefix sums tells each workgroup which job and which tile it
 * takes (a binary search, wave-uniform), then decodes its tile with the
 * job's own H plan (default r and beta).  A step's result does not depend
 * on the map or the tiles, so every job's output equals what
 * simplex_map_launch gives for it alone.  Batched tiles: rho = 256 for CA2
 * (256 threads, one workgroup per tile), rho = 64 for CA3 (128 threads).
 *
 * The table travels from pinned host memory to device memory with an
 * asynchronous copy on `stream`, then the launch follows on `stream`; the
 * call returns without synchronising.  Tables are cut from a 32 MiB byte
 * ring per device (pinned host staging plus a device copy, allocated on
 * the first call and kept until the process ends); a table's bytes are
 * reused once the event recorded after its launch has completed, and the
 * call waits on the host only when the ring is full.  Jobs of one class are
 * launched together up to 4096 per launch (more are split over several
 * launches).
 *
 * Errors: SMAP_EINVAL for njobs < 0, a NULL `jobs` with njobs > 0, a job
 * with an unsupported (m, op), a negative n, NULL or overlapping buffers;
 * SMAP_ERANGE for sizes beyond the index range; SMAP_EHIP if an allocation,
 * copy or launch fails.  All jobs are checked before anything is enqueued.
 * njobs == 0 is a no-op.
 */
int simplex_batch_launch(const struct simplex_job *jobs, int32_t njobs, void *stream);

/*
 * Steps every job of `jobs[0..njobs)` with the H map in ONE persistent
 * launch for all classes (CA2 and CA3 jobs mixed), through a device-side
 * work queue of H-mapped block ranges.  A work unit is one H-mapped tile
 * (CA2, rho = 256) or one of the 4 sub-blocks of an H-mapped tile (CA3,
 * rho = 64); the units of all jobs are concatenated, job after job.  The
 * grid holds only as many workgroups (256 threads) as the device runs at
 * once — occupancy times compute units, or max_workgroups if that is
 * smaller and non-zero — and each workgroup claims unit after unit with an
 * atomic add on a head counter in device memory, until the head reaches
 * the tail (the unit count, fixed at launch); a claimed unit is mapped to
 * its job by a binary search over the unit prefix sums and decoded with
 * the job's own H plan (Section 4; the blocks of a job's reduced grid are
 * the units).  Outputs equal those of simplex_map_launch for each job
 * alone.
 *
 * Tables (head counter, prefix sums, jobs) come from the same ring as
 * simplex_batch_launch's and travel with an asynchronous copy on `stream`;
 * the call returns without synchronising.  Up to 4096 jobs go in one
 * launch (more are split over several launches).  max_workgroups: 0 for
 * the device's resident count, or a smaller positive cap (a cap of 1 runs
 * every unit on one workgroup).  Errors are those of simplex_batch_launch,
 * plus SMAP_EINVAL for max_workgroups < 0.
 */
int simplex_queue_launch(const struct simplex_job *jobs, int32_t njobs, int32_t max_workgroups,
                         void *stream);

/*
 * Captures ONE persistent work-queue launch (simplex_queue_launch) over the
 * fixed job set jobs[0..njobs) into a graph, for replay with
 * simplex_graph_launch and release with simplex_graph_destroy.  The job
 * table (head counter, unit prefix sums, jobs' plans and pointers) is
 * copied once, at creation, into device memory that the graph owns (freed
 * by simplex_graph_destroy); each replay first clears the head counter with
 * a one-workgroup fill kernel (the graph holds no memset node), then runs
 * the queue kernel.  The jobs' buffers must stay valid while the graph
 * exists; a replay reads buf_in and writes buf_out of every job, so
 * replays that overlap on the device race on those buffers (and on the
 * head counter).  njobs is at most 4096 (SMAP_ERANGE beyond);
 * max_workgroups as for simplex_queue_launch.  Errors: those of
 * simplex_queue_launch, SMAP_EINVAL for a NULL graph or njobs < 1,
 * SMAP_EHIP if the allocation, copy, capture or instantiation fails.
 */
int simplex_queue_graph_create(const struct simplex_job *jobs, int32_t njobs, int32_t max_workgroups,
                               void **graph);

/*
 * For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the persistent
 * work-queue launch of simplex_queue_launch, with the same jobs, kernel and
 * results, but its job table (head counter, unit prefix sums, jobs) kept in
 * a fixed device array inside the library instead of the allocated ring.
 * No call allocates or frees device or pinned memory; the array (about
 * 100 KB per device, for at most 256 jobs) and a pageable host staging copy
 * are taken on the first call on a device and held until the process ends.
 * The table travels with an asynchronous copy on `stream`, the head counter
 * starting at zero as part of it (no memset); before rewriting the staging
 * copy, a call waits on the host for the previous call's copy to finish.
 * Every call on a device shares that device's array and leaves the last
 * call's table in it: calls on one device must be ordered (one stream, or
 * streams the caller synchronises); calls that overlap on the device race.
 * Errors: those of simplex_queue_launch, and SMAP_ERANGE for njobs > 256.
 */
int simplex_queue_launch_static(const struct simplex_job *jobs, int32_t njobs, int32_t max_workgroups,
                                void *stream);

/* ---- serving loop -------------------------------------------------------
 *
 * A request stream of automaton-step jobs (the continuous-batching serving
 * loop).  Each job's input is already resident on the device; its output
 * is placed in a device arena whose size is the memory budget.
 */
struct simplex_serve_job {
    int32_t m;            /* 2 (op SMAP_OP_CA2) or 3 (op SMAP_OP_CA3) */
    int32_t op;
    int64_t n;
    const void *buf_in;   /* device, (n+1)^m uint8 cells */
    double arrival_s;     /* arrival time, seconds after the start of the run;
                             non-decreasing over the job array */
};

/* What happened to one job, in seconds after the start of the run.  Host
 * clock times are exact; done_s comes from a device event and is placed on
 * the host clock through the start event (whose own time is taken as the
 * midpoint of its record-and-wait, an uncertainty of a few microseconds). */
struct simplex_serve_record {
    double admit_s;       /* output memory granted (host) */
    double launch_s;      /* its launch enqueued (host) */
    double done_s;        /* its launch finished on the device (device event) */
    double release_s;     /* completion seen and memory returned (host) */
    uint64_t out_offset;  /* byte offset of its output in the arena */
    int32_t batch;        /* index of the launch group that ran it */
    int32_t status;       /* SMAP_OK, or the error of its launch */
};

#define SMAP_SERVE_SEQUENTIAL 0  /* one simplex_map_launch per job, in arrival order */
#define SMAP_SERVE_BATCHED 1     /* continuous batching with simplex_batch_launch */
#define SMAP_SERVE_PERSISTENT 2  /* continuous batching with simplex_queue_launch */

/*
 * Replays `jobs` in real time on the current device and returns when every
 * job has completed.  The inputs must be ready before the call (the loop
 * runs on streams of its own: synchronise the device after producing them).  Admission is by memory: a job is admitted, in arrival
 * order, once its (n+1)^m output bytes (rounded up to 256) fit in the
 * arena [arena, arena + arena_bytes); its memory returns to the arena when
 * its launch has completed, unless keep_outputs is non-zero (then every
 * output stays where it was written, and the arena must hold all of them).
 *
 * SMAP_SERVE_SEQUENTIAL: each admitted job is launched alone with the H map
 * as soon as it is admitted, all on one stream.
 * SMAP_SERVE_BATCHED: admitted jobs wait for a launch slot; whenever fewer
 * than `max_inflight` batches are running, all admitted, not yet launched
 * jobs go out as one simplex_batch_launch.  Batches alternate between two
 * streams of the default priority (created and destroyed by the call), so
 * consecutive batches overlap on the device.  Jobs that arrive while
 * others run join the next batch.
 * SMAP_SERVE_PERSISTENT: as SMAP_SERVE_BATCHED, but each batch goes out as
 * one simplex_queue_launch (all classes in one persistent launch).
 * Before the clock starts, one tiny step
 * of each class runs on every stream of the loop (a kernel's first launch
 * in a process otherwise pays for loading its code object), on 16 KiB of
 * zeroed device memory the library keeps with its job tables (never on the
 * arena or a job's buffers).
 *
 * records (may be NULL) receives one entry per job.  Errors: SMAP_EINVAL for
 * bad arguments (including a job that could never fit the arena),
 * SMAP_EHIP for a runtime failure; the run stops at the first error after
 * waiting for the work already enqueued.
 */
int simplex_serve_run(const struct simplex_serve_job *jobs, int32_t njobs, void *arena,
                      uint64_t arena_bytes, int32_t mode, int32_t max_inflight,
                      int32_t keep_outputs, struct simplex_serve_record *records);

#ifdef __cplusplus
}
#endif

#endif /* SIMPLEXMAP_H */
