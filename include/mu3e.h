/*
 * mu3e.h -- C ABI of the MI355X (gfx950) online event selection for Mu3e.
 *
 * Method: V. Henkys, B. Schmidt, N. Berger, "Online Event Selection for
 * Mu3e using GPUs" (arXiv 2206.11535):
 *   Section IV-A  Selection Cuts (eq. sel-cut-delta-lambda, eq. sel-cut-phi,
 *                 eq. rt-cut; Alg. 2)
 *   Section IV-B  Track Reconstruction (eq. objective-function, triplet fit
 *                 linearised around the transverse circle, weighted mean
 *                 curvature, eq. objective-function-global, chi2 < 32; Alg. 3)
 *   Section IV-C  Vertex Fit (circle intersections, weighted 2D vertex,
 *                 eq. track-error, z back-projection, vertex chi2, signal
 *                 tests; Alg. 4)
 *   Section V     frame flow (Alg. 1), "marked for storage" on overflow.
 *
 * Conventions.  Units mm, MeV, tesla, radian.  Field along +z; positive
 * charges turn clockwise seen from +z and have positive signed circumradius
 * and curvature.  Hits are float32 structure-of-arrays, sorted by frame and
 * then layer; frame f, layer l owns hits [layer_offsets[4f+l],
 * layer_offsets[4f+l+1]).  Indices and counts are int32, flags uint32.
 *
 * Memory.  Unless stated otherwise every pointer is a DEVICE pointer and
 * every buffer is owned by the caller; the library never allocates on these
 * paths.  Scratch memory is a caller-provided workspace whose size is
 * queried first.  Every call is asynchronous on the given HIP stream
 * (NULL = default stream) and re-entrant for distinct workspaces.
 *
 * Errors.  Argument errors are reported synchronously as a negative status
 * and nothing is launched.  Conditions only known on the device (a candidate
 * list in the workspace filled up) are reported in the workspace's status
 * word, readable after the stream has been synchronised (mu3e_debug_t), and
 * every frame they touched carries MU3E_LIST_FULL | MU3E_KEEP: a frame is
 * either fully processed or kept.
 * Exceeding a *method* cap (max_triplets, max_tracks, max_combos) is not an
 * error: the frame's overflow flag is set and the frame is kept, as the
 * paper's implementation marks such frames for storage.  max_layer_hits is a
 * capacity of this implementation, not of the method (frame-local hit
 * indices are packed in 10 bits): a frame above it is kept unprocessed, the
 * same fail-safe.
 */
#ifndef MU3E_H
#define MU3E_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MU3E_OK = 0,
  MU3E_ERR_INVALID_ARG = -1,   /* null pointer, negative size, bad parameter */
  MU3E_ERR_HIP = -2,           /* a HIP runtime call failed                   */
  MU3E_ERR_CAPACITY = -3,      /* workspace too small for the request         */
  MU3E_ERR_UNSUPPORTED = -4    /* parameter beyond what the kernels support   */
} mu3e_status;

/* Per-frame flag bits (frame_flags). */
enum {
  MU3E_KEEP = 1u,          /* frame is kept (any other bit set)                */
  MU3E_TRIPLET_OVF = 2u,   /* more than max_triplets triplets passed the cuts  */
  MU3E_TRACK_OVF = 4u,     /* more than max_tracks tracks passed chi2 < max    */
  MU3E_COMBO_OVF = 8u,     /* more than max_combos e+e+e- triples passed dE    */
  MU3E_VERTEX = 16u,       /* a signal-like vertex was found                   */
  MU3E_HITS_OVF = 32u,     /* a layer holds more than max_layer_hits hits
                              (a capacity flag, see above)                     */
  MU3E_LIST_FULL = 64u     /* a workspace list of this call was full before the
                              frame was done (its selected triplets, the
                              float64 re-evaluation queue, or the vertex
                              stage's track table): the frame is kept without
                              the later stages, never passed on incomplete;
                              its triplet count stays exact                   */
};

/* Largest per-layer hit count the kernels process.  Layers are staged in LDS
 * in tiles of 64 or 128 hits; a frame with a larger layer runs tile by tile. */
#define MU3E_MAX_LAYER_HITS 1023

/* Hits of a batch of frames (device pointers).  layer and sensor may be NULL
 * for calls that do not need them. */
typedef struct {
  const float *x, *y, *z;            /* [n_hits] mm                              */
  const uint16_t *layer, *sensor;    /* [n_hits]                                 */
  const int32_t *layer_offsets;      /* [4*n_frames+1], non-decreasing, [0] = 0  */
  int32_t n_frames, n_hits;          /* both >= 0: every entry point refuses a
                                        negative count (MU3E_ERR_INVALID_ARG)    */
} mu3e_hits_t;

typedef struct { float lo, hi; } mu3e_window_t;   /* pass iff lo <= q <= hi */

/* Selection parameters (host struct, passed by pointer, copied at launch). */
typedef struct {
  float r_layer[4];          /* nominal layer radii (25, 31, 73, 85)              */
  float z_half[4];           /* layer half lengths                                */
  float b_tesla;             /* solenoid field                                    */
  float x_over_x0;           /* radiation length fraction per layer               */
  float sigma_pixel;         /* pixel resolution (pitch / sqrt 12)                */
  mu3e_window_t dlambda;     /* tan(lambda_12) - tan(lambda_01)                   */
  mu3e_window_t cosphi01;    /* cos of the azimuth between layer-0/1 hits         */
  mu3e_window_t cosphi12;    /* cos of the azimuth between layer-1/2 hits         */
  mu3e_window_t rtc_abs;     /* |signed transverse circumradius|                  */
  float chi2_track_max;      /* keep tracks with chi2_global < this (32)          */
  int32_t max_triplets;      /* cap of the selected-triplet list (768)            */
  int32_t max_tracks;        /* cap of the track list                             */
  int32_t max_combos;        /* cap of the energy-passing e+e+e- triple list      */
  int32_t max_layer_hits;    /* capacity, <= MU3E_MAX_LAYER_HITS                  */
  float de_max;              /* |sum E - m_mu| <= de_max                          */
  float r_target;            /* target radius (19)                                */
  float target_tol;          /* intersections within r_target + target_tol        */
  float chi2_vertex_max;     /* vertex chi2 <= this                               */
  float d_target_max;        /* distance of the vertex to the target surface      */
  float p_sum_max;           /* |vector sum of the three momenta|                 */
} mu3e_params_t;

/* Optional debug view, filled on return of mu3e_select_frames (host struct
 * holding device pointers into the caller's workspace).  The triplet list
 * is handed out to the waves of the cuts kernel in chunks (each wave starts
 * with one of its own, further ones cost one atomic each); a frame's
 * triplets may span chunks.  The track stage stores its
 * result for every triplet in place (no shared counter).  After the stream
 * is synchronised:
 *   counters[0]  triplets selected in total (true count)
 *   counters[2]  status bits: 1 the triplet list was full, 2 the float64
 *                re-evaluation list or the vertex-stage track table was
 *                full, 4 a frame's layer_offsets were malformed (decreasing,
 *                negative or beyond n_hits; that frame was skipped)
 *   counters[7]  triplet entries handed out in chunks of a fixed size
 *                (also past the capacity)
 *   chunks       [max_chunks][4]: start, count, fitted, 0 -- chunk c holds
 *                triplet entries [start, start + count); the rows in use are
 *                those with start + chunk size <= triplet_capacity, i.e. the
 *                first min(counters[7], triplet_capacity) / chunk size rows,
 *                and chunk c starts at c * chunk size
 *   triplets     [triplet_capacity][2]: frame, packed frame-local
 *                indices i0 | i1 << 10 | i2 << 20 (hit = layer_offsets[4f+l] + il)
 *   tracks       [triplet_capacity][4], parallel to triplets: code (1 the
 *                triplet starts an accepted track, 0 not, 2 undecided: only
 *                when the re-evaluation list was full), frame-local
 *                layer-3 index i3, float bits of kappa_bar, float bits of
 *                chi2_global
 * Triplets of frames flagged MU3E_TRIPLET_OVF may appear in the list; they
 * are never fitted (code 0).  Accepted tracks per frame are in
 * frame_counts[3f + 1]. */
typedef struct {
  const int32_t *counters;
  const int32_t *triplets;
  const int32_t *tracks;
  int32_t triplet_capacity, track_capacity;
  const int32_t *chunks;
  int32_t max_chunks, chunk_size;
} mu3e_debug_t;

/* Text of a status code; any int is accepted ("unknown status" outside the
 * enumeration). */
const char *mu3e_status_string(int status);

/* Workspace bytes for mu3e_select_frames over n_frames frames with room for
 * triplet_capacity (<= 2^30) selected triplets and track_capacity tracks of
 * vertex candidate frames in total.  The triplet list is shared by all waves
 * of the cuts in chunks of triplet_capacity / (2 * waves) entries (clamped to
 * [64, 4096]; waves = 20 per compute unit, or the plan's persistent waves),
 * so allow about twice the expected number of selected triplets.  Whatever
 * the capacities, no frame is passed on incomplete: a frame whose selected
 * triplets did not all fit, whose undecided track could not be queued for
 * the float64 re-evaluation, or whose tracks did not fit the vertex table is
 * flagged MU3E_LIST_FULL | MU3E_KEEP (kept for storage, as the paper keeps
 * an overflowing frame), and the run reports it in counters[2]
 * (mu3e_debug_t); larger capacities only lower the number of such frames.
 * Returns 0 for invalid sizes. */
size_t mu3e_select_workspace_size(int32_t n_frames, int32_t triplet_capacity,
                                  int32_t track_capacity);

/* The whole selection (Sections IV-A..IV-C, Alg. 1) for every frame:
 *   frame_flags  [n_frames]     MU3E_* bits
 *   frame_counts [3*n_frames]   triplets passing the cuts, tracks passing the
 *                               chi2 cut, e+e+e- triples passing the energy
 *                               test (exact counts; a stage skipped after an
 *                               overflow reports 0)
 *   frame_vertex [4*n_frames]   x, y, z, chi2 of the minimum-chi2 passing
 *                               vertex, NaN if none
 * dbg may be NULL.  Layer and sensor arrays are not read. */
mu3e_status mu3e_select_frames(const mu3e_hits_t *hits, const mu3e_params_t *params,
                               uint32_t *frame_flags, int32_t *frame_counts,
                               float *frame_vertex, void *workspace, size_t workspace_bytes,
                               int32_t triplet_capacity, int32_t track_capacity,
                               mu3e_debug_t *dbg, hipStream_t stream);

/* mu3e_select_frames that also records stage_events[0..4] on the stream:
 * before the first kernel, then after the cuts (Alg. 2), track (Alg. 3),
 * vertex-preparation and vertex (Alg. 4) kernels, for per-stage timing with
 * hipEventElapsedTime.  The events are created and owned by the caller;
 * stage_events may be NULL. */
mu3e_status mu3e_select_frames_timed(const mu3e_hits_t *hits, const mu3e_params_t *params,
                                     uint32_t *frame_flags, int32_t *frame_counts,
                                     float *frame_vertex, void *workspace, size_t workspace_bytes,
                                     int32_t triplet_capacity, int32_t track_capacity,
                                     mu3e_debug_t *dbg, hipStream_t stream,
                                     hipEvent_t *stage_events);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * mu3e_select_frames with its workspace taken from a library-owned static
 * device array of MU3E_STATIC_SCRATCH_BYTES (64 MiB; one copy per GPU the
 * library runs on, held until the process ends), so the call allocates
 * nothing.  The caller still owns the hits and the outputs.  A request whose
 * workspace (mu3e_select_workspace_size of n_frames, triplet_capacity,
 * track_capacity) exceeds the array returns MU3E_ERR_CAPACITY before
 * anything is launched; e.g. 100,000 nominal-rate frames fit with
 * triplet_capacity 2^21 and track_capacity 65536.  The first call on a device
 * resolves the array's address there (with that device current).  Every
 * call on a GPU uses that GPU's one array: calls that overlap in time on one
 * GPU (on different streams, or from different threads) race and give
 * undefined results, so serialise them (e.g. one stream).  The array keeps
 * the last call's contents; the counters that must start at zero are cleared
 * by the call's first kernel.  dbg (nullable) then points into the array and
 * stays valid until the next call on that GPU. */
#define MU3E_STATIC_SCRATCH_BYTES (64u << 20)
mu3e_status mu3e_select_frames_static(const mu3e_hits_t *hits, const mu3e_params_t *params,
                                      uint32_t *frame_flags, int32_t *frame_counts,
                                      float *frame_vertex, int32_t triplet_capacity,
                                      int32_t track_capacity, mu3e_debug_t *dbg,
                                      hipStream_t stream);

/* Single triplet fit (Section IV-B) of n explicit triplets of global hit
 * indices trip[n][3] (layer order 0,1,2 or 1,2,3).  out[n][8]: kappa,
 * sigma^2_kappa, chi2_min, R*, sigma^2_R, signed circumradius, theta_C1,
 * theta_C2.  A degenerate triplet (collinear in the transverse plane) or one
 * with a hit index outside [0, n_hits) gives NaN in all eight fields. */
mu3e_status mu3e_fit_triplets(const mu3e_hits_t *hits, const int32_t *trip, int32_t n,
                              const mu3e_params_t *params, float *out, hipStream_t stream);

/* Adjoint of the single triplet fit (Section IV-B: the chi2 of the
 * linearised multiple-scattering fit) with respect to the hit coordinates:
 * grad_xyz[n_hits][3] += sum_t grad_chi2[t] * d chi2_t / d(x, y, z) over the
 * three hits of each triplet trip[n][3].  grad_xyz is accumulated, not
 * overwritten (zero it first for a plain gradient); the additions are
 * float32 atomics, so their order, and the last bits, vary between calls.
 * The forward fit is recomputed (nothing is saved between the calls); its
 * discrete choices (minor arc, branches) stay fixed.  Degenerate triplets
 * and triplets with a hit index outside [0, n_hits) add nothing.  Caller
 * owns all buffers; n = 0 is a valid call that launches nothing. */
mu3e_status mu3e_fit_triplets_backward(const mu3e_hits_t *hits, const int32_t *trip, int32_t n,
                                       const mu3e_params_t *params, const float *grad_chi2,
                                       float *grad_xyz, hipStream_t stream);

/* Tracks grouped by frame: frame f owns tracks [frame_offsets[f],
 * frame_offsets[f+1]) of hit[n_tracks][4] (global hit indices, layers 0..3). */
typedef struct {
  const int32_t *hit;
  const int32_t *frame_offsets;      /* [n_frames+1] */
  int32_t n_frames, n_tracks;
} mu3e_tracks_t;

/* Workspace bytes of mu3e_vertex for n_tracks tracks (0 if n_tracks < 0). */
size_t mu3e_vertex_workspace_size(int32_t n_tracks);

/* Vertex stage (Section IV-C, Alg. 4) on given tracks: the track parameters
 * are recomputed from the hits in float64, e+e+e- triples pass the energy
 * test, the vertex estimate and the three signal tests decide MU3E_VERTEX.
 *   frame_flags  [n_frames]   MU3E_TRACK_OVF | MU3E_COMBO_OVF | MU3E_VERTEX |
 *                             MU3E_KEEP (overwritten)
 *   frame_combos [n_frames]   energy-passing triples
 *   frame_vertex [4*n_frames] as in mu3e_select_frames
 * Tracks with a hit index outside [0, n_hits) are ignored; a frame whose
 * range is malformed (decreasing or beyond n_tracks) forms no triple. */
mu3e_status mu3e_vertex(const mu3e_hits_t *hits, const mu3e_tracks_t *tracks,
                        const mu3e_params_t *params, uint32_t *frame_flags,
                        int32_t *frame_combos, float *frame_vertex, void *workspace,
                        size_t workspace_bytes, hipStream_t stream);

/* mu3e_vertex that also lists the e+e+e- triples passing the energy test
 * (the debug view of Alg. 4's preliminary check): rows triples[r][4] =
 * {frame, track a, track b, track c} (global track indices into
 * tracks->hit; a and b the positive tracks, c the negative one), in no
 * particular order.  *n_triples (a device int32 the caller zeroes before the
 * call) receives the number of passing triples; rows beyond
 * triple_capacity are not written.  triples may be NULL (then the call is
 * mu3e_vertex). */
mu3e_status mu3e_vertex_debug(const mu3e_hits_t *hits, const mu3e_tracks_t *tracks,
                              const mu3e_params_t *params, uint32_t *frame_flags,
                              int32_t *frame_combos, float *frame_vertex, void *workspace,
                              size_t workspace_bytes, int32_t *triples, int32_t triple_capacity,
                              int32_t *n_triples, hipStream_t stream);

/* Refined vertex of listed e+e+e- track triples: the more precise vertex
 * reconstruction that Section VII names as the next step after the rough
 * estimate of Section IV-C.  The refined vertex v minimises
 *   J(v, phi) = sum_k |H_k(phi_k) - v|^2 / sigma_k^2
 * jointly over v and one turning angle phi_k per track, H_k being track k's
 * helix (the transverse circle of the vertex stage with the track's dip) and
 * sigma_k^2 eq. track-error's variance at the track's closest approach to
 * the rough estimate, held fixed; J has 3 degrees of freedom.  Only triples
 * whose rough estimate passes the three signal tests are refined; the rough
 * estimate is the start.  Track parameters are recomputed from the hits
 * once per track (into the workspace, at least
 * mu3e_vertex_workspace_size(tracks->n_tracks) bytes) and the fit runs in
 * float64 (Gauss-Newton, at most 16 steps).
 *   triples  [n][4]   rows {frame, a, b, c} of global track indices into
 *                     tracks->hit (the rows mu3e_vertex_debug writes; the
 *                     frame column is not read; tracks->frame_offsets is
 *                     not read either)
 *   n_valid           optional device int32: only rows [0, min(n, *n_valid))
 *                     are processed (the count mu3e_vertex_debug writes), so
 *                     the two calls chain without a host synchronisation;
 *                     NULL processes all n rows.  Rows beyond are untouched.
 *   out      [n][8]   float64: refined x, y, z (mm), J; rough x, y, z, chi2
 *   status   [n]      the Gauss-Newton steps used (>= 1, converged); 0 the
 *                     rough estimate does not pass (out all NaN); -1 no
 *                     convergence (out[0..3] hold the last iterate); -2 a
 *                     track index outside [0, n_tracks), a hit index outside
 *                     [0, n_hits) or a failed track fit (out all NaN).
 * Caller owns all buffers; n = 0 launches nothing.  A workspace below the
 * size gives MU3E_ERR_CAPACITY. */
mu3e_status mu3e_vertex_refine(const mu3e_hits_t *hits, const mu3e_tracks_t *tracks, const int32_t *triples,
                               int32_t n, const int32_t *n_valid, const mu3e_params_t *params, double *out,
                               int32_t *status, void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ---- Chunk ingest (Section V-A) ------------------------------------------
 * A chunk is a fixed-size buffer written by the readout and copied to the
 * GPU as is (from pinned host memory, one stream per chunk in flight):
 *   bytes [0, 12 n)                 n hit records {float x, y, z} (mm), sorted
 *                                   by frame and then layer
 *   int32 [4F+1] just before the    layer offsets: frame f, layer l owns
 *   last four bytes                 records [off[4f+l], off[4f+l+1]); off[0] = 0,
 *                                   off[4F] = n
 *   int32, the last four bytes      F, the number of frames in the chunk
 * The space between the records and the offsets is unused.  The tail is
 * read from byte (chunk_bytes & ~3) - 4 backwards. */

/* Unpacks a chunk (device pointer, 4-byte aligned, chunk_bytes long) into SoA
 * hits x, y, z [max_hits] and layer_offsets [4*max_frames+1] (device
 * buffers owned by the caller), padding frames F .. max_frames-1 as empty so
 * that a selection or a plan bound to max_frames frames and max_hits hits
 * runs any chunk.  info [2] (device) receives {F, n}; a chunk whose tail is
 * inconsistent (F < 0 or > max_frames, offsets overlapping the records,
 * off[0] != 0, n > max_hits) yields {-1, -1} and no frames (all offsets 0).
 * Offsets that decrease inside a consistent tail are passed on: the
 * selection skips such frames and reports them (status bit 4). */
mu3e_status mu3e_chunk_unpack(const void *chunk, int64_t chunk_bytes, int32_t max_frames,
                              int32_t max_hits, float *x, float *y, float *z,
                              int32_t *layer_offsets, int32_t *info, hipStream_t stream);

/* ---- Frame pairs (tracks across a frame boundary, Section VII) -----------
 * Builds the overlapping frame pairs of a batch: merged frame g (0 <= g <
 * n_frames - 1) holds, per layer, the hits of frame g followed by those of
 * frame g + 1.  Outputs (device, caller-owned): x, y, z [capacity] with
 * capacity >= 2 * n_hits (else MU3E_ERR_CAPACITY), layer_offsets
 * [4 * (n_frames - 1) + 1] with layer_offsets[4g + l] = lo[4g + l] +
 * lo[4g + 4 + l] - lo[4].  Running the selection on the merged frames
 * (n_frames - 1 frames, layer_offsets[4 (n_frames - 1)] hits) finds the
 * tracks whose hits fall into two consecutive frames: a hit with local
 * index k on layer l of merged frame g comes from frame g when k is below
 * frame g's count on that layer, else from frame g + 1.  Needs n_frames >= 2. */
mu3e_status mu3e_pair_frames(const mu3e_hits_t *hits, float *x, float *y, float *z,
                             int32_t *layer_offsets, int64_t capacity, hipStream_t stream);

/* ---- Batched form ------------------------------------------------------
 * A plan captures the whole selection of one batch of frames into a HIP
 * graph around one persistent kernel: waves take the frames of the batch
 * cyclically, except a tail of steal_percent % of them which they claim
 * frames_per_claim frames at a time from shared counters (work stealing over
 * uneven frames), and run the Selection Cuts of each frame; with fuse_fits the same waves also fit
 * the pending survivors of their frames 64 at a time, otherwise a fit kernel
 * follows in the graph.  The float64 re-evaluation and the vertex stage
 * follow in the same graph.  Outputs are identical to mu3e_select_frames.
 * The plan binds the hit, output and workspace buffers given here: refill
 * them and call mu3e_plan_run again.  Runs of one plan (or of plans sharing
 * a workspace) must not overlap; plans with their own buffers may run at the
 * same time on different streams (several batches in flight, each batch's
 * latency-bound stages overlapping another's cuts). */
typedef struct mu3e_plan mu3e_plan_t;

typedef struct {
  int32_t waves_per_cu;       /* persistent waves per compute unit (0: default 16;
                                 capped by occupancy)                           */
  int32_t frames_per_claim;   /* frames taken per work-stealing claim (0: 4)   */
  int32_t fuse_fits;          /* 1: the persistent waves also fit (see above)  */
  int32_t steal_percent;      /* 0..100: share of the frames (the tail of the
                                 batch) taken by work stealing; the rest is
                                 dealt cyclically                              */
  int32_t tile_hits;          /* LDS tile of the cuts: hits per layer staged at
                                 once, 64 or 128 (0: 128); a frame with a
                                 layer above it runs tile by tile.  Smaller
                                 tiles take half the LDS, so more waves fit
                                 on a compute unit                             */
  int32_t sub_batches;        /* 1..4 (0: 1): the batch is split into this many
                                 contiguous ranges of frames, each with its own
                                 part of the workspace; the cuts of one run
                                 while the fits and vertex stage of the one
                                 before run on another stream                  */
} mu3e_tuning_t;

/* Workspace bytes of a plan over n_frames frames with the given capacities
 * split over sub_batches (0 or 1: the same as mu3e_select_workspace_size).
 * Returns 0 for invalid sizes. */
size_t mu3e_plan_workspace_size(int32_t n_frames, int32_t triplet_capacity,
                                int32_t track_capacity, int32_t sub_batches);

/* Workspace as mu3e_plan_workspace_size (the capacities are split evenly
 * over the sub-batches).  tuning may be NULL.  Allocates the plan object,
 * two graphs per sub-batch, and a stream and two events per sub-batch after
 * the first (host and driver memory; the streams have the default
 * priority). */
mu3e_status mu3e_plan_create(mu3e_plan_t **plan, const mu3e_hits_t *hits,
                             const mu3e_params_t *params, uint32_t *frame_flags,
                             int32_t *frame_counts, float *frame_vertex, void *workspace,
                             size_t workspace_bytes, int32_t triplet_capacity,
                             int32_t track_capacity, const mu3e_tuning_t *tuning);

/* One run of the batch (asynchronous; no allocation): sub-batch 0 on the
 * given stream, sub-batch j > 0 on the plan's stream j, each as two graph
 * launches (cuts; fits and vertex stage); the cuts of sub-batch j wait for
 * those of sub-batch j - 1, and the given stream waits for every
 * sub-batch, so work queued on it afterwards sees the whole batch done. */
mu3e_status mu3e_plan_run(mu3e_plan_t *plan, hipStream_t stream);

/* The same kernel sequence as mu3e_plan_run, launched directly on the given
 * stream (no graph; the sub-batches one after another) with four events per
 * sub-batch, events[4j .. 4j+3] (caller-created, timing enabled, 4 *
 * sub_batches in all), recorded before and after its persistent kernel,
 * after its fit kernel and after its last kernel, so that kernel durations
 * can be measured on the stream they run on.  Identical outputs. */
mu3e_status mu3e_plan_run_timed(mu3e_plan_t *plan, hipStream_t stream, hipEvent_t *events);

/* The debug view of sub-batch 0 (as mu3e_select_frames fills it) and the
 * tuning in effect; either pointer may be NULL. */
mu3e_status mu3e_plan_info(const mu3e_plan_t *plan, mu3e_debug_t *dbg, mu3e_tuning_t *tuning);

/* The debug view of sub-batch `part` (0 <= part < sub_batches in effect) and
 * its frames [first_frame, first_frame + n_frames) of the batch; the frame
 * numbers in its triplet list are relative to first_frame.  Any output
 * pointer may be NULL. */
mu3e_status mu3e_plan_part_info(const mu3e_plan_t *plan, int32_t part, mu3e_debug_t *dbg,
                                int32_t *first_frame, int32_t *n_frames);

void mu3e_plan_destroy(mu3e_plan_t *plan);

/* ---- Alignment (differentiable form) ---------------------------------
 * theta[n_sensors][4] = (tx, ty, tz, alpha) per sensor: a hit h on sensor s
 * (hits->sensor, required here) is moved to R_z(alpha_s) h + (tx, ty, tz)_s
 * before the triplet fit of Section IV-B.  trip[n][3] are global hit indices
 * of triplets on consecutive layers (a frozen set, e.g. both triplets of
 * every accepted track); n_sensors <= 2048. */

/* chi2[n]: the triplet-fit chi2 of each triplet after alignment (float32
 * fit); NaN for a degenerate triplet or an index out of range. */
mu3e_status mu3e_align_chi2(const mu3e_hits_t *hits, const int32_t *trip, int32_t n,
                            const float *theta, int32_t n_sensors, const mu3e_params_t *params,
                            float *chi2, hipStream_t stream);

/* Workspace bytes of mu3e_align_backward (0 if n_sensors is out of range). */
size_t mu3e_align_workspace_size(int32_t n_sensors);

/* Hand-written adjoint: grad_theta[n_sensors][4] (overwritten) =
 * sum_t grad_chi2[t] * d chi2_t / d theta, through the circumcircle, the
 * linearised fit and the Highland width; the discrete choices of the fit
 * stay fixed.  Accumulation in float64. */
mu3e_status mu3e_align_backward(const mu3e_hits_t *hits, const int32_t *trip, int32_t n,
                                const float *theta, int32_t n_sensors,
                                const mu3e_params_t *params, const float *grad_chi2,
                                float *grad_theta, void *workspace, size_t workspace_bytes,
                                hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* MU3E_H */
