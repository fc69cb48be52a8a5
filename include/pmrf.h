/*
 * pmrf.h -- C ABI of the MI355X (gfx950) EM optimisation path of DPP-PMRF
 * (Lessley, Perciano, Heinemann, Camp, Childs, Bethel: "DPP-PMRF: Rethinking
 * Optimization for a Probabilistic Graphical Model Using Data-Parallel
 * Primitives", LDAV 2018, arXiv:1809.05018).
 *
 * The problem statement of Alg. 1 / Alg. 2 (inputs: image, oversegmentation,
 * number of labels; outputs: segmentation and estimated parameters) is taken
 * at the point where the paper says the optimisation consumes a graph
 * (Sec. 5): the caller hands over the region-adjacency graph of the
 * oversegmentation as CSR plus one intensity per region, and receives one
 * label per region plus the per-label mean and standard deviation.
 *
 * Conventions for every call:
 *  - Return value: PMRF_OK (0) or a negative pmrf_status.  On an error found
 *    on the host, no caller-visible output has been written.  The message of
 *    the last error on the calling thread is pmrf_last_error().
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *    memory (for example torch tensors' data_ptr() on a ROCm device).
 *  - The caller owns every buffer it passes.  The library owns only the opaque
 *    host object pmrf_hoods (freed with pmrf_hoods_free).  The library never
 *    allocates device memory at run time: buffers it needs come in as a caller
 *    workspace (pmrf_em_run_noalloc uses a static device array instead).
 *  - Device work is enqueued on the given HIP stream (hipStream_t passed as
 *    void*, NULL = the null stream) and is asynchronous; results are valid
 *    after the stream is synchronised.  Errors that only the device can see
 *    (a starting label outside [0, L), a non-positive starting sigma, a
 *    non-finite intensity) are reported in counters[PMRF_CTR_STATUS].
 *  - Labels are int32; intensities, parameters and energies are IEEE double.
 */
#ifndef PMRF_H
#define PMRF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pmrf_status;
#define PMRF_OK 0
#define PMRF_EINVAL (-1)       /* bad argument or malformed graph */
#define PMRF_ENOMEM (-2)       /* a caller buffer is too small, or host allocation failed */
#define PMRF_EDEVICE (-3)      /* a HIP runtime call failed */
#define PMRF_EUNSUPPORTED (-4) /* valid request outside what this version supports (k != 1, L > 16, neighbourhood > 1024, n > 2^26 - 1) */
/* device-reported codes, in counters[PMRF_CTR_STATUS] */
#define PMRF_EBADLABEL (-10)   /* a starting label outside [0, L) */
#define PMRF_EBADPARAM (-11)   /* a starting sigma <= 0 or a non-finite mu / sigma */
#define PMRF_ERANGE (-12)      /* reserved: not returned by this version */
#define PMRF_ETIMEOUT (-13)    /* reserved: not returned by this version (no kernel waits on another block) */

/* Thread-local text of the last error (never NULL; "" if none). */
const char *pmrf_last_error(void);

/* Version of this ABI (incremented on any incompatible change). */
int32_t pmrf_abi_version(void);

/* ------------------------------------------------------------------------
 * Neighbourhoods (Sec. 3.1: a k-neighbourhood is a maximal clique together
 * with every vertex within k edges of it, here k = 1; Sec. 3.2.1 and the
 * construction steps of Sec. 3.2.2, "Construction of Neighborhoods").
 *
 * Maximal cliques are listed in canonical order (each clique ascending, the
 * list in lexicographic order), neighbourhood h belongs to clique h, and the
 * members of a neighbourhood are in ascending vertex order.  An isolated
 * vertex is a clique (and a neighbourhood) of its own.  Every vertex is
 * "owned" by its position in the first clique that contains it; that element
 * sees all of the vertex's neighbours and decides its label.
 * ------------------------------------------------------------------------ */
typedef struct pmrf_hoods pmrf_hoods;

typedef struct {
  int64_t n;            /* vertices */
  int64_t H;            /* maximal cliques = neighbourhoods */
  int64_t M;            /* neighbourhood elements, sum of sizes */
  int64_t A;            /* in-neighbourhood adjacency entries */
  int64_t max_hood;     /* largest neighbourhood */
  int64_t tiles;        /* wave-sized work packets of the device layout */
  int64_t device_bytes; /* exact size of the device copy written by pmrf_hoods_upload */
} pmrf_hoods_info;

/* Build the neighbourhoods of an undirected graph given as CSR (host).
 * row_ptr[n+1] (row_ptr[0] = 0, non-decreasing) and col_idx[row_ptr[n]]
 * with each row strictly ascending, no self loops, every edge present in both
 * directions.  k is the neighbourhood radius, 1..8 (the paper uses k = 1):
 * a neighbourhood holds its clique and every vertex within k edges of it.
 * n = 0 is allowed (empty problem).  *out receives a new host object.
 * Errors: PMRF_EINVAL (malformed CSR, NULL pointers, k < 1), PMRF_EUNSUPPORTED
 * (k > 8, a neighbourhood above 1024 members, n above 2^26 - 1 = 67108863
 * vertices, 2^30 or more neighbourhood elements), PMRF_ENOMEM. */
pmrf_status pmrf_build_neighborhoods(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t k,
                                     pmrf_hoods **out);

/* The same construction on the device (Alg. 2, "enumerate maximal cliques"
 * and "construct k-neighborhoods", as data-parallel passes: Sec. 3.2.2 Find /
 * Count / Get Neighbors and Remove Duplicate Neighbors).  d_row_ptr[n+1] and
 * d_col_idx[d_row_ptr[n]] are device arrays on the current device with the
 * CSR rules above (checked on the device).  Work is enqueued on hip_stream
 * (NULL: the null stream); the call synchronises that stream several times
 * to size its arrays and returns when the structure is complete.  The result
 * equals pmrf_build_neighborhoods' in every exported array and in the layout
 * pmrf_hoods_upload writes, byte for byte; its layout and canonical arrays
 * stay in device memory owned by the object (hipMalloc; released by
 * pmrf_hoods_free), and pmrf_hoods_upload copies device to device.  Its
 * temporaries come stream-ordered from a memory pool the library creates
 * per device (freeing them synchronises nothing else), which keeps up to
 * 1 GiB of freed blocks for the next build until the process ends.  The
 * caller keeps ownership of the CSR, which is not needed afterwards.
 * Errors: as pmrf_build_neighborhoods, plus PMRF_EUNSUPPORTED when one
 * neighbourhood gathers more than 8192 candidate entries (its members'
 * rows, duplicates included) or a clique level would exceed 2^30 member
 * entries, and PMRF_EDEVICE / PMRF_ENOMEM for HIP failures. */
pmrf_status pmrf_build_neighborhoods_device(int32_t n, const int32_t *d_row_ptr, const int32_t *d_col_idx, int32_t k,
                                            void *hip_stream, pmrf_hoods **out);

/* Device memory held by a structure from pmrf_build_neighborhoods_device:
 * *d_layout = its own copy of the layout (info.device_bytes bytes, on the
 * device it was built on, 256-byte aligned), which may be passed wherever an
 * uploaded buffer is expected (d_hoodbuf) while the object lives;
 * *held_bytes = all device memory the object holds (layout and canonical
 * arrays).  A host-built structure gives NULL and 0.  Either output may be
 * NULL.  Errors: PMRF_EINVAL (hoods NULL). */
pmrf_status pmrf_hoods_device_buffer(const pmrf_hoods *hoods, void **d_layout, int64_t *held_bytes);

pmrf_status pmrf_hoods_get_info(const pmrf_hoods *hoods, pmrf_hoods_info *info);

/* Host copies of the canonical structure (for inspection and tests):
 * hood_ptr[H+1], hood_vid[M], clique_ptr[H+1], clique_vid[clique members],
 * owner[n] = element index (into hood_vid) owning each vertex.  Any output
 * may be NULL.  clique sizes total = clique_ptr[H]. */
pmrf_status pmrf_hoods_export(const pmrf_hoods *hoods, int64_t *hood_ptr, int32_t *hood_vid, int64_t *clique_ptr,
                              int32_t *clique_vid, int64_t *owner);

/* Copy the device layout of the neighbourhoods into a caller device buffer of
 * at least info.device_bytes bytes (256-byte aligned), enqueued on stream.
 * The host object must outlive every run that uses this buffer. */
pmrf_status pmrf_hoods_upload(const pmrf_hoods *hoods, void *d_buf, int64_t bytes, void *hip_stream);

/* Replication by label (Sec. 3.2.2, "Replicate Neighborhoods By Label"), in the
 * paper's layout: for each neighbourhood h, for each label l, its members in
 * order; test_label = l, old_index = position in the flat neighbourhood array,
 * hood_id = h.  Each output has L*M entries (host).  The HIP path never
 * materialises these arrays; this call exports them for inspection. */
pmrf_status pmrf_replicate_indices(const pmrf_hoods *hoods, int32_t L, int32_t *test_label, int64_t *old_index,
                                   int32_t *hood_id);

/* Same replication for an arbitrary flat neighbourhood array given by its
 * offsets hood_ptr[H+1] (host). */
pmrf_status pmrf_replicate_hood_array(int64_t H, const int64_t *hood_ptr, int32_t L, int32_t *test_label,
                                      int64_t *old_index, int32_t *hood_id);

void pmrf_hoods_free(pmrf_hoods *hoods);

/* ------------------------------------------------------------------------
 * EM optimisation (Alg. 2, EM loop; Sec. 3.2.2 "EM Parameter Estimation").
 *
 * Iteration t, from labels x_t and parameters theta_t = (mu_l, sigma_l):
 *   E(h,j,l) = (y_v - mu_l)^2 / (2 sigma_l^2) + ln sigma_l
 *              + beta * #{u in N(v), u in hood h : x_t(u) != l}
 *     for every neighbourhood h, member v = hood_h[j], label l
 *     (Gaussian likelihood energy plus Potts prior energy, Sec. 2.1)
 *   m(h,j) = min_l E(h,j,l), lowest label on ties; S_h = sum_j m(h,j);
 *   T_t = sum_h S_h                                  ("Neighborhood Energy Sums")
 *   x_{t+1}(v) = argmin at the owner element of v    ("Update Output Labels")
 *   theta_{t+1}: per label, mean and population standard deviation of y over
 *   the vertices labelled l in x_{t+1} (floored at sigma_min; a label with no
 *   vertex keeps its parameters)                     ("Update Parameters")
 *   a neighbourhood has converged at t when |S_h^t - S_h^{t-w}| < conv_tol for
 *   w = 1..conv_window; the total T likewise        ("MAP / EM Convergence Check")
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t L;                /* number of labels, 2..16 */
  double beta;              /* Potts weight, finite, >= 0 */
  int32_t max_iters;        /* EM iterations, >= 0 (the paper uses a fixed 20) */
  int32_t conv_window;      /* convergence window, 1..8 (paper: 3) */
  double conv_tol;          /* absolute convergence threshold, >= 0 (paper: 1e-4) */
  int32_t early_exit;       /* 1: stop after the iteration at which every neighbourhood converged */
  int32_t init_from_labels; /* 1: first replace (mu, sigma) by the parameter update of the starting labels */
  double sigma_min;         /* floor of sigma, > 0 (default 1e-3) */
  double tie_eps;           /* a label decision with energy gap below this is counted as a near tie (1e-9) */
  int32_t scatter_rule;     /* PMRF_SCATTER_*: which neighbourhood's label decision stands for a vertex */
} pmrf_em_params;

/* Scatter rules of the label update ("Update Output Labels": every element
 * (h, v) scatters its arg-minimum to vertex v; the paper leaves the write
 * conflicts between the ~20 neighbourhoods holding a vertex open).
 *  OWNER: the element in the first clique (canonical order) holding v; it sees
 *         every graph neighbour of v, so the update is synchronous ICM on the
 *         graph (default).
 *  LAST:  the element in the last neighbourhood (canonical order) holding v,
 *         the outcome of a serial Scatter over the neighbourhood-major array.
 *  MIN:   the element of v with the smallest minimum energy, the first in
 *         canonical order on ties; a near tie also counts another element of
 *         v within tie_eps of that minimum at a different label.  Runs a
 *         per-vertex pass after each iteration's energies. */
#define PMRF_SCATTER_OWNER 0
#define PMRF_SCATTER_LAST 1
#define PMRF_SCATTER_MIN 2

/* Fill p with the defaults: L = 2, beta = 0.5, max_iters = 20, conv_window = 3,
 * conv_tol = 1e-4, early_exit = 0, init_from_labels = 0, sigma_min = 1e-3,
 * tie_eps = 1e-9, scatter_rule = PMRF_SCATTER_OWNER. */
void pmrf_em_params_default(pmrf_em_params *p);

/* counters[] layout (int64, device) */
#define PMRF_CTR_STATUS 0      /* 0 or a device-reported PMRF_E* code */
#define PMRF_CTR_ITERS 1       /* iterations executed */
#define PMRF_CTR_MAP_CONV 2    /* first iteration at which every neighbourhood had converged, or -1 */
#define PMRF_CTR_EM_CONV 3     /* first iteration at which the total T had converged, or -1 */
#define PMRF_CTR_NEAR_TIES 4   /* near ties summed over iterations */
#define PMRF_CTR_EVALS 5       /* energy evaluations = M * L * iterations */
#define PMRF_NCOUNTERS 8

/* Exact device workspace size for pmrf_em_run with these hoods and params. */
pmrf_status pmrf_em_workspace_bytes(const pmrf_hoods *hoods, const pmrf_em_params *params, int64_t *bytes);

/* Run params->max_iters EM iterations on one graph (device buffers, stream-ordered).
 *  d_hoodbuf      the buffer filled by pmrf_hoods_upload for these hoods
 *  d_y[n]         region intensities (read only)
 *  d_labels[n]    in: starting labels x_0 in [0, L); out: labels after the last iteration
 *  d_mu[L], d_sigma[L]  in: starting parameters; out: parameters after the last iteration
 *  d_hood_energy[H]     out: S_h of the last iteration (NULL: not written)
 *  d_trace[max_iters]   out: T_t per iteration (NULL: not written)
 *  d_iter_stats[2*max_iters]  out: per iteration {near ties, neighbourhoods not converged} (NULL: not written)
 *  d_counters[PMRF_NCOUNTERS] out: PMRF_CTR_* (required)
 *  d_ws, ws_bytes       workspace of at least pmrf_em_workspace_bytes bytes, 256-byte aligned;
 *                       its contents on entry do not matter
 * Results do not depend on the launch configuration: counts are exact
 * integers and every FP64 sum (neighbourhood sums, energy totals, the
 * per-label sums of the parameter update) is taken in a fixed order set by the
 * graph alone.  Runs that share a workspace or outputs must not overlap in
 * time. */
pmrf_status pmrf_em_run(const pmrf_hoods *hoods, const void *d_hoodbuf, const double *d_y, int32_t *d_labels,
                        double *d_mu, double *d_sigma, double *d_hood_energy, double *d_trace, int64_t *d_iter_stats,
                        int64_t *d_counters, void *d_ws, int64_t ws_bytes, const pmrf_em_params *params,
                        void *hip_stream);

/* Allocation-free variant of pmrf_em_run, for callers that cannot allocate
 * device memory: work recorded under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Arguments and results are those of
 * pmrf_em_run without d_ws / ws_bytes: the workspace is a static device array
 * of PMRF_NOALLOC_WS_BYTES bytes that the library holds on every GPU it runs
 * on, until the process ends.  The call allocates nothing (no hipMalloc, no
 * graph capture, no timing events): its kernels are launched directly on the
 * stream, and its results are bitwise those of pmrf_em_run.
 * Errors: as pmrf_em_run, plus PMRF_ENOMEM, returned before any device call,
 * when the run needs more workspace than PMRF_NOALLOC_WS_BYTES
 * (pmrf_em_workspace_bytes gives the need; the 100k-region slice at L = 2
 * needs about 6.5 MB).
 * Every call on one GPU uses that GPU's one array, which keeps the last call's
 * contents (a run initialises whatever part of it it reads): calls that
 * overlap in time on one GPU (other streams or threads) race and must be
 * serialised by the caller. */
#define PMRF_NOALLOC_WS_BYTES (64LL << 20)
pmrf_status pmrf_em_run_noalloc(const pmrf_hoods *hoods, const void *d_hoodbuf, const double *d_y, int32_t *d_labels,
                                double *d_mu, double *d_sigma, double *d_hood_energy, double *d_trace,
                                int64_t *d_iter_stats, int64_t *d_counters, const pmrf_em_params *params,
                                void *hip_stream);

/* ------------------------------------------------------------------------
 * Batched optimisation: many graphs (for example the slices of a volume, which
 * the paper processes one by one, Sec. 4.3.1) advanced together, one launch
 * per EM iteration covering every graph.  Each item is exactly the argument
 * set of pmrf_em_run; each graph's results are bitwise identical to running it
 * alone.  Items may have different L, beta and iteration counts.
 * ------------------------------------------------------------------------ */
typedef struct {
  const pmrf_hoods *hoods;
  const void *d_hoodbuf;
  const double *d_y;
  int32_t *d_labels;
  double *d_mu;
  double *d_sigma;
  double *d_hood_energy;
  double *d_trace;
  int64_t *d_iter_stats;
  int64_t *d_counters;
  pmrf_em_params params;
} pmrf_em_item;

pmrf_status pmrf_em_batch_workspace_bytes(int32_t B, const pmrf_em_item *items, int64_t *bytes);

pmrf_status pmrf_em_batch(int32_t B, const pmrf_em_item *items, void *d_ws, int64_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * Launch configuration (does not change any result, only speed: every
 * reduction order is fixed by the graph, not by the launch shape).
 *  mode: 0 = automatic: an argument set runs as direct launches (as mode 3)
 *        the first time it is seen and as in mode 1 from its second run on, so
 *        one-off argument sets never pay a graph capture;
 *        1 = the run's kernels are captured once per distinct argument set
 *        into a HIP graph (a cache of the 128 most recent sets) and the graph
 *        is replayed on the caller's stream; the iteration kernel has one block
 *        per superchunk of every graph (4, 8 or 16 chunks of 10 work packets,
 *        set by the graph's size; a single graph of at most 256 superchunks
 *        whose blocks have at least 4 waves runs one launch per EM iteration,
 *        the parameter update of the previous iteration included, otherwise a
 *        one-block parameter-update launch follows each iteration launch);
 *        2 = as 1, but the iteration kernel is a persistent grid of
 *        blocks_per_cu blocks per compute unit that walk all superchunks;
 *        3 = direct launches on the caller's stream (one block per superchunk).
 *        While kernel timing is on (pmrf_profile_begin), runs use direct
 *        launches with the grid of the selected mode.
 *  waves_per_block: 1..16 (0 = automatic: a single graph one wave per chunk
 *        of its superchunks, a batch 4)
 *  tiles_per_wave: reserved (0)
 *  blocks_per_cu: blocks per compute unit in mode 2 (0 = automatic: 5)
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t mode;
  int32_t waves_per_block;
  int32_t tiles_per_wave;
  int32_t blocks_per_cu;
} pmrf_launch;

pmrf_status pmrf_set_launch(const pmrf_launch *launch);
pmrf_status pmrf_get_launch(pmrf_launch *launch);

/* Counts since the library was loaded (host ints): runs that captured a new
 * HIP graph, runs replayed from the graph cache, runs launched directly. */
pmrf_status pmrf_launch_stats(int64_t *captures, int64_t *replays, int64_t *direct);

/* ------------------------------------------------------------------------
 * Kernel timing for measurement.  Between pmrf_profile_begin and
 * pmrf_profile_end the work kernels of every EM iteration made by this
 * process (the energy / argmin / sum / label / statistics kernels: the
 * iteration kernel, and a separate packet kernel where one runs) carry a pair of HIP
 * events on their stream, which the runtime stamps with the first kernel's
 * dispatch begin and the last one's end (hipExtLaunchKernel).
 * pmrf_profile_end waits for the last event and returns the summed
 * begin-to-end time in milliseconds and the number of timed iterations
 * (every iteration launches at least one block, also for an empty graph).
 * Timing does not change any result.  Not thread safe: one measuring thread
 * at a time.
 * ------------------------------------------------------------------------ */
pmrf_status pmrf_profile_begin(void);
pmrf_status pmrf_profile_end(double *total_ms, int64_t *launches);

/* ------------------------------------------------------------------------
 * Image in, segmentation out (the input and output of the paper's Alg. 2:
 * an image with its oversegmentation in, a labelling of the pixels out; the
 * optimisation in between takes the regions' graph, Sec. 5).
 *
 * pmrf_image_graph: the region adjacency graph and the region means of an
 * oversegmented 8-bit image, on the device.  d_regions (int32, height x width,
 * row-major) holds each pixel's region id in [0, n); d_pixels (uint8, same
 * layout) the intensities.  Regions u != v are adjacent when a pixel of u and
 * a pixel of v are horizontal or vertical neighbours (4-connectivity).
 * Outputs: d_row_ptr (int32[n + 1]) and d_col_idx (int32[col_capacity]) the
 * symmetric CSR with every row ascending (the form pmrf_build_neighborhoods
 * takes, after a copy to the host), d_means (double[n]) the sum of a region's
 * pixel values over its pixel count (0 for a region without pixels), *nnz
 * (host) the number of adjacency entries.  d_ws: a device workspace of at
 * least pmrf_image_graph_workspace_bytes(width, height, n) bytes.  The call
 * waits for the stream once (the entry count and the id check come back to the
 * host; every intermediate size stays on the device) and returns with the
 * outputs enqueued.  Errors: PMRF_EINVAL (NULL or negative
 * argument, a region id outside [0, n): nothing written), PMRF_ENOMEM
 * (workspace too small; col_capacity below the entry count, which is then in
 * *nnz: nothing else written), PMRF_EUNSUPPORTED (more than 2^28 pixels),
 * PMRF_EDEVICE.  Results are deterministic (integer sums, sorted edges).
 *
 * pmrf_labels_to_pixels: d_out[p] = d_labels[d_regions[p]] as uint8 for
 * npixels pixels (255 where the id is outside [0, n) or the label outside
 * [0, 255)); stream-ordered, nothing waited for.
 *
 * pmrf_confusion: d_counts[a * k + b] (int64[k * k], device) = number of
 * pixels p with d_a[p] = a and d_b[p] = b, for a, b < k (pixels with a value
 * >= k in either image are not counted); 1 <= k <= 16.  With a = the
 * segmentation and b = the ground truth these are the TP, TN, FP and FN counts
 * of the verification metrics (precision, recall, accuracy) and the void
 * fraction of the porosity (Sec. 4.2.1).  Stream-ordered.
 * ------------------------------------------------------------------------ */
pmrf_status pmrf_image_graph_workspace_bytes(int32_t width, int32_t height, int32_t n, int64_t *bytes);
pmrf_status pmrf_image_graph(const int32_t *d_regions, const uint8_t *d_pixels, int32_t width, int32_t height,
                             int32_t n, int32_t *d_row_ptr, int32_t *d_col_idx, int64_t col_capacity,
                             double *d_means, int64_t *nnz, void *d_ws, int64_t ws_bytes, void *hip_stream);
/* pmrf_volume_graph: the same for a volume (depth slices of height x width,
 * slice-major): regions are also adjacent across consecutive slices
 * (6-connectivity), the 3-D graphs the paper names as the next step
 * (Sec. 5).  pmrf_image_graph is this call with depth 1; arguments, limits
 * (at most 2^28 voxels) and errors as there. */
pmrf_status pmrf_volume_graph_workspace_bytes(int32_t width, int32_t height, int32_t depth, int32_t n,
                                              int64_t *bytes);
pmrf_status pmrf_volume_graph(const int32_t *d_regions, const uint8_t *d_voxels, int32_t width, int32_t height,
                              int32_t depth, int32_t n, int32_t *d_row_ptr, int32_t *d_col_idx, int64_t col_capacity,
                              double *d_means, int64_t *nnz, void *d_ws, int64_t ws_bytes, void *hip_stream);
pmrf_status pmrf_labels_to_pixels(const int32_t *d_regions, const int32_t *d_labels, int64_t npixels, int32_t n,
                                  uint8_t *d_out, void *hip_stream);
pmrf_status pmrf_confusion(const uint8_t *d_a, const uint8_t *d_b, int64_t npixels, int32_t k, int64_t *d_counts,
                           void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PMRF_H */
