/*
 * prism.h -- C ABI of the MI355X PRISM / multislice STEM simulation library.
 *
 * The operations follow the statement of the method in Pryor, Ophus and Miao,
 * "A Streaming Multi-GPU Implementation of Image Simulation Algorithms for
 * Scanning Transmission Electron Microscopy" (2017):
 *   - projected potential slices   ("Calculation of the Projected Potentials", Fig. 1a-b)
 *   - compact S-matrix build       (Fig. 1f-h, Eqs. 1-2, "PRISM Probe Simulations")
 *   - PRISM probe outputs          (Fig. 1i-k, "PRISM Probe Simulations")
 *   - multislice probe outputs     (Fig. 1c-e, Eqs. 1-2, "Multislice Probe Simulations")
 *
 * Conventions common to every entry point
 *   - Units: lengths in Angstrom, energies in eV, angles in rad, potentials
 *     projected over a slice in V*A.
 *   - Grids are square: n x n pixels over an Lx = Ly = L cell, pixel pitch
 *     L/n, n a power of two in [64, 2048].  Arrays are row-major [y][x].
 *   - Complex values are interleaved float pairs (re, im) ("complex64").
 *   - Every function returns PRISM_OK (0) or a negative PRISM_E_* code and
 *     then sets a thread-local message readable with prism_last_error().
 *     No C++ exception crosses this boundary.
 *   - Ownership: the caller owns every buffer and the HIP stream.  Pointers
 *     documented as "device" must be device memory of the current HIP device;
 *     pointers documented as "host" are read during the call only.  The
 *     library allocates no device memory: scratch space comes in through a
 *     caller-provided workspace whose size the *_plan / *_workspace call
 *     reports (prism_probe_outputs_noalloc alone uses the library's fixed
 *     scratch array instead).  `stream` is a hipStream_t (NULL = the default
 *     stream).
 *   - Execution: work is queued on `stream` and the call returns without
 *     waiting for it, except where a function says it uploads host tables:
 *     those calls copy small host-computed tables into the workspace and wait
 *     for that copy on `stream` before queuing kernels.
 */
#ifndef PRISM_H
#define PRISM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PRISM_OK              0
#define PRISM_E_INVAL        -1   /* argument out of its documented range, NULL pointer */
#define PRISM_E_UNSUPPORTED  -2   /* valid physics, but a size this library does not build */
#define PRISM_E_NOMEM        -3   /* host allocation failed */
#define PRISM_E_DEVICE       -4   /* a HIP runtime call or kernel launch failed */
#define PRISM_E_WORKSPACE    -5   /* workspace pointer NULL or smaller than required */

/* ---- arithmetic of the beam contraction (probe synthesis) -------------- */
#define PRISM_FP32           0    /* FP32 products, FP32 accumulation                   */
#define PRISM_SPLIT_BF16X3   1    /* hi*hi + hi*lo + lo*hi BF16 MFMA, FP32 accumulation */
#define PRISM_BF16           2    /* hi*hi BF16 MFMA, FP32 accumulation (error reported) */

/* ---- structures -------------------------------------------------------- */
typedef struct prism_atom {
    double x, y, z;          /* position in A; x, y are wrapped into the cell */
    int32_t species;         /* index into the species table                   */
    int32_t pad;
} prism_atom;

/* Projected potential of one species as a sum of 2D Gaussians:
 * V(r) = sum_i amp[i] / (2 pi width[i]^2) exp(-r^2 / (2 width[i]^2)),
 * truncated at r < 6 max_i width[i].  amp = 2D integral (V*A^2), width = std-dev (A). */
typedef struct prism_species {
    int32_t n_gauss;         /* 1..4 */
    int32_t pad;
    double amp[4];
    double width[4];
} prism_species;

/* Simulation grid: the cell is cut into n_slices = ceil(Lz/dz) slabs along z. */
typedef struct prism_grid {
    int32_t n;               /* pixels per side */
    int32_t n_slices;        /* filled by prism_grid_init */
    double cell[3];          /* Lx, Ly, Lz (A); Lx must equal Ly */
    double dz;               /* slice thickness (A) */
} prism_grid;

/* Compact S-matrix geometry.  Inputs: grid, E0, alpha_max, f.  The rest is
 * filled by prism_smatrix_plan. */
typedef struct prism_smatrix_desc {
    prism_grid grid;
    double E0;               /* beam energy (eV) */
    double alpha_max;        /* largest beam angle = probe semi-angle (rad) */
    int32_t f;               /* interpolation factor: every f-th plane wave per axis */
    int32_t beam_batch;      /* input: beams propagated per launch, 0 = all; bounds the workspace */
    int32_t n_beams;         /* |B_f| */
    int32_t ns;              /* S-matrix side n/2 */
    int32_t m_win;           /* probe window side ns/f */
    int32_t pad;
    double lambda;           /* relativistic wavelength (A) */
    double sigma;            /* interaction constant (rad / (V*A)) */
    double alpha_aa;         /* anti-aliasing angle lambda*n/(4L) (rad) */
    size_t smatrix_bytes;    /* n_beams * ns * ns * 8 */
    size_t build_ws_bytes;   /* workspace of prism_build_smatrix for min(beam_batch, n_beams) beams per launch */
} prism_smatrix_desc;

/* Coherent probe aberrations carried by the probe coefficients ("PRISM Probe
 * Simulations"): exp(-i chi(q)), chi = pi lambda C1 |q|^2 + (pi/2) C3 lambda^3 |q|^4.
 * C1 (defocus) and C3 (spherical aberration) in A; C1 > 0 equals free
 * propagation of the probe over C1 before the specimen. */
typedef struct prism_aberrations {
    double C1;
    double C3;
} prism_aberrations;

/* Probe-synthesis plan (host side of a plan whose tables live in device memory). */
typedef struct prism_probe_plan {
    int64_t n_probes;
    int32_t n_bins;          /* detector bins (3D output depth) */
    int32_t n_tiles;         /* work tiles of the contraction: (tiling phase, 16 x 16 S-grid
                                pixel tile) pairs that at least one window overlaps */
    int64_t n_entries;       /* (work tile, probe) pairs */
    int32_t max_per_tile;    /* largest probe count of one work tile */
    int32_t n_binned;        /* window pixels that fall in a detector bin */
    double dalpha;           /* bin width (rad) */
    size_t plan_bytes;       /* device bytes of the plan tables */
    size_t ws_bytes;         /* workspace of prism_probe_outputs for all probes at once */
    double C1, C3;           /* aberrations the plan was made with */
    size_t off[10];          /* internal: offsets of the tables inside the plan buffer */
} prism_probe_plan;

/* ---- grid ---------------------------------------------------------------- */

/* Validate a grid and fill n_slices = ceil(Lz/dz).
 * Errors: PRISM_E_INVAL (n <= 0, dz <= 0, cell <= 0, NULL), PRISM_E_UNSUPPORTED
 * (Lx != Ly, n not a power of two in [64, 2048]). */
int prism_grid_init(const double cell[3], double dz, int32_t n, prism_grid* out);

/* ---- projected potential ("Calculation of the Projected Potentials") ------ */

/* Workspace bytes for prism_project_potential with n_atoms atoms. */
int prism_project_potential_workspace(int64_t n_atoms, size_t* bytes);

/* V[s][y][x] (device, float32, n_slices*n*n) = sum over atoms whose slab is s
 * (s = clamp(floor(z/dz), 0, n_slices-1)) of their Gaussian terms at the
 * minimum-image distance.  atoms, species: host arrays.  Uploads host tables.
 * Errors: PRISM_E_INVAL (bad species index, n_gauss outside 1..4, width <= 0,
 * cutoff 6*max(width) not below L/2), PRISM_E_WORKSPACE, PRISM_E_DEVICE. */
int prism_project_potential(const prism_atom* atoms, int64_t n_atoms,
                            const prism_species* species, int32_t n_species,
                            const prism_grid* grid, float* V,
                            void* ws, size_t ws_bytes, void* stream);

/* ---- compact S-matrix (Fig. 1g-h, Eqs. 1-2) ------------------------------- */

/* Fill the derived fields of *d: lambda, sigma, alpha_aa, beams B_f = every
 * f-th Fourier index (kx, ky) per axis with lambda*sqrt(kx^2+ky^2)/L <= alpha_max,
 * ns = n/2, m_win = ns/f, and the byte sizes.
 * Errors: PRISM_E_INVAL (E0 <= 0, alpha_max <= 0, f < 1, beam_batch < 0),
 * PRISM_E_UNSUPPORTED (alpha_max >= alpha_aa, f not dividing ns, m_win outside
 * [16, 512]). */
int prism_smatrix_plan(prism_smatrix_desc* d);

/* Copy the beam list (kx, ky pairs, host int32 [cap][2]) in the order of the
 * S-matrix layers.  Errors: PRISM_E_INVAL when cap < n_beams. */
int prism_beam_list(const prism_smatrix_desc* d, int32_t* k_out, int32_t cap);

/* Build S[b][my][mx] (device complex64, n_beams*ns*ns): plane wave
 * exp(2 pi i (kx x + ky y)/n) of beam b, transmitted by exp(i sigma V_s)
 * (Eq. 1) and propagated by the band-limited Fresnel propagator
 * [|q| < 1/(4 dx)] exp(-i pi lambda |q|^2 dz) (Eq. 2) through every slice,
 * stored in real space on every second pixel (exact by the band limit).
 * V: device float32 [n_slices][n][n].  Uploads host tables.
 * Errors: PRISM_E_INVAL, PRISM_E_WORKSPACE (ws_bytes < d->build_ws_bytes),
 * PRISM_E_DEVICE. */
int prism_build_smatrix(const prism_smatrix_desc* d, const float* V, void* S,
                        void* ws, size_t ws_bytes, void* stream);

/* Layers first .. first + count - 1 of the S-matrix of prism_build_smatrix
 * (beams in the order of prism_beam_list), bit-identical to the same layers
 * of the whole build; the other layers of S are not written.  S is the
 * whole S-matrix (n_beams layers).  For callers that issue a large build in
 * parts, e.g. a serving loop that keeps other requests' work from queuing
 * behind all of it.  Same workspace as prism_build_smatrix (sized by
 * beam_batch, not by count).  Uploads host tables.
 * Errors: as prism_build_smatrix; PRISM_E_INVAL when the range is not inside
 * [0, n_beams). */
int prism_build_smatrix_range(const prism_smatrix_desc* d, const float* V, void* S, int32_t first,
                              int32_t count, void* ws, size_t ws_bytes, void* stream);

/* Streams used by prism_build_smatrix (process-wide), n in 1..4, or 0 (the
 * default) for a count chosen by grid size: 4 for n <= 1024, 1 above.  Every
 * beam batch is split into n parts, run on `stream` and on n - 1
 * partner streams that the library creates once per caller stream (default
 * priority, kept until the process ends), each part one slice behind the
 * previous one, so that row and column passes of different beams run
 * together.  The call still returns with all work ordered on `stream`, and
 * the S-matrix is identical to the one-stream build (n = 1).  Batches of
 * fewer than n beams use as many streams as beams.  At most 32 caller
 * streams get partners; builds on any further caller stream run on that
 * stream alone.
 * Errors: PRISM_E_INVAL (n outside 0..4). */
int prism_set_build_streams(int32_t n);

/* ---- PRISM probe outputs (Fig. 1i-k) -------------------------------------- */

/* Plan the synthesis of n_probes probes at probe_xy (host float64 [n][2], A):
 * window centres (nearest S-grid pixel), the (pixel tile, probe) cover lists,
 * and the detector bin tables.  dalpha: bin width (rad); n_bins <= 0 selects
 * ceil(alpha_aa / dalpha).  ab: aberrations, NULL for none.  Fills *plan
 * (sizes) only. */
int prism_probe_plan_init(const prism_smatrix_desc* d, const double* probe_xy, int64_t n_probes,
                          double dalpha, int32_t n_bins, const prism_aberrations* ab,
                          prism_probe_plan* plan);

/* Compute the plan tables and upload them into plan_dev (device, plan->plan_bytes).
 * Uploads host tables (waits for the copy on `stream`).  The plan must have
 * been made by prism_probe_plan_init for these positions: every size the
 * kernels use (entries, tiles, largest probe count of a tile, binned pixels)
 * is checked.  Errors: PRISM_E_INVAL (NULL, a plan for other positions or for
 * a detector map), PRISM_E_DEVICE. */
int prism_probe_plan_upload(const prism_smatrix_desc* d, const double* probe_xy,
                            const prism_probe_plan* plan, void* plan_dev, void* stream);

/* Virtual detectors (Fig. 1e: detector outputs are sums of the diffraction
 * intensity over detector regions; "Description of Algorithms": 2D, 3D or
 * 4D outputs).  Instead of annular bins, the caller's detector map assigns
 * each pixel of the probe window's Fourier grid to a detector:
 * detector_map: host int32 [m_win][m_win], FFT order ([ky][kx], pitch f/L),
 * entries -1 (no detector) or a detector index in [0, n_bins); any shape of
 * detector (segments, inner/outer dark field, quadrants of a differential
 * phase contrast detector).  n_bins in [1, 4096].  The plan records
 * dalpha = 0.  out[p][b] of prism_probe_outputs is then the sum of
 * |FFT_M(psi_p)|^2 / M^4 over the pixels mapped to b.  The map is read during
 * the call only.  Errors: PRISM_E_INVAL (NULL map, an entry outside
 * [-1, n_bins), n_bins outside [1, 4096]), as prism_probe_plan_init. */
int prism_probe_plan_init_map(const prism_smatrix_desc* d, const double* probe_xy, int64_t n_probes,
                              const int32_t* detector_map, int32_t n_bins, const prism_aberrations* ab,
                              prism_probe_plan* plan);

/* prism_probe_plan_upload for a plan made by prism_probe_plan_init_map, with
 * the same map.  Errors: as prism_probe_plan_upload; PRISM_E_INVAL for an
 * annular plan or an invalid map. */
int prism_probe_plan_upload_map(const prism_smatrix_desc* d, const double* probe_xy,
                                const int32_t* detector_map, const prism_probe_plan* plan,
                                void* plan_dev, void* stream);

/* out[p][bin] (device float32 [n_probes][n_bins]) = sum over the bin's window
 * pixels of |FFT_M(psi_p)|^2 / M^4, where
 * psi_p[v][u] = sum_b c_b(p) S_b[(cy - M/2 + v) mod ns][(cx - M/2 + u) mod ns],
 * c_b(p) = |B_f|^(-1/2) exp(-2 pi i (kx_b x_p + ky_b y_p)/L) exp(-i chi(q_b)).
 * precision: PRISM_FP32, PRISM_SPLIT_BF16X3 or PRISM_BF16.  Fully asynchronous.
 * Errors: PRISM_E_INVAL, PRISM_E_WORKSPACE (ws_bytes < plan->ws_bytes), PRISM_E_DEVICE. */
int prism_probe_outputs(const prism_smatrix_desc* d, const void* S,
                        const prism_probe_plan* plan, const void* plan_dev,
                        int32_t precision, float* out,
                        void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (work under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * prism_probe_outputs with the same kernels and result, its workspace taken
 * from a fixed scratch array of PRISM_NOALLOC_SCRATCH_BYTES that the library
 * holds on each GPU it runs on until the process ends.  The caller passes the
 * inputs (S, the uploaded plan) and the output as for prism_probe_outputs.
 * The call allocates nothing on the device.  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (on different streams or
 * from different threads) race and must not be issued.  Fully asynchronous.
 * Errors: PRISM_E_WORKSPACE when the plan's workspace (plan->ws_bytes)
 * exceeds PRISM_NOALLOC_SCRATCH_BYTES; otherwise as prism_probe_outputs. */
#define PRISM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int prism_probe_outputs_noalloc(const prism_smatrix_desc* d, const void* S,
                                const prism_probe_plan* plan, const void* plan_dev,
                                int32_t precision, float* out, void* stream);

/* 4D output (Fig. 1e/k, "the entire probe diffraction pattern"):
 * out4d[p][ky][kx] (device float32 [n_probes][m_win][m_win], FFT order on the
 * window's Fourier grid, pitch f/L) = |FFT_M(psi_p)|^2 / M^4, psi_p as in
 * prism_probe_outputs.  Same workspace as prism_probe_outputs.  Fully
 * asynchronous.  Errors: PRISM_E_INVAL, PRISM_E_WORKSPACE, PRISM_E_DEVICE. */
int prism_probe_diffraction(const prism_smatrix_desc* d, const void* S,
                            const prism_probe_plan* plan, const void* plan_dev,
                            int32_t precision, float* out4d,
                            void* ws, size_t ws_bytes, void* stream);

/* One request's probe synthesis inside a batched call (all pointers borrowed
 * for the call; device pointers as in prism_probe_outputs). */
typedef struct prism_probe_job {
    const prism_smatrix_desc* desc;   /* host */
    const void* S;                    /* device complex64 [n_beams][ns][ns] */
    const prism_probe_plan* plan;     /* host */
    const void* plan_dev;             /* device plan tables */
    float* out;                       /* device float32 [n_probes][n_bins] (3D output), or NULL */
    float* diffraction;               /* device float32 [n_probes][m_win][m_win] (4D output), or NULL */
    float out_scale;                  /* out = out_scale * bin sums, diffraction =
                                         out_scale * intensities ...                       */
    int32_t accumulate;               /* ... + the previous contents of out (and of
                                         diffraction) when 1, e.g. averaging frozen-phonon
                                         configurations of the 3D or 4D output; 0 or 1 */
} prism_probe_job;

/* Workspace bytes of prism_probe_outputs_batched for these jobs. */
int prism_probe_batch_workspace(const prism_probe_job* jobs, int32_t n_jobs, size_t* bytes);

/* Probe outputs of several independent jobs (different S-matrices, grids,
 * interpolation factors and probe sets) in one pass on one stream: the
 * windowed contractions of all jobs share launches, as do the window
 * transforms of jobs with the same window side.  Each job's result is the
 * one prism_probe_outputs gives for it alone (same kernels, same order of
 * operations).  Fully asynchronous.
 * Errors: PRISM_E_INVAL, PRISM_E_WORKSPACE, PRISM_E_DEVICE. */
int prism_probe_outputs_batched(const prism_probe_job* jobs, int32_t n_jobs, int32_t precision,
                                void* ws, size_t ws_bytes, void* stream);

/* ---- multislice probe outputs (Fig. 1c-e) --------------------------------- */

/* Workspace bytes for multislice_outputs over n_probes probes processed
 * `batch` at a time. */
int multislice_workspace(const prism_grid* grid, int32_t batch, int64_t n_probes, size_t* bytes);

/* out[p][bin] (device float32 [n_probes][n_bins]): hard-aperture probe
 * (lambda |q| <= alpha_max) with coefficients |B_1|^(-1/2) exp(-2 pi i q.r_p)
 * exp(-i chi(q)) (ab: aberrations, NULL for none),
 * transmitted and propagated through every slice (Eqs. 1-2), then
 * |Psi(q)|^2 / n^4 summed over annular bins of width dalpha up to alpha_aa.
 * probe_xy: host float64 [n_probes][2].  V: device float32 [n_slices][n][n].
 * The probes are processed `batch` at a time inside ws.  Uploads host tables.
 * Errors: PRISM_E_INVAL, PRISM_E_UNSUPPORTED, PRISM_E_WORKSPACE, PRISM_E_DEVICE. */
int multislice_outputs(const prism_grid* grid, double E0, double alpha_max, const prism_aberrations* ab,
                       const float* V, const double* probe_xy, int64_t n_probes, double dalpha,
                       int32_t n_bins, int32_t batch, float* out, void* ws, size_t ws_bytes, void* stream);

/* multislice_outputs with the caller's detector map over the n x n Fourier
 * grid (host int32 [n][n], FFT order [ky][kx], pitch 1/L; entries -1 or a
 * detector in [0, n_bins), n_bins in [1, 4096]) instead of annular bins:
 * out[p][b] = sum over the pixels mapped to b of |Psi(q)|^2 / n^4 (pixels
 * outside the propagator's band carry no intensity).  Uses the workspace of
 * multislice_workspace.  Errors: as multislice_outputs; PRISM_E_INVAL for a
 * NULL or invalid map. */
int multislice_outputs_map(const prism_grid* grid, double E0, double alpha_max, const prism_aberrations* ab,
                           const float* V, const double* probe_xy, int64_t n_probes,
                           const int32_t* detector_map, int32_t n_bins, int32_t batch, float* out,
                           void* ws, size_t ws_bytes, void* stream);

/* ---- streaming memory model ("Streaming Data for Very Large Simulations") --- */
/* For cells whose potential or S-matrix should not be resident in device
 * memory: the large arrays stay in host memory (page-locked, e.g. from
 * hipHostMalloc, for the copies to be asynchronous) and only the subset the
 * current step needs is staged through small device buffers.  Copies are
 * issued on the caller's copy streams and overlap the kernels running on the
 * compute stream; each staging buffer is double-buffered and guarded by HIP
 * events, so the copy of the next slice (or beam chunk) proceeds while the
 * current one is processed.  The results are those of the single-transfer
 * entry points: the build and multislice give bit-identical outputs; the
 * streamed synthesis sums its beam chunks in order into FP32 windows.
 *
 * Streams: `stream` runs the kernels; `h2d_stream` and `d2h_stream` carry
 * the host-to-device and device-to-host copies (they may be the same stream,
 * or `stream` itself, at the cost of overlap).  The copies start after the
 * work enqueued on `stream` before the call.  On return all work is enqueued
 * and `stream` is made to wait for every copy, so the results (including
 * host-side S) are complete once `stream` has drained.  The host
 * arrays must stay alive and unmodified until then.  HIP events are created
 * and destroyed per call; no device memory is allocated. */

/* Device workspace of prism_build_smatrix_streaming: two potential-slice
 * buffers, one transmission slice, the wave buffer of one beam batch and two
 * S staging buffers of one batch. */
int prism_streaming_build_workspace(const prism_smatrix_desc* d, size_t* bytes);

/* Same S-matrix as prism_build_smatrix (bit-identical), with V in host memory
 * (float32 [n_slices][n][n]) and S written to host memory
 * (complex64 [n_beams][ns][ns]).  Every beam batch streams all slices of V
 * (one slice ahead) and its finished S layers are copied out while the next
 * batch runs.
 * Errors: PRISM_E_INVAL, PRISM_E_WORKSPACE, PRISM_E_DEVICE. */
int prism_build_smatrix_streaming(const prism_smatrix_desc* d, const float* V_host, void* S_host,
                                  void* ws, size_t ws_bytes, void* stream, void* h2d_stream,
                                  void* d2h_stream);

/* Device workspace of prism_probe_outputs_streaming with beam_chunk beams
 * staged at a time (two S chunk buffers, the coefficients of one chunk, the
 * windows of all probes). */
int prism_probe_streaming_workspace(const prism_smatrix_desc* d, const prism_probe_plan* plan,
                                    int32_t beam_chunk, size_t* bytes);

/* prism_probe_outputs (out, or the 4D output out4d when out is NULL) with S in
 * host memory (complex64 [n_beams][ns][ns]): beam chunks are copied in one
 * chunk ahead and their windowed contractions accumulate into the FP32
 * windows before the window transform.  beam_chunk in [1, n_beams].
 * Errors: PRISM_E_INVAL, PRISM_E_WORKSPACE, PRISM_E_DEVICE. */
int prism_probe_outputs_streaming(const prism_smatrix_desc* d, const void* S_host,
                                  const prism_probe_plan* plan, const void* plan_dev,
                                  int32_t precision, int32_t beam_chunk, float* out, float* out4d,
                                  void* ws, size_t ws_bytes, void* stream, void* h2d_stream);

/* Device workspace of prism_probe_outputs_chunked with beam_chunk beams per
 * chunk (coefficients and split S of one chunk, the windows of all probes). */
int prism_probe_chunked_workspace(const prism_smatrix_desc* d, const prism_probe_plan* plan,
                                  int32_t beam_chunk, size_t* bytes);

/* prism_probe_outputs (out, or the 4D output out4d when out is NULL) with S in
 * device memory, contracted beam_chunk beams at a time into FP32 windows:
 * the MFMA precisions then need a split copy of one chunk of S instead of
 * all of it (workspace for S-matrices too large to duplicate).  The result
 * equals prism_probe_outputs_streaming's for the same chunk size.  Fully
 * asynchronous.  Errors: PRISM_E_INVAL, PRISM_E_WORKSPACE, PRISM_E_DEVICE. */
int prism_probe_outputs_chunked(const prism_smatrix_desc* d, const void* S,
                                const prism_probe_plan* plan, const void* plan_dev,
                                int32_t precision, int32_t beam_chunk, float* out, float* out4d,
                                void* ws, size_t ws_bytes, void* stream);

/* Device workspace of multislice_outputs_streaming. */
int multislice_streaming_workspace(const prism_grid* grid, int32_t batch, int64_t n_probes,
                                   size_t* bytes);

/* multislice_outputs (bit-identical) with V in host memory (float32
 * [n_slices][n][n]): each probe batch streams the slices one ahead through
 * two device slice buffers, as the paper's streaming multislice keeps only
 * the current slice of the potential on the device.
 * Errors: as multislice_outputs. */
int multislice_outputs_streaming(const prism_grid* grid, double E0, double alpha_max,
                                 const prism_aberrations* ab, const float* V_host,
                                 const double* probe_xy, int64_t n_probes, double dalpha,
                                 int32_t n_bins, int32_t batch, float* out, void* ws,
                                 size_t ws_bytes, void* stream, void* h2d_stream);

/* ---- detector geometry ------------------------------------------------------ */

/* map[ky][kx] (host int32 [m][m], FFT order) = floor(alpha / dalpha) with
 * alpha = lambda * sqrt(kx^2 + ky^2) / Lw, or -1 when alpha >= alpha_aa or the
 * bin is >= n_bins.  Every step is a correctly rounded float64 operation. */
int prism_detector_bin_map(double lambda, double Lw, double alpha_aa, double dalpha,
                           int32_t n_bins, int32_t m, int32_t* map);

/* Detector extent of a grid ("Multislice Probe Simulations", Fig. 1e: annular
 * bins up to the largest angle the band-limited propagation of Eq. 2 keeps):
 * alpha_aa = lambda n / (4 L), the anti-aliasing angle, and
 * n_bins = ceil(alpha_aa / dalpha), the bin count that multislice_outputs and
 * prism_probe_plan_init use when given n_bins <= 0.  `alpha_aa` may be NULL.
 * Host only.  Errors: PRISM_E_INVAL (E0 <= 0, dalpha <= 0, NULL n_bins or grid),
 * those of prism_grid_init for the grid. */
int prism_detector_default_bins(const prism_grid* grid, double E0, double dalpha, int32_t* n_bins,
                                double* alpha_aa);

/* ---- kernel timing (diagnostics) --------------------------------------------- */

#define PRISM_K_PASS_A         0   /* row pass: inverse row DFT, transmission, forward row DFT */
#define PRISM_K_PASS_B         1   /* column pass: forward column DFT, propagator, inverse column DFT */
#define PRISM_K_FINAL          2   /* S-matrix real-space store */
#define PRISM_K_TRANSMISSION   3   /* exp(i sigma V); also the first slice's row spectrum */
#define PRISM_K_COEFFICIENTS   4   /* probe coefficients */
#define PRISM_K_CONTRACT       5   /* windowed beam contraction */
#define PRISM_K_WINDOW         6   /* window FFT, |Psi|^2, detector sums */
#define PRISM_K_POTENTIAL      7   /* projected potential */
#define PRISM_K_BIN_REDUCE     8   /* multislice detector sums */
#define PRISM_K_SPLIT          9   /* S-matrix to split-BF16 records (MFMA precisions) */
#define PRISM_K_FIRST         10   /* first slice of an S-matrix build (plane waves from the row spectrum) */
#define PRISM_TIMING_CLASSES  11

/* While enabled (per calling thread), every kernel launch of the library is
 * bracketed by HIP events recorded on its stream. */
int prism_timing_enable(int32_t enable);
/* Drop pending events and zero the totals of the calling thread. */
int prism_timing_reset(void);
/* Total device milliseconds and launch count of kernel class `cls` since the
 * last reset; waits for the recorded events.  Errors: PRISM_E_INVAL, PRISM_E_DEVICE. */
int prism_timing_read(int32_t cls, double* total_ms, int64_t* launches);

/* Diagnostic: copies `bytes` (a multiple of 16) from src to dst (device,
 * 16-byte aligned, not overlapping) with one 16-byte load and store per
 * thread, the plain streaming pattern that calibrates the HBM bandwidth the
 * propagation passes are compared with.  Enqueued on `stream`.
 * Errors: PRISM_E_INVAL, PRISM_E_DEVICE. */
int prism_device_copy(const void* src, void* dst, size_t bytes, void* stream);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* prism_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PRISM_H */
