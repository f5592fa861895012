/*
 * hmd.h -- C ABI of libhmd: an MI355X (gfx950) NEMD channel micro-solver and
 * the surrogates of a hybrid continuum-atomistic channel-flow scheme.
 *
 * Method: D. Stephenson, J. R. Kermode, D. A. Lockerby, "Accelerating a
 * hybrid continuum-atomistic fluidic model with on-the-fly machine learning"
 * (arXiv:1603.04628).
 *
 * Conventions for every call
 *   - Reduced Lennard-Jones units: eps = sigma = m = k_B = 1.
 *   - Host arrays passed in are owned by the caller and copied before the call
 *     returns; host arrays passed out are caller-allocated with the stated size.
 *   - Device memory, HIP streams and graphs are owned by the library and freed
 *     by the matching *_free / hmd_destroy.
 *   - Every int-returning call returns HMD_OK (0) or a negative hmd_status; a
 *     message is kept per context and read with hmd_last_error().  No C++
 *     exception crosses this boundary.
 *   - A context and everything created from it is NOT thread-safe: use one
 *     context per host thread.  Calls on one context run in order on its
 *     stream and return after their results are on the host.
 */
#ifndef HMD_H
#define HMD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HMD_OK = 0,
    HMD_EINVAL = -1,     /* bad argument (null pointer, size, range)            */
    HMD_EDEVICE = -2,    /* a HIP runtime call failed                           */
    HMD_ENOMEM = -3,     /* host or device allocation failed                    */
    HMD_EUNSTABLE = -4,  /* MD blew up: non-finite state or an atom left the gap */
    HMD_ENOTCONV = -5,   /* sampled flux not stationary (critical shear), Sec. 3.2 */
    HMD_ENOTSPD = -6,    /* GP covariance not positive definite                 */
    HMD_ENOSYS = -7      /* not available in this library                       */
} hmd_status;

typedef struct hmd_ctx hmd_ctx;
typedef struct hmd_sys hmd_sys;
typedef struct hmd_batch hmd_batch;
typedef struct hmd_gp hmd_gp;
typedef struct hmd_ens hmd_ens;
typedef struct hmd_hybrid hmd_hybrid;

/* ------------------------------------------------------------------------
 * MD model parameters (Appendix A of the paper: shifted LJ fluid, frozen
 * FCC walls, velocity Verlet, Berendsen thermostat on one velocity component,
 * periodic in x (streamwise) and z (spanwise); body force of Eq. momentumEq).
 * hmd_md_params_default() fills the stated defaults:
 *   rho 0.8, T0 1, rc 2.5, eps_wf 1, sigma_wf 1, rho_wall 1, wall_layers 4,
 *   thermo_axis 1 (y), dt 0.005, tau_T 0.1, Lx = Lz = 12 (nominal, snapped to
 *   whole wall cubes), bin_dy 0.25, n_equil 0, n_blocks 0, n_fluid 0
 *   (= round(rho Lx Lz h)), delta 1 (first lattice plane above a wall).
 * ------------------------------------------------------------------------ */
typedef struct {
    double rho, T0, rc, eps_wf, sigma_wf, rho_wall;
    int wall_layers, thermo_axis;
    double dt, tau_T, Lx_nom, Lz_nom, bin_dy;
    int64_t n_equil;
    /* standard error of the sampled flux: 0 = Geyer's initial monotone
     * sequence estimator over the per-step series (default); 2..1024 = the
     * standard deviation of that many contiguous block means / sqrt(n) */
    int n_blocks;
    int64_t n_fluid;
    double delta;
    /* Implementation choices (results agree to the force tolerance):
     * force_path 0: cell list rebuilt every step, forces over the 27
     * neighbouring cells; 1: Verlet pair list (cut-off rc + skin) rebuilt
     * from the cell list whenever an atom has moved skin/2 since the last
     * build; 2: the same lists for workgroups that each own a tile of whole
     * cell columns and read their neighbours' positions from LDS (16-bit
     * list entries); 3: path 2 with every tile on the position-index
     * fallback that a tile takes when its neighbourhood exceeds the LDS
     * capacity (for tests; reported as path 2); -1: the library's tuned
     * choice.  cell_w: minimum cell width (0: rc, or rc + skin for the pair
     * lists).  tile_alpha (tiled path): each system's tiles take the column
     * count that minimises (padded lanes + tile_alpha x staged atoms) per
     * home atom; 0 = fill the lanes, larger values favour wider tiles that
     * stage less halo per atom.  graph_chunk: steps per captured graph of
     * the whole-run calls (even; 0 = 100).  force_path -1 applies what
     * md_autotune chose for the workload, where it has run. */
    int force_path;
    double skin, cell_w;
    double tile_alpha;
    int graph_chunk;
    /* pressure 1: sampled steps also record the normal pressure the fluid
     * exerts on the walls, (F_lo,y - F_hi,y) / (2 Lx Lz) (the cross-section
     * average of P_yy, by the yy momentum balance; Alg. 1's pressure output
     * of an MD run), into a per-step series beside the flux; results then
     * carry p and p_se.  Pair paths only (force_path 0 is rejected); the
     * force kernel of a sampled step then costs a few instructions more per
     * pair.  0 (default): no pressure. */
    int pressure;
} hmd_md_params;

void hmd_md_params_default(hmd_md_params* p);

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * run on, or NULL for a library-owned stream (default priority).  `params`
 * may be NULL for the defaults.  *out receives the context. */
int hmd_create(const hmd_md_params* params, int device, void* hip_stream, hmd_ctx** out);
void hmd_destroy(hmd_ctx* ctx);
const char* hmd_last_error(const hmd_ctx* ctx);
/* Achievable rates of the context's device, for the rooflines beside the
 * published peaks.  Each kernel runs once to warm up, then five timed times:
 * out[0] FP32 fused multiply-add TFLOP/s (eight independent chains per
 * thread, unpacked as this library is compiled), out[1] FP32 reciprocals
 * per second (x 1e12), out[2] the time of a reciprocal in fused
 * multiply-adds, out[3] GB/s of a 1 GiB device copy (bytes read plus
 * written).  `out` is a caller-owned host array of 4 doubles.  Allocates
 * and frees 2 GiB on the device; ENOMEM if it cannot, EINVAL for a null
 * pointer, EDEVICE for a failed launch.  Synchronises the context's stream. */
int hmd_measure_peaks(hmd_ctx* ctx, double* out);
/* Replace (or read) the MD parameters used by later calls on this context. */
int hmd_set_params(hmd_ctx* ctx, const hmd_md_params* params);
int hmd_get_params(const hmd_ctx* ctx, hmd_md_params* params);

/* ------------------------------------------------------------------------
 * The micro-solve.  A job is one NEMD channel (Sec. 2.1, quasi-steady
 * subdomain run): channel height h (gap between the innermost wall planes),
 * body-force acceleration g along +x (g = F/m of Eq. momentumEq, i.e.
 * F_ext/m - (1/rho) dp/dx), Philox seed, number of sampling steps after
 * params.n_equil equilibration steps.
 * Result: mean mass flow rate per unit span q' = sum(m v_x)/(Lx Lz) over the
 * sampled steps, its standard error from the per-step series (Sec. 2.3: the
 * noise of a run is the standard deviation of its mean, from the raw
 * time-instantaneous data; estimator per params.n_blocks, see
 * md_series_stats), J = q'/h, the sampled
 * kinetic temperatures per component, the potential energy per atom at the
 * end, the fluid atom count and a per-job status (HMD_OK, HMD_EUNSTABLE,
 * HMD_ENOTCONV).
 * ------------------------------------------------------------------------ */
/* rho: fluid density of this job (atoms N_f = round(rho Lx Lz h)); <= 0
 * takes params.rho. */
typedef struct { double h, g; uint64_t seed; int64_t n_sample; double rho; } hmd_md_job;
/* p, p_se: mean wall normal pressure and its standard error (same
 * estimator as the flux) when params.pressure is on, else 0. */
typedef struct {
    double flux, flux_se, jflux, T[3], pe; int64_t n_fluid; int status; double p, p_se;
} hmd_md_result;

/* One job; flux and se receive q' and its standard error.  Returns the job's
 * status (a failed run returns HMD_EUNSTABLE / HMD_ENOTCONV with the values
 * still written). */
int md_flux(hmd_ctx* ctx, double h, double g, uint64_t seed, int64_t steps, double* flux, double* se);

/* n jobs of any heights and forces run together as one batch (one flattened
 * launch per kernel, step loop replayed as a HIP graph).  out[n] receives
 * per-job results, each with its own status; the call returns HMD_OK unless
 * the batch as a whole could not run. */
int md_flux_batch(hmd_ctx* ctx, const hmd_md_job* jobs, int n, hmd_md_result* out);
/* Device-pointer form (interop with a framework's tensors): jobs stay on the
 * host (the geometry is built there); flux, SE and status of each job land in
 * the device arrays d_flux[n], d_se[n], d_status[n] through copies on
 * `stream` (NULL: the context's stream), complete when the call returns. */
int md_flux_batch_dev(hmd_ctx* ctx, const hmd_md_job* jobs, int n, double* d_flux, double* d_se, int* d_status,
                      void* stream);

/* Staged form of md_flux_batch, for timing the step loop alone: create sets
 * up and uploads every system; run advances all systems by `steps` steps
 * (the equilibration + sampling schedule counts from creation); results
 * writes what md_flux_batch would; graph_chunk > 0 replays the step loop as a
 * HIP graph of that many steps (even), 0 launches kernels one by one. */
int md_batch_create(hmd_ctx* ctx, const hmd_md_job* jobs, int n, hmd_batch** out);
int md_batch_run(hmd_batch* b, int64_t steps, int graph_chunk);
int md_batch_results(hmd_batch* b, hmd_md_result* out);
/* Set the state of one system of a batch (atom id order, n_fluid x 3
 * doubles each), e.g. a warm start from a stored state; the forces are
 * recomputed.  The step count and sampling schedule are unchanged. */
int md_batch_set_state(hmd_batch* b, int sim, const double* x, const double* v);
/* The same for m systems at once (one upload): system sims[j] takes x[j]
 * and v[j] (n_fluid x 3 doubles each, atom id order); the others keep
 * their state.  EINVAL for an index out of range or given twice. */
int md_batch_set_states(hmd_batch* b, int m, const int* sims, const double* const* x, const double* const* v);
/* The states of every system (one download): x[k] and v[k] receive system
 * k's positions and velocities (n_fluid x 3 doubles each, atom id order);
 * a null x[k] or v[k] skips it. */
int md_batch_get_states(hmd_batch* b, double* const* x, double* const* v);
/* The sampled flux series q'(t) of one system (Sec. 2.1 flow rate per step):
 * *n receives its length, q (nullable, *n doubles) the values.  One entry
 * per sampled step while n_sample <= 65536; beyond, each entry is the mean
 * of B = ceil(n_sample / 65536) consecutive steps (the first n_sample mod B
 * sampled steps are left out).  Entries past the steps run so far read 0.
 * EINVAL for a batch created with n_sample = 0. */
int md_batch_series(hmd_batch* b, int sim, double* q, int64_t* n);
/* The sampled wall-pressure series of one system (params.pressure on), laid
 * out as md_batch_series; EINVAL with pressure off. */
int md_batch_pressure_series(hmd_batch* b, int sim, double* p, int64_t* n);
/* Fluid atoms summed over the batch (for atom-step rates). */
int64_t md_batch_atoms(const hmd_batch* b);
/* Average duration in ms of each kernel over the md_batch_run calls made
 * since timing was switched on: names are "integrate", "keys", "scan",
 * "scatter", "reorder", "list", "force"; "graph_step" gives the average time
 * of one step of the stamped graph replays.  Direct launches are timed by
 * HIP events on the batch's stream.  Graph replays (graph_chunk > 0): one
 * replay in ten is a graph whose kernels of ten evenly spaced steps are
 * bracketed by clock-stamp kernels (a kernel's time is the difference of its
 * stamps less that of two adjacent stamps with nothing between them, at the
 * device's wall-clock rate), timed by events and read back; the other
 * replays run the plain graph without host synchronisation.  Stamped graph
 * replays also give "list_rebuild" and "list_idle": the list build's mean
 * time on stamped steps that rebuild the pair lists and on those that do
 * not, so that a per-step figure can be weighted by the exact rebuild rate
 * (md_batch_list_builds) rather than by the rebuilds that fell on stamped
 * steps. */
int md_batch_set_timing(hmd_batch* b, int on);
int md_batch_kernel_ms(const hmd_batch* b, const char* kernel, double* ms, int64_t* launches);
/* In-cutoff pairs at the current positions, summed over the batch:
 * ordered fluid-fluid pairs (each unordered pair counted twice, once per
 * atom of the full neighbour sum) and wall-fluid pairs.  Runs one extra
 * force evaluation (forces unchanged). */
int md_batch_pair_count(hmd_batch* b, int64_t* fluid_pairs, int64_t* wall_pairs);
/* Number of Verlet pair-list builds made since the batch was created or its
 * state last set (Sec. 2.1 neighbour search; 0 on the cell path).  A build
 * happens whenever some atom of the batch has moved more than half the skin
 * since the previous one. */
int md_batch_list_builds(hmd_batch* b, int64_t* builds);
/* One system of a batch, for checks at full batch size: its state (atom id
 * order, n_fluid x 3 each; x and v may be null to ask for n_fluid only) and
 * the forces at that state (recomputed, FP32, n_fluid x 3) with its
 * potential energy. */
int md_batch_get_state(hmd_batch* b, int sim, double* x, double* v, int64_t* n_fluid);
int md_batch_forces(hmd_batch* b, int sim, float* f, double* pe);
/* The implementation choices in use: force path (0 cell, 1 pair list),
 * pair-list skin, threads per block, pair-list capacity per atom. */
int md_batch_config(const hmd_batch* b, int* path, double* skin, int* tpb, int* list_cap);
/* All implementation choices of a batch, 8 doubles: force path, skin,
 * threads per block, tile_alpha, cell width in use (sigma), graph chunk of
 * whole-run calls, tiles (tiled path) and pair-list capacity. */
int md_batch_tuning(const hmd_batch* b, double out[8]);

/* Autotuner (the project's own): picks the force path, pair-list skin (0.05
 * steps), tile size (tile_alpha), cell width and graph chunk for these jobs
 * by timing them.  One warm-up batch of the default configuration runs
 * probe_steps steps from the start lattice; every candidate then starts from
 * that warmed state and is timed over probe_steps steps of graph replays.
 * The search is coordinate descent: path and threads per block, then skin,
 * then tile_alpha, then cell width, then graph chunk, each axis at the best
 * of the previous ones.  The winner is kept for later batches of the same
 * workload signature on this context (number of systems, total atoms to a
 * factor of 2, box, mean height to 1 sigma) and used when force_path is -1.
 * table (nullable, room for 64 rows of 7 doubles): per candidate path,
 * skin, threads per block, tile_alpha, cell width parameter, graph chunk, ms
 * per step; n_rows receives the number of candidates timed. */
int md_autotune(hmd_ctx* ctx, const hmd_md_job* jobs, int n, int probe_steps, double* table, int* n_rows);
void md_batch_free(hmd_batch* b);

/* ------------------------------------------------------------------------
 * Mean and standard error of sampled series (Sec. 2.3: the noise level of an
 * MD run is the standard deviation of its mean output, estimated from the
 * raw time-instantaneous data).  x holds S series of n samples each, row k
 * at x + k ld (ld >= n).  n_blocks = 0: Geyer's initial monotone sequence
 * estimator (Statistical Science 7 (1992) 473, Sec. 3.3): from the
 * autocovariances gamma_t = (1/n) sum_{i<n-t} (x_i - mean)(x_{i+t} - mean),
 * the pair sums gamma_2k + gamma_2k+1 are summed while positive, each
 * replaced by the smallest so far, sigma^2 = -gamma_0 + 2 sum, SE =
 * sqrt(sigma^2 / n) (gamma_0 / n when the sum is not positive).  n_blocks in
 * 2..1024: the standard deviation of n_blocks contiguous block means over
 * sqrt(n_blocks), a remainder of n mod n_blocks dropped from the front.
 * out receives 4 doubles per series: mean, SE, mean of the first half,
 * mean of the second half (of the block means for the block rule).
 * EINVAL unless 1 <= S <= 65535, n >= 2, ld >= n and n >= n_blocks.  All
 * arithmetic FP64 on the device; the host form copies x in and out back and
 * returns when done.
 * ------------------------------------------------------------------------ */
int md_series_stats(hmd_ctx* ctx, const double* x, int S, int64_t n, int64_t ld, int n_blocks, double* out);
/* Device-pointer form: d_x (S rows, stride ld) and d_out (4 S doubles) are
 * device arrays; queued on `stream` (NULL: the context's stream) without
 * waiting.  The autocovariances need S n doubles of scratch, which the
 * context allocates on first use and keeps (growing it waits for the
 * device); calls of one context on different streams must not overlap. */
int md_series_stats_dev(hmd_ctx* ctx, const double* d_x, int S, int64_t n, int64_t ld, int n_blocks, double* d_out,
                        void* stream);
/* Allocation-free form of md_series_stats_dev, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid it): same arguments, results and kernels, but the
 * autocovariance scratch is a fixed array of 2^21 doubles (16 MiB) in device
 * memory, one per GPU, held until the process ends; this call allocates and
 * frees nothing.  EINVAL when n_blocks = 0 and S n > 2^21 (the block rule
 * needs no scratch).  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (other streams, other contexts or threads) race
 * and must be serialised by the caller.  Nothing in the scratch needs to
 * start at zero (each call writes every entry it reads).  Queued on `stream`
 * (NULL: the context's stream) without waiting. */
int md_series_stats_noalloc(hmd_ctx* ctx, const double* d_x, int S, int64_t n, int64_t ld, int n_blocks,
                            double* d_out, void* stream);

/* ------------------------------------------------------------------------
 * Single-system hooks (tests, checkpoint/restart).  Atom order in every
 * array below is the atom id order fixed at creation.
 * ------------------------------------------------------------------------ */
int md_sys_create(hmd_ctx* ctx, double h, double g, uint64_t seed, hmd_sys** out);
/* n_fluid, n_wall, box = {Lx, h, Lz}, ncell = {nx, ny, nz} fluid cells. */
int md_sys_info(hmd_sys* s, int64_t* n_fluid, int64_t* n_wall, double box[3], int ncell[3]);
/* x, v: n_fluid x 3 doubles, row-major.  set_state recomputes forces. */
int md_set_state(hmd_sys* s, const double* x, const double* v);
int md_get_state(hmd_sys* s, double* x, double* v, int64_t* n_fluid);
/* FP32 pair forces (plus g is NOT included) for the current positions:
 * f is n_fluid x 3 floats; pe (nullable) the shifted potential energy. */
int md_compute_forces(hmd_sys* s, float* f, double* pe);
/* Cell lists of the current positions: cell_of_atom[n_fluid] (fluid cell
 * index (cz*ny + cy)*nx + cx), cell_count[nx*ny*nz], order[n_fluid] = atom ids
 * cell-major (order within a cell = the library's stable sort order). */
int md_cell_lists(hmd_sys* s, uint32_t* cell_of_atom, uint32_t* cell_count, uint32_t* order);
/* Advance `steps` steps; thermostat_on = 0 gives NVE (plus the body force);
 * energy_trace (nullable, `steps` doubles): total energy per atom after each
 * step. */
int md_run(hmd_sys* s, int64_t steps, int thermostat_on, double* energy_trace);
/* Wall-normal profile accumulated over the sampled steps: per bin of width
 * params.bin_dy from y = 0, the sum of v_x and the atom count (ceil(h/bin_dy)
 * doubles each). */
int md_sys_profile(hmd_sys* s, double* mvx, double* cnt);
/* Pair path only: the Verlet lists of the last build, per atom id, as sorted
 * neighbour ids (fluid ids, or N_f + wall index for wall atoms); counts has
 * n_fluid entries, idx up to cap entries, total receives the entry count. */
int md_neighbor_lists(hmd_sys* s, uint32_t* counts, uint32_t* idx, int64_t cap, int64_t* total);
int md_sys_config(hmd_sys* s, int* path, double* skin, int* tpb, int* list_cap);
void md_sys_free(hmd_sys* s);

/* ------------------------------------------------------------------------
 * Gaussian-process surrogate (Sec. 2.2): squared-exponential kernel
 * (Eq. quadraticKernelEq) on inputs normalised by the mean separation of the
 * database inputs (Eq. d2Eq), noisy covariance C = K + sigma_n^2 I
 * (Eq. covarianceEq), posterior mean and variance (Eqs. predMeanEq,
 * predVarEq), log marginal likelihood (Eq. evidenceEq).  Prior mean zero.
 * X is row-major n x d (1 <= d <= 4); y the outputs; y_se (nullable)
 * per-point standard errors.  Readings: the mean separation is the mean of
 * |x_ik - x_jk| over pairs i < j (a quarter of range[k] with fewer than two
 * points, or when scale_mode = 1); with out_scale the outputs are divided by
 * their RMS before fitting; sigma_n < 0 means mean(y_se) in those units.
 * gp_append refits (the normalisation moves with the data) except when the
 * normalisation, noise and output scale are all fixed, where it extends the
 * Cholesky factor by one row.  L^-1 is kept beside the factor (extended
 * by a row on such an append) so that a query costs one triangular
 * product.  At most 6144 points (EINVAL beyond).  All arithmetic FP64 on
 * the device; ENOTSPD when the covariance is not positive definite.
 * ------------------------------------------------------------------------ */
typedef struct {
    double sigma_f, ell, sigma_n;  /* sigma_n < 0: mean(y_se) / output scale */
    int scale_mode;                /* 0: mean pairwise separation; 1: fixed ranges */
    double range[4];               /* per-input ranges for scale_mode 1 / fallback */
    int out_scale;                 /* 1: divide y by its RMS before fitting */
    /* noise_mode 1: heteroscedastic noise, each point's own (y_se_i / output
     * scale)^2 on the diagonal of C in place of sigma_n^2.  kernel 1: the
     * periodic kernel of App. B (Eq. periodicKernel),
     * sigma_f^2 exp(-2 sin^2(pi |t - t'| / period) / ell^2), on a single
     * input (d = 1) with no input normalisation. */
    int noise_mode;
    int kernel;
    double period;
} hmd_gp_hyper;

void hmd_gp_hyper_default(hmd_gp_hyper* h);
int gp_fit(hmd_ctx* ctx, const double* X, const double* y, const double* y_se, int n, int d,
           const hmd_gp_hyper* hyper, hmd_gp** out);
/* Append one observation (Alg. 1: database growth and covariance update). */
int gp_append(hmd_gp* gp, const double* x, double y, double y_se);
/* mean[m], var[m] (latent posterior variance, output units^2). */
int gp_predict(hmd_gp* gp, const double* Xs, int m, double* mean, double* var);
/* Device-pointer form (Eqs. predMeanEq, predVarEq): dXs is m x d row-major in
 * device memory, dmean[m] and dvar[m] are device arrays; the kernels are
 * queued on `stream` (NULL: the context's stream) and the call returns
 * without waiting.  The GP's scratch is shared by its calls: calls on
 * different streams must not overlap. */
int gp_predict_dev(hmd_gp* gp, const double* dXs, int m, double* dmean, double* dvar, void* stream);
int gp_log_marginal(hmd_gp* gp, double* lml);
/* Hyperparameters that maximise Eq. evidenceEq (Sec. 2.3: the paper's
 * sigma_f and l; App. B: l and sigma_n of the periodic kernel): mask bit 0
 * sigma_f, bit 1 ell, bit 2 sigma_n (uniform noise only; it is then held
 * explicitly, in output units).  The evidence may have several local
 * maxima: a grid of 17 points per chosen parameter, a quarter decade apart
 * over two decades either side of the current values, picks the start of
 * cyclic golden-section searches over the logarithm of each chosen
 * parameter (bracket: a factor 10 either side of the current value), every
 * evaluation a refit on the device, until a cycle gains less than 1e-12
 * relative.  Cost: 17^m refits for m chosen parameters, then the search.  The GP is left fitted at the optimum;
 * *lml (nullable) receives the maximum.  Later appends keep the optimised
 * values. */
int gp_optimize(hmd_gp* gp, int mask, double* lml);
/* The hyperparameters in use (after gp_optimize, the optimised ones). */
int gp_hyper_get(const hmd_gp* gp, hmd_gp_hyper* hyper);
/* The database inputs (n x d row-major into X, nullable) and *n, *d. */
int gp_inputs(const hmd_gp* gp, double* X, int* n, int* d);
/* The database outputs and their standard errors as given to gp_fit and
 * gp_append (n doubles each, nullable): with gp_inputs, a copy of the
 * database, e.g. to start another march from it (Sec. 3.4). */
int gp_outputs(const hmd_gp* gp, double* y, double* y_se);
int gp_size(const hmd_gp* gp);
/* The normalisation in use: per-input denominators of Eq. d2Eq (d values),
 * the output scale and sigma_n in scaled units (each nullable). */
int gp_scales(const hmd_gp* gp, double* scale, double* s_q, double* sigma_n);
void gp_free(hmd_gp* gp);

/* ------------------------------------------------------------------------
 * MLP deep ensemble (a learned surrogate beside the GP; not in the paper):
 * `members` nets of 2 -> hidden -> hidden -> 1 with tanh (hidden <= 64),
 * FP32 weights and accumulation, trained full-batch on the mean squared
 * error with Adam (beta 0.9/0.999, eps 1e-8) by the library's own
 * forward/backward kernels.  Inputs are standardised by the training mean
 * and standard deviation, outputs divided by their RMS; weights start
 * Glorot-uniform from Philox4x32-10 (key = seed, counter (p div 4, member,
 * 2, 0), word p mod 4 for flat parameter p), biases at zero.  Flat parameter
 * order: W1[hidden x 2], b1, W2[hidden x hidden], b2, W3[1 x hidden], b3.
 * X is row-major n x 2.
 * ------------------------------------------------------------------------ */
/* bootstrap 1: member k trains on a resample of the n points drawn with
 * replacement (draw j is point (r n) >> 32 for the Philox4x32-10 word r of
 * counter (j div 4, k, 3, 0), word j mod 4, key = seed): its loss weights
 * each squared residual by the point's count; standardisation uses the
 * whole set.  0: every member trains on the whole set. */
typedef struct { int members, hidden, iters; double lr; uint64_t seed; int bootstrap; } hmd_ens_cfg;

void hmd_ens_cfg_default(hmd_ens_cfg* c);
int ens_fit(hmd_ctx* ctx, const double* X, const double* y, int n, const hmd_ens_cfg* cfg, hmd_ens** out);
/* mean[m], std[m] (sample standard deviation over members). */
int ens_predict(hmd_ens* e, const double* Xs, int m, double* mean, double* std);
/* Device-pointer form: dXs is m x 2 row-major in device memory, dmean[m] and
 * dstd[m] device arrays; queued on `stream` (NULL: the context's stream)
 * without waiting.  Scratch is shared by the ensemble's calls, as for
 * gp_predict_dev. */
int ens_predict_dev(hmd_ens* e, const double* dXs, int m, double* dmean, double* dstd, void* stream);
/* Final training loss per member (MSE on scaled outputs), members values. */
int ens_loss(const hmd_ens* e, double* loss);
/* Gradients of the MSE loss of member `k` for its initial parameters
 * (test hook): grad receives the flattened parameter gradient. */
int ens_grad_init(hmd_ctx* ctx, const double* X, const double* y, int n, const hmd_ens_cfg* cfg,
                  int member, double* params, double* grad, int* n_params);
int ens_members(const hmd_ens* e);
/* Online learning: add one training point (kept on the host), and retrain
 * every member from its initial weights on the whole training set. */
int ens_append(hmd_ens* e, const double* x, double y);
int ens_refit(hmd_ens* e);
int ens_size(const hmd_ens* e);
void ens_free(hmd_ens* e);

/* ------------------------------------------------------------------------
 * Hybrid macro solve (Alg. 1).  Sections i = 0..n-1 at s_i = (i + 1/2) ds,
 * ds = L / n, of a channel h(s) = h0 (1 + amp cos(2 pi s / L)).  Per macro
 * step (t = step count):
 *   p_i = p_out + c2 (rho_i - rho_ref)            (linear equation of state)
 *   dp/ds_i = (p_{i+1} - p_{i-1}) / (2 ds), ghosts p_{-1} = p_in(t),
 *             p_n = p_out, p_in(t) = p_out + dp_mean (1 + dp_amp sin(2 pi t / period))
 *   g_i = -(1/rho_i) dp/ds_i                      (Eq. momentumEq, F_ext = 0)
 *   with mirror on, the query is (h_i, |g_i|) and the answer takes the sign
 *   of g_i: the channel and its walls are symmetric under s -> -s, so the
 *   flux is odd in the body force, q(h, -g) = -q(h, g), and every surrogate
 *   point and MD run stays at g >= 0
 *   surrogate mean and standard deviation at (h_i, g_i); the section falls
 *   back to the micro-solver when std > max(tau_rel |mean|, tau_abs)
 *   (tau_abs alone is the paper's absolute sigma_t); fallback results join
 *   the surrogate's database (the GP refits at once, the ensemble every
 *   refit_every new points); every audit_every-th surrogate answer is also
 *   run and counted as passing when |mean - q_MD| <= 2 SE_MD
 *   rho_i h_i -= dt_macro (q_{i+1/2} - q_{i-1/2}) / ds  (Eq. continuityEq per
 *   unit span; faces average the neighbours, boundary faces carry the
 *   boundary section's flux)
 * All sections that fall back in one step run as one MD batch.  The MD
 * protocol is the context's parameters (box, n_equil) with md_sample
 * sampling steps; seeds count up from `seed`.
 * ------------------------------------------------------------------------ */
typedef struct {
    int n_sections;
    double h0, amp, L, dt_macro, rho_ref, p_out, dp_mean, dp_amp, period, c2;
    double tau_rel, tau_abs;
    int surrogate;     /* 0: GP, 1: MLP ensemble */
    int audit_every;   /* every k-th surrogate answer is re-run with MD (0: off) */
    int64_t md_sample; /* sampling steps of each fallback MD run */
    int refit_every;   /* ensemble: retrain after this many new MD points */
    uint64_t seed;     /* first MD seed */
    int mirror;        /* 1: use q(h, -g) = -q(h, g) (default), 0: query g as it is */
    int audit_batch;   /* audits wait until this many are pending, then run as one
                          MD batch (0: in the step that drew them) */
    /* Warm starts (Alg. 1 "find nearest prior input", "pseudoMD"; Sec. 2.4):
     * with warm_start on, a fallback run starts from the final state of the
     * earlier fallback run of the same height (equal within a relative 1e-9)
     * whose input has the largest covariance with the new one, i.e. the
     * smallest squared distance (dh^2 + dg^2, ties to the earliest), else
     * from the lattice; its
     * equilibration is the start-up time of the 1-D channel flow with Navier
     * slip (viscosity pseudo_nu, slip length pseudo_slip) from the prior's
     * body force (0 from the lattice) to the new one, until the flow rate is
     * within pseudo_tol of its new steady value (relative to the larger of
     * the two steady flow rates), in steps, at least n_min_warm
     * (n_min_cold from the lattice).  The runs of one step share a batch and
     * step together, so the batch equilibrates for the longest of them.
     * Audits always start from the lattice with params.n_equil. */
    int warm_start;
    double pseudo_nu, pseudo_slip, pseudo_tol;
    int64_t n_min_warm, n_min_cold;
    /* geometry 1: the paper's benchmark channel (Sec. 2.1), periodic in s
     * (the first section at inlet and outlet), sections at s_i = i L / n
     * (Eq. subsEq, 0-based), h = amp h0 (cos(2 pi s / L) - 1) + h0 (Eq.
     * heightEq: h_1 = h0, a = amp h0), driven by the uniform external force
     * per unit mass f_amp sin(2 pi t / f_period) (Eq. extForcing1, t in macro
     * steps); pressure gradient and face fluxes wrap around, and p_out,
     * dp_mean, dp_amp and period are unused.  geometry 0: the channel above. */
    int geometry;
    double f_amp, f_period;
    /* eos 1: the paper's full input set (Sec. 2.2; Alg. 1 with both GPs).
     * The section pressure is the mean of a pressure GP p(h, rho) (attached
     * with hybrid_set_pressure_gp, built from pre-simulations: md_flux_batch
     * with params.pressure on, g = 0, over a density sweep per height)
     * instead of the linear law; the flux GP takes three inputs (h, rho, |g|);
     * every fallback runs at its section's density and also returns the
     * wall pressure, which joins the pressure GP when that (h, rho) is not in
     * it yet (an entry within a relative 1e-9 in both inputs counts as
     * present).  The boundary pressures p_out and p_in(t) are then absolute.
     * Needs surrogate 0 and no warm starts.  eos 0: the linear law. */
    int eos;
} hmd_hybrid_cfg;
typedef struct {
    int64_t steps, md_calls, audited, audit_pass, queries, md_failed;
    double wall_s, md_wall_s, md_atom_steps, surrogate_wall_s;
    /* audits run apart from the fallback batch: their time and atom-steps
     * (included in wall_s, excluded from md_wall_s and md_atom_steps) */
    double audit_wall_s, audit_atom_steps;
    /* fallback runs: equilibration atom-steps run, warm starts, and the
     * atom-steps the same runs would have taken from the lattice with
     * params.n_equil */
    double md_equil_atom_steps;
    int64_t warm_starts;
    double md_atom_steps_cold;
    /* audits that also pass when the surrogate's own predicted standard
     * deviation is counted: |mean - q_MD| <= 2 sqrt(std^2 + SE_MD^2) */
    int64_t audit_pass_cal;
    /* eos 1: fallback pressures appended to the pressure GP */
    int64_t p_appends;
} hmd_hybrid_stats;

/* A replacement micro-solver: given n (h, g) pairs, write the mean flux and
 * its standard error; return 0 on success.  Used instead of batched MD when
 * set (coupling another solver, or a known law in tests). */
typedef int (*hmd_micro_fn)(void* user, int n, const double* h, const double* g, double* q, double* se);
/* The same for eos 1: inputs (h, rho, g), outputs flux, its SE, wall
 * pressure and its SE. */
typedef int (*hmd_micro_p_fn)(void* user, int n, const double* h, const double* rho, const double* g, double* q,
                              double* se, double* p, double* p_se);

void hmd_hybrid_cfg_default(hmd_hybrid_cfg* c);
/* Runs the audits still pending (audit_batch > 0) and returns the stats. */
int hybrid_flush_audits(hmd_hybrid* hy, hmd_hybrid_stats* out);
/* Exactly one of gp / ens matches cfg->surrogate; the hybrid borrows it
 * (the caller frees it after hybrid_free).  rho starts at rho_ref. */
int hybrid_create(hmd_ctx* ctx, const hmd_hybrid_cfg* cfg, hmd_gp* gp, hmd_ens* ens, hmd_hybrid** out);
int hybrid_set_micro(hmd_hybrid* hy, hmd_micro_fn fn, void* user);
int hybrid_set_micro_p(hmd_hybrid* hy, hmd_micro_p_fn fn, void* user);
/* eos 1: the pressure GP over (h, rho) (2 inputs), borrowed like the flux
 * GP; its current inputs count as present for the append rule. */
int hybrid_set_pressure_gp(hmd_hybrid* hy, hmd_gp* pgp);
/* eos 1: the section pressures of the last step and their GP standard
 * deviations (n_sections doubles each, nullable); eos 0: the linear law. */
int hybrid_get_pressure(hmd_hybrid* hy, double* p, double* p_std);
/* Forcing variants of Sec. 3.4 (the variable-frequency and
 * variable-amplitude cases): on the periodic channel (geometry 1), macro
 * step k takes F_ext / m = f[k] in place of Eq. extForcing1's sinusoid.
 * f is n host doubles, copied; n = 0 restores the sinusoid.  EINVAL for
 * geometry 0, a non-finite entry, or (from hybrid_step) a step at or past
 * the end of the table. */
int hybrid_set_forcing(hmd_hybrid* hy, const double* f, int64_t n);
/* Overwrite the density of every section (n_sections doubles). */
int hybrid_set_rho(hmd_hybrid* hy, const double* rho);
/* The fallback plan of the last macro step, per section (each nullable):
 * prior[i] = index (in order of recording) of the earlier fallback run it
 * starts from, -1 from the lattice, -2 when the section did not fall back;
 * n_equil[i] its start-up in steps (0 when it did not fall back);
 * *batch_equil the equilibration of the step's batch.  Every fallback run
 * that converged is recorded, also under a replacement micro-solver, where
 * the plan is computed the same way but no state is stored or used. */
int hybrid_last_plan(hmd_hybrid* hy, int* prior, int64_t* n_equil, int64_t* batch_equil);
/* One macro step; out (nullable) receives the cumulative statistics. */
int hybrid_step(hmd_hybrid* hy, hmd_hybrid_stats* out);
/* rho, q, q_std, g (n_sections doubles), from_md (n_sections bytes); each
 * nullable. */
int hybrid_get(hmd_hybrid* hy, double* rho, double* q, double* q_std, double* g, uint8_t* from_md);
void hybrid_free(hmd_hybrid* hy);

#ifdef __cplusplus
}
#endif
#endif /* HMD_H */
