/*
 * tpx.h — C-ABI of the MI355X (gfx950) library for ultra-low-memory FWI
 * gradients with randomized trace estimation (Louboutin & Herrmann,
 * "Ultra-low memory seismic inversion with randomized trace estimation").
 *
 * The library computes, on one GPU, the objective of Eq. (2)
 *     J(m) = 1/2 || F(m; q) - d_obs ||_2^2
 * for the isotropic acoustic wave equation  m u_tt - Lap u = q
 * (m = squared slowness), its exact adjoint-state gradient (Eq. 3) and the
 * probed approximation of Eq. (4) / Algorithm 1, in which the time axis of the
 * forward and adjoint wavefields is compressed on the fly by r probing vectors
 * so that only N x r values per pass are kept instead of N x n_t.
 *
 * Discretisation (the paper names none; these are this library's readings):
 *   - second order in time (leapfrog), 4th or 8th order centred Laplacian;
 *   - nbl absorbing nodes added on every face, with the damped equation
 *     m u_tt + m d u_t - Lap u = q, d = dmax * (distance into layer / nbl)^2,
 *     dmax = 3 damp_vmax / (2 nbl h) ln(1/damp_R), u_t centred;
 *   - the model is padded by edge replication; fields vanish outside the box;
 *   - point sources and receivers use bilinear (2D) / trilinear (3D) weights;
 *   - u^{-1} = u^0 = 0; step k = 0..nt-2 injects q^k and yields u^{k+1};
 *     traces d^k = R u^k for k = 0..nt-1;
 *   - the adjoint is the discrete adjoint of that recurrence:
 *     lambda^{nt} = lambda^{nt-1} = 0; step k = nt-1..1 injects
 *     R^T dd^k / dt^2 and yields lambda^{k-1};
 *   - exact gradient, cropped to the physical grid:
 *     g = - sum_{s=1}^{nt-1} u^s * (lambda^{s-1} - 2 lambda^s + lambda^{s+1});
 *   - probed gradient: ubar_j = sum_s Z[s,j] u^s,
 *     vbar_j = sum_s Z[s,j] (lambda^{s-1} - 2 lambda^s + lambda^{s+1}),
 *     g~ = -c sum_shots sum_j ubar_j * vbar_j  (c = 1/r for random probes,
 *     1 for the identity, `scale` for an explicit Z).
 *
 * Units: m (lengths), ms (time), km/s = m/ms (velocity), kHz; m in ms^2/m^2.
 * Layouts (C order, x fastest): models and gradients [z][y][x] over the
 * physical grid (2D: [z][x]); traces [shot][t][rec]; wavelets [shot][t];
 * probing matrices [shot][t][r].
 *
 * Memory and streams: every device buffer, including the workspace, is
 * allocated and owned by the caller; the library never allocates device
 * memory.  Each call validates its arguments on the host before any launch,
 * then enqueues its work on `stream` (a hipStream_t passed as void*, NULL =
 * the null stream) and returns; outputs are valid once the stream reaches the
 * end of the call.  A call stages its geometry tables in pinned host memory
 * owned by the library and uploads them into the workspace asynchronously, on
 * the same stream; it never waits for the stream.
 * Two calls may run concurrently on different streams if their workspaces
 * and outputs do not overlap.  A call may be captured into a HIP graph (stream
 * capture in relaxed mode; the contraction overlap option off): the tables it
 * uploads during capture get pinned host copies that the library keeps for
 * the life of the process, so every replay reads them.  No C++ exception
 * crosses this boundary.
 */
#ifndef TPX_H
#define TPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TPX_OK = 0,
    TPX_E_INVAL = 1,   /* bad sizes, null pointers, unsupported order or kind     */
    TPX_E_CFL = 2,     /* dt above the leapfrog stability limit for damp_vmax      */
    TPX_E_GEOM = 3,    /* a source or receiver lies outside [0, (n-1) h]           */
    TPX_E_NOMEM = 4,   /* workspace / state smaller than required                  */
    TPX_E_DEVICE = 5,  /* a HIP runtime error (message in tpx_last_error)          */
    TPX_E_NUMERIC = 6, /* a non-finite or non-positive model value was found       */
    TPX_E_STATE = 7    /* state buffer does not match the problem it is used with  */
} tpx_status;

/* Message of the last non-OK status returned on the calling thread. */
const char *tpx_last_error(void);
const char *tpx_version(void);

/* Grid and time axis.  2D problems use axes x and z: ndim = 2, n[1] = 1. */
typedef struct {
    int32_t ndim;        /* 2 or 3 */
    int64_t n[3];        /* physical nodes along x, y, z (each >= 2 when active) */
    double h;            /* grid spacing, m */
    int32_t nbl;         /* absorbing-layer width in nodes, >= 0 */
    int32_t space_order; /* 4 or 8 */
    double dt;           /* ms */
    int32_t nt;          /* time samples, >= 2 */
    double damp_vmax;    /* km/s: damping profile, and the CFL check */
    double damp_R;       /* reflection coefficient of the layer, in (0, 1] */
} tpx_grid;

/* Acquisition.  Positions are HOST arrays (read during the call only);
 * the wavelet is a DEVICE array. */
typedef struct {
    int32_t nshots;         /* S >= 1: shots are batched in one launch */
    int32_t nrec;           /* receivers per shot, >= 0 */
    const double *src_pos;  /* host [S][3] (x, y, z) in m */
    const double *rec_pos;  /* host [S][nrec][3] */
    const float *wavelet;   /* device [S][nt], q^k */
} tpx_geom;

typedef enum {
    TPX_PROBE_RADEMACHER = 0, /* random +-1 (Randomized trace estimation) */
    TPX_PROBE_GAUSS_B64 = 1,  /* "Gaussian": (popcount(w) - 32) / 4, unit variance */
    TPX_PROBE_IDENTITY = 2,   /* Z = I, requires r == nt: exact gradient */
    TPX_PROBE_EXPLICIT = 3,   /* caller-provided Z (e.g. an orthonormal basis) */
    TPX_PROBE_RANGE_FINDER = 4 /* Q = qr(D_obs D_obs^T Z) per shot, Z Rademacher
                                  (Choice of the probing matrix Q, Eq. 6):
                                  orthonormal, c = 1.  Needs the observed data,
                                  so gradient calls and jobs only (the split
                                  forward/backward pair takes it as EXPLICIT
                                  from tpx_range_finder_probes); 1 <= r <=
                                  min(64, nrec, nt). */
} tpx_probe_kind;

/* Probing (Eq. 1, Eq. 4).  Random entries are Philox4x64-10 (Salmon et al.,
 * SC'11) at counter (t+1, j, shot, 0), key (seed, 0), first output word w:
 * Rademacher 1 - 2 (w >> 63); Gauss-B64 (popcount(w) - 32) / 4. */
typedef struct {
    int32_t kind;      /* tpx_probe_kind */
    int32_t r;         /* number of probing vectors, >= 1 */
    uint64_t seed;
    const float *Z;    /* EXPLICIT only: device [S][nt][r] */
    double scale;      /* EXPLICIT only: the factor c of the imaging condition */
    int32_t block;     /* time steps per probe contraction; 0 = library default */
    int32_t keep_vbar; /* 0: fold the adjoint accumulation into the gradient
                          (no vbar array); 1: accumulate vbar, then image */
    int32_t dtt_side;  /* which pass probes the second time difference:
                          0: ubar_j = sum_s Z[s,j] u^s (s = 1..nt-1) and
                             vbar_j = sum_s Z[s,j] (lam^{s-1} - 2 lam^s + lam^{s+1});
                          1 (Algorithm 1 as printed): ubar_j = sum_k Z[k,j]
                             (u^{k+1} - 2 u^k + u^{k-1}) and vbar_j = sum_k Z[k,j]
                             lam^k (k = 0..nt-2).  Both are unbiased estimators of
                             the gradient of Eq. 3 and equal it for Z = I. */
    int32_t imaging;   /* imaging condition applied to the probed fields:
                          0: pointwise product, g = -c sum_j ubar_j vbar_j (Eq. 4);
                          1: space-only linear operator D = grad applied to the
                             probed fields (Eq. 5), g = -c sum_j grad ubar_j .
                             grad vbar_j with centred differences, 0 on the
                             outermost physical nodes; needs keep_vbar = 1. */
} tpx_probe;

/* Call identifiers for tpx_workspace_bytes. */
enum {
    TPX_CALL_FORWARD = 0,
    TPX_CALL_ADJOINT = 1,
    TPX_CALL_GRADIENT_PROBED = 2,
    TPX_CALL_GRADIENT_FULL = 3,
    TPX_CALL_FORWARD_PROBED = 4,
    TPX_CALL_BACKWARD_PROBED = 5,
    TPX_CALL_RANGE_FINDER = 6,
    TPX_CALL_OBJECTIVE = 7
};

/* Device workspace (bytes) that `call` needs for this problem; 0 on invalid
 * arguments (see tpx_last_error).  `probe` may be NULL for calls without
 * probing.  Full-history storage (TPX_CALL_GRADIENT_FULL) grows with nt. */
size_t tpx_workspace_bytes(int32_t call, const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe);

/* Bytes of the state that tpx_forward_probed hands to tpx_backward_probed:
 * the probed forward wavefield ubar, S x r x N_phys floats, followed by a
 * 256-byte header naming the problem and probe set it was computed for. */
size_t tpx_state_bytes(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe);

/* Forward modelling F(m; q), Eq. (2):  d[S][nt][nrec] (device). */
tpx_status tpx_forward(const tpx_grid *grid, const tpx_geom *geom, const float *m, float *d,
                       void *ws, size_t ws_bytes, void *stream);

/* Objective of Eq. (2) at m: forward modelling, then J = 1/2 ||F(m; q) - d_obs||^2
 * summed over every trace sample (FP64 partial sums in a fixed order, so the
 * value is run-to-run identical).  J is one device double; d_out (device
 * [S][nt][nrec], may be NULL) receives F(m; q).  This is the function value
 * that a line search along a model update needs, without back-propagation. */
tpx_status tpx_objective(const tpx_grid *grid, const tpx_geom *geom, const float *m, const float *d_obs,
                         double *J, float *d_out, void *ws, size_t ws_bytes, void *stream);

/* Adjoint of the source-to-trace map: q_adj[S][nt] = F^T d_in (device),
 * q_adj^k = dt^2 S lambda^k.  <F q, d> = <q, F^T d> to rounding. */
tpx_status tpx_adjoint(const tpx_grid *grid, const tpx_geom *geom, const float *m, const float *d_in,
                       float *q_adj, void *ws, size_t ws_bytes, void *stream);

/* Probed gradient (Eq. 4, Algorithm 1): forward with on-the-fly probing,
 * residual and objective, adjoint with on-the-fly probing, imaging.
 * g (device, physical grid) is overwritten; J (device double) receives the
 * objective; d_out (device [S][nt][nrec], may be NULL) receives F(m; q). */
tpx_status tpx_gradient_probed(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe,
                               const float *m, const float *d_obs, float *g, double *J, float *d_out,
                               void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the probed
 * gradient of tpx_gradient_probed, with the same arguments and results, but
 * no workspace argument.  Its workspace is a static device array of the
 * library, TPX_NOALLOC_SCRATCH_BYTES (64 MiB) on each GPU, held until the
 * process ends; the call neither allocates nor frees memory.  Problems whose
 * probed workspace exceeds that size (tpx_workspace_bytes with
 * TPX_CALL_GRADIENT_PROBED and the contraction-overlap option off) return
 * TPX_E_NOMEM before any launch.  The geometry tables are copied from pageable
 * host memory and the call waits for that copy (hipStreamSynchronize on
 * `stream`), so, unlike the other calls, it does wait for the stream once;
 * contractions always run in stream order.  Every call on one GPU shares that
 * GPU's array and leaves its contents behind (each call initialises what it
 * reads): calls that overlap in time on one GPU race and give wrong results,
 * so serialise them (one stream, or one call at a time). */
#define TPX_NOALLOC_SCRATCH_BYTES (64u << 20)
tpx_status tpx_gradient_probed_noalloc(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe,
                                       const float *m, const float *d_obs, float *g, double *J, float *d_out,
                                       void *stream);

/* Exact gradient (Eq. 3) from the stored forward history (N x nt values):
 * the conventional reference path.  Returns TPX_E_NOMEM when the history does
 * not fit the workspace. */
tpx_status tpx_gradient_full(const tpx_grid *grid, const tpx_geom *geom, const float *m, const float *d_obs,
                             float *g, double *J, float *d_out, void *ws, size_t ws_bytes, void *stream);

/* Split form for differentiation: the forward pass with probing writes the
 * traces d and the probed wavefield ubar into `state`; the backward pass
 * back-propagates grad_d (the gradient of a loss with respect to d) and images
 * with the stored ubar.  g = (dd/dm)^T grad_d in the probed approximation. */
tpx_status tpx_forward_probed(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe,
                              const float *m, float *d, void *state, size_t state_bytes,
                              void *ws, size_t ws_bytes, void *stream);
tpx_status tpx_backward_probed(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe,
                               const float *m, const float *grad_d, const void *state, size_t state_bytes,
                               float *g, void *ws, size_t ws_bytes, void *stream);

/* Resumable probed-gradient job, for servers that interleave several
 * gradients on one GPU.  tpx_job_create validates, uploads the geometry tables
 * and enqueues the set-up work on `stream`; each tpx_job_advance enqueues at
 * most `max_steps` further time steps (plus the probe contractions, residual
 * and imaging that fall due) and sets *finished once everything is enqueued.
 * The outputs g, J (and d_out) are valid when the stream has executed the last
 * advance.  m, d_obs, g, J, d_out and ws must stay allocated until then, and
 * successive calls of one job must be ordered on the device (the same stream,
 * or streams joined by events).  Jobs with separate workspaces are
 * independent: a job's results do not depend on what runs beside it. */
typedef struct tpx_job tpx_job;
tpx_status tpx_job_create(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe, const float *m,
                          const float *d_obs, float *g, double *J, float *d_out, void *ws, size_t ws_bytes,
                          void *stream, tpx_job **job);
tpx_status tpx_job_advance(tpx_job *job, int32_t max_steps, void *stream, int32_t *finished);
tpx_status tpx_job_progress(const tpx_job *job, int64_t *steps_done, int64_t *steps_total);
void tpx_job_destroy(tpx_job *job);

/* Library-wide options.  TPX_OPT_OVERLAP_CONTRACTIONS (default 0): each
 * time block's probe contraction runs on an auxiliary HIP stream owned by the
 * library, concurrently with the next block of time steps, and is joined back
 * into the caller's stream before the pass ends (the ring then holds 2b + 3
 * instead of b + 2 slots).  The option changes workspace sizes: set it before
 * sizing a workspace, not between sizing and use. */
enum { TPX_OPT_OVERLAP_CONTRACTIONS = 1, TPX_OPT_MATRIX_CORES = 2, TPX_OPT_FUSED_STEPS_3D = 3, TPX_OPT_STEPS_2D = 4 };
/* TPX_OPT_FUSED_STEPS_3D (default 0): 3D launches advance two leapfrog steps
 * at a time (as 2D launches always do) instead of one.  Results are bitwise
 * the same either way; only speed differs. */
/* TPX_OPT_STEPS_2D (default 3): the most leapfrog steps one 2D launch
 * advances, 3 or 2.  Three-step launches (temporal blocking over three levels:
 * u^{k-1}, u^k and beta read once, three new levels written) need their own
 * injection tables and a plain forward/adjoint ring of six levels instead of
 * four, so the option changes workspace sizes: set it before sizing a
 * workspace.  Results are bitwise the same for any setting. */
/* TPX_OPT_MATRIX_CORES (default 1): the probe contractions of the time
 * blocks are dense products (r x b by b x points) and can run on the matrix
 * cores when r is a multiple of 16: bfloat16 MFMA with each FP32 field value
 * split exactly into three bfloat16 parts and FP32 accumulation.  Probes exact
 * in bfloat16 (Rademacher, GAUSS_B64, identity) take three products per tile;
 * other probes (explicit, range finder) are split in three as well and take
 * six, the dropped terms below 2^-21 of each product.  Value 0: never; 1: the
 * folded adjoint contraction when r >= 32 and the ubar/vbar accumulations
 * when r >= 64 (where they measured faster than the vector units); 2: every
 * contraction.  Explicit probes must be 16-byte aligned to qualify, and a
 * ring slot (one level of all shots) must hold fewer than 2^32 floats.  Results
 * agree with the FP32 path to rounding (not bitwise).  Workspace sizes do
 * not depend on this option. */
tpx_status tpx_set_option(int32_t option, int64_t value);
int64_t tpx_get_option(int32_t option);

/* Device-side checks of the last call that used `ws`, after waiting for
 * `stream`: TPX_E_NUMERIC if the model held a non-finite or non-positive
 * value, TPX_E_CFL if it held a velocity above damp_vmax, TPX_E_STATE if
 * tpx_backward_probed was given a state that a forward pass of another
 * problem or probe set (kind, r, seed, side, explicit Z, grid, shots, nt)
 * wrote.  The backward pass itself runs regardless; its result is then
 * meaningless. */
tpx_status tpx_check_workspace(const void *ws, void *stream);

/* Kernel timing for measurement: while enabled, each run of consecutive
 * launches of one kernel kind on one stream is bracketed by a pair of HIP
 * events on that stream (no events between the kernels of a run).  Enabling
 * clears earlier records; tpx_profile_read waits for the recorded events and
 * returns the summed duration and the launch count of one kernel kind. */
enum {
    TPX_KERNEL_STEP = 0,      /* one leapfrog step with fused injection/sampling  */
    TPX_KERNEL_ACCUM_FWD = 1, /* forward probe contraction                        */
    TPX_KERNEL_ACCUM_ADJ = 2, /* adjoint probe contraction (or fold)              */
    TPX_KERNEL_ACCUM_FULL = 3,/* full-history imaging term                        */
    TPX_KERNEL_STEP2 = 4,     /* two fused leapfrog steps in one launch           */
    TPX_KERNEL_STEP3 = 5      /* three fused leapfrog steps in one launch (2D)    */
};
void tpx_profile_enable(int32_t on);
tpx_status tpx_profile_read(int32_t kind, double *total_ms, int64_t *launches);

/* Probes from the range of the data covariance (Choice of the probing
 * matrix Q, Eq. 6): for every shot, D = d_obs[shot] as an nt x nrec matrix,
 * Z = the shot's Rademacher probes (probe->seed), Q[shot] = the orthonormal
 * factor of the reduced QR of D D^T Z, computed in FP64 and stored as float
 * Q[S][nt][r] (device).  Use it as EXPLICIT probes with scale 1.  Only
 * grid->nt, geom->nshots and geom->nrec are used of the problem; the
 * workspace is tpx_workspace_bytes(TPX_CALL_RANGE_FINDER, ...).
 * probe->kind must be TPX_PROBE_RANGE_FINDER; E_INVAL unless
 * 1 <= r <= min(64, nrec, nt). */
tpx_status tpx_range_finder_probes(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe,
                                   const float *d_obs, float *Q, void *ws, size_t ws_bytes, void *stream);

/* Probing matrix of one shot as the GPU generates it: Z[nt][r] (device). */
tpx_status tpx_probe_matrix(const tpx_probe *probe, int32_t nt, int32_t shot, float *Z, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TPX_H */
