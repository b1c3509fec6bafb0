/*
 * etpic -- C ABI of the envelope-tracking particle-mesh step on AMD MI355X.
 *
 * The step is the data-parallel particle part of the envelope-tracking
 * EM-FEMPIC method (Ramachandran, Crawford, O'Connor, Luginsland, Shanker):
 *   gather  : fields at each particle from the Whitney edge (E) and face (B)
 *             expansions (Formulation, "Discretization in Space and Time"),
 *             whose complex envelope DoFs are modulated by the carrier
 *             e^{j w t} and taken as the real part (Particle Push section,
 *             the Lorentz update with the fast carrier treated analytically);
 *   push    : a Lorentz update at the fine step (the "simpler" scheme of the
 *             Particle Push section), here the Boris rotation, with a
 *             tet-to-tet walk of the straight path;
 *   deposit : the edge DoFs of G, the time integral of the current, which is
 *             q times the path integral of the trajectory (eq. g_def; edge
 *             DoFs g_l = <W1_l, G>; the trajectory summed over fine steps,
 *             eq. G_integral and the sum that follows it).
 *
 * Conventions (all arrays are plain pointers):
 *  - tet rows list vertex ids in ascending order; barycentrics lam1..lam3 refer
 *    to local vertices 1..3 of that order and lam0 = 1 - lam1 - lam2 - lam3;
 *  - local edges (0,1),(0,2),(0,3),(1,2),(1,3),(2,3); local face k is opposite
 *    local vertex k;
 *  - edges are (a<b) pairs numbered lexicographically and oriented a->b; faces
 *    are (a<b<c) triples numbered lexicographically, oriented by
 *    (r_b - r_a) x (r_c - r_a);
 *  - complex DoFs are interleaved (re, im) float64 pairs (complex128 layout);
 *  - the physical fields are Re{env * e^{j w t}} + dc with t = step*dt.
 *
 * Ownership: every device buffer is the caller's.  The library allocates no
 * device memory; what it keeps on the device lives in buffers the caller
 * allocates (e.g. torch tensors) and hands in after a size query:
 *   context workspace   etpic_workspace_bytes  -> etpic_workspace_bind
 *   mesh tables         etpic_mesh_sizes       -> etpic_mesh_upload
 *   field-step solver   etpic_field_bytes      -> etpic_field_setup
 *   Gauss-law solver    etpic_ns_bytes         -> etpic_ns_setup
 *   downshifted rows    etpic_ds_rows_bytes    -> etpic_ds_rows_bind
 *   projector object    etpic_qh_bytes         -> etpic_qh_bind
 * Each buffer must be 256-byte aligned, at least the queried size, and stay
 * valid (not freed, not written by the caller) while the object that was
 * given it is in use: until the next bind/upload/setup of the same kind, a
 * new mesh upload (which drops the mesh-derived ones: field, Gauss-law and
 * downshifted buffers must then be given again), or destruction.  Particle
 * arrays, field DoFs, outputs, the adjoint workspace and the downshifted
 * history are caller-owned too and must stay valid until the work queued on
 * `stream` has finished.  Host resources taken by etpic_create: one pinned
 * 8-byte word (the sort's run-length statistic is read into it without
 * blocking) and a fixed pool of HIP events for ETPIC_STEP_TIMING; none
 * afterwards.
 *
 * Errors: every entry point returns an etpic status (0 = OK).  On failure the
 * message is available from etpic_last_error() (thread-local).  Errors found
 * inside kernels (walk hop cap, NaN) set bits in a device status word that
 * etpic_check() reads.  No C++ exception crosses this boundary.  A context is
 * not thread-safe: use one context per host thread, and order the calls made
 * on one context (same stream, or synchronise between streams): its step
 * calls share a small device work queue.
 * `stream` is a hipStream_t passed as void* (NULL = default stream).
 */
#ifndef ETPIC_H
#define ETPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum etpic_status {
    ETPIC_OK = 0,
    ETPIC_EINVAL = -1,    /* bad argument (null pointer, size, precision) */
    ETPIC_ESTATE = -2,    /* no mesh uploaded yet */
    ETPIC_EHIP = -3,      /* HIP runtime error; message carries hipGetErrorString */
    ETPIC_EMESH = -4,     /* unsorted row, degenerate tet or non-manifold face */
    ETPIC_EPARTICLE = -5, /* particle tet index out of range */
    ETPIC_EWALK = -6,     /* a particle exceeded the walk hop cap */
    ETPIC_ENAN = -7,      /* non-finite value met in a kernel */
    ETPIC_ENOCONV = -8,   /* iterative solve did not converge */
    ETPIC_EIO = -9        /* checkpoint file missing, unreadable, corrupt or not writable */
};

enum etpic_precision {
    ETPIC_FP64 = 0,  /* gather, push and deposit in float64; velocities float64 */
    ETPIC_MIXED = 1, /* gather and push in float32 on tet-local barycentrics,
                        velocities float32; positions, deposit and charge float64 */
    ETPIC_MIXED_FIXED = 2 /* ETPIC_MIXED with the barycentrics stored as uint32
                        fixed point (lam = u * 2^-32; the lam[k] arrays hold
                        uint32): 56 B per particle-step instead of 80.  Each
                        step's end point is rounded to that grid (lam_0 =
                        1 - sum stays >= 0) and the step's piece is deposited
                        up to the rounded point, so the stored end points and
                        the deposit agree exactly (continuity to float64
                        rounding); the position quantum is 2^-32 of the tet
                        size.  The particle steps (etpic_gather_push_deposit,
                        etpic_run_steps, etpic_sort_run_steps,
                        etpic_coarse_step), etpic_sort, etpic_vertex_charge,
                        etpic_particles_locate / _positions and
                        etpic_stream_probe take it; the downshifted, Gauss-law
                        loop and electromagnetic loop entry points return
                        EINVAL for it */
};

/* bits of the device status word read by etpic_check */
enum etpic_device_flags {
    ETPIC_DEV_HOPCAP = 1u, /* walk hop cap reached (particle left where it stopped) */
    ETPIC_DEV_NAN = 2u,    /* non-finite field or velocity */
    ETPIC_DEV_BADTET = 4u  /* tet index outside [0, N_t) */
};

/* flags of etpic_gather_push_deposit */
enum etpic_step_flags {
    ETPIC_STEP_XCD_REMAP = 1u, /* map consecutive particle blocks to one XCD (default on) */
    ETPIC_STEP_TIMING = 2u,    /* time the particle kernel of each step with HIP events (etpic_kernel_time) */
    /* slices of 64 particles per wavefront of the particle kernel; without one
     * of these the library picks 1, 4 or 16 from the last sort's (etpic_sort,
     * etpic_sort_run_steps, etpic_ds_sort) mean, over particles, of the number
     * of particles in the same tet (1 before any sort).  Longer slices cut
     * same-address atomics where thousands of particles share a tet. */
    ETPIC_STEP_SLICES_1 = 4u,
    ETPIC_STEP_SLICES_4 = 8u,
    ETPIC_STEP_SLICES_16 = 16u,
    /* two slices per wavefront, the second slice's particle state requested
     * before the first one's per-tet rows are read (the float32 forms; float64
     * and the sorting and charge-scattering forms run one slice instead).
     * Without a slice flag the library takes it for the float32 forms where
     * the sort left one slice and the mesh's float32 per-tet rows (160 B per
     * tet) exceed the 256 MB Infinity Cache. */
    ETPIC_STEP_SLICES_2 = 512u,
    /* queue the particles that leave their tet by 64-particle slice, the path
     * the library otherwise takes only when more than 2^23 particles leave
     * their tet in one step (exercises that path); in the sorting step of
     * etpic_sort_run_steps, whose overflow path is a scan of all particles,
     * take that scan instead */
    ETPIC_STEP_WALK_BY_SLICE = 32u,
    /* as ETPIC_STEP_TIMING, and also the coefficient, walk and edge-gather
     * kernels.  Each timed dispatch costs the stream a few microseconds of
     * idle time after it, so a throughput measurement times the particle
     * kernel only and takes this breakdown in a run of its own. */
    ETPIC_STEP_TIMING_ALL = 256u
    /* bit 31 is the library's own and is ignored in the flags passed in */
};

#define ETPIC_HOP_CAP 64

typedef struct etpic_ctx etpic_ctx;

/* Particle state, structure of arrays on the device, length n each (n <= 2^29).
 * lam[k]: float64 barycentric lam_{k+1} in the particle's tet (for
 *         ETPIC_MIXED_FIXED: uint32 fixed point, u = lam * 2^32, the pointer
 *         reinterpreted).
 * vel[k]: velocity component k at the half step (v^{n-1/2} in, v^{n+1/2} out);
 *         float64 for ETPIC_FP64, float32 for ETPIC_MIXED.
 * tet:    int32 tet index.  id: int64 particle id, carried by etpic_sort (may be NULL). */
typedef struct {
    int64_t n;
    double *lam[3];
    void *vel[3];
    int32_t *tet;
    int64_t *id;
} etpic_particles;

/* Field DoFs on the device.  e_env: 2*N_e float64 (complex edge envelope);
 * e_dc: N_e float64 or NULL (real unmodulated edge DoFs); b_env: 2*N_f float64
 * (complex face envelope); b_dc: N_f float64 or NULL (real unmodulated face DoFs). */
typedef struct {
    const double *e_env;
    const double *e_dc;
    const double *b_env;
    const double *b_dc;
} etpic_fields;

/* Species: charge q [C], mass m [kg], macroparticle weight w. */
typedef struct {
    double q, m, w;
} etpic_species;

/* Thread-local message of the last failing call ("" if none). */
const char *etpic_last_error(void);

/* Create a context bound to HIP device `device`.  *out receives the handle.
 * Takes no device memory: bind a workspace (below) before any other call that
 * launches work (ESTATE otherwise). */
int etpic_create(etpic_ctx **out, int device);

/* Destroy a context (its host resources; the device buffers it was given are
 * the caller's to free afterwards).  NULL is accepted. */
int etpic_destroy(etpic_ctx *ctx);

/* Bytes of the context workspace: the device status word, the reduction and
 * run-length words, the walk counters and the two queues of particles that
 * left their tet (2^23 entries each).  Host only. */
int etpic_workspace_bytes(size_t *bytes);

/* Give the context its workspace (device, 256-byte aligned, at least
 * etpic_workspace_bytes; zeroes what must start at zero, synchronously).
 * Rebinding replaces the previous one.  Errors: EINVAL (null, misaligned or
 * short buffer), EHIP. */
int etpic_workspace_bind(etpic_ctx *ctx, void *dev_buf, size_t bytes);

/* Host only (no context, no GPU): the mesh tables' device size.  Builds the
 * canonical numbering as etpic_mesh_upload does (Appendix A: the sets N, E,
 * F, T); counts_out[4] = {N_n, N_e, N_f, N_t}; *dev_bytes = the buffer
 * etpic_mesh_upload needs.  Errors: EINVAL, EMESH. */
int etpic_mesh_sizes(int64_t n_vert, const double *xyz_host, int64_t n_tet, const int32_t *tet_vert_host,
                     int64_t counts_out[4], size_t *dev_bytes);

/* Upload a tet mesh (Appendix A: the sets N, E, F, T) into the caller's
 * device buffer dev_buf (256-byte aligned, at least the etpic_mesh_sizes
 * bytes).  Host arrays: xyz_host[3*n_vert] (x,y,z per vertex),
 * tet_vert_host[4*n_tet] ascending per row.  Builds the canonical
 * edges/faces, tet->edge/face/neighbour tables and the barycentric gradients
 * on the host and fills the device tables in dev_buf (synchronously): topology,
 * gradient, push and geometry rows, the per-step coefficient table, point-location
 * grid, incidences, sort counters and the per-tet current slots.  Replaces any
 * previous mesh (and forgets its field, Gauss-law and downshifted buffers).
 * Errors: EINVAL (bad input, short buffer), EMESH, EHIP. */
int etpic_mesh_upload(etpic_ctx *ctx, int64_t n_vert, const double *xyz_host, int64_t n_tet,
                      const int32_t *tet_vert_host, void *dev_buf, size_t bytes);

/* Host only (no context, no GPU): the canonical numbering of a mesh, as
 * etpic_mesh_upload would build it.  counts_out[4] = {N_n, N_e, N_f, N_t};
 * edge_vert_host (2*N_e int32) and face_vert_host (3*N_f int32) are filled when
 * non-NULL (call once with NULLs to size them).  Errors: EINVAL, EMESH. */
int etpic_mesh_canonical(int64_t n_vert, const double *xyz_host, int64_t n_tet, const int32_t *tet_vert_host,
                         int64_t counts_out[4], int32_t *edge_vert_host, int32_t *face_vert_host);

/* counts_out[4] = {N_n, N_e, N_f, N_t} of the uploaded mesh.  ESTATE if none. */
int etpic_mesh_counts(const etpic_ctx *ctx, int64_t counts_out[4]);

/* Canonical edge list, host buffer of 2*N_e int32 (a<b per edge). */
int etpic_mesh_edges(const etpic_ctx *ctx, int32_t *edge_vert_host);

/* Canonical face list, host buffer of 3*N_f int32 (a<b<c per face). */
int etpic_mesh_faces(const etpic_ctx *ctx, int32_t *face_vert_host);

/* Particle upload from Cartesian positions (Problem Statement: particles are
 * points r_p; this library keeps each as its tet and barycentrics).
 * xyz[0..2]: device float64 arrays of length p->n (x, y, z of each point).
 * hint: device int32[p->n] start tets, or NULL; an entry outside [0, N_t)
 * means "no hint".  Each point is located by a straight walk from the centroid
 * of its start tet (the hint, else the tet registered for the point's cell of a
 * uniform grid built at mesh upload); p->tet and p->lam receive the tet and
 * lam_1..3 = grad lam_k . (x - r_0) of that tet (a point on a shared face may
 * land in either tet).  p->vel and p->id are not touched.  Synchronises
 * `stream`.  A point outside a boundary face by at most 1e-10 in barycentric
 * terms counts as on it (lam may then be slightly negative).  Points outside
 * the mesh, non-finite points, and points the straight
 * walk cannot reach (a non-convex domain without a good hint) get tet -1 and
 * make the call return EPARTICLE with their count; the others are located.
 * precision says how lam is stored (ETPIC_MIXED_FIXED: rounded to the
 * fixed-point grid).  Errors: EINVAL, ESTATE, EPARTICLE, EHIP. */
int etpic_particles_locate(etpic_ctx *ctx, const etpic_particles *p, int precision, const double *const xyz[3],
                           const int32_t *hint, void *stream);

/* Host checkpoint of the particle state of a time loop, so that a run
 * resumes where it stopped: (tet, lam_1..3, v, id) and the step index.
 * Fields, currents and charges are the caller's arrays and are not part of
 * it.  The file (a 136-byte header, then the arrays as stored on the device,
 * see checkpoint_host.hpp) carries the FNV-1a checksum of every array and of
 * the header, and a hash of the uploaded mesh: a checkpoint is read back only
 * on the same mesh (same vertex coordinates and tet vertex ids, bit for bit).
 *
 * etpic_checkpoint_write: copies the particles (device, p->n of them, stored
 * as `precision` says) to `path` through host chunks of 16 MiB on `stream`
 * (ordered after the work already queued there; synchronous on return).  It
 * writes `path`.tmp and renames it, so an existing checkpoint is replaced
 * whole or not at all.  The id array is saved when p->id is non-null.
 * Errors: EINVAL, ESTATE (no mesh), EIO (file), EHIP. */
int etpic_checkpoint_write(etpic_ctx *ctx, const etpic_particles *p, int precision, int64_t step, const char *path,
                           void *stream);

/* Header of a checkpoint file, host only (no context, no GPU): particle
 * count, precision, step index, whether ids are stored (each output may be
 * NULL).  EIO for a missing, short, foreign or corrupt header or a file whose
 * size does not match it. */
int etpic_checkpoint_info(const char *path, int64_t *n, int *precision, int64_t *step, int *has_id);

/* Reads a checkpoint into the particle arrays of p (device, allocated by the
 * caller with p->n = the checkpoint's count; etpic_checkpoint_info gives it)
 * and returns its step index in *step (may be NULL).  The checkpoint's
 * precision must equal `precision`, and p->id must be given exactly when the
 * checkpoint holds ids (EINVAL otherwise); a checkpoint of another mesh is
 * EMESH.  Every array's checksum is checked as it is read: EIO on a mismatch,
 * after which the particle arrays hold partly read data.  Synchronous. */
int etpic_checkpoint_read(etpic_ctx *ctx, const etpic_particles *p, int precision, const char *path, int64_t *step,
                          void *stream);

/* Cartesian positions x = sum_k lam_k r_k of the particles into the device
 * float64 arrays xyz[0..2] (length p->n).  A tet index outside [0, N_t) gives
 * NaN and the BADTET device flag.  precision says how lam is stored.
 * Asynchronous on `stream`. */
int etpic_particles_positions(etpic_ctx *ctx, const etpic_particles *p, int precision, double *const xyz[3],
                              void *stream);

/* One fine step of every particle, asynchronous on `stream`:
 * gather E, B at (x^n, t_n = step*dt) with the carrier (cos w t_n, sin w t_n)
 * evaluated on the host in float64; Boris update v^{n-1/2} -> v^{n+1/2};
 * walk the straight path x^n -> x^n + dt v^{n+1/2} through the mesh
 * (specular reflection at the domain boundary, hop cap ETPIC_HOP_CAP);
 * dG[N_e] += q w * (path integral of each Whitney edge function);
 * rho[N_n] += q w * lam_k(x^{n+1}) if rho != NULL.
 * dG and rho accumulate (the caller zeroes them).  The particle state is
 * updated in place.  Errors: EINVAL, ESTATE, EHIP; in-kernel errors via
 * etpic_check. */
int etpic_gather_push_deposit(etpic_ctx *ctx, const etpic_particles *p, int precision, const etpic_species *sp,
                              const etpic_fields *f, int64_t step, double dt, double omega, double *dG,
                              double *rho, uint32_t flags, void *stream);

/* nsteps consecutive steps (times (step0 + j) dt, j = 0..nsteps-1) with the same
 * field DoFs: the same result as nsteps calls of etpic_gather_push_deposit,
 * with rho (if not NULL) deposited after the last step only.  Between two
 * steps the walk of one and the coefficient pass of the next run in one
 * kernel launch.  With ETPIC_STEP_TIMING, etpic_kernel_time books that shared
 * launch as walk time (the coefficient time of all but the first step is 0).
 * Asynchronous on `stream`.  Errors as etpic_gather_push_deposit. */
int etpic_run_steps(etpic_ctx *ctx, const etpic_particles *p, int precision, const etpic_species *sp,
                    const etpic_fields *f, int64_t step0, int nsteps, double dt, double omega, double *dG,
                    double *rho, uint32_t flags, void *stream);

/* One coarse field step of the particles at the fine step (Particle Push
 * section: fields known at the coarse step dt_coarse are reconstructed at the
 * fine step with the quadratic Lagrange basis N_{n,k} of eqs. newmark_L /
 * newmark_N, the trajectories advanced at the fine step and the path integral
 * summed over the fine steps, eq. G_integral and the sum after it).
 * snap[0], snap[1], snap[2]: the field DoFs (same layout as
 * etpic_gather_push_deposit) at t_coarse - dt_coarse, t_coarse and
 * t_coarse + dt_coarse; the dc DoFs are taken from snap[1].  The particles
 * advance from t_coarse to t_coarse + dt_coarse in fine_steps steps of
 * dt = dt_coarse / fine_steps; fine step j gathers at t_j = t_coarse + j dt
 * with the envelope sum_k N_{n,k}(t_j) snap[k] modulated by e^{j w t_j}
 * (carrier at the fine time), then pushes, walks and deposits exactly as
 * etpic_gather_push_deposit.  dG accumulates the deposit of all fine steps;
 * rho, if not NULL, receives q w lam_k at the end of the last fine step.
 * flags as for etpic_gather_push_deposit; consecutive fine steps share
 * launches as in etpic_run_steps.  Asynchronous on `stream`.
 * Errors: EINVAL, ESTATE, EHIP; in-kernel errors via etpic_check. */
int etpic_coarse_step(etpic_ctx *ctx, const etpic_particles *p, int precision, const etpic_species *sp,
                      const etpic_fields snap[3], double t_coarse, double dt_coarse, int fine_steps, double omega,
                      double *dG, double *rho, uint32_t flags, void *stream);

/* Counting sort of the particles by tet (histogram, exclusive scan, scatter):
 * src -> dst (distinct buffers, same n and precision); the order among
 * particles of one tet is unspecified.  Asynchronous on `stream`. */
int etpic_sort(etpic_ctx *ctx, const etpic_particles *src, const etpic_particles *dst, int precision,
               void *stream);

/* etpic_sort(src -> dst) followed by etpic_run_steps on dst, with the sort's
 * scatter folded into the first step: the first step's particle kernel reads
 * the particles of src in their order and writes them, pushed, at their
 * tet-sorted positions of dst, so the particle state crosses HBM once for
 * both (used for the periodic re-sort).  Each particle's result, and the
 * placement of the tets' groups, are those of the two calls; the order within
 * a tet is unspecified as for etpic_sort, and dG / rho agree to the float64
 * atomics' summation order.  src is read only.  Requirements on src and dst
 * as for etpic_sort, on the step arguments as for etpic_run_steps;
 * nsteps >= 1.  Asynchronous on `stream`.  Errors as etpic_run_steps. */
int etpic_sort_run_steps(etpic_ctx *ctx, const etpic_particles *src, const etpic_particles *dst, int precision,
                         const etpic_species *sp, const etpic_fields *f, int64_t step0, int nsteps, double dt,
                         double omega, double *dG, double *rho, uint32_t flags, void *stream);

/* rho[N_n] += q w * lam_k for the four vertices of every particle's tet
 * (the W0 shape; Formulation, the particle charge density).  Same-tet runs of
 * consecutive particles are summed in the wavefront before the float64
 * atomics; where the last sort found long runs (as the particle kernel picks
 * its slices) each wavefront covers 4 or 16 slices of 64 particles and carries
 * a run across them.  precision says how lam is stored.  Asynchronous. */
int etpic_vertex_charge(etpic_ctx *ctx, const etpic_particles *p, int precision, const etpic_species *sp, double *rho,
                        void *stream);

/* Discrete continuity residual r = D^T dG - (rho_new - rho_old), D the edge-vertex
 * incidence (-1 tail, +1 head) (section on discretization and exact charge
 * conservation).  Synchronises `stream`; out_host[0] = max|r|,
 * out_host[1] = max|rho_old|.  Both maxima propagate NaN: if any entry of dG,
 * rho_new or rho_old is not finite the function still writes out_host (NaN or
 * inf) and returns ETPIC_ENAN. */
int etpic_gauss_residual(etpic_ctx *ctx, const double *dG, const double *rho_new, const double *rho_old,
                         double out_host[2], void *stream);

/* Slices of 64 particles per wavefront that the last particle-kernel launch of
 * a step call used (1: k_push; 2: k_push_pipe, two pipelined slices; 4 or 16:
 * k_push_slices<S>; 0 before any step).  Host only. */
int etpic_last_push_slices(const etpic_ctx *ctx, int *slices);

/* Measurement aid, not a step of the method: the particle kernel's HBM access
 * pattern alone (the same launch shape and XCD block order, non-temporal loads
 * of tet, lambda_1..3 and v, non-temporal stores of lambda_1..3 and v in
 * place; 100 B per particle in float64, 76 B with float32 velocities) with no
 * arithmetic, so that the streaming rate that pattern reaches on the device can
 * be timed beside the particle kernel.  The particle arrays are rewritten with
 * their own values (unchanged).  flags: ETPIC_STEP_XCD_REMAP or 0.
 * Asynchronous on `stream`; EINVAL for a bad descriptor or precision. */
int etpic_stream_probe(etpic_ctx *ctx, const etpic_particles *p, int precision, uint32_t flags, void *stream);

/* etpic_gauss_residual without any allocation, for callers that cannot
 * allocate device memory (loops that log the residual every step under an
 * allocation-free policy, harnesses that forbid hipMalloc).  Same arguments,
 * result and errors as etpic_gauss_residual (the maxima are the same numbers).
 * Its scratch is a file-scope device array of 16 KB (1,024 partial pairs and
 * the result pair), one per GPU for the life of the process, whose address
 * etpic_create takes on the context's device; any mesh size is served (the
 * vertices are visited by a grid-stride loop over at most 1,024 blocks), and
 * a mesh beyond 2^31 - 1 vertices is refused with EINVAL.  Calls on one GPU
 * share that array: calls that overlap on one GPU (two streams, two threads)
 * race and must be serialised by the caller.  Synchronises `stream`. */
int etpic_gauss_residual_noalloc(etpic_ctx *ctx, const double *dG, const double *rho_new, const double *rho_old,
                                 double out_host[2], void *stream);

/* ---- Downshifted integrator ------------------------------------------------
 * The Particle Push section's scheme that treats the carrier analytically in
 * the velocity update.  Over a step [t_n, t_n + dt] the envelope fields sampled
 * at the particle (E~, B~ from the Whitney expansions, and the dc DoFs) and the
 * velocity are interpolated in time by the Lagrange basis N_k on the nodes
 * t_n, t_{n-1}, t_{n-2}, and the carrier is integrated exactly against them:
 *   v^{n+1} = v^n + q/m sum_k (Re E~_k M^r_k + Im E~_k M^i_k + Edc_k P_k)
 *           + q/m sum_{j,k} v^{n-j} x (Re B~_k L^r_jk + Im B~_k L^i_jk + Bdc_k Q_jk),
 * M^r_k = int N_k cos(wt), M^i_k = -int N_k sin(wt), L^r_jk = int N_j N_k
 * cos(wt), L^i_jk = -int N_j N_k sin(wt) (the section's operators), P_k = int
 * N_k, Q_jk = int N_j N_k over the step.  Positions advance by the
 * fourth-order Adams-Bashforth stencil in the velocities (eq. newtons); the
 * path r^n -> r^{n+1} is walked and deposited exactly as in
 * etpic_gather_push_deposit (same dG, rho and continuity law).  At a wall the
 * velocity and the velocity samples kept for later steps are mirrored.  With
 * fewer than three earlier downshifted steps the orders ramp up: K =
 * min(hist, 2) + 1 nodes and Adams-Bashforth order min(hist, 3) + 1.
 * Precision: ETPIC_FP64, or ETPIC_MIXED (float32 samples, velocities and
 * velocity update, float64 positions, barycentric increments and deposit,
 * as the mixed fine-step form). */

/* Bytes of the per-tet complex-envelope rows of the downshifted step (72
 * float64 per tet of the uploaded mesh), and binding of the caller's buffer
 * (device, 256-byte aligned) that holds them; etpic_ds_steps needs it (ESTATE
 * otherwise) and rebuilds the rows at each call.  A mesh upload forgets it. */
int etpic_ds_rows_bytes(const etpic_ctx *ctx, size_t *bytes);
int etpic_ds_rows_bind(etpic_ctx *ctx, void *dev_buf, size_t bytes);

/* Size of the history buffer for n particles: 48 arrays of length n of the
 * velocity type (float64, float32 for ETPIC_MIXED): velocity ring v^m in slot
 * m mod 4; E and B samples, real part, imaginary part and dc part, of step m
 * in slot m mod 2.  Host only. */
int etpic_ds_history_bytes(int64_t n, int precision, size_t *bytes_out);

/* nsteps downshifted steps from step0 (t_n = n dt) with fixed field DoFs.
 * p: particles of `precision`, p->vel = v^n in, v^{n+nsteps} out.  hist: the history
 * buffer (device, 8-byte aligned, at least etpic_ds_history_bytes), whose
 * slots are addressed by the step number, so successive calls must continue
 * the numbering; hist0 = number of downshifted steps already taken with this
 * buffer (0 for a fresh start: the buffer is then not read); the calls that
 * share a history either all give dc edge DoFs or none does (without them the
 * E dc samples are neither stored nor read).  Re-sort with etpic_ds_sort,
 * which moves the history with the particles (etpic_sort does not: restart
 * with hist0 = 0 after it).  dG accumulates the deposit of all steps, rho (if not NULL)
 * receives q w lam_k after the last one.  flags as for
 * etpic_gather_push_deposit (XCD_REMAP, TIMING, WALK_BY_SLICE).  The
 * complex-envelope rows go to the buffer of etpic_ds_rows_bind.
 * Asynchronous on `stream`.  Errors: EINVAL, ESTATE, EHIP; in-kernel errors
 * via etpic_check. */
int etpic_ds_steps(etpic_ctx *ctx, const etpic_particles *p, int precision, void *hist, size_t hist_bytes,
                   const etpic_species *sp, const etpic_fields *f, int64_t step0, int nsteps, int hist0, double dt,
                   double omega, double *dG, double *rho, uint32_t flags, void *stream);

/* etpic_sort of particles src -> dst that also moves their downshifted
 * history hist_src -> hist_dst (distinct device buffers of at least
 * hist_bytes = etpic_ds_history_bytes(n, precision)), so the steps continue
 * with the same numbering and hist0.  Asynchronous on `stream`.  Errors as
 * etpic_sort. */
int etpic_ds_sort(etpic_ctx *ctx, const etpic_particles *src, const etpic_particles *dst, int precision,
                  const void *hist_src, void *hist_dst, size_t hist_bytes, void *stream);

/* ---- Differentiation (float64 form only) --------------------------------
 * Reverse-mode derivative of nsteps particle steps with respect to the
 * complex edge envelope, for a loss of the final particle state, with step
 * checkpointing (the state is kept every `checkpoint_every` steps and each
 * segment is recomputed from its checkpoint during the reverse sweep).  The
 * gradient follows the convention dL/dRe(e) + j dL/dIm(e) (the one PyTorch
 * uses for real losses of complex tensors).  The face envelope and the dc
 * DoFs are held fixed; the tet sequence and wall reflections of every step
 * are those of the forward run (the step map is piecewise smooth). */

/* Device workspace in bytes for n particles, nsteps steps, checkpoint_every >= 1. */
int etpic_adjoint_workspace(const etpic_ctx *ctx, int64_t n, int nsteps, int checkpoint_every, size_t *bytes_out);

/* nsteps float64 steps (times step0, step0+1, ...) of the particles p, in
 * place, exactly as etpic_gather_push_deposit, recording the checkpoints in
 * `workspace` (device, >= etpic_adjoint_workspace bytes).  dG (N_e)
 * accumulates the deposit, or NULL to discard it.  Asynchronous. */
int etpic_forward_checkpointed(etpic_ctx *ctx, const etpic_particles *p, const etpic_species *sp,
                               const etpic_fields *f, int64_t step0, int nsteps, double dt, double omega,
                               int checkpoint_every, void *workspace, size_t workspace_bytes, double *dG,
                               void *stream);

/* Reverse sweep of the run recorded by etpic_forward_checkpointed (same n,
 * species, fields, step0, nsteps, dt, omega, checkpoint_every, workspace).
 * vbar[k], xbar[k]: device float64 arrays of n.  In: adjoints of the final
 * velocity (v^{n+1/2} after the last step) and final Cartesian position.  Out:
 * adjoints of the initial velocity and position.  grad_e (2*N_e float64,
 * interleaved complex) accumulates the envelope gradient.  Asynchronous. */
int etpic_backward(etpic_ctx *ctx, int64_t n, const etpic_species *sp, const etpic_fields *f, int64_t step0,
                   int nsteps, double dt, double omega, int checkpoint_every, void *workspace,
                   size_t workspace_bytes, double *const vbar[3], double *const xbar[3], double *grad_e,
                   void *stream);

/* ---- Field-coefficient update (side path, timed separately) ---------------
 * Eliminating the face envelope from the envelope Maxwell curl equations
 * (Formulation: the curl equations with the carrier) and testing with the
 * Whitney edge functions gives, for the complex edge envelope e,
 *     M e'' + 2 j w M e' + (K - w^2 M) e = -e^{-j w t} g''
 * with M = eps-weighted edge mass matrix, K = (1/mu)-weighted curl-curl
 * matrix (Appendix A: [*eps] and the curl matrices) and g the deposited edge
 * DoFs of G.  It is stepped with Newmark-beta, gamma = 1/2, beta = 1/4
 * (Formulation), in acceleration form; the implicit system
 *     A = (1 + j w dt - w^2 dt^2 / 4) M + (dt^2 / 4) K
 * is complex symmetric and solved by Jacobi-preconditioned COCG with a CSR
 * sparse matrix-vector product.  Boundary edges are perfect-conductor
 * (tangential field zero).  The face envelope follows the envelope Faraday law
 * (j w + d/dt) b = -C e (C the face-edge incidence, (C e)_f = e_ab + e_bc - e_ac
 * for face (a<b<c)) with the trapezoidal rule.  Run on a state without
 * gradient part (D^T [*eps] u = 0 at the inner nodes) and driven by the
 * source of etpic_sol_source, the same step is the solenoidal system of the
 * quasi-Helmholtz split (etpic_em_steps with ETPIC_EM_SPLIT); driven by the
 * plain source it carries a gradient part that only etpic_ns_correct makes
 * obey Gauss' law. */

/* Bytes of the field-step solver for permittivity eps and permeability mu
 * (assembles M and K on the host, kept for the etpic_field_setup call that
 * follows with the same eps and mu). */
int etpic_field_bytes(etpic_ctx *ctx, double eps, double mu, size_t *bytes);

/* Field step dt, carrier w, permittivity eps, permeability mu: M, K, the
 * Jacobi preconditioner and the COCG work vectors in the caller's buffer
 * (device, 256-byte aligned, at least etpic_field_bytes).  Replaces the
 * previous setup.  Errors: EINVAL (bad parameters, short buffer), ESTATE (no
 * mesh), EMESH, EHIP. */
int etpic_field_setup(etpic_ctx *ctx, double dt, double omega, double eps, double mu, void *dev_buf, size_t bytes);

/* Number of stored entries of the CSR pattern (M and K share it). */
int etpic_field_nnz(const etpic_ctx *ctx, int64_t *nnz_out);

/* y = alpha M x + beta K x for complex x, y (2*N_e float64 each, device),
 * complex alpha, real beta.  Asynchronous. */
int etpic_field_spmv(etpic_ctx *ctx, const double *x, double *y, double alpha_re, double alpha_im, double beta,
                     void *stream);

/* One field step to time t_next: u = e, v = e', a = e'' (2*N_e float64 each,
 * complex, device, updated in place), b = face envelope (2*N_f, in place),
 * gdd = g'' at t_next (N_e float64, device, NULL = 0).  COCG stops when
 * ||r|| / ||rhs|| <= tol (tested on the device every iteration, read by the
 * host every 5) or after max_iter;
 * *iters_out, *resid_out report it.  Synchronises `stream`.  ENOCONV (state
 * left unchanged) if the tolerance is not reached. */
int etpic_field_step(etpic_ctx *ctx, double t_next, double *u, double *v, double *a, double *b, const double *gdd,
                     double tol, int max_iter, int *iters_out, double *resid_out, void *stream);

/* ---- Non-solenoidal field of the quasi-Helmholtz split (Quasi Helmholtz or
 * Coulomb gauge, Discrete System, eq. ns_equation; operators of App. A).
 * Gauss' law is solved on its own: with D the node-to-edge incidence (the
 * discrete gradient [grad]; -1 at an edge's lower vertex id, +1 at its
 * higher), [*eps] the Whitney edge mass and C_z the map that grounds the wall
 * nodes (vertices of boundary faces),
 *     C_z^T D^T [*eps] D C_z x = -C_z^T (D^T e^{-j w t} G + e^{-j w t} rho0),
 *     e_ns = D C_z x.
 * G is the real path integral of the deposited current (the dG of the step
 * calls, summed); rho0 the nodal charge present when that sum started (D^T G
 * counts only the change).  D^T [*eps] D is the linear-element stiffness
 * eps int grad W0_i . grad W0_j; it is real, so the solve is real and the
 * carrier phase e^{-j w t} multiplies its solution.  Float64 throughout. */

/* Bytes of the Gauss-law solver for permittivity eps (assembles the nodal
 * operator on the host, kept for the etpic_ns_setup call that follows). */
int etpic_ns_bytes(etpic_ctx *ctx, double eps, size_t *bytes);

/* The nodal operator for permittivity eps, its Jacobi preconditioner and the
 * CG work vectors in the caller's buffer (device, 256-byte aligned, at least
 * etpic_ns_bytes).  Replaced by the next call, forgotten by a mesh upload. */
int etpic_ns_setup(etpic_ctx *ctx, double eps, void *dev_buf, size_t bytes);

/* Stored entries of the nodal operator (wall rows count one each) and, if
 * wall_nodes_out is not NULL, the number of grounded wall nodes. */
int etpic_ns_info(const etpic_ctx *ctx, int64_t *nnz_out, int64_t *wall_nodes_out);

/* flags of etpic_ns_solve and etpic_ns_run_steps */
enum etpic_ns_flags {
    /* start the CG from the solution of the previous solve on this context
     * (x = 0 after etpic_ns_setup) instead of from zero: in a time loop the
     * field changes little from one step to the next */
    ETPIC_NS_WARM = 64u
};

/* Solve eq. ns_equation.  G: N_e float64 (device, NULL = 0); rho0: N_n
 * float64 (device, NULL = 0); t, omega: the carrier phase.  Outputs (device,
 * either may be NULL but not both): x_out = nodal coefficients, 2*N_n float64
 * (complex, interleaved; 0 on the wall), e_out = edge coefficients of the
 * non-solenoidal electric field, 2*N_e float64 (complex).  flags: 0 or
 * ETPIC_NS_WARM.  Preconditioned CG stops when ||r|| / ||b|| <= tol (tested
 * on the device every iteration, read by the host every 10) or after
 * max_iter; *iters_out and *resid_out (may be NULL) report it.  No source
 * (b = 0) gives x = 0 without iterations.  Synchronises `stream`.  ENOCONV
 * (outputs untouched) if the tolerance is not reached. */
int etpic_ns_solve(etpic_ctx *ctx, const double *G, const double *rho0, double t, double omega, double *x_out,
                   double *e_out, double tol, int max_iter, uint32_t flags, int *iters_out, double *resid_out,
                   void *stream);

/* The particles in the field of their own charge: the loop field -> particles
 * -> G -> field closed through eq. ns_equation (the non-solenoidal part of
 * the split only; no solenoidal field is computed).  Every steps_per_solve
 * steps, at t = (step0 + j) dt: solve eq. ns_equation from G and rho0
 * (warm-started after the first solve, and for the first too with
 * ETPIC_NS_WARM) and set e_work = D y (+ ext->e_dc): the field of the charge
 * is quasi-static, so it enters the steps as real, unmodulated edge DoFs and
 * is held over the steps up to the next solve (the multi-rate use: fields at
 * the coarse step, particles at the fine one).  Then those steps (as
 * etpic_run_steps) in the fields {ext->e_env, e_work, ext->b_env, ext->b_dc}
 * (without ext: no other field), their path integrals added to G.
 * G: N_e float64 (device, in place), the running path integral of the
 * current; rho0: N_n float64 (device, NULL = 0), the charge when G was zero;
 * e_work: N_e float64 (device, caller-owned; holds the last solve's edge DoFs
 * on return; must not be ext->e_dc).  One species per call.  flags:
 * ETPIC_STEP_* flags of the particle steps, ETPIC_NS_WARM.  *iters_out (may
 * be NULL): CG iterations summed over the solves.  Synchronises `stream` once
 * per solve.  ENOCONV stops the loop at the solve that failed (the particles
 * have taken the steps before it). */
int etpic_ns_run_steps(etpic_ctx *ctx, const etpic_particles *p, int precision, const etpic_species *sp,
                       const etpic_fields *ext, int64_t step0, int nsteps, int steps_per_solve, double dt,
                       double omega, double *G, const double *rho0, double *e_work, double tol, int max_iter,
                       uint32_t flags, int *iters_out, void *stream);

/* Gauss-law correction of a field-step state (the property the split is
 * for: Gauss' law exact for the fields, Discrete System).  For the complex
 * edge envelope u (2*N_e float64, device; e.g. the u of etpic_field_step,
 * zero on boundary edges) returns e_out = u + D y (2*N_e, device; may alias
 * u), y complex on the nodes, zero on the wall, from
 *     D^T [*eps] D y = -(e^{-j w t} (D^T G + rho0) + D^T [*eps] u)
 * at the other nodes, so that D^T [*eps] e_out = -e^{-j w t}(D^T G + rho0):
 * the curl of e_out is that of u (C D = 0) and its divergence is the
 * deposited charge's.  [*eps] is the field step's mass, so etpic_field_setup
 * and etpic_ns_setup must have been called with the same eps (EINVAL
 * otherwise).  Two real CG solves (the real and imaginary parts), warm-started
 * from the previous call's with ETPIC_NS_WARM; *iters_out = their sum,
 * *resid_out = the larger residual.  Synchronises `stream`; ENOCONV leaves
 * e_out untouched. */
int etpic_ns_correct(etpic_ctx *ctx, const double *G, const double *rho0, double t, double omega, const double *u,
                     double *e_out, double tol, int max_iter, uint32_t flags, int *iters_out, double *resid_out,
                     void *stream);

/* Source of the solenoidal system of the split (eq. sol_disc; the projector
 * P^Lambda_e taken orthogonal in the [*eps] inner product, whose range is
 * that of the cotree unknowns' fields, and its transpose applied to the
 * source of the field step):
 *     gs = gdd - [*eps] D y,  D^T [*eps] D y = D^T gdd at the inner nodes,
 * y zero on the wall, so that D^T gs = 0 at the inner nodes and the field
 * step driven by gs keeps a state without gradient part free of one (the
 * curl-curl stiffness annihilates gradients).  gdd, gs_out: N_e float64
 * (device; gs_out may be gdd); on edges of boundary faces gs = gdd.  Needs
 * etpic_field_setup and etpic_ns_setup with the same eps (ESTATE / EINVAL);
 * uses the field step's work vectors.  One real CG solve, stopping and
 * reporting as etpic_ns_solve; flags: 0 or ETPIC_NS_WARM (start from this
 * function's previous solution).  Synchronises `stream`; ENOCONV leaves
 * gs_out untouched. */
int etpic_sol_source(etpic_ctx *ctx, const double *gdd, double *gs_out, double tol, int max_iter, uint32_t flags,
                     int *iters_out, double *resid_out, void *stream);

/* flag of etpic_em_steps */
enum etpic_em_flags {
    /* the loop in the form of the split: the field step takes the source of
     * etpic_sol_source (u, v, a then stay free of a gradient part; they must
     * start so, e.g. zero, or etpic_ns_correct's e minus its gradient) and
     * e = u + the field of eq. ns_equation from G and rho0 (etpic_ns_solve);
     * one real solve each, as many as the correction takes */
    ETPIC_EM_SPLIT = 128u
};

/* The electromagnetic loop with Gauss' law exact for the fields (the loop
 * field -> particles -> G -> field of the split, with the implicit field
 * step for the solenoidal part and etpic_ns_correct for the rest).  Uses the
 * dt and omega of etpic_field_setup.  For each of nsteps steps, t = (step0 +
 * j) dt: one particle step (as etpic_run_steps) in the fields {e, b} at t,
 * its path integral added to G; the field step (etpic_field_step) to t + dt
 * with the source g'' = (G - 2 G_hist[0..N_e) + G_hist[N_e..2N_e)) / dt^2,
 * the second difference of G one step behind; G_hist shifted (G one and two
 * steps back); e = the Gauss correction of u at t + dt with G and rho0.
 * State (device, caller-owned, in place): u, v, a, e 2*N_e float64 complex
 * (e must hold the field of step step0 on entry, e.g. etpic_ns_correct of
 * u), b 2*N_f complex, G N_e float64 (the running path integral), G_hist
 * 2*N_e float64 (zero for a start from rest), rho0 N_n float64 or NULL (the
 * charge when G was zero).  One species per call.  flags: ETPIC_STEP_* of
 * the particle steps, ETPIC_NS_WARM for the first correction (or the first
 * solves of the split form), ETPIC_EM_SPLIT for the split form.  *iters_out:
 * COCG and CG iterations summed.  Synchronises `stream` several times per
 * step; ENOCONV stops the loop at the solve that failed. */
int etpic_em_steps(etpic_ctx *ctx, const etpic_particles *p, int precision, const etpic_species *sp, int64_t step0,
                   int nsteps, double *u, double *v, double *a, double *b, double *e, double *G, double *G_hist,
                   const double *rho0, double tol, int max_iter, uint32_t flags, int *iters_out, void *stream);

/* ---- Quasi-Helmholtz projectors (Quasi Helmholtz or Coulomb gauge section,
 * eqs. proj_es, proj_el, bfld_projector, efld_projected; App. A):
 *     P^Lambda_b = I - div^T (div div^T)^-1 div          (face DoFs),
 *     P^Sigma_e  = Sigma (Sigma^T Sigma)^+ Sigma^T,  P^Lambda_e = I - P^Sigma_e
 *                                                        (edge DoFs),
 * with Sigma = eps0 M_g = [*eps] D (the gradient of a hat function is a signed
 * sum of Whitney edge functions, so M_g = [*eps] D / eps0), D the node-edge
 * incidence, [*eps] the Whitney edge mass (all rows, no boundary condition)
 * and div = [*rho]^-1 M_d the signed tet-face incidence (+1 where the face's
 * global normal, right-handed in its ascending vertex order, points out of
 * the tet).  + is the Moore-Penrose pseudoinverse: Sigma^T Sigma has the
 * constants as null space and the nodal solution returned is the one
 * orthogonal to them.  The projector object keeps its own copy of the mesh
 * tables (same canonical numbering as etpic_mesh_upload) and work vectors, on
 * the device in the caller's buffer (etpic_qh_bind); it is independent of
 * etpic_ctx.  Errors: etpic status codes, the
 * message from etpic_qh_last_error() (thread-local).  Vectors are complex,
 * 2*N float64 interleaved, on the device; calls synchronise `stream`. */
typedef struct etpic_qh etpic_qh;

/* Thread-local message of the last failing etpic_qh_* call. */
const char *etpic_qh_last_error(void);

/* Build the projector object on HIP device `device` for the mesh (xyz: 3*nv
 * float64, tet_vert: 4*nt int32 ascending per row, host; the mesh must be
 * connected, else EMESH) and permittivity eps: its tables are built on the
 * host; the device part is given by etpic_qh_bind.  *out receives the handle. */
int etpic_qh_create(etpic_qh **out, int device, int64_t nv, const double *xyz, int64_t nt, const int32_t *tet_vert,
                    double eps);

/* Device bytes of the object (mesh tables, edge mass, work vectors), and the
 * binding of the caller's buffer (device, 256-byte aligned, at least that
 * size) that receives them (synchronously).  The projections need it
 * (ESTATE otherwise). */
int etpic_qh_bytes(const etpic_qh *qh, size_t *bytes);
int etpic_qh_bind(etpic_qh *qh, void *dev_buf, size_t bytes);

/* Destroy the object (its host tables; the bound buffer is the caller's).
 * NULL accepted. */
void etpic_qh_destroy(etpic_qh *qh);

/* counts_out = {N_n, N_e, N_f, N_t, stored entries of [*eps]}. */
int etpic_qh_counts(const etpic_qh *qh, int64_t counts_out[5]);

/* b_out = P^Lambda_b b (2*N_f float64 each; may alias).  CG on div div^T
 * stops when ||r|| / ||div b|| <= tol (tested on the device every iteration,
 * read by the host every 10) or after max_iter: ENOCONV, b_out untouched.
 * *iters_out, *resid_out (may be NULL) report it. */
int etpic_qh_project_b(etpic_qh *qh, const double *b, double *b_out, double tol, int max_iter, int *iters_out,
                       double *resid_out, void *stream);

/* For edge DoFs d (2*N_e float64): d_sigma = P^Sigma_e d, d_lambda =
 * P^Lambda_e d (2*N_e each) and e_ns = (Sigma^T Sigma)^+ Sigma^T d (2*N_n),
 * so that d = Sigma e_ns + P^Lambda_e d (eq. efld_projected).  Any output may
 * be NULL, not all; none may alias d.  Jacobi-preconditioned CG on Sigma^T
 * Sigma with the stopping rule of etpic_qh_project_b (residual relative to
 * ||Sigma^T d||); ENOCONV leaves the outputs untouched. */
int etpic_qh_project_e(etpic_qh *qh, const double *d, double *d_sigma, double *d_lambda, double *e_ns, double tol,
                       int max_iter, int *iters_out, double *resid_out, void *stream);

/* Tree-cotree maps of the split (Discrete System; the maps [C^e_c], [C^b_c]
 * of App. A), host only, no device needed.  For the mesh (arguments as
 * etpic_mesh_canonical, same canonical numbering): edge_tree_host[e] = 1 for
 * the edges of a spanning tree of the vertex graph (breadth first from the
 * lowest vertex of each component), 0 for the cotree edges; face_tree_host[f]
 * = 1 for the faces of a spanning tree of the dual graph (tets plus one
 * exterior node joined by the boundary faces), 0 for the cotree faces.  [C^e_c]
 * and [C^b_c] select the cotree edges and faces in ascending id: with a
 * connected mesh there are N_e - N_n + 1 and N_f - N_t of them, the
 * dimensions of the discretely divergence-free edge and face fields, and the
 * tree values of such a field follow from its cotree values.  counts_out =
 * {tree edges, cotree edges, tree faces, cotree faces}.  Errors as
 * etpic_mesh_canonical, message from etpic_qh_last_error(). */
int etpic_tree_cotree(int64_t n_vert, const double *xyz_host, int64_t n_tet, const int32_t *tet_vert_host,
                      uint8_t *edge_tree_host, uint8_t *face_tree_host, int64_t counts_out[4]);

/* The solenoidal system of eq. sol_disc (Quasi Helmholtz section, Discrete
 * System) on the cotree unknowns, with the blocks as App. A prints them
 * (Euclidean projectors P^Lambda_b, P^Lambda_e of the object `qh` of the same
 * mesh; [curl] = C the signed face-edge incidence; [*mu^-1] the Whitney face
 * mass; C_e, C_b the cotree edges and faces of etpic_tree_cotree, ascending;
 * C_z the nodes off the conducting wall, ascending).  Created on the host
 * from the mesh (as given to etpic_qh_create) and mu; the device part lives
 * in the caller's buffer (etpic_cotree_bytes, etpic_cotree_bind: 256-byte
 * aligned).  Vectors are complex (re, im) float64 pairs on the device; the
 * calls synchronise.  Errors: EINVAL, ESTATE (not bound), EMESH, EHIP,
 * ENOCONV (an inner projector solve or the step's GMRES did not reach its
 * tolerance); message from etpic_qh_last_error(). */
typedef struct etpic_cotree etpic_cotree;
int etpic_cotree_create(etpic_cotree **out, const etpic_qh *qh, int64_t nv, const double *xyz, int64_t nt,
                        const int32_t *tet_vert, double mu);
int etpic_cotree_bytes(const etpic_cotree *z, size_t *bytes);
int etpic_cotree_bind(etpic_cotree *z, void *dev_buf, size_t bytes);
void etpic_cotree_destroy(etpic_cotree *z);

/* counts_out = {cotree edges N_ec, cotree faces N_fc, nodes off the wall N_z,
 * stored face-mass entries} */
int etpic_cotree_counts(const etpic_cotree *z, int64_t counts_out[4]);

/* y = Z_block x for block 11 (x: N_fc -> y: N_fc), 12 (N_ec -> N_fc), 13
 * (N_z -> N_fc), 21 (N_ec -> N_ec), 22 (N_fc -> N_ec), 23 (N_z -> N_ec), each
 * applied matrix-free; tol and max_iter bound the projector solve it needs
 * (blocks 11, 12, 21, 22).  Z13 is the curl of a gradient and comes out at
 * rounding level. */
int etpic_cotree_apply(etpic_cotree *z, etpic_qh *qh, int block, const double *x, double *y, double tol,
                       int max_iter, void *stream);

/* b_out = P^Lambda_b C_b bs: the divergence-free face field (N_f) the
 * blocks attach to the cotree unknowns bs (N_fc). */
int etpic_cotree_b_field(etpic_cotree *z, etpic_qh *qh, const double *bs, double *b_out, double tol, int max_iter,
                         void *stream);

/* One step of eq. sol_disc, time derivatives by the trapezoidal rule over
 * [t_n, t_n + dt] with carrier frequency omega (a = 1/dt + j omega/2):
 *   Z11 (a B1 - conj(a) B0) + Z12 (E1 + E0)/2 = 0,
 *   Z21 (a E1 - conj(a) E0) - Z22 (B1 + B0)/2 = src
 * (Z13 E_ns = 0 identically; src, N_ec or NULL, is the Ampere right-hand side
 * at the midpoint: the current and E_ns terms on the cotree edges).  The
 * state is b (N_f, the face field P^Lambda_b C_b B_s, in/out) and es (N_ec,
 * in/out).  Faraday's rows hold on every face, so b advances explicitly; the
 * Ampere rows are one system on the cotree edges, solved by restarted GMRES
 * (relative residual tol, at most max_iter iterations, each with one
 * P^Lambda_e solve to inner_tol / inner_max) from the guess es; iters_out and
 * resid_out (may be NULL) report it.  The printed Z21 is not symmetric and,
 * from a few cells per side on, indefinite: GMRES then needs many iterations
 * or does not converge (ENOCONV: es holds the last iterate, b is left as it
 * was). */
int etpic_cotree_step(etpic_cotree *z, etpic_qh *qh, double dt, double omega, double *b, double *es,
                      const double *src, double tol, int max_iter, double inner_tol, int inner_max, int *iters_out,
                      double *resid_out, void *stream);

/* Kernel times of the steps launched with ETPIC_STEP_TIMING since the last
 * reset, from HIP start and stop events bound to each kernel's own dispatch
 * on the launch stream (hipExtLaunchKernel: no marker packets between the
 * kernels, so the timing does not stretch the step), summed over the steps:
 * ms_out[0] = particle kernel (gather, push, in-tet deposit) of the steps
 * that update the particles in place, ms_out[1] = per-tet coefficient kernel
 * where it runs alone, ms_out[2] = walk kernel (with the next step's
 * coefficient pass where the two share a launch, and the gather of the
 * per-tet current sums onto the edges at the end of a call), ms_out[3] =
 * particle kernel of the steps that also sort (the first step of
 * etpic_sort_run_steps); [1] and [2] only for steps run with
 * ETPIC_STEP_TIMING_ALL (0 otherwise).  launches_out (may be NULL) = number of timed steps
 * of each kind: [0] in place, [1] sorting.  Synchronises on the events;
 * reset != 0 clears the record afterwards. */
int etpic_kernel_time(etpic_ctx *ctx, double ms_out[4], int64_t launches_out[2], int reset);

/* Synchronise `stream`, return and clear the device status word in *device_flags.
 * Returns EWALK / ENAN / EPARTICLE for the first set bit, OK otherwise. */
int etpic_check(etpic_ctx *ctx, void *stream, uint32_t *device_flags);

#ifdef __cplusplus
}
#endif
#endif /* ETPIC_H */
