/*
 * lbfd.h -- C ABI of the MI355X (gfx950) solver for the hybrid lattice-
 * Boltzmann colour-gradient / finite-difference method for two-phase flow
 * with soluble surfactants (Ba, Liu, Li, Yang; arXiv 2311.15242).
 *
 * One time step (lbfd_step) is the method's whole per-step path:
 *   - interface geometry and forces: colour function (eq 6), normal and
 *     curvature (eq 7), modified Langmuir equation of state (eq 8),
 *     interfacial force with the Marangoni term (eqs 5 and 9), buoyancy
 *     (Sec 3.4), fluid velocity (eq 10);
 *   - MRT collision with the correction and forcing terms (eqs 1-4,
 *     Appendix A eqs 36-43), recolouring (eqs 11-12) and propagation
 *     (eq 13) with periodic or half-way bounce-back boundaries;
 *   - finite-difference transport of the interface and bulk surfactant
 *     concentrations psi and phi (eqs 20-22) with WENO3 convection
 *     (eqs 25-27), conservative diffusion (eq 28), the modified
 *     Crank-Nicolson scheme (eqs 23-24) solved by red-black SOR, and the
 *     rescaling that restores the total surfactant (Sec 2.2).
 *
 * Conventions
 *   - Lattice units, dx = dt = 1. Grids are nx * ny * nz nodes (nz = 1 in
 *     2-D), node index n = x + nx * (y + ny * z), x fastest.
 *   - Device memory: the caller allocates one device workspace of the size
 *     lbfd_workspace_bytes reports and keeps it alive until lbfd_destroy;
 *     the handle only borrows it. The handle allocates nothing on the device
 *     except transient buffers inside lbfd_read_field / lbfd_set_state /
 *     lbfd_write_field; lbfd_read_field_noalloc stages through a fixed
 *     library-owned array instead and allocates nothing.
 *   - Streams: every device operation is enqueued on the stream given to
 *     lbfd_create (a hipStream_t passed as void*; NULL is the null stream).
 *     lbfd_step is asynchronous; lbfd_observables, lbfd_read_field and
 *     lbfd_set_state synchronise that stream.
 *   - Host arrays exchanged with the library are FP64 whatever the storage
 *     precision, laid out [component][z][y][x].
 *   - Every call returns an lbfd_status; no call aborts or exits. A handle
 *     is used from one host thread at a time.
 */
#ifndef LBFD_H
#define LBFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBFD_OK = 0,
    LBFD_EINVAL = -1,       /* bad argument, shape or parameter */
    LBFD_ENOMEM = -2,       /* host allocation failed */
    LBFD_EHIP = -3,         /* a HIP runtime call failed */
    LBFD_ENONFINITE = -4,   /* a non-finite total surfactant or mass was detected */
    LBFD_ESOR = -5,         /* SOR reached sor_max_sweeps above tolerance */
    LBFD_EWORKSPACE = -6,   /* workspace missing or smaller than required */
    LBFD_EUNSUPPORTED = -7, /* valid but not supported combination */
    LBFD_ESCRATCH = -8      /* request larger than the fixed scratch buffer (lbfd_read_field_noalloc) */
} lbfd_status;

typedef enum { LBFD_D2Q9 = 0, LBFD_D3Q19 = 1 } lbfd_lattice;

/* Storage precision. FP64: FP64 everywhere. FP32: FP32 storage and
 * arithmetic. FP16DEV / BF16DEV: populations stored as 16-bit deviations
 * from the local equilibrium of the node they left, all other fields FP32,
 * FP32 arithmetic. Global sums (masses, total surfactant) are FP64 in every
 * mode. */
typedef enum { LBFD_FP64 = 0, LBFD_FP32 = 1, LBFD_FP16DEV = 2, LBFD_BF16DEV = 3 } lbfd_precision;

typedef enum { LBFD_PERIODIC = 0, LBFD_WALL = 1 } lbfd_bc;

/* Parameters, lattice units. */
typedef struct {
    int32_t lattice;             /* lbfd_lattice */
    int32_t precision;           /* lbfd_precision */
    int32_t nx, ny, nz;          /* each >= 4 (nz = 1 for D2Q9); nx*ny*nz < 2^28 (FP64: < 2^27) */
    int32_t bc[3];               /* per axis x,y,z: periodic, or half-way walls at -1/2 and n-1/2 */
    double wall_u[6][3];         /* wall velocities at -x,+x,-y,+y,-z,+z */
    double rhoR0, rhoB0;         /* pure-fluid densities, red (dispersed) and blue (eq 6) */
    double muR0, muB0;           /* pure-fluid dynamic viscosities (eq 43) */
    double alphaR;               /* sound-speed parameter of red (Appendix A); blue from eq 42 */
    double beta;                 /* recolouring segregation parameter (0.7) */
    double sigma0, E0;           /* clean interfacial tension and elasticity number (eq 8) */
    double psi_inf;              /* maximum interface concentration (eq 8) */
    double sigma_min_ratio;      /* sigma_min / sigma0 (0.1, below eq 8) */
    double Ds, Db;               /* interface and bulk surfactant diffusivities (eqs 20-21) */
    double ra, rd;               /* adsorption and desorption coefficients (eq 22) */
    int32_t source_mode;         /* 0: j of eq 22; 1: adsorption only, j = ra psi_inf phi (Sec 3.1) */
    double gravity[3];           /* body force F_b = (rho - rho_ref) * gravity (Sec 3.4; see buoyancy_ref) */
    double sor_omega;            /* SOR relaxation factor (1.2 in Sec 2.2) */
    double sor_tol;              /* stop at max|residual| <= sor_tol * max|rhs| (red-black ordering;
                                    with sor_omega = 1 the test after sweep s is the red residual at
                                    the start of sweep s + 1, whose red half is then kept) */
    int32_t sor_max_sweeps;      /* sweeps launched per step; LBFD_ESOR if still above tolerance */
    double weno_eps;             /* WENO3 epsilon (1e-6, Sec 2.2) */
    int32_t rescale;             /* 1: restore the initial total surfactant each step */
    int32_t fd_enable;           /* 0: psi and phi frozen (flow only) */
    int32_t q_literal;           /* 3-D correction factor: 0 = 1 - 3 cs^2, 1 = printed 1 - cs^2 */
    double eps_n;                /* regularisation of the interface normal (1e-12) */
    int32_t recolour_literal;    /* recolouring weight: 0 = local rest equilibrium, 1 = lattice w_i */
    double fd_eps;               /* background support added to the FD weights G and X (1e-10 FP64,
                                    1e-6 FP32): keeps psi, phi defined where the interface delta
                                    function and the bulk indicator of eqs 20-21 vanish */
    double upwind_eps;           /* |u_a| <= upwind_eps weighs both WENO differences by 1/2 (eq 25 is
                                    0/0 at u = 0); 1e-12 keeps rounding noise out of the upwind choice */
    int32_t buoyancy_ref;        /* F_b = (rho - rho_ref) gravity with rho_ref = rhoB0 (0, as printed in
                                    Sec 3.4) or the mean density of the domain (1: no net force on a
                                    periodic domain; fixed when the fields are initialised or set) */
    int32_t eos_mode;            /* 0: Langmuir law of eq 8, floored at sigma_min beyond the CMC;
                                    1: linear law sigma = sigma0 (1 - E0 psi / psi_inf) of Sec 3.2 */
} lbfd_params;

/* Initial state: up to 16 red drops or bubbles with a tanh colour profile of
 * width `width`, uniform psi0, bulk phi0_out outside (rhoN < 0) and phi0_in
 * inside, and an optional linear shear flow u_x = shear_rate (y - (ny-1)/2). */
typedef struct {
    int32_t n;
    double cx[16], cy[16], cz[16], r[16];
    double width;
    double psi0, phi0_out, phi0_in;
    double shear_rate;
} lbfd_init;

/* Observables of the current state, all FP64. */
typedef struct {
    int64_t step;
    double mass_R, mass_B;       /* sums of rho^R and rho^B */
    double total_surf;           /* sum of (G psi + X phi), G = |grad rhoN| + fd_eps, X = 1 - rhoN + fd_eps */
    double drift_pre;            /* relative change of total_surf in the last step before rescaling */
    double velocity[3];          /* eq 33 per component: sum u N / sum N, N = [rhoN >= 0] (eq 34) */
    double centroid[3];          /* weight (1 + rhoN)/2 */
    double second[6];            /* central second moments xx,yy,zz,xy,xz,yz, same weight */
    double wsum, nsum;           /* sum of the weight, sum of N */
    double psi_av;               /* sum G psi / sum G */
    double psi_min, psi_max;     /* over nodes with |rhoN| <= 0.5 */
    double p_in, p_out;          /* mean sum_k rho^k (cs^k)^2 over rhoN > 0.99 and rhoN < -0.99 */
    double deformation;          /* (L - B)/(L + B) from the second-moment eigenvalues */
    int32_t sor_sweeps[2];       /* full sweeps after which psi and phi met the tolerance (last step) */
    int32_t status;              /* sticky device error status (lbfd_status) */
} lbfd_obs;

/* Field identifiers for lbfd_read_field. Counts are per node. */
typedef enum {
    LBFD_FIELD_F = 0,      /* total populations f_i (Q), after propagation */
    LBFD_FIELD_RHOR = 3,   /* rho^R (1) */
    LBFD_FIELD_RHOB = 4,   /* rho^B (1) */
    LBFD_FIELD_RHON = 5,   /* colour function rhoN (1) */
    LBFD_FIELD_U = 6,      /* fluid velocity (D) */
    LBFD_FIELD_PSI = 7,    /* interface surfactant psi (1), rescaled */
    LBFD_FIELD_PHI = 8,    /* bulk surfactant phi (1), rescaled */
    LBFD_FIELD_FORCE = 9,  /* interfacial + body force (D) */
    LBFD_FIELD_G = 10,     /* |grad rhoN| (1) */
    LBFD_FIELD_SPREV = 11, /* S at the previous step (1), for the AB2 term of eq 24 */
    LBFD_FIELD_BPREV = 12  /* B at the previous step (1) */
} lbfd_field;

typedef struct lbfd_handle lbfd_handle;

/* Bytes of device workspace the parameters need (256-byte aligned). */
int lbfd_workspace_bytes(const lbfd_params *p, size_t *bytes);

/* Validate parameters and bind a handle to a caller-owned device workspace
 * (d_workspace, at least lbfd_workspace_bytes) and stream. *out is set on
 * success. Errors: EINVAL (shape < 4, non-positive density or viscosity,
 * alpha outside (0,1), unknown lattice/precision), EWORKSPACE, ENOMEM. */
int lbfd_create(const lbfd_params *p, void *d_workspace, size_t bytes, void *stream, lbfd_handle **out);

/* Initial fields (see lbfd_init) on the device; sets the step counter to 0
 * (so the first FD step is the Euler step of eq 23) and records the initial
 * total surfactant as the rescaling target. Asynchronous. */
int lbfd_init_fields(lbfd_handle *h, const lbfd_init *init);

/* Replace the state: populations f (Q*N), rhoR and rhoB (N each, the colour
 * split of f), psi, phi, and the previous-step sources Sprev, Bprev (N each;
 * NULL = zero). `step` selects eq 23 (0) or eq 24 (>0); M0 is the rescaling
 * target. Synchronises the stream. */
int lbfd_set_state(lbfd_handle *h, const double *f, const double *rhoR, const double *rhoB,
                   const double *psi, const double *phi, const double *Sprev, const double *Bprev,
                   int64_t step, double M0);

/* Advance n >= 0 time steps. Asynchronous; errors found on the device are
 * reported by the next synchronising call. */
int lbfd_step(lbfd_handle *h, int64_t n);

/* Compute the observables of the current state (FP64 reductions on the
 * device) into *out. Synchronises the stream. */
int lbfd_observables(lbfd_handle *h, lbfd_obs *out);

/* Copy one field of the current state to host memory as FP64; `count`
 * must equal components * nodes. Synchronises the stream. */
int lbfd_read_field(lbfd_handle *h, int32_t field, double *host, size_t count);

/* lbfd_read_field without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). The field is converted to FP64 in a fixed device staging
 * array owned by the library (one per device, LBFD_SCRATCH_DOUBLES doubles =
 * 64 MiB, held until the process ends) and copied to `host`; arguments and
 * result are those of lbfd_read_field. The call allocates nothing: no hipMalloc,
 * hipFree or allocating library routine. All calls on one device share that
 * array and it keeps the last call's contents, so calls that overlap on one
 * device (from several host threads or handles) race; serialise them.
 * Synchronises the handle's stream. Errors: EINVAL (unknown field, count not
 * components * nodes, null pointer), ESCRATCH (count > LBFD_SCRATCH_DOUBLES;
 * use lbfd_read_field), EHIP. */
#define LBFD_SCRATCH_DOUBLES ((size_t)8 << 20)
int lbfd_read_field_noalloc(lbfd_handle *h, int32_t field, double *host, size_t count);

/* Per-kernel timing with HIP events on the handle's stream: enable (non-zero)
 * or disable (0); enabling clears the accumulators. enable = 1 times every
 * kernel class; enable = 1 | (mask << 1) times only the classes whose bits
 * are set in mask (class k = the k-th name reported by lbfd_profile_read),
 * which keeps the event overhead off the other launches. */
int lbfd_profile(lbfd_handle *h, int32_t enable);

/* Accumulated milliseconds and launch counts per kernel class since the last
 * lbfd_profile(h, 1); names[k] point to static strings. Synchronises. */
int lbfd_profile_read(lbfd_handle *h, int32_t max_kernels, const char **names, double *ms, int64_t *launches,
                      int32_t *n_kernels);

/* Overwrite one FD field from count = N FP64 host values in node order:
 * LBFD_FIELD_PSI or LBFD_FIELD_PHI (physical values; the force is recomputed
 * from the new psi) or LBFD_FIELD_SPREV / LBFD_FIELD_BPREV (the AB2 source
 * histories of eq 24). The rescaling target M0 is kept. Other fields:
 * LBFD_EUNSUPPORTED (use lbfd_set_state). Synchronous. Errors: EINVAL (count
 * or null pointer), EHIP. */
int lbfd_write_field(lbfd_handle *h, int32_t field, const double *host, size_t count);

/* Advance psi and phi by k >= 0 FD updates (Sec 2.2, eqs 20-28) with the flow
 * frozen at the current state: rhoN, G and u of the current populations, the
 * weights of the new time level equal to those of the current one. The LB
 * populations and the step count do not change; the force is recomputed from
 * the new psi. The quantity the learned surrogate approximates, and its
 * fallback. No-op when fd_enable is 0. Errors: EINVAL (null handle, k < 0). */
int lbfd_fd_substeps(lbfd_handle *h, int64_t k);

/* Switch the FD part of lbfd_step off (enable = 0: the LB part advances with
 * psi and phi held, as between the updates of the learned surrogate) or back
 * on (the default). Errors: EINVAL (null handle). */
int lbfd_set_fd(lbfd_handle *h, int32_t enable);

/* Graph replay of lbfd_step (enable != 0, the default) or plain launches
 * (enable = 0). A call that advances four or more steps, with profiling off,
 * records two steps once per buffer-role state into a HIP graph (captured on
 * a private stream of default priority) and replays it on the handle's
 * stream; steps before the second one, or before an extrapolation history
 * exists, and an odd last step are launched directly. The results are
 * identical either way. Errors: EINVAL (null handle). */
int lbfd_set_graphs(lbfd_handle *h, int32_t enable);

/* Launch shape of the solver's kernels: a tuning choice that never changes the
 * results (every node's arithmetic and the red-black order of the solve are the
 * same; the FP64 reductions keep their own fixed shape). */
typedef struct {
    int32_t rows;           /* workgroups of the step's node kernels: 64 x rows nodes, rows = 1, 2 or 4
                               (default 4) */
    int32_t sor_wg_per_cu;  /* persistent grid of the SOR half-sweeps: workgroups of 256 per compute unit,
                               1..32 (default 8), capped at one per 256 nodes of a colour */
    int32_t sor_narrow;     /* workgroups of the sweeps past the third (they usually only find the systems
                               converged): 8..65536, a multiple of 8 (default 256) */
} lbfd_tuning;

/* Set or read a handle's launch shape (lbfd_set_tuning synchronises the stream
 * and drops captured graphs). Errors: EINVAL (null pointer, value out of range),
 * EHIP. */
int lbfd_set_tuning(lbfd_handle *h, const lbfd_tuning *t);
int lbfd_get_tuning(const lbfd_handle *h, lbfd_tuning *t);

/* Release the handle (not the caller's workspace or stream). */
void lbfd_destroy(lbfd_handle *h);

/* Static description of a status code. */
const char *lbfd_strerror(int status);

/* ---- Batches: independent instances stepped together ----------------------
 *
 * A batch holds n independent instances (a parameter sweep of uneven grids,
 * say), each an ordinary handle on its own slice of one caller-owned device
 * workspace, and advances all of them with one launch per kernel class instead
 * of one per instance. The method per instance is unchanged: the same time
 * step as lbfd_step. The instances share the lattice, the precision,
 * fd_enable and sor_max_sweeps; grid sizes, boundaries and physical parameters
 * are free. Each instance is initialised, observed and read through the
 * single-instance calls on the handle lbfd_batch_instance returns (those calls
 * synchronise the batch's stream); it is not stepped on its own. */
typedef struct lbfd_batch lbfd_batch;

/* Bytes of device workspace for a batch of the n parameter blocks p[0..n-1]. */
int lbfd_batch_workspace_bytes(const lbfd_params *p, int32_t n, size_t *bytes);

/* Create a batch on a caller-owned workspace (256-byte aligned, at least
 * lbfd_batch_workspace_bytes) and stream. Errors: EINVAL (n outside 1..65536,
 * an invalid parameter block, or lattice, precision, fd_enable or
 * sor_max_sweeps differing between instances), EWORKSPACE, ENOMEM, EHIP. */
int lbfd_batch_create(const lbfd_params *p, int32_t n, void *d_workspace, size_t bytes, void *stream,
                      lbfd_batch **out);

/* Handle of instance i (owned by the batch), or NULL when i is out of range. */
lbfd_handle *lbfd_batch_instance(lbfd_batch *b, int32_t i);

/* Advance every instance n >= 0 steps. All instances must be at the same step
 * (initialised, or set to the same step, together), else EINVAL. Asynchronous. */
int lbfd_batch_step(lbfd_batch *b, int64_t n);

/* Launch shape of every instance of a batch: `rows` for the node kernels and
 * `sor_narrow` for the SOR sweeps past the third, which run over the instances
 * still converging (the first three sweeps launch one workgroup per SOR tile of
 * every instance, so `sor_wg_per_cu` does not change the batch's launches).
 * Errors: EINVAL, EHIP. */
int lbfd_batch_set_tuning(lbfd_batch *b, const lbfd_tuning *t);

/* Graph replay of lbfd_batch_step, as lbfd_set_graphs for one handle. */
int lbfd_batch_set_graphs(lbfd_batch *b, int32_t enable);

/* Release the batch and its instance handles (not the workspace or stream). */
void lbfd_batch_destroy(lbfd_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LBFD_H */
