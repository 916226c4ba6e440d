/* Learned surrogate of k frozen-flow FD substeps: C ABI of liblbfd.so.
 *
 * A method addition (the paper has no surrogate). The FD update of Sec 2.2
 * (eqs 20-28) applied k times with the flow held at the current state (the
 * operation lbfd_fd_substeps performs) is approximated by a small network:
 * four 3x3x3 "valid" convolutions, channels 6 -> 32 -> 32 -> 32 -> 7, ReLU
 * after the first three, BF16 weights and activations with FP32 accumulation
 * on the matrix cores, FP32 master weights trained with Adam.
 *
 * Inputs per node (channels-last, BF16, padded to 16 channels with zeros):
 * psi/psi_inf, phi/phi_s, rhoN, u_x/u_s, u_y/u_s, u_z/u_s (u_z = 0 in 2-D).
 * Outputs per node (FP32, 7 channels), read in a conservative form: flux
 * coefficients f_psi,a and f_phi,a (a = x, y, z) and an exchange s. With the
 * weights of eqs 20-21 held over the substeps, W = G + fd_eps and X = 1 - rhoN +
 * fd_eps, the flux of W psi through the face between n and n + e_a is
 * (W[n] + W[n + e_a])/2 f_psi,a[n] (likewise X phi with X), the exchange from
 * bulk to interface at n is W[n] s[n], and the changes over the k substeps are
 *   W dpsi = dpsi_s (W s - sum_a (face flux out - face flux in)),
 *   X dphi = dphi_s (- sum_a (face flux out - face flux in)) - dpsi_s W s,
 * so the total surfactant sum (W psi + X phi) is conserved by construction on
 * a periodic grid. Grids are (z, y, x) with x fastest; an input grid of
 * d x h x w nodes gives (d-8) x (h-8) x (w-8) outputs. A training tile of T^3
 * outputs is scored on its interior [1, T-2]^3, where every face it needs lies
 * in the tile.
 *
 * Parameter vector (FP32, lbfd_sg_n_params() entries): for each layer in turn
 * the weights w[a][p][q][i][o] (tap offsets a, p, q in z, y, x; input channel
 * i; output channel o) in row-major order, then the biases b[o].
 *
 * Device pointers are on the device of the stream given at creation. Calls
 * are asynchronous on that stream unless they return host data.
 * Errors: LBFD_EINVAL (bad sizes, null pointers, or a solver grid that is not
 * periodic on every axis for the whole-field calls), LBFD_EWORKSPACE,
 * LBFD_ENOMEM, LBFD_EHIP. */
#ifndef LBFD_SURROGATE_H
#define LBFD_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#include "lbfd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbfd_sg lbfd_sg;

typedef struct {
    int32_t tile;       /* output edge of a training tile (its input edge is tile + 8), 3..64 */
    int32_t max_batch;  /* most tiles per lbfd_sg_gradient / lbfd_sg_train_step / lbfd_sg_tiles call, >= 1,
                           with max_batch (tile + 6)^3 < 2^31 (LBFD_EINVAL otherwise) */
    int32_t field[3];   /* largest solver grid (nx, ny, nz) for the whole-field calls; 0s: none */
    int32_t k;          /* FD substeps one application replaces (>= 1) */
    double lr, beta1, beta2, adam_eps;             /* Adam */
    double psi_inf, phi_s, u_s, dpsi_s, dphi_s;    /* channel scales (all > 0) */
    double drift_tol;   /* lbfd_sg_advance falls back to the FD update when the network's
                           update changes the total surfactant (at the frozen weights,
                           before any rescaling) by more than this relative amount, or
                           when it is implausible: not finite, or a change of psi (phi)
                           above 20 dpsi_s (20 dphi_s) where W (X) >= 1e-3 */
} lbfd_sg_params;

typedef struct {
    int64_t blocks;     /* surrogate applications attempted */
    int64_t accepted;   /* applications kept */
    int64_t fallbacks;  /* applications replaced by lbfd_fd_substeps */
    double max_drift;   /* largest |pre-rescale drift| of a kept application */
    double last_drift;  /* drift of the last application (kept or not) */
} lbfd_sg_report;

/* Number of FP32 parameters (66631). */
int64_t lbfd_sg_n_params(void);

/* Device workspace for the surrogate described by p. */
int lbfd_sg_workspace_bytes(const lbfd_sg_params *p, size_t *bytes);

/* Create on a caller-owned workspace (256-byte aligned, at least
 * lbfd_sg_workspace_bytes) and stream. Weights start at zero: load them with
 * lbfd_sg_set_params. */
int lbfd_sg_create(const lbfd_sg_params *p, void *d_workspace, size_t bytes, void *stream, lbfd_sg **out);

/* Master weights from / to host memory (n = lbfd_sg_n_params()). Setting them
 * resets the Adam moments and the step count. Synchronous. */
int lbfd_sg_set_params(lbfd_sg *s, const float *host, int64_t n);
int lbfd_sg_get_params(lbfd_sg *s, float *host, int64_t n);

/* Network on B grids of d x h x w input nodes (d_in: BF16 bit patterns,
 * [B][d][h][w][16]); d_out: FP32 [B][d-8][h-8][w-8][7]. B * d * h * w and
 * the intermediate grids must fit the workspace (the tile batch or the
 * whole-field grid it was sized for). */
int lbfd_sg_forward(lbfd_sg *s, const uint16_t *d_in, int32_t B, int32_t d, int32_t h, int32_t w, float *d_out);

/* Mean squared error of the network's conservative form on B training tiles
 * (d_in as above with d = h = w = tile + 8; d_target: FP32
 * [B][tile][tile][tile][4] = (W dpsi / dpsi_s, X dphi / dphi_s, W, X) per
 * output node, as lbfd_sg_tiles writes it), over both fields and the tiles'
 * interior nodes, and its gradient in parameter order (host, n entries).
 * Synchronous. */
int lbfd_sg_gradient(lbfd_sg *s, const uint16_t *d_in, const float *d_target, int32_t B, double *loss,
                     float *host_grad, int64_t n);

/* One Adam step on B training tiles; *loss (if not NULL) receives the loss
 * before the step (synchronous only when loss is not NULL). */
int lbfd_sg_train_step(lbfd_sg *s, const uint16_t *d_in, const float *d_target, int32_t B, double *loss);

/* Input channels of the solver's current state on its grid with a periodic
 * halo of 4 nodes: d_feat is BF16 [nz+8][ny+8][nx+8][16] (2-D: nz = 1, the
 * single plane repeated). */
int lbfd_sg_features(lbfd_handle *h, lbfd_sg *s, uint16_t *d_feat);

/* The solver's current psi and phi (physical values, FP32 [N][2]). */
int lbfd_sg_snapshot(lbfd_handle *h, lbfd_sg *s, float *d_snap);

/* Training tiles: inputs cropped from a feature grid (as lbfd_sg_features
 * wrote it) and targets over the tile's output nodes: the changes of the
 * conserved densities, W (psi now - d_snap psi) / dpsi_s and
 * X (phi now - d_snap phi) / dphi_s, and the weights W, X of the current state
 * (FP32 [B][tile][tile][tile][4]). Tile b has its output corner
 * at node (org[3b], org[3b+1], org[3b+2]) = (x, y, z) with x + tile <= nx,
 * y + tile <= ny, z + tile <= nz (so training tiles come from 3-D grids). */
int lbfd_sg_tiles(lbfd_handle *h, lbfd_sg *s, const uint16_t *d_feat, const float *d_snap,
                  const int32_t *host_org, int32_t B, uint16_t *d_in, float *d_target);

/* Advance the solver by nblocks blocks of k steps in surrogate mode. Each
 * block first advances psi and phi by k frozen-flow substeps with the network
 * (whole grid, one application, in the conservative form above) and checks the
 * change it makes to the total surfactant before any rescaling against
 * drift_tol, and its plausibility (see drift_tol); if a check fails the
 * network's result is
 * discarded and lbfd_fd_substeps(k) is applied instead. Then the lattice
 * Boltzmann part advances k steps with psi and phi held (lagged coupling).
 * rep (if not NULL) accumulates counts over the call. Synchronises once per
 * block (the drift check is read on the host). */
int lbfd_sg_advance(lbfd_handle *h, lbfd_sg *s, int64_t nblocks, lbfd_sg_report *rep);

/* Change the fallback threshold of lbfd_sg_advance (tol >= 0). */
int lbfd_sg_set_drift_tol(lbfd_sg *s, double tol);

/* Change the Adam step size used by the following lbfd_sg_train_step calls
 * (finite lr > 0, else LBFD_EINVAL); the moments and the step count are kept, so a
 * caller can decay the step size over a training run. */
int lbfd_sg_set_lr(lbfd_sg *s, double lr);

/* Release the surrogate (not the workspace or stream). */
void lbfd_sg_destroy(lbfd_sg *s);

#ifdef __cplusplus
}
#endif

#endif
