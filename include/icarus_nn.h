/*
 * icarus_nn.h -- C-ABI of the warm-start network (not in the paper).
 *
 * The paper relaxes the heliosphere for 8 simulated days before the period
 * of interest (Sect. 3: relaxation time = slow-wind crossing time to the
 * outer boundary).  This network maps a 0.1 AU boundary map to an initial
 * state close to the relaxed wind, so that the relaxation needs fewer steps;
 * the plain radial-expansion start (Sect. 2.1) remains the fallback.
 *
 * Network per sample, on the (theta, phi) grid of the map:
 *   features X [n_theta][n_phi][C], C = 8 normalised boundary primitives,
 *   plus (coord = 1) two colatitude channels t and 2 t^2 - 1, t running
 *   from -1 to 1 across the grid's colatitude range, so the encoder knows
 *   how far a column sits from the theta boundaries
 *   conv 3 x nk C -> c1, SiLU, over colatitude offsets -1..1 and longitude
 *   offsets phi_lo..phi_hi (nk = phi_hi - phi_lo + 1): plasma at longitude
 *   phi and radius r left the inner boundary at phi + Omega (r - r_in) / v_r
 *   in the co-rotating frame, so a window reaching far to positive offsets
 *   sees the footpoints of every radius;
 *   conv 3x3 c1 -> c2, SiLU   (both periodic in phi, edge-clamped in theta)
 *   per (theta, phi) column: Linear c2 -> hidden, SiLU; Linear hidden -> n_r*8
 *   output Y [n_theta*n_phi][n_r][8]: normalised residual of the state over
 *   the radial expansion of the map (log-ratio for rho and p, offsets in
 *   units of 100 km/s for velocities, of |B_r|+|B_phi| of the expansion for B).
 * Products: BF16 operands on MFMA with FP32 accumulation.  Parameters: FP32
 * masters (updated by Adam) with BF16 copies used by the products.
 * Parameter vector order: W1 [3*nk*C][c1], b1 [c1], W2 [9*c1][c2], b2 [c2],
 * W3 [c2][hidden], b3 [hidden], W4 [hidden][n_r*8], b4 [n_r*8]; weights
 * row-major [in][out]; conv input index = tap*C + channel with
 * tap = (dtheta+1)*nk + (dphi-phi_lo) (nk = 3, phi_lo = -1 in the second
 * convolution).
 *
 * Conventions: as in icarus_hip.h (status codes, caller-owned 256-byte
 * aligned device workspace, work enqueued on the given HIP stream).  "dev"
 * pointers are device memory, "host" pointers host memory.
 */
#ifndef ICARUS_NN_H
#define ICARUS_NN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ICR_NN_OK = 0, ICR_NN_ERR_ARG = -1, ICR_NN_ERR_HIP = -4 };

typedef struct {
  int n_theta, n_phi, n_r;  /* grid of the solver the network serves      */
  int c1, c2, hidden;       /* encoder channels and decoder width         */
  int batch_max;            /* samples per forward/backward call          */
  int phi_lo, phi_hi;       /* first-layer longitude offsets, inclusive:
                               phi_lo <= 0 <= phi_hi, window <= n_phi     */
  int coord;                /* 1: two colatitude input channels (C = 10),
                               0: none (C = 8)                            */
} icr_nn_shape;

typedef struct icr_nn icr_nn;

const char *icr_nn_last_error(void);
int icr_nn_param_count(const icr_nn_shape *shape, long long *n);
int icr_nn_workspace_bytes(const icr_nn_shape *shape, size_t *bytes);
int icr_nn_create(const icr_nn_shape *shape, void *dev_workspace, size_t bytes,
                  void *hip_stream, icr_nn **out);
void icr_nn_destroy(icr_nn *n);

/* FP32 parameters (host, param_count floats); setting resets Adam. */
int icr_nn_set_params(icr_nn *n, const float *host);
int icr_nn_get_params(icr_nn *n, float *host);

/* Forward pass of `batch` samples: x_dev [batch][n_theta][n_phi][8] FP32,
 * y_dev [batch][n_theta*n_phi][n_r*8] FP32 (NULL: keep on the device). */
int icr_nn_forward(icr_nn *n, int batch, const float *x_dev, float *y_dev);

/* Forward + backward of the mean squared error against t_dev (same layout
 * as y).  The gradients stay on the device for icr_nn_adam_step; loss
 * (host, may be NULL) and grad_host (param_count floats, may be NULL)
 * receive copies. */
int icr_nn_loss_grad(icr_nn *n, int batch, const float *x_dev,
                     const float *t_dev, double *loss, float *grad_host);

/* One Adam step with bias correction on the FP32 masters. */
int icr_nn_adam_step(icr_nn *n, float lr, float beta1, float beta2, float eps);

/* Features of `batch` SI maps [batch][8][n_theta][n_phi] (dev) with
 * colatitude centres thc_dev [n_theta]: ln(rho/rho0), v_r/100 km/s - 5,
 * v_theta/100 km/s, inertial v_phi/100 km/s, ln(p/p0), B/250 nT, then with
 * coord = 1 the colatitude channels t, 2 t^2 - 1 (t = -1 at the first
 * colatitude centre, 1 at the last); x_dev [batch][n_theta][n_phi][C]. */
int icr_nn_encode_map(icr_nn *n, int batch, const double *maps_dev,
                      const double *thc_dev, double omega, double r_in,
                      float *x_dev);

/* Training target from a primitive SI state [8][n_phi][n_theta][n_r] (dev)
 * and its map [8][n_theta][n_phi] (dev); rc_dev: cell-centre radii [n_r] m. */
int icr_nn_encode_target(icr_nn *n, const double *map_dev, const double *state_dev,
                         const double *rc_dev, const double *thc_dev, double omega,
                         double r_in, double gamma, float *t_dev);

/* Inverse: primitive SI state (dev) from a network output y_dev (one sample). */
int icr_nn_decode_state(icr_nn *n, const double *map_dev, const float *y_dev,
                        const double *rc_dev, const double *thc_dev, double omega,
                        double r_in, double gamma, double *state_dev);

/* The BF16 MFMA product used by the network, for tests:
 * C[m][n] = sum_k A(m,k) B(k,n) (+ bias[n]) with A(m,k) = A[m*lda+k]
 * (trans_a = 0) or A[k*lda+m] (trans_a = 1), B(k,n) = B[k*ldb+n]
 * (trans_b = 0) or B[n*ldb+k] (trans_b = 1); A, B BF16 bit patterns, C FP32. */
int icr_nn_gemm_bf16(int trans_a, int trans_b, int M, int N, int K, const void *A,
                     int lda, const void *B, int ldb, float *C, int ldc,
                     const float *bias, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* ICARUS_NN_H */
