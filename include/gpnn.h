/*
 * gpnn.h -- C-ABI of the warm-start network for imaginary-time ground-state searches:
 * a small 3D convolutional decoder, trained on ground states produced by the
 * split-step Crank-Nicolson solver (gp.h), that maps a problem's trap and
 * nonlinearity (nu_x, nu_y, nu_z, g) to a positive ground-state guess psi on the
 * solver's grid.  The paper's method starts imaginary-time propagation from a
 * Gaussian (program summary (i)); this network only changes the starting state, the
 * propagation that follows is the paper's.  Forward and backward passes run on
 * gfx950 BF16 matrix cores (MFMA) with FP32 accumulation; weights are FP32 masters with
 * BF16 copies; training uses Adam (Kingma and Ba, Algorithm 1).
 *
 * Network (nsteps = number of x2 upsampling stages S, channels ch[0..S]):
 *   z0 = (nu_x, nu_y, nu_z, ln g) standardised by in_mean / in_std
 *   a1 = silu(W1 z0 + b1)                       W1 [hidden][4]
 *   a2 = silu(W2 a1 + b2)                       W2 [base^3 ch0][hidden]; a2 read as a
 *                                               [base][base][base][ch0] volume
 *   stage s: u = nearest x2 upsampling of a;  a = silu(conv3x3x3(u; Cs) + cs)
 *                                               Cs [27][ch_s][ch_{s-1}], zero padding,
 *                                               tap t = (a*3+b)*3+c for offset (a-1,b-1,c-1)
 *   f = wh . a_S + bh + ln G,  psi = exp(min(f, 10))
 *   ln G = 1/4 sum ln(nu/pi) - 1/2 sum nu x^2 (the normalised Gaussian ground state at g=0),
 *   x_i = (i - (N-1)/2) dx, N = base * 2^S.
 * Loss: L = (1/n) sum_samples dx^3 sum_points (psi - target)^2.
 *
 * Parameter vector (FP32, this order): W1, b1, W2, b2, then per stage Cs, cs, then wh
 * [ch_S], bh [1].  Activations are BF16, channels last ([sample][x][y][z][channel]).
 *
 * Requirements: hidden and ch[0..S] multiples of 16, ch[S] in {16, 32, 64}; 1 <= S <= 6;
 * base >= 1; N <= 1024; max_batch >= 1.  Violations return GPNN_ERR_INVALID.
 *
 * Ownership: the model owns its parameters, gradients, Adam moments, BF16 copies and
 * activation buffers (sized for max_batch).  Inputs and outputs are caller device
 * buffers.  The stream is borrowed; calls are stream-ordered and do not synchronise
 * unless stated.  A model is not thread-safe.  Return codes: 0 or a negative
 * GPNN_ERR_*; nothing aborts or prints.
 */
#ifndef GPNN_H
#define GPNN_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { GPNN_OK = 0, GPNN_ERR_INVALID = -1, GPNN_ERR_HIP = -2, GPNN_ERR_OOM = -3, GPNN_ERR_STATE = -4 };

typedef struct gpnn gpnn;

typedef struct {
  int32_t base;        /* edge of the first feature volume */
  int32_t hidden;      /* width of the hidden dense layer */
  int32_t nstage;      /* S */
  int32_t ch[7];       /* ch[0..S] */
  int32_t max_batch;   /* largest n accepted by gpnn_forward */
  double dx;           /* spacing of the output grid */
  double in_mean[4], in_std[4];
} gpnn_arch;

int gpnn_create(const gpnn_arch* a, void* hip_stream, gpnn** out);
int gpnn_destroy(gpnn* m);
/* number of FP32 parameters */
int gpnn_param_count(gpnn* m, int64_t* n);
/* copy all parameters from host memory (n FP32 in the documented order); resets the
 * Adam moments and refreshes the BF16 copies.  Synchronises. */
int gpnn_set_params(gpnn* m, const float* host, int64_t n);
/* copy parameters / gradients of the last gpnn_loss_backward to host memory.  Synchronises. */
int gpnn_get_params(gpnn* m, float* host, int64_t n);
int gpnn_get_grads(gpnn* m, float* host, int64_t n);

/* Forward pass for n <= max_batch problems.  params_dev: n x 4 FP32 device array of raw
 * (nu_x, nu_y, nu_z, g), nu > 0, g > 0.  out_dev: n x N^3 values, FP32
 * (out_complex64 = 0), complex64 (1) or complex128 (2) with zero imaginary part, laid out
 * as the solver's psi ([x][y][z], z fastest), so a complex output can start the solver
 * in place.  The activations are kept for gpnn_loss_backward / gpnn_backward (FP32
 * output only); out_dev must stay valid until then. */
int gpnn_forward(gpnn* m, const float* params_dev, int32_t n, void* out_dev, int32_t out_complex64);
/* Loss against target_dev (n x N^3 FP32, same layout) for the last forward pass (which
 * must have written FP32 output), and the gradient of the loss with respect to every
 * parameter (overwritten, not accumulated).  loss (nullable, host): the loss;
 * synchronises when given. */
int gpnn_loss_backward(gpnn* m, const float* target_dev, double* loss);
/* Backward pass of the last forward pass (which must have written FP32 output) from an
 * upstream gradient: grad_psi_dev (n x N^3 FP32, the output's layout) holds dL/dpsi for
 * whatever loss the caller computes.  Every parameter gradient is overwritten (not
 * accumulated; the caller sums several passes on the host if it needs to).  With
 * dL/dpsi = 2 (psi - t) dx^3 / n it gives gpnn_loss_backward's gradients.  No sync. */
int gpnn_backward(gpnn* m, const void* grad_psi_dev);
/* One Adam update of every parameter with the gradients of the last backward pass;
 * t >= 1 is the update count (bias correction).  Refreshes the BF16 copies. */
int gpnn_adam_step(gpnn* m, float lr, float beta1, float beta2, float eps, int64_t t);

/* Kernel-level entry points (device pointers, BF16 as uint16 bit patterns), used by
 * the tests to check each kernel; they allocate temporaries and synchronise.
 *
 * gpnn_conv: y[p, o] = act(sum_t sum_i w[t, o, i] x[p + off_t, i] + bias[o]) * gate'
 *   ks = 3: x [n][d][d][d][cin], 27 taps; ks = 1: x [n][cin], one tap (dense layer).
 *   bias nullable; act 0 = identity, 1 = silu; gate (nullable, [n..][cout] BF16): when
 *   given, the result is multiplied by silu'(gate) instead (backward through silu);
 *   pre (nullable) receives the value before the activation.  cin multiple of 16,
 *   cout multiple of 16.
 * gpnn_conv_wgrad: dw[t, o, i] = sum_p dy[p, o] x[p + off_t, i] (FP32 [taps][cout][cin]),
 *   db[o] = sum_p dy[p, o] (nullable). */
int gpnn_conv(int32_t ks, int32_t n, int32_t d, int32_t cin, int32_t cout, const void* x, const void* w,
              const float* bias, int32_t act, const void* gate, void* y, void* pre, void* hip_stream);
int gpnn_conv_wgrad(int32_t ks, int32_t n, int32_t d, int32_t cin, int32_t cout, const void* dy, const void* x,
                    float* dw, float* db, void* hip_stream);

const char* gpnn_last_error(gpnn* m);

#ifdef __cplusplus
}
#endif
#endif
