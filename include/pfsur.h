/*
 * pfsur.h -- C ABI of the learned 16-step surrogate that runs beside the phase-field
 * lattice Boltzmann solver (libpflb), on AMD gfx950 with BF16 matrix cores.
 *
 * The surrogate is not part of the paper.  It maps the macroscopic state (phi, P, rho u)
 * of a D2Q9 periodic domain at step n to the state at step n + 16 through a 4-level
 * convolutional U-Net (17 circular-padded 3x3 convolutions with 32/64/128/256 channels
 * and SiLU, 2x2 average pooling, nearest 2x upsampling with skip concatenation, and a
 * 1x1 head predicting the normalised residual).  Convolutions are implicit GEMMs on
 * BF16 MFMA with FP32 accumulation; weights are kept as FP32 masters with BF16 copies.
 * The plain lattice Boltzmann step is the fallback and the reference for the surrogate's
 * error (pflb_advance_guarded).
 *
 * Conventions (as in pflb.h): device pointers unless stated "host"; the caller owns
 * activations, batches and workspaces; the library owns the weights and optimiser
 * state of a context.  Tensors are NHWC: [B][H][W][C], C fastest.  Returns 0 or a
 * negative PFLB_ERR_* code.  A context is not safe for concurrent calls from several
 * host threads; calls on one stream are ordered.
 */
#ifndef PFSUR_H
#define PFSUR_H

#include <stddef.h>

#include "pflb.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PFSUR_IN_CH   8   /* input channels: phi, P, J_x, J_y, log10(rho_H/rho_L), 3 zero */
#define PFSUR_OUT_CH  4   /* output channels: normalised residual of phi, P, J_x, J_y    */
#define PFSUR_STEPS  16   /* lattice Boltzmann steps one surrogate application replaces  */

/* Geometry and the normalisation of the fields.
 *   H, W         grid (multiples of 8, >= 16)
 *   max_batch    largest batch a workspace is sized for (>= 1)
 *   in_shift[4], in_scale[4]   x_c = (field_c - shift_c) * scale_c for phi, P, J_x, J_y
 *   out_scale[4] field_c(n+16) = field_c(n) + out_c * out_scale[c]
 *   lrr_scale    channel 4 = log10(rho_H / rho_L) * lrr_scale */
typedef struct pfsur_cfg {
    int H, W;
    int max_batch;
    float in_shift[4];
    float in_scale[4];
    float out_scale[4];
    float lrr_scale;
} pfsur_cfg;

typedef struct pfsur_ctx pfsur_ctx;

/* Number of FP32 parameters: for every 3x3 layer in network order (e0a, e0b, e1a, e1b,
 * e2a, e2b, b3a, b3b, u2, d2a, d2b, u1, d1a, d1b, u0, d0a, d0b) its weights
 * [Cout][3][3][Cin] then its bias [Cout]; then the head's [4][32] and [4]. */
size_t pfsur_num_params(void);

/* Create a context on the current device: allocates the FP32 master weights, their
 * BF16 copies and the Adam moments (zero weights until pfsur_set_params). */
int pfsur_create(const pfsur_cfg* cfg, pfsur_ctx** out);
void pfsur_destroy(pfsur_ctx* ctx);
const char* pfsur_last_error(const pfsur_ctx* ctx);

/* Parameters to / from a HOST float array of pfsur_num_params() values (layout above).
 * Setting parameters also resets the Adam state. */
int pfsur_set_params(pfsur_ctx* ctx, const float* host);
int pfsur_get_params(pfsur_ctx* ctx, float* host);

/* Bytes of the caller's device workspace for a batch (training = 1: forward
 * activations plus the backward buffers). */
size_t pfsur_workspace_bytes(const pfsur_cfg* cfg, int batch, int training);

/* Where 3x3 layer `layer` (0..16, network order as listed above) reads and writes its
 * activations in the workspace of (cfg, batch, training), so that a caller can inspect
 * every layer's BF16 activations after pfsur_forward or a training step.  All buffers
 * are NHWC BF16 at the resolution (H >> level, W >> level) of their level.
 *   in_off      byte offset of the input buffer, or (size_t)-1 for the network input x
 *   in_cs/in_c0 its channel stride and the first channel the layer reads (Cin of them)
 *   in_mode     0: read at the layer's resolution; 1: nearest 2x upsampling of a buffer
 *               at level + 1; 2: the 2x2 averages of the level above, already stored
 *               compact at the layer's resolution by the producing layer
 *   out_off, out_cs, out_c0   the output buffer (SiLU activations, Cout channels); at
 *               inference the last layer's activations are not stored (its epilogue
 *               feeds the 1x1 head straight away)
 *   pool_off, pool_cs   the buffer that also receives the 2x2 averages of the output
 *               (BF16 of 0.25 (((a(y,x) + a(y,x+1)) + a(y+1,x)) + a(y+1,x+1)) of the stored
 *               BF16 activations, summed in float32), or (size_t)-1
 * Returns PFLB_OK or PFLB_ERR_PARAM (invalid cfg, batch or layer). */
typedef struct pfsur_layer_io {
    size_t in_off, out_off, pool_off;
    int in_cs, in_c0, in_mode, out_cs, out_c0, pool_cs;
    int Cin, Cout, level;
} pfsur_layer_io;
int pfsur_layer_io_of(const pfsur_cfg* cfg, int batch, int training, int layer,
                      pfsur_layer_io* out);

/* Pack a batch of solver fields into the network input x (BF16 NHWC, PFSUR_IN_CH).  The
 * network works with the velocity u = J / rho(phi), rho(phi) = rho_L + clamp(phi, 0, 1)
 * (rho_H - rho_L), not with the momentum J, whose values span the density ratio: channels
 * (phi - s0) k0, (P - s1) k1, (u_x - s2) k2, (u_y - s3) k3 (s = in_shift, k = in_scale),
 * log10(rho_H/rho_L) lrr_scale, then zeros.
 *   phi, P [batch][H][W], J [batch][2][H][W] (the pflb_read layout per sample),
 *   rho[batch][2] host array of (rho_L, rho_H) per sample, finite and > 0. */
int pfsur_pack(pfsur_ctx* ctx, const float* phi, const float* P, const float* J,
               const double* rho, int batch, void* x, void* stream);

/* Training target from two solver states of the same batch, 16 steps apart:
 * y [batch][H][W][4] FP32, y_c = (f1_c - f0_c) / out_scale[c] for f = (phi, P, u_x, u_y)
 * (layouts and rho as in pfsur_pack). */
int pfsur_pack_target(pfsur_ctx* ctx, const float* phi0, const float* P0, const float* J0,
                      const float* phi1, const float* P1, const float* J1, const double* rho,
                      int batch, float* y, void* stream);

/* out [batch][H][W][4] FP32 = network(x) (x: BF16 NHWC [batch][H][W][8]). */
int pfsur_forward(pfsur_ctx* ctx, const void* x, float* out, int batch, void* workspace,
                  void* stream);

/* Apply a predicted residual in place: phi and P advance by out_c * out_scale[c], the
 * velocity J / rho(phi) likewise, and J becomes rho(phi_new) u_new (phi, P [batch][H][W],
 * J [batch][2][H][W]; rho as in pfsur_pack). */
int pfsur_apply(pfsur_ctx* ctx, const float* out, float* phi, float* P, float* J,
                const double* rho, int batch, void* stream);

/* One training step on (x, y): forward, MSE loss against y [batch][H][W][4] FP32,
 * backward, Adam with learning rate lr (beta1 0.9, beta2 0.999, eps 1e-8).  *loss
 * (host) receives the batch loss of the forward pass; synchronous. */
int pfsur_train_step(pfsur_ctx* ctx, const void* x, const float* y, int batch, float lr,
                     float* loss, void* workspace, void* stream);

/* Gradients of the MSE loss with respect to all parameters, without an update, into a
 * HOST array of pfsur_num_params() floats (for checking against a reference). */
int pfsur_gradients(pfsur_ctx* ctx, const void* x, const float* y, int batch, float* host_grad,
                    float* loss, void* workspace, void* stream);

/* Guarded advance of a batch of D2Q9 lattice Boltzmann contexts by `windows` x 16 steps
 * (the surrogate's densities per context are the contexts' own rho_L, rho_H).
 * For each window the surrogate predicts, in one batched forward pass, the state 16
 * steps ahead of every context; the prediction for context k is accepted when
 * |sum(phi_out) - sum(phi_0)| <= mass_tol * |sum(phi_0)|, sum(phi_0) the context's sum
 * at the start of the call (the method conserves it, so accepted windows cannot add up
 * to a drift beyond mass_tol), when the largest speed the
 * hand-over would give, max |J| / rho' with rho' = rho_L + phi (rho_H - rho_L) +
 * rho_dif lap(phi) / 4 (Eq. 13's density where the context uses it; rho' <= 0 counts as
 * infinite), is at most u_max (a state handed over with an unphysical speed would make
 * the plain steps after it unstable) and, on every
 * check_every-th window (0: never), when max|phi_out - phi_LB| <= phi_tol against 16
 * plain steps taken from the same state.  An accepted prediction becomes the context's
 * new state (pflb_reconstruct); otherwise the 16 plain steps are taken.  A context whose
 * state is non-finite at the start of a window ends the call with PFLB_ERR_NONFINITE
 * before that window hands over a prediction or takes a fallback (on a checked window
 * every context has by then taken the window's plain steps, its reference).
 *   lbs[batch]  contexts (periodic, nx = W, ny = H), batch <= max_batch
 *   work        pfsur_guard_work_bytes(cfg, batch) bytes of device memory, 256-aligned
 *   *n_fallback (host) number of (window, context) pairs that fell back.
 * Synchronous.  If an error is returned part-way, each context holds a valid state (the
 * one before or after its current window) but the windows done so far may differ
 * between contexts. */
size_t pfsur_guard_work_bytes(const pfsur_cfg* cfg, int batch);
int pflb_advance_guarded(pflb_ctx* const* lbs, int batch, pfsur_ctx* sur, int windows,
                         double mass_tol, double phi_tol, double u_max, int check_every,
                         int* n_fallback, void* work, void* stream);

/* pflb_advance_guarded that also records each decision and the quantities it rests on:
 * trace (host, NULL: none) receives windows x batch records of PFSUR_TRACE_FIELDS
 * doubles, record (window w, context k) at trace[(w * batch + k) * PFSUR_TRACE_FIELDS]:
 *   [0] sum(phi_0)  [1] sum(phi_in) of the window  [2] sum(phi_out) of the prediction
 *   [3] max |J_out| / rho'(phi_out)  [4] max |phi_out - phi_LB| (NaN if not checked)
 *   [5] 1 accepted, 0 fell back.
 * Sums are float64 over the float32 read-out fields in a fixed order. */
#define PFSUR_TRACE_FIELDS 6
int pflb_advance_guarded_trace(pflb_ctx* const* lbs, int batch, pfsur_ctx* sur, int windows,
                               double mass_tol, double phi_tol, double u_max, int check_every,
                               int* n_fallback, double* trace, void* work, void* stream);

/* The accept rule of pflb_advance_guarded, a pure host function (1 accept, 0 reject):
 * accept iff |sum_out - sum_in| <= mass_tol * |sum_in| (false for non-finite sums;
 * pflb_advance_guarded passes the sum at the start of the call as sum_in),
 * speed <= u_max (false if non-finite) and, when checked != 0, phi_err <= phi_tol. */
int pfsur_guard_accept(double sum_in, double sum_out, double mass_tol, double speed,
                       double u_max, int checked, double phi_err, double phi_tol);

/* Building blocks, stateless (no context): one circular-padded 3x3 convolution as the
 * network computes it, for testing and reuse.
 *   mode 0: x is [batch][H][W][Cin]; mode 1: x is [batch][H/2][W/2][Cin], read through
 *   2x nearest upsampling (H, W even); mode 2: x is [batch][2H][2W][Cin], read through
 *   2x2 average pooling (each pooled value rounded to BF16).
 *   x BF16 NHWC, Cin a multiple of 8; w BF16 [Cout][3][3][Cin]; b FP32 [Cout] or NULL.
 * pfsur_conv_fwd writes y_pre FP32 [batch][H][W][Cout] = conv(x) + b and/or
 * y_act BF16 = act ? silu(y_pre) : y_pre (either may be NULL).
 * pfsur_conv_wgrad writes dw FP32 [Cout][3][3][Cin] = sum_p dy[p, o] x_mode[p + tap, c]
 * and db FP32 [Cout] = sum_p dy[p, o] (NULL: skip) from dy BF16 [batch][H][W][Cout]
 * (Cout a multiple of 8), using `work` of pfsur_conv_wgrad_work_bytes() bytes.
 * Requires batch * H * W <= 2^26. */
int pfsur_conv_fwd(const void* x, int batch, int H, int W, int Cin, int Cout, int mode,
                   const void* w, const float* b, int act, float* y_pre, void* y_act,
                   void* stream);
size_t pfsur_conv_wgrad_work_bytes(int batch, int H, int W, int Cin, int Cout);
int pfsur_conv_wgrad(const void* x, const void* dy, int batch, int H, int W, int Cin, int Cout,
                     int mode, float* dw, float* db, void* work, void* stream);

/* Checkpoint / restore the parameters and optimiser state (host file). */
int pfsur_save(pfsur_ctx* ctx, const char* path);
int pfsur_load(pfsur_ctx* ctx, const char* path);

#ifdef __cplusplus
}
#endif

#endif /* PFSUR_H */
