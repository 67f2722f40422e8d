/*
 * unet.h -- C ABI of the U-Net part of the MI355X Helmholtz library: the
 * network used as error predictor inside the preconditioners of section 3.2
 * (coarse-grid correction with Jacobi smoothing, Algorithm 2; deflation
 * beside an SL V-cycle, eq. 3.4), its encoder-solver variant (section 3.3,
 * eq. 3.5) and its supervised training (section 3.4, eq. 3.7-3.9) with Adam.
 *
 * Conventions are those of helm.h (device pointers owned by the caller,
 * void* streams, 0 / >0 / <0 return codes, helm_last_error()).
 *
 * Network: L levels of widths w_0..w_{L-1}.  Level l applies twice
 * [3x3 convolution (zero padding, no bias) -> batch normalisation ->
 * LeakyReLU(0.2)]; 2x2 max pooling between levels; on the way up a bilinear
 * x2 upsampling (half-pixel centres, edges clamped) concatenated as
 * [upsampled, skip] and the same double convolution; a 1x1 convolution with
 * bias to out_ch channels.  BN uses eps 1e-5 and momentum 0.1; inference uses
 * the running statistics.  Weights and activations are bf16 on the device
 * with FP32 accumulation; FP32 master weights and Adam moments are kept.
 *
 * Parameter order (flat FP32 arrays): for each 3x3 convolution in forward
 * order (enc0a, enc0b, enc1a, ..., dec{L-2}a, dec{L-2}b, ..., dec0a, dec0b):
 * weight [cout][cin][3][3], BN weight [cout], BN bias [cout]; then the head
 * weight [out_ch][w_0] and bias [out_ch] (absent for an encoder).  Buffers:
 * for each convolution the BN running mean [cout] and running variance [cout].
 * cin counts the concatenated inputs in order: [input (+ context)] for the
 * down convolutions, [upsampled, skip (+ context)] for the up convolutions.
 */
#ifndef UNET_H
#define UNET_H

#include "helm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct unet_net unet_net;

typedef struct {
    int in_ch;      /* real input channels: 3 = (Re r, Im r, kappa)           */
    int out_ch;     /* output channels: 2 = (Re e, Im e)                       */
    int levels;     /* resolution levels, 1..6                                  */
    int widths[6];  /* channels per level; each a multiple of 32               */
    int context;    /* 1: solver of an encoder-solver pair: level l's context
                       (w_l channels) is the last input of its first down
                       convolution and of its first up convolution           */
    int head;       /* 1: 1x1 head; 0: encoder (in_ch 1, context 0) whose
                       outputs are the per-level contexts                    */
    int arch;       /* 0: the network above (default).  1: the paper's own
                       network (section 3.1, eq. 3.1-3.3) on the FINE grid:
                       in_ch 4 = (Re r^, Im r^, kappa^2, gamma), levels L
                       below the fine grid with widths c_1..c_L (any >= 1);
                       level l: x = elu(BN(R_l x)) with R_l a 5x5 stride-2
                       convolution, then ResNet blocks x = elu(BN(x + K2
                       elu(BN(K1 x)))) with 3x3 K1, K2 (one per level, three
                       at level L); up: y = cat(BN(P elu(y)), x^(l)) with P a
                       5x5 stride-2 transposed convolution (padding 2, output
                       padding 1); output e = P_1 elu(y^(1)) (2 channels, with
                       a bias).  Parameters per layer in that order: weight
                       (convolution [cout][cin][5|3][5|3], transposed
                       [cin][cout][5][5]), BN weight and bias (the output
                       layer: its bias); buffers: BN running mean and variance
                       per layer.  FP32 throughout; head 1, context 0.        */
} unet_cfg;

/* Create a network with zero parameters (set them with unet_set_params). */
int unet_create(const unet_cfg *cfg, unet_net **out);
void unet_destroy(unet_net *net);
/* Number of FP32 parameters / buffer entries in the flat orders above. */
long long unet_num_params(const unet_net *net);
long long unet_num_buffers(const unet_net *net);

/* Copy parameters and BN buffers in (device float arrays of the sizes above);
 * resets the Adam state and step count.  buffers may be NULL (mean 0, var 1). */
int unet_set_params(unet_net *net, const float *params, const float *buffers, void *stream);
/*
 * Seeded initial parameters: 3x3 weights Kaiming-normal over the real input
 * fan-in with the LeakyReLU(0.2) gain (std sqrt(2 / (1 + 0.2^2) / (9 cin))),
 * BN weight 1 and bias 0, head weight normal with std sqrt(1 / w_0), head
 * bias 0; running statistics mean 0, variance 1; Adam state reset.  Normals
 * from splitmix64 and the Box-Muller transform.  Synchronises `stream`.
 */
int unet_init(unet_net *net, unsigned long long seed, void *stream);
/* Copy the FP32 master parameters and buffers out (either may be NULL). */
int unet_get_params(unet_net *net, float *params, float *buffers, void *stream);

/*
 * unet_forward -- plain network application.
 *   x   : device float [B][in_ch][H][W]; H, W divisible by 2^(levels-1)
 *         (arch 1: H = W divisible by 2^levels)
 *   out : device float [B][out_ch][H][W]
 *   training = 0: BN with running statistics; 1: batch statistics (the
 *   running statistics are not updated).
 */
int unet_forward(unet_net *net, const float *x, int B, int H, int W, float *out, int training,
                 void *stream);

/*
 * unet_infer -- the network as error predictor for residuals on the fine
 * grid of medium h (the network runs on the grid n/2):
 *   e = P s Net(R(h^2 r) / s, kappa_c),  s = RMS over the coarse grid of
 *   |R(h^2 r)|,  kappa_c the slowness injected at the coarse points.
 * R, P: full-weighting restriction and bilinear prolongation (eq. 2.9); the
 * h^2 scaling follows section 3.4; s makes the map positively homogeneous.
 * arch 1 (the paper's network, whose transfers are learned):
 *   e = s Net(h^2 r / s, kappa^2, gamma) on the fine grid, s = RMS of |h^2 r|.
 * An all-zero residual gives e = 0.
 *   r, e : complex64 [nrhs][n][n]; must not overlap.
 */
int unet_infer(unet_net *net, helm_handle *h, const float *r, float *e, int nrhs, void *stream);

/* One training batch of (residual, error, coarse slowness) triples. */
typedef struct {
    int nb;               /* samples                                             */
    int n;                /* fine grid size (network on n/2)                     */
    const float *r;       /* complex64 [nb][n][n] residuals                      */
    const float *e;       /* complex64 [nb][n][n] errors (A e = r)               */
    const float *kappa_c; /* float [nb][n/2][n/2] coarse slowness                */
    /* arch 1 only (the paper's network reads the fine medium): slowness and
       attenuation, float [nb][n][n], or [n][n] shared by the batch when
       fine_shared is 1; NULL for arch 0 */
    const float *kappa_f, *gamma_f;
    int fine_shared;
} unet_batch;

typedef struct {
    float lr;             /* default 1e-3 */
    float beta1, beta2;   /* default 0.9, 0.999 */
    float eps;            /* default 1e-8 */
} unet_train_opts;

/*
 * unet_loss_grad -- loss of eq. 3.7 in the scaled form used here,
 *   loss = mean_b || P Net(R(h^2 r_b)/s_b, kappa_c) - e_b / s_b ||^2 / n^2,
 * with training-mode BN, and its gradient.  loss_out: host double.
 * grads: device float [num_params] receiving the gradient (may be NULL).
 */
int unet_loss_grad(unet_net *net, const unet_batch *batch, double *loss_out, float *grads,
                   void *stream);

/*
 * unet_train_step -- unet_loss_grad, one Adam step (bias-corrected, no weight
 * decay) on the FP32 masters, bf16 weights re-rounded from them, and the BN
 * running statistics updated.  loss_out: host double (loss before the step);
 * opts may be NULL.  Synchronises `stream` to read the loss.
 */
int unet_train_step(unet_net *net, const unet_batch *batch, const unet_train_opts *opts,
                    double *loss_out, void *stream);

/*
 * Encoder-solver pair (section 3.3, eq. 3.5).  The encoder is the same
 * skeleton without a head, applied to the coarse slowness kappa_c (one input
 * channel); its output at level l (the up-path output, the bottleneck output
 * at the last level) is the context f^(l), [nb][nc >> l][nc >> l][w_l].
 * The solver (context = 1) concatenates f^(l) to the input of its first down
 * convolution and of its first up convolution at level l.
 */

/*
 * unet_pair_encode -- run the encoder (inference BN) on kappa_c, device float
 * [nb][nc][nc], and store the contexts in the solver (a copy the solver owns:
 * the encoder may then be reused or destroyed).  With nb = 1 the context is
 * shared by every sample of later solver calls (one medium, many right-hand
 * sides: the encoder runs once per medium); with nb > 1, sample b of a
 * unet_forward batch of size nb uses context b.  helm_fgmres_solve and
 * unet_infer need the nb = 1 form for the problem's medium (nc = n/2).
 */
int unet_pair_encode(unet_net *encoder, unet_net *solver, const float *kappa_c, int nb, int nc,
                     void *stream);

/*
 * unet_pair_encode_medium -- unet_pair_encode for the medium of handle h:
 * the encoder runs on the slowness injected at the coarse points of h (the
 * network grid n/2) and the solver keeps that one context (nb = 1).  The
 * handle keeps a float [n/2][n/2] buffer for the coarse slowness.
 */
int unet_pair_encode_medium(unet_net *encoder, unet_net *solver, helm_handle *h, void *stream);

/*
 * unet_pair_loss_grad -- the loss of unet_loss_grad with the solver fed
 * the contexts the encoder computes (training-mode BN in both) from each
 * sample's batch->kappa_c; gradients of both networks (joint training).
 * enc_grads / sol_grads: device float arrays of each network's num_params (may
 * be NULL).  Leaves the solver without a context (encode again before use).
 */
int unet_pair_loss_grad(unet_net *encoder, unet_net *solver, const unet_batch *batch,
                        double *loss_out, float *enc_grads, float *sol_grads, void *stream);

/* unet_pair_loss_grad, then one Adam step of each network (as unet_train_step). */
int unet_pair_train_step(unet_net *encoder, unet_net *solver, const unet_batch *batch,
                         const unet_train_opts *opts, double *loss_out, void *stream);

/*
 * Training state.  unet_save writes, and unet_load restores, everything a
 * training run needs to continue bit for bit: the FP32 master parameters, the
 * BN running statistics, the Adam moments and step count (section 3.4 trains
 * with Adam) and the training-data cursor (the seed and the next sample index
 * of helm_training_triples_seeded).  The file is a host file at `path`
 * (written to path + ".tmp", then renamed): the 8-byte tag "HELMUNT1", int32
 * in_ch, out_ch, levels, widths[6] (0 past levels), context, head, arch; int64
 * num_params, num_buffers; int32 Adam step; uint64 data seed, next sample
 * index; FP32 parameters, buffers, first moments, second moments, all
 * little-endian.  unet_load requires a network of the same configuration
 * (else HELM_E_INVALID, nothing changed), re-rounds the bf16 weights and
 * drops the solver's context maps (encode again).  Both synchronise `stream`.
 */
int unet_save(unet_net *net, const char *path, void *stream);
int unet_load(unet_net *net, const char *path, void *stream);
/* The training-data cursor kept with the state (0, 0 after unet_create). */
int unet_set_cursor(unet_net *net, unsigned long long seed, unsigned long long next_index);
int unet_get_cursor(const unet_net *net, unsigned long long *seed, unsigned long long *next_index);

#ifdef __cplusplus
}
#endif

#endif /* UNET_H */
