/*
 * imsim_mpnn: a learned estimator of the expected spread sigma(S), trained on
 * Monte Carlo estimates from the simulator (ims_simulate_sets), and used to
 * rank candidate seeds inside the greedy loop of influence maximization
 * (paper Section 2, "Influence Maximization": greedy needs sigma(S + v) for
 * many v, each an expensive Monte Carlo estimate; Section 4 compares greedy
 * seed sets against degree and random heuristics).  The paper does not define
 * a network; the one here is this library's design.
 *
 * Network (one graph, a batch of B seed sets, node-major rows r = v * B + b):
 *   x_v      = [s_v, log(1 + outdeg v), log(1 + indeg v), log(1 + sum over
 *               arcs (v,u) of a_vu), 0 x 12]       (IMS_MPNN_IN = 16 values)
 *   h^0 = x;  h^{l+1}_v = ReLU([h^l_v | sum over arcs (u,v) of a_uv h^l_u] W_l + b_l),
 *             l = 0, 1, 2, hidden width 64
 *   yhat_v   = 1 if v in S, else sigmoid(h^3_v . w_o + b_o)
 *   pred(S)  = sum over v of yhat_v             (estimate of sigma(S))
 *   loss     = mean over the batch of ((pred(S) - target(S)) / n)^2
 * a_uv is the per-arc weight given at creation (the IC probability of the
 * arc).  Weights enter the arithmetic rounded to bf16; activations and
 * gradients are stored in bf16; every sum accumulates in fp32; biases are
 * fp32.  All reductions use a fixed order: results are deterministic.
 *
 * Parameters are one caller-owned fp32 device array of IMS_MPNN_NPARAMS
 * values laid out as the offsets below (W_l row-major [2 * width_in][64],
 * rows 0..width_in-1 multiply h_v, the rest the aggregate).
 *
 * Conventions as in imsim.h: 0 or a negative IMS_E_* code, message in
 * ims_last_error(); "host" pointers are read during the call only; "device"
 * pointers are caller-owned; work is enqueued on `stream`.
 */
#ifndef IMSIM_MPNN_H
#define IMSIM_MPNN_H

#include <stdint.h>

#include "imsim.h"

#ifdef __cplusplus
extern "C" {
#endif

#define IMS_MPNN_IN 16
#define IMS_MPNN_HIDDEN 64
#define IMS_MPNN_MAX_BATCH 256
#define IMS_MPNN_OFF_W0 0       /* [32][64]  */
#define IMS_MPNN_OFF_B0 2048    /* [64]      */
#define IMS_MPNN_OFF_W1 2112    /* [128][64] */
#define IMS_MPNN_OFF_B1 10304   /* [64]      */
#define IMS_MPNN_OFF_W2 10368   /* [128][64] */
#define IMS_MPNN_OFF_B2 18560   /* [64]      */
#define IMS_MPNN_OFF_WO 18624   /* [64]      */
#define IMS_MPNN_OFF_BO 18688   /* [1]       */
#define IMS_MPNN_NPARAMS 18689

/* Internal tensors readable with ims_mpnn_fetch after a forward (and a
 * backward), rows = n * B of the last forward, bf16 unless stated. */
enum {
    IMS_MPNN_T_X0 = 0,   /* [rows][16] input features                     */
    IMS_MPNN_T_M0 = 1,   /* [rows][16] aggregate of X0                    */
    IMS_MPNN_T_H1 = 2,   /* [rows][64]                                    */
    IMS_MPNN_T_M1 = 3,
    IMS_MPNN_T_H2 = 4,
    IMS_MPNN_T_M2 = 5,
    IMS_MPNN_T_H3 = 6,
    IMS_MPNN_T_YHAT = 7, /* [rows] fp32 per-node estimate                 */
    IMS_MPNN_T_DZ3 = 8,  /* [rows][64] loss gradient of layer-3 pre-activation */
    IMS_MPNN_T_DH2 = 9,  /* [rows][64] gradient of h^2 through W_2's self rows */
    IMS_MPNN_T_DM2 = 10, /* [rows][64] gradient of the layer-2 aggregate  */
    IMS_MPNN_T_DZ2 = 11,
    IMS_MPNN_T_DH1 = 12,
    IMS_MPNN_T_DM1 = 13,
    IMS_MPNN_T_DZ1 = 14,
    IMS_MPNN_T_COUNT = 15
};

typedef struct ims_mpnn ims_mpnn;

/* Plan for one graph: out-CSR (host offsets int64[n+1], indices uint32[m])
 * with arc weights a (host float[m], out-CSR order, finite), and the largest
 * batch (1 .. IMS_MPNN_MAX_BATCH).  Builds the in-CSR, the node features and
 * a workspace of about 12 * 128 * n * max_batch bytes.  Synchronous. */
int ims_mpnn_create(int64_t n, int64_t m, const int64_t* offsets, const uint32_t* indices, const float* arc_weight,
                    uint32_t max_batch, ims_mpnn** out);
int ims_mpnn_destroy(ims_mpnn* p);

/* Glorot-uniform weights (fan-in counts only the 4 real input features at
 * layer 0), zero biases, from a splitmix64 stream of `seed`.  Host output
 * float[IMS_MPNN_NPARAMS]. */
int ims_mpnn_init_params(uint64_t seed, float* params);

/* pred[b] (device float[n_sets]) = estimate of sigma(set b) for the sets given
 * as host set_offsets uint32[n_sets+1] / set_nodes (duplicates allowed, ids
 * < n), 1 <= n_sets <= max_batch.  Keeps every activation for a following
 * backward. */
int ims_mpnn_forward(ims_mpnn* p, const float* params, const uint32_t* set_offsets, const uint32_t* set_nodes,
                     uint32_t n_sets, float* pred, void* stream);

/* Gradient of the loss of the last forward against target (device
 * float[n_sets]) into grads (device float[IMS_MPNN_NPARAMS], overwritten);
 * loss (device float[1]) may be NULL.  params must be those of the forward. */
int ims_mpnn_backward(ims_mpnn* p, const float* params, const float* target, float* grads, float* loss, void* stream);

/* One Adam step (bias-corrected; step counts from 1) on device arrays of
 * `count` floats: params -= lr * mhat / (sqrt(vhat) + eps). */
int ims_mpnn_adam_step(float* params, const float* grads, float* m, float* v, int64_t count, float lr, float beta1,
                       float beta2, float eps, uint32_t step, void* stream);

/* Copy internal tensor `tensor` (IMS_MPNN_T_*) of the last forward/backward
 * into host memory (at most `bytes`; *written = bytes copied).  Waits for
 * `stream`.  Inspection hook for tests. */
int ims_mpnn_fetch(ims_mpnn* p, int tensor, void* host_out, int64_t bytes, int64_t* written, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* IMSIM_MPNN_H */
