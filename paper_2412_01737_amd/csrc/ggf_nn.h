// Launch interface of the learned block proposal (network and block moves).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ggf_device.h"
#include "ggf_launch.h"

#define GGF_NN_NPARAMS 19682
#define GGF_BLOCK_RMAX 128   /* 4 Majoranas x every link of a 4 x 4 patch */

struct NNArgs {
  int P;                       // patch side (1, 2 or 4)
  const uint16_t *wq;          // bfloat16 weights
  const float *params;         // float32 master parameters (biases read from here)
  const ChainDev *chains;
  const int8_t *links;
};

struct BlockLaunch {
  LaunchCtx lc;
  NNArgs nn;
  double *A, *Wf;
  void *D;
  const size_t *d_off;
  int *U, *rcnt;
  unsigned long long *bprop, *bacc;   // per chain: proposed, accepted, links changed, updates of G
  int patch, parity, kmax;
  // delayed block moves: largest pending rank (0 = apply each accepted move at once) and the
  // decision's move (Wn, Un, rn, mode) with its pending-move products (E, Fm)
  int pend;
  double *E, *Fm, *Wn;
  int *Un, *rn, *mode;
  double rho;                  // move rate of the proposal
};

void ggf_nn_forward_launch(const NNArgs &a, const int *ex_chain, const int *ex_patch, int n_ex, float *logits,
                           hipStream_t s);
void ggf_nn_grad_launch(const NNArgs &a, const int *ex_chain, const int *ex_patch, int n_ex, float *gpart,
                        int nslices, double *lpart, float *grad, double *loss, hipStream_t s);
void ggf_nn_adam_launch(float *p, uint16_t *wq, float *m, float *v, const float *g, float lr, int t, hipStream_t s);
void ggf_nn_quantize_launch(const float *p, uint16_t *wq, hipStream_t s);
void ggf_nn_examples_launch(int *ex_chain, int *ex_patch, int n_ex, uint32_t t, uint32_t k0, uint32_t k1, int n_chains,
                            int npatch, hipStream_t s);
void ggf_block_decide_launch(const BlockLaunch &bl, hipStream_t s);
void ggf_block_update_launch(const BlockLaunch &bl, int grid, hipStream_t s);
void ggf_block_merge_launch(const BlockLaunch &bl, hipStream_t s);
void ggf_block_pending_launch(const BlockLaunch &bl, bool list, hipStream_t s);
