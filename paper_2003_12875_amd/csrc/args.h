// args.h -- kernel argument blocks of the streaming NLL kernels: plain data
// seen by the host runtime and by the device code (compiled ahead of time
// or at run time).
#pragma once

#include <stdint.h>

#include "plan.h"

namespace nllmi {

// State of a gradient-descent fit (device arrays).
struct GDState {
  double* th_acc;   // n_sets * P  last accepted point
  double* g_acc;    // n_sets * P  its gradient
  double* th_prop;  // n_sets * P  point being evaluated
  double* f_acc;    // n_sets      its NLL (+inf before the first acceptance)
  double* eta;      // n_sets      step size (BHHH: damping lambda)
  int* last_status; // n_sets
  double* b_acc;    // n_sets * P * P  BHHH: matrix at the last accepted point
};

struct SingleArgs {
  const double* cols[kMaxObs];  // SoA event columns (device)
  int64_t n;
  const double* theta;          // n_param (device)
  double* nll_out;              // 1 (device)
  double* grad_out;             // n_param (device) or null
  double* bhhh_out;             // n_param^2 (device): BHHH matrix (evaluation)
  double* partials;             // grid * (NA + 1) double-double pairs
  PerTheta* pt_out;             // per-point constants left by block 0 (evaluation)
  PerTheta* consts;             // fit: constants of the proposal being evaluated,
                                // written by the previous step's finishing kernel
  int* status;                  // accumulated status bits
  const double* glx;            // 256-point Gauss-Legendre rule on [-1, 1]
  const double* glw;
  GDState gd;                   // fit mode: theta = gd.th_prop, set 0
  const double* wsum;           // weighted events: the weights' sum W (device, 1)
  // gradient-descent fit, double-buffered by step parity (k_single_fit):
  const double* partials_prev;  // the previous step's block records (null at the first step)
  GDState gd_out;               // the state the update writes (gd is the one it reads)
  PerTheta* consts_out;         // constants of the proposal this step evaluates
  double* aux;                  // a leaf's per-point tables (kAuxWords) beside the
                                // fit's constants in consts (first step, BHHH steps)
};

// The chunks of the batched pass: the events [0, n) in K rounds of G
// chunks, chunk j = r G + b streamed by block b in round r.  Rounds
// 0 .. K-2 have chunks of C events; the last round splits the remaining
// L = n - base events, base = (K - 1) G C, into G equal shares.
struct ChunkGrid {
  int64_t n, C, base, L;
  int32_t G, K;
};
#ifndef __HIPCC_RTC__
inline ChunkGrid make_chunk_grid(int64_t n, int G, int64_t C) {
  ChunkGrid g;
  g.n = n;
  g.C = C;
  g.G = G;
  g.K = n > 0 ? (int32_t)((n + (int64_t)G * C - 1) / ((int64_t)G * C)) : 1;
  g.base = (int64_t)(g.K - 1) * G * C;
  g.L = n - g.base;
  return g;
}
#endif

// One work item of the batched pass: events [start, end) of one set.
struct WorkItem {
  int64_t start, end;
  int32_t set, flag;  // flag: the offsets were malformed (no events)
};

struct SetsArgs {
  const double* cols[kMaxObs];
  int n_sets;
  const int64_t* offsets;   // n_sets + 1 (device)
  int64_t tile;             // events per work item
  const int64_t* tile_off;  // n_sets + 1 prefix of item counts (device)
  const int* set_flag;      // n_sets: 1 = malformed offsets
  const WorkItem* items;    // tile_off[n_sets] work items in set (and event) order
  const int64_t* chunk_first;  // G K + 1: the first item of each chunk (ChunkGrid)
  int32_t rounds;               // K: block b streams the items of chunks b, G + b, ..., (K-1) G + b
  PerTheta* consts;         // n_sets
  double* aux;              // n_sets * kAuxWords: a leaf's per-point tables, or null
  double* partials;         // items * (NA + 1) double-double pairs
  const double* theta;      // n_sets * P (evaluation mode)
  double* nll_out;          // n_sets
  double* grad_out;         // n_sets * P or null
  int* status_out;          // n_sets or null
  GDState gd;               // fit mode
  const double* glx;
  const double* glw;
};

}  // namespace nllmi
