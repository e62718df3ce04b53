// Batched solves: state and launchers shared by batched.cpp and kernels_batch.hip.
#pragma once

#include <vector>

#include "gabp_internal.h"

namespace gabp {

// per (system, right-hand side) status bits
constexpr uint32_t kPairDone = 1u;       // converged, failed or given up: x is final
constexpr uint32_t kPairFailed = 2u;     // non-finite values or stagnated refinement
constexpr uint32_t kPairHasBest = 4u;    // refinement: an improving trial exists
constexpr uint32_t kPairInnerDone = 8u;  // refinement: inner solve of this step finished
constexpr uint32_t kPairNewBest = 16u;   // refinement: last check produced a new best

struct PairStat {
  double rel_res2;
  double res_inf;
  int32_t sweeps;
  int32_t outer;
};

struct Batch {
  int32_t nsys = 0, R = 1;
  int64_t N = 0;                       // external rows (sum of system sizes)
  std::vector<int32_t> h_ext_off, h_int_off;
  // device
  int32_t* ext_off = nullptr;          // [nsys+1] external row offsets
  int32_t* int_off = nullptr;          // [nsys+1] internal (slice-aligned) row offsets
  int32_t* slice_sys = nullptr;        // [nslices] system of every slice
  int32_t* sys_slice0 = nullptr;       // [nsys+1] first slice of every system
  int32_t* sys_on = nullptr;           // [nsys] system is sweeping
  int32_t* sys_live = nullptr;         // [nsys] system has unfinished pairs (refinement)
  int32_t* count = nullptr;            // [1] systems still sweeping after a check
  uint32_t* flags = nullptr;           // [nsys*R]
  PairStat* stat = nullptr;            // [nsys*R]
  double* scale = nullptr;             // [nsys*R] refinement scale ||r||_inf
  double* best = nullptr;              // [nsys*R] best trial residual of the inner solve
  double* rn = nullptr;                // [nsys*R] residual norm at the outer step start
  int32_t* since = nullptr;            // [nsys*R] checks since the last new best
  int32_t* inner = nullptr;            // [nsys*R] sweeps of the current inner solve
  double* partials = nullptr;          // [nslices*R*3]
  double* norms = nullptr;             // [nsys*R*3]: sum r^2, max|r|, sum b^2
  double* b = nullptr;                 // [n_int*R] internal right-hand sides
  double* x = nullptr;                 // [n_int*R]
  double* r = nullptr;                 // [n_int*R]
  float* r32 = nullptr;                // [n_int*R]
  float* d32 = nullptr;                // [n_int*R]
  float* dbest32 = nullptr;            // [n_int*R]
  double* msg64[2] = {nullptr, nullptr};   // [(epad+1)*R]
  float* msg32[2] = {nullptr, nullptr};    // [(epad+1)*R]
  int32_t* host_count = nullptr;       // pinned
};

hipError_t batch_mean32(const gabp_ctx* c, const Batch* B, const float* msg_in, float* msg_out,
                        float* x, hipStream_t s);
hipError_t batch_mean64(const gabp_ctx* c, const Batch* B, const double* msg_in,
                        double* msg_out, double* x, hipStream_t s);
hipError_t batch_joint64(const gabp_ctx* c, const Batch* B, const double* lam_in,
                         const double* msg_in, double* lam_out, double* msg_out, double* x,
                         hipStream_t s);
hipError_t batch_residual(const gabp_ctx* c, const Batch* B, const int32_t* gate,
                          const double* x, const float* dx, double* r, hipStream_t s);
hipError_t batch_decide_plain(const Batch* B, double tol, int k_swept, hipStream_t s);
hipError_t batch_ir_outer_begin(const Batch* B, double tol, hipStream_t s);
hipError_t batch_ir_inner_check(const Batch* B, double tol, double inner_tol, int patience,
                                int k_swept, int inner_max, hipStream_t s);
hipError_t batch_ir_outer_end(const Batch* B, hipStream_t s);
hipError_t batch_copy_best(const gabp_ctx* c, const Batch* B, hipStream_t s);
hipError_t batch_apply_best(const gabp_ctx* c, const Batch* B, hipStream_t s);
hipError_t batch_cast(const gabp_ctx* c, const Batch* B, hipStream_t s);
hipError_t batch_zero_msgs32(const gabp_ctx* c, const Batch* B, float* msg, hipStream_t s);
hipError_t batch_zero_msgs64(const gabp_ctx* c, const Batch* B, double* msg, hipStream_t s);
hipError_t batch_pack(const gabp_ctx* c, const Batch* B, const double* Bx, double* bi,
                      hipStream_t s);
hipError_t batch_unpack(const gabp_ctx* c, const Batch* B, const double* xi, double* X,
                        hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);

void batch_free(Batch* B);

}  // namespace gabp
