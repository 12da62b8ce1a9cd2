// The Kronecker operator through rectangular real cos/sin factors (rect.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

namespace kpme {

struct RectArgs {
  bool fp64;
  int K[3];            // grid points per axis
  int n[3];            // real Fourier rows per axis, min(2M + 1, K)
  const void* F[3];    // [n_j][K_j] rows 1, cos, sin (row-major)
  const void* Ft[3];   // [K_j][n_j] their transposes
  const void* D;       // [n1][n2][n3] sum_r omega_r d_r1 (x) d_r2 (x) d_r3
  const void* Q;       // grid in  [K1][K2][K3]
  void* Phi;           // grid out [K1][K2][K3]
  void* wa;            // two work arrays of K1 K2 K3 values
  void* wb;
  void* handle;        // rocBLAS handle (the plan's)
  const double* sumQ;  // sum(Q) (device)
  double c0;           // the correction constant
  double* epart;       // finalize partials of sum Q Phi, or NULL
};

// Real Fourier rows 1, cos(2 pi m g / K), sin(...) for m = 1..M (no sine row at
// m = K / 2), row-major [rows][K]; *modes receives the mode of each row.
std::vector<double> rect_rows(int K, int M, std::vector<int>* modes);
// The diagonal weights d of an even mode vector a on those rows.
std::vector<double> rect_weights(const std::vector<double>& a, const std::vector<int>& modes);

hipError_t rect_create_handle(void** handle);
void rect_destroy_handle(void* handle);
// Phi (without the correction) = F^T D F Q in three thin products each way.
hipError_t launch_rect_apply(const RectArgs& a, hipStream_t st);
// Phi -= c0 sum(Q) and the energy partials.
hipError_t launch_rect_finalize(const RectArgs& a, hipStream_t st);

}  // namespace kpme
