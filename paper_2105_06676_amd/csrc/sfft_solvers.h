// Whole-solve entry points shared by the C ABI, the batch and the server.
// A non-null `pool` gives a solve one device region for all its buffers (at
// least the matching *_footprint bytes; the server's per-request arena block);
// otherwise the solve uses the device context's per-stream buffers.
#pragma once

#include <vector>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>

namespace sfft {

// StencilFFT-P on 7-smooth extents, radius <= 2 (fused pass schedule).
void solve_periodic_dense(void* grid, bool f64, int d, const int64_t* dims, int64_t B, const double* coeffs, int r,
                          int64_t T, hipStream_t st);
// StencilFFT-P on any extents (chirp-z transforms along axes with a prime factor above 7).
void solve_periodic_any(void* grid, bool f64, int d, const int64_t* dims, const double* coeffs, int r, int64_t T,
                        hipStream_t st, void* pool = nullptr);
size_t periodic_any_footprint(bool f64, int d, const int64_t* dims);
// StencilFFT-P for radius up to kMaxGeneralR (7-smooth extents, unfused schedule).
void solve_periodic_general(void* grid, bool f64, int d, const int64_t* dims, const double* coeffs, int r,
                            int64_t T, hipStream_t st, void* pool = nullptr);
size_t periodic_general_footprint(bool f64, int d, const int64_t* dims, int r);
// m coupled fields (or, with q_coeffs, an implicit stencil Q a_{t+1} = S a_t on
// one field) on extents with a prime factor above 7: complex per-axis transforms
// (chirp-z on those axes), the symbol-matrix power on the full spectrum.
void solve_fields_any(void* grid, bool f64, int m, int d, const int64_t* dims, const double* coeffs, int r,
                      int64_t T, hipStream_t st, const double* q_coeffs = nullptr);
struct FieldParams;
std::vector<double> field_constants(int m, int d, const double* coeffs, int r, const double* q_coeffs,
                                    FieldParams* fp);
// StencilFFT-A with RecursiveBoundary; bc 0: fixed frame, 1: reflecting frame.
void solve_aperiodic(void* grid, bool f64, int d, const int64_t* dims, const double* coeffs, int r, int64_t T,
                     int bc, hipStream_t st);
void solve_aperiodic_pooled(void* grid, bool f64, int d, const int64_t* dims, const double* coeffs, int r,
                            int64_t T, int bc, hipStream_t st, void* pool, size_t cap);
size_t aperiodic_footprint(bool f64, int d, const int64_t* dims, const double* coeffs, int r, int64_t T, int bc);
struct Verifier;
// The aperiodic solve's bookkeeping with nothing enqueued, every pass schedule and
// base case checked against its buffers.
void verify_aperiodic(bool f64, int d, const int64_t* dims, const double* coeffs, int r, int64_t T, int bc,
                      Verifier* v);

}  // namespace sfft
