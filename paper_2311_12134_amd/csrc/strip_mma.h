// A 16-row strip of a product C = A B with K = KD (a multiple of 4, default NB = 64) on
// the matrix cores, for one wavefront: rows [0, 16) of the strip, CB blocks of 16 columns.  A and B are read
// through functors a(i, k) and b(k, j) returning the storage's complex type.
//   float2  : FP32 MFMA 16x16x4 with three real products (Ar Br, Ai Bi, (Ar+Ai)(Br+Bi));
//             D lane l, register r -> (row 4 (l/16) + r, column l % 16) of a block.
//   double2 : FP64 MFMA 16x16x4 with four real products;
//             D lane l, register r -> (row l/16 + 4 r, column l % 16) of a block.
// A lane l supplies A (row l % 16, k l / 16) and B (k l / 16, column l % 16).
#pragma once

#include "lsms_internal.h"

namespace lsms {

template <typename T, int CB, int KD = NB>
struct StripMma;

template <int CB, int KD>
struct StripMma<float2, CB, KD> {
  typedef float f4v __attribute__((ext_vector_type(4)));
  f4v t1[CB], t2[CB], t3[CB];
  __device__ void zero() {
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      t1[c] = f4v{0, 0, 0, 0};
      t2[c] = f4v{0, 0, 0, 0};
      t3[c] = f4v{0, 0, 0, 0};
    }
  }
  template <typename FA, typename FB>
  __device__ void run(FA a_at, FB b_at, int lane) {
    const int ii = lane & 15, kq = lane >> 4;
#pragma unroll 4
    for (int k4 = 0; k4 < KD; k4 += 4) {
      const float2 a = a_at(ii, k4 + kq);
      const float as = a.x + a.y;
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const float2 b = b_at(k4 + kq, c * 16 + ii);
        t1[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, t1[c], 0, 0, 0);
        t2[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, t2[c], 0, 0, 0);
        t3[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(as, b.x + b.y, t3[c], 0, 0, 0);
      }
    }
  }
  // as run, with this lane's A values (row l % 16, k 4 q + l / 16) already in registers
  template <typename FB>
  __device__ void run_regs(const float2 (&a)[KD / 4], FB b_at, int lane) {
    const int ii = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int q = 0; q < KD / 4; ++q) {
      const float as = a[q].x + a[q].y;
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const float2 b = b_at(4 * q + kq, c * 16 + ii);
        t1[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q].x, b.x, t1[c], 0, 0, 0);
        t2[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q].y, b.y, t2[c], 0, 0, 0);
        t3[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(as, b.x + b.y, t3[c], 0, 0, 0);
      }
    }
  }
  __device__ static int row(int r, int lane) { return 4 * (lane >> 4) + r; }
  __device__ double2 value(int c, int r) const {
    return make_double2((double)(t1[c][r] - t2[c][r]), (double)(t3[c][r] - t1[c][r] - t2[c][r]));
  }
};

template <int CB, int KD>
struct StripMma<double2, CB, KD> {
  typedef double d4v __attribute__((ext_vector_type(4)));
  d4v re[CB], im[CB];
  __device__ void zero() {
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      re[c] = d4v{0, 0, 0, 0};
      im[c] = d4v{0, 0, 0, 0};
    }
  }
  template <typename FA, typename FB>
  __device__ void run(FA a_at, FB b_at, int lane) {
    const int ii = lane & 15, kq = lane >> 4;
#pragma unroll 4
    for (int k4 = 0; k4 < KD; k4 += 4) {
      const double2 a = a_at(ii, k4 + kq);
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const double2 b = b_at(k4 + kq, c * 16 + ii);
        re[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, re[c], 0, 0, 0);
        re[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, re[c], 0, 0, 0);
        im[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, im[c], 0, 0, 0);
        im[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, im[c], 0, 0, 0);
      }
    }
  }
  template <typename FB>
  __device__ void run_regs(const double2 (&a)[KD / 4], FB b_at, int lane) {
    const int ii = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int q = 0; q < KD / 4; ++q) {
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const double2 b = b_at(4 * q + kq, c * 16 + ii);
        re[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q].x, b.x, re[c], 0, 0, 0);
        re[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[q].y, b.y, re[c], 0, 0, 0);
        im[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q].x, b.y, im[c], 0, 0, 0);
        im[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q].y, b.x, im[c], 0, 0, 0);
      }
    }
  }
  __device__ static int row(int r, int lane) { return (lane >> 4) + 4 * r; }
  __device__ double2 value(int c, int r) const { return make_double2(re[c][r], im[c][r]); }
};

}  // namespace lsms
