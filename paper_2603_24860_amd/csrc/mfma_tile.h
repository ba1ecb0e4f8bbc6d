// MFMA 16x16x4 tile core for gfx950, shared by the GEMM-shaped kernels.
//
// A workgroup of 256 threads (4 waves in a 2x2 arrangement) computes a
// BM x BN tile of C = A * B^T with A (BM x K) and B (BN x K) staged in LDS
// row-major along K.  One MFMA step consumes K = 4: lane l supplies row
// (l & 15) of a 16-row fragment at K slot (l >> 4).  Because K is a pure
// reduction index, the kernels permute it so that lane l reads the four
// consecutive K values kk + 4 (l >> 4) + i (i = 0..3) with one vector LDS
// read and feeds them to four successive MFMAs.  The output layout of the
// 16x16 block is: lane l holds column (l & 15), rows 4 (l >> 4) + j, j = 0..3
// for the f32 instruction.  The f64 instruction places row g + 4 j in lane
// (g, j) instead; Mfma<double>::arow() permutes which A row each lane feeds so
// that both types end with the f32 output layout.
#pragma once
#include <hip/hip_runtime.h>

namespace bse {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
  typedef f32x4 acc_t;
  typedef f32x4 frag_t;
  // A row (within the 16-row fragment) that lane row r feeds
  static __device__ __forceinline__ int arow(int r) { return r; }
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  typedef f64x4 acc_t;
  typedef f64x4 frag_t;
  static __device__ __forceinline__ int arow(int r) { return 4 * (r & 3) + (r >> 2); }
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// Four consecutive K values of one row from LDS (16-byte aligned address).
template <typename T> __device__ __forceinline__ typename Mfma<T>::frag_t lds_frag(const T *p);
template <> __device__ __forceinline__ f32x4 lds_frag<float>(const float *p) {
  return *reinterpret_cast<const f32x4 *>(p);
}
template <> __device__ __forceinline__ f64x4 lds_frag<double>(const double *p) {
  const double2 lo = *reinterpret_cast<const double2 *>(p);
  const double2 hi = *reinterpret_cast<const double2 *>(p + 2);
  f64x4 r;
  r[0] = lo.x; r[1] = lo.y; r[2] = hi.x; r[3] = hi.y;
  return r;
}

// Row pitch (elements) of an LDS tile with BK columns: 16 bytes of padding.
template <typename T, int BK> struct Pitch {
  static constexpr int value = BK + 16 / int(sizeof(T));
};

// Accumulates one BK-deep slab: acc[MI][NI] += A_lds[wm0.., :] * B_lds[wn0.., :]^T
template <typename T, int MI, int NI, int BK>
__device__ __forceinline__ void mfma_slab(typename Mfma<T>::acc_t (&acc)[MI][NI], const T *As,
                                          const T *Bs, int wm0, int wn0, int lane) {
  constexpr int P = Pitch<T, BK>::value;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < BK; kk += 16) {
    typename Mfma<T>::frag_t a[MI], b[NI];
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
      a[mi] = lds_frag<T>(As + (wm0 + 16 * mi + Mfma<T>::arow(r)) * P + kk + 4 * g);
#pragma unroll
    for (int ni = 0; ni < NI; ++ni)
      b[ni] = lds_frag<T>(Bs + (wn0 + 16 * ni + r) * P + kk + 4 * g);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < NI; ++ni) acc[mi][ni] = Mfma<T>::mma(a[mi][i], b[ni][i], acc[mi][ni]);
  }
}

// The same with A stored K-major: At[k * PT + row] (the four K values of a
// lane are read one by one down a column; the 16 rows of a fragment are
// consecutive in LDS).
template <typename T, int MI, int NI, int BK, int PT>
__device__ __forceinline__ void mfma_slab_at(typename Mfma<T>::acc_t (&acc)[MI][NI], const T *At,
                                             const T *Bs, int wm0, int wn0, int lane) {
  constexpr int P = Pitch<T, BK>::value;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < BK; kk += 16) {
    typename Mfma<T>::frag_t a[MI], b[NI];
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a[mi][i] = At[(kk + 4 * g + i) * PT + wm0 + 16 * mi + Mfma<T>::arow(r)];
#pragma unroll
    for (int ni = 0; ni < NI; ++ni)
      b[ni] = lds_frag<T>(Bs + (wn0 + 16 * ni + r) * P + kk + 4 * g);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < NI; ++ni) acc[mi][ni] = Mfma<T>::mma(a[mi][i], b[ni][i], acc[mi][ni]);
  }
}

template <typename T, int MI, int NI>
__device__ __forceinline__ void acc_zero(typename Mfma<T>::acc_t (&acc)[MI][NI]) {
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[mi][ni][j] = T(0);
}

template <typename T> struct Cplx;
template <> struct Cplx<float> { typedef float2 type; };
template <> struct Cplx<double> { typedef double2 type; };

}  // namespace bse
