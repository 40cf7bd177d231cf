// Device building blocks of the batched 3D complex FFT (gfx950, wave64).
//
// A 3D transform of the plane-wave basis is split into a plane pass (the two
// fastest axes, y and z, in LDS) and a column pass (the slowest axis, x, in
// LDS).  Within LDS each 1D transform runs as in-place mixed-radix
// Cooley-Tukey stages: decimation in frequency (forward, natural order in,
// digit-reversed order out) and decimation in time (inverse, digit-reversed
// in, natural out).  G space is therefore never put back in natural order;
// the kinetic and Poisson multipliers are laid out in the same digit-reversed
// order on the host.  Each stage is one radix-r butterfly per (line, index)
// work item; butterflies of a stage touch disjoint elements, so a stage needs
// one barrier and no scratch buffer.
#pragma once
#include <hip/hip_runtime.h>

namespace nct {

template <typename R>
struct cpx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b) {  // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename R>
__device__ __forceinline__ cpx<R> cscale(cpx<R> a, R s) { return {a.x * s, a.y * s}; }
// multiply by dir * i (dir = +1 or -1)
template <typename R, int DIR>
__device__ __forceinline__ cpx<R> mul_i(cpx<R> a) {
  if constexpr (DIR > 0) return {-a.y, a.x};
  else return {a.y, -a.x};
}

// exp(2 pi i k / 16) and exp(2 pi i k / 12), exact symmetric constants.
#define NCT_C8 0.92387953251128675613
#define NCT_S8 0.38268343236508977173
#define NCT_H2 0.70710678118654752440
#define NCT_R3 0.86602540378443864676
__device__ __forceinline__ constexpr double w16c(int k) {
  constexpr double t[16] = {1.0, NCT_C8, NCT_H2, NCT_S8, 0.0, -NCT_S8, -NCT_H2, -NCT_C8,
                            -1.0, -NCT_C8, -NCT_H2, -NCT_S8, 0.0, NCT_S8, NCT_H2, NCT_C8};
  return t[k & 15];
}
__device__ __forceinline__ constexpr double w16s(int k) {
  constexpr double t[16] = {0.0, NCT_S8, NCT_H2, NCT_C8, 1.0, NCT_C8, NCT_H2, NCT_S8,
                            0.0, -NCT_S8, -NCT_H2, -NCT_C8, -1.0, -NCT_C8, -NCT_H2, -NCT_S8};
  return t[k & 15];
}
__device__ __forceinline__ constexpr double w12c(int k) {
  constexpr double t[12] = {1.0, NCT_R3, 0.5, 0.0, -0.5, -NCT_R3, -1.0, -NCT_R3, -0.5, 0.0, 0.5, NCT_R3};
  return t[k % 12];
}
__device__ __forceinline__ constexpr double w12s(int k) {
  constexpr double t[12] = {0.0, 0.5, NCT_R3, 1.0, NCT_R3, 0.5, 0.0, -0.5, -NCT_R3, -1.0, -NCT_R3, -0.5};
  return t[k % 12];
}
// cos / sin of 2 pi e / RR for RR in {2,3,4,6,8,12,16}
template <int RR>
__device__ __forceinline__ constexpr double wc(int e) {
  if constexpr (16 % RR == 0) return w16c(e * (16 / RR));
  else return w12c(e * (12 / RR));
}
template <int RR>
__device__ __forceinline__ constexpr double ws(int e) {
  if constexpr (16 % RR == 0) return w16s(e * (16 / RR));
  else return w12s(e * (12 / RR));
}

// ---------------------------------------------------------------- small DFTs in registers
// y_k = sum_q x_q exp(DIR 2 pi i q k / RAD), natural order in and out.
template <typename R, int DIR, int RAD>
__device__ __forceinline__ void dft(cpx<R>* x);

template <typename R, int DIR>
__device__ __forceinline__ void dft2(cpx<R>* x) {
  cpx<R> a = x[0];
  x[0] = a + x[1];
  x[1] = a - x[1];
}
template <typename R, int DIR>
__device__ __forceinline__ void dft3(cpx<R>* x) {
  const R c = R(-0.5);
  const R s = R(DIR) * R(NCT_R3);
  cpx<R> t1 = x[1] + x[2];
  cpx<R> t2 = x[1] - x[2];
  cpx<R> m = {x[0].x + c * t1.x, x[0].y + c * t1.y};
  cpx<R> is = {-s * t2.y, s * t2.x};
  x[0] = x[0] + t1;
  x[1] = m + is;
  x[2] = m - is;
}
template <typename R, int DIR>
__device__ __forceinline__ void dft4(cpx<R>* x) {
  cpx<R> a = x[0] + x[2], b = x[0] - x[2], c = x[1] + x[3], d = x[1] - x[3];
  cpx<R> jd = mul_i<R, DIR>(d);
  x[0] = a + c;
  x[2] = a - c;
  x[1] = b + jd;
  x[3] = b - jd;
}
// RR = R1 * R2 in registers: R2 DFTs of size R1 (stride R2), twiddles, R1 DFTs of size R2,
// then the digit permutation back to natural order (free: register renaming).
template <typename R, int DIR, int R1, int R2>
__device__ __forceinline__ void dft_split(cpx<R>* x) {
  constexpr int RR = R1 * R2;
#pragma unroll
  for (int b = 0; b < R2; ++b) {
    cpx<R> t[R1];
#pragma unroll
    for (int q = 0; q < R1; ++q) t[q] = x[b + q * R2];
    dft<R, DIR, R1>(t);
#pragma unroll
    for (int p = 0; p < R1; ++p) {
      const int e = (b * p) % RR;
      if (e == 0) {
        x[b + p * R2] = t[p];
      } else {
        const cpx<R> w = {R(wc<RR>(e)), R(DIR) * R(ws<RR>(e))};
        x[b + p * R2] = cmul(t[p], w);
      }
    }
  }
  cpx<R> y[RR];
#pragma unroll
  for (int p = 0; p < R1; ++p) {
    cpx<R> t[R2];
#pragma unroll
    for (int q = 0; q < R2; ++q) t[q] = x[p * R2 + q];
    dft<R, DIR, R2>(t);
#pragma unroll
    for (int p2 = 0; p2 < R2; ++p2) y[p + R1 * p2] = t[p2];
  }
#pragma unroll
  for (int k = 0; k < RR; ++k) x[k] = y[k];
}

template <typename R, int DIR, int RAD>
__device__ __forceinline__ void dft(cpx<R>* x) {
  if constexpr (RAD == 1) {
  } else if constexpr (RAD == 2) {
    dft2<R, DIR>(x);
  } else if constexpr (RAD == 3) {
    dft3<R, DIR>(x);
  } else if constexpr (RAD == 4) {
    dft4<R, DIR>(x);
  } else if constexpr (RAD == 6) {
    dft_split<R, DIR, 3, 2>(x);
  } else if constexpr (RAD == 8) {
    dft_split<R, DIR, 4, 2>(x);
  } else if constexpr (RAD == 12) {
    dft_split<R, DIR, 4, 3>(x);
  } else if constexpr (RAD == 16) {
    dft_split<R, DIR, 4, 4>(x);
  } else {
    static_assert(RAD == 2, "unsupported radix");
  }
}

// ---------------------------------------------------------------- radix plans
// Radix of DIF stage s for a line of length N (0 = no such stage).  Radices stay <= 8 where a
// two-stage plan allows it, so a butterfly's data and twiddles fit in registers together.
__host__ __device__ constexpr int plan_radix(int N, int s) {
  switch (N) {
    case 4: return s == 0 ? 4 : 0;
    case 6: return s == 0 ? 6 : 0;
    case 8: return s == 0 ? 8 : 0;
    case 12: return s == 0 ? 4 : (s == 1 ? 3 : 0);
    case 16: return s == 0 ? 4 : (s == 1 ? 4 : 0);
    case 24: return s == 0 ? 8 : (s == 1 ? 3 : 0);
    case 32: return s == 0 ? 8 : (s == 1 ? 4 : 0);
    case 36: return s == 0 ? 6 : (s == 1 ? 6 : 0);
    case 48: return s == 0 ? 8 : (s == 1 ? 6 : 0);
    case 64: return s == 0 ? 8 : (s == 1 ? 8 : 0);
    case 72: return s == 0 ? 8 : (s == 1 ? 3 : (s == 2 ? 3 : 0));
    case 96: return s == 0 ? 8 : (s == 1 ? 12 : 0);
    case 128: return s == 0 ? 8 : (s == 1 ? 4 : (s == 2 ? 4 : 0));
    default: return 0;
  }
}
__host__ __device__ constexpr int plan_nstages(int N) {
  int k = 0;
  while (k < 4 && plan_radix(N, k) != 0) ++k;
  return k;
}
__host__ __device__ constexpr int plan_span(int N, int s) {
  int L = N;
  for (int i = 0; i < s; ++i) L /= plan_radix(N, i);
  return L;
}

// ---------------------------------------------------------------- one LDS stage
// NCT_TW_PRODUCTS (tuning macro): FP64 radix-8 butterflies read w1, w2 and w4 (1), w1 and w2 (2)
// or w1 (3) from the table and form the other twiddles as products (at most three roundings).
// Fewer values in flight: with three reads the FP64 64^2 plane pass spilled 56 instead of 72 B
// per lane and ran 5575 instead of 5455 GB/s (64^3 x 256), and the FP64 48^2 one no longer
// spills; two reads are what leave the forward FP64 64^2 kernel without spill.
#ifndef NCT_TW_PRODUCTS
#define NCT_TW_PRODUCTS 2
#endif
// Butterfly of stage STAGE on its RAD operands x (in place); b: index within the stage's block,
// tw[e] = exp(-2 pi i e / N).  Forward (DIF): DFT then twiddles; inverse (DIT): conjugate
// twiddles then DFT.
template <typename R, int N, int STAGE, bool FWD>
__device__ __forceinline__ void stage_butterfly(cpx<R>* x, const cpx<R>* tw, int b) {
  constexpr int RAD = plan_radix(N, STAGE);
  constexpr int SPAN = plan_span(N, STAGE);
  constexpr int M = SPAN / RAD;
  constexpr int TWS = N / SPAN;
  if constexpr (M > 1) {
    cpx<R> w[RAD - 1];
    if constexpr (NCT_TW_PRODUCTS && sizeof(R) == 8 && RAD == 8) {
      // FP64 radix 8: few table reads, the other twiddles as products of them, which keeps
      // fewer values in flight than seven reads
      const cpx<R> w1 = tw[b * TWS];
      const cpx<R> w2 = NCT_TW_PRODUCTS >= 3 ? cmul(w1, w1) : tw[b * 2 * TWS];
      const cpx<R> w4 = NCT_TW_PRODUCTS >= 2 ? cmul(w2, w2) : tw[b * 4 * TWS];
      w[0] = w1;
      w[1] = w2;
      w[3] = w4;
      w[2] = cmul(w1, w2);
      w[4] = cmul(w1, w4);
      w[5] = cmul(w2, w4);
      w[6] = cmul(w[2], w4);
    } else {
#pragma unroll
      for (int p = 1; p < RAD; ++p) w[p - 1] = tw[b * p * TWS];
    }
    if constexpr (FWD) {
      dft<R, -1, RAD>(x);
#pragma unroll
      for (int p = 1; p < RAD; ++p) x[p] = cmul(x[p], w[p - 1]);
    } else {
#pragma unroll
      for (int p = 1; p < RAD; ++p) x[p] = cmulc(x[p], w[p - 1]);
      dft<R, +1, RAD>(x);
    }
  } else {
    dft<R, FWD ? -1 : +1, RAD>(x);
  }
}

// Lines of length N at lds + line*LS + k*ES.  Work item it -> (line = it % NLINES, butterfly),
// so that neighbouring lanes work on neighbouring lines.
template <typename R, int N, int STAGE, int NLINES, int LS, int ES, bool FWD>
__device__ __forceinline__ void lds_stage(cpx<R>* lds, const cpx<R>* tw, int tid, int nt) {
  constexpr int RAD = plan_radix(N, STAGE);
  constexpr int SPAN = plan_span(N, STAGE);
  constexpr int M = SPAN / RAD;
  constexpr int NBF = N / RAD;
  constexpr int TOTAL = NLINES * NBF;
  for (int it = tid; it < TOTAL; it += nt) {
    const int line = it % NLINES;
    const int bfi = it / NLINES;
    const int blk = bfi / M;
    const int b = bfi - blk * M;
    cpx<R>* base = lds + line * LS + (blk * SPAN + b) * ES;
    cpx<R> x[RAD];
#pragma unroll
    for (int q = 0; q < RAD; ++q) x[q] = base[q * M * ES];
    stage_butterfly<R, N, STAGE, FWD>(x, tw, b);
#pragma unroll
    for (int q = 0; q < RAD; ++q) base[q * M * ES] = x[q];
  }
}

// A stage whose operands come from memory through ld(g) instead of LDS (g = line*GLS + k*GES,
// positions in an unpadded plane), results to LDS: the first stage of a transform fused with
// the load of its input.  Every load of the thread is issued before its first butterfly; a
// barrier precedes the butterflies (twiddles and earlier LDS writes visible) and follows the
// LDS writes.
template <typename R, int N, int STAGE, int NLINES, int LS, int ES, int GLS, int GES, int NT, bool FWD,
          typename LD>
__device__ __forceinline__ void stage_from(cpx<R>* lds, const cpx<R>* tw, int tid, LD ld) {
  constexpr int RAD = plan_radix(N, STAGE);
  constexpr int SPAN = plan_span(N, STAGE);
  constexpr int M = SPAN / RAD;
  constexpr int TOTAL = NLINES * (N / RAD);
  constexpr int IT = (TOTAL + NT - 1) / NT;
  cpx<R> x[IT][RAD];
#pragma unroll
  for (int u = 0; u < IT; ++u) {
    const int it = tid + u * NT;
    if ((u + 1) * NT <= TOTAL || it < TOTAL) {  // only a last, partial round has idle items
      const int line = it % NLINES;
      const int bfi = it / NLINES;
      const int blk = bfi / M;
      const int k0 = blk * SPAN + (bfi - blk * M);
#pragma unroll
      for (int q = 0; q < RAD; ++q) x[u][q] = ld(line * GLS + (k0 + q * M) * GES);
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < IT; ++u) {
    const int it = tid + u * NT;
    if (it < TOTAL) {
      const int line = it % NLINES;
      const int bfi = it / NLINES;
      const int blk = bfi / M;
      const int b = bfi - blk * M;
      stage_butterfly<R, N, STAGE, FWD>(x[u], tw, b);
      cpx<R>* base = lds + line * LS + (blk * SPAN + b) * ES;
#pragma unroll
      for (int q = 0; q < RAD; ++q) base[q * M * ES] = x[u][q];
    }
  }
  __syncthreads();
}

// A stage reading LDS whose results go to st(g, l, v, u) (g: unpadded position as above, l: the
// LDS position, v: the value, u: what pre(g) returned for that position, loaded before the
// butterflies) instead of back to LDS: the last stage of a transform fused with the store of its
// output.  No barrier.
template <typename R, int N, int STAGE, int NLINES, int LS, int ES, int GLS, int GES, int NT, bool FWD,
          typename PRE, typename ST>
__device__ __forceinline__ void stage_to(const cpx<R>* lds, const cpx<R>* tw, int tid, PRE pre, ST st) {
  constexpr int RAD = plan_radix(N, STAGE);
  constexpr int SPAN = plan_span(N, STAGE);
  constexpr int M = SPAN / RAD;
  constexpr int TOTAL = NLINES * (N / RAD);
  constexpr int IT = (TOTAL + NT - 1) / NT;
  using U = decltype(pre(0));
  U u[IT][RAD];
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int it = tid + k * NT;
    if ((k + 1) * NT <= TOTAL || it < TOTAL) {
      const int line = it % NLINES;
      const int bfi = it / NLINES;
      const int blk = bfi / M;
      const int k0 = blk * SPAN + (bfi - blk * M);
#pragma unroll
      for (int q = 0; q < RAD; ++q) u[k][q] = pre(line * GLS + (k0 + q * M) * GES);
    }
  }
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int it = tid + k * NT;
    if (it < TOTAL) {
      const int line = it % NLINES;
      const int bfi = it / NLINES;
      const int blk = bfi / M;
      const int b = bfi - blk * M;
      const int k0 = blk * SPAN + b;
      const cpx<R>* base = lds + line * LS + k0 * ES;
      cpx<R> x[RAD];
#pragma unroll
      for (int q = 0; q < RAD; ++q) x[q] = base[q * M * ES];
      stage_butterfly<R, N, STAGE, FWD>(x, tw, b);
#pragma unroll
      for (int q = 0; q < RAD; ++q)
        st(line * GLS + (k0 + q * M) * GES, line * LS + (k0 + q * M) * ES, x[q], u[k][q]);
    }
  }
}

// All stages of a line transform, a barrier after each stage.
template <typename R, int N, int NLINES, int LS, int ES, bool FWD>
__device__ __forceinline__ void lds_fft(cpx<R>* lds, const cpx<R>* tw, int tid, int nt) {
  constexpr int NS = plan_nstages(N);
  static_assert(NS >= 1 && NS <= 3, "line length not supported");
  if constexpr (FWD) {
    lds_stage<R, N, 0, NLINES, LS, ES, true>(lds, tw, tid, nt);
    __syncthreads();
    if constexpr (NS > 1) {
      lds_stage<R, N, 1, NLINES, LS, ES, true>(lds, tw, tid, nt);
      __syncthreads();
    }
    if constexpr (NS > 2) {
      lds_stage<R, N, 2, NLINES, LS, ES, true>(lds, tw, tid, nt);
      __syncthreads();
    }
  } else {
    if constexpr (NS > 2) {
      lds_stage<R, N, 2, NLINES, LS, ES, false>(lds, tw, tid, nt);
      __syncthreads();
    }
    if constexpr (NS > 1) {
      lds_stage<R, N, 1, NLINES, LS, ES, false>(lds, tw, tid, nt);
      __syncthreads();
    }
    lds_stage<R, N, 0, NLINES, LS, ES, false>(lds, tw, tid, nt);
    __syncthreads();
  }
}

// Forward / inverse 2D transform of an NY x NZ plane held at lds[y*PZ + z].
template <typename R, int NY, int NZ, int PZ>
__device__ __forceinline__ void plane_fft_fwd(cpx<R>* lds, const cpx<R>* twy, const cpx<R>* twz,
                                              int tid, int nt) {
  // rows: NY lines of length NZ, line stride PZ, element stride 1
  lds_fft<R, NZ, NY, PZ, 1, true>(lds, twz, tid, nt);
  // columns: NZ lines of length NY, line stride 1, element stride PZ
  lds_fft<R, NY, NZ, 1, PZ, true>(lds, twy, tid, nt);
}
template <typename R, int NY, int NZ, int PZ>
__device__ __forceinline__ void plane_fft_inv(cpx<R>* lds, const cpx<R>* twy, const cpx<R>* twz,
                                              int tid, int nt) {
  lds_fft<R, NY, NZ, 1, PZ, false>(lds, twy, tid, nt);
  lds_fft<R, NZ, NY, PZ, 1, false>(lds, twz, tid, nt);
}

// Inverse 2D transform of a plane read through ld(y*NZ + z) (digit-reversed (y,z) order, as the
// forward transform leaves it) into lds[y*PZ + z]: the first column stage is fused with the load.
// No barrier is needed before the call; one follows it.
template <typename R, int NY, int NZ, int PZ, int NT, typename LD>
__device__ __forceinline__ void plane_fft_inv_from(cpx<R>* lds, const cpx<R>* twy, const cpx<R>* twz, int tid,
                                                   LD ld) {
  constexpr int NS = plan_nstages(NY);
  stage_from<R, NY, NS - 1, NZ, 1, PZ, 1, NZ, NT, false>(lds, twy, tid, ld);
  if constexpr (NS > 2) {
    lds_stage<R, NY, 1, NZ, 1, PZ, false>(lds, twy, tid, NT);
    __syncthreads();
  }
  if constexpr (NS > 1) {
    lds_stage<R, NY, 0, NZ, 1, PZ, false>(lds, twy, tid, NT);
    __syncthreads();
  }
  lds_fft<R, NZ, NY, PZ, 1, false>(lds, twz, tid, NT);
}
// Forward 2D transform of lds[y*PZ + z] whose output goes to st(y*NZ + z, y*PZ + z, value,
// pre(y*NZ + z)): the last column stage is fused with the store.  Needs a barrier before the call; none follows it.
template <typename R, int NY, int NZ, int PZ, int NT, typename PRE, typename ST>
__device__ __forceinline__ void plane_fft_fwd_to(cpx<R>* lds, const cpx<R>* twy, const cpx<R>* twz, int tid,
                                                 PRE pre, ST st) {
  constexpr int NS = plan_nstages(NY);
  lds_fft<R, NZ, NY, PZ, 1, true>(lds, twz, tid, NT);
  if constexpr (NS > 1) {
    lds_stage<R, NY, 0, NZ, 1, PZ, true>(lds, twy, tid, NT);
    __syncthreads();
  }
  if constexpr (NS > 2) {
    lds_stage<R, NY, 1, NZ, 1, PZ, true>(lds, twy, tid, NT);
    __syncthreads();
  }
  stage_to<R, NY, NS - 1, NZ, 1, PZ, 1, NZ, NT, true>(lds, twy, tid, pre, st);
}

// Workgroup index remap so that consecutive logical indices run on one XCD.
// The hardware deals workgroups round-robin to the 8 XCDs (block b -> XCD b % 8).
__device__ __forceinline__ int xcd_logical(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int k = b & 7;
  return k * q + (k < r ? k : r) + (b >> 3);
}

}  // namespace nct
