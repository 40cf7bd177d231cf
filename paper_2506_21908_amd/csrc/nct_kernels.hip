// HIP kernels of the non-collinear TDDFT step for gfx950 (MI355X), wave64.
//
// H application (Eq. HNC-SDFT / TDSDFT) as two passes over HBM:
//   column pass  (k_xpass):  DFT_x -> multiply 1/2|G|^2/N -> IDFT_x on the
//                            (y,z)-transformed states, tiles of TC columns in LDS;
//   plane pass   (k_plane_stage): per (state, x-plane), both spinor components:
//                            IDFT_yz -> T w; V w with the 2x2 local potential
//                            [v + b.sigma]; + projector scatter rows; Taylor
//                            (Horner) update out = alpha x + c H w; sphere rows of
//                            out for the next projection; DFT_yz of out for the
//                            next column pass.
// Densities, exchange, Hartree and reductions are FP64.  The projector
// contraction <beta|psi> and its scatter-back run on the matrix cores
// (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>

#include "nct_fft.hpp"
#include "nct_internal.hpp"

namespace nct {

// threads per plane workgroup: smallest power of two >= 64 with at most 9 points per thread
__host__ __device__ constexpr int plane_nt(int np) {
  int nt = 64;
  while (nt < 1024 && (np + nt - 1) / nt > 9) nt *= 2;
  return nt;
}
template <int NY, int NZ>
constexpr size_t plane_lds_bytes(size_t elem) {
  return (size_t(NY) * (NZ + 1) + NY + NZ) * elem;
}

// ---------------------------------------------------------------- block reductions
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  // wave64 butterfly then a fixed-order sum over waves: deterministic
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int k = 0; k < NT / 64; ++k) s += red[k];
  }
  return s;  // valid on thread 0
}

// ---------------------------------------------------------------- streamed global access
// Cache policy of the large streamed operands (the state-sized buffers), chosen per system from
// the size of one state set: M = 0 plain loads and stores; M = 1 non-temporal (streaming)
// stores; M = 2 non-temporal loads as well.  Streaming keeps buffers that will not be re-read
// from the caches before eviction from displacing the shared fields and twiddles; for state
// sets small enough to stay cache-resident between passes plain accesses are faster.
template <int M, typename R>
__device__ __forceinline__ cpx<R> ld_stream(const cpx<R>* p) {
  if constexpr (M >= 2) {
    typedef R v2 __attribute__((ext_vector_type(2)));
    const v2 t = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return cpx<R>{t.x, t.y};
  } else {
    return *p;
  }
}
template <int M, typename R>
__device__ __forceinline__ void st_stream(cpx<R>* p, cpx<R> v) {
  if constexpr (M >= 1) {
    typedef R v2 __attribute__((ext_vector_type(2)));
    v2 t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, reinterpret_cast<v2*>(p));
  } else {
    *p = v;
  }
}

// Bloch phase exp(i q.d) of one sphere row (q: Bloch vector, d: the row's displacement from its
// atom).  Rows gathered for the projections carry it, scattered rows its conjugate.
// (q passed as scalars: an addressable local array would live in scratch memory)
__device__ __forceinline__ cpx<double> bloch_phase(double q0, double q1, double q2, const double* d) {
  double sn, cs;
  sincos(q0 * d[0] + q1 * d[1] + q2 * d[2], &sn, &cs);
  return {cs, sn};
}
__device__ __forceinline__ cpx<float> bloch_phase(float q0, float q1, float q2, const float* d) {
  float sn, cs;
  sincosf(q0 * d[0] + q1 * d[1] + q2 * d[2], &sn, &cs);
  return {cs, sn};
}

// ---------------------------------------------------------------- plane pass: fused H stage
template <typename R, int NY, int NZ, int M>
__global__ __launch_bounds__(plane_nt(NY* NZ)) void k_plane_stage(StageArgs<R> a, ProjTables pt,
                                                                   const cpx<R>* __restrict__ twy_g,
                                                                   const cpx<R>* __restrict__ twz_g,
                                                                   int S, int NX) {
  constexpr int NP = NY * NZ;
  constexpr int NT = plane_nt(NP);
  constexpr int PZ = NZ + 1;
  constexpr int PPT = (NP + NT - 1) / NT;
  extern __shared__ double4 smem_d4[];
  cpx<R>* plane = reinterpret_cast<cpx<R>*>(smem_d4);
  cpx<R>* twy = plane + NY * PZ;
  cpx<R>* twz = twy + NY;
  const int tid = threadIdx.x;
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  const int x = L / S;
  const int i = L - x * S;
  for (int k = tid; k < NY; k += NT) twy[k] = twy_g[k];
  for (int k = tid; k < NZ; k += NT) twz[k] = twz_g[k];
  const size_t N = size_t(NX) * NP;
  size_t off[2];
  off[0] = (size_t(2 * i) * NX + x) * NP;
  off[1] = (size_t(2 * i + 1) * NX + x) * NP;
  const cpx<R>* __restrict__ tin = reinterpret_cast<const cpx<R>*>(a.tmp_in);
  cpx<R> hv[2][PPT];

  // 1) kinetic part: inverse 2D transform of the column-pass output, both spinors
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int e = tid + j * NT;
      if (e < NP) plane[(e / NZ) * PZ + (e % NZ)] = ld_stream<M>(&tin[off[s] + e]);
    }
    __syncthreads();
    plane_fft_inv<R, NY, NZ, PZ>(plane, twy, twz, tid, NT);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int e = tid + j * NT;
      if (e < NP) hv[s][j] = plane[(e / NZ) * PZ + (e % NZ)];
    }
    __syncthreads();
  }

  // 2) local 2x2 potential and Taylor update, pointwise
  const cpx<R>* __restrict__ win = reinterpret_cast<const cpx<R>*>(a.w_in);
  const cpx<R>* __restrict__ xb = reinterpret_cast<const cpx<R>*>(a.x_base);
  const R* __restrict__ F = a.fields;
  const R lx = a.lg[0] * R(x) + a.lg[3];  // laser potential of this plane, less its y, z terms
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int e = tid + j * NT;
    if (e < NP) {
      const size_t p = size_t(x) * NP + e;
      const R v = F[p] + (lx + a.lg[1] * R(e / NZ) + a.lg[2] * R(e % NZ));
      const R bx = F[N + p] + a.bext[0];
      const R by = F[2 * N + p] + a.bext[1];
      const R bz = F[3 * N + p] + a.bext[2];
      const cpx<R> wu = ld_stream<M>(&win[off[0] + e]);
      const cpx<R> wd = ld_stream<M>(&win[off[1] + e]);
      // up' = (v+bz) up + (bx - i by) dn ; dn' = (bx + i by) up + (v - bz) dn
      cpx<R> hu, hd;
      hu.x = hv[0][j].x + (v + bz) * wu.x + bx * wd.x + by * wd.y;
      hu.y = hv[0][j].y + (v + bz) * wu.y + bx * wd.y - by * wd.x;
      hd.x = hv[1][j].x + bx * wu.x - by * wu.y + (v - bz) * wd.x;
      hd.y = hv[1][j].y + bx * wu.y + by * wu.x + (v - bz) * wd.y;
      cpx<R> ou = {a.cre * hu.x - a.cim * hu.y, a.cre * hu.y + a.cim * hu.x};
      cpx<R> od = {a.cre * hd.x - a.cim * hd.y, a.cre * hd.y + a.cim * hd.x};
      if (xb) {
        const cpx<R> xu = ld_stream<M>(&xb[off[0] + e]);
        const cpx<R> xd = ld_stream<M>(&xb[off[1] + e]);
        ou.x += a.alpha * xu.x;
        ou.y += a.alpha * xu.y;
        od.x += a.alpha * xd.x;
        od.y += a.alpha * xd.y;
      }
      hv[0][j] = ou;
      hv[1][j] = od;
    }
  }

  // 3) per spinor: projector rows, outputs, forward 2D transform
  const cpx<R>* __restrict__ Y = reinterpret_cast<const cpx<R>*>(a.Y);
  cpx<R>* __restrict__ Wr = reinterpret_cast<cpx<R>*>(a.W);
  cpx<R>* __restrict__ wout = reinterpret_cast<cpx<R>*>(a.w_out);
  cpx<R>* __restrict__ acc = reinterpret_cast<cpx<R>*>(a.acc);
  cpx<R>* __restrict__ tout = reinterpret_cast<cpx<R>*>(a.tmp_out);
  const int r0 = pt.pr_off ? pt.pr_off[x] : 0;
  const int r1 = pt.pr_off ? pt.pr_off[x + 1] : 0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int e = tid + j * NT;
      if (e < NP) plane[(e / NZ) * PZ + (e % NZ)] = hv[s][j];
    }
    __syncthreads();
    const size_t rowbase = size_t(2 * i + s) * pt.Jtot;
    const bool kq = a.kv != nullptr;
    R q0 = 0, q1 = 0, q2 = 0;
    if (kq) {
      const R* k0 = a.kv + 3 * (a.state_off + i);
      q0 = k0[0] + a.ka[0];
      q1 = k0[1] + a.ka[1];
      q2 = k0[2] + a.ka[2];
    }
    const R* disp = reinterpret_cast<const R*>(pt.disp);
    if (Y) {
      for (int r = r0; r < r1; ++r) {
        const int jb = pt.pr_begin[r], je = pt.pr_end[r];
        for (int J = jb + tid; J < je; J += NT) {
          const int e = pt.pidx[J];
          cpx<R> y = Y[rowbase + J];
          if (kq) y = cmulc(y, bloch_phase(q0, q1, q2, disp + 3 * J));
          cpx<R>& d = plane[(e / NZ) * PZ + (e % NZ)];
          d.x += a.cre * y.x - a.cim * y.y;
          d.y += a.cre * y.y + a.cim * y.x;
        }
        __syncthreads();
      }
    }
    if (Wr) {
      for (int r = r0; r < r1; ++r) {
        const int jb = pt.pr_begin[r], je = pt.pr_end[r];
        for (int J = jb + tid; J < je; J += NT) {
          const int e = pt.pidx[J];
          cpx<R> o = plane[(e / NZ) * PZ + (e % NZ)];
          if (kq) o = cmul(o, bloch_phase(q0, q1, q2, disp + 3 * J));
          Wr[rowbase + J] = o;
        }
      }
    }
    if (wout || acc) {
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        const int e = tid + j * NT;
        if (e < NP) {
          const cpx<R> o = plane[(e / NZ) * PZ + (e % NZ)];
          if (wout) st_stream<M>(&wout[off[s] + e], o);
          if (acc) {
            cpx<R> q = acc[off[s] + e];
            acc[off[s] + e] = q + o;
          }
        }
      }
    }
    if (tout) {
      __syncthreads();
      plane_fft_fwd<R, NY, NZ, PZ>(plane, twy, twz, tid, NT);
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        const int e = tid + j * NT;
        if (e < NP) st_stream<M>(&tout[off[s] + e], plane[(e / NZ) * PZ + (e % NZ)]);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- plane pass, two halves
// Same stage as k_plane_stage, with the two spinor components of the (state, x-plane) held as
// two LDS planes and transformed concurrently by the two halves of the workgroup; the pointwise
// 2x2 update then reads both planes.  Used when two planes fit in LDS.
// Threads per spinor half: plane_nt's choice capped at NCT_PLANE2_NTH_MAX (tuning macro), except
// FP64 48^2 planes.  There LDS admits two workgroups per CU, and 256 threads per half at 98 VGPRs
// keep only 16 waves per CU; 384 threads (6 points each, 2304 = 6 x 384) with a register target
// of 6 waves per SIMD (80 VGPRs) keep 24 and measured 3 % faster on MI355X.  320 and 448 threads
// (a partial last round) and 512 (spills at 64 VGPRs) measured slower.
#ifndef NCT_PLANE2_NTH_MAX_F64
#define NCT_PLANE2_NTH_MAX_F64 512
#endif
#ifndef NCT_PLANE2_NTH_MAX_F32
#define NCT_PLANE2_NTH_MAX_F32 512
#endif
template <typename R>
__host__ __device__ constexpr int plane2_nth(int np) {
  if (sizeof(R) == 8 && np == 48 * 48) return 384;
  const int cap = sizeof(R) == 8 ? NCT_PLANE2_NTH_MAX_F64 : NCT_PLANE2_NTH_MAX_F32;
  return plane_nt(np) > cap ? cap : plane_nt(np);
}
// Minimum waves per SIMD the register allocation of the two-half kernel must allow, where LDS
// admits more workgroups per CU than the registers would: FP64 48^2 (above), and FP32 64^2,
// whose two 66 KB workgroups of 16 waves need 8 waves per SIMD: at 68 VGPRs only one fitted, at
// 63 both do (measured 1159 -> 949 us per launch at 64^3 x 256).
template <typename R>
__host__ __device__ constexpr int plane2_min_waves(int np) {
  if (sizeof(R) == 8 && np == 48 * 48) return 6;
  if (sizeof(R) == 4 && np == 64 * 64) return 8;
  return 1;
}
template <int NY, int NZ>
constexpr size_t plane2_lds_bytes(size_t elem) {
  return (size_t(2) * NY * (NZ + 1) + NY + NZ) * elem;
}
// LDS budget of the two-plane kernel (tuning macro; 160 KiB per CU less a margin)
#ifndef NCT_PLANE2_MAX_LDS
#define NCT_PLANE2_MAX_LDS (160 * 1024 - 1024)
#endif
template <typename R, int NY, int NZ>
constexpr bool plane2_fits() {
  return plane2_lds_bytes<NY, NZ>(sizeof(cpx<R>)) <= NCT_PLANE2_MAX_LDS;
}

template <typename R, int NY, int NZ, int M>
__global__ __launch_bounds__(2 * plane2_nth<R>(NY* NZ), plane2_min_waves<R>(NY* NZ)) void k_plane_stage2(StageArgs<R> a, ProjTables pt,
                                                                          const cpx<R>* __restrict__ twy_g,
                                                                          const cpx<R>* __restrict__ twz_g,
                                                                          int S, int NX) {
  constexpr int NP = NY * NZ;
  constexpr int NTH = plane2_nth<R>(NP);
  constexpr int NT = 2 * NTH;
  constexpr int PZ = NZ + 1;
  constexpr int PL = NY * PZ;
  constexpr int PPH = (NP + NTH - 1) / NTH;
  constexpr int PPT = (NP + NT - 1) / NT;
#ifndef NCT_PLANE2_G_F64
#define NCT_PLANE2_G_F64 3
#endif
#ifndef NCT_PLANE2_G_F32
#define NCT_PLANE2_G_F32 3
#endif
  // pointwise points per load batch (2 for FP64 48^2, where 3 spills at that case's register target)
  constexpr int G = (sizeof(R) == 8 && NP == 48 * 48) ? 2 : (sizeof(R) == 8 ? NCT_PLANE2_G_F64 : NCT_PLANE2_G_F32);
  extern __shared__ double4 smem_d4[];
  cpx<R>* planes = reinterpret_cast<cpx<R>*>(smem_d4);
  cpx<R>* twy = planes + 2 * PL;
  cpx<R>* twz = twy + NY;
  const int tid = threadIdx.x;
  const int h = tid / NTH;
  const int th = tid - h * NTH;
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  const int x = L / S;
  const int i = L - x * S;
  for (int k = tid; k < NY; k += NT) twy[k] = twy_g[k];
  for (int k = tid; k < NZ; k += NT) twz[k] = twz_g[k];
  const size_t N = size_t(NX) * NP;
  const size_t off0 = (size_t(2 * i) * NX + x) * NP;
  const size_t off1 = (size_t(2 * i + 1) * NX + x) * NP;
  const size_t offh = h ? off1 : off0;
  cpx<R>* pl = planes + h * PL;

  // 1) kinetic part: each half loads and inverse-transforms its spinor's plane (the first
  //    transform stage works on the loaded values)
  {
    const cpx<R>* __restrict__ tin = reinterpret_cast<const cpx<R>*>(a.tmp_in) + offh;
    plane_fft_inv_from<R, NY, NZ, PZ, NTH>(pl, twy, twz, th, [&](int g) { return ld_stream<M>(&tin[g]); });
  }

  // 2) 2x2 local potential and Taylor update over the whole plane (both spinors per point)
  {
    const cpx<R>* __restrict__ win = reinterpret_cast<const cpx<R>*>(a.w_in);
    const cpx<R>* __restrict__ xb = reinterpret_cast<const cpx<R>*>(a.x_base);
    const bool xsep = xb && (a.x_base != a.w_in);
    const R* __restrict__ F = a.fields;
    const R lx = a.lg[0] * R(x) + a.lg[3];  // laser potential of this plane, less its y, z terms
#pragma unroll
    for (int j0 = 0; j0 < PPT; j0 += G) {
      cpx<R> wu[G], wd[G], xu[G], xd[G];
      R fv[G], fx[G], fy[G], fz[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (j0 + g < PPT) {
          const int e = min(tid + (j0 + g) * NT, NP - 1);  // clamped: loads unconditional
          const size_t p = size_t(x) * NP + e;
          wu[g] = ld_stream<M>(&win[off0 + e]);
          wd[g] = ld_stream<M>(&win[off1 + e]);
          if (xsep) {
            xu[g] = ld_stream<M>(&xb[off0 + e]);
            xd[g] = ld_stream<M>(&xb[off1 + e]);
          } else {
            xu[g] = wu[g];
            xd[g] = wd[g];
          }
          fv[g] = F[p];
          fx[g] = F[N + p];
          fy[g] = F[2 * N + p];
          fz[g] = F[3 * N + p];
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int e = tid + (j0 + g) * NT;
        if (j0 + g < PPT && e < NP) {
          const int q = (e / NZ) * PZ + (e % NZ);
          const cpx<R> tu = planes[q], td = planes[PL + q];
          const R v = fv[g] + (lx + a.lg[1] * R(e / NZ) + a.lg[2] * R(e % NZ));
          const R bx = fx[g] + a.bext[0], by = fy[g] + a.bext[1], bz = fz[g] + a.bext[2];
          cpx<R> hu, hd;
          hu.x = tu.x + (v + bz) * wu[g].x + bx * wd[g].x + by * wd[g].y;
          hu.y = tu.y + (v + bz) * wu[g].y + bx * wd[g].y - by * wd[g].x;
          hd.x = td.x + bx * wu[g].x - by * wu[g].y + (v - bz) * wd[g].x;
          hd.y = td.y + bx * wu[g].y + by * wu[g].x + (v - bz) * wd[g].y;
          cpx<R> ou = {a.cre * hu.x - a.cim * hu.y, a.cre * hu.y + a.cim * hu.x};
          cpx<R> od = {a.cre * hd.x - a.cim * hd.y, a.cre * hd.y + a.cim * hd.x};
          if (xb) {
            ou.x += a.alpha * xu[g].x;
            ou.y += a.alpha * xu[g].y;
            od.x += a.alpha * xd[g].x;
            od.y += a.alpha * xd[g].y;
          }
          planes[q] = ou;
          planes[PL + q] = od;
        }
      }
    }
  }
  __syncthreads();

  // 3) projector rows, outputs, forward transform; each half its own spinor
  const cpx<R>* __restrict__ Y = reinterpret_cast<const cpx<R>*>(a.Y);
  cpx<R>* __restrict__ Wr = reinterpret_cast<cpx<R>*>(a.W);
  cpx<R>* __restrict__ wout = reinterpret_cast<cpx<R>*>(a.w_out);
  cpx<R>* __restrict__ acc = reinterpret_cast<cpx<R>*>(a.acc);
  cpx<R>* __restrict__ tout = reinterpret_cast<cpx<R>*>(a.tmp_out);
  const int r0 = pt.pr_off ? pt.pr_off[x] : 0;
  const int r1 = pt.pr_off ? pt.pr_off[x + 1] : 0;
  const size_t rowbase = size_t(2 * i + h) * pt.Jtot;
  const bool kq = a.kv != nullptr;
  R q0 = 0, q1 = 0, q2 = 0;
  if (kq) {
    const R* k0 = a.kv + 3 * (a.state_off + i);
    q0 = k0[0] + a.ka[0];
    q1 = k0[1] + a.ka[1];
    q2 = k0[2] + a.ka[2];
  }
  const R* disp = reinterpret_cast<const R*>(pt.disp);
  if (Y) {
    for (int r = r0; r < r1; ++r) {
      const int jb = pt.pr_begin[r], je = pt.pr_end[r];
      for (int J = jb + th; J < je; J += NTH) {
        const int e = pt.pidx[J];
        cpx<R> y = Y[rowbase + J];
        if (kq) y = cmulc(y, bloch_phase(q0, q1, q2, disp + 3 * J));
        cpx<R>& d = pl[(e / NZ) * PZ + (e % NZ)];
        d.x += a.cre * y.x - a.cim * y.y;
        d.y += a.cre * y.y + a.cim * y.x;
      }
      __syncthreads();
    }
  }
  if (Wr) {
    for (int r = r0; r < r1; ++r) {
      const int jb = pt.pr_begin[r], je = pt.pr_end[r];
      for (int J = jb + th; J < je; J += NTH) {
        const int e = pt.pidx[J];
        cpx<R> o = pl[(e / NZ) * PZ + (e % NZ)];
        if (kq) o = cmul(o, bloch_phase(q0, q1, q2, disp + 3 * J));
        Wr[rowbase + J] = o;
      }
    }
  }
  if (acc) {
    cpx<R> v[PPH];
#pragma unroll
    for (int j = 0; j < PPH; ++j) v[j] = acc[offh + min(th + j * NTH, NP - 1)];
#pragma unroll
    for (int j = 0; j < PPH; ++j) {
      const int e = th + j * NTH;
      if (e < NP) acc[offh + e] = v[j] + pl[(e / NZ) * PZ + (e % NZ)];
    }
  }
  if (wout) {
#pragma unroll
    for (int j = 0; j < PPH; ++j) {
      const int e = th + j * NTH;
      if (e < NP) st_stream<M>(&wout[offh + e], pl[(e / NZ) * PZ + (e % NZ)]);
    }
  }
  if (tout) {
    __syncthreads();
    cpx<R>* __restrict__ to = tout + offh;
    plane_fft_fwd_to<R, NY, NZ, PZ, NTH>(pl, twy, twz, th, [](int) { return 0; },
                                         [&](int g, int, cpx<R> v, int) { st_stream<M>(&to[g], v); });
  }
}

// ---------------------------------------------------------------- plane pass, one plane in LDS
// Same stage as k_plane_stage2 for planes where two LDS planes would admit only one workgroup per
// CU but one plane admits two (FP64 64^2: 67 KB; FP32 96^2: 76 KB).  The spinor components go
// through the single LDS plane one after the other: the up component's kinetic part waits in
// registers (PPT values per thread, the last of them in a private LDS slot per thread) while the
// down component is transformed; after the 2x2 update the up result waits there again while the
// down result is finished and transformed forward.
// Two resident workgroups per CU interleave their memory and transform phases.
// Threads per workgroup (tuning macro) and the point batch of the 2x2 update.
#ifndef NCT_PLANER_NT
#define NCT_PLANER_NT 512
#endif
// NCT_PLANER_OFF (tuning macro) keeps those planes on the two-plane kernel.
template <typename R, int NY, int NZ>
constexpr bool planer_use() {
#ifdef NCT_PLANER_OFF
  return false;
#else
  return plane2_lds_bytes<NY, NZ>(sizeof(cpx<R>)) > 80 * 1024 &&
         plane_lds_bytes<NY, NZ>(sizeof(cpx<R>)) <= 80 * 1024 - 512;
#endif
}

// Values per thread of the held spinor component that live in LDS left over by the plane
// (tuning macro NCT_PLANER_KL: at most that many, within the 80 KB of two workgroups per CU).
// One slot takes four of the 128 VGPRs off the held values: FP64 64^2 spills 36 instead of 56 B
// per lane and its plane pass runs 5707 instead of 5575 GB/s (64^3 x 256).
#ifndef NCT_PLANER_KL
#define NCT_PLANER_KL 1
#endif
template <typename R, int NY, int NZ>
constexpr int planer_kl() {
  constexpr size_t spare = 80 * 1024 - 512 - plane_lds_bytes<NY, NZ>(sizeof(cpx<R>));
  constexpr int fit = int(spare / (size_t(NCT_PLANER_NT) * sizeof(cpx<R>)));
  constexpr int ppt = (NY * NZ + NCT_PLANER_NT - 1) / NCT_PLANER_NT;
  constexpr int kl = NCT_PLANER_KL < fit ? NCT_PLANER_KL : fit;
  return kl < ppt ? kl : ppt;
}
template <typename R, int NY, int NZ>
constexpr size_t planer_lds_bytes() {
  return plane_lds_bytes<NY, NZ>(sizeof(cpx<R>)) + size_t(planer_kl<R, NY, NZ>()) * NCT_PLANER_NT * sizeof(cpx<R>);
}

// ACC: the kernel carries the adjoint's accumulation acc += w_out (only the adjoint passes acc).
template <typename R, int NY, int NZ, int M, bool ACC>
__global__ __launch_bounds__(NCT_PLANER_NT, 4) void k_plane_stage_r(StageArgs<R> a, ProjTables pt,
                                                                     const cpx<R>* __restrict__ twy_g,
                                                                     const cpx<R>* __restrict__ twz_g,
                                                                     int S, int NX) {
  constexpr int NP = NY * NZ;
  constexpr int NT = NCT_PLANER_NT;
  constexpr int PZ = NZ + 1;
  constexpr int PPT = (NP + NT - 1) / NT;
  constexpr int KR = PPT - planer_kl<R, NY, NZ>();  // held values in registers, the rest in LDS
#ifndef NCT_PLANER_G_F64  // points per load batch of the FP64 2x2 update (tuning macro)
#define NCT_PLANER_G_F64 2
#endif
  constexpr int G = sizeof(R) == 8 ? NCT_PLANER_G_F64 : 3;  // points per load batch of the 2x2 update
  extern __shared__ double4 smem_d4[];
  cpx<R>* pl = reinterpret_cast<cpx<R>*>(smem_d4);
  cpx<R>* twy = pl + NY * PZ;
  cpx<R>* twz = twy + NY;
  cpx<R>* kus = twz + NZ;  // [PPT - KR][NT]: each thread's own held values beyond KR
  const int tid = threadIdx.x;
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  const int x = L / S;
  const int i = L - x * S;
  for (int k = tid; k < NY; k += NT) twy[k] = twy_g[k];
  for (int k = tid; k < NZ; k += NT) twz[k] = twz_g[k];
  const size_t N = size_t(NX) * NP;
  const size_t off0 = (size_t(2 * i) * NX + x) * NP;
  const size_t off1 = (size_t(2 * i + 1) * NX + x) * NP;
  const cpx<R>* __restrict__ tin = reinterpret_cast<const cpx<R>*>(a.tmp_in);

  // 1) kinetic part of the up component (inverse 2D transform), kept in registers (the first KR
  //    values of each thread) and in the thread's own LDS slots (the rest)
  plane_fft_inv_from<R, NY, NZ, PZ, NT>(pl, twy, twz, tid, [&](int g) { return ld_stream<M>(&tin[off0 + g]); });
  cpx<R> ku[KR > 0 ? KR : 1];
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int e = min(tid + j * NT, NP - 1);
    const cpx<R> v = pl[(e / NZ) * PZ + (e % NZ)];
    if (j < KR) ku[j < KR ? j : 0] = v;
    else kus[(j - KR) * NT + tid] = v;
  }
  __syncthreads();
  // 2) kinetic part of the down component, left in LDS
  plane_fft_inv_from<R, NY, NZ, PZ, NT>(pl, twy, twz, tid, [&](int g) { return ld_stream<M>(&tin[off1 + g]); });

  // 3) 2x2 local potential and Taylor update: up result back into ku, down result into LDS
  {
    const cpx<R>* __restrict__ win = reinterpret_cast<const cpx<R>*>(a.w_in);
    const cpx<R>* __restrict__ xb = reinterpret_cast<const cpx<R>*>(a.x_base);
    const bool xsep = xb && (a.x_base != a.w_in);
    const R* __restrict__ F = a.fields;
    const R lx = a.lg[0] * R(x) + a.lg[3];  // laser potential of this plane, less its y, z terms
#pragma unroll
    for (int j0 = 0; j0 < PPT; j0 += G) {
      cpx<R> wu[G], wd[G], xu[G], xd[G];
      R fv[G], fx[G], fy[G], fz[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (j0 + g < PPT) {
          const int e = min(tid + (j0 + g) * NT, NP - 1);  // clamped: loads unconditional
          const size_t p = size_t(x) * NP + e;
          wu[g] = ld_stream<M>(&win[off0 + e]);
          wd[g] = ld_stream<M>(&win[off1 + e]);
          if (xsep) {
            xu[g] = ld_stream<M>(&xb[off0 + e]);
            xd[g] = ld_stream<M>(&xb[off1 + e]);
          } else {
            xu[g] = wu[g];
            xd[g] = wd[g];
          }
          fv[g] = F[p];
          fx[g] = F[N + p];
          fy[g] = F[2 * N + p];
          fz[g] = F[3 * N + p];
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int j = j0 + g;
        const int e = tid + j * NT;
        if (j < PPT && e < NP) {
          const int q = (e / NZ) * PZ + (e % NZ);
          const cpx<R> tu = j < KR ? ku[j < KR ? j : 0] : kus[(j - KR) * NT + tid], td = pl[q];
          const R v = fv[g] + (lx + a.lg[1] * R(e / NZ) + a.lg[2] * R(e % NZ));
          const R bx = fx[g] + a.bext[0], by = fy[g] + a.bext[1], bz = fz[g] + a.bext[2];
          cpx<R> hu, hd;
          hu.x = tu.x + (v + bz) * wu[g].x + bx * wd[g].x + by * wd[g].y;
          hu.y = tu.y + (v + bz) * wu[g].y + bx * wd[g].y - by * wd[g].x;
          hd.x = td.x + bx * wu[g].x - by * wu[g].y + (v - bz) * wd[g].x;
          hd.y = td.y + bx * wu[g].y + by * wu[g].x + (v - bz) * wd[g].y;
          cpx<R> ou = {a.cre * hu.x - a.cim * hu.y, a.cre * hu.y + a.cim * hu.x};
          cpx<R> od = {a.cre * hd.x - a.cim * hd.y, a.cre * hd.y + a.cim * hd.x};
          if (xb) {
            ou.x += a.alpha * xu[g].x;
            ou.y += a.alpha * xu[g].y;
            od.x += a.alpha * xd[g].x;
            od.y += a.alpha * xd[g].y;
          }
          if (j < KR) ku[j < KR ? j : 0] = ou;
          else kus[(j - KR) * NT + tid] = ou;
          pl[q] = od;
        }
      }
    }
  }
  __syncthreads();

  // 4) per component (down, then up): projector rows, outputs, forward transform
  const cpx<R>* __restrict__ Y = reinterpret_cast<const cpx<R>*>(a.Y);
  cpx<R>* __restrict__ Wr = reinterpret_cast<cpx<R>*>(a.W);
  cpx<R>* __restrict__ wout = reinterpret_cast<cpx<R>*>(a.w_out);
  cpx<R>* __restrict__ acc = reinterpret_cast<cpx<R>*>(a.acc);
  cpx<R>* __restrict__ tout = reinterpret_cast<cpx<R>*>(a.tmp_out);
  const int r0 = pt.pr_off ? pt.pr_off[x] : 0;
  const int r1 = pt.pr_off ? pt.pr_off[x + 1] : 0;
  const bool kq = a.kv != nullptr;
  R q0 = 0, q1 = 0, q2 = 0;
  if (kq) {
    const R* k0 = a.kv + 3 * (a.state_off + i);
    q0 = k0[0] + a.ka[0];
    q1 = k0[1] + a.ka[1];
    q2 = k0[2] + a.ka[2];
  }
  const R* disp = reinterpret_cast<const R*>(pt.disp);
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const int h = 1 - pass;  // spinor component finished in this pass
    const size_t offh = h ? off1 : off0;
    if (pass == 1) {
      // the down component's forward transform has read LDS for the last time: reuse it for up
      __syncthreads();
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        const int e = tid + j * NT;
        if (e < NP) pl[(e / NZ) * PZ + (e % NZ)] = j < KR ? ku[j < KR ? j : 0] : kus[(j - KR) * NT + tid];
      }
      __syncthreads();
    }
    const size_t rowbase = size_t(2 * i + h) * pt.Jtot;
    if (Y) {
      for (int r = r0; r < r1; ++r) {
        const int jb = pt.pr_begin[r], je = pt.pr_end[r];
        for (int J = jb + tid; J < je; J += NT) {
          const int e = pt.pidx[J];
          cpx<R> y = Y[rowbase + J];
          if (kq) y = cmulc(y, bloch_phase(q0, q1, q2, disp + 3 * J));
          cpx<R>& d = pl[(e / NZ) * PZ + (e % NZ)];
          d.x += a.cre * y.x - a.cim * y.y;
          d.y += a.cre * y.y + a.cim * y.x;
        }
        __syncthreads();
      }
    }
    if (Wr) {
      for (int r = r0; r < r1; ++r) {
        const int jb = pt.pr_begin[r], je = pt.pr_end[r];
        for (int J = jb + tid; J < je; J += NT) {
          const int e = pt.pidx[J];
          cpx<R> o = pl[(e / NZ) * PZ + (e % NZ)];
          if (kq) o = cmul(o, bloch_phase(q0, q1, q2, disp + 3 * J));
          Wr[rowbase + J] = o;
        }
      }
    }
    if (ACC && acc) {
      cpx<R> v[PPT];
#pragma unroll
      for (int j = 0; j < PPT; ++j) v[j] = acc[offh + min(tid + j * NT, NP - 1)];
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        const int e = tid + j * NT;
        if (e < NP) acc[offh + e] = v[j] + pl[(e / NZ) * PZ + (e % NZ)];
      }
    }
    if (wout) {
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        const int e = tid + j * NT;
        if (e < NP) st_stream<M>(&wout[offh + e], pl[(e / NZ) * PZ + (e % NZ)]);
      }
    }
    if (tout) {
      __syncthreads();
      cpx<R>* __restrict__ to = tout + offh;
      plane_fft_fwd_to<R, NY, NZ, PZ, NT>(pl, twy, twz, tid, [](int) { return 0; },
                                          [&](int g, int, cpx<R> v, int) { st_stream<M>(&to[g], v); });
    }
  }
}

// ---------------------------------------------------------------- plane pass: transform only
// SRC: what `in` holds: 0 complex values; 1 a spin density rho_v (real, [4][N]; the transform
// takes n = rho_uu + rho_dd), 2 a real array (the transform takes it as the real part).
template <typename R, int NY, int NZ, int SRC = 0>
__global__ __launch_bounds__(plane_nt(NY* NZ)) void k_plane_fwd(const cpx<R>* in, cpx<R>* out,
                                                                 cpx<R>* W, ProjTables pt,
                                                                 const cpx<R>* __restrict__ twy_g,
                                                                 const cpx<R>* __restrict__ twz_g,
                                                                 int B, int NX, KTables<R> kt) {
  constexpr int NP = NY * NZ;
  constexpr int NT = plane_nt(NP);
  constexpr int PZ = NZ + 1;
  extern __shared__ double4 smem_d4[];
  cpx<R>* plane = reinterpret_cast<cpx<R>*>(smem_d4);
  cpx<R>* twy = plane + NY * PZ;
  cpx<R>* twz = twy + NY;
  const int tid = threadIdx.x;
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  const int x = L / B;
  const int b = L - x * B;
  for (int k = tid; k < NY; k += NT) twy[k] = twy_g[k];
  for (int k = tid; k < NZ; k += NT) twz[k] = twz_g[k];
  const size_t off = (size_t(b) * NX + x) * NP;
  if constexpr (SRC == 0) {
    for (int e = tid; e < NP; e += NT) plane[(e / NZ) * PZ + (e % NZ)] = in[off + e];
  } else {
    const R* rin = reinterpret_cast<const R*>(in);
    const size_t Nall = size_t(NX) * NP;
    for (int e = tid; e < NP; e += NT)
      plane[(e / NZ) * PZ + (e % NZ)] = cpx<R>{SRC == 1 ? rin[off + e] + rin[Nall + off + e] : rin[off + e], R(0)};
  }
  __syncthreads();
  if (W && pt.pr_off) {
    const size_t rowbase = size_t(b) * pt.Jtot;
    const bool kq = kt.kv != nullptr;
    R q0 = 0, q1 = 0, q2 = 0;
    if (kq) {
      const R* k0 = kt.kv + 3 * (kt.state_off + b / 2);
      q0 = k0[0] + kt.ka[0];
      q1 = k0[1] + kt.ka[1];
      q2 = k0[2] + kt.ka[2];
    }
    const R* disp = reinterpret_cast<const R*>(pt.disp);
    for (int r = pt.pr_off[x]; r < pt.pr_off[x + 1]; ++r) {
      for (int J = pt.pr_begin[r] + tid; J < pt.pr_end[r]; J += NT) {
        const int e = pt.pidx[J];
        cpx<R> o = plane[(e / NZ) * PZ + (e % NZ)];
        if (kq) o = cmul(o, bloch_phase(q0, q1, q2, disp + 3 * J));
        W[rowbase + J] = o;
      }
    }
    __syncthreads();
  }
  plane_fft_fwd<R, NY, NZ, PZ>(plane, twy, twz, tid, NT);
  for (int e = tid; e < NP; e += NT) out[off + e] = plane[(e / NZ) * PZ + (e % NZ)];
}

template <typename R, int NY, int NZ>
__global__ __launch_bounds__(plane_nt(NY* NZ)) void k_plane_inv(const cpx<R>* in, cpx<R>* out,
                                                                 R scale,
                                                                 const cpx<R>* __restrict__ twy_g,
                                                                 const cpx<R>* __restrict__ twz_g,
                                                                 int B, int NX) {
  constexpr int NP = NY * NZ;
  constexpr int NT = plane_nt(NP);
  constexpr int PZ = NZ + 1;
  extern __shared__ double4 smem_d4[];
  cpx<R>* plane = reinterpret_cast<cpx<R>*>(smem_d4);
  cpx<R>* twy = plane + NY * PZ;
  cpx<R>* twz = twy + NY;
  const int tid = threadIdx.x;
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  const int x = L / B;
  const int b = L - x * B;
  for (int k = tid; k < NY; k += NT) twy[k] = twy_g[k];
  for (int k = tid; k < NZ; k += NT) twz[k] = twz_g[k];
  const size_t off = (size_t(b) * NX + x) * NP;
  for (int e = tid; e < NP; e += NT) plane[(e / NZ) * PZ + (e % NZ)] = in[off + e];
  __syncthreads();
  plane_fft_inv<R, NY, NZ, PZ>(plane, twy, twz, tid, NT);
  for (int e = tid; e < NP; e += NT) out[off + e] = cscale(plane[(e / NZ) * PZ + (e % NZ)], scale);
}

// ---------------------------------------------------------------- column pass along x
// widest column-pass tile (64, 32, 16 columns) whose LDS footprint stays within a budget
// (tuning macros, bytes per workgroup).  FP32 at 96 points takes 64 columns (48 KB, three
// 512-thread workgroups per CU): 4717 against 4535 GB/s with 32 columns (96^3 x 512).
#ifndef NCT_XPASS_TILE_MAX_F64
#define NCT_XPASS_TILE_MAX_F64 32768
#endif
#ifndef NCT_XPASS_TILE_MAX_F32
#define NCT_XPASS_TILE_MAX_F32 49152
#endif
template <typename R>
constexpr int xpass_tc(int nx) {
  const int b = int(sizeof(R)) * 2;
  const int cap = sizeof(R) == 8 ? NCT_XPASS_TILE_MAX_F64 : NCT_XPASS_TILE_MAX_F32;
  if (nx * 64 * b <= cap) return 64;
  if (nx * 32 * b <= cap) return 32;
  return 16;
}
constexpr int XP_NT = 256;  // threads of the energy column pass
// threads of the column pass per precision (tuning macros); FP32 tiles of 64 columns whose first
// stage has at least 512 butterflies take NCT_XPASS_NT_F32_WIDE: at 64 points 512 threads
// measured 4848 against 4571 GB/s (64^3 x 256), while the 48-point tile (384 butterflies) and
// the 32-column tile at 96 points lost with 512 (4324 against 4402, 4256 against 4543 GB/s), and
// the 64-column tile at 96 points with 256 (4159 against 4717 GB/s).  FP64 at 64 points keeps 32
// columns: a 64-column tile (64 KB, two workgroups per CU) measured 4940 GB/s with 512 threads and
// 4630 with 256, against 4960.
#ifndef NCT_XPASS_NT_F64
#define NCT_XPASS_NT_F64 256
#endif
#ifndef NCT_XPASS_NT_F32
#define NCT_XPASS_NT_F32 256
#endif
#ifndef NCT_XPASS_NT_F32_WIDE
#define NCT_XPASS_NT_F32_WIDE 512
#endif
template <typename R, int NX, int TC>
__host__ __device__ constexpr int xp_nt() {
  if constexpr (sizeof(R) == 4 && TC == 64 && TC * NX / plan_radix(NX, 0) >= 512) return NCT_XPASS_NT_F32_WIDE;
  return sizeof(R) == 8 ? NCT_XPASS_NT_F64 : NCT_XPASS_NT_F32;
}

// Column pass: one workgroup per tile of TC consecutive yz columns x NX planes of one batch
// entry (spinor component).  The first forward x stage works on the values as they are loaded.
template <typename R, int NX, int TC, int M>
__global__ __launch_bounds__((xp_nt<R, NX, TC>())) void k_xpass(const cpx<R>* src, cpx<R>* dst, int NYZ,
                                                 const R* __restrict__ g2x,
                                                 const R* __restrict__ g2yz, R kscale, int mode,
                                                 const cpx<R>* __restrict__ twx_g, KTables<R> kt) {
  __shared__ cpx<R> tile[NX * TC];
  __shared__ cpx<R> tw[NX];
  const int tid = threadIdx.x;
  const int tiles = NYZ / TC;
  const int b = blockIdx.x / tiles;
  const int q0 = (blockIdx.x - b * tiles) * TC;
  for (int k = tid; k < NX; k += xp_nt<R, NX, TC>()) tw[k] = twx_g[k];
  const cpx<R>* srcb = src + size_t(b) * NX * NYZ + q0;
  cpx<R>* dstb = dst + size_t(b) * NX * NYZ + q0;
  {
    // forward DFT along x; its last stage applies the kinetic (mode 0) or Poisson (mode 1)
    // factor as it writes back; the inverse DFT's last stage stores to dst
    constexpr int NS = plan_nstages(NX);
    if constexpr (NS > 1) {
      stage_from<R, NX, 0, TC, 1, TC, 1, TC, xp_nt<R, NX, TC>(), true>(
          tile, tw, tid, [&](int e) { return ld_stream<M>(&srcb[size_t(e / TC) * NYZ + (e % TC)]); });
    } else {
      for (int e = tid; e < NX * TC; e += xp_nt<R, NX, TC>()) tile[e] = ld_stream<M>(&srcb[size_t(e / TC) * NYZ + (e % TC)]);
      __syncthreads();
    }
    if constexpr (NS > 2) {
      lds_stage<R, NX, 1, TC, 1, TC, true>(tile, tw, tid, xp_nt<R, NX, TC>());
      __syncthreads();
    }
    stage_to<R, NX, NS - 1, TC, 1, TC, 1, TC, xp_nt<R, NX, TC>(), true>(
        tile, tw, tid, [](int) { return 0; }, [&](int e, int l, cpx<R> v, int) {
          R g;
          if (kt.kv) {  // |G + k|^2 of this spinor component's state
            const R* k = kt.kv + 3 * (kt.state_off + b / 2);
            const R gx = kt.gx[e / TC] + (k[0] + kt.ka[0]);
            const R gy = kt.gy[q0 + (e % TC)] + (k[1] + kt.ka[1]);
            const R gz = kt.gz[q0 + (e % TC)] + (k[2] + kt.ka[2]);
            g = gx * gx + gy * gy + gz * gz;
          } else {
            g = g2x[e / TC] + g2yz[q0 + (e % TC)];
          }
          R m;
          if (mode == 0) m = kscale * g;
          else m = g > R(0) ? kscale / g : R(0);
          tile[l] = cscale(v, m);
        });
    __syncthreads();
    if constexpr (NS > 2) {
      lds_stage<R, NX, 2, TC, 1, TC, false>(tile, tw, tid, xp_nt<R, NX, TC>());
      __syncthreads();
    }
    if constexpr (NS > 1) {
      lds_stage<R, NX, 1, TC, 1, TC, false>(tile, tw, tid, xp_nt<R, NX, TC>());
      __syncthreads();
    }
    stage_to<R, NX, 0, TC, 1, TC, 1, TC, xp_nt<R, NX, TC>(), false>(
        tile, tw, tid, [](int) { return 0; }, [&](int e, int, cpx<R> v, int) {
          st_stream<M>(&dstb[size_t(e / TC) * NYZ + (e % TC)], v);
        });
  }
}

template <typename R, int NX, int TC>
__global__ __launch_bounds__(XP_NT) void k_xpass_energy(const cpx<R>* src, int NYZ,
                                                        const R* __restrict__ g2x,
                                                        const R* __restrict__ g2yz, R kscale,
                                                        const cpx<R>* __restrict__ twx_g,
                                                        double* part, KTables<R> kt) {
  __shared__ cpx<R> tile[NX * TC];
  __shared__ cpx<R> tw[NX];
  __shared__ double red[XP_NT / 64];
  const int tid = threadIdx.x;
  const int tiles = NYZ / TC;
  const int b = blockIdx.x / tiles;
  const int tl = blockIdx.x - b * tiles;
  const int q0 = tl * TC;
  for (int k = tid; k < NX; k += XP_NT) tw[k] = twx_g[k];
  const size_t base = size_t(b) * NX * NYZ + q0;
  constexpr int PER = (NX * TC + XP_NT - 1) / XP_NT;
  {
    cpx<R> v[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int e = min(tid + j * XP_NT, NX * TC - 1);  // clamped: every load unconditional
      v[j] = src[base + size_t(e / TC) * NYZ + (e % TC)];
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int e = tid + j * XP_NT;
      if (e < NX * TC) tile[e] = v[j];
    }
  }
  __syncthreads();
  lds_fft<R, NX, TC, 1, TC, true>(tile, tw, tid, XP_NT);
  double s1 = 0.0, s2 = 0.0;
  for (int e = tid; e < NX * TC; e += XP_NT) {
    const int xx = e / TC, c = e - (e / TC) * TC;
    double g;
    if (kt.kv) {
      const R* k = kt.kv + 3 * (kt.state_off + b / 2);
      const double gx = double(kt.gx[xx]) + double(k[0] + kt.ka[0]);
      const double gy = double(kt.gy[q0 + c]) + double(k[1] + kt.ka[1]);
      const double gz = double(kt.gz[q0 + c]) + double(k[2] + kt.ka[2]);
      g = gx * gx + gy * gy + gz * gz;
    } else {
      g = double(g2x[xx]) + double(g2yz[q0 + c]);
    }
    const double a2 = double(tile[e].x) * double(tile[e].x) + double(tile[e].y) * double(tile[e].y);
    s1 += double(kscale) * g * a2;
    s2 += a2;
  }
  const double t1 = block_sum<XP_NT>(s1, red);
  const double t2 = block_sum<XP_NT>(s2, red);
  if (tid == 0) {
    part[size_t(blockIdx.x) * 2 + 0] = t1;
    part[size_t(blockIdx.x) * 2 + 1] = t2;
  }
}

// ---------------------------------------------------------------- density (Eq. density4)
template <typename R>
__global__ __launch_bounds__(256) void k_density(const cpx<R>* __restrict__ psi,
                                                 const double* __restrict__ occ, int S, size_t N,
                                                 double* __restrict__ rho) {
  const size_t p = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (p >= N) return;
  double uu = 0, dd = 0, udr = 0, udi = 0;
#pragma unroll 4
  for (int i = 0; i < S; ++i) {
    const double f = occ[i];
    const cpx<R> u = psi[size_t(2 * i) * N + p];
    const cpx<R> d = psi[size_t(2 * i + 1) * N + p];
    const double ux = u.x, uy = u.y, dx = d.x, dy = d.y;
    uu += f * (ux * ux + uy * uy);
    dd += f * (dx * dx + dy * dy);
    udr += f * (ux * dx + uy * dy);   // Re(u d*)
    udi += f * (uy * dx - ux * dy);   // Im(u d*)
  }
  rho[p] = uu;
  rho[N + p] = dd;
  rho[2 * N + p] = udr;
  rho[3 * N + p] = udi;
}

// ---------------------------------------------------------------- exchange + fields (FP64)
// Locally collinear Slater exchange (Eqs. LC+ALDA2, LC+ALDA):
//   n_s = (n +/- |m|)/2, v_s = -(6/pi)^(1/3) n_s^(1/3), vbar = (v_up+v_dn)/2,
//   b_xc = (v_up - v_dn)/2 m/|m| (0 below threshold), e_x = -(3/4)(6/pi)^(1/3) sum n_s^(4/3).
// v_up - v_dn is evaluated as -(6/pi)^(1/3) (n_up - n_dn) / (n_up^(2/3) + (n_up n_dn)^(1/3) + n_dn^(2/3)).
// Dual number v + d e (e^2 = 0) for forward-mode derivatives of the correlation potentials in
// the adjoint; the elementary functions below take double or dual.  cbrt's derivative at 0 is
// taken as 0 (the one-sided value of the clamped channel).
struct dnum {
  double v, d;
};
__device__ __forceinline__ dnum operator+(dnum a, dnum b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ dnum operator-(dnum a, dnum b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ dnum operator*(dnum a, dnum b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ dnum operator/(dnum a, dnum b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
__device__ __forceinline__ dnum operator+(double a, dnum b) { return {a + b.v, b.d}; }
__device__ __forceinline__ dnum operator+(dnum a, double b) { return {a.v + b, a.d}; }
__device__ __forceinline__ dnum operator-(double a, dnum b) { return {a - b.v, -b.d}; }
__device__ __forceinline__ dnum operator-(dnum a, double b) { return {a.v - b, a.d}; }
__device__ __forceinline__ dnum operator*(double a, dnum b) { return {a * b.v, a * b.d}; }
__device__ __forceinline__ dnum operator*(dnum a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ dnum operator/(double a, dnum b) { return {a / b.v, -a * b.d / (b.v * b.v)}; }
__device__ __forceinline__ dnum operator/(dnum a, double b) { return {a.v / b, a.d / b}; }
__device__ __forceinline__ double xval(double x) { return x; }
__device__ __forceinline__ double xval(dnum x) { return x.v; }
__device__ __forceinline__ double xcbrt(double x) { return cbrt(x); }
__device__ __forceinline__ dnum xcbrt(dnum x) {
  const double c = cbrt(x.v);
  return {c, c != 0.0 ? x.d / (3.0 * c * c) : 0.0};
}
__device__ __forceinline__ double xsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ dnum xsqrt(dnum x) {
  const double r = sqrt(x.v);
  return {r, x.d / (2.0 * r)};
}
__device__ __forceinline__ double xlog1p(double x) { return log1p(x); }
__device__ __forceinline__ dnum xlog1p(dnum x) { return {log1p(x.v), x.d / (1.0 + x.v)}; }
__device__ __forceinline__ double xclamp01(double x) { return fmin(fmax(x, 0.0), 1.0); }
__device__ __forceinline__ dnum xclamp01(dnum x) {
  if (x.v < 0.0) return {0.0, 0.0};
  if (x.v > 1.0) return {1.0, 0.0};
  return x;
}

// PW92 LSDA correlation (J. P. Perdew and Y. Wang, Phys. Rev. B 45, 13244 (1992)).
// G(rs) = -2A(1 + a1 rs) ln[1 + 1/(2A(b1 rs^1/2 + b2 rs + b3 rs^3/2 + b4 rs^2))] and dG/drs.
template <typename T>
__device__ __forceinline__ void pw92_g(T rs, T srs, double A, double a1, double b1, double b2, double b3,
                                       double b4, T& g, T& dg) {
  const T q0 = -2.0 * A * (1.0 + a1 * rs);
  const T q1 = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs);
  const T q1p = A * (b1 / srs + 2.0 * b2 + 3.0 * b3 * srs + 4.0 * b4 * rs);
  const T lg = xlog1p(1.0 / q1);
  g = q0 * lg;
  dg = -2.0 * A * a1 * lg - q0 * q1p / (q1 * q1 + q1);
}
// Locally collinear PW92 at density n and |m| = mu: vbar = (v_up + v_dn)/2, bmag = (v_up - v_dn)/2
// (the field along m/|m|), ec = n eps_c; zero where n <= 1e-30.  T = dnum carries the derivative
// along the direction given in n.d, mu.d; T = double is the plain evaluation.
template <typename T>
__device__ void pw92_lc(T n, T mu, T& vbar, T& bmag, T& ec) {
  vbar = bmag = ec = T{};
  if (!(xval(n) > 1e-30)) return;
  const T rs = xcbrt(0.75 / (3.14159265358979323846 * n));
  const T srs = xsqrt(rs);
  const T z = xclamp01(mu / n);
  T e0, d0, e1, d1, ma, dma;
  pw92_g(rs, srs, 0.031091, 0.21370, 7.5957, 3.5876, 1.6382, 0.49294, e0, d0);    // zeta = 0
  pw92_g(rs, srs, 0.015545, 0.20548, 14.1189, 6.1977, 3.3662, 0.62517, e1, d1);   // zeta = 1
  pw92_g(rs, srs, 0.016887, 0.11125, 10.357, 3.6231, 0.88026, 0.49671, ma, dma);  // -alpha_c
  const T ac = 0.0 - ma, dac = 0.0 - dma;
  const double fpp0 = 1.709921;
  const double fden = 0.5198420997897464;  // 2^(4/3) - 2
  const T cu = xcbrt(1.0 + z), cd = xcbrt(1.0 - z);
  const T f = ((1.0 + z) * cu + (1.0 - z) * cd - 2.0) / fden;
  const T fp = (4.0 / 3.0) * (cu - cd) / fden;
  const T z3 = z * z * z, z4 = z3 * z;
  const T eps = e0 + ac * f * (1.0 - z4) / fpp0 + (e1 - e0) * f * z4;
  const T drs = d0 * (1.0 - f * z4) + d1 * f * z4 + dac * f * (1.0 - z4) / fpp0;
  const T dz = 4.0 * z3 * f * (e1 - e0 - ac / fpp0) + fp * (z4 * (e1 - e0) + (1.0 - z4) * ac / fpp0);
  vbar = eps - rs / 3.0 * drs - z * dz;
  bmag = dz;
  ec = n * eps;
}
__global__ __launch_bounds__(256) void k_fields(const double* __restrict__ rho,
                                                const double* __restrict__ vext,
                                                const double* __restrict__ vH, int xc, double thr,
                                                int ny, int nz, double hx, double hy, double hz,
                                                double cx, double cy, double cz, size_t N,
                                                double* __restrict__ fields,
                                                float* __restrict__ f32, double* __restrict__ part) {
  __shared__ double red[4];
  const size_t p = size_t(blockIdx.x) * 256 + threadIdx.x;
  double n = 0, mx = 0, my = 0, mz = 0, eloc = 0, eh = 0, ex = 0, dx = 0, dy = 0, dz = 0;
  if (p < N) {
    const double ruu = rho[p], rdd = rho[N + p], rr = rho[2 * N + p], ri = rho[3 * N + p];
    n = ruu + rdd;
    mx = 2.0 * rr;
    my = -2.0 * ri;
    mz = ruu - rdd;
    const double ve = vext ? vext[p] : 0.0;
    const double vh = vH ? vH[2 * p] : 0.0;  // real part of the complex Poisson output
    double vbar = 0.0, bx = 0.0, by = 0.0, bz = 0.0;
    if (xc) {
      const double c = 1.2407009817988000;  // (6/pi)^(1/3)
      const double mu = sqrt(mx * mx + my * my + mz * mz);
      const double nu = fmax(0.5 * (n + mu), 0.0);
      const double nd = fmax(0.5 * (n - mu), 0.0);
      const double cu = cbrt(nu), cd = cbrt(nd);
      vbar = -0.5 * c * (cu + cd);
      ex = -0.75 * c * (nu * cu + nd * cd);
      double bmag = 0.0;
      if (mu >= thr) {
        const double den = cu * cu + cu * cd + cd * cd;
        bmag = den > 0.0 ? -0.5 * c * (nu - nd) / den : 0.0;
      }
      if (xc >= 2) {
        double vc, bc, ec;
        pw92_lc<double>(n, mu, vc, bc, ec);
        vbar += vc;
        ex += ec;
        if (mu >= thr) bmag += bc;
      }
      if (mu >= thr) {
        const double s = bmag / mu;
        bx = s * mx;
        by = s * my;
        bz = s * mz;
      }
    }
    const double v = ve + vh + vbar;
    fields[p] = v;
    fields[N + p] = bx;
    fields[2 * N + p] = by;
    fields[3 * N + p] = bz;
    if (f32) {
      f32[p] = float(v);
      f32[N + p] = float(bx);
      f32[2 * N + p] = float(by);
      f32[3 * N + p] = float(bz);
    }
    eloc = ve * n;
    eh = 0.5 * vh * n;
    const size_t nyz = size_t(ny) * nz;
    const int ix = int(p / nyz);
    const int rem = int(p - size_t(ix) * nyz);
    const int iy = rem / nz;
    const int iz = rem - iy * nz;
    dx = (ix * hx - cx) * n;
    dy = (iy * hy - cy) * n;
    dz = (iz * hz - cz) * n;
  }
  const double vals[kFieldTot] = {n, mx, my, mz, eloc, eh, ex, 0.0, dx, dy, dz, 0.0};
#pragma unroll
  for (int k = 0; k < kFieldTot; ++k) {
    const double t = (k == 7 || k == 11) ? 0.0 : block_sum<256>(vals[k], red);
    if (threadIdx.x == 0) part[size_t(blockIdx.x) * kFieldTot + k] = t;
  }
}

// out[w] = sum_r part[r*width + w], fixed order; copy0, if given, receives out[0] as well
__global__ __launch_bounds__(256) void k_reduce_rows(const double* __restrict__ part, int nrows,
                                                     int width, double* __restrict__ out,
                                                     double* __restrict__ copy0) {
  __shared__ double red[4];
  for (int w = 0; w < width; ++w) {
    double s = 0.0;
    for (int r = threadIdx.x; r < nrows; r += 256) s += part[size_t(r) * width + w];
    const double t = block_sum<256>(s, red);
    if (threadIdx.x == 0) {
      out[w] = t;
      if (w == 0 && copy0) *copy0 = t;
    }
  }
}

__global__ void k_add_bext(const double* __restrict__ f, int ny, int nz, size_t N, double b0,
                           double b1, double b2, double l0, double l1, double l2, double l3,
                           double* __restrict__ out) {
  const size_t p = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (p < N) {
    const size_t nyz = size_t(ny) * nz;
    const int ix = int(p / nyz);
    const int rem = int(p - size_t(ix) * nyz);
    const int iy = rem / nz;
    const int iz = rem - iy * nz;
    out[p] = f[p] + (l0 * ix + l1 * iy + l2 * iz + l3);
    out[N + p] = f[N + p] + b0;
    out[2 * N + p] = f[2 * N + p] + b1;
    out[3 * N + p] = f[3 * N + p] + b2;
  }
}
__global__ void k_to_float(const double* __restrict__ in, size_t n, float* __restrict__ out) {
  const size_t p = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (p < n) out[p] = float(in[p]);
}

// ---------------------------------------------------------------- projectors on the matrix cores
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename R>
struct mfma16;
// Output element r of lane l is D[row(r, l/16)][l%16]: the f64 instruction interleaves the
// four row groups across registers, the f32 one keeps four consecutive rows per lane.
template <>
struct mfma16<double> {
  typedef d4v acc;
  static __device__ __forceinline__ int row(int r, int kl) { return 4 * r + kl; }
  static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct mfma16<float> {
  typedef f4v acc;
  static __device__ __forceinline__ int row(int r, int kl) { return 4 * kl + r; }
  static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

constexpr int KC = 64;  // contraction K chunk per wave
constexpr int KU = 4;   // k-steps whose operands are loaded together

// Cpart[a][kc][p][i] = sum_{k in chunk} conj(beta[a][k][p]) W[i][k], k = 2 (J - off_a) + s.
// One wave: PP/16 output tiles of 16 projectors x 16 states; A/B operands as
// A[row = lane%16][k = lane/16], B[k = lane/16][col = lane%16]; D rows from mfma16::row.
template <typename R, int PP>
__global__ __launch_bounds__(64) void k_proj_contract(ProjTables pt, const cpx<R>* __restrict__ W,
                                                      int S, cpx<double>* __restrict__ Cpart) {
  using M = mfma16<R>;
  constexpr int NMT = PP / 16;
  const int a = blockIdx.x, nt = blockIdx.y, kc = blockIdx.z;
  const int off = pt.row_off[a];
  const int K = 2 * (pt.row_off[a + 1] - off);
  const int nch_a = (K + KC - 1) / KC;
  if (kc >= nch_a) return;
  const int lane = threadIdx.x;
  const int col = lane & 15, kl = lane >> 4;
  const int i = nt * 16 + col;
  const cpx<R>* __restrict__ beta = reinterpret_cast<const cpx<R>*>(pt.beta);
  typename M::acc ar[NMT], ai[NMT];
#pragma unroll
  for (int mt = 0; mt < NMT; ++mt) {
    ar[mt] = M::zero();
    ai[mt] = M::zero();
  }
  const int kend = min(K, kc * KC + KC);
  for (int k0 = kc * KC; k0 < kend; k0 += 4 * KU) {
    cpx<R> bw[KU], bb[KU][NMT];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int k = k0 + 4 * u + kl;
      const bool ok = k < kend;
      const int kk = ok ? k : kc * KC;  // clamped index, value zeroed below
      const int J = off + (kk >> 1), s = kk & 1;
      const cpx<R> w = W[size_t(2 * min(i, S - 1) + s) * pt.Jtot + J];
      bw[u] = (ok && i < S) ? w : cpx<R>{R(0), R(0)};
#pragma unroll
      for (int mt = 0; mt < NMT; ++mt) {
        const cpx<R> v = beta[(size_t(2 * off) + kk) * PP + mt * 16 + col];
        bb[u][mt] = ok ? v : cpx<R>{R(0), R(0)};
      }
    }
#pragma unroll
    for (int u = 0; u < KU; ++u) {
#pragma unroll
      for (int mt = 0; mt < NMT; ++mt) {
        ar[mt] = M::op(bb[u][mt].x, bw[u].x, ar[mt]);
        ar[mt] = M::op(bb[u][mt].y, bw[u].y, ar[mt]);
        ai[mt] = M::op(bb[u][mt].x, bw[u].y, ai[mt]);
        ai[mt] = M::op(-bb[u][mt].y, bw[u].x, ai[mt]);
      }
    }
  }
  const int nch = pt.max_kchunks;
#pragma unroll
  for (int mt = 0; mt < NMT; ++mt) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = mt * 16 + M::row(r, kl);
      if (i < S)
        Cpart[((size_t(a) * nch + kc) * PP + p) * S + i] = {double(ar[mt][r]), double(ai[mt][r])};
    }
  }
}

// C[a][p][i] = dV sum_kc Cpart (chunk order); EC = E[a][p] C (R precision)
template <typename R>
__global__ __launch_bounds__(256) void k_proj_reduce(ProjTables pt, const cpx<double>* __restrict__ Cpart,
                                                     int S, double dV, cpx<double>* __restrict__ C,
                                                     cpx<R>* __restrict__ EC) {
  const size_t idx = size_t(blockIdx.x) * 256 + threadIdx.x;
  const size_t total = size_t(pt.natoms) * pt.PP * S;
  if (idx >= total) return;
  const int i = int(idx % S);
  const int p = int((idx / S) % pt.PP);
  const int a = int(idx / (size_t(S) * pt.PP));
  const int K = 2 * (pt.row_off[a + 1] - pt.row_off[a]);
  const int nch_a = (K + KC - 1) / KC;
  const size_t stride = size_t(pt.PP) * S;
  const cpx<double>* src = Cpart + (size_t(a) * pt.max_kchunks * pt.PP + p) * S + i;
  double sr = 0, si = 0;
  int kc = 0;
  for (; kc + 8 <= nch_a; kc += 8) {
    cpx<double> v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[size_t(kc + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sr += v[u].x;
      si += v[u].y;
    }
  }
  for (; kc < nch_a; ++kc) {
    const cpx<double> v = src[size_t(kc) * stride];
    sr += v.x;
    si += v.y;
  }
  sr *= dV;
  si *= dV;
  C[idx] = {sr, si};
  const double e = pt.energy[size_t(a) * pt.PP + p];
  EC[idx] = {R(e * sr), R(e * si)};
}

// Y[i][s][J] = sum_p beta[J][s][p] EC[a][p][i]; rows k = 2 (J - off_a) + s
template <typename R, int PP>
__global__ __launch_bounds__(64) void k_proj_scatter(ProjTables pt, const cpx<R>* __restrict__ EC,
                                                     int S, cpx<R>* __restrict__ Y) {
  using M = mfma16<R>;
  constexpr int KS = PP / 4;
  const int a = blockIdx.x, rt = blockIdx.y, nt = blockIdx.z;
  const int off = pt.row_off[a];
  const int K2 = 2 * (pt.row_off[a + 1] - off);
  if (rt * 16 >= K2) return;
  const int lane = threadIdx.x;
  const int col = lane & 15, kl = lane >> 4;
  const int row = rt * 16 + col;
  const int i = nt * 16 + col;
  const cpx<R>* __restrict__ beta = reinterpret_cast<const cpx<R>*>(pt.beta);
  cpx<R> xb[KS], ec[KS];
#pragma unroll
  for (int u = 0; u < KS; ++u) {
    const int p = 4 * u + kl;
    const cpx<R> bv = beta[(size_t(2 * off) + min(row, K2 - 1)) * PP + p];
    xb[u] = row < K2 ? bv : cpx<R>{R(0), R(0)};
    const cpx<R> ev = EC[(size_t(a) * PP + p) * S + min(i, S - 1)];
    ec[u] = i < S ? ev : cpx<R>{R(0), R(0)};
  }
  typename M::acc yr = M::zero(), yi = M::zero();
#pragma unroll
  for (int u = 0; u < KS; ++u) {
    yr = M::op(xb[u].x, ec[u].x, yr);
    yr = M::op(-xb[u].y, ec[u].y, yr);
    yi = M::op(xb[u].x, ec[u].y, yi);
    yi = M::op(xb[u].y, ec[u].x, yi);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int rr = rt * 16 + M::row(r, kl);
    if (rr < K2 && i < S) {
      const int J = off + (rr >> 1), s = rr & 1;
      Y[size_t(2 * i + s) * pt.Jtot + J] = {yr[r], yi[r]};
    }
  }
}

// ---------------------------------------------------------------- adjoint kernels
// Pair reduction of one adjoint Taylor stage:
//   g[0][p] += gamma sum_i Im(mu_i^dagger w_i),  g[1+q][p] += gamma sum_i Im(mu_i^dagger sigma_q w_i)
// i.e. dL = sum_r (g_v dv + g_b . db) for a perturbation dH = dv + db.sigma of the stage
// w_k = x + (-i gamma) H w_{k-1} with adjoint mu_k.
template <typename R>
__global__ __launch_bounds__(256) void k_pair(const cpx<R>* __restrict__ mu, const cpx<R>* __restrict__ w,
                                              int S, size_t N, double gamma, double* __restrict__ g) {
  const size_t p = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (p >= N) return;
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll 2
  for (int i = 0; i < S; ++i) {
    const cpx<R> mu_u = mu[size_t(2 * i) * N + p], mu_d = mu[size_t(2 * i + 1) * N + p];
    const cpx<R> w_u = w[size_t(2 * i) * N + p], w_d = w[size_t(2 * i + 1) * N + p];
    const double ar = mu_u.x, ai = mu_u.y, br = mu_d.x, bi = mu_d.y;
    const double ur = w_u.x, ui = w_u.y, dr = w_d.x, di = w_d.y;
    // Im(conj(a) u) = ar ui - ai ur
    const double im_au = ar * ui - ai * ur, im_bd = br * di - bi * dr;
    const double im_ad = ar * di - ai * dr, im_bu = br * ui - bi * ur;
    const double re_ad = ar * dr + ai * di, re_bu = br * ur + bi * ui;
    s0 += im_au + im_bd;                 // 1
    s1 += im_ad + im_bu;                 // sigma_x: conj(a) d + conj(b) u
    s2 += -re_ad + re_bu;                // sigma_y: -i conj(a) d + i conj(b) u  -> Im = -Re(a*d) + Re(b*u)
    s3 += im_au - im_bd;                 // sigma_z
  }
  g[p] += gamma * s0;
  g[N + p] += gamma * s1;
  g[2 * N + p] += gamma * s2;
  g[3 * N + p] += gamma * s3;
}

// Transpose of the field map (v, b) <- (n, m) at the density rho, for gradients g = (g_v, g_b):
//   g_n = P g_v + dvbar/dn g_v + dbeta/dn (mhat.g_b)
//   g_m = [dvbar/dmu g_v + dbeta/dmu (mhat.g_b)] mhat + (beta/mu)(g_b - mhat (mhat.g_b))
// with beta = (v_up - v_dn)/2, v_s' = -(1/3)(6/pi)^(1/3) n_s^(-2/3) (0 on a clamped channel),
// b_xc = 0 (and its derivatives) below the |m| threshold.  pg = P g_v (Poisson) or null.
// part[blk][0..2] = block sums of g_b (for dL/dB_ext).
__global__ __launch_bounds__(256) void k_field_adjoint(const double* __restrict__ rho,
                                                       const double* __restrict__ g,
                                                       const double* __restrict__ pg, int xc,
                                                       double thr, size_t N, double* __restrict__ gnm,
                                                       double* __restrict__ part) {
  __shared__ double red[4];
  const size_t p = size_t(blockIdx.x) * 256 + threadIdx.x;
  double gbx = 0, gby = 0, gbz = 0;
  if (p < N) {
    const double gv = g[p];
    gbx = g[N + p];
    gby = g[2 * N + p];
    gbz = g[3 * N + p];
    double gn = pg ? pg[2 * p] : 0.0;  // real part of the complex Poisson output
    double gmx = 0, gmy = 0, gmz = 0;
    if (xc) {
      // v = vbar(n, |m|), b = bmag(n, |m|) m/|m| (|m| >= thr); with J the Jacobian of
      // (vbar, bmag) in (n, |m|) and g_r = mhat.g_b:
      //   g_n += J00 g_v + J10 g_r,  g_m = (J01 g_v + J11 g_r) mhat + (bmag/|m|)(g_b - mhat g_r)
      const double c = 1.2407009817988000;  // (6/pi)^(1/3)
      const double ruu = rho[p], rdd = rho[N + p], rr = rho[2 * N + p], ri = rho[3 * N + p];
      const double n = ruu + rdd, mx = 2.0 * rr, my = -2.0 * ri, mz = ruu - rdd;
      const double mu = sqrt(mx * mx + my * my + mz * mz);
      const double nu = 0.5 * (n + mu), nd = 0.5 * (n - mu);
      const double cu = nu > 0 ? cbrt(nu) : 0.0, cd = nd > 0 ? cbrt(nd) : 0.0;
      // exchange: v_s depends on n_s alone, dv_s/dn_s = du, dd
      const double du = nu > 0 ? -(c / 3.0) / (cu * cu) : 0.0;
      const double dd = nd > 0 ? -(c / 3.0) / (cd * cd) : 0.0;
      double j00 = 0.25 * (du + dd), j01 = 0.25 * (du - dd), j10 = j01, j11 = j00;
      double bmag = 0.0;
      if (mu >= thr) {
        const double nuc = fmax(nu, 0.0), ndc = fmax(nd, 0.0);
        const double den = cu * cu + cu * cd + cd * cd;
        bmag = den > 0.0 ? -0.5 * c * (nuc - ndc) / den : 0.0;
      }
      if (xc >= 2) {  // PW92 correlation: its Jacobian from two dual evaluations
        dnum vb, bm, ec;
        pw92_lc<dnum>(dnum{n, 1.0}, dnum{mu, 0.0}, vb, bm, ec);
        j00 += vb.d;
        j10 += bm.d;
        pw92_lc<dnum>(dnum{n, 0.0}, dnum{mu, 1.0}, vb, bm, ec);
        j01 += vb.d;
        j11 += bm.d;
        if (mu >= thr) bmag += bm.v;
      }
      gn += j00 * gv;
      if (mu >= thr) {
        const double hx = mx / mu, hy = my / mu, hz = mz / mu;
        const double mg = hx * gbx + hy * gby + hz * gbz;
        const double bom = bmag / mu;
        gn += j10 * mg;
        const double radial = j01 * gv + j11 * mg;
        gmx = radial * hx + bom * (gbx - hx * mg);
        gmy = radial * hy + bom * (gby - hy * mg);
        gmz = radial * hz + bom * (gbz - hz * mg);
      }
    }
    gnm[p] = gn;
    gnm[N + p] = gmx;
    gnm[2 * N + p] = gmy;
    gnm[3 * N + p] = gmz;
  }
  const double v3[3] = {gbx, gby, gbz};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double t = block_sum<256>(v3[k], red);
    if (threadIdx.x == 0) part[size_t(blockIdx.x) * 4 + k] = t;
  }
  if (threadIdx.x == 0) part[size_t(blockIdx.x) * 4 + 3] = 0.0;
}

// lam_i (+)= 2 f_i [g_n + g_m . sigma] psi_i   (adjoint of n = sum f psi^dag psi, m = sum f psi^dag sigma psi)
template <typename R>
__global__ __launch_bounds__(256) void k_density_backprop(const cpx<R>* __restrict__ psi,
                                                          const double* __restrict__ occ,
                                                          const double* __restrict__ gnm, int S,
                                                          size_t N, int add, cpx<R>* __restrict__ lam) {
  const size_t idx = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= size_t(S) * N) return;
  const int i = int(idx / N);
  const size_t p = idx - size_t(i) * N;
  const double f = 2.0 * occ[i];
  const double gn = gnm[p], gx = gnm[N + p], gy = gnm[2 * N + p], gz = gnm[3 * N + p];
  const cpx<R> u = psi[size_t(2 * i) * N + p], d = psi[size_t(2 * i + 1) * N + p];
  const double ux = u.x, uy = u.y, dx = d.x, dy = d.y;
  // up' = (gn + gz) u + (gx - i gy) d ; dn' = (gx + i gy) u + (gn - gz) d
  double ox = (gn + gz) * ux + gx * dx + gy * dy;
  double oy = (gn + gz) * uy + gx * dy - gy * dx;
  double px = gx * ux - gy * uy + (gn - gz) * dx;
  double py = gx * uy + gy * ux + (gn - gz) * dy;
  cpx<R>& lu = lam[size_t(2 * i) * N + p];
  cpx<R>& ld = lam[size_t(2 * i + 1) * N + p];
  if (add) {
    ox = f * ox + double(lu.x);
    oy = f * oy + double(lu.y);
    px = f * px + double(ld.x);
    py = f * py + double(ld.y);
  } else {
    ox *= f;
    oy *= f;
    px *= f;
    py *= f;
  }
  lu = {R(ox), R(oy)};
  ld = {R(px), R(py)};
}


// ---------------------------------------------------------------- observables row
__global__ __launch_bounds__(256) void k_obs_row(ObsInputs in, double* __restrict__ row) {
  __shared__ double red[4];
  __shared__ double maxerr[256];
  const int tid = threadIdx.x;
  double ekin = 0.0, mx = 0.0, enl = 0.0;
  for (int i = tid; i < in.S; i += 256) {
    double e = 0.0, nn = 0.0;
    for (int s = 0; s < 2; ++s) {
      for (int t = 0; t < in.ntiles; ++t) {
        const double* q = in.epart + (size_t(2 * i + s) * in.ntiles + t) * 2;
        e += q[0];
        nn += q[1];
      }
    }
    ekin += in.occ[i] * e * in.dV;
    mx = fmax(mx, fabs(nn * in.invN * in.dV - 1.0));
  }
  if (in.C) {
    const size_t total = size_t(in.natoms) * in.PP * in.S;
    const cpx<double>* C = reinterpret_cast<const cpx<double>*>(in.C);
    for (size_t idx = tid; idx < total; idx += 256) {
      const int i = int(idx % in.S);
      const int p = int((idx / in.S) % in.PP);
      const int a = int(idx / (size_t(in.S) * in.PP));
      const cpx<double> c = C[idx];
      enl += in.occ[i] * in.energy[size_t(a) * in.PP + p] * (c.x * c.x + c.y * c.y);
    }
  }
  const double Ekin = block_sum<256>(ekin, red);
  const double Enl = block_sum<256>(enl, red);
  maxerr[tid] = mx;
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int k = 0; k < 256; ++k) m = fmax(m, maxerr[k]);
    const double* ft = in.field_tot;
    const double dV = in.dV;
    const double Ne = ft[0] * dV, Mx = ft[1] * dV, My = ft[2] * dV, Mz = ft[3] * dV;
    const double Eloc = (ft[4] + in.efield[0] * ft[8] + in.efield[1] * ft[9] + in.efield[2] * ft[10]) * dV;
    const double EH = ft[5] * dV, Exc = ft[6] * dV;
    const double EZ = in.muB_B[0] * Mx + in.muB_B[1] * My + in.muB_B[2] * Mz;
    row[0] = in.t;
    row[1] = Ne;
    row[2] = Mx;
    row[3] = My;
    row[4] = Mz;
    row[5] = Ekin + Eloc + Enl + EH + Exc + EZ;
    row[6] = Ekin;
    row[7] = Eloc;
    row[8] = Enl;
    row[9] = EH;
    row[10] = Exc;
    row[11] = EZ;
    row[12] = m;
  }
}

// ---------------------------------------------------------------- small pointwise kernels
// lam_i = scale f_i (w . sigma) psi_i
template <typename R>
__global__ void k_seed(const cpx<R>* __restrict__ psi, const double* __restrict__ occ, int S,
                       size_t N, double w0, double w1, double w2, double scale,
                       cpx<R>* __restrict__ lam) {
  const size_t idx = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= size_t(S) * N) return;
  const int i = int(idx / N);
  const size_t p = idx - size_t(i) * N;
  const double f = scale * occ[i];
  const cpx<R> u = psi[size_t(2 * i) * N + p];
  const cpx<R> d = psi[size_t(2 * i + 1) * N + p];
  // (w.sigma) (u, d) = (w2 u + (w0 - i w1) d, (w0 + i w1) u - w2 d)
  const double ux = u.x, uy = u.y, dx = d.x, dy = d.y;
  const double ox = w2 * ux + w0 * dx + w1 * dy;
  const double oy = w2 * uy + w0 * dy - w1 * dx;
  const double px = w0 * ux - w1 * uy - w2 * dx;
  const double py = w0 * uy + w1 * ux - w2 * dy;
  lam[size_t(2 * i) * N + p] = {R(f * ox), R(f * oy)};
  lam[size_t(2 * i + 1) * N + p] = {R(f * px), R(f * py)};
}

// y = (a_re + i a_im) x + b y
template <typename R>
__global__ void k_axpby(cpx<R>* __restrict__ y, const cpx<R>* __restrict__ x, size_t count,
                        R are, R aim, R b) {
  const size_t idx = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= count) return;
  const cpx<R> xv = x[idx];
  const cpx<R> yv = y[idx];
  y[idx] = {are * xv.x - aim * xv.y + b * yv.x, are * xv.y + aim * xv.x + b * yv.y};
}

// rows[S][2][Jtot] *= exp(i dA.d_J)
template <typename R>
__global__ __launch_bounds__(256) void k_rephase_rows(cpx<R>* __restrict__ rows, const R* __restrict__ disp,
                                                      int Jtot, size_t total, R a0, R a1, R a2) {
  const size_t p = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (p >= total) return;
  const int J = int(p % size_t(Jtot));
  rows[p] = cmul(rows[p], bloch_phase(a0, a1, a2, disp + 3 * J));
}

// ---------------------------------------------------------------- initial spin-density matrix
__global__ __launch_bounds__(256) void k_dm_init(int nx, int ny, int nz, double hx, double hy,
                                                 double hz, double Lx, double Ly, double Lz, int natoms,
                                                 const double* __restrict__ atoms,
                                                 const double* __restrict__ moments,
                                                 double* __restrict__ rho) {
  const size_t N = size_t(nx) * ny * nz;
  const size_t p = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (p >= N) return;
  const size_t nyz = size_t(ny) * nz;
  const int ix = int(p / nyz);
  const int rem = int(p - size_t(ix) * nyz);
  const int iy = rem / nz, iz = rem - (rem / nz) * nz;
  const double r[3] = {ix * hx, iy * hy, iz * hz};
  const double L[3] = {Lx, Ly, Lz};
  double best = 1e300;
  int owner = 0;
  for (int a = 0; a < natoms; ++a) {
    double d2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double d = __dsub_rn(r[k], atoms[6 * a + k]);
      d = __dsub_rn(d, __dmul_rn(L[k], rint(d / L[k])));
      d2 = __dadd_rn(d2, __dmul_rn(d, d));
    }
    if (d2 < best) {
      best = d2;
      owner = a;
    }
  }
  const double Z = atoms[6 * owner + 3], sg = atoms[6 * owner + 4];
  const double n = Z * pow(2.0 * 3.14159265358979323846 * sg * sg, -1.5) * exp(-best / (2.0 * sg * sg));
  const double mx = moments[3 * owner] / Z, my = moments[3 * owner + 1] / Z, mz = moments[3 * owner + 2] / Z;
  rho[p] = n * (1.0 + mz) / 2.0;
  rho[N + p] = n * (1.0 - mz) / 2.0;
  rho[2 * N + p] = n * mx / 2.0;
  rho[3 * N + p] = -n * my / 2.0;
}

// ---------------------------------------------------------------- orthonormalisation (ground state)
// Overlap of a run of states and the triangular change of basis that orthonormalises them.  Both
// are dense complex contractions on the matrix cores with FP64 operands and FP64 accumulation in
// either precision (the overlap is a norm reduction over 2N terms).

// Partial Gram matrices over K-chunks: part[c][i][j] = sum_{k in chunk c} conj(A[i][k]) A[j][k]
// for the tile pairs (ti <= tj) of 32 x 32 state tiles; A is [S][K] (states are rows of K = 2N
// complex values).  Four waves per workgroup, one 16 x 16 output tile each.
constexpr int GRAM_T = 32;   // output tile (states)
constexpr int GRAM_KB = 16;  // k values staged per iteration
template <typename R>
__global__ __launch_bounds__(256) void k_gram_partial(const cpx<R>* __restrict__ A, int S, size_t K,
                                                      size_t kchunk, cpx<double>* __restrict__ part) {
  using M = mfma16<double>;
  __shared__ cpx<double> sa[GRAM_T][GRAM_KB + 1];
  __shared__ cpx<double> sb[GRAM_T][GRAM_KB + 1];
  const int T = (S + GRAM_T - 1) / GRAM_T;
  int pidx = blockIdx.x, ti = 0;
  while (pidx >= T - ti) {
    pidx -= T - ti;
    ++ti;
  }
  const int tj = ti + pidx;
  const size_t k0 = size_t(blockIdx.y) * kchunk;
  const size_t k1 = min(K, k0 + kchunk);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int wi = w >> 1, wj = w & 1;
  const int c = lane & 15, kl = lane >> 4;
  M::acc cr = M::zero(), ci = M::zero();
  for (size_t kb = k0; kb < k1; kb += GRAM_KB) {
#pragma unroll
    for (int e = tid; e < GRAM_T * GRAM_KB; e += 256) {
      const int r = e / GRAM_KB, kk = e % GRAM_KB;
      const size_t k = kb + kk;
      const int ri = ti * GRAM_T + r, rj = tj * GRAM_T + r;
      cpx<double> va = {0.0, 0.0}, vb = {0.0, 0.0};
      if (k < k1 && ri < S) {
        const cpx<R> v = A[size_t(ri) * K + k];
        va = {double(v.x), double(v.y)};
      }
      if (k < k1 && rj < S) {
        const cpx<R> v = A[size_t(rj) * K + k];
        vb = {double(v.x), double(v.y)};
      }
      sa[r][kk] = va;
      sb[r][kk] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GRAM_KB; ks += 4) {
      const cpx<double> a = sa[wi * 16 + c][ks + kl];  // A operand: row i, column k
      const cpx<double> b = sb[wj * 16 + c][ks + kl];  // B operand: row k, column j
      cr = M::op(a.x, b.x, cr);
      cr = M::op(a.y, b.y, cr);
      ci = M::op(a.x, b.y, ci);
      ci = M::op(-a.y, b.x, ci);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = ti * GRAM_T + wi * 16 + M::row(r, kl);
    const int j = tj * GRAM_T + wj * 16 + c;
    if (i < S && j < S) part[(size_t(blockIdx.y) * S + i) * S + j] = {cr[r], ci[r]};
  }
}

// out[i][j] = scale sum_c part[c][i][j] (chunk order) for j >= i, and its conjugate at [j][i].
__global__ __launch_bounds__(256) void k_gram_reduce(const cpx<double>* __restrict__ part, int S, int nchunks,
                                                     double scale, cpx<double>* __restrict__ out) {
  const size_t idx = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= size_t(S) * S) return;
  const int i = int(idx / S), j = int(idx - size_t(i) * S);
  if (j < i) return;
  double sr = 0.0, si = 0.0;
  for (int cch = 0; cch < nchunks; ++cch) {
    const cpx<double> v = part[(size_t(cch) * S + i) * S + j];
    sr += v.x;
    si += v.y;
  }
  out[size_t(i) * S + j] = {scale * sr, scale * si};
  if (j != i) out[size_t(j) * S + i] = {scale * sr, -scale * si};
}

// D[j][p] = sum_{i <= j} Mt[i][j] A[i][p] (Mt upper triangular, FP64): the states D_j = sum_i
// A_i M_ij.  One workgroup: 64 states j x 64 columns p; wave w owns states w*16 .. w*16+15 and
// four 16-column MFMA tiles.  Only i below the tile's last j contribute.
constexpr int BT_J = 64;
constexpr int BT_P = 64;
constexpr int BT_KI = 16;
template <typename R>
__global__ __launch_bounds__(256) void k_basis_transform(const cpx<R>* __restrict__ A,
                                                         const cpx<double>* __restrict__ Mt, int S,
                                                         size_t K, cpx<R>* __restrict__ D) {
  using M = mfma16<double>;
  __shared__ cpx<double> sm[BT_J][BT_KI + 1];   // [j][i]
  __shared__ cpx<double> sx[BT_KI][BT_P + 1];   // [i][p]
  const int j0 = blockIdx.y * BT_J;
  const size_t p0 = size_t(blockIdx.x) * BT_P;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int c = lane & 15, kl = lane >> 4;
  M::acc dr[4], di[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    dr[h] = M::zero();
    di[h] = M::zero();
  }
  const int iend = min(S, j0 + BT_J);
  for (int i0 = 0; i0 < iend; i0 += BT_KI) {
#pragma unroll
    for (int e = tid; e < BT_KI * BT_J; e += 256) {
      const int il = e / BT_J, jl = e % BT_J;
      const int i = i0 + il, j = j0 + jl;
      sm[jl][il] = (i < S && j < S) ? Mt[size_t(i) * S + j] : cpx<double>{0.0, 0.0};
    }
#pragma unroll
    for (int e = tid; e < BT_KI * BT_P; e += 256) {
      const int il = e / BT_P, pl = e % BT_P;
      const int i = i0 + il;
      const size_t pp = p0 + pl;
      cpx<double> v = {0.0, 0.0};
      if (i < S && pp < K) {
        const cpx<R> a = A[size_t(i) * K + pp];
        v = {double(a.x), double(a.y)};
      }
      sx[il][pl] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BT_KI; ks += 4) {
      const cpx<double> a = sm[w * 16 + c][ks + kl];  // A operand: row j, column i
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const cpx<double> b = sx[ks + kl][h * 16 + c];  // B operand: row i, column p
        dr[h] = M::op(a.x, b.x, dr[h]);
        dr[h] = M::op(-a.y, b.y, dr[h]);
        di[h] = M::op(a.x, b.y, di[h]);
        di[h] = M::op(a.y, b.x, di[h]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int h = 0; h < 4; ++h) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = j0 + w * 16 + M::row(r, kl);
      const size_t pp = p0 + h * 16 + c;
      if (j < S && pp < K) D[size_t(j) * K + pp] = {R(dr[h][r]), R(di[h][r])};
    }
  }
}

// ---------------------------------------------------------------- static scratch
// Temporaries of the allocation-free entry point.  Host code never passes this name to a kernel:
// it takes the per-device address from static_scratch().
static __device__ __align__(256) unsigned char scratch[NCT_STATIC_SCRATCH_BYTES];

hipError_t static_scratch(void** ptr, size_t* bytes) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {  // once per device, with that device current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = NCT_STATIC_SCRATCH_BYTES;
  return hipSuccess;
}

// ================================================================ launchers
static inline unsigned nblocks(size_t n, unsigned bs) { return unsigned((n + bs - 1) / bs); }

LaunchEvents& launch_events() {
  static thread_local LaunchEvents ev;
  return ev;
}

// Every dispatch goes through here: with timing events pending they ride on the dispatch itself.
template <typename F, typename... Args>
static void nct_launch(F kern, dim3 grid, dim3 block, size_t lds, hipStream_t st, Args... args) {
  LaunchEvents& ev = launch_events();
  if (ev.stop) {
    hipExtLaunchKernelGGL(kern, grid, block, std::uint32_t(lds), st, ev.used ? nullptr : ev.start,
                          ev.stop, 0u, args...);
    ev.used = true;
  } else {
    hipLaunchKernelGGL(kern, grid, block, lds, st, args...);
  }
}

#define NCT_PLANE_PAIRS(X) \
  X(8, 8) X(12, 12) X(16, 16) X(24, 24) X(32, 32) X(48, 48) X(64, 64) X(96, 96) \
  X(8, 16) X(16, 8) X(12, 16) X(16, 12) X(16, 24) X(24, 16)
#define NCT_LINES(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96)

bool plane_pair_supported(int ny, int nz) {
#define X(a, b) if (ny == a && nz == b) return true;
  NCT_PLANE_PAIRS(X)
#undef X
  return false;
}
bool line_supported(int n) {
#define X(a) if (n == a) return true;
  NCT_LINES(X)
#undef X
  return false;
}

template <typename K>
static hipError_t set_lds(K kern, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

template <typename R, int A, int B, int M>
static hipError_t launch_plane_stage_m(int S, int NX, const StageArgs<R>& a, const ProjTables& pt,
                                       const void* twy, const void* twz, hipStream_t st) {
  const unsigned grid = unsigned(S) * unsigned(NX);
  const auto ty = reinterpret_cast<const cpx<R>*>(twy);
  const auto tz = reinterpret_cast<const cpx<R>*>(twz);
  if constexpr (planer_use<R, A, B>()) {
    constexpr size_t ldsr = planer_lds_bytes<R, A, B>();
    // FP64 stages without accumulation take an instantiation without that path: four fewer
    // live values leave the FP64 64^2 kernel without register spill.  FP32 keeps one
    // instantiation: without the path the compiler allocates the FP32 96^2 kernel worse (36 B of
    // spill per lane instead of 28).
    auto kernr = k_plane_stage_r<R, A, B, M, true>;
    if constexpr (sizeof(R) == 8) {
      if (!a.acc) kernr = k_plane_stage_r<R, A, B, M, false>;
    }
    hipError_t er = set_lds(kernr, ldsr);
    if (er != hipSuccess) return er;
    nct_launch(kernr, dim3(grid), dim3(NCT_PLANER_NT), ldsr, st, a, pt, ty, tz, S, NX);
  } else if constexpr (plane2_fits<R, A, B>()) {
    constexpr size_t lds2 = plane2_lds_bytes<A, B>(sizeof(cpx<R>));
    auto kern2 = k_plane_stage2<R, A, B, M>;
    hipError_t e2 = set_lds(kern2, lds2);
    if (e2 != hipSuccess) return e2;
    nct_launch(kern2, dim3(grid), dim3(2 * plane2_nth<R>(A * B)), lds2, st, a, pt, ty, tz, S, NX);
  } else {
    constexpr size_t lds = plane_lds_bytes<A, B>(sizeof(cpx<R>));
    auto kern = k_plane_stage<R, A, B, M>;
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess) return e;
    nct_launch(kern, dim3(grid), dim3(plane_nt(A * B)), lds, st, a, pt, ty, tz, S, NX);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_plane_stage(const int n[3], int S, const StageArgs<R>& a, const ProjTables& pt,
                              const void* twy, const void* twz, hipStream_t st) {
#define X(A, B)                                                                              \
  if (n[1] == A && n[2] == B) {                                                              \
    if (a.cache_mode >= 2) return launch_plane_stage_m<R, A, B, 2>(S, n[0], a, pt, twy, twz, st); \
    if (a.cache_mode == 1) return launch_plane_stage_m<R, A, B, 1>(S, n[0], a, pt, twy, twz, st); \
    return launch_plane_stage_m<R, A, B, 0>(S, n[0], a, pt, twy, twz, st);                  \
  }
  NCT_PLANE_PAIRS(X)
#undef X
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_plane_fwd(const int n[3], int B, const void* in, void* out, void* W,
                            const ProjTables* pt, const void* twy, const void* twz, hipStream_t st,
                            KTables<R> kt) {
  const unsigned grid = unsigned(B) * unsigned(n[0]);
  ProjTables none;
  const ProjTables& p = pt ? *pt : none;
#define X(A, BB)                                                                            \
  if (n[1] == A && n[2] == BB) {                                                            \
    constexpr size_t lds = plane_lds_bytes<A, BB>(sizeof(cpx<R>));                          \
    auto kern = k_plane_fwd<R, A, BB>;                                                      \
    hipError_t e = set_lds(kern, lds);                                                      \
    if (e != hipSuccess) return e;                                                          \
    nct_launch(kern, dim3(grid), dim3(plane_nt(A * BB)), lds, st,                   \
                       reinterpret_cast<const cpx<R>*>(in), reinterpret_cast<cpx<R>*>(out),  \
                       reinterpret_cast<cpx<R>*>(W), p,                                     \
                       reinterpret_cast<const cpx<R>*>(twy), reinterpret_cast<const cpx<R>*>(twz), \
                       B, n[0], kt);                                                        \
    return hipGetLastError();                                                               \
  }
  NCT_PLANE_PAIRS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_plane_fwd_real(const int n[3], const double* in, int src, void* out, const void* twy,
                                 const void* twz, hipStream_t st) {
  const unsigned grid = unsigned(n[0]);
#define X(A, BB)                                                                            \
  if (n[1] == A && n[2] == BB) {                                                            \
    constexpr size_t lds = plane_lds_bytes<A, BB>(sizeof(cpx<double>));                     \
    auto kern = src == 1 ? k_plane_fwd<double, A, BB, 1> : k_plane_fwd<double, A, BB, 2>;  \
    hipError_t e = set_lds(kern, lds);                                                      \
    if (e != hipSuccess) return e;                                                          \
    nct_launch(kern, dim3(grid), dim3(plane_nt(A * BB)), lds, st,                            \
               reinterpret_cast<const cpx<double>*>(in), reinterpret_cast<cpx<double>*>(out), \
               static_cast<cpx<double>*>(nullptr), ProjTables{},                             \
               reinterpret_cast<const cpx<double>*>(twy), reinterpret_cast<const cpx<double>*>(twz), \
               1, n[0], KTables<double>{});                                                  \
    return hipGetLastError();                                                               \
  }
  NCT_PLANE_PAIRS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_dm_init(const int n[3], const double cell[3], int natoms, const double* atoms,
                          const double* moments, double* rho, hipStream_t st) {
  const size_t N = size_t(n[0]) * n[1] * n[2];
  nct_launch(k_dm_init, dim3(nblocks(N, 256)), dim3(256), 0, st, n[0], n[1], n[2], cell[0] / n[0],
             cell[1] / n[1], cell[2] / n[2], cell[0], cell[1], cell[2], natoms, atoms, moments, rho);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_rephase_rows(const ProjTables& pt, void* rows, int S, const double dA[3],
                               hipStream_t st) {
  if (pt.natoms == 0 || pt.Jtot == 0) return hipSuccess;
  const size_t total = size_t(S) * 2 * pt.Jtot;
  nct_launch(k_rephase_rows<R>, dim3(nblocks(total, 256)), dim3(256), 0, st,
             reinterpret_cast<cpx<R>*>(rows), reinterpret_cast<const R*>(pt.disp), pt.Jtot, total,
             R(dA[0]), R(dA[1]), R(dA[2]));
  return hipGetLastError();
}

template <typename R>
hipError_t launch_plane_inv(const int n[3], int B, const void* in, void* out, R scale,
                            const void* twy, const void* twz, hipStream_t st) {
  const unsigned grid = unsigned(B) * unsigned(n[0]);
#define X(A, BB)                                                                            \
  if (n[1] == A && n[2] == BB) {                                                            \
    constexpr size_t lds = plane_lds_bytes<A, BB>(sizeof(cpx<R>));                          \
    auto kern = k_plane_inv<R, A, BB>;                                                      \
    hipError_t e = set_lds(kern, lds);                                                      \
    if (e != hipSuccess) return e;                                                          \
    nct_launch(kern, dim3(grid), dim3(plane_nt(A * BB)), lds, st,                   \
                       reinterpret_cast<const cpx<R>*>(in), reinterpret_cast<cpx<R>*>(out),  \
                       scale, reinterpret_cast<const cpx<R>*>(twy),                         \
                       reinterpret_cast<const cpx<R>*>(twz), B, n[0]);                      \
    return hipGetLastError();                                                               \
  }
  NCT_PLANE_PAIRS(X)
#undef X
  return hipErrorInvalidValue;
}

template <typename R, int NX, int TC>
static hipError_t launch_xpass_tc(int B, int NYZ, const void* src, void* dst, const R* g2x, const R* g2yz,
                                  R kscale, int mode, const void* twx, int cache_mode, hipStream_t st,
                                  KTables<R> kt) {
  const int tiles = NYZ / TC;
  const auto s_ = reinterpret_cast<const cpx<R>*>(src);
  const auto d_ = reinterpret_cast<cpx<R>*>(dst);
  const auto t_ = reinterpret_cast<const cpx<R>*>(twx);
  // one tile per workgroup (a second, prefetched tile per workgroup measured no faster on
  // MI355X and costs occupancy)
  const dim3 grid(unsigned(B) * unsigned(tiles));
  if (cache_mode >= 2)
    nct_launch((k_xpass<R, NX, TC, 2>), grid, dim3(xp_nt<R, NX, TC>()), 0, st, s_, d_, NYZ, g2x, g2yz, kscale, mode, t_, kt);
  else if (cache_mode == 1)
    nct_launch((k_xpass<R, NX, TC, 1>), grid, dim3(xp_nt<R, NX, TC>()), 0, st, s_, d_, NYZ, g2x, g2yz, kscale, mode, t_, kt);
  else
    nct_launch((k_xpass<R, NX, TC, 0>), grid, dim3(xp_nt<R, NX, TC>()), 0, st, s_, d_, NYZ, g2x, g2yz, kscale, mode, t_, kt);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_xpass(const int n[3], int B, const void* src, void* dst, const R* g2x,
                        const R* g2yz, R kscale, int mode, const void* twx, hipStream_t st,
                        int cache_mode, KTables<R> kt) {
  const int NYZ = n[1] * n[2];
#define X(A)                                                                                \
  if (n[0] == A) {                                                                          \
    constexpr int TCP = xpass_tc<R>(A);                                                     \
    if (NYZ % TCP == 0)                                                                     \
      return launch_xpass_tc<R, A, TCP>(B, NYZ, src, dst, g2x, g2yz, kscale, mode, twx, cache_mode, st, kt); \
    return launch_xpass_tc<R, A, 16>(B, NYZ, src, dst, g2x, g2yz, kscale, mode, twx, cache_mode, st, kt); \
  }
  NCT_LINES(X)
#undef X
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_xpass_energy(const int n[3], int B, const void* src, const R* g2x,
                               const R* g2yz, R kscale, const void* twx, double* part,
                               int* ntiles_out, hipStream_t st, KTables<R> kt) {
  const int NYZ = n[1] * n[2];
#define X(A)                                                                                \
  if (n[0] == A) {                                                                          \
    constexpr int TCP = xpass_tc<R>(A);                                                     \
    if (NYZ % TCP == 0) {                                                                   \
      *ntiles_out = NYZ / TCP;                                                              \
      nct_launch((k_xpass_energy<R, A, TCP>), dim3(unsigned(B) * unsigned(NYZ / TCP)), \
                         dim3(XP_NT), 0, st, reinterpret_cast<const cpx<R>*>(src), NYZ, g2x,  \
                         g2yz, kscale, reinterpret_cast<const cpx<R>*>(twx), part, kt);      \
    } else {                                                                                \
      *ntiles_out = NYZ / 16;                                                               \
      nct_launch((k_xpass_energy<R, A, 16>), dim3(unsigned(B) * unsigned(NYZ / 16)),  \
                         dim3(XP_NT), 0, st, reinterpret_cast<const cpx<R>*>(src), NYZ, g2x,  \
                         g2yz, kscale, reinterpret_cast<const cpx<R>*>(twx), part, kt);      \
    }                                                                                       \
    return hipGetLastError();                                                               \
  }
  NCT_LINES(X)
#undef X
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_density(const void* psi, const double* occ, int S, size_t N, double* rho,
                          hipStream_t st) {
  nct_launch((k_density<R>), dim3(nblocks(N, 256)), dim3(256), 0, st,
                     reinterpret_cast<const cpx<R>*>(psi), occ, S, N, rho);
  return hipGetLastError();
}

hipError_t launch_fields(const double* rho, const double* vext, const double* vH, int xc,
                         double thr, const int n[3], const double cell[3], double* fields,
                         float* fields32, double* part, int* nblk_out, hipStream_t st) {
  const size_t N = size_t(n[0]) * n[1] * n[2];
  const unsigned nb = nblocks(N, 256);
  *nblk_out = int(nb);
  nct_launch(k_fields, dim3(nb), dim3(256), 0, st, rho, vext, vH, xc, thr, n[1], n[2],
                     cell[0] / n[0], cell[1] / n[1], cell[2] / n[2], 0.5 * cell[0], 0.5 * cell[1],
                     0.5 * cell[2], N, fields, fields32, part);
  return hipGetLastError();
}

hipError_t launch_reduce_rows(const double* part, int nrows, int width, double* out,
                              hipStream_t st, double* copy0) {
  nct_launch(k_reduce_rows, dim3(1), dim3(256), 0, st, part, nrows, width, out, copy0);
  return hipGetLastError();
}
hipError_t launch_add_bext(const double* fields, const int n[3], const double b[3],
                           const double lg[4], double* out, hipStream_t st) {
  const size_t N = size_t(n[0]) * n[1] * n[2];
  nct_launch(k_add_bext, dim3(nblocks(N, 256)), dim3(256), 0, st, fields, n[1], n[2], N,
                     b[0], b[1], b[2], lg[0], lg[1], lg[2], lg[3], out);
  return hipGetLastError();
}
hipError_t launch_to_float(const double* in, size_t n, float* out, hipStream_t st) {
  nct_launch(k_to_float, dim3(nblocks(n, 256)), dim3(256), 0, st, in, n, out);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_proj_contract(const ProjTables& pt, const void* W, int S, double dV,
                                void* Cpart, void* C, void* EC, hipStream_t st) {
  if (pt.natoms == 0) return hipSuccess;
  const unsigned ntile = unsigned((S + 15) / 16);
  const dim3 grid(pt.natoms, ntile, pt.max_kchunks);
  if (pt.PP == 16)
    nct_launch((k_proj_contract<R, 16>), grid, dim3(64), 0, st, pt,
                       reinterpret_cast<const cpx<R>*>(W), S, reinterpret_cast<cpx<double>*>(Cpart));
  else
    nct_launch((k_proj_contract<R, 32>), grid, dim3(64), 0, st, pt,
                       reinterpret_cast<const cpx<R>*>(W), S, reinterpret_cast<cpx<double>*>(Cpart));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t total = size_t(pt.natoms) * pt.PP * S;
  nct_launch((k_proj_reduce<R>), dim3(nblocks(total, 256)), dim3(256), 0, st, pt,
                     reinterpret_cast<const cpx<double>*>(Cpart), S, dV,
                     reinterpret_cast<cpx<double>*>(C), reinterpret_cast<cpx<R>*>(EC));
  return hipGetLastError();
}

template <typename R>
hipError_t launch_proj_scatter(const ProjTables& pt, const void* EC, int S, void* Y,
                               hipStream_t st) {
  if (pt.natoms == 0) return hipSuccess;
  const unsigned ntile = unsigned((S + 15) / 16);
  const dim3 grid(pt.natoms, pt.max_rowtiles, ntile);
  if (pt.PP == 16)
    nct_launch((k_proj_scatter<R, 16>), grid, dim3(64), 0, st, pt,
                       reinterpret_cast<const cpx<R>*>(EC), S, reinterpret_cast<cpx<R>*>(Y));
  else
    nct_launch((k_proj_scatter<R, 32>), grid, dim3(64), 0, st, pt,
                       reinterpret_cast<const cpx<R>*>(EC), S, reinterpret_cast<cpx<R>*>(Y));
  return hipGetLastError();
}

int gram_chunks(int S, size_t K) {
  const int T = (S + GRAM_T - 1) / GRAM_T;
  const size_t pairs = size_t(T) * (T + 1) / 2;
  size_t nc = (2048 + pairs - 1) / pairs;                              // enough workgroups
  nc = std::min<size_t>(nc, 256);
  nc = std::min<size_t>(nc, std::max<size_t>(1, (size_t(64) << 20) / (size_t(S) * S * 16)));  // partials <= 64 MiB
  nc = std::min<size_t>(nc, std::max<size_t>(1, K / (4 * GRAM_KB)));   // chunks of >= 64 values
  return int(std::max<size_t>(nc, 1));
}

template <typename R>
hipError_t launch_gram(const void* A, int S, size_t K, double scale, void* part, int nchunks, void* out,
                       hipStream_t st) {
  if (S <= 0 || nchunks <= 0) return hipErrorInvalidValue;
  const int T = (S + GRAM_T - 1) / GRAM_T;
  const unsigned pairs = unsigned(T) * unsigned(T + 1) / 2;
  size_t kchunk = (K + nchunks - 1) / nchunks;
  kchunk = (kchunk + GRAM_KB - 1) / GRAM_KB * GRAM_KB;
  const unsigned used = unsigned((K + kchunk - 1) / kchunk);
  nct_launch((k_gram_partial<R>), dim3(pairs, used), dim3(256), 0, st, reinterpret_cast<const cpx<R>*>(A), S, K,
             kchunk, reinterpret_cast<cpx<double>*>(part));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  nct_launch(k_gram_reduce, dim3(nblocks(size_t(S) * S, 256)), dim3(256), 0, st,
             reinterpret_cast<const cpx<double>*>(part), S, int(used), scale, reinterpret_cast<cpx<double>*>(out));
  return hipGetLastError();
}

template <typename R>
hipError_t launch_basis_transform(const void* A, const void* Mt, int S, size_t K, void* D, hipStream_t st) {
  if (S <= 0) return hipErrorInvalidValue;
  const dim3 grid(unsigned((K + BT_P - 1) / BT_P), unsigned((S + BT_J - 1) / BT_J));
  nct_launch((k_basis_transform<R>), grid, dim3(256), 0, st, reinterpret_cast<const cpx<R>*>(A),
             reinterpret_cast<const cpx<double>*>(Mt), S, K, reinterpret_cast<cpx<R>*>(D));
  return hipGetLastError();
}

hipError_t launch_obs_row(const ObsInputs& in, double* row, hipStream_t st) {
  nct_launch(k_obs_row, dim3(1), dim3(256), 0, st, in, row);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_seed(const void* psi, const double* occ, int S, size_t N, double w0, double w1,
                       double w2, double scale, void* lam, hipStream_t st) {
  nct_launch((k_seed<R>), dim3(nblocks(size_t(S) * N, 256)), dim3(256), 0, st,
                     reinterpret_cast<const cpx<R>*>(psi), occ, S, N, w0, w1, w2, scale,
                     reinterpret_cast<cpx<R>*>(lam));
  return hipGetLastError();
}
template <typename R>
hipError_t launch_axpby(void* y, const void* x, size_t count, R a_re, R a_im, R b,
                        hipStream_t st) {
  nct_launch((k_axpby<R>), dim3(nblocks(count, 256)), dim3(256), 0, st,
                     reinterpret_cast<cpx<R>*>(y), reinterpret_cast<const cpx<R>*>(x), count, a_re,
                     a_im, b);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_pair(const void* mu, const void* w, int S, size_t N, double gamma, double* g,
                       hipStream_t st) {
  nct_launch((k_pair<R>), dim3(nblocks(N, 256)), dim3(256), 0, st,
                     reinterpret_cast<const cpx<R>*>(mu), reinterpret_cast<const cpx<R>*>(w), S, N,
                     gamma, g);
  return hipGetLastError();
}
hipError_t launch_field_adjoint(const double* rho, const double* g, const double* pg, int xc,
                                double thr, size_t N, double* gnm, double* part, int* nblk_out,
                                hipStream_t st) {
  const unsigned nb = nblocks(N, 256);
  *nblk_out = int(nb);
  nct_launch(k_field_adjoint, dim3(nb), dim3(256), 0, st, rho, g, pg, xc, thr, N, gnm, part);
  return hipGetLastError();
}
template <typename R>
hipError_t launch_density_backprop(const void* psi, const double* occ, const double* gnm, int S,
                                   size_t N, int add, void* lam, hipStream_t st) {
  nct_launch((k_density_backprop<R>), dim3(nblocks(size_t(S) * N, 256)), dim3(256), 0, st,
                     reinterpret_cast<const cpx<R>*>(psi), occ, gnm, S, N, add,
                     reinterpret_cast<cpx<R>*>(lam));
  return hipGetLastError();
}

// explicit instantiations
#define NCT_INST(R)                                                                                \
  template hipError_t launch_plane_stage<R>(const int*, int, const StageArgs<R>&, const ProjTables&, \
                                            const void*, const void*, hipStream_t);                \
  template hipError_t launch_plane_fwd<R>(const int*, int, const void*, void*, void*,              \
                                          const ProjTables*, const void*, const void*, hipStream_t, \
                                          KTables<R>);                                             \
  template hipError_t launch_rephase_rows<R>(const ProjTables&, void*, int, const double*,       \
                                             hipStream_t);                                         \
  template hipError_t launch_plane_inv<R>(const int*, int, const void*, void*, R, const void*,     \
                                          const void*, hipStream_t);                               \
  template hipError_t launch_xpass<R>(const int*, int, const void*, void*, const R*, const R*, R,  \
                                      int, const void*, hipStream_t, int, KTables<R>);             \
  template hipError_t launch_xpass_energy<R>(const int*, int, const void*, const R*, const R*, R,  \
                                             const void*, double*, int*, hipStream_t, KTables<R>); \
  template hipError_t launch_density<R>(const void*, const double*, int, size_t, double*,          \
                                        hipStream_t);                                              \
  template hipError_t launch_proj_contract<R>(const ProjTables&, const void*, int, double, void*,  \
                                              void*, void*, hipStream_t);                          \
  template hipError_t launch_proj_scatter<R>(const ProjTables&, const void*, int, void*,           \
                                             hipStream_t);                                         \
  template hipError_t launch_seed<R>(const void*, const double*, int, size_t, double, double,      \
                                     double, double, void*, hipStream_t);                          \
  template hipError_t launch_axpby<R>(void*, const void*, size_t, R, R, R, hipStream_t);          \
  template hipError_t launch_pair<R>(const void*, const void*, int, size_t, double, double*,      \
                                     hipStream_t);                                               \
  template hipError_t launch_density_backprop<R>(const void*, const double*, const double*, int,  \
                                                 size_t, int, void*, hipStream_t);               \
  template hipError_t launch_gram<R>(const void*, int, size_t, double, void*, int, void*, hipStream_t); \
  template hipError_t launch_basis_transform<R>(const void*, const void*, int, size_t, void*, hipStream_t);
NCT_INST(double)
NCT_INST(float)

}  // namespace nct
