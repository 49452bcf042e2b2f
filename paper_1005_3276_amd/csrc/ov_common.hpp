// ov_common.hpp -- device building blocks for gfx950 (CDNA4, wave64).
//
// Internal field layout ("spin-planar"): one system's spinor field of V sites is
// four planes of V complex numbers, plane s holding spin component s of every
// site in lexicographic order i = x + X*(y + Y*(z + Z*t)).  A wavefront of 64
// consecutive sites therefore loads 64 consecutive complex numbers per plane:
// 1 KiB (FP64) or 512 B (FP32) per load instruction, fully coalesced.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ov {

template <class R> struct cplx_of;
template <> struct cplx_of<double> { using type = double2; };
template <> struct cplx_of<float> { using type = float2; };
template <class R> using c2 = typename cplx_of<R>::type;

template <class V> __device__ __forceinline__ V cmul_i(V a) { return V{-a.y, a.x}; }  // i*a

// Global-memory access.  Field and scalar buffers are reached through plain pointers held
// in descriptors, which the compiler accesses with flat instructions; a flat access counts
// on the LDS/scalar wait counter as well, so every LDS access, cross-lane reduction or
// scalar load after it would also wait for all loads in flight.  These helpers access the
// buffers in address space 1 (global instructions, vector memory counter only).
#define OV_GLOBAL __attribute__((address_space(1)))
template <class R>
using ev2 = R __attribute__((ext_vector_type(2)));

template <class R>
__device__ __forceinline__ c2<R> ldg2(const c2<R>* p, size_t k) {
  const ev2<R> e = ((const OV_GLOBAL ev2<R>*)p)[k];
  return c2<R>{e.x, e.y};
}

template <class R>
__device__ __forceinline__ void stg2(c2<R>* p, size_t k, c2<R> v) {
  ((OV_GLOBAL ev2<R>*)p)[k] = ev2<R>{v.x, v.y};
}

template <class T>
__device__ __forceinline__ T ldg(const T* p, size_t k) {
  return ((const OV_GLOBAL T*)p)[k];
}

// Per-system geometry.  bc is the time-boundary phase of the fermion (+1/-1).
struct Geo {
  int X, Y, Z, T;
  int V;
  int bc;
};

// Wilson term of H_W = g5 D_W(-M0) at one site (Sec. 2.2 operators with the
// Wilson-term sign fixed by the momentum-space forms of Sec. 3.1):
//   D_W psi_x = (4 - M0) psi_x - 1/2 sum_mu [(1 - g_mu) psi_{x+mu} + (1 + g_mu) psi_{x-mu}]
//             = (4 - M0) psi_x - 1/2 sum_mu S_mu + 1/2 sum_mu g_mu D_mu,
//   S_mu = psi_{x+mu} + psi_{x-mu},  D_mu = psi_{x+mu} - psi_{x-mu}.
// gamma basis of Sec. 2.1 (x,y,z -> gamma_1,2,3; t -> gamma_0):
//   g_x D = ( i D3,  i D2, -i D1, -i D0)
//   g_y D = (   D3,  -D2,  -D1,    D0)
//   g_z D = ( i D2, -i D3, -i D0,  i D1)
//   g_t D = (   D2,   D3,   D0,    D1)
// g5 = diag(-1,-1,1,1) flips the sign of spins 0,1 of the result.
template <class R>
__device__ __forceinline__ void load_sp(const c2<R>* __restrict__ f, int V, int i, c2<R> v[4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) v[s] = ldg2<R>(f, (size_t)s * V + i);
}

template <class R>
__device__ __forceinline__ void store_sp(c2<R>* __restrict__ f, int V, int i, const c2<R> v[4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) stg2<R>(f, (size_t)s * V + i, v[s]);
}

// The nine spinors the stencil reads at site i, loaded in one batch so that
// all 36 loads are in flight together (the caller may overlap other work
// before consuming them).  Time-boundary phases are applied at load time.
template <class R>
struct Nbr {
  c2<R> c[4], xf[4], xb[4], yf[4], yb[4], zf[4], zb[4], tf[4], tb[4];
};

template <class R>
__device__ __forceinline__ void load_nbr(const c2<R>* __restrict__ f, const Geo& g, int i,
                                         Nbr<R>& nb) {
  const int X = g.X, Y = g.Y, Z = g.Z, T = g.T, V = g.V;
  int r = i;
  const int x = r % X; r /= X;
  const int y = r % Y; r /= Y;
  const int z = r % Z;
  const int t = r / Z;
  const int XY = X * Y, XYZ = XY * Z;
  load_sp<R>(f, V, i, nb.c);
  load_sp<R>(f, V, (x + 1 < X) ? i + 1 : i + 1 - X, nb.xf);
  load_sp<R>(f, V, (x > 0) ? i - 1 : i - 1 + X, nb.xb);
  load_sp<R>(f, V, (y + 1 < Y) ? i + X : i + X - XY, nb.yf);
  load_sp<R>(f, V, (y > 0) ? i - X : i - X + XY, nb.yb);
  load_sp<R>(f, V, (z + 1 < Z) ? i + XY : i + XY - XYZ, nb.zf);
  load_sp<R>(f, V, (z > 0) ? i - XY : i - XY + XYZ, nb.zb);
  load_sp<R>(f, V, (t + 1 < T) ? i + XYZ : i + XYZ - V, nb.tf);
  load_sp<R>(f, V, (t > 0) ? i - XYZ : i - XYZ + V, nb.tb);
}

// H_W at site i from its loaded neighbourhood.
template <class R>
__device__ __forceinline__ void hw_compute(const Nbr<R>& nb, const Geo& g, int i, R diag,
                                           c2<R> out[4]) {
  using C = c2<R>;
  const int T = g.T;
  const int t = i / (g.X * g.Y * g.Z);
  C a[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) a[s] = C{diag * nb.c[s].x, diag * nb.c[s].y};
  C S[4], D[4];
  const R h = R(0.5);
  // ---- x
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    S[s] = C{nb.xf[s].x + nb.xb[s].x, nb.xf[s].y + nb.xb[s].y};
    D[s] = C{h * (nb.xf[s].x - nb.xb[s].x), h * (nb.xf[s].y - nb.xb[s].y)};
  }
  {
    const C g0 = cmul_i(D[3]), g1 = cmul_i(D[2]), g2 = cmul_i(D[1]), g3 = cmul_i(D[0]);
    a[0] = C{a[0].x - h * S[0].x + g0.x, a[0].y - h * S[0].y + g0.y};
    a[1] = C{a[1].x - h * S[1].x + g1.x, a[1].y - h * S[1].y + g1.y};
    a[2] = C{a[2].x - h * S[2].x - g2.x, a[2].y - h * S[2].y - g2.y};
    a[3] = C{a[3].x - h * S[3].x - g3.x, a[3].y - h * S[3].y - g3.y};
  }
  // ---- y
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    S[s] = C{nb.yf[s].x + nb.yb[s].x, nb.yf[s].y + nb.yb[s].y};
    D[s] = C{h * (nb.yf[s].x - nb.yb[s].x), h * (nb.yf[s].y - nb.yb[s].y)};
  }
  a[0] = C{a[0].x - h * S[0].x + D[3].x, a[0].y - h * S[0].y + D[3].y};
  a[1] = C{a[1].x - h * S[1].x - D[2].x, a[1].y - h * S[1].y - D[2].y};
  a[2] = C{a[2].x - h * S[2].x - D[1].x, a[2].y - h * S[2].y - D[1].y};
  a[3] = C{a[3].x - h * S[3].x + D[0].x, a[3].y - h * S[3].y + D[0].y};
  // ---- z
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    S[s] = C{nb.zf[s].x + nb.zb[s].x, nb.zf[s].y + nb.zb[s].y};
    D[s] = C{h * (nb.zf[s].x - nb.zb[s].x), h * (nb.zf[s].y - nb.zb[s].y)};
  }
  {
    const C g0 = cmul_i(D[2]), g1 = cmul_i(D[3]), g2 = cmul_i(D[0]), g3 = cmul_i(D[1]);
    a[0] = C{a[0].x - h * S[0].x + g0.x, a[0].y - h * S[0].y + g0.y};
    a[1] = C{a[1].x - h * S[1].x - g1.x, a[1].y - h * S[1].y - g1.y};
    a[2] = C{a[2].x - h * S[2].x - g2.x, a[2].y - h * S[2].y - g2.y};
    a[3] = C{a[3].x - h * S[3].x + g3.x, a[3].y - h * S[3].y + g3.y};
  }
  // ---- t (boundary phase bc on wrapping hops)
  {
    const R phf = (t + 1 == T && g.bc < 0) ? R(-1) : R(1);
    const R phb = (t == 0 && g.bc < 0) ? R(-1) : R(1);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const C u = C{phf * nb.tf[s].x, phf * nb.tf[s].y};
      const C w = C{phb * nb.tb[s].x, phb * nb.tb[s].y};
      S[s] = C{u.x + w.x, u.y + w.y};
      D[s] = C{h * (u.x - w.x), h * (u.y - w.y)};
    }
    a[0] = C{a[0].x - h * S[0].x + D[2].x, a[0].y - h * S[0].y + D[2].y};
    a[1] = C{a[1].x - h * S[1].x + D[3].x, a[1].y - h * S[1].y + D[3].y};
    a[2] = C{a[2].x - h * S[2].x + D[0].x, a[2].y - h * S[2].y + D[0].y};
    a[3] = C{a[3].x - h * S[3].x + D[1].x, a[3].y - h * S[3].y + D[1].y};
  }
  // g5
  out[0] = C{-a[0].x, -a[0].y};
  out[1] = C{-a[1].x, -a[1].y};
  out[2] = a[2];
  out[3] = a[3];
}

template <class R>
__device__ __forceinline__ void hw_site(const c2<R>* __restrict__ f, const Geo& g, int i,
                                        R diag, c2<R> out[4]) {
  Nbr<R> nb;
  load_nbr<R>(f, g, i, nb);
  hw_compute<R>(nb, g, i, diag, out);
}

template <class V> __device__ __forceinline__ double norm2_sp(const V v[4]) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double re = (double)v[k].x, im = (double)v[k].y;
    s += re * re + im * im;
  }
  return s;
}

// ---------------------------------------------------------------- reductions
// Deterministic: fixed shuffle tree inside each wave64, then waves summed in
// index order by thread 0.  Returns the block total to every thread.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Wave total returned to every lane (butterfly: same bits in every lane).
__device__ __forceinline__ double wave_sum_all(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int MAXW = 16>
__device__ __forceinline__ double block_sum(double v, double* lds /* >= MAXW+1 */) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  if (lane == 0) lds[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += lds[k];
    lds[MAXW] = s;
  }
  __syncthreads();
  const double r = lds[MAXW];
  __syncthreads();
  return r;
}

// Sum of n partials in fixed order: thread j accumulates j, j+B, ... then a
// block_sum.  Every block that calls this on the same data gets the same bits.
template <int MAXW = 16>
__device__ __forceinline__ double sum_partials(const double* __restrict__ p, int n, double* lds) {
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) s += p[j];
  return block_sum<MAXW>(s, lds);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// Remap so that each XCD works on one contiguous range of logical blocks, which
// keeps the y/z/t stencil neighbours of a block in the same L2.
__device__ __forceinline__ int xcd_logical_block(int nb) {
  const int b = blockIdx.x;
  const int q = nb >> 3, rem = nb & 7;
  const int xcd = b & 7, k = b >> 3;
  return xcd * q + (xcd < rem ? xcd : rem) + k;
}

}  // namespace ov
