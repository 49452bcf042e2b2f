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
  for (int s = 0; s < 4; ++s) v[s] = f[(size_t)s * V + i];
}

template <class R>
__device__ __forceinline__ void store_sp(c2<R>* __restrict__ f, int V, int i, const c2<R> v[4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) f[(size_t)s * V + i] = v[s];
}

template <class R>
__device__ __forceinline__ void hw_site(const c2<R>* __restrict__ f, const Geo& g, int i,
                                        R diag, c2<R> out[4]) {
  using C = c2<R>;
  const int X = g.X, Y = g.Y, Z = g.Z, T = g.T, V = g.V;
  int r = i;
  const int x = r % X; r /= X;
  const int y = r % Y; r /= Y;
  const int z = r % Z;
  const int t = r / Z;
  const int XY = X * Y, XYZ = XY * Z;

  C c[4];
  load_sp<R>(f, V, i, c);
  C a[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) a[s] = C{diag * c[s].x, diag * c[s].y};

  C pf[4], pb[4], S[4], D[4];
  const R h = R(0.5);
  // ---- x
  {
    const int jf = (x + 1 < X) ? i + 1 : i + 1 - X;
    const int jb = (x > 0) ? i - 1 : i - 1 + X;
    load_sp<R>(f, V, jf, pf);
    load_sp<R>(f, V, jb, pb);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      S[s] = C{pf[s].x + pb[s].x, pf[s].y + pb[s].y};
      D[s] = C{h * (pf[s].x - pb[s].x), h * (pf[s].y - pb[s].y)};
    }
    C g0 = cmul_i(D[3]), g1 = cmul_i(D[2]), g2 = cmul_i(D[1]), g3 = cmul_i(D[0]);
    a[0] = C{a[0].x - h * S[0].x + g0.x, a[0].y - h * S[0].y + g0.y};
    a[1] = C{a[1].x - h * S[1].x + g1.x, a[1].y - h * S[1].y + g1.y};
    a[2] = C{a[2].x - h * S[2].x - g2.x, a[2].y - h * S[2].y - g2.y};
    a[3] = C{a[3].x - h * S[3].x - g3.x, a[3].y - h * S[3].y - g3.y};
  }
  // ---- y
  {
    const int jf = (y + 1 < Y) ? i + X : i + X - XY;
    const int jb = (y > 0) ? i - X : i - X + XY;
    load_sp<R>(f, V, jf, pf);
    load_sp<R>(f, V, jb, pb);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      S[s] = C{pf[s].x + pb[s].x, pf[s].y + pb[s].y};
      D[s] = C{h * (pf[s].x - pb[s].x), h * (pf[s].y - pb[s].y)};
    }
    a[0] = C{a[0].x - h * S[0].x + D[3].x, a[0].y - h * S[0].y + D[3].y};
    a[1] = C{a[1].x - h * S[1].x - D[2].x, a[1].y - h * S[1].y - D[2].y};
    a[2] = C{a[2].x - h * S[2].x - D[1].x, a[2].y - h * S[2].y - D[1].y};
    a[3] = C{a[3].x - h * S[3].x + D[0].x, a[3].y - h * S[3].y + D[0].y};
  }
  // ---- z
  {
    const int jf = (z + 1 < Z) ? i + XY : i + XY - XYZ;
    const int jb = (z > 0) ? i - XY : i - XY + XYZ;
    load_sp<R>(f, V, jf, pf);
    load_sp<R>(f, V, jb, pb);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      S[s] = C{pf[s].x + pb[s].x, pf[s].y + pb[s].y};
      D[s] = C{h * (pf[s].x - pb[s].x), h * (pf[s].y - pb[s].y)};
    }
    C g0 = cmul_i(D[2]), g1 = cmul_i(D[3]), g2 = cmul_i(D[0]), g3 = cmul_i(D[1]);
    a[0] = C{a[0].x - h * S[0].x + g0.x, a[0].y - h * S[0].y + g0.y};
    a[1] = C{a[1].x - h * S[1].x - g1.x, a[1].y - h * S[1].y - g1.y};
    a[2] = C{a[2].x - h * S[2].x - g2.x, a[2].y - h * S[2].y - g2.y};
    a[3] = C{a[3].x - h * S[3].x + g3.x, a[3].y - h * S[3].y + g3.y};
  }
  // ---- t (boundary phase bc on wrapping hops)
  {
    const bool wf = (t + 1 == T), wb = (t == 0);
    const int jf = wf ? i + XYZ - V : i + XYZ;
    const int jb = wb ? i - XYZ + V : i - XYZ;
    load_sp<R>(f, V, jf, pf);
    load_sp<R>(f, V, jb, pb);
    const R phf = (wf && g.bc < 0) ? R(-1) : R(1);
    const R phb = (wb && g.bc < 0) ? R(-1) : R(1);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const C u = C{phf * pf[s].x, phf * pf[s].y};
      const C w = C{phb * pb[s].x, phb * pb[s].y};
      S[s] = C{u.x + w.x, u.y + w.y};
      D[s] = C{h * (u.x - w.x), h * (u.y - w.y)};
    }
    a[0] = C{a[0].x - h * S[0].x + D[2].x, a[0].y - h * S[0].y + D[2].y};
    a[1] = C{a[1].x - h * S[1].x + D[3].x, a[1].y - h * S[1].y + D[3].y};
    a[2] = C{a[2].x - h * S[2].x + D[0].x, a[2].y - h * S[2].y + D[0].y};
    a[3] = C{a[3].x - h * S[3].x + D[1].x, a[3].y - h * S[3].y + D[1].y};
  }
  out[0] = C{-a[0].x, -a[0].y};
  out[1] = C{-a[1].x, -a[1].y};
  out[2] = a[2];
  out[3] = a[3];
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
