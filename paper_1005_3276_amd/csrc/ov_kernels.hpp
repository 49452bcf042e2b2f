// ov_kernels.hpp -- HIP kernels of the overlap hot path (gfx950).
//
// Every kernel works on a *batch* of systems: one system is one right-hand
// side on one lattice.  A launch covers sum_s nblk_s workgroups; workgroup b
// is remapped XCD-contiguously to a logical block L, which belongs to system
// s with sys[s].blk0 <= L < sys[s].blk0 + sys[s].nblk.  Systems may live on
// lattices of different sizes (uneven batches) and carry their own scalars,
// iteration counts and convergence flags.
//
// Multi-shift CG, Krylov-basis form.  For (H^2 + b_k) y_k = psi the shifted
// solutions are linear combinations of the base residuals r_j, with scalar
// coefficients that follow from the base CG scalars alone (Jegerlehner's
// recurrences).  The pole sum needed by the sign function is
//     eps = H sum_k a_k y_k = sum_j d_j t_j,   t_j = H P_j,
// so one pass of the base CG on H^2 that keeps every t_j (HBM is 288 GB) plus
// one combination pass replaces the n_poles shifted search directions of the
// textbook algorithm.  Per iteration only two vectors are read and one written
// in each of the two stencil kernels:
//     k_ms_t:  t_n = H r_n + beta_{n-1} t_{n-1}         (= H P_n, P never stored)
//     k_ms_r:  r_{n+1} = r_n - alpha_n H t_n
// The scalar reductions are finished redundantly by every workgroup of the
// next kernel (fixed summation order -> identical bits in every workgroup), so
// no grid barrier, atomic or host round trip is needed inside an iteration.
#pragma once

#include "ov_common.hpp"

namespace ov {

constexpr int MAXP = 32;      // max poles
constexpr int NTHREADS = 256; // default workgroup size (4 waves)

// Device descriptor of one system for one phase of a solve.
struct SysDev {
  Geo g;
  int nblk;    // workgroups of this system in a launch
  int blk0;    // first logical workgroup
  int spb;     // sites per workgroup
  int pad0;
  int* active;              // host-controlled on/off flag (batched solves); may be null
  // multi-shift
  void* basis;              // t_j slots, slot stride 4V complex
  void* r;                  // r_n, n >= 1
  const void* src;          // r_0
  double* part_a;           // [nblk] |t_n|^2 partials
  double* part_b;           // [nblk] |r_n|^2 partials (source partials for n = 0)
  double* h_rho;            // [cap+1]
  double* h_alpha;          // [cap+1]
  double* h_zeta;           // [(cap+1) * MAXP]
  unsigned int* h_active;   // [cap+1] shift masks
  int* h_ctl;               // [4]: done, n_done, status, sticky error (host-reset)
  long long* stat;          // [4]: inner iterations, multi-shift solves, max N, max N of the
                            //      current outer iteration (cleared by k_cg_p)
  double* dstat;            // [2]: max shift residual of the last multi-shift, (unused)
  double* coef_term;        // [MAXP * cap]
  double* coef_c;           // [cap+1]
  double* coef_d;           // [cap]
  double* coef_d2;          // [cap] non-null: also the coefficients of H r(A)^2 psi (k_ms_coef)
  double* coef_sq;          // [(2 MAXP + 2) cap] scratch of those coefficients
  // epilogue / CG
  const double2* phi;       // [V] background scalar
  const void* e_in;         // operator input psi (spin-planar, kernel precision)
  void* e_out;              // operator output
  void* e_out2;             // optional g5 * output (next multi-shift source)
  double* part_c;           // [nblk] partials of |e_out|^2 or |r|^2
  void* cg_x;               // CG vectors (kernel precision)
  void* cg_p;
  void* cg_r;
  void* cg_z;               // preconditioned residual z = P r (PCG); null: z = r
  const double2* cg_b;      // FP64 right-hand side (true residual)
  void* cg_r64;             // FP64 true residual out
  void* cg_x64;             // FP64 solution (reliable updates)
  double* cg_s;             // per-system CG scalars (see CG_* below)
  double m_re, m_im;        // fermion mass
  double pc_re, pc_im;      // mass of the preconditioner M0 (m, or the RMS of c = m + g phi)
  double shift;             // sigma of a shifted solve (MdagM + sigma) x = b; 0 otherwise
  double g_re, g_im;        // Yukawa coupling
  double2* shx;             // multi-shift CG on MdagM: nshift solutions (FP64 planar)
  double2* shp;             //   and nshift search directions
  const double* shc;        //   per-shift coefficients (SHC_* layout)
  int nshift;
  void* fft_tmp;            // momentum-space scratch field (kernel precision)
  int off_xy, off_z, off_t; // first workgroup of this system in each transform pass
  int xc;                   // x values per workgroup in the t pass (divides X, xc T <= 64)
  double* pcs;              // [V] preconditioner scale per momentum (k_pcg_table), or null
};

// CG scalar slots
// CG_RR holds rho = <r, z> (= |r|^2 without a preconditioner); CG_R2 holds |r|^2 of
// the preconditioned recursion.
enum { CG_RR = 0, CG_RR_OLD, CG_PAP, CG_ALPHA, CG_BETA, CG_BB, CG_RTRUE, CG_R2, CG_NSLOT = 8 };

struct MsParams {
  int np;               // poles
  int cap;              // basis capacity (max iterations)
  double tol;           // shift tolerance
  double diag;          // 4 - M0
  double sigma[MAXP];   // shifts b_k
  double coef[MAXP];    // residues a_k
  int zm;               // > 0: z-marching passes over zm planes per workgroup (ZmMarch)
  unsigned long long* tstamp;  // non-null: per workgroup (start, end, sites) stamps
};

__device__ __forceinline__ int find_sys(const SysDev* __restrict__ sys, int nsys, int L) {
  int s = 0;
  for (int k = 1; k < nsys; ++k)
    if (sys[k].blk0 <= L) s = k;
  return s;
}

// ------------------------------------------------------------------ pack
// ABI complex128 (V,4) AoS (optionally times g5, times scale) <-> spin-planar R.
template <class R>
__global__ void k_pack(const SysDev* __restrict__ sys, const int* __restrict__ bmap, int nb_total,
                       const double2* const* __restrict__ src, void* const* __restrict__ dst,
                       double scale) {
  const int L = xcd_logical_block(nb_total);
  const int s = bmap[L];
  const SysDev& S = sys[s];
  const int V = S.g.V;
  const int lb = L - S.blk0;
  const double2* in = src[s];
  c2<R>* out = (c2<R>*)dst[s];
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double2 v = in[(size_t)i * 4 + k];
      out[(size_t)k * V + i] = c2<R>{(R)(scale * v.x), (R)(scale * v.y)};
    }
  }
}

template <class R>
__global__ void k_unpack(const SysDev* __restrict__ sys, const int* __restrict__ bmap, int nb_total,
                         void* const* __restrict__ src, double2* const* __restrict__ dst) {
  const int L = xcd_logical_block(nb_total);
  const int s = bmap[L];
  const SysDev& S = sys[s];
  const int V = S.g.V;
  const int lb = L - S.blk0;
  const c2<R>* in = (const c2<R>*)src[s];
  double2* out = dst[s];
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const c2<R> v = in[(size_t)k * V + i];
      out[(size_t)i * 4 + k] = double2{(double)v.x, (double)v.y};
    }
  }
}

// out = a * in over n complex128 values (ABI layout).
__global__ void k_scale_copy(double2* __restrict__ out, const double2* __restrict__ in, double a,
                             size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const double2 v = in[i];
    out[i] = double2{a * v.x, a * v.y};
  }
}

// dst += a * src: planar FP64 src (spin-planar) added into the ABI's complex128 AoS dst.
__global__ void k_unpack_axpy(const SysDev* __restrict__ sys, const int* __restrict__ bmap,
                              int nb_total, void* const* __restrict__ src,
                              double2* const* __restrict__ dst, double a) {
  const int L = xcd_logical_block(nb_total);
  const int s = bmap[L];
  const SysDev& S = sys[s];
  const int V = S.g.V;
  const int lb = L - S.blk0;
  const double2* in = (const double2*)src[s];
  double2* out = dst[s];
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double2 v = in[(size_t)k * V + i];
      double2& o = out[(size_t)i * 4 + k];
      o = double2{o.x + a * v.x, o.y + a * v.y};
    }
  }
}

// ---------------------------------------------------------- plain stencil
// out = H_W in; optional |out|^2 partials.  in/out per system from e_in/e_out.
template <class R>
__global__ void __launch_bounds__(256) k_hw(const SysDev* __restrict__ sys, const int* __restrict__ bmap,
                                             int nb_total, double diag, int want_norm) {
  __shared__ double lds[17];
  const int L = xcd_logical_block(nb_total);
  const int s = bmap[L];
  const SysDev& S = sys[s];
  const Geo g = S.g;
  const int lb = L - S.blk0;
  const c2<R>* in = (const c2<R>*)S.e_in;
  c2<R>* out = (c2<R>*)S.e_out;
  const int i0 = lb * S.spb;
  const int i1 = min(g.V, i0 + S.spb);
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    c2<R> o[4];
    hw_site<R>(in, g, i, (R)diag, o);
    store_sp<R>(out, g.V, i, o);
    if (want_norm) acc += norm2_sp(o);
  }
  if (want_norm) {
    const double tot = block_sum(acc, lds);
    if (threadIdx.x == 0) S.part_c[lb] = tot;
  }
}

// out = H_W in with the block's own sites staged in LDS: a block of spb
// consecutive sites covers whole x rows (and, at 16^4 with 256 sites, a whole
// xy plane), so its x and y neighbours are read from LDS and only the centre
// and the z and t neighbours come through the vector cache (5 of 9 spinor
// loads).  Neighbours outside the block fall back to global loads.
// Dynamic LDS: 4 * spb complex values.
template <class R>
__device__ __forceinline__ void nb_lds(const c2<R>* __restrict__ f, const c2<R>* sh, int V, int spb,
                                       int i0, int i1, int j, c2<R> v[4]) {
  if (j >= i0 && j < i1) {
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = sh[s * spb + (j - i0)];
  } else {
    load_sp<R>(f, V, j, v);
  }
}

template <class R>
__device__ __forceinline__ void load_nbr_staged(const c2<R>* __restrict__ f, const Geo& g, int i,
                                                const c2<R>* sh, int spb, int i0, int i1,
                                                Nbr<R>& nb) {
  const int X = g.X, Y = g.Y, Z = g.Z, T = g.T, V = g.V;
  int r = i;
  const int x = r % X; r /= X;
  const int y = r % Y; r /= Y;
  const int z = r % Z;
  const int t = r / Z;
  const int XY = X * Y, XYZ = XY * Z;
  load_sp<R>(f, V, (z + 1 < Z) ? i + XY : i + XY - XYZ, nb.zf);
  load_sp<R>(f, V, (z > 0) ? i - XY : i - XY + XYZ, nb.zb);
  load_sp<R>(f, V, (t + 1 < T) ? i + XYZ : i + XYZ - V, nb.tf);
  load_sp<R>(f, V, (t > 0) ? i - XYZ : i - XYZ + V, nb.tb);
#pragma unroll
  for (int s = 0; s < 4; ++s) nb.c[s] = sh[s * spb + (i - i0)];
  nb_lds<R>(f, sh, V, spb, i0, i1, (x + 1 < X) ? i + 1 : i + 1 - X, nb.xf);
  nb_lds<R>(f, sh, V, spb, i0, i1, (x > 0) ? i - 1 : i - 1 + X, nb.xb);
  nb_lds<R>(f, sh, V, spb, i0, i1, (y + 1 < Y) ? i + X : i + X - XY, nb.yf);
  nb_lds<R>(f, sh, V, spb, i0, i1, (y > 0) ? i - X : i - X + XY, nb.yb);
}

// Stage the block's sites [i0, i1) of f into sh (planar, 4 * spb values).
template <class R>
__device__ __forceinline__ void stage_block(const c2<R>* __restrict__ f, int V, int spb, int i0,
                                            int i1, c2<R>* sh) {
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
#pragma unroll
    for (int s = 0; s < 4; ++s) sh[s * spb + (i - i0)] = f[(size_t)s * V + i];
  }
  __syncthreads();
}

template <class R>
__global__ void __launch_bounds__(256) k_hw_lds(const SysDev* __restrict__ sys, const int* __restrict__ bmap,
                                                 int nb_total, double diag) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  c2<R>* sh = (c2<R>*)dyn_lds;
  const int L = xcd_logical_block(nb_total);
  const SysDev& S = sys[bmap[L]];
  const Geo g = S.g;
  const int lb = L - S.blk0;
  const c2<R>* in = (const c2<R>*)S.e_in;
  c2<R>* out = (c2<R>*)S.e_out;
  const int spb = S.spb;
  const int i0 = lb * spb;
  const int i1 = min(g.V, i0 + spb);
  stage_block<R>(in, g.V, spb, i0, i1, sh);
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    Nbr<R> nb;
    load_nbr_staged<R>(in, g, i, sh, spb, i0, i1, nb);
    c2<R> o[4];
    hw_compute<R>(nb, g, i, (R)diag, o);
    store_sp<R>(out, g.V, i, o);
  }
}

// out = H_W in, z-marching form: a workgroup owns one xy plane (X Y <= 256
// sites, one per thread) of one time slice and walks ZC consecutive z planes.
// The z neighbours stay in registers (the plane below, the current one, the
// plane above), the x and y neighbours come from the current plane staged in
// LDS, so each output site reads (ZC + 2)/ZC centre spinors plus its two time
// neighbours from the memory hierarchy instead of nine spinors.  Every system
// of the table has the same lattice.  Grid: nsys * T * (Z / ZC) workgroups.
// Streaming store of a site's spinor: marked non-temporal so that the output lines do
// not push the input planes, which neighbouring workgroups still read, out of L2.
template <class R>
__device__ __forceinline__ void store_sp_nt(c2<R>* __restrict__ f, int V, int i, const c2<R> v[4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const ev2<R> e = {v[s].x, v[s].y};
    __builtin_nontemporal_store(e, (OV_GLOBAL ev2<R>*)(f + (size_t)s * V + i));
  }
}

template <class R, int ZC>
__global__ void __launch_bounds__(256) k_hw_zm(const SysDev* __restrict__ sys, double diag) {
  __shared__ c2<R> sh[4 * 256];
  const Geo g = sys[0].g;
  const int X = g.X, Y = g.Y, Z = g.Z, T = g.T, V = g.V;
  const int XY = X * Y, XYZ = XY * Z;
  const int nzc = Z / ZC;
  // XCD-contiguous order: the workgroups of neighbouring time slices share an L2,
  // which then serves the time-neighbour reads.  FP64 takes the time slices fastest
  // (time neighbours in consecutive workgroups, loaded together: 48 fields at 16^4 read
  // 1.14x instead of 1.23x the algorithmic bytes, 5.14 -> 5.43 TB/s); FP32, with more
  // workgroups resident, reuses them as well with the z chunks fastest (1.04x; 1.09x
  // the other way round).
  const int b = xcd_logical_block(gridDim.x);
  const int s = b / (T * nzc);
  constexpr bool t_fast = sizeof(R) == sizeof(double);
  const int t = t_fast ? b % T : (b / nzc) % T;
  const int z0 = (t_fast ? (b / T) % nzc : b % nzc) * ZC;
  const SysDev& S = sys[s];
  const c2<R>* in = (const c2<R>*)S.e_in;
  c2<R>* out = (c2<R>*)S.e_out;
  const int j = threadIdx.x;
  const bool on = j < XY;
  const int x = on ? j % X : 0, y = on ? j / X : 0;
  const int tf_off = (t + 1 < T) ? XYZ : XYZ - V;
  const int tb_off = (t > 0) ? -XYZ : V - XYZ;
  const int jxf = y * X + ((x + 1 < X) ? x + 1 : 0);
  const int jxb = y * X + ((x > 0) ? x - 1 : X - 1);
  const int jyf = ((y + 1 < Y) ? y + 1 : 0) * X + x;
  const int jyb = ((y > 0) ? y - 1 : Y - 1) * X + x;
  auto site = [&](int z) { return j + XY * (z + Z * t); };
  auto zwrap = [&](int z) { return z < 0 ? z + Z : (z >= Z ? z - Z : z); };
  // software pipeline: the plane above and the time neighbours of the next plane
  // are loaded one step ahead
  c2<R> prev[4], cur[4], next[4], tf[4], tb[4];
  if (on) {
    load_sp<R>(in, V, site(zwrap(z0 - 1)), prev);
    load_sp<R>(in, V, site(z0), cur);
    load_sp<R>(in, V, site(zwrap(z0 + 1)), next);
    load_sp<R>(in, V, site(z0) + tf_off, tf);
    load_sp<R>(in, V, site(z0) + tb_off, tb);
  }
#pragma unroll
  for (int zi = 0; zi < ZC; ++zi) {
    const int z = z0 + zi;
    const int i = site(z);
    c2<R> next2[4], tf2[4], tb2[4];
    if (on && zi + 1 < ZC) {
      load_sp<R>(in, V, site(zwrap(z + 2)), next2);
      load_sp<R>(in, V, site(z + 1) + tf_off, tf2);
      load_sp<R>(in, V, site(z + 1) + tb_off, tb2);
    }
    __syncthreads();  // the previous plane's LDS reads are done
    if (on) {
#pragma unroll
      for (int q = 0; q < 4; ++q) sh[q * 256 + j] = cur[q];
    }
    __syncthreads();
    if (on) {
      Nbr<R> nb;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        nb.c[q] = cur[q];
        nb.xf[q] = sh[q * 256 + jxf];
        nb.xb[q] = sh[q * 256 + jxb];
        nb.yf[q] = sh[q * 256 + jyf];
        nb.yb[q] = sh[q * 256 + jyb];
        nb.zf[q] = next[q];
        nb.zb[q] = prev[q];
        nb.tf[q] = tf[q];
        nb.tb[q] = tb[q];
      }
      c2<R> o[4];
      hw_compute<R>(nb, g, i, (R)diag, o);
      store_sp_nt<R>(out, V, i, o);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        prev[q] = cur[q];
        cur[q] = next[q];
        next[q] = next2[q];
        tf[q] = tf2[q];
        tb[q] = tb2[q];
      }
    }
  }
}

// H_W of f on the sites of a workgroup that owns zc consecutive z planes of one
// time slice (X Y == blockDim.x; the block's sites i0 .. i0 + zc X Y - 1, zc
// dividing Z), in the z-marching order of k_hw_zm: plane z below and above in
// registers, the current plane in LDS (sh: 4 X Y values) for the x and y
// neighbours.  Next to the stencil operands each site may take one more spinor
// of its own (the epilogue operand, from ep).  begin() issues the loads of the
// first plane, so that a caller puts them in flight before its scalar work (a
// workgroup whose system has converged reads no more than that); with PIPE, run()
// loads the operands of plane k + 1 while plane k is computed (two register sets),
// else after it.  For each site, epi(i, w, e) receives w = (H_W f)_i and the epilogue
// operand e and returns a partial sum; run() returns the total.  Every thread of the
// block must call run().
template <class R, bool PIPE>
struct ZmMarch {
  const c2<R>* f;
  const c2<R>* ep;
  int V, XY, Z, base, z0, tf_off, tb_off, jxf, jxb, jyf, jyb;
  c2<R> prev[4], cur[4], next[4], tf[4], tb[4], e[4];
  c2<R> next2[4], tf2[4], tb2[4], e2[4];  // PIPE: operands of the following plane

  __device__ __forceinline__ int plane(int z) const { return base + XY * (z < Z ? z : z - Z); }

  // operands of the plane after the one at site index i (z index z of that plane)
  __device__ __forceinline__ void load_ahead(int i, int z) {
    const int i2 = i + XY;  // plane z + 1 < Z
    load_sp<R>(f, V, plane(z + 2), next2);
    load_sp<R>(f, V, i2 + tf_off, tf2);
    load_sp<R>(f, V, i2 + tb_off, tb2);
    if (ep) load_sp<R>(ep, V, i2, e2);
  }

  __device__ __forceinline__ void begin(const c2<R>* __restrict__ f_, const c2<R>* __restrict__ ep_,
                                        const Geo& g, int i0) {
    f = f_;
    ep = ep_;
    const int X = g.X, Y = g.Y, T = g.T;
    V = g.V;
    Z = g.Z;
    XY = X * Y;
    const int XYZ = XY * Z;
    const int j = threadIdx.x;
    const int x = j % X, y = j / X;
    const int p0 = i0 / XY;  // z0 + Z t
    const int t = p0 / Z;
    z0 = p0 - Z * t;
    tf_off = (t + 1 < T) ? XYZ : XYZ - V;
    tb_off = (t > 0) ? -XYZ : V - XYZ;
    jxf = y * X + ((x + 1 < X) ? x + 1 : 0);
    jxb = y * X + ((x > 0) ? x - 1 : X - 1);
    jyf = ((y + 1 < Y) ? y + 1 : 0) * X + x;
    jyb = ((y > 0) ? y - 1 : Y - 1) * X + x;
    base = j + XYZ * t;
    const int i = plane(z0);
    load_sp<R>(f, V, plane(z0 > 0 ? z0 - 1 : Z - 1), prev);
    load_sp<R>(f, V, i, cur);
    load_sp<R>(f, V, plane(z0 + 1), next);
    load_sp<R>(f, V, i + tf_off, tf);
    load_sp<R>(f, V, i + tb_off, tb);
    if (ep) load_sp<R>(ep, V, i, e);
  }

  template <class Epi>
  __device__ __forceinline__ double run(int zc, const Geo& g, R diag, c2<R>* sh, Epi epi) {
    const int j = threadIdx.x;
    double acc = 0.0;
    for (int k = 0; k < zc; ++k) {
      const int i = plane(z0 + k);
      if (PIPE && k + 1 < zc) load_ahead(i, z0 + k);
      __syncthreads();  // reads of the previous plane are done
#pragma unroll
      for (int q = 0; q < 4; ++q) sh[q * XY + j] = cur[q];
      __syncthreads();
      Nbr<R> nb;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        nb.c[q] = cur[q];
        nb.xf[q] = sh[q * XY + jxf];
        nb.xb[q] = sh[q * XY + jxb];
        nb.yf[q] = sh[q * XY + jyf];
        nb.yb[q] = sh[q * XY + jyb];
        nb.zf[q] = next[q];
        nb.zb[q] = prev[q];
        nb.tf[q] = tf[q];
        nb.tb[q] = tb[q];
      }
      c2<R> w[4];
      hw_compute<R>(nb, g, i, diag, w);
      acc += epi(i, w, e);
      if (PIPE) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          prev[q] = cur[q];
          cur[q] = next[q];
          next[q] = next2[q];
          tf[q] = tf2[q];
          tb[q] = tb2[q];
          e[q] = e2[q];
        }
      } else if (k + 1 < zc) {
        const int i2 = i + XY;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          prev[q] = cur[q];
          cur[q] = next[q];
        }
        load_sp<R>(f, V, plane(z0 + k + 2), next);
        load_sp<R>(f, V, i2 + tf_off, tf);
        load_sp<R>(f, V, i2 + tb_off, tb);
        if (ep) load_sp<R>(ep, V, i2, e);
      }
    }
    return acc;
  }
};

// First site of z-marching workgroup lb of a system (lb < T Z / zc).  As in k_hw_zm, FP64
// takes the time slices fastest, so that time-neighbouring planes belong to consecutive
// workgroups (loaded together, served by one L2); FP32 keeps the z chunks fastest.
template <class R>
__device__ __forceinline__ int zm_first_site(const SysDev& S, int lb) {
  if (sizeof(R) == sizeof(double)) {
    const int nzc = (S.g.Z * S.g.X * S.g.Y) / S.spb;  // z chunks per time slice
    return ((lb % S.g.T) * nzc + lb / S.g.T) * S.spb;
  }
  return lb * S.spb;
}

// The z-marching passes prefetch the next plane's operands in FP32 only (ZM = 2): in
// FP64 the second register set would halve the co-resident workgroups of large launches
// and measured no faster on small ones.

// ------------------------------------------------------- multi-shift: t pass
// Iteration n.  Finishes rho_n = |r_n|^2 (partials of the previous kernel),
// advances the shift recurrences, decides convergence, then
//   t_n = H r_n + beta_{n-1} t_{n-1}  -> basis slot n,  partial |t_n|^2.
// Latency layout: every independent load (control word, partials, scalar
// history, the nine stencil operands and t_{n-1}) is issued before any of them
// is consumed, and each wave finishes the reduction and the shift recurrences
// on its own (identical bits in every wave), so the only barrier is the final
// block reduction.
// ZM: 0 plain passes, 1 z-marching, 2 z-marching with the next plane prefetched.
// CF: read the system's on/off flag and the done word before the stencil operands, so
// that a workgroup with nothing to do returns without reading them (large batched
// launches, where other workgroups hide the extra round trip); else the operands go out
// first and the check follows (a single system's launch waits for memory once).
template <class R, int ZM, bool CF>
__device__ __forceinline__ int ms_t_block(const SysDev& S, int lb, int n, const MsParams* mp,
                                          double* lds, c2<R>* sh) {
  const int lane = threadIdx.x & 63;
  const Geo g = S.g;
  const int np = mp->np;
  const int nblk = S.nblk;

  const int act_sys = S.active ? *S.active : 1;
  const int done = (n > 0) ? S.h_ctl[0] : 0;
  // partials of rho_n (this lane's share, summed in a fixed order)
  double pr = 0.0;
  for (int j = lane; j < nblk; j += 64) pr += ldg(S.part_b, j);
  // scalar history for lane k = shift k
  const int k = lane;
  double zk1 = 1.0, zk2 = 1.0, a1 = 0.0, a2 = 1.0, rho_m1 = 1.0, rho_m2 = 1.0, rho0 = 0.0;
  unsigned int act_prev = 0xffffffffu;
  if (n > 0) {
    act_prev = S.h_active[n - 1];
    rho_m1 = S.h_rho[n - 1];
    a1 = S.h_alpha[n - 1];
    rho0 = S.h_rho[0];
    if (k < np) zk1 = S.h_zeta[(size_t)(n - 1) * MAXP + k];
    if (n >= 2) {
      a2 = S.h_alpha[n - 2];
      rho_m2 = S.h_rho[n - 2];
      if (k < np) zk2 = S.h_zeta[(size_t)(n - 2) * MAXP + k];
    }
  }
  // stencil operands
  const size_t slot = (size_t)4 * g.V;
  const c2<R>* rin = (const c2<R>*)(n == 0 ? S.src : S.r);
  c2<R>* tn = (c2<R>*)S.basis + (size_t)n * slot;
  const c2<R>* tp = (const c2<R>*)S.basis + (size_t)(n > 0 ? n - 1 : 0) * slot;
  const int i0 = ZM ? zm_first_site<R>(S, lb) : lb * S.spb;
  const int i1 = min(g.V, i0 + S.spb);
  int i = i0 + threadIdx.x;
  constexpr bool zm = ZM > 0;  // z-marching (mp->zm planes per workgroup)
  const bool have = !zm && i < i1;
  Nbr<R> nb;
  c2<R> q[4];
  ZmMarch<R, ZM == 2> zmm;
  if (CF && (!act_sys || done)) return 0;
  if (zm) zmm.begin(rin, n > 0 ? tp : nullptr, g, i0);
  if (have) {
    load_nbr<R>(rin, g, i, nb);
    if (n > 0) load_sp<R>(tp, g.V, i, q);
  }
  if (!act_sys || done) return 0;

  // rho_n and the shift recurrences, per wave
  const double rho = wave_sum_all(pr);
  const double srho = sqrt(rho);
  if (n == 0) rho0 = rho;
  const double thr = mp->tol * sqrt(rho0);
  bool act = false;
  double zn = 1.0;
  if (n == 0) {
    act = (k < np) && (srho > thr);
  } else if (k < np) {
    zn = zk1;
    if (act_prev & (1u << k)) {
      const double b2 = (n >= 2) ? rho_m1 / rho_m2 : 0.0;  // beta_{n-2}
      const double den = a2 * zk2 * (1.0 + a1 * mp->sigma[k]) + a1 * b2 * (zk2 - zk1);
      zn = zk1 * zk2 * a2 / den;
      act = fabs(zn) * srho > thr;
    }
  }
  const unsigned int amask = (unsigned int)__ballot(act);
  int status = 0;
  if (n > 0 && (!(rho >= 0.0) || !isfinite(rho))) status = 1;  // breakdown
  int stop = (amask == 0) || status != 0;
  if (!stop && n >= mp->cap) { stop = 1; status = 2; }            // basis exhausted
  if (lb == 0 && threadIdx.x < 64) {
    if (k < np) S.h_zeta[(size_t)n * MAXP + k] = zn;
    if (k == 0) {
      S.h_rho[n] = rho;
      S.h_active[n] = amask;
      if (stop) {
        S.h_ctl[1] = n;
        S.h_ctl[2] = status;
      }
      // one word: 0 while iterating, n + 1 once finished at iteration n
      __hip_atomic_store(&S.h_ctl[0], stop ? n + 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (stop) return 0;
  const R beta = (R)((n > 0) ? rho / rho_m1 : 0.0);

  double acc = 0.0;
  if (zm) {
    acc = zmm.run(mp->zm, g, (R)mp->diag, sh, [&](int ii, c2<R>* o, const c2<R>* qq) -> double {
      if (n > 0) {
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2)
          o[k2] = c2<R>{o[k2].x + beta * qq[k2].x, o[k2].y + beta * qq[k2].y};
      }
      store_sp_nt<R>(tn, g.V, ii, o);
      return norm2_sp(o);
    });
    i = i1;  // every site done
  }
  if (have) {
    c2<R> o[4];
    hw_compute<R>(nb, g, i, (R)mp->diag, o);
    if (n > 0) {
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) o[k2] = c2<R>{o[k2].x + beta * q[k2].x, o[k2].y + beta * q[k2].y};
    }
    store_sp_nt<R>(tn, g.V, i, o);
    acc = norm2_sp(o);
  }
  // remaining sites of this block (sites per thread > 1)
  for (i += blockDim.x; !zm && i < i1; i += blockDim.x) {
    c2<R> o[4];
    hw_site<R>(rin, g, i, (R)mp->diag, o);
    if (n > 0) {
      load_sp<R>(tp, g.V, i, q);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) o[k2] = c2<R>{o[k2].x + beta * q[k2].x, o[k2].y + beta * q[k2].y};
    }
    store_sp_nt<R>(tn, g.V, i, o);
    acc += norm2_sp(o);
  }
  const double tot = block_sum(acc, lds);
  if (threadIdx.x == 0) S.part_a[lb] = tot;
  return i1 - i0;
}

template <class R, int ZM, bool CF>
__device__ __forceinline__ int ms_r_block(const SysDev& S, int lb, int n, const MsParams* mp,
                                          double* lds, c2<R>* sh) {
  const int lane = threadIdx.x & 63;
  const Geo g = S.g;
  const int nblk = S.nblk;
  const int act_sys = S.active ? *S.active : 1;
  const int done = S.h_ctl[0];
  double pg = 0.0;
  for (int j = lane; j < nblk; j += 64) pg += ldg(S.part_a, j);
  const double rho = S.h_rho[n];
  const size_t slot = (size_t)4 * g.V;
  const c2<R>* tn = (const c2<R>*)S.basis + (size_t)n * slot;
  const c2<R>* rin = (const c2<R>*)(n == 0 ? S.src : S.r);
  c2<R>* rout = (c2<R>*)S.r;
  const int i0 = ZM ? zm_first_site<R>(S, lb) : lb * S.spb;
  const int i1 = min(g.V, i0 + S.spb);
  int i = i0 + threadIdx.x;
  constexpr bool zm = ZM > 0;
  const bool have = !zm && i < i1;
  Nbr<R> nb;
  c2<R> r[4];
  ZmMarch<R, ZM == 2> zmm;
  if (CF && (!act_sys || done)) return 0;
  if (zm) zmm.begin(tn, rin, g, i0);
  if (have) {
    load_nbr<R>(tn, g, i, nb);
    load_sp<R>(rin, g.V, i, r);
  }
  if (!act_sys || done) return 0;
  const double gam = wave_sum_all(pg);
  const double alpha_d = rho / gam;
  const int stop = !(gam > 0.0) || !isfinite(alpha_d);
  if (lb == 0 && threadIdx.x == 0) {
    S.h_alpha[n] = alpha_d;
    if (stop) {
      S.h_ctl[1] = n;
      S.h_ctl[2] = 1;
      __hip_atomic_store(&S.h_ctl[0], n + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (stop) return 0;
  const R alpha = (R)alpha_d;
  double acc = 0.0;
  if (zm) {
    acc = zmm.run(mp->zm, g, (R)mp->diag, sh, [&](int ii, c2<R>* w, const c2<R>* r0) -> double {
      c2<R> rr[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) rr[k] = r0[k];
#pragma unroll
      for (int k = 0; k < 4; ++k) rr[k] = c2<R>{rr[k].x - alpha * w[k].x, rr[k].y - alpha * w[k].y};
      store_sp_nt<R>(rout, g.V, ii, rr);
      return norm2_sp(rr);
    });
    i = i1;
  }
  if (have) {
    c2<R> w[4];
    hw_compute<R>(nb, g, i, (R)mp->diag, w);
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = c2<R>{r[k].x - alpha * w[k].x, r[k].y - alpha * w[k].y};
    store_sp_nt<R>(rout, g.V, i, r);
    acc = norm2_sp(r);
  }
  for (i += blockDim.x; !zm && i < i1; i += blockDim.x) {
    c2<R> w[4];
    hw_site<R>(tn, g, i, (R)mp->diag, w);
    load_sp<R>(rin, g.V, i, r);
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = c2<R>{r[k].x - alpha * w[k].x, r[k].y - alpha * w[k].y};
    store_sp_nt<R>(rout, g.V, i, r);
    acc += norm2_sp(r);
  }
  const double tot = block_sum(acc, lds);
  if (threadIdx.x == 0) S.part_b[lb] = tot;
  return i1 - i0;
}

// Kernel-duration sampling: once every wave of the workgroup is done, thread 0 stores
// the workgroup's start and end wall-clock stamps and the sites it processed (0 for a
// system that sat the launch out) in its own three words (vector stores, no atomics); the
// host takes max(end) - min(start) over the workgroups and counts the processed sites' bytes.
__device__ __forceinline__ void stamp_block(unsigned long long* ts, unsigned long long t0,
                                            int sites) {
  __syncthreads();
  if (threadIdx.x == 0) {
    ts[3 * blockIdx.x] = t0;
    ts[3 * blockIdx.x + 1] = wall_clock64();
    ts[3 * blockIdx.x + 2] = (unsigned long long)(sites > 0 ? sites : 0);
  }
}

// Iteration n, t pass: finishes rho_n = |r_n|^2 from the previous kernel's
// partials, advances the shift recurrences, decides convergence, then
//   t_n = H r_n + beta_{n-1} t_{n-1}  -> basis slot n,  partial |t_n|^2.
// Latency layout: every independent load (control word, partials, scalar
// history, the nine stencil operands and t_{n-1}) is issued before any of them
// is consumed, and each wave finishes the reduction and the shift recurrences
// on its own (identical bits in every wave), so the only barrier is the final
// block reduction.
template <class R, int ZM, bool CF>
__global__ void __launch_bounds__(256) k_ms_t(const SysDev* __restrict__ sys,
                                              const int* __restrict__ bmap, int nb_total, int n,
                                              const MsParams mp_) {
  __shared__ double lds[17];
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  unsigned long long t0 = 0;
  if (mp_.tstamp && threadIdx.x == 0) t0 = wall_clock64();
  const int L = xcd_logical_block(nb_total);
  const SysDev& S = sys[bmap[L]];
  const int sites = ms_t_block<R, ZM, CF>(S, L - S.blk0, n, &mp_, lds, ZM ? (c2<R>*)dyn_lds : nullptr);
  if (mp_.tstamp) stamp_block(mp_.tstamp, t0, sites);
}

// Iteration n, r pass:
//   alpha_n = rho_n / |t_n|^2;  r_{n+1} = r_n - alpha_n H t_n;  partial |r_{n+1}|^2.
template <class R, int ZM, bool CF>
__global__ void __launch_bounds__(256) k_ms_r(const SysDev* __restrict__ sys,
                                              const int* __restrict__ bmap, int nb_total, int n,
                                              const MsParams mp_) {
  __shared__ double lds[17];
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  unsigned long long t0 = 0;
  if (mp_.tstamp && threadIdx.x == 0) t0 = wall_clock64();
  const int L = xcd_logical_block(nb_total);
  const SysDev& S = sys[bmap[L]];
  const int sites = ms_r_block<R, ZM, CF>(S, L - S.blk0, n, &mp_, lds, ZM ? (c2<R>*)dyn_lds : nullptr);
  if (mp_.tstamp) stamp_block(mp_.tstamp, t0, sites);
}

// ------------------------------------------------ multi-shift: persistent form
// All iterations of one multi-shift solve in a single cooperative launch: the
// t and r passes are separated by grid barriers instead of kernel boundaries.
// Every spin is bounded: a barrier that does not complete within the limit
// raises `abort` and every workgroup leaves, so the launch always drains.
struct GridBar {
  unsigned int count;  // arrivals in the current barrier
  unsigned int gen;    // barrier generation
  int abort;           // set by a workgroup whose wait timed out
  int pad;
};

constexpr long long kSpinLimit = 1LL << 20;

// Grid barrier.  Each wave first waits for its own stores to complete, the
// workgroup meets, then one thread per workgroup publishes the workgroup's
// writes device-wide (agent-scope release: L2 write-back), arrives with a
// relaxed atomic, polls the generation with relaxed atomic loads (no cache
// invalidation per poll) and finally acquires once (agent-scope invalidate).
__device__ __forceinline__ bool grid_sync(GridBar* gb, unsigned int nblocks) {
  __shared__ int sh_ok;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned int g0 = __hip_atomic_load(&gb->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned int arrived =
        __hip_atomic_fetch_add(&gb->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&gb->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(&gb->gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long long spins = 0;
      while (__hip_atomic_load(&gb->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit ||
            __hip_atomic_load(&gb->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          ok = 0;
          break;
        }
      }
      if (!ok) __hip_atomic_store(&gb->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    sh_ok = ok;
  }
  __syncthreads();
  return sh_ok != 0;
}

// True when every participating system finished at an iteration <= n.  A
// system that finishes at n' writes n' + 1 in one word, so a workgroup that
// runs ahead into iteration n + 1 can never change this answer for iteration n.
__device__ __forceinline__ bool all_done(const SysDev* __restrict__ sys, int nsys, int n) {
  for (int s = 0; s < nsys; ++s) {
    const SysDev& S = sys[s];
    if (S.active && *S.active == 0) continue;
    const int d = __hip_atomic_load(&S.h_ctl[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (d == 0 || d - 1 > n) return false;
  }
  return true;
}

// Launch with exactly `grid` co-resident workgroups (cooperative launch).
// Workgroup b handles logical blocks j, j + grid, ... with j its XCD-contiguous
// index.  Every workgroup runs the same barriers and leaves at the same
// iteration (after L iterations, or once all_done holds after a barrier).
template <class R>
__global__ void __launch_bounds__(256) k_ms_persistent(const SysDev* __restrict__ sys, int nsys,
                                                       const int* __restrict__ bmap, int nb_total,
                                                       int L, const MsParams mp_, GridBar* gb) {
  __shared__ double lds[17];
  const int grid = gridDim.x;
  const int j0 = xcd_logical_block(grid);
  for (int n = 0; n < L; ++n) {
    for (int Lb = j0; Lb < nb_total; Lb += grid) {
      const SysDev& S = sys[bmap[Lb]];
      ms_t_block<R, 0, false>(S, Lb - S.blk0, n, &mp_, lds, (c2<R>*)nullptr);
      __syncthreads();
    }
    if (!grid_sync(gb, grid)) return;
    for (int Lb = j0; Lb < nb_total; Lb += grid) {
      const SysDev& S = sys[bmap[Lb]];
      ms_r_block<R, 0, false>(S, Lb - S.blk0, n, &mp_, lds, (c2<R>*)nullptr);
      __syncthreads();
    }
    if (!grid_sync(gb, grid)) return;
    if (all_done(sys, nsys, n)) return;
  }
}

__global__ void k_bar_reset(GridBar* gb) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    gb->count = 0;
    gb->abort = 0;
  }
}

// ------------------------------------------------- multi-shift: coefficients
// One workgroup per system.  Shift k ran N_k iterations (first n with its bit
// clear in h_active).  With z^j = zeta_k^j, alpha_{j,k} = alpha_j z^{j+1}/z^j,
// beta_{j,k} = beta_j (z^{j+1}/z^j)^2 and p_k^j = sum_{i<=j} z^i prod beta_{.,k} r_i:
//   y_k = sum_j z^j S_k^j r_j,  S_k^j = alpha_{j,k} + beta_{j,k} S_k^{j+1},  S_k^{N_k} = 0,
//   acc = sum_j c_j r_j,  c_j = sum_k a_k z^j S_k^j,
//   eps = H acc = sum_j d_j t_j,  d_j = c_j - beta_j c_{j+1}   (H r_j = t_j - beta_{j-1} t_{j-1}).
constexpr int COEF_LDS_ITERS = 160;  // history rows staged in LDS (larger N reads global)

// LDS of k_ms_coef.  The staged path works on these arrays only (no pointer that may
// point to either LDS or global memory: such accesses compile to flat instructions, and
// each of them waits for every global store in flight).
struct CoefLds {
  int N;
  int nk[MAXP];
  double res[MAXP];
  double rho[COEF_LDS_ITERS + 1], alpha[COEF_LDS_ITERS + 1], c[COEF_LDS_ITERS + 1];
  unsigned int act[COEF_LDS_ITERS + 1];
  double zeta[(COEF_LDS_ITERS + 1) * MAXP];
  double u[MAXP][COEF_LDS_ITERS + 1];   // recurrence factors, then the terms (k, j)
  double cp[MAXP][COEF_LDS_ITERS + 1];
  double g[COEF_LDS_ITERS + 1], td[COEF_LDS_ITERS + 1], to[COEF_LDS_ITERS + 1];
};

// Second function of the same Krylov space (entries with coef_d2 set):
//   w = H r(A)^2 psi = sum_j d2_j t_j,   so that eps^2 psi = A r(A)^2 psi = H w.
// The CG scalars give the Lanczos tridiagonal of A on v_j = (-1)^j r_j / |r_j|:
//   T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},  T_j,j+1 = sqrt(beta_j)/alpha_j,
// and r(A)^2 psi ~ |psi| V r(T)^2 e_1 with r(T)^2 e_1 = sum_l a_l (T + b_l)^-1 g,
// g = sum_k a_k (T + b_k)^-1 e_1: 2 np tridiagonal solves (T + b is positive definite,
// elimination without pivoting is stable), one thread per shift.  Coefficients on r_j:
// c2_j = |psi| (-1)^j h_j / |r_j|; on t_j: d2_j = c2_j - beta_j c2_{j+1}.
// Work arrays U, CP ([MAXP][ld]), G, TD, TO ([N]) all in LDS or all in global memory.
__device__ __forceinline__ void coef_second(const SysDev& S, const MsParams* mp, int N,
                                            const double* rho, const double* alph, double* U,
                                            double* CP, double* G, double* TD, double* TO,
                                            int ld) {
  const int np = mp->np;
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    TD[j] = 1.0 / alph[j] + (j > 0 ? (rho[j] / rho[j - 1]) / alph[j - 1] : 0.0);
    TO[j] = sqrt(rho[j + 1] / rho[j]) / alph[j];
  }
  __syncthreads();
  auto solve = [&](int k, bool from_g) {
    double* u = U + (size_t)k * ld;
    double* cp = CP + (size_t)k * ld;
    const double bk = mp->sigma[k];
    // forward elimination; the next row's operands are read ahead of the division
    double cprev = 0.0, dprev = 0.0, ol = 0.0;
    double td = TD[0], rhs = from_g ? G[0] : 1.0;
    for (int j = 0; j < N; ++j) {
      const double to = TO[j];
      double td_n = 0.0, rhs_n = 0.0;
      if (j + 1 < N) {
        td_n = TD[j + 1];
        rhs_n = from_g ? G[j + 1] : 0.0;
      }
      const double inv = 1.0 / (td + bk - ol * cprev);
      const double cj = j + 1 < N ? to * inv : 0.0;
      const double dj = (rhs - ol * dprev) * inv;
      cp[j] = cj;
      u[j] = dj;
      cprev = cj;
      dprev = dj;
      ol = to;
      td = td_n;
      rhs = rhs_n;
    }
    double un = dprev;
    for (int j = N - 2; j >= 0; --j) {
      un = u[j] - cp[j] * un;
      u[j] = un;
    }
  };
  if (threadIdx.x < np) solve(threadIdx.x, false);
  __syncthreads();
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    double g = 0.0;
    for (int k = 0; k < np; ++k) g += mp->coef[k] * U[(size_t)k * ld + j];
    G[j] = g;
  }
  __syncthreads();
  if (threadIdx.x < np) solve(threadIdx.x, true);
  __syncthreads();
  const double sr0 = sqrt(rho[0]);
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    double h = 0.0;
    for (int k = 0; k < np; ++k) h += mp->coef[k] * U[(size_t)k * ld + j];
    G[j] = sr0 * ((j & 1) ? -h : h) / sqrt(rho[j]);  // c2_j
  }
  __syncthreads();
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    const double cn = (j + 1 < N) ? G[j + 1] : 0.0;
    S.coef_d2[j] = G[j] - (rho[j + 1] / rho[j]) * cn;
  }
}

__global__ void __launch_bounds__(256) k_ms_coef(const SysDev* __restrict__ sys, int nsys,
                                                 int launched, const MsParams mp_) {
  __shared__ CoefLds L;
  const int s = blockIdx.x;
  if (s >= nsys) return;
  const SysDev& S = sys[s];
  if (S.active && *S.active == 0) return;
  const MsParams* mp = &mp_;
  const int np = mp->np;
  const int cap = mp->cap;
  if (threadIdx.x == 0) {
    int N;
    if (S.h_ctl[0]) {
      N = S.h_ctl[1];
      if (S.h_ctl[2]) S.h_ctl[3] |= 1 << S.h_ctl[2];
    } else {  // not finished within the launched iterations: use what exists
      N = launched > 0 ? launched - 1 : 0;
      S.h_ctl[1] = N;
      S.h_ctl[3] |= 1 << 2;
    }
    L.N = N;
  }
  for (int k = threadIdx.x; k < MAXP; k += blockDim.x) L.res[k] = 0.0;
  __syncthreads();
  const int N = L.N;
  if (N <= COEF_LDS_ITERS) {
    // stage rows 0..N of the history (coalesced)
    for (int j = threadIdx.x; j <= N; j += blockDim.x) {
      L.rho[j] = S.h_rho[j];
      L.alpha[j] = S.h_alpha[j];
      L.act[j] = S.h_active[j];
    }
    for (int q = threadIdx.x; q < (N + 1) * MAXP; q += blockDim.x) L.zeta[q] = S.h_zeta[q];
    __syncthreads();
    // N_k, the first iteration with shift k inactive: one wave per shift, a ballot per
    // 64 iterations
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int k = threadIdx.x >> 6; k < np; k += nw) {
      int nk = N;
      for (int j0 = 0; j0 < N; j0 += 64) {
        const int j = j0 + lane;
        const unsigned long long m = __ballot(j < N && !(L.act[j] & (1u << k)));
        if (m) {
          nk = j0 + __ffsll((long long)m) - 1;
          break;
        }
      }
      if (lane == 0) L.nk[k] = nk;
    }
    // the recurrence factors alpha_{j,k}, beta_{j,k} for every (k, j) at once; the
    // per-shift chains below are then multiply-adds on LDS operands
    for (int q = threadIdx.x; q < np * N; q += blockDim.x) {
      const int k = q / N, j = q - k * N;
      const double zj = L.zeta[j * MAXP + k];
      const double zr = L.zeta[(j + 1) * MAXP + k] / zj;
      L.u[k][j] = L.alpha[j] * zr;
      L.cp[k][j] = (L.rho[j + 1] / L.rho[j]) * zr * zr;
    }
    __syncthreads();
    const double rho0 = L.rho[0];
    for (int k = threadIdx.x; k < np; k += blockDim.x) {
      const int Nk = L.nk[k];
      double Sk = 0.0;
      for (int j = Nk - 1; j >= 0; --j) {
        Sk = L.u[k][j] + L.cp[k][j] * Sk;
        L.u[k][j] = mp->coef[k] * L.zeta[j * MAXP + k] * Sk;  // term (k, j)
      }
      for (int j = Nk; j < N; ++j) L.u[k][j] = 0.0;
      if (rho0 > 0.0) L.res[k] = fabs(L.zeta[Nk * MAXP + k]) * sqrt(L.rho[Nk] / rho0);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
      double c = 0.0;
      for (int k = 0; k < np; ++k) c += L.u[k][j];
      L.c[j] = c;
      S.coef_c[j] = c;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
      const double cn = (j + 1 < N) ? L.c[j + 1] : 0.0;
      S.coef_d[j] = L.c[j] - (L.rho[j + 1] / L.rho[j]) * cn;
    }
    if (S.coef_d2 && N > 0)
      coef_second(S, mp, N, L.rho, L.alpha, &L.u[0][0], &L.cp[0][0], L.g, L.td, L.to,
                  COEF_LDS_ITERS + 1);
  } else {
    // long histories read global memory (terms through the entry's coef_term)
    const double* rho = S.h_rho;
    const double* alph = S.h_alpha;
    const double* zeta = S.h_zeta;
    const double rho0 = rho[0];
    for (int k = threadIdx.x; k < np; k += blockDim.x) {
      int Nk = N;
      for (int j = 0; j < N; ++j)
        if (!(S.h_active[j] & (1u << k))) { Nk = j; break; }
      double Sk = 0.0;
      for (int j = Nk - 1; j >= 0; --j) {
        const double zj = zeta[(size_t)j * MAXP + k];
        const double zr = zeta[(size_t)(j + 1) * MAXP + k] / zj;
        const double aj = alph[j] * zr;
        const double bj = (rho[j + 1] / rho[j]) * zr * zr;
        Sk = aj + bj * Sk;
        S.coef_term[(size_t)k * cap + j] = mp->coef[k] * zj * Sk;
      }
      for (int j = Nk; j < N; ++j) S.coef_term[(size_t)k * cap + j] = 0.0;
      if (rho0 > 0.0) L.res[k] = fabs(zeta[(size_t)Nk * MAXP + k]) * sqrt(rho[Nk] / rho0);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
      double c = 0.0;
      for (int k = 0; k < np; ++k) c += S.coef_term[(size_t)k * cap + j];
      S.coef_c[j] = c;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
      const double cn = (j + 1 < N) ? S.coef_c[j + 1] : 0.0;
      S.coef_d[j] = S.coef_c[j] - (rho[j + 1] / rho[j]) * cn;
    }
    if (S.coef_d2 && N > 0) {
      __syncthreads();  // the terms are consumed: coef_term becomes TO
      coef_second(S, mp, N, rho, alph, S.coef_sq, S.coef_sq + (size_t)MAXP * cap,
                  S.coef_sq + (size_t)2 * MAXP * cap, S.coef_sq + (size_t)2 * MAXP * cap + cap,
                  S.coef_term, cap);
    }
  }
  if (threadIdx.x == 0) {  // statistics, off the critical path
    double mx = 0.0;
    for (int k = 0; k < np; ++k) mx = fmax(mx, L.res[k]);
    S.dstat[0] = mx;
    S.stat[0] += N;
    S.stat[1] += 1;
    if (N > S.stat[2]) S.stat[2] = N;
    if (N > S.stat[3]) S.stat[3] = N;  // max N since the host last cleared it
  }
}

// ---------------------------------------------- combination + epilogues
enum EpiMode {
  EPI_SIGN = 0,     // out = eps
  EPI_DOV = 1,      // out = psi + g5 eps
  EPI_DOVDAG = 2,   // out = psi + eps            (multi-shift source was g5 psi)
  EPI_M = 3,        // out = psi + g5 eps + Y psi;   out2 = g5 out;  partial |out|^2
  EPI_MDAG = 4,     // out = psi + eps + Y^dag psi
  EPI_MDAG_CG = 5,  // q = psi + eps + Y^dag psi;  x += alpha p;  r -= alpha q;  partial |r|^2
  EPI_MDAG_RES = 6  // r64 = b - (psi + eps + Y^dag psi) (+ low-precision copy in cg_r); partial |r64|^2
};

// c+ = m + g phi, c- = m* + g* phi*;  Y psi = c- psi_{0,1} (P-) + c+ psi_{2,3} (P+).
template <class R>
__global__ void __launch_bounds__(256) k_ms_combine(const SysDev* __restrict__ sys, const int* __restrict__ bmap,
                                                     int nb_total, int mode) {
  __shared__ double lds[17];
  const int L = xcd_logical_block(nb_total);
  const int s = bmap[L];
  const SysDev& S = sys[s];
  if (S.active && *S.active == 0) return;
  const int lb = L - S.blk0;
  const Geo g = S.g;
  const int V = g.V;
  const size_t slot = (size_t)4 * V;
  const int N = S.h_ctl[1];
  const double* __restrict__ d = S.coef_d;
  const c2<R>* basis = (const c2<R>*)S.basis;
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  double alpha = 0.0;
  if (mode == EPI_MDAG_CG) alpha = S.cg_s[CG_ALPHA];
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double2 e[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) e[k] = double2{0.0, 0.0};
    int j = 0;
    for (; j + 1 < N; j += 2) {
      const double d0 = d[j], d1 = d[j + 1];
      const c2<R>* b0 = basis + (size_t)j * slot;
      const c2<R>* b1 = b0 + slot;
      c2<R> v0[4], v1[4];
      load_sp<R>(b0, V, i, v0);
      load_sp<R>(b1, V, i, v1);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        e[k].x += d0 * (double)v0[k].x + d1 * (double)v1[k].x;
        e[k].y += d0 * (double)v0[k].y + d1 * (double)v1[k].y;
      }
    }
    if (j < N) {
      const double d0 = d[j];
      c2<R> v0[4];
      load_sp<R>(basis + (size_t)j * slot, V, i, v0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        e[k].x += d0 * (double)v0[k].x;
        e[k].y += d0 * (double)v0[k].y;
      }
    }
    if (mode == EPI_SIGN) {
      c2<R> o[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) o[k] = c2<R>{(R)e[k].x, (R)e[k].y};
      store_sp<R>((c2<R>*)S.e_out, V, i, o);
      continue;
    }
    c2<R> p[4];
    load_sp<R>((const c2<R>*)S.e_in, V, i, p);
    double2 o[4];
    if (mode == EPI_DOV || mode == EPI_M) {
      o[0] = double2{(double)p[0].x - e[0].x, (double)p[0].y - e[0].y};
      o[1] = double2{(double)p[1].x - e[1].x, (double)p[1].y - e[1].y};
      o[2] = double2{(double)p[2].x + e[2].x, (double)p[2].y + e[2].y};
      o[3] = double2{(double)p[3].x + e[3].x, (double)p[3].y + e[3].y};
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) o[k] = double2{(double)p[k].x + e[k].x, (double)p[k].y + e[k].y};
    }
    if (mode >= EPI_M) {
      const double2 ph = S.phi[i];
      // c+ = m + g phi ; c- = conj(m) + conj(g) conj(phi)
      double cpr = S.m_re + S.g_re * ph.x - S.g_im * ph.y;
      double cpi = S.m_im + S.g_re * ph.y + S.g_im * ph.x;
      double cmr = S.m_re + S.g_re * ph.x - S.g_im * ph.y;
      double cmi = -S.m_im - (S.g_re * ph.y + S.g_im * ph.x);
      if (mode != EPI_M) { cpi = -cpi; cmi = -cmi; }  // adjoint: conjugate coefficients
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double cr = (k < 2) ? cmr : cpr, ci = (k < 2) ? cmi : cpi;
        const double pr = (double)p[k].x, pi = (double)p[k].y;
        o[k].x += cr * pr - ci * pi;
        o[k].y += cr * pi + ci * pr;
      }
    }
    if (mode == EPI_MDAG_CG) {
      // x += alpha p ; r -= alpha q
      c2<R> xv[4], pv[4], rv[4];
      load_sp<R>((const c2<R>*)S.cg_x, V, i, xv);
      load_sp<R>((const c2<R>*)S.cg_p, V, i, pv);
      load_sp<R>((const c2<R>*)S.cg_r, V, i, rv);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        xv[k] = c2<R>{(R)((double)xv[k].x + alpha * (double)pv[k].x),
                      (R)((double)xv[k].y + alpha * (double)pv[k].y)};
        rv[k] = c2<R>{(R)((double)rv[k].x - alpha * o[k].x), (R)((double)rv[k].y - alpha * o[k].y)};
      }
      store_sp<R>((c2<R>*)S.cg_x, V, i, xv);
      store_sp<R>((c2<R>*)S.cg_r, V, i, rv);
      acc += norm2_sp(rv);
      continue;
    }
    if (mode == EPI_MDAG_RES) {
      double2 rr[4];
      const double2* b = S.cg_b;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double2 bv = b[(size_t)i * 4 + k];
        rr[k] = double2{bv.x - o[k].x, bv.y - o[k].y};
      }
      store_sp<double>((double2*)S.cg_r64, V, i, rr);
      if (S.cg_r) {
        c2<R> lo[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) lo[k] = c2<R>{(R)rr[k].x, (R)rr[k].y};
        store_sp<R>((c2<R>*)S.cg_r, V, i, lo);
      }
      acc += norm2_sp(rr);
      continue;
    }
    c2<R> ov[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) ov[k] = c2<R>{(R)o[k].x, (R)o[k].y};
    store_sp<R>((c2<R>*)S.e_out, V, i, ov);
    if (mode == EPI_M) {
      acc += norm2_sp(ov);
      if (S.e_out2) {
        c2<R> g5o[4] = {c2<R>{-ov[0].x, -ov[0].y}, c2<R>{-ov[1].x, -ov[1].y}, ov[2], ov[3]};
        store_sp<R>((c2<R>*)S.e_out2, V, i, g5o);
      }
    }
  }
  if (mode == EPI_M || mode == EPI_MDAG_CG || mode == EPI_MDAG_RES) {
    const double tot = block_sum(acc, lds);
    if (threadIdx.x == 0) {
      if (S.part_c) S.part_c[lb] = tot;
      if (mode == EPI_M && S.part_b) S.part_b[lb] = tot;  // rho_0 of the next multi-shift
    }
  }
}

// ------------------------------------------------------- multi-shift setup
// Source partials |src|^2 -> part_b (and src = g5 e_in when g5_src).
template <class R>
__global__ void __launch_bounds__(256) k_ms_prep(const SysDev* __restrict__ sys, const int* __restrict__ bmap,
                                                  int nb_total, int g5_src) {
  __shared__ double lds[17];
  const int L = xcd_logical_block(nb_total);
  const int s = bmap[L];
  const SysDev& S = sys[s];
  if (S.active && *S.active == 0) return;
  const int lb = L - S.blk0;
  const int V = S.g.V;
  // optional: src = g5 * e_in  (writes the multi-shift source buffer)
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    c2<R> v[4];
    if (g5_src) {
      load_sp<R>((const c2<R>*)S.e_in, V, i, v);
      v[0] = c2<R>{-v[0].x, -v[0].y};
      v[1] = c2<R>{-v[1].x, -v[1].y};
      store_sp<R>((c2<R>*)S.src, V, i, v);
    } else {
      load_sp<R>((const c2<R>*)S.src, V, i, v);
    }
    acc += norm2_sp(v);
  }
  const double tot = block_sum(acc, lds);
  if (threadIdx.x == 0) S.part_b[lb] = tot;
}

// Deterministic synthetic field for tuning runs: a hash of the site and spin
// mapped to [-1, 1) in both components, written to src.
template <class R>
__global__ void __launch_bounds__(256) k_fill(const SysDev* __restrict__ sys,
                                              const int* __restrict__ bmap, int nb_total) {
  const int L = xcd_logical_block(nb_total);
  const SysDev& S = sys[bmap[L]];
  const int lb = L - S.blk0;
  const int V = S.g.V;
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  c2<R>* out = (c2<R>*)S.src;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      unsigned int h = (unsigned int)(i * 4 + k) * 2654435761u + 0x9e3779b9u;
      h ^= h >> 15; h *= 2246822519u; h ^= h >> 13;
      const unsigned int h2 = h * 3266489917u + 374761393u;
      out[(size_t)k * V + i] = c2<R>{(R)((double)(h & 0xffffff) / 8388608.0 - 1.0),
                                     (R)((double)(h2 & 0xffffff) / 8388608.0 - 1.0)};
    }
  }
}

// ------------------------------------------------- momentum-space operators
// The theory has no gauge field, so every translation-invariant operator built
// from H_W is diagonal in momentum space (the FFT route of Sec. 7.2).  For a
// field ~ exp(+i p.x), D_W(p) = w + i gamma.s with w = 4 - M0 - sum cos p_mu,
// s_mu = sin p_mu, H_W(p)^2 = s2 = w^2 + |s|^2.  Every Dirac operator form is
//   D(p) = a0 + i c gamma.s :
//   overlap, rational sign R = sum_k a_k / (s2 + b_k):  a0 = 1 + R w, c = R;
//   overlap, exact sign R = 1 / sqrt(s2):                a0 = 1 + R w, c = R;
//   Dslash = (1 - D_ov/2)^-1 D_ov (exact sign, Sec. 2.2): a0 = 0,
//     c = 2 / (sqrt(s2) - w) = 2 (sqrt(s2) + w) / |s|^2  (finite when no momentum
//     has every component in {0, pi}: antiperiodic time, T even).
// The free fermion matrix of the preconditioner (Sec. 7.3),
//   M0 = D + m P+ + m* P- = a + i mu g5 + i c gamma.s,  a = a0 + Re m, mu = Im m,
// has M0^-1 = (a - i mu g5 - i c gamma.s) / (a^2 + mu^2 + c^2 |s|^2), and M0^-dag
// the same with + signs.
// Fields go through per-axis DFTs of L <= 64 points: forward e^{-2 pi i j k/L},
// inverse e^{+2 pi i j k/L} with 1/V.  Antiperiodic time is handled by the
// twist e^{-i pi t/T} before the forward and e^{+i pi t/T} after the inverse
// transform, which puts p_t on (2n+1) pi / T.
// SYM_PCG: the scalar (M0^dag M0)^-1 = M0^-1 M0^-dag of the free-field operator, the
// preconditioner of CG on MdagM (Sec. 7.3 in its split form; same iterates).
enum SymKind { SYM_D = 0, SYM_D_DAG = 1, SYM_M0INV = 2, SYM_M0INV_DAG = 3, SYM_BOSON = 4,
               SYM_PCG = 5 };
enum DiracForm { DIRAC_RATIONAL = 0, DIRAC_EXACT = 1, DIRAC_DSLASH = 2 };

struct SymParams {
  int kind;
  int form;           // DiracForm
  int periodic;       // 1: periodic time (scalar fields) whatever the fermion boundary
  int np;
  double diag;        // 4 - M0
  double a[MAXP];     // residues a_k of the sign rational
  double b[MAXP];     // shifts b_k
};

// System of workgroup b in a transform pass (which: 0 xy, 1 z, 2 t).
__device__ __forceinline__ int find_sys(const SysDev* __restrict__ sys, int nsys, int b, int which) {
  int s = 0;
  for (int k = 1; k < nsys; ++k) {
    const int o = which == 0 ? sys[k].off_xy : (which == 1 ? sys[k].off_z : sys[k].off_t);
    if (o <= b) s = k;
  }
  return s;
}

// Twiddle table e^{sgn 2 pi i j / L}, evaluated in FP64 and stored in the transform's
// precision (an FP32 transform reads 8-byte entries from LDS).
template <class R>
__device__ __forceinline__ void twiddles(c2<R>* tw, int L, double sgn) {
  for (int j = threadIdx.x; j < L; j += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)j / (double)L, &sn, &cs);
    tw[j] = c2<R>{(R)cs, (R)(sgn * sn)};
  }
}

template <class R>
__device__ __forceinline__ c2<R> cmad(c2<R> acc, c2<R> a, c2<R> w) {
  return c2<R>{acc.x + a.x * w.x - a.y * w.y, acc.y + a.x * w.y + a.y * w.x};
}

// x and y axes of one (z, t, spin) plane.  inv = 0: e_in -> fft_tmp with the
// time twist; inv = 1: fft_tmp -> e_out with the untwist and 1/V.  Needs
// X, Y <= 64 and X Y <= 1024.
template <class R>
__global__ void __launch_bounds__(256) k_fft_xy(const SysDev* __restrict__ sys, int nsys, int inv,
                                                int periodic) {
  __shared__ c2<R> A[1024], B[1024];
  __shared__ c2<R> twx[64], twy[64];
  const SysDev& S = sys[find_sys(sys, nsys, blockIdx.x, 0)];
  if (S.active && *S.active == 0) return;
  const int X = S.g.X, Y = S.g.Y, Z = S.g.Z, T = S.g.T, V = S.g.V;
  const int loc = blockIdx.x - S.off_xy;
  const int spin = loc & 3;
  const int zt = loc >> 2;  // z + Z t
  const int t = zt / Z;
  const int XY = X * Y;
  const c2<R>* in = (const c2<R>*)(inv ? S.fft_tmp : S.e_in) + (size_t)spin * V + (size_t)zt * XY;
  c2<R>* out = (c2<R>*)(inv ? S.e_out : S.fft_tmp) + (size_t)spin * V + (size_t)zt * XY;
  const double sgn = inv ? 1.0 : -1.0;
  twiddles<R>(twx, X, sgn);
  twiddles<R>(twy, Y, sgn);
  double tr = 1.0, ti = 0.0;  // twist (forward) / untwist and normalisation (inverse)
  if (S.g.bc < 0 && !periodic) sincospi(sgn * (double)t / (double)T, &ti, &tr);
  if (inv) {
    tr /= (double)V;
    ti /= (double)V;
  }
  for (int i = threadIdx.x; i < XY; i += blockDim.x) {
    const c2<R> v = in[i];
    A[i] = inv ? v : c2<R>{(R)(v.x * tr - v.y * ti), (R)(v.x * ti + v.y * tr)};
  }
  __syncthreads();
  for (int i = threadIdx.x; i < XY; i += blockDim.x) {  // x axis
    const int kx = i % X, y = i / X;
    c2<R> acc{(R)0, (R)0};
    int w = 0;
    for (int x = 0; x < X; ++x) {
      acc = cmad<R>(acc, A[y * X + x], twx[w]);
      w += kx;
      if (w >= X) w -= X;
    }
    B[i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < XY; i += blockDim.x) {  // y axis
    const int kx = i % X, ky = i / X;
    c2<R> acc{(R)0, (R)0};
    int w = 0;
    for (int y = 0; y < Y; ++y) {
      acc = cmad<R>(acc, B[y * X + kx], twy[w]);
      w += ky;
      if (w >= Y) w -= Y;
    }
    out[i] = inv ? c2<R>{(R)(acc.x * tr - acc.y * ti), (R)(acc.x * ti + acc.y * tr)} : acc;
  }
}

// z axis of the (x, z) slab of one (y, t, spin), in place on fft_tmp.
// Needs Z <= 64 and X Z <= 1024.
template <class R>
__global__ void __launch_bounds__(256) k_fft_z(const SysDev* __restrict__ sys, int nsys, int inv) {
  __shared__ c2<R> A[1024];
  __shared__ c2<R> tw[64];
  const SysDev& S = sys[find_sys(sys, nsys, blockIdx.x, 1)];
  if (S.active && *S.active == 0) return;
  const int X = S.g.X, Y = S.g.Y, Z = S.g.Z, V = S.g.V;
  const int loc = blockIdx.x - S.off_z;
  const int spin = loc & 3;
  const int yt = loc >> 2;  // y + Y t
  const int y = yt % Y, t = yt / Y;
  c2<R>* f = (c2<R>*)S.fft_tmp + (size_t)spin * V;
  twiddles<R>(tw, Z, inv ? 1.0 : -1.0);
  const int n = X * Z;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int x = e % X, z = e / X;
    A[e] = f[x + X * (y + Y * (z + Z * t))];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int x = e % X, kz = e / X;
    c2<R> acc{(R)0, (R)0};
    int w = 0;
    for (int z = 0; z < Z; ++z) {
      acc = cmad<R>(acc, A[z * X + x], tw[w]);
      w += kz;
      if (w >= Z) w -= Z;
    }
    f[x + X * (y + Y * (kz + Z * t))] = acc;  // every read of f happened before the barrier
  }
}

// Free-field Dirac operator at one momentum: D = a0 + i c gamma.s (s_mu = sin p_mu,
// w the Wilson term), for the form's sign function.
__device__ __forceinline__ void free_symbol(const SymParams& sp, double s2sin, double w,
                                            double& a0, double& c) {
  const double s2 = w * w + s2sin;
  if (sp.form == DIRAC_DSLASH) {
    const double sq = sqrt(s2);
    a0 = 0.0;
    c = (w > 0.0) ? 2.0 * (sq + w) / s2sin : 2.0 / (sq - w);
  } else {
    double Rr = 0.0;
    if (sp.form == DIRAC_EXACT) {
      Rr = 1.0 / sqrt(s2);
    } else {
      for (int k = 0; k < sp.np; ++k) Rr += sp.a[k] / (s2 + sp.b[k]);
    }
    a0 = 1.0 + Rr * w;
    c = Rr;
  }
}

// The preconditioner of CG on MdagM at one momentum: M0^dag M0 = (a^2 + mu^2 + c^2 |s|^2) 1
// is a scalar (a shifted solve takes the free shifted operator, M0^dag M0 + sigma), so
// P = (M0^dag M0 + sigma)^-1 is one number per momentum.
__device__ __forceinline__ double pcg_scale(const SymParams& sp, double m_re, double m_im,
                                            double shift, double s2sin, double w) {
  double a0, c;
  free_symbol(sp, s2sin, w, a0, c);
  const double A = a0 + m_re;
  return 1.0 / (A * A + m_im * m_im + c * c * s2sin + shift);
}

// Momentum-space operator on the four spin components v of one momentum.
__device__ __forceinline__ void apply_symbol(const SymParams& sp, double m_re, double m_im,
                                             double shift, double sx, double sy, double sz,
                                             double st, double w, double2 v[4]) {
  const double s2sin = sx * sx + sy * sy + sz * sz + st * st;
  if (sp.kind == SYM_PCG) {
    const double sc = pcg_scale(sp, m_re, m_im, shift, s2sin, w);
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = double2{v[k].x * sc, v[k].y * sc};
    return;
  }
  double a0, c;
  free_symbol(sp, s2sin, w, a0, c);
  // out = (A v + i (cg gamma.s v + c5 g5 v)) * scale
  double A = a0, cg = c, c5 = 0.0, scale = 1.0;
  if (sp.kind == SYM_D_DAG) {
    cg = -c;
  } else if (sp.kind == SYM_M0INV || sp.kind == SYM_M0INV_DAG) {
    A = a0 + m_re;
    const double sg = sp.kind == SYM_M0INV ? -1.0 : 1.0;
    cg = sg * c;
    c5 = sg * m_im;
    scale = 1.0 / (A * A + m_im * m_im + c * c * s2sin);
  }
  // G = gamma.s v in the basis of Sec. 2.1 (the one of the Wilson stencil)
  double2 G[4];
  G[0] = double2{-sx * v[3].y + sy * v[3].x - sz * v[2].y + st * v[2].x,
                 sx * v[3].x + sy * v[3].y + sz * v[2].x + st * v[2].y};
  G[1] = double2{-sx * v[2].y - sy * v[2].x + sz * v[3].y + st * v[3].x,
                 sx * v[2].x - sy * v[2].y - sz * v[3].x + st * v[3].y};
  G[2] = double2{sx * v[1].y - sy * v[1].x + sz * v[0].y + st * v[0].x,
                 -sx * v[1].x - sy * v[1].y - sz * v[0].x + st * v[0].y};
  G[3] = double2{sx * v[0].y + sy * v[0].x - sz * v[1].y + st * v[1].x,
                 -sx * v[0].x + sy * v[0].y + sz * v[1].x + st * v[1].y};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double g5 = k < 2 ? -1.0 : 1.0;
    const double hr = cg * G[k].x + c5 * g5 * v[k].x;
    const double hi = cg * G[k].y + c5 * g5 * v[k].y;
    v[k] = double2{(A * v[k].x - hi) * scale, (A * v[k].y + hr) * scale};
  }
}

// t axis forward, the momentum-space operator on all four spins, t axis
// inverse, in place on fft_tmp.  Workgroup: (chunk of xc x values, y, z);
// needs T <= 64 and xc T <= 256.
template <class R>
__global__ void __launch_bounds__(256) k_fft_t_sym(const SysDev* __restrict__ sys, int nsys,
                                                   const SymParams sp) {
  __shared__ c2<R> A[1024], B[1024];
  __shared__ c2<R> twf[64], twi[64];
  __shared__ double2 csx[64], cst[64];  // (sin, cos) of the block's x momenta and of every t momentum
  const SysDev& S = sys[find_sys(sys, nsys, blockIdx.x, 2)];
  if (S.active && *S.active == 0) return;
  const int X = S.g.X, Y = S.g.Y, Z = S.g.Z, T = S.g.T, V = S.g.V;
  const int XC = S.xc;
  const int loc = blockIdx.x - S.off_t;
  const int nxc = X / XC;
  const int xb = (loc % nxc) * XC;
  const int yz = loc / nxc;  // y + Y z
  const int y = yz % Y, z = yz / Y;
  c2<R>* f = (c2<R>*)S.fft_tmp;
  twiddles<R>(twf, T, -1.0);
  twiddles<R>(twi, T, 1.0);
  const double tshift = (S.g.bc < 0 && !sp.periodic) ? 1.0 : 0.0;
  for (int j = threadIdx.x; j < XC + T; j += blockDim.x) {
    double sn, cs;
    if (j < XC) {
      sincospi(2.0 * (double)(xb + j) / (double)X, &sn, &cs);
      csx[j] = double2{sn, cs};
    } else {
      sincospi((2.0 * (j - XC) + tshift) / (double)T, &sn, &cs);
      cst[j - XC] = double2{sn, cs};
    }
  }
  const int n = 4 * XC * T;  // element e = (spin T + t) XC + xl
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int xl = e % XC, q = e / XC;
    const int t = q % T, spin = q / T;
    A[e] = f[(size_t)spin * V + (xb + xl) + X * (y + Y * (z + Z * t))];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n; e += blockDim.x) {  // forward t
    const int xl = e % XC, q = e / XC;
    const int kt = q % T, spin = q / T;
    c2<R> acc{(R)0, (R)0};
    int w = 0;
    for (int t = 0; t < T; ++t) {
      acc = cmad<R>(acc, A[(spin * T + t) * XC + xl], twf[w]);
      w += kt;
      if (w >= T) w -= T;
    }
    B[e] = acc;
  }
  __syncthreads();
  double sy, cy, sz, cz;
  sincospi(2.0 * (double)y / (double)Y, &sy, &cy);
  sincospi(2.0 * (double)z / (double)Z, &sz, &cz);
  for (int q = threadIdx.x; q < XC * T; q += blockDim.x) {  // operator at (kx, ky, kz, kt)
    const int xl = q % XC, kt = q / XC;
    const double sx = csx[xl].x, cx = csx[xl].y, st = cst[kt].x, ct = cst[kt].y;
    const double w = sp.diag - (cx + cy + cz + ct);
    double2 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const c2<R> u = B[(k * T + kt) * XC + xl];
      v[k] = double2{(double)u.x, (double)u.y};
    }
    if (sp.kind == SYM_BOSON) {
      // scalar fields in planes 0-2: D_2 = 1 + w/s (scalar part of the exact overlap
      // operator), then 1 - D_2/2 twice; plane 3 unused
      const double d2 = 1.0 + w / sqrt(w * w + sx * sx + sy * sy + sz * sz + st * st);
      v[0] = double2{d2 * v[0].x, d2 * v[0].y};
      const double k2 = 1.0 - 0.5 * d2;
      v[1] = double2{k2 * v[1].x, k2 * v[1].y};
      v[2] = double2{k2 * v[2].x, k2 * v[2].y};
      v[3] = double2{0.0, 0.0};
    } else {
      const bool m0 = sp.kind == SYM_M0INV || sp.kind == SYM_M0INV_DAG || sp.kind == SYM_PCG;
      apply_symbol(sp, m0 ? S.pc_re : S.m_re, m0 ? S.pc_im : S.m_im, S.shift, sx, sy, sz, st, w,
                   v);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) A[(k * T + kt) * XC + xl] = c2<R>{(R)v[k].x, (R)v[k].y};
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n; e += blockDim.x) {  // inverse t
    const int xl = e % XC, q = e / XC;
    const int t = q % T, spin = q / T;
    c2<R> acc{(R)0, (R)0};
    int w = 0;
    for (int kt = 0; kt < T; ++kt) {
      acc = cmad<R>(acc, A[(spin * T + kt) * XC + xl], twi[w]);
      w += t;
      if (w >= T) w -= T;
    }
    f[(size_t)spin * V + (xb + xl) + X * (y + Y * (z + Z * t))] = acc;
  }
}

// ------------------------------------------- transforms of fixed length
// Lines of compile-time length N (N = 2^a 3^b) transformed in registers: mixed-radix
// Cooley-Tukey, decimation in time, every index a constant after unrolling, twiddles
// e^{sgn 2 pi i m / N} folded into the code from a constant table.

// cos and sin of 2 pi j / n at compile time: reduction to |r| <= pi/4 by quadrants,
// then the Taylor series (terms to r^25: below 1e-17 there).
struct CS {
  double c, s;
};
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr CS ce_cossin(long long j, long long n) {
  j %= n;
  if (j < 0) j += n;
  // quadrant q = round(4 j / n), r = 2 pi (j / n - q / 4)
  const long long q = (8 * j + n) / (2 * n);
  const double r = kTwoPi * ((double)(4 * j - q * n) / (double)(4 * n));
  const double r2 = r * r;
  double sn = r, cs = 1.0, ts = r, tc = 1.0;
  for (int k = 1; k <= 12; ++k) {
    ts *= -r2 / (double)((2 * k) * (2 * k + 1));
    tc *= -r2 / (double)((2 * k - 1) * (2 * k));
    sn += ts;
    cs += tc;
  }
  switch (q & 3) {
    case 0: return CS{cs, sn};
    case 1: return CS{-sn, cs};
    case 2: return CS{-cs, -sn};
    default: return CS{sn, -cs};
  }
}

template <int N>
struct TwTable {
  double c[N], s[N];
  constexpr TwTable() : c(), s() {
    for (int j = 0; j < N; ++j) {
      const CS v = ce_cossin(j, N);
      c[j] = v.c;
      s[j] = v.s;
    }
  }
};
template <int N>
constexpr TwTable<N> kTw{};

template <class R>
__host__ __device__ __forceinline__ c2<R> cmul(c2<R> a, R wr, R wi) {
  return c2<R>{a.x * wr - a.y * wi, a.x * wi + a.y * wr};
}

// out[k] = sum_j a[j] e^{SGN 2 pi i j k / N}, in place, natural order in and out.
template <class R, int N, int SGN>
struct LineFft {
  static_assert(N >= 1, "length");
  static constexpr int P = (N % 2 == 0) ? 2 : 3;
  static constexpr int Q = N / P;
  static_assert(N == 1 || N % P == 0, "lengths are 2^a 3^b");
  __host__ __device__ static __forceinline__ void run(c2<R> (&a)[N]) {
    if constexpr (N == 1) {
      return;
    } else {
      c2<R> sub[P][Q];
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int q = 0; q < Q; ++q) sub[p][q] = a[q * P + p];
#pragma unroll
      for (int p = 0; p < P; ++p) LineFft<R, Q, SGN>::run(sub[p]);
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        c2<R> t[P];
        t[0] = sub[0][k];
#pragma unroll
        for (int p = 1; p < P; ++p) {
          const int m = (p * k) % N;
          t[p] = cmul<R>(sub[p][k], (R)kTw<N>.c[m], (R)(SGN * kTw<N>.s[m]));
        }
        if constexpr (P == 2) {
          a[k] = c2<R>{t[0].x + t[1].x, t[0].y + t[1].y};
          a[k + Q] = c2<R>{t[0].x - t[1].x, t[0].y - t[1].y};
        } else {
          // radix 3: w3 = e^{SGN 2 pi i / 3} = -1/2 + SGN i sqrt(3)/2
          const R h = (R)0.8660254037844386467637231707529 * (R)SGN;
          const c2<R> sp{t[1].x + t[2].x, t[1].y + t[2].y};
          const c2<R> sm{t[1].x - t[2].x, t[1].y - t[2].y};
          const c2<R> m0{t[0].x - (R)0.5 * sp.x, t[0].y - (R)0.5 * sp.y};
          a[k] = c2<R>{t[0].x + sp.x, t[0].y + sp.y};
          a[k + Q] = c2<R>{m0.x - h * sm.y, m0.y + h * sm.x};
          a[k + 2 * Q] = c2<R>{m0.x + h * sm.y, m0.y - h * sm.x};
        }
      }
    }
  }
};

// Forward (inverse) transform of the x, y and z axes of one (time slice, spin) of a
// system, through LDS: e_in -> fft_tmp with the time twist (fft_tmp -> e_out with the
// untwist and 1/V).  Replaces k_fft_xy + k_fft_z for lattices whose spatial extents
// have templates.  Workgroup b of the run starting at system s0: system s0 + b / (4 T),
// spin b % 4, time slice (b / 4) % T.  LDS rows padded by one value against bank
// conflicts of the x lines.
template <class R, int NX, int NY, int NZ, int INV>
__global__ void __launch_bounds__(256) k_fft_xyz(const SysDev* __restrict__ sys, int s0,
                                                 int periodic) {
  constexpr int PX = NX + 1;
  constexpr int NV = NX * NY * NZ;
  constexpr int SGN = INV ? 1 : -1;
  __shared__ c2<R> A[PX * NY * NZ];
  const int T = sys[s0].g.T;
  const int b = blockIdx.x;
  const SysDev& S = sys[s0 + b / (4 * T)];
  if (S.active && *S.active == 0) return;
  const int spin = b & 3;
  const int t = (b >> 2) % T;
  const int V = S.g.V;
  const size_t off = (size_t)spin * V + (size_t)t * NV;
  const c2<R>* in = (const c2<R>*)(INV ? S.fft_tmp : S.e_in) + off;
  c2<R>* out = (c2<R>*)(INV ? S.e_out : S.fft_tmp) + off;
  double tr = 1.0, ti = 0.0;  // twist (forward) / untwist and normalisation (inverse)
  if (S.g.bc < 0 && !periodic) sincospi((double)SGN * (double)t / (double)T, &ti, &tr);
  if (INV) {
    tr /= (double)V;
    ti /= (double)V;
  }
  const R rr = (R)tr, ri = (R)ti;
  {
    // every load of the volume in flight before the first LDS store (256 threads)
    constexpr int NL = (NV + 255) / 256;
    c2<R> v[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int i = q * 256 + (int)threadIdx.x;
      if (i < NV) v[q] = ldg2<R>(in, i);
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int i = q * 256 + (int)threadIdx.x;
      if (i < NV) A[i % NX + PX * (i / NX)] = INV ? v[q] : cmul<R>(v[q], rr, ri);
    }
  }
  __syncthreads();
  for (int l = threadIdx.x; l < NY * NZ; l += blockDim.x) {  // x lines
    c2<R> a[NX];
#pragma unroll
    for (int x = 0; x < NX; ++x) a[x] = A[x + PX * l];
    LineFft<R, NX, SGN>::run(a);
#pragma unroll
    for (int x = 0; x < NX; ++x) A[x + PX * l] = a[x];
  }
  __syncthreads();
  for (int l = threadIdx.x; l < NX * NZ; l += blockDim.x) {  // y lines
    const int x = l % NX, z = l / NX;
    c2<R> a[NY];
#pragma unroll
    for (int y = 0; y < NY; ++y) a[y] = A[x + PX * (y + NY * z)];
    LineFft<R, NY, SGN>::run(a);
#pragma unroll
    for (int y = 0; y < NY; ++y) A[x + PX * (y + NY * z)] = a[y];
  }
  __syncthreads();
  for (int l = threadIdx.x; l < NX * NY; l += blockDim.x) {  // z lines
    c2<R> a[NZ];
#pragma unroll
    for (int z = 0; z < NZ; ++z) a[z] = A[l % NX + PX * (l / NX + NY * z)];
    LineFft<R, NZ, SGN>::run(a);
#pragma unroll
    for (int z = 0; z < NZ; ++z) A[l % NX + PX * (l / NX + NY * z)] = a[z];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NV; i += blockDim.x) {
    const c2<R> v = A[i % NX + PX * (i / NX)];
    stg2<R>(out, i, INV ? cmul<R>(v, rr, ri) : v);
  }
}

// The preconditioner's scale per momentum of every system (sites of the table's
// partition; momentum (kx, ky, kz, kt) at the site index of (x, y, z, t)), for
// k_fft_t_pcg: the same arithmetic as the SYM_PCG symbol.
__global__ void __launch_bounds__(256) k_pcg_table(const SysDev* __restrict__ sys,
                                                   const int* __restrict__ bmap, int nb_total,
                                                   const SymParams sp) {
  const int L = xcd_logical_block(nb_total);
  const SysDev& S = sys[bmap[L]];
  const int lb = L - S.blk0;
  const int X = S.g.X, Y = S.g.Y, Z = S.g.Z, T = S.g.T, V = S.g.V;
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  const double tshift = (S.g.bc < 0 && !sp.periodic) ? 1.0 : 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    int r = i;
    const int kx = r % X; r /= X;
    const int ky = r % Y; r /= Y;
    const int kz = r % Z;
    const int kt = r / Z;
    double sx, cx, sy, cy, sz, cz, st, ct;
    sincospi(2.0 * (double)kx / (double)X, &sx, &cx);
    sincospi(2.0 * (double)ky / (double)Y, &sy, &cy);
    sincospi(2.0 * (double)kz / (double)Z, &sz, &cz);
    sincospi((2.0 * kt + tshift) / (double)T, &st, &ct);
    const double w = sp.diag - (cx + cy + cz + ct);
    const double s2sin = sx * sx + sy * sy + sz * sz + st * st;
    S.pcs[i] = pcg_scale(sp, S.pc_re, S.pc_im, S.shift, s2sin, w);
  }
}

// t axis forward, the preconditioner's scale, t axis inverse, in place on fft_tmp: the
// t pass of z = P r.  P does not mix spins, so one thread owns one (site, spin) line of
// NT values in registers; a wave reads 64 consecutive sites of one time slice per load
// (coalesced), and no LDS is needed.  Workgroup (64 threads) b of the run starting at
// system s0: system s0 + b / (4 nchunk), chunk of 64 sites (b / 4) % nchunk, spin b % 4
// (the four spins of a chunk are neighbours, so they share the scale lines in L2).
template <class R, int NT>
__global__ void __launch_bounds__(64) k_fft_t_pcg(const SysDev* __restrict__ sys, int s0,
                                                  int nchunk) {
  const int b = blockIdx.x;
  const SysDev& S = sys[s0 + b / (4 * nchunk)];
  if (S.active && *S.active == 0) return;
  const int XYZ = S.g.X * S.g.Y * S.g.Z;
  const int site = ((b >> 2) % nchunk) * 64 + (int)threadIdx.x;
  if (site >= XYZ) return;
  c2<R>* f = (c2<R>*)S.fft_tmp + (size_t)(b & 3) * S.g.V + site;
  const double* sc = S.pcs + site;
  c2<R> a[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) a[t] = ldg2<R>(f, (size_t)t * XYZ);
  LineFft<R, NT, -1>::run(a);
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const double m = ldg(sc, (size_t)k * XYZ);
    a[k] = c2<R>{(R)((double)a[k].x * m), (R)((double)a[k].y * m)};
  }
  LineFft<R, NT, 1>::run(a);
#pragma unroll
  for (int t = 0; t < NT; ++t) stg2<R>(f, (size_t)t * XYZ, a[t]);
}

// Yukawa epilogue of a momentum-space D (psi = e_in, D psi already in e_out):
//   mode 0:  e_out = D psi + Y psi,           partial |e_out|^2 -> part_c, part_b
//   mode 1:  e_out = D^dag psi + Y^dag psi
//   mode 2:  r64 = b - (D^dag psi + Y^dag psi)  (+ copy in cg_r when set),
//            partial |r64|^2 -> part_c   (FP64 only)
// c+ = m + g phi, c- = m* + g* phi*;  Y psi = c- P- psi + c+ P+ psi (spins 0,1 / 2,3).
template <class R>
__global__ void __launch_bounds__(256) k_yuk(const SysDev* __restrict__ sys, const int* __restrict__ bmap,
                                              int nb_total, int mode) {
  __shared__ double lds[17];
  const int L = xcd_logical_block(nb_total);
  const SysDev& S = sys[bmap[L]];
  if (S.active && *S.active == 0) return;
  const int lb = L - S.blk0;
  const int V = S.g.V;
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    c2<R> p[4], w[4];
    load_sp<R>((const c2<R>*)S.e_in, V, i, p);
    load_sp<R>((const c2<R>*)S.e_out, V, i, w);
    const double2 ph = S.phi[i];
    double cpr = S.m_re + S.g_re * ph.x - S.g_im * ph.y;
    double cpi = S.m_im + S.g_re * ph.y + S.g_im * ph.x;
    const double cmr = cpr;
    double cmi = -cpi;
    if (mode != 0) {  // adjoint: conjugate coefficients
      cpi = -cpi;
      cmi = -cmi;
    }
    double2 o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double cr = (k < 2) ? cmr : cpr, ci = (k < 2) ? cmi : cpi;
      const double pr = (double)p[k].x, pi = (double)p[k].y;
      o[k] = double2{(double)w[k].x + cr * pr - ci * pi, (double)w[k].y + cr * pi + ci * pr};
    }
    if (S.shift != 0.0 && mode == 1) {  // (MdagM + sigma) p: p = cg_p
      c2<R> q[4];
      load_sp<R>((const c2<R>*)S.cg_p, V, i, q);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        o[k] = double2{o[k].x + S.shift * (double)q[k].x, o[k].y + S.shift * (double)q[k].y};
    }
    if (mode == 2) {
      double2 rr[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double2 bv = S.cg_b[(size_t)i * 4 + k];
        rr[k] = double2{bv.x - o[k].x, bv.y - o[k].y};
      }
      if (S.shift != 0.0) {  // (MdagM + sigma) x: x = cg_x64
        double2 x[4];
        load_sp<double>((const double2*)S.cg_x64, V, i, x);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          rr[k] = double2{rr[k].x - S.shift * x[k].x, rr[k].y - S.shift * x[k].y};
      }
      store_sp<double>((double2*)S.cg_r64, V, i, rr);
      if (S.cg_r) {
        c2<R> lo[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) lo[k] = c2<R>{(R)rr[k].x, (R)rr[k].y};
        store_sp<R>((c2<R>*)S.cg_r, V, i, lo);
      }
      acc += norm2_sp(rr);
      continue;
    }
    c2<R> ov[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) ov[k] = c2<R>{(R)o[k].x, (R)o[k].y};
    store_sp<R>((c2<R>*)S.e_out, V, i, ov);
    if (mode == 0) acc += norm2_sp(ov) + S.shift * norm2_sp(p);  // <p, (MdagM + sigma) p>
  }
  if (mode != 1) {
    const double tot = block_sum(acc, lds);
    if (threadIdx.x == 0) {
      S.part_c[lb] = tot;
      if (mode == 0 && S.part_b) S.part_b[lb] = tot;
    }
  }
}

// ------------------------------------------------ locality probe (Sec. 3.2)
// norm[i] = ||psi_i|| (psi = e_in, FP64 planar) for the sites of one system.
__global__ void __launch_bounds__(256) k_site_norm(const SysDev* __restrict__ sys,
                                                    const int* __restrict__ bmap, int nb_total,
                                                    double* __restrict__ norm) {
  const int L = xcd_logical_block(nb_total);
  const SysDev& S = sys[bmap[L]];
  const int lb = L - S.blk0;
  const int V = S.g.V;
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double2 v[4];
    load_sp<double>((const double2*)S.e_in, V, i, v);
    norm[i] = sqrt(norm2_sp(v));
  }
}

// f[r] = max norm[i] over the sites at taxi-driver distance r from the origin,
// r = sum_mu min(x_mu, L_mu - x_mu).  One workgroup per r.
__global__ void __launch_bounds__(256) k_shell_max(const Geo g, const double* __restrict__ norm,
                                                    double* __restrict__ f) {
  __shared__ double red[256];
  const int r = blockIdx.x;
  double m = 0.0;
  for (int i = threadIdx.x; i < g.V; i += blockDim.x) {
    int q = i;
    const int x = q % g.X; q /= g.X;
    const int y = q % g.Y; q /= g.Y;
    const int z = q % g.Z;
    const int t = q / g.Z;
    const int d = min(x, g.X - x) + min(y, g.Y - y) + min(z, g.Z - z) + min(t, g.T - t);
    if (d == r) m = fmax(m, norm[i]);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) f[r] = red[0];
}

// ----------------------------------------- multi-shift CG on MdagM (RHMC layers)
// (MdagM + beta_i) X_i = b for every shift on the Krylov space of the base CG
// (beta = 0), with Jegerlehner's zeta recurrences (the rational functions of
// MdagM of Sec. 7.3).  Per system the coefficient block shc holds, per shift i,
// (a_i, z_i, b_i, act_i) at 4 i: x_i += a_i p_i; p_i = z_i r + b_i p_i while
// act_i != 0; the residues alpha_i at SHC_RES + i and a0 at SHC_A0.
enum { SHC_RES = 4 * MAXP, SHC_A0 = 5 * MAXP, SHC_LEN = 5 * MAXP + 1 };

// mode 0: x_i = 0, p_i = r (cg_r, FP64).  mode 1: the update above.
__global__ void __launch_bounds__(256) k_shift(const SysDev* __restrict__ sys, const int* __restrict__ bmap,
                                                int nb_total, int mode) {
  const int L = xcd_logical_block(nb_total);
  const SysDev& S = sys[bmap[L]];
  if (S.active && *S.active == 0) return;
  const int lb = L - S.blk0;
  const int V = S.g.V;
  const size_t slot = (size_t)4 * V;
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  const double* cf = S.shc;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double2 r[4];
    load_sp<double>((const double2*)S.cg_r, V, i, r);
    for (int k = 0; k < S.nshift; ++k) {
      double2* xk = S.shx + (size_t)k * slot;
      double2* pk = S.shp + (size_t)k * slot;
      if (mode == 0) {
        double2 z[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) z[q] = double2{0.0, 0.0};
        store_sp<double>(xk, V, i, z);
        store_sp<double>(pk, V, i, r);
        continue;
      }
      if (cf[4 * k + 3] == 0.0) continue;
      const double a = cf[4 * k], zz = cf[4 * k + 1], bb = cf[4 * k + 2];
      double2 x[4], pv[4];
      load_sp<double>(xk, V, i, x);
      load_sp<double>(pk, V, i, pv);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        x[q] = double2{x[q].x + a * pv[q].x, x[q].y + a * pv[q].y};
        pv[q] = double2{zz * r[q].x + bb * pv[q].x, zz * r[q].y + bb * pv[q].y};
      }
      store_sp<double>(xk, V, i, x);
      store_sp<double>(pk, V, i, pv);
    }
  }
}

// e_out = a0 b + sum_i alpha_i x_i (b = cg_b, complex128 AoS; e_out FP64 planar).
__global__ void __launch_bounds__(256) k_rat_combine(const SysDev* __restrict__ sys,
                                                      const int* __restrict__ bmap, int nb_total) {
  const int L = xcd_logical_block(nb_total);
  const SysDev& S = sys[bmap[L]];
  const int lb = L - S.blk0;
  const int V = S.g.V;
  const size_t slot = (size_t)4 * V;
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  const double a0 = S.shc[SHC_A0];
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double2 o[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 bv = S.cg_b[(size_t)i * 4 + q];
      o[q] = double2{a0 * bv.x, a0 * bv.y};
    }
    for (int k = 0; k < S.nshift; ++k) {
      const double al = S.shc[SHC_RES + k];
      double2 x[4];
      load_sp<double>(S.shx + (size_t)k * slot, V, i, x);
#pragma unroll
      for (int q = 0; q < 4; ++q) o[q] = double2{o[q].x + al * x[q].x, o[q].y + al * x[q].y};
    }
    store_sp<double>((double2*)S.e_out, V, i, o);
  }
}

// e_out *= f (FP64 planar).
__global__ void __launch_bounds__(256) k_scale(const SysDev* __restrict__ sys, const int* __restrict__ bmap,
                                                int nb_total, double f) {
  const int L = xcd_logical_block(nb_total);
  const SysDev& S = sys[bmap[L]];
  const int lb = L - S.blk0;
  const int V = S.g.V;
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double2 v[4];
    load_sp<double>((const double2*)S.e_out, V, i, v);
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = double2{f * v[q].x, f * v[q].y};
    store_sp<double>((double2*)S.e_out, V, i, v);
  }
}

// ----------------------------- inner MdagM in Ginsparg-Wilson form (Sec. 2.2)
// With D = 1 + g5 eps and eps^2 = 1, D^dag D = D + D^dag (the Ginsparg-Wilson
// relation at a = 1), so with the site-local Y = c- P- + c+ P+
//   MdagM v = (1 + |1 + c|^2) v + (1 + c*) g5 eps(v) + eps(g5 (1 + Y) v)
// per spin component (c = c- on spins 0,1 and c+ on spins 2,3).  The two signs
// are independent, so one two-source multi-shift solve replaces the two
// dependent ones of M then M^dag.  For the rational eps the result differs from
// MdagM by (1 - eps^2) v, i.e. by the approximation error: the inner solver
// uses it, the FP64 true residuals use M then M^dag.
//
// prep (entries A = ta[s], B = tb[s]; v = A.e_in): B.src = g5 (1 + Y) v, the
// source partials |v|^2 -> A.part_b and |B.src|^2 -> B.part_b (rho_0 of both
// multi-shift solves), and B's per-outer-iteration counter stat[3] cleared.
template <class R>
__global__ void __launch_bounds__(512) k_gw_prep(const SysDev* __restrict__ ta,
                                                  const SysDev* __restrict__ tb,
                                                  const int* __restrict__ bmap, int nb_total) {
  __shared__ double lds[17];
  const int L = xcd_logical_block(nb_total);
  const int s = bmap[L];
  const SysDev& A = ta[s];
  const SysDev& B = tb[s];
  if (A.active && *A.active == 0) return;
  const int lb = L - A.blk0;
  const int V = A.g.V;
  const int i0 = lb * A.spb;
  const int i1 = min(V, i0 + A.spb);
  if (lb == 0 && threadIdx.x == 0) B.stat[3] = 0;
  double av = 0.0, as = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    c2<R> v[4];
    load_sp<R>((const c2<R>*)A.e_in, V, i, v);
    const double2 ph = A.phi[i];
    const double cpr = A.m_re + A.g_re * ph.x - A.g_im * ph.y;
    const double cpi = A.m_im + A.g_re * ph.y + A.g_im * ph.x;
    c2<R> o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double cr = cpr, ci = (k < 2) ? -cpi : cpi;  // c- = conj(c+)
      const double vr = (double)v[k].x, vi = (double)v[k].y;
      const double g5 = k < 2 ? -1.0 : 1.0;
      o[k] = c2<R>{(R)(g5 * (vr + cr * vr - ci * vi)), (R)(g5 * (vi + cr * vi + ci * vr))};
    }
    store_sp<R>((c2<R>*)B.src, V, i, o);
    av += norm2_sp(v);
    as += norm2_sp(o);
  }
  const double tv = block_sum(av, lds);
  const double ts = block_sum(as, lds);
  if (threadIdx.x == 0) {
    A.part_b[lb] = tv;
    B.part_b[lb] = ts;
  }
}

// e = sum_{j < N} d_j t_j at site i (FP64 accumulation, two slots per step).
template <class R>
__device__ __forceinline__ void basis_sum(const c2<R>* __restrict__ basis,
                                          const double* __restrict__ d, int N, size_t slot, int V,
                                          int i, double2 e[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) e[k] = double2{0.0, 0.0};
  int j = 0;
  for (; j + 1 < N; j += 2) {
    const double d0 = d[j], d1 = d[j + 1];
    const c2<R>* b0 = basis + (size_t)j * slot;
    c2<R> v0[4], v1[4];
    load_sp<R>(b0, V, i, v0);
    load_sp<R>(b0 + slot, V, i, v1);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      e[k].x += d0 * (double)v0[k].x + d1 * (double)v1[k].x;
      e[k].y += d0 * (double)v0[k].y + d1 * (double)v1[k].y;
    }
  }
  if (j < N) {
    const double d0 = d[j];
    c2<R> v0[4];
    load_sp<R>(basis + (size_t)j * slot, V, i, v0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      e[k].x += d0 * (double)v0[k].x;
      e[k].y += d0 * (double)v0[k].y;
    }
  }
}

// combine: e1 = sum_j dA_j tA_j (entry A: eps(v)), e23 = sum_j dB_j tB_j (entry
// B: eps(g5 (1 + Y) v)), w = (1 + |1 + c|^2) v + (1 + c*) g5 e1 + e23 -> A.e_out;
// partial Re <v, w> -> A.part_a (the passes' partials are dead by then; k_cg_misc op 7
// reduces them while it writes part_c).  v = A.e_in.
template <class R>
__global__ void __launch_bounds__(512) k_gw_combine(const SysDev* __restrict__ ta,
                                                     const SysDev* __restrict__ tb,
                                                     const int* __restrict__ bmap, int nb_total) {
  __shared__ double lds[17];
  const int L = xcd_logical_block(nb_total);
  const int s = bmap[L];
  const SysDev& A = ta[s];
  const SysDev& B = tb[s];
  if (A.active && *A.active == 0) return;
  const int lb = L - A.blk0;
  const int V = A.g.V;
  const size_t slot = (size_t)4 * V;
  const int NA = A.h_ctl[1], NB = B.h_ctl[1];
  const int i0 = lb * A.spb;
  const int i1 = min(V, i0 + A.spb);
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double2 e1[4], e2[4];
    basis_sum<R>((const c2<R>*)A.basis, A.coef_d, NA, slot, V, i, e1);
    basis_sum<R>((const c2<R>*)B.basis, B.coef_d, NB, slot, V, i, e2);
    c2<R> v[4];
    load_sp<R>((const c2<R>*)A.e_in, V, i, v);
    const double2 ph = A.phi[i];
    const double cpr = A.m_re + A.g_re * ph.x - A.g_im * ph.y;
    const double cpi = A.m_im + A.g_re * ph.y + A.g_im * ph.x;
    c2<R> w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double cr = cpr, ci = (k < 2) ? -cpi : cpi;
      const double g5 = k < 2 ? -1.0 : 1.0;
      const double a = 1.0 + (1.0 + cr) * (1.0 + cr) + ci * ci + A.shift;  // 1 + |1 + c|^2 + sigma
      // (1 + c*) g5 e1
      const double br = 1.0 + cr, bi = -ci;
      const double fr = g5 * (br * e1[k].x - bi * e1[k].y);
      const double fi = g5 * (br * e1[k].y + bi * e1[k].x);
      const double vr = (double)v[k].x, vi = (double)v[k].y;
      const double wr = a * vr + fr + e2[k].x, wi = a * vi + fi + e2[k].y;
      w[k] = c2<R>{(R)wr, (R)wi};
      acc += vr * wr + vi * wi;
    }
    store_sp<R>((c2<R>*)A.e_out, V, i, w);
  }
  const double tot = block_sum(acc, lds);
  if (threadIdx.x == 0) A.part_a[lb] = tot;  // part_a: free once the passes are done
}

// ------------------------ FP64 true residual in Ginsparg-Wilson form (Sec. 2.2)
// For any Hermitian eps, D = 1 + g5 eps gives D^dag D = 1 + g5 eps + eps g5 + eps^2, so
//   MdagM x = |1 + c|^2 x + (1 + c*) g5 eps(x) + eps(g5 (1 + Y) x) + eps^2 x
// exactly (rational eps included).  One multi-shift with the two sources x (entry A)
// and g5 (1 + Y) x (entry B) provides eps(x), eps(g5 (1 + Y) x) and, from the Krylov
// space of x, w = H r(A)^2 x (coef_d2), with eps^2 x = H w: the true residual needs one
// multi-shift depth instead of two (M, then M^dag).
// combine: P = |1 + c|^2 x + (1 + c*) g5 e1 + e23 -> A.e_out, w -> A.e_out2; x = A.e_in.
__global__ void __launch_bounds__(512) k_truth_combine(const SysDev* __restrict__ ta,
                                                       const SysDev* __restrict__ tb,
                                                       const int* __restrict__ bmap, int nb_total) {
  const int L = xcd_logical_block(nb_total);
  const int s = bmap[L];
  const SysDev& A = ta[s];
  const SysDev& B = tb[s];
  if (A.active && *A.active == 0) return;
  const int lb = L - A.blk0;
  const int V = A.g.V;
  const size_t slot = (size_t)4 * V;
  const int NA = A.h_ctl[1], NB = B.h_ctl[1];
  const int i0 = lb * A.spb;
  const int i1 = min(V, i0 + A.spb);
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double2 e1[4], w[4], e2[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) e1[k] = w[k] = double2{0.0, 0.0};
    for (int j = 0; j < NA; ++j) {
      const double d = A.coef_d[j], d2 = A.coef_d2[j];
      double2 t[4];
      load_sp<double>((const double2*)A.basis + (size_t)j * slot, V, i, t);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        e1[k] = double2{e1[k].x + d * t[k].x, e1[k].y + d * t[k].y};
        w[k] = double2{w[k].x + d2 * t[k].x, w[k].y + d2 * t[k].y};
      }
    }
    basis_sum<double>((const double2*)B.basis, B.coef_d, NB, slot, V, i, e2);
    double2 x[4];
    load_sp<double>((const double2*)A.e_in, V, i, x);
    const double2 ph = A.phi[i];
    const double cpr = A.m_re + A.g_re * ph.x - A.g_im * ph.y;
    const double cpi = A.m_im + A.g_re * ph.y + A.g_im * ph.x;
    double2 P[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double cr = cpr, ci = (k < 2) ? -cpi : cpi;
      const double g5 = k < 2 ? -1.0 : 1.0;
      const double a = (1.0 + cr) * (1.0 + cr) + ci * ci;  // |1 + c|^2
      const double br = 1.0 + cr, bi = -ci;                // 1 + c*
      const double fr = g5 * (br * e1[k].x - bi * e1[k].y);
      const double fi = g5 * (br * e1[k].y + bi * e1[k].x);
      P[k] = double2{a * x[k].x + fr + e2[k].x, a * x[k].y + fi + e2[k].y};
    }
    store_sp<double>((double2*)A.e_out, V, i, P);
    store_sp<double>((double2*)A.e_out2, V, i, w);
  }
}

// finish, P = e_out, w = e_out2 (H w = eps^2 x):
//   mode 0 (true residual): r64 = b - P - H w -> cg_r64 (b = cg_b, AoS), low-precision
//          copy in cg_r when set, partial |r64|^2 -> part_c;
//   mode 1 (product): W = P + H w = MdagM x -> cg_r64, partial Re <x, W> -> part_c, x = e_in.
template <class R>
__global__ void __launch_bounds__(512) k_truth_finish(const SysDev* __restrict__ sys,
                                                      const int* __restrict__ bmap, int nb_total,
                                                      double diag, int mode) {
  __shared__ double lds[17];
  const int L = xcd_logical_block(nb_total);
  const SysDev& S = sys[bmap[L]];
  if (S.active && *S.active == 0) return;
  const int lb = L - S.blk0;
  const Geo g = S.g;
  const int V = g.V;
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double2 hw[4], P[4], rr[4];
    hw_site<double>((const double2*)S.e_out2, g, i, diag, hw);
    load_sp<double>((const double2*)S.e_out, V, i, P);
    if (mode == 1) {
      double2 x[4];
      load_sp<double>((const double2*)S.e_in, V, i, x);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        rr[k] = double2{P[k].x + hw[k].x, P[k].y + hw[k].y};
        acc += x[k].x * rr[k].x + x[k].y * rr[k].y;
      }
      store_sp<double>((double2*)S.cg_r64, V, i, rr);
      continue;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double2 bv = S.cg_b[(size_t)i * 4 + k];
      rr[k] = double2{bv.x - P[k].x - hw[k].x, bv.y - P[k].y - hw[k].y};
    }
    if (S.shift != 0.0) {  // (MdagM + sigma) x: x = e_in
      double2 x[4];
      load_sp<double>((const double2*)S.e_in, V, i, x);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        rr[k] = double2{rr[k].x - S.shift * x[k].x, rr[k].y - S.shift * x[k].y};
    }
    store_sp<double>((double2*)S.cg_r64, V, i, rr);
    if (S.cg_r) {
      c2<R> lo[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) lo[k] = c2<R>{(R)rr[k].x, (R)rr[k].y};
      store_sp<R>((c2<R>*)S.cg_r, V, i, lo);
    }
    acc += norm2_sp(rr);
  }
  const double tot = block_sum(acc, lds);
  if (threadIdx.x == 0) S.part_c[lb] = tot;
}

// ------------------------------------------------- RHMC bosonic action (eq. acws)
// phi: complex128 [V] (site order).  Pack planes of e_out2 (FP64 planar):
// 0 = phi, 1 = W' = m phi + (g/2) phi^2, 2 = conj(W'), 3 = 0.
__global__ void __launch_bounds__(256) k_boson_pack(const SysDev* __restrict__ sys,
                                                     const int* __restrict__ bmap, int nb_total) {
  const int L = xcd_logical_block(nb_total);
  const SysDev& S = sys[bmap[L]];
  const int lb = L - S.blk0;
  const int V = S.g.V;
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  const double lr = 0.5 * S.g_re, li = 0.5 * S.g_im;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const double2 f = S.phi[i];
    const double f2r = f.x * f.x - f.y * f.y, f2i = 2.0 * f.x * f.y;
    const double wr = S.m_re * f.x - S.m_im * f.y + lr * f2r - li * f2i;
    const double wi = S.m_re * f.y + S.m_im * f.x + lr * f2i + li * f2r;
    double2 v[4] = {f, double2{wr, wi}, double2{wr, -wi}, double2{0.0, 0.0}};
    store_sp<double>((double2*)S.e_in, V, i, v);
  }
}

// From the transformed planes (e_out: D_2 phi, K W', K conj(W'), K = 1 - D_2/2):
//   S partials  2 Re conj(phi) D_2 phi + Re conj(W') K W'  -> part_c
//   G = 2 [2 D_2 phi + conj(m + g phi) K W']   (G_out, may be null)
//   F = -K conj(W')                            (F_out, may be null)
__global__ void __launch_bounds__(256) k_boson_finish(const SysDev* __restrict__ sys,
                                                       const int* __restrict__ bmap, int nb_total,
                                                       double2* __restrict__ G_out,
                                                       double2* __restrict__ F_out) {
  __shared__ double lds[17];
  const int L = xcd_logical_block(nb_total);
  const SysDev& S = sys[bmap[L]];
  const int lb = L - S.blk0;
  const int V = S.g.V;
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double2 a[4], t[4];
    load_sp<double>((const double2*)S.e_in, V, i, a);   // phi, W', conj W'
    load_sp<double>((const double2*)S.e_out, V, i, t);  // D_2 phi, K W', K conj W'
    const double2 f = a[0], w = a[1];
    acc += 2.0 * (f.x * t[0].x + f.y * t[0].y) + (w.x * t[1].x + w.y * t[1].y);
    if (G_out) {
      // conj(m + g phi)
      const double cr = S.m_re + S.g_re * f.x - S.g_im * f.y;
      const double ci = -(S.m_im + S.g_re * f.y + S.g_im * f.x);
      const double pr = cr * t[1].x - ci * t[1].y, pi = cr * t[1].y + ci * t[1].x;
      G_out[i] = double2{2.0 * (2.0 * t[0].x + pr), 2.0 * (2.0 * t[0].y + pi)};
    }
    if (F_out) F_out[i] = double2{-t[2].x, -t[2].y};
  }
  const double tot = block_sum(acc, lds);
  if (threadIdx.x == 0) S.part_c[lb] = tot;
}

// Molecular-dynamics updates on complex128 [n] arrays: y += a (x1 + x2) (x2 may be
// null); optional partial |y|^2 per workgroup into part (null: none).
__global__ void __launch_bounds__(256) k_md_axpy(double2* __restrict__ y, double a,
                                                  const double2* __restrict__ x1,
                                                  const double2* __restrict__ x2, int n,
                                                  double* __restrict__ part) {
  __shared__ double lds[17];
  double acc = 0.0;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double2 v = y[i];
    if (x1) {
      double2 d = x1[i];
      if (x2) d = double2{d.x + x2[i].x, d.y + x2[i].y};
      v = double2{v.x + a * d.x, v.y + a * d.y};
      y[i] = v;
    }
    acc = v.x * v.x + v.y * v.y;
  }
  if (part) {
    const double tot = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
  }
}

// ------------------------------------------------------------ CG kernels
// CG scalars of system s from partial sums (part_c; part_b for rho = <r, z>):
//   op 0: start, rho = |r|^2;  1: alpha = rho / <p, w>;  2: beta, rho = |r|^2;
//   3 / 7: reliable update (true |r|^2 replaces the recursive one; 7 restarts);
//   4: |b|^2;  5: true |r|^2 only;
//   preconditioned (PCG, z = P r):  9: beta, rho = <r, z>, |r|^2;  10: start;
//   11 / 12: reliable update from the true residual (|r|^2 set by op 5; 12 restarts).
__global__ void k_cg_scalar(const SysDev* __restrict__ sys, int nsys, int op) {
  __shared__ double lds[17];
  const int s = blockIdx.x;
  if (s >= nsys) return;
  const SysDev& S = sys[s];
  if (S.active && *S.active == 0) return;
  const double v = (op >= 10) ? 0.0 : sum_partials(S.part_c, S.nblk, lds);
  const double rz = (op >= 9) ? sum_partials(S.part_b, S.nblk, lds) : 0.0;
  if (threadIdx.x == 0) {
    double* c = S.cg_s;
    if (op == 0) {
      c[CG_RR] = v;
      c[CG_RR_OLD] = v;
      c[CG_BETA] = 0.0;
      c[CG_R2] = v;
    } else if (op == 1) {
      c[CG_PAP] = v;
      c[CG_ALPHA] = c[CG_RR] / v;
    } else if (op == 2) {
      c[CG_RR_OLD] = c[CG_RR];
      c[CG_RR] = v;
      c[CG_BETA] = v / c[CG_RR_OLD];
      c[CG_R2] = v;
    } else if (op == 3 || op == 7) {  // reliable update: recursive |r|^2 -> true one
      // Keep the search direction unless the true residual exceeds the recursive
      // one by more than 2x (the recursion drifted) or a restart is forced (op 7,
      // a stalled recursion): then restart with p = r.
      const double rec = c[CG_RR];
      c[CG_RTRUE] = v;
      c[CG_RR] = v;
      c[CG_R2] = v;
      c[CG_BETA] = (op == 7 || v > 4.0 * rec) ? 0.0 : v / c[CG_RR_OLD];
    } else if (op == 5) {  // true residual only (no CG state change)
      c[CG_RTRUE] = v;
    } else if (op == 9) {
      c[CG_RR_OLD] = c[CG_RR];
      c[CG_RR] = rz;
      c[CG_BETA] = rz / c[CG_RR_OLD];
      c[CG_R2] = v;
    } else if (op == 10) {  // start from r = b (|b|^2 set by op 4)
      c[CG_RR] = rz;
      c[CG_RR_OLD] = rz;
      c[CG_BETA] = 0.0;
      c[CG_R2] = c[CG_BB];
    } else if (op == 11 || op == 12) {
      const double rec = c[CG_R2];
      const double rt = c[CG_RTRUE];
      c[CG_R2] = rt;
      c[CG_RR] = rz;
      c[CG_BETA] = (op == 12 || rt > 4.0 * rec) ? 0.0 : rz / c[CG_RR_OLD];
    } else if (op == 4) {  // norm of b
      c[CG_BB] = v;
    }
  }
}

// stat[3] = 0 for the nsys entries (the per-update maximum of multi-shift iterations).
__global__ void k_stat3_clear(const SysDev* __restrict__ sys, int nsys) {
  for (int s = threadIdx.x; s < nsys; s += blockDim.x)
    if (sys[s].stat) sys[s].stat[3] = 0;
}

// h_ctl[3] = 0 (the sticky multi-shift error bits) for the nsys entries, so that the
// next multi-shift solves can be checked on their own.
__global__ void k_ctl3_clear(const SysDev* __restrict__ sys, int nsys) {
  for (int s = threadIdx.x; s < nsys; s += blockDim.x)
    if (sys[s].h_ctl) sys[s].h_ctl[3] = 0;
}

// Zero n 32-bit words (a fill kernel rather than a memset node, so that the clear is
// an ordinary kernel also when a caller captures the stream into a graph).
__global__ void __launch_bounds__(256) k_zero32(unsigned int* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// p = z + beta p (z = cg_z, or r without a preconditioner; beta from cg_s;
// use_beta = 0 -> p = z); partial |p|^2 -> part_b.
template <class R>
__global__ void __launch_bounds__(512) k_cg_p(const SysDev* __restrict__ sys, const int* __restrict__ bmap,
                                               int nb_total, int use_beta) {
  __shared__ double lds[17];
  const int L = xcd_logical_block(nb_total);
  const int s = bmap[L];
  const SysDev& S = sys[s];
  if (S.active && *S.active == 0) return;
  const int lb = L - S.blk0;
  const int V = S.g.V;
  const double beta = use_beta ? S.cg_s[CG_BETA] : 0.0;
  use_beta = use_beta && beta != 0.0;  // restart: p = r, the old p is never read
  if (lb == 0 && threadIdx.x == 0) S.stat[3] = 0;
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    c2<R> r[4], p[4];
    load_sp<R>((const c2<R>*)(S.cg_z ? S.cg_z : S.cg_r), V, i, r);
    if (use_beta) {
      load_sp<R>((const c2<R>*)S.cg_p, V, i, p);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        p[k] = c2<R>{(R)((double)r[k].x + beta * (double)p[k].x),
                     (R)((double)r[k].y + beta * (double)p[k].y)};
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) p[k] = r[k];
    }
    store_sp<R>((c2<R>*)S.cg_p, V, i, p);
    acc += norm2_sp(p);
  }
  const double tot = block_sum(acc, lds);
  if (threadIdx.x == 0) S.part_b[lb] = tot;
}

// k_cg_p followed by k_gw_prep in one pass (the Ginsparg-Wilson inner operator):
// p = z + beta p -> cg_p; the second multi-shift source g5 (1 + Y) p -> B.src; partials
// |p|^2 -> part_b (the CG table's and entry A's, one buffer) and |g5 (1 + Y) p|^2 ->
// B.part_b.  S: CG table, A and B: the two entries of the inner multi-shift.
template <class R>
__global__ void __launch_bounds__(512) k_cg_p_gw(const SysDev* __restrict__ sys,
                                                 const SysDev* __restrict__ ta,
                                                 const SysDev* __restrict__ tb,
                                                 const int* __restrict__ bmap, int nb_total,
                                                 int use_beta) {
  __shared__ double lds[17];
  const int L = xcd_logical_block(nb_total);
  const int s = bmap[L];
  const SysDev& S = sys[s];
  const SysDev& A = ta[s];
  const SysDev& B = tb[s];
  if (S.active && *S.active == 0) return;
  const int lb = L - S.blk0;
  const int V = S.g.V;
  const double beta = use_beta ? S.cg_s[CG_BETA] : 0.0;
  use_beta = use_beta && beta != 0.0;  // restart: p = z, the old p is never read
  if (lb == 0 && threadIdx.x == 0) {
    S.stat[3] = 0;
    B.stat[3] = 0;
  }
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  double av = 0.0, as = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    c2<R> r[4], p[4];
    load_sp<R>((const c2<R>*)(S.cg_z ? S.cg_z : S.cg_r), V, i, r);
    if (use_beta) {
      load_sp<R>((const c2<R>*)S.cg_p, V, i, p);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        p[k] = c2<R>{(R)((double)r[k].x + beta * (double)p[k].x),
                     (R)((double)r[k].y + beta * (double)p[k].y)};
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) p[k] = r[k];
    }
    store_sp<R>((c2<R>*)S.cg_p, V, i, p);
    const double2 ph = A.phi[i];
    const double cpr = A.m_re + A.g_re * ph.x - A.g_im * ph.y;
    const double cpi = A.m_im + A.g_re * ph.y + A.g_im * ph.x;
    c2<R> o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double cr = cpr, ci = (k < 2) ? -cpi : cpi;  // c- = conj(c+)
      const double vr = (double)p[k].x, vi = (double)p[k].y;
      const double g5 = k < 2 ? -1.0 : 1.0;
      o[k] = c2<R>{(R)(g5 * (vr + cr * vr - ci * vi)), (R)(g5 * (vi + cr * vi + ci * vr))};
    }
    store_sp<R>((c2<R>*)B.src, V, i, o);
    av += norm2_sp(p);
    as += norm2_sp(o);
  }
  const double tv = block_sum(av, lds);
  const double ts = block_sum(as, lds);
  if (threadIdx.x == 0) {
    S.part_b[lb] = tv;
    B.part_b[lb] = ts;
  }
}

// Fill / axpy helpers used by the reliable-update solver.
//   op 0: x64 += x (low precision), x = 0
//   op 1: r = b (FP64 AoS -> planar R), partial |b|^2 -> part_c
//   op 2: x = 0
//   op 3: x64 += e_out (low precision), x = 0        (preconditioned fold-in)
//   op 4: partial |r|^2 -> part_c
//   op 5: x += alpha p, r -= alpha e_in, partial |r|^2 -> part_c
//   op 6: partial Re <r, z> -> part_b  (z = cg_z)
//   op 7: op 5 with alpha = rho / Re <p, w> from the partials in part_a, reduced by every
//         workgroup in the fixed order of k_cg_scalar (identical bits everywhere);
//         workgroup 0 records PAP and ALPHA
template <class R>
__global__ void __launch_bounds__(512) k_cg_misc(const SysDev* __restrict__ sys, const int* __restrict__ bmap,
                                                  int nb_total, int op) {
  __shared__ double lds[17];
  const int L = xcd_logical_block(nb_total);
  const int s = bmap[L];
  const SysDev& S = sys[s];
  if (S.active && *S.active == 0) return;
  const int lb = L - S.blk0;
  const int V = S.g.V;
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  double alpha7 = 0.0;
  const bool own_alpha = op == 7;
  if (own_alpha) {
    const double pap = sum_partials(S.part_a, S.nblk, lds);
    alpha7 = S.cg_s[CG_RR] / pap;
    if (lb == 0 && threadIdx.x == 0) {
      S.cg_s[CG_PAP] = pap;
      S.cg_s[CG_ALPHA] = alpha7;
    }
    op = 5;
  }
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    if (op == 0) {
      c2<R> xv[4];
      double2 xh[4];
      load_sp<R>((const c2<R>*)S.cg_x, V, i, xv);
      load_sp<double>((const double2*)S.cg_x64, V, i, xh);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        xh[k] = double2{xh[k].x + (double)xv[k].x, xh[k].y + (double)xv[k].y};
        xv[k] = c2<R>{(R)0, (R)0};
      }
      store_sp<double>((double2*)S.cg_x64, V, i, xh);
      store_sp<R>((c2<R>*)S.cg_x, V, i, xv);
    } else if (op == 1) {
      c2<R> rv[4];
      double2 bv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        bv[k] = S.cg_b[(size_t)i * 4 + k];
        rv[k] = c2<R>{(R)bv[k].x, (R)bv[k].y};
      }
      store_sp<R>((c2<R>*)S.cg_r, V, i, rv);
      acc += norm2_sp(bv);
    } else if (op == 2) {
      c2<R> z[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) z[k] = c2<R>{(R)0, (R)0};
      store_sp<R>((c2<R>*)S.cg_x, V, i, z);
    } else if (op == 3) {
      c2<R> xv[4];
      double2 xh[4];
      load_sp<R>((const c2<R>*)S.e_out, V, i, xv);
      load_sp<double>((const double2*)S.cg_x64, V, i, xh);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        xh[k] = double2{xh[k].x + (double)xv[k].x, xh[k].y + (double)xv[k].y};
        xv[k] = c2<R>{(R)0, (R)0};
      }
      store_sp<double>((double2*)S.cg_x64, V, i, xh);
      store_sp<R>((c2<R>*)S.cg_x, V, i, xv);
    } else if (op == 4) {
      c2<R> rv[4];
      load_sp<R>((const c2<R>*)S.cg_r, V, i, rv);
      acc += norm2_sp(rv);
    } else if (op == 5) {
      const double alpha = own_alpha ? alpha7 : S.cg_s[CG_ALPHA];
      c2<R> xv[4], pv[4], rv[4], qv[4];
      load_sp<R>((const c2<R>*)S.cg_x, V, i, xv);
      load_sp<R>((const c2<R>*)S.cg_p, V, i, pv);
      load_sp<R>((const c2<R>*)S.cg_r, V, i, rv);
      load_sp<R>((const c2<R>*)S.e_in, V, i, qv);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        xv[k] = c2<R>{(R)((double)xv[k].x + alpha * (double)pv[k].x),
                      (R)((double)xv[k].y + alpha * (double)pv[k].y)};
        rv[k] = c2<R>{(R)((double)rv[k].x - alpha * (double)qv[k].x),
                      (R)((double)rv[k].y - alpha * (double)qv[k].y)};
      }
      store_sp<R>((c2<R>*)S.cg_x, V, i, xv);
      store_sp<R>((c2<R>*)S.cg_r, V, i, rv);
      acc += norm2_sp(rv);
    } else if (op == 6) {
      c2<R> rv[4], zv[4];
      load_sp<R>((const c2<R>*)S.cg_r, V, i, rv);
      load_sp<R>((const c2<R>*)S.cg_z, V, i, zv);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        acc += (double)rv[k].x * (double)zv[k].x + (double)rv[k].y * (double)zv[k].y;
    }
  }
  if (op == 1 || op == 4 || op == 5) {
    const double tot = block_sum(acc, lds);
    if (threadIdx.x == 0) S.part_c[lb] = tot;
  } else if (op == 6) {
    const double tot = block_sum(acc, lds);
    if (threadIdx.x == 0) S.part_b[lb] = tot;
  }
}

// ------------------------------------------------------------------ force
// dS/dphi_x = -g [ Y_x^dag P+ X_x + X_x^dag P- Y_x ]  and  G_x = 2 conj(dS/dphi_x),
// summed over the nsys right-hand sides (same lattice, same phi) in index order.
// X = e_in, Y = e_out (FP64 planar) per system; G complex128 [V].
__global__ void __launch_bounds__(256) k_force(const SysDev* __restrict__ sys, int nsys,
                                                int nb0, double2* __restrict__ G) {
  const int L = xcd_logical_block(nb0);
  const SysDev& S0 = sys[0];
  const int V = S0.g.V;
  const int i0 = L * S0.spb;
  const int i1 = min(V, i0 + S0.spb);
  const double g_re = S0.g_re, g_im = S0.g_im;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double gr = 0.0, gi = 0.0;
    for (int s = 0; s < nsys; ++s) {
      double2 X[4], Y[4];
      load_sp<double>((const double2*)sys[s].e_in, V, i, X);
      load_sp<double>((const double2*)sys[s].e_out, V, i, Y);
      // t = sum_{s=2,3} conj(Y_s) X_s + sum_{s=0,1} conj(X_s) Y_s
      double tr = 0.0, ti = 0.0;
#pragma unroll
      for (int k = 2; k < 4; ++k) {
        tr += Y[k].x * X[k].x + Y[k].y * X[k].y;
        ti += Y[k].x * X[k].y - Y[k].y * X[k].x;
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        tr += X[k].x * Y[k].x + X[k].y * Y[k].y;
        ti += X[k].x * Y[k].y - X[k].y * Y[k].x;
      }
      // dS/dphi = -g t ;  G = 2 conj(dS/dphi)
      const double fr = -(g_re * tr - g_im * ti);
      const double fi = -(g_re * ti + g_im * tr);
      gr += 2.0 * fr;
      gi += -2.0 * fi;
    }
    G[i] = double2{gr, gi};
  }
}

// Partials of |c_x|^2 = |m + g phi_x|^2 over the sites of each system -> part_c.
__global__ void __launch_bounds__(256) k_c_norm(const SysDev* __restrict__ sys,
                                                const int* __restrict__ bmap, int nb_total) {
  __shared__ double lds[17];
  const int L = xcd_logical_block(nb_total);
  const SysDev& S = sys[bmap[L]];
  const int lb = L - S.blk0;
  const int V = S.g.V;
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const double2 ph = S.phi[i];
    const double cr = S.m_re + S.g_re * ph.x - S.g_im * ph.y;
    const double ci = S.m_im + S.g_re * ph.y + S.g_im * ph.x;
    acc += cr * cr + ci * ci;
  }
  const double tot = block_sum(acc, lds);
  if (threadIdx.x == 0) S.part_c[lb] = tot;
}

// Re <xi, X> partials (xi AoS complex128 from cg_b, X planar FP64 e_in) -> part_c
__global__ void __launch_bounds__(256) k_dot_re(const SysDev* __restrict__ sys, const int* __restrict__ bmap,
                                                 int nb_total) {
  __shared__ double lds[17];
  const int L = xcd_logical_block(nb_total);
  const int s = bmap[L];
  const SysDev& S = sys[s];
  const int lb = L - S.blk0;
  const int V = S.g.V;
  const int i0 = lb * S.spb;
  const int i1 = min(V, i0 + S.spb);
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double2 X[4];
    load_sp<double>((const double2*)S.e_in, V, i, X);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double2 b = S.cg_b[(size_t)i * 4 + k];
      acc += b.x * X[k].x + b.y * X[k].y;
    }
  }
  const double tot = block_sum(acc, lds);
  if (threadIdx.x == 0) S.part_c[lb] = tot;
}

}  // namespace ov
