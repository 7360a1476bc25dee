// mesh.hip -- mesh kernels of the hot path (gfx950): the Poisson solve of
// Eq. (3) in 7-point finite-difference form (FFT along the periodic x,y,
// tridiagonal along z between the electrodes), the FP64 residual used to
// refine an FP32 solve, the field of Eq. (4) and the grains' charge on the mesh.
//
// Poisson: phi = V(t) k / nz + psi, psi = 0 on both electrodes; per interior
// plane the RHS b = -dx^2 rho / eps0 is transformed along x then y, each
// Fourier mode (m, n) solves psi_{k-1} - (2 + lambda_mn) psi_k + psi_{k+1} = b_k,
// lambda_mn = 4 sin^2(pi m / nx) + 4 sin^2(pi n / ny), and the inverse
// transform returns psi.  The tridiagonal factors are computed once per run.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.hpp"
#include "launch.hpp"

namespace pic {

template <typename T>
using cplx = typename std::conditional<sizeof(T) == 8, double2, float2>::type;

template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename C>
__device__ __forceinline__ C cadd(C a, C b) {
  C r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <typename C>
__device__ __forceinline__ C csub(C a, C b) {
  C r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}
// multiply by -i (fwd = true) or +i
template <typename C>
__device__ __forceinline__ C cmi(C a, bool fwd) {
  C r;
  if (fwd) {
    r.x = a.y;
    r.y = -a.x;
  } else {
    r.x = -a.y;
    r.y = a.x;
  }
  return r;
}

// one radix-R butterfly of a Stockham stage: legs x[k xs] in, y[j ys] out,
// twiddled by w_N^{j p s}; R is a compile-time constant so the legs stay in
// registers
template <int R, typename C>
__device__ __forceinline__ void butterfly(const C* x, C* y, int xs, int ys, int N, int p, int s,
                                          const C* __restrict__ tw, bool forward) {
  C a[R], out[R];
#pragma unroll
  for (int k = 0; k < R; ++k) a[k] = x[k * xs];
  if constexpr (R == 2) {
    out[0] = cadd(a[0], a[1]);
    out[1] = csub(a[0], a[1]);
  } else if constexpr (R == 4) {
    const C t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    const C t2 = cadd(a[1], a[3]), t3 = cmi(csub(a[1], a[3]), forward);
    out[0] = cadd(t0, t2);
    out[1] = cadd(t1, t3);
    out[2] = csub(t0, t2);
    out[3] = csub(t1, t3);
  } else {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      C acc = a[0];
#pragma unroll
      for (int k = 1; k < R; ++k) {
        C w = tw[((j * k) % R) * (N / R)];
        if (forward) w.y = -w.y;
        acc = cadd(acc, cmul(a[k], w));
      }
      out[j] = acc;
    }
  }
  y[0] = out[0];
  // j p s < N: the stages keep n s = N and p < n / R
#pragma unroll
  for (int j = 1; j < R; ++j) {
    C w = tw[j * p * s];
    if (forward) w.y = -w.y;
    y[j * ys] = cmul(out[j], w);
  }
}

// the stages of one transform of L lines of length N held in LDS; element e
// of line l at buf[l * ls + e * es]; returns the buffer that holds the result
template <typename C>
__device__ C* fft_stages(C* src, C* dst, int N, int L, int ls, int es, const int* fac, int nfac,
                         const C* __restrict__ tw, bool forward) {
  // neighbouring threads take neighbouring elements of a line when elements
  // are contiguous, else neighbouring lines (no LDS bank conflicts either way)
  const bool lfast = es != 1;
  int n = N, s = 1;
  for (int f = 0; f < nfac; ++f) {
    const int r = fac[f];
    const int m = n / r;
    const int per_line = N / r;
    for (int b = threadIdx.x; b < L * per_line; b += blockDim.x) {
      const int l = lfast ? b % L : b / per_line;
      const int t = lfast ? b / L : b - l * per_line;
      const int p = t / s, q = t - p * s;
      const C* x = src + l * ls + (q + s * p) * es;
      C* y = dst + l * ls + (q + s * r * p) * es;
      const int xs = s * m * es, ys = s * es;
      switch (r) {
        case 2: butterfly<2>(x, y, xs, ys, N, p, s, tw, forward); break;
        case 3: butterfly<3>(x, y, xs, ys, N, p, s, tw, forward); break;
        case 4: butterfly<4>(x, y, xs, ys, N, p, s, tw, forward); break;
        default: butterfly<5>(x, y, xs, ys, N, p, s, tw, forward); break;
      }
    }
    __syncthreads();
    C* tmp = src;
    src = dst;
    dst = tmp;
    n = m;
    s *= r;
  }
  return src;
}

// ---------------------------------------------------------------- FFT lines
// One block transforms L lines of length N held in LDS, ping-ponging between
// two buffers through the Stockham stages (decimation in frequency):
//   y[q + s (r p + j)] = w_n^{j p} sum_k x[q + s (p + k m)] w_r^{j k},  m = n / r,
// then n <- m, s <- s r; the output ends in natural order.  Every twiddle is
// w_N^t from one table of the N-th roots of unity.
struct FftGeom {
  int N;             // line length
  int nfac;
  int fac[12];       // radices, each 2, 3, 4 or 5
  int L;             // lines per block
  int lines_per_plane;
  long elem_stride, line_stride, plane_stride;  // in elements of the work array
  long real_plane_offset;  // added to the real array offset (phi: one wall plane)
};

enum { IN_COMPLEX = 0, IN_REAL = 1 };
enum { OUT_COMPLEX = 0, OUT_REAL_LIFT = 1, OUT_REAL_ACCUM = 2, OUT_REAL_STORE = 3 };

template <typename T, int IN, int OUT>
__global__ __launch_bounds__(256) void fft_lines_kernel(FftGeom g, const cplx<T>* __restrict__ tw,
                                                        int forward, cplx<T>* __restrict__ work,
                                                        const double* __restrict__ rin,
                                                        double in_scale, double* __restrict__ rout,
                                                        double out_scale, RfDrive rf, int nz,
                                                        const int* __restrict__ skip) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  if (skip && *skip) return;  // a refinement sweep after convergence
  const double V = OUT == OUT_REAL_LIFT ? rf_voltage(rf) : 0.0;
  C* buf0 = reinterpret_cast<C*>(smem_raw);
  C* buf1 = buf0 + g.L * g.N;
  const int N = g.N, L = g.L;
  const int blocks_per_plane = g.lines_per_plane / L;
  const int plane = blockIdx.x / blocks_per_plane;
  const int l0 = (blockIdx.x % blocks_per_plane) * L;
  const long pbase = (long)plane * g.plane_stride;
  const bool e_fast = g.elem_stride == 1;

  for (int idx = threadIdx.x; idx < L * N; idx += blockDim.x) {
    const int l = e_fast ? idx / N : idx % L;
    const int e = e_fast ? idx % N : idx / L;
    const long off = pbase + (long)(l0 + l) * g.line_stride + (long)e * g.elem_stride;
    C v;
    if (IN == IN_REAL) {
      v.x = (T)(rin[off] * in_scale);
      v.y = (T)0;
    } else {
      v = work[off];
    }
    buf0[l * N + e] = v;
  }
  __syncthreads();

  C* src = fft_stages(buf0, buf1, N, L, N, 1, g.fac, g.nfac, tw, forward != 0);

  for (int idx = threadIdx.x; idx < L * N; idx += blockDim.x) {
    const int l = e_fast ? idx / N : idx % L;
    const int e = e_fast ? idx % N : idx / L;
    const long off = pbase + (long)(l0 + l) * g.line_stride + (long)e * g.elem_stride;
    const C v = src[l * N + e];
    if (OUT == OUT_COMPLEX) {
      work[off] = v;
    } else if (OUT == OUT_REAL_LIFT) {
      // interior plane k = plane + 1 of phi
      rout[off + g.real_plane_offset] =
          (double)v.x * out_scale + V * (double)(plane + 1) / (double)nz;
    } else if (OUT == OUT_REAL_STORE) {
      rout[off] = (double)v.x * out_scale;
    } else {
      rout[off] += (double)v.x * out_scale;
    }
  }
}

// ---------------------------------------------------------------- FFT planes
// One block transforms one whole plane (nx * ny points) in LDS: the x lines,
// then the y lines, with the same Stockham stages as above on strided lines,
// so a 2-D transform costs one read and one write of the plane.  Used when
// two plane buffers fit in LDS.
struct Fft2Geom {
  int nx, ny;
  int nfx, fx[12];
  int nfy, fy[12];
};

constexpr int kPlaneThreads = 1024;

template <typename T, int IN, int OUT>
__global__ __launch_bounds__(kPlaneThreads) void fft_plane_kernel(Fft2Geom g, const cplx<T>* __restrict__ tw_x,
                                                        const cplx<T>* __restrict__ tw_y,
                                                        int forward, cplx<T>* __restrict__ work,
                                                        const double* __restrict__ rin,
                                                        double in_scale, double* __restrict__ rout,
                                                        double out_scale, RfDrive rf, int nz,
                                                        const int* __restrict__ skip) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  if (skip && *skip) return;  // a refinement sweep after convergence
  const int nx = g.nx, ny = g.ny, np = nx * ny;
  C* b0 = reinterpret_cast<C*>(smem_raw);
  C* b1 = b0 + np;
  const int plane = blockIdx.x;
  const long pbase = (long)plane * np;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    C v;
    if (IN == IN_REAL) {
      v.x = (T)(rin[pbase + i] * in_scale);
      v.y = (T)0;
    } else {
      v = work[pbase + i];
    }
    b0[i] = v;
  }
  __syncthreads();
  C* res;
  if (forward) {  // x lines (rows, contiguous), then y lines (columns)
    res = fft_stages(b0, b1, nx, ny, nx, 1, g.fx, g.nfx, tw_x, true);
    C* other = res == b0 ? b1 : b0;
    res = fft_stages(res, other, ny, nx, 1, nx, g.fy, g.nfy, tw_y, true);
  } else {  // y lines, then x lines
    res = fft_stages(b0, b1, ny, nx, 1, nx, g.fy, g.nfy, tw_y, false);
    C* other = res == b0 ? b1 : b0;
    res = fft_stages(res, other, nx, ny, nx, 1, g.fx, g.nfx, tw_x, false);
  }
  const double V = OUT == OUT_REAL_LIFT ? rf_voltage(rf) : 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const C v = res[i];
    if (OUT == OUT_COMPLEX) {
      work[pbase + i] = v;
    } else if (OUT == OUT_REAL_LIFT) {
      // interior plane k = plane + 1 of phi
      rout[pbase + np + i] = (double)v.x * out_scale + V * (double)(plane + 1) / (double)nz;
    } else if (OUT == OUT_REAL_STORE) {
      rout[pbase + i] = (double)v.x * out_scale;
    } else {
      rout[pbase + i] += (double)v.x * out_scale;
    }
  }
}

// The refinement's residual r = b - A psi of one interior plane formed where
// the plane transform loads its input, then the forward 2-D transform of r
// into work, as fft_plane_kernel<T, IN_REAL, OUT_COMPLEX> does after a
// separate residual pass (the same r in FP64, the same rounding to T; r is
// not stored).  The plane's sums of r^2 and b^2 go to partials[2 k],
// partials[2 k + 1], added in a fixed order (per wave, then the waves in
// turn).  With kRhs the kernel forms b first, as rhs_residual_kernel does
// (scale rho plus the grains' shares in the table's order; block 0 freezes
// Q_g), and stores it; otherwise it reads b.
template <typename T, bool kRhs>
__global__ __launch_bounds__(kPlaneThreads) void residual_fft_kernel(
    Fft2Geom g, const cplx<T>* __restrict__ tw_x, const cplx<T>* __restrict__ tw_y,
    cplx<T>* __restrict__ work, const double* __restrict__ psi, double* __restrict__ b, RhsArgs a,
    double* __restrict__ partials, const int* __restrict__ skip) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  __shared__ double s_r[kPlaneThreads / 64], s_b[kPlaneThreads / 64];
  __shared__ int s_e[2];
  if (skip && *skip) return;  // a refinement sweep after convergence
  const int nx = g.nx, ny = g.ny, np = nx * ny;
  const int K = (int)gridDim.x;
  C* b0 = reinterpret_cast<C*>(smem_raw);
  C* b1 = b0 + np;
  const int k = blockIdx.x;
  const long pbase = (long)k * np;
  if (kRhs) {
    if (k == 0)
      for (int q = (int)threadIdx.x; q < a.ng; q += (int)blockDim.x)
        a.Q[q] = (double)((long long)a.counts[2 * q + 1] - (long long)a.counts[2 * q]) * a.we;
    if (threadIdx.x < 2) {  // the table's entries of this plane
      const long key = pbase + (threadIdx.x ? (long)np : 0);
      int lo = 0, hi = a.ntab;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((long)a.tab[mid].node < key) lo = mid + 1;
        else hi = mid;
      }
      s_e[threadIdx.x] = lo;
    }
    __syncthreads();
  }
  double rr = 0.0, bb = 0.0;
  for (int pn = (int)threadIdx.x; pn < np; pn += kPlaneThreads) {
    const long i = pbase + pn;
    double bi;
    if (kRhs) {
      bi = a.scale * (double)a.rho[i + np];
      for (int e = s_e[0]; e < s_e[1]; ++e) {
        const GrainShare t = a.tab[e];
        if (t.node != i) continue;
        const long long net = (long long)a.counts[2 * t.g + 1] - (long long)a.counts[2 * t.g];
        if (net != 0) bi += a.scale * (double)(net * t.part);
      }
      b[i] = bi;
    } else {
      bi = b[i];
    }
    const int y = pn / nx, x = pn - y * nx;
    const long row = i - x, pl = i - (long)y * nx - x;
    const double c = psi[i];
    const double xp = psi[row + (x + 1 == nx ? 0 : x + 1)];
    const double xm = psi[row + (x == 0 ? nx - 1 : x - 1)];
    const double yp = psi[pl + (long)(y + 1 == ny ? 0 : y + 1) * nx + x];
    const double ym = psi[pl + (long)(y == 0 ? ny - 1 : y - 1) * nx + x];
    const double zp = k + 1 < K ? psi[i + np] : 0.0;
    const double zm = k > 0 ? psi[i - np] : 0.0;
    const double Ax = xp + xm + yp + ym + zp + zm - 6.0 * c;
    const double ri = bi - Ax;
    rr += ri * ri;
    bb += bi * bi;
    C v;
    v.x = (T)ri;
    v.y = (T)0;
    b0[pn] = v;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    rr += __shfl_xor(rr, off, 64);
    bb += __shfl_xor(bb, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_r[threadIdx.x >> 6] = rr;
    s_b[threadIdx.x >> 6] = bb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sr = 0.0, sb = 0.0;
    for (int w = 0; w < kPlaneThreads / 64; ++w) {
      sr += s_r[w];
      sb += s_b[w];
    }
    partials[2 * k] = sr;
    partials[2 * k + 1] = sb;
  }
  C* res = fft_stages(b0, b1, nx, ny, nx, 1, g.fx, g.nfx, tw_x, true);
  C* other = res == b0 ? b1 : b0;
  res = fft_stages(res, other, ny, nx, 1, nx, g.fy, g.nfy, tw_y, true);
  for (int i = (int)threadIdx.x; i < np; i += kPlaneThreads) work[pbase + i] = res[i];
}

// ---------------------------------------------------------------- tridiagonal, chunked
// The two sweeps of the tridiagonal solve as first-order affine recurrences,
// each split into kTriChunks chunks along z per mode:
//   forward  y_k = f_k (d_k - y_{k-1})   = a_k y_{k-1} + f_k d_k,  a_k = -f_k,
//   backward x_k = y_k - f_k x_{k+1}     = a_k x_{k+1} + y_k.
// Each thread composes the affine map of its chunk, the maps of the earlier
// chunks give its incoming value (LDS), and the chunk is re-run from it.  The
// recursion depth drops from K to K / kTriChunks + kTriChunks.
constexpr int kTriChunks = 16;
constexpr int kTriModes = 16;  // modes per block (16 x 16 = 256 threads)

// d is stored in T; the recurrences run in TC with the factorisation in TC
// (the FP32 correction solves use TC = double: the lowest modes' tridiagonal
// systems are the worst conditioned part of the solve)
template <typename T, typename TC, int kTriMaxLen>  // rows per chunk held in registers
__global__ __launch_bounds__(256) void thomas_chunked_kernel(cplx<T>* __restrict__ d,
                                                             const TC* __restrict__ inv, int K,
                                                             long modes,
                                                             const int* __restrict__ skip) {
  using C = cplx<TC>;
  if (skip && *skip) return;  // a refinement sweep after convergence
  __shared__ TC s_A[kTriChunks][kTriModes];
  __shared__ C s_B[kTriChunks][kTriModes];
  const int lm = threadIdx.x % kTriModes, c = threadIdx.x / kTriModes;
  const long mn = (long)blockIdx.x * kTriModes + lm;
  const bool on = mn < modes;
  const int len = (K + kTriChunks - 1) / kTriChunks;
  const int k0 = c * len;
  const int k1 = min(K, k0 + len);
  C v[kTriMaxLen];
  TC f[kTriMaxLen];
#pragma unroll
  for (int i = 0; i < kTriMaxLen; ++i) {
    if (on && i < k1 - k0) {
      const cplx<T> a = d[(long)(k0 + i) * modes + mn];
      v[i].x = (TC)a.x;
      v[i].y = (TC)a.y;
      f[i] = inv[(long)(k0 + i) * modes + mn];
    }
  }
  // forward sweep: the chunk's map y_out = A y_in + B
  TC A = (TC)1;
  C B;
  B.x = B.y = (TC)0;
#pragma unroll
  for (int i = 0; i < kTriMaxLen; ++i) {
    if (i < k1 - k0) {
      A = -f[i] * A;
      B.x = f[i] * (v[i].x - B.x);
      B.y = f[i] * (v[i].y - B.y);
    }
  }
  s_A[c][lm] = A;
  s_B[c][lm] = B;
  __syncthreads();
  C y;
  y.x = y.y = (TC)0;
  for (int cc = 0; cc < c; ++cc) {
    const TC a = s_A[cc][lm];
    const C b = s_B[cc][lm];
    y.x = a * y.x + b.x;
    y.y = a * y.y + b.y;
  }
#pragma unroll
  for (int i = 0; i < kTriMaxLen; ++i) {
    if (i < k1 - k0) {
      y.x = f[i] * (v[i].x - y.x);
      y.y = f[i] * (v[i].y - y.y);
      v[i] = y;
    }
  }
  __syncthreads();
  // backward sweep from the chunk's end: x_start = A x_next + B
  A = (TC)1;
  B.x = B.y = (TC)0;
#pragma unroll
  for (int i = kTriMaxLen - 1; i >= 0; --i) {
    if (i < k1 - k0) {
      A = -f[i] * A;
      B.x = v[i].x - f[i] * B.x;
      B.y = v[i].y - f[i] * B.y;
    }
  }
  s_A[c][lm] = A;
  s_B[c][lm] = B;
  __syncthreads();
  C x;
  x.x = x.y = (TC)0;
  for (int cc = kTriChunks - 1; cc > c; --cc) {
    const TC a = s_A[cc][lm];
    const C b = s_B[cc][lm];
    x.x = a * x.x + b.x;
    x.y = a * x.y + b.y;
  }
#pragma unroll
  for (int i = kTriMaxLen - 1; i >= 0; --i) {
    if (i < k1 - k0) {
      x.x = v[i].x - f[i] * x.x;
      x.y = v[i].y - f[i] * x.y;
      cplx<T> o;
      o.x = (T)x.x;
      o.y = (T)x.y;
      if (on) d[(long)(k0 + i) * modes + mn] = o;
    }
  }
}

// ---------------------------------------------------------------- tridiagonal
// one thread per Fourier mode; inv[k][mode] = 1 / (diag - inv[k-1][mode]) is
// the factorisation, computed once per run (for more than 16 x 32 planes; the
// arithmetic is in TC, the forward sweep's intermediates are stored in T)
template <typename T, typename TC>
__global__ void thomas_kernel(cplx<T>* __restrict__ d, const TC* __restrict__ inv, int K,
                              long modes, const int* __restrict__ skip) {
  if (skip && *skip) return;  // a refinement sweep after convergence
  // the loads of a batch of planes are issued together: the recursion only
  // waits on arithmetic, not on one memory round trip per plane
  using C = cplx<TC>;
  constexpr int B = 8;
  const long mn = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (mn >= modes) return;
  auto ld = [&](long i) {
    const cplx<T> a = d[i];
    C r;
    r.x = (TC)a.x;
    r.y = (TC)a.y;
    return r;
  };
  auto st = [&](long i, const C& v) {
    cplx<T> o;
    o.x = (T)v.x;
    o.y = (T)v.y;
    d[i] = o;
  };
  C prev;
  prev.x = prev.y = (TC)0;
  for (int k0 = 0; k0 < K; k0 += B) {
    C cur[B];
    TC f[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (k0 + b < K) {
        cur[b] = ld((long)(k0 + b) * modes + mn);
        f[b] = inv[(long)(k0 + b) * modes + mn];
      }
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (k0 + b < K) {
        cur[b].x = (cur[b].x - prev.x) * f[b];
        cur[b].y = (cur[b].y - prev.y) * f[b];
        prev = cur[b];
        st((long)(k0 + b) * modes + mn, cur[b]);
      }
    }
  }
  // back substitution from the last plane: x_k = d'_k - inv_k x_{k+1}
  C next;
  next.x = next.y = (TC)0;
  for (int k1 = K - 1; k1 >= 0; k1 -= B) {
    C cur[B];
    TC f[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (k1 - b >= 0) {
        cur[b] = ld((long)(k1 - b) * modes + mn);
        f[b] = inv[(long)(k1 - b) * modes + mn];
      }
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (k1 - b >= 0) {
        cur[b].x -= f[b] * next.x;
        cur[b].y -= f[b] * next.y;
        next = cur[b];
        st((long)(k1 - b) * modes + mn, cur[b]);
      }
    }
  }
}

// ---------------------------------------------------------------- RHS
// b (interior planes) = scale * rho (all nodes); FP64 form rho in units of w e
__global__ void rhs_f64_kernel(const double* __restrict__ rho, double scale, double* __restrict__ b,
                               long plane, long n_int) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_int) b[i] = scale * rho[i + plane];
}

// CIC nodes and weights of a grain (its position is at least one cell inside)
__device__ __forceinline__ void grain_nodes(const double* gpos, int g, int nx, int ny, long n[8],
                                            double w[8], float off[3], int cell[3]) {
  const double X = gpos[3 * g], Y = gpos[3 * g + 1], Z = gpos[3 * g + 2];
  const int i0 = (int)floor(X), j0 = (int)floor(Y), k0 = (int)floor(Z);
  const double fx = X - i0, fy = Y - j0, fz = Z - k0;
  const int i1 = i0 + 1 == nx ? 0 : i0 + 1, j1 = j0 + 1 == ny ? 0 : j0 + 1;
  const int ii[2] = {i0, i1}, jj[2] = {j0, j1};
  for (int t = 0; t < 8; ++t) {
    const int a = t & 1, b = (t >> 1) & 1, c = t >> 2;
    n[t] = ii[a] + (long)nx * (jj[b] + (long)ny * (k0 + c));
    w[t] = (a ? fx : 1.0 - fx) * (b ? fy : 1.0 - fy) * (c ? fz : 1.0 - fz);
  }
  off[0] = (float)fx;
  off[1] = (float)fy;
  off[2] = (float)fz;
  cell[0] = i0;
  cell[1] = j0;
  cell[2] = k0;
}

// the same exact split of the macro charge as the particle deposit (FP32R)
__device__ __forceinline__ void grain_split(long long Q, double fx, double fy, double fz,
                                            long long part[8]) {
  const long long qx = (long long)floor(fx * 16777216.0);
  const long long qy = (long long)floor(fy * 16777216.0);
  const long long qz = (long long)floor(fz * 16777216.0);
  long long ax[2];
  ax[1] = (Q * qx) >> 24;
  ax[0] = Q - ax[1];
  for (int a = 0; a < 2; ++a) {
    const long long y1 = (ax[a] * qy) >> 24;
    const long long yy[2] = {ax[a] - y1, y1};
    for (int b = 0; b < 2; ++b) {
      const long long z1 = (yy[b] * qz) >> 24;
      part[a + 2 * b] = yy[b] - z1;
      part[a + 2 * b + 4] = z1;
    }
  }
}

// Grain charges at the start of the step: Q_g = (C_i - C_e) w e is frozen for
// the step's MD kernel, and the grains' CIC charge is added to the RHS.
// mode 0: FP64 (b += scale_w * net * W); mode 1: FP32R (b += scale_fixed * net * part)
__global__ void grain_rhs_kernel(const unsigned long long* __restrict__ counts, const double* gpos,
                                 int ng, int nx, int ny, int nz, double we, double* __restrict__ Q,
                                 double* __restrict__ b, double scale, int mode, long long Qp) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const long plane = (long)nx * ny;
  for (int g = 0; g < ng; ++g) {
    const long long net = (long long)counts[2 * g + 1] - (long long)counts[2 * g + 0];
    Q[g] = (double)net * we;
    if (!b || net == 0) continue;
    long n[8];
    double w[8];
    float off[3];
    int cell[3];
    grain_nodes(gpos, g, nx, ny, n, w, off, cell);
    long long part[8];
    if (mode == 1) {
      const double X = gpos[3 * g], Y = gpos[3 * g + 1], Z = gpos[3 * g + 2];
      grain_split(Qp, X - floor(X), Y - floor(Y), Z - floor(Z), part);
    }
    for (int t = 0; t < 8; ++t) {
      const long k = n[t] / plane;
      if (k < 1 || k > nz - 1) continue;
      const double add = mode == 1 ? scale * (double)(net * part[t]) : scale * (double)net * w[t];
      b[n[t] - plane] += add;
    }
  }
}

// The same in parallel for up to kGrainPairs / 8 grains: thread p takes
// corner t = p % 8 of grain g = p / 8; the first (grain, corner) pair of each
// node adds, in (grain, corner) order, every contribution to that node, so the
// sums are those of the serial loop above, bit for bit.
constexpr int kGrainPairs = 2048;
__global__ __launch_bounds__(256) void grain_rhs_par_kernel(
    const unsigned long long* __restrict__ counts, const double* gpos, int ng, int nx, int ny,
    int nz, double we, double* __restrict__ Q, double* __restrict__ b, double scale, int mode,
    long long Qp) {
  __shared__ long s_node[kGrainPairs];
  __shared__ double s_add[kGrainPairs];
  const long plane = (long)nx * ny;
  const int npair = 8 * ng;
  for (int p = threadIdx.x; p < npair; p += blockDim.x) {
    const int g = p >> 3, t = p & 7;
    const long long net = (long long)counts[2 * g + 1] - (long long)counts[2 * g + 0];
    if (t == 0) Q[g] = (double)net * we;
    long n[8];
    double w[8];
    float off[3];
    int cell[3];
    grain_nodes(gpos, g, nx, ny, n, w, off, cell);
    long long part[8];
    if (mode == 1) {
      const double X = gpos[3 * g], Y = gpos[3 * g + 1], Z = gpos[3 * g + 2];
      grain_split(Qp, X - floor(X), Y - floor(Y), Z - floor(Z), part);
    }
    const long k = n[t] / plane;
    const bool in = b && net != 0 && k >= 1 && k <= nz - 1;
    s_node[p] = in ? n[t] : -1;
    s_add[p] = mode == 1 ? scale * (double)(net * part[t]) : scale * (double)net * w[t];
  }
  __syncthreads();
  for (int p = threadIdx.x; p < npair; p += blockDim.x) {
    const long node = s_node[p];
    if (node < 0) continue;
    bool first = true;
    for (int q = 0; q < p && first; ++q) first = s_node[q] != node;
    if (!first) continue;
    double v = b[node - plane];
    for (int q = p; q < npair; ++q)
      if (s_node[q] == node) v += s_add[q];
    b[node - plane] = v;
  }
}

// unit (1 C) charge of grain g on the RHS, for its unit field
__global__ void unit_rhs_kernel(const double* gpos, int g, int nx, int ny, int nz, double scale,
                                double* __restrict__ b) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const long plane = (long)nx * ny;
  long n[8];
  double w[8];
  float off[3];
  int cell[3];
  grain_nodes(gpos, g, nx, ny, n, w, off, cell);
  for (int t = 0; t < 8; ++t) {
    const long k = n[t] / plane;
    if (k >= 1 && k <= nz - 1) b[n[t] - plane] += scale * w[t];
  }
}

// copy grain g's field (interleaved double pairs) on its cube into U[g][3][side^3]
__global__ void extract_cube_kernel(const double2* __restrict__ E, const int* gcell, int g, int c,
                                    int nx, int ny, double* __restrict__ U) {
  const int side = 2 * c + 2;
  const long cube = (long)side * side * side;
  const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= cube) return;
  const int cx = (int)(l % side), cy = (int)((l / side) % side), cz = (int)(l / (side * side));
  int i = gcell[3 * g] - c + cx, j = gcell[3 * g + 1] - c + cy;
  const int k = gcell[3 * g + 2] - c + cz;
  i = ((i % nx) + nx) % nx;
  j = ((j % ny) + ny) % ny;
  const long n = i + (long)nx * (j + (long)ny * k);
  const double2 a = E[2 * n], bz = E[2 * n + 1];
  double* Ug = U + (long)g * 3 * cube;
  Ug[l] = a.x;
  Ug[cube + l] = a.y;
  Ug[2 * cube + l] = bz.x;
}

// ---------------------------------------------------------------- refinement
// r = b - A psi on the interior nodes (psi = 0 on the electrodes), FP64;
// with NORMS, also the per-block partial sums of ||r||^2 and ||b||^2
template <bool NORMS>
__global__ __launch_bounds__(256) void residual_kernel(const double* __restrict__ psi,
                                                       const double* __restrict__ b,
                                                       double* __restrict__ r, int nx, int ny,
                                                       int K, double* __restrict__ partials,
                                                       const int* __restrict__ skip) {
  __shared__ double s_r[256], s_b[256];
  if (skip && *skip) return;  // a refinement sweep after convergence
  const long plane = (long)nx * ny;
  // grid: x over the plane's nodes, y over the planes
  const int pn = (int)(blockIdx.x * blockDim.x + threadIdx.x), k = (int)blockIdx.y;
  const long i = (long)k * plane + pn;
  double rr = 0.0, bb = 0.0;
  if (pn < plane && k < K) {
    const int y = pn / nx, x = pn - y * nx;
    const long row = i - x, pl = i - (long)y * nx - x;
    const double c = psi[i];
    const double xp = psi[row + (x + 1 == nx ? 0 : x + 1)];
    const double xm = psi[row + (x == 0 ? nx - 1 : x - 1)];
    const double yp = psi[pl + (long)(y + 1 == ny ? 0 : y + 1) * nx + x];
    const double ym = psi[pl + (long)(y == 0 ? ny - 1 : y - 1) * nx + x];
    const double zp = k + 1 < K ? psi[i + plane] : 0.0;
    const double zm = k > 0 ? psi[i - plane] : 0.0;
    const double Ax = xp + xm + yp + ym + zp + zm - 6.0 * c;
    const double bi = b[i];
    const double ri = bi - Ax;
    r[i] = ri;
    rr = ri * ri;
    bb = bi * bi;
  }
  if (!NORMS) return;
  s_r[threadIdx.x] = rr;
  s_b[threadIdx.x] = bb;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s_r[threadIdx.x] += s_r[threadIdx.x + off];
      s_b[threadIdx.x] += s_b[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const long blk = (long)blockIdx.y * gridDim.x + blockIdx.x;
    partials[2 * blk] = s_r[0];
    partials[2 * blk + 1] = s_b[0];
  }
}

// The FP32R right-hand side and the first residual of the refinement in one
// pass: b = scale rho on the interior nodes plus, at the grains' CIC nodes,
// scale (net_g part) for each share in the table's order (the order of the
// separate grain kernels: by grain, then corner), then r = b - A psi and the
// block's norm partials, as residual_kernel.  Block (0, 0) also freezes the
// grains' charges Q_g = net_g w e for the step.  net_g = C_i - C_e.
__global__ __launch_bounds__(256) void rhs_residual_kernel(
    const long long* __restrict__ rho, double scale, const GrainShare* __restrict__ tab, int ntab,
    const unsigned long long* __restrict__ counts, int ng, double we, double* __restrict__ Q,
    double* __restrict__ b, const double* __restrict__ psi, double* __restrict__ r, int nx,
    int ny, int K, double* __restrict__ partials) {
  __shared__ double s_r[256], s_b[256];
  __shared__ int s_e[2];
  const long plane = (long)nx * ny;
  const int pn0 = (int)(blockIdx.x * blockDim.x), k = (int)blockIdx.y;
  const int pn = pn0 + (int)threadIdx.x;
  const long i = (long)k * plane + pn;
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int g = (int)threadIdx.x; g < ng; g += (int)blockDim.x)
      Q[g] = (double)((long long)counts[2 * g + 1] - (long long)counts[2 * g]) * we;
  if (threadIdx.x < 2) {  // the table's entries of this block's node range
    const long key = (long)k * plane + pn0 + (threadIdx.x ? (long)blockDim.x : 0);
    int lo = 0, hi = ntab;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((long)tab[mid].node < key) lo = mid + 1;
      else hi = mid;
    }
    s_e[threadIdx.x] = lo;
  }
  __syncthreads();
  double rr = 0.0, bb = 0.0;
  if (pn < plane && k < K) {
    double bi = scale * (double)rho[i + plane];
    for (int e = s_e[0]; e < s_e[1]; ++e) {
      const GrainShare t = tab[e];
      if (t.node != i) continue;
      const long long net = (long long)counts[2 * t.g + 1] - (long long)counts[2 * t.g];
      if (net != 0) bi += scale * (double)(net * t.part);
    }
    b[i] = bi;
    const int y = pn / nx, x = pn - y * nx;
    const long row = i - x, pl = i - (long)y * nx - x;
    const double c = psi[i];
    const double xp = psi[row + (x + 1 == nx ? 0 : x + 1)];
    const double xm = psi[row + (x == 0 ? nx - 1 : x - 1)];
    const double yp = psi[pl + (long)(y + 1 == ny ? 0 : y + 1) * nx + x];
    const double ym = psi[pl + (long)(y == 0 ? ny - 1 : y - 1) * nx + x];
    const double zp = k + 1 < K ? psi[i + plane] : 0.0;
    const double zm = k > 0 ? psi[i - plane] : 0.0;
    const double Ax = xp + xm + yp + ym + zp + zm - 6.0 * c;
    const double ri = bi - Ax;
    r[i] = ri;
    rr = ri * ri;
    bb = bi * bi;
  }
  s_r[threadIdx.x] = rr;
  s_b[threadIdx.x] = bb;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s_r[threadIdx.x] += s_r[threadIdx.x + off];
      s_b[threadIdx.x] += s_b[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const long blk = (long)blockIdx.y * gridDim.x + blockIdx.x;
    partials[2 * blk] = s_r[0];
    partials[2 * blk + 1] = s_b[0];
  }
}

// sum of the per-block partial norms (one block); then the stopping test of
// the refinement after `sweep` FP32 solves (0: the residual of the starting
// guess): ctl[0] = 1 once ||r||^2 <= tol2 ||b||^2 (or r = 0), ctl[1] = sweeps
// done in this solve, ctl[2] += 1 when the last allowed sweep (last != 0)
// ends above the tolerance
__global__ __launch_bounds__(1024) void norm_reduce_kernel(const double* __restrict__ partials,
                                                           int nb, double* __restrict__ norms,
                                                           int* __restrict__ ctl, double tol2,
                                                           int sweep, int last) {
  __shared__ double s_r[1024], s_b[1024];
  if (sweep > 0 && ctl[0]) return;  // converged before this sweep
  double rr = 0.0, bb = 0.0;
  for (int i = threadIdx.x; i < nb; i += 1024) {
    rr += partials[2 * i];
    bb += partials[2 * i + 1];
  }
  s_r[threadIdx.x] = rr;
  s_b[threadIdx.x] = bb;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s_r[threadIdx.x] += s_r[threadIdx.x + off];
      s_b[threadIdx.x] += s_b[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    norms[0] = s_r[0];
    norms[1] = s_b[0];
    const int done = s_r[0] <= tol2 * s_b[0] || s_r[0] == 0.0;
    ctl[0] = done;
    ctl[1] = sweep;
    if (last && !done) ctl[2] += 1;
  }
}

__global__ void walls_kernel(double* __restrict__ phi, long plane, int nz, RfDrive rf) {
  const double V = rf_voltage(rf);
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= plane) return;
  phi[n] = 0.0;
  phi[(long)nz * plane + n] = V;
}

// ---------------------------------------------------------------- field
// E = -grad phi from a stored phi (field readouts; the step's fields come
// from field_out_kernel).  Stored interleaved per node: FP64 as two double
// pairs (Ex,Ey),(Ez,0); FP32 as one float4 (Ex,Ey,Ez,0).
template <typename OutT>
__global__ void efield_kernel(const double* __restrict__ phi, OutT* __restrict__ E, int nx, int ny,
                              int nz, double dx) {
  const long plane = (long)nx * ny;
  // grid: x over the plane's nodes, y over the planes
  const int pn = (int)(blockIdx.x * blockDim.x + threadIdx.x), k = (int)blockIdx.y;
  if (pn >= plane) return;
  const long n = (long)k * plane + pn;
  const int y = pn / nx, x = pn - y * nx;
  double ex, ey, ez;
  node_field<false>(phi, nx, ny, nz, dx, 0.0, x, y, k, ex, ey, ez);
  if constexpr (std::is_same<OutT, double2>::value) {
    E[2 * n] = make_double2(ex, ey);
    E[2 * n + 1] = make_double2(ez, 0.0);
  } else {
    E[n] = make_float4((float)ex, (float)ey, (float)ez, 0.0f);
  }
}

// ---------------------------------------------------------------- readouts
__global__ void e_out_kernel(const double2* __restrict__ E2, const float4* __restrict__ E4,
                             double* __restrict__ out, long nn) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  if (E2) {
    const double2 a = E2[2 * n], b = E2[2 * n + 1];
    out[n] = a.x;
    out[nn + n] = a.y;
    out[2 * nn + n] = b.x;
  } else {
    const float4 a = E4[n];
    out[n] = a.x;
    out[nn + n] = a.y;
    out[2 * nn + n] = a.z;
  }
}

// total rho: plasma accumulator plus grains.  FP64 form: out = conv * (acc + net W);
// FP32R: fixed = acc + net * part (exact), out = conv * fixed.
__global__ void rho_out_kernel(const double* __restrict__ acc64, const long long* __restrict__ accfx,
                               double conv, double* __restrict__ out, long long* __restrict__ outfx,
                               long nn) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  if (acc64) {
    out[n] = acc64[n];
  } else {
    outfx[n] = accfx[n];
  }
}

__global__ void rho_grains_kernel(const unsigned long long* __restrict__ counts, const double* gpos,
                                  int ng, int nx, int ny, double* __restrict__ acc,
                                  long long* __restrict__ fx, long long Qp) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int g = 0; g < ng; ++g) {
    const long long net = (long long)counts[2 * g + 1] - (long long)counts[2 * g + 0];
    long n[8];
    double w[8];
    float off[3];
    int cell[3];
    grain_nodes(gpos, g, nx, ny, n, w, off, cell);
    long long part[8];
    const double X = gpos[3 * g], Y = gpos[3 * g + 1], Z = gpos[3 * g + 2];
    grain_split(Qp, X - floor(X), Y - floor(Y), Z - floor(Z), part);
    for (int t = 0; t < 8; ++t) {
      if (acc) acc[n[t]] += (double)net * w[t];
      if (fx) fx[n[t]] += net * part[t];
    }
  }
}

__global__ void scale_kernel(const double* __restrict__ in, const long long* __restrict__ infx,
                             double conv, double* __restrict__ out, long nn) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  out[n] = conv * (in ? in[n] : (double)infx[n]);
}

// time averages: phi_k into the rf-phase bin of step k, one sample counted
__global__ void avg_phi_kernel(const double* __restrict__ phi, double* __restrict__ acc, long nn,
                               AvgBins avg, unsigned long long* __restrict__ cnt) {
  const int b = phase_bin(*avg.step, avg.f_rf, avg.dt, avg.nbins);
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n == 0) cnt[b] += 1ull;
  if (n < nn) acc[avg.stride * b + n] += phi[n];
}

// the averages over bins b0..b1-1: phi (u < n_plain) and the moments (times wv)
__global__ void avg_out_kernel(const double* __restrict__ acc, int b0, int b1, long stride,
                               long total, long n_plain, const unsigned long long* __restrict__ cnt,
                               double wv, double* __restrict__ out) {
  const long u = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= total) return;
  double s = 0.0;
  unsigned long long c = 0;
  for (int b = b0; b < b1; ++b) {
    s += acc[stride * b + u];
    c += cnt[b];
  }
  out[u] = c ? s / (double)c * (u < n_plain ? 1.0 : wv) : 0.0;
}

// phi of the unit-charge solve on grain g's MD cube: Uphi[g][side^3]
__global__ void extract_cube_phi_kernel(const double* __restrict__ phi, const int* gcell, int g,
                                        int c, int nx, int ny, double* __restrict__ Uphi) {
  const int side = 2 * c + 2;
  const long cube = (long)side * side * side;
  const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= cube) return;
  const int cx = (int)(l % side), cy = (int)((l / side) % side), cz = (int)(l / (side * side));
  int i = gcell[3 * g] - c + cx, j = gcell[3 * g + 1] - c + cy;
  const int k = gcell[3 * g + 2] - c + cz;
  i = ((i % nx) + nx) % nx;
  j = ((j % ny) + ny) % ny;
  Uphi[(long)g * cube + l] = phi[i + (long)nx * (j + (long)ny * k)];
}

// The potential on the nodes of the fine grid: the mesh potential with the
// cloud-in-cell weights of the node (a node on the domain's upper face in the
// last cell), plus for each grain whose MD cube holds the node's cell
// Q_g (1 / (4 pi eps0 max(r, a)) - its unit mesh potential at the node), the
// PPPM split of the field applied to the potential.  With avg.step set the
// value is added to the rf-phase bin's sums.
__global__ __launch_bounds__(256) void fine_phi_kernel(const double* __restrict__ phi,
                                                       MdTables md,
                                                       const double* __restrict__ Uphi,
                                                       FineBox fb, int nx, int ny, int nz,
                                                       double dx, double radius,
                                                       double* __restrict__ out, AvgBins avg) {
  if (avg.step) out += avg.stride * phase_bin(*avg.step, avg.f_rf, avg.dt, avg.nbins);
  const long u = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= fb.fn) return;
  const long ii = u % fb.mx, jj = (u / fb.mx) % fb.my, kk = u / (fb.mx * fb.my);
  const double X[3] = {fb.o[0] + fb.h * (double)ii, fb.o[1] + fb.h * (double)jj,
                       fb.o[2] + fb.h * (double)kk};
  const int n3[3] = {nx, ny, nz};
  int cl[3];
  double f[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cl[a] = (int)floor(X[a]);
    if (cl[a] > n3[a] - 1) cl[a] = n3[a] - 1;
    f[a] = X[a] - (double)cl[a];
  }
  const int i1 = cl[0] + 1 == nx ? 0 : cl[0] + 1, j1 = cl[1] + 1 == ny ? 0 : cl[1] + 1;
  double w[8];
  double v = 0.0;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int a = t & 1, b = (t >> 1) & 1, cc = t >> 2;
    w[t] = (a ? f[0] : 1.0 - f[0]) * (b ? f[1] : 1.0 - f[1]) * (cc ? f[2] : 1.0 - f[2]);
    v += w[t] * phi[(a ? i1 : cl[0]) + (long)nx * ((b ? j1 : cl[1]) + (long)ny * (cl[2] + cc))];
  }
  if (md.n_grains > 0) {
    // the periodic bounding box of the cubes: which grains' cubes hold this cell
    int bx = cl[0] - md.bx0, by = cl[1] - md.by0;
    const int bz = cl[2] - md.bz0;
    if (bx < 0) bx += nx;
    if (by < 0) by += ny;
    if (bx < md.bsx && by < md.bsy && bz >= 0 && bz < md.bsz) {
      const uint32_t e = md.cell_list[((long)bz * md.bsy + by) * md.bsx + bx];
      const int first = (int)(e >> 8), cnt = (int)(e & 255u);
      const int c = md.cutoff, side = md.side;
      const long cube = (long)side * side * side;
      for (int q = 0; q < cnt; ++q) {
        const int g = md.grain_idx[first + q];
        double r2 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          double dd = X[a] - md.gpos[3 * g + a];
          if (a < 2) dd -= (double)n3[a] * floor(dd / (double)n3[a] + 0.5);
          r2 += dd * dd;
        }
        double r = sqrt(r2) * dx;
        if (r < radius) r = radius;
        // the node's corners in the cube's node frame
        int ox = cl[0] - md.gcell[3 * g], oy = cl[1] - md.gcell[3 * g + 1];
        ox -= nx * (int)floor((double)ox / nx + 0.5);
        oy -= ny * (int)floor((double)oy / ny + 0.5);
        ox += c;
        oy += c;
        const int oz = cl[2] - md.gcell[3 * g + 2] + c;
        double unit = 0.0;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int a = t & 1, b = (t >> 1) & 1, cc = t >> 2;
          unit += w[t] * Uphi[(long)g * cube + ((long)(oz + cc) * side + (oy + b)) * side + (ox + a)];
        }
        v += md.Q[g] * (1.0 / (4.0 * kPi * kEps0 * r) - unit);
      }
    }
  }
  if (avg.step) out[u] += v;
  else out[u] = v;
}

__global__ void zero_f64_kernel(double* a, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}
__global__ void zero_i64_kernel(long long* a, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}
__global__ void zero_i32_kernel(int* a, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

// ---------------------------------------------------------------- launchers
static inline int nb256(long n) { return (int)((n + 255) / 256); }

static FftGeom make_geom(const FftPlanHost& P, bool along_x, int nx, int ny, long plane) {
  FftGeom g{};
  g.N = along_x ? nx : ny;
  const int* f = along_x ? P.fac_x : P.fac_y;
  g.nfac = along_x ? P.nfac_x : P.nfac_y;
  for (int i = 0; i < g.nfac; ++i) g.fac[i] = f[i];
  g.lines_per_plane = along_x ? ny : nx;
  g.L = along_x ? P.L_x : P.L_y;
  g.elem_stride = along_x ? 1 : nx;
  g.line_stride = along_x ? nx : 1;
  g.plane_stride = plane;
  g.real_plane_offset = plane;
  return g;
}

template <typename T>
static void fft_launch(const FftGeom& g, int planes, const void* tw, int forward, int in_mode,
                       int out_mode, void* work, const double* rin, double in_scale, double* rout,
                       double out_scale, RfDrive rf, int nz, hipStream_t st,
                       const int* skip = nullptr) {
  using C = cplx<T>;
  const int blocks = planes * (g.lines_per_plane / g.L);
  const size_t lds = 2 * sizeof(C) * g.L * g.N;
  const C* t = (const C*)tw;
  C* w = (C*)work;
  if (in_mode == IN_REAL && out_mode == OUT_COMPLEX)
    hipLaunchKernelGGL((fft_lines_kernel<T, IN_REAL, OUT_COMPLEX>), dim3(blocks), dim3(256), lds, st,
                       g, t, forward, w, rin, in_scale, rout, out_scale, rf, nz, skip);
  else if (in_mode == IN_COMPLEX && out_mode == OUT_COMPLEX)
    hipLaunchKernelGGL((fft_lines_kernel<T, IN_COMPLEX, OUT_COMPLEX>), dim3(blocks), dim3(256), lds,
                       st, g, t, forward, w, rin, in_scale, rout, out_scale, rf, nz, skip);
  else if (out_mode == OUT_REAL_LIFT)
    hipLaunchKernelGGL((fft_lines_kernel<T, IN_COMPLEX, OUT_REAL_LIFT>), dim3(blocks), dim3(256), lds,
                       st, g, t, forward, w, rin, in_scale, rout, out_scale, rf, nz, skip);
  else if (out_mode == OUT_REAL_STORE)
    hipLaunchKernelGGL((fft_lines_kernel<T, IN_COMPLEX, OUT_REAL_STORE>), dim3(blocks), dim3(256),
                       lds, st, g, t, forward, w, rin, in_scale, rout, out_scale, rf, nz, skip);
  else
    hipLaunchKernelGGL((fft_lines_kernel<T, IN_COMPLEX, OUT_REAL_ACCUM>), dim3(blocks), dim3(256),
                       lds, st, g, t, forward, w, rin, in_scale, rout, out_scale, rf, nz, skip);
}

// 2-D plane transforms when two plane buffers fit in 64 KB of LDS
constexpr size_t kPlaneLds = 65536;

template <typename T>
static void fft_plane_launch(const FftPlanHost& P, int nx, int ny, int planes, const void* tw_x,
                             const void* tw_y, int forward, int in_mode, int out_mode, void* work,
                             const double* rin, double* rout, double out_scale, RfDrive rf, int nz,
                             hipStream_t st, const int* skip = nullptr) {
  using C = cplx<T>;
  Fft2Geom g{};
  g.nx = nx;
  g.ny = ny;
  g.nfx = P.nfac_x;
  g.nfy = P.nfac_y;
  for (int i = 0; i < 12; ++i) {
    g.fx[i] = P.fac_x[i];
    g.fy[i] = P.fac_y[i];
  }
  const size_t lds = 2 * sizeof(C) * (size_t)nx * ny;
  const C* tx = (const C*)tw_x;
  const C* ty = (const C*)tw_y;
  C* w = (C*)work;
  if (in_mode == IN_REAL)
    hipLaunchKernelGGL((fft_plane_kernel<T, IN_REAL, OUT_COMPLEX>), dim3(planes), dim3(kPlaneThreads), lds, st,
                       g, tx, ty, forward, w, rin, 1.0, rout, out_scale, rf, nz, skip);
  else if (out_mode == OUT_REAL_LIFT)
    hipLaunchKernelGGL((fft_plane_kernel<T, IN_COMPLEX, OUT_REAL_LIFT>), dim3(planes),
                       dim3(kPlaneThreads), lds, st, g, tx, ty, forward, w, rin, 1.0, rout, out_scale, rf, nz, skip);
  else if (out_mode == OUT_REAL_STORE)
    hipLaunchKernelGGL((fft_plane_kernel<T, IN_COMPLEX, OUT_REAL_STORE>), dim3(planes),
                       dim3(kPlaneThreads), lds, st, g, tx, ty, forward, w, rin, 1.0, rout, out_scale, rf, nz, skip);
  else
    hipLaunchKernelGGL((fft_plane_kernel<T, IN_COMPLEX, OUT_REAL_ACCUM>), dim3(planes),
                       dim3(kPlaneThreads), lds, st, g, tx, ty, forward, w, rin, 1.0, rout, out_scale, rf, nz, skip);
}

// the tridiagonal solves of every mode: work in T, the factorisation inv and
// the arithmetic in double (both forms)
template <typename T>
static void tridiag_launch(void* work, const void* inv, int K, long modes, hipStream_t st,
                           const int* skip = nullptr) {
  using C = cplx<T>;
  const int len = (K + kTriChunks - 1) / kTriChunks;
  const int blocks = (int)((modes + kTriModes - 1) / kTriModes);
  if (len <= 16)
    hipLaunchKernelGGL((thomas_chunked_kernel<T, double, 16>), dim3(blocks), dim3(256), 0, st,
                       (C*)work, (const double*)inv, K, modes, skip);
  else if (len <= 32)
    hipLaunchKernelGGL((thomas_chunked_kernel<T, double, 32>), dim3(blocks), dim3(256), 0, st,
                       (C*)work, (const double*)inv, K, modes, skip);
  else
    hipLaunchKernelGGL((thomas_kernel<T, double>), dim3(nb256(modes)), dim3(256), 0, st, (C*)work,
                       (const double*)inv, K, modes, skip);
}

// one FFT + tridiagonal + inverse FFT solve of A psi = b (T = double or float);
// out_mode OUT_REAL_LIFT writes phi (with the lift), OUT_REAL_ACCUM adds to psi
template <typename T>
static void solve_once(const FftPlanHost& P, int nx, int ny, int nz, const double* b, void* work,
                       const void* tw_x, const void* tw_y, const void* inv, int out_mode,
                       double* out, RfDrive rf, hipStream_t st, const int* skip = nullptr) {
  const long plane = (long)nx * ny;
  const int K = nz - 1;
  if (2 * sizeof(cplx<T>) * (size_t)plane <= kPlaneLds) {
    fft_plane_launch<T>(P, nx, ny, K, tw_x, tw_y, 1, IN_REAL, OUT_COMPLEX, work, b, nullptr, 0.0,
                        rf, nz, st, skip);
    tridiag_launch<T>(work, inv, K, plane, st, skip);
    fft_plane_launch<T>(P, nx, ny, K, tw_x, tw_y, 0, IN_COMPLEX, out_mode, work, nullptr, out,
                        1.0 / (double)plane, rf, nz, st, skip);
    return;
  }
  const FftGeom gx = make_geom(P, true, nx, ny, plane);
  const FftGeom gy = make_geom(P, false, nx, ny, plane);
  fft_launch<T>(gx, K, tw_x, 1, IN_REAL, OUT_COMPLEX, work, b, 1.0, nullptr, 0.0, rf, nz, st, skip);
  fft_launch<T>(gy, K, tw_y, 1, IN_COMPLEX, OUT_COMPLEX, work, nullptr, 0.0, nullptr, 0.0, rf, nz,
                st, skip);
  tridiag_launch<T>(work, inv, K, plane, st, skip);
  fft_launch<T>(gy, K, tw_y, 0, IN_COMPLEX, OUT_COMPLEX, work, nullptr, 0.0, nullptr, 0.0, rf, nz,
                st, skip);
  fft_launch<T>(gx, K, tw_x, 0, IN_COMPLEX, out_mode, work, nullptr, 0.0, out,
                1.0 / (double)plane, rf, nz, st, skip);
}

void launch_solve_f64(const FftPlanHost& P, int nx, int ny, int nz, const double* b, void* work,
                      const void* tw_x, const void* tw_y, const void* inv, double* phi, RfDrive rf,
                      hipStream_t st) {
  solve_once<double>(P, nx, ny, nz, b, work, tw_x, tw_y, inv, OUT_REAL_LIFT, phi, rf, st);
  hipLaunchKernelGGL(walls_kernel, dim3(nb256((long)nx * ny)), dim3(256), 0, st, phi,
                     (long)nx * ny, nz, rf);
}

// FP32 solves refined in FP64, starting from the psi the previous solve left
// (zero after loading): r = b - A psi; then up to `sweeps` times
// { psi += solve32(r); r = b - A psi }, stopping once ||r|| <= tol ||b||
// (phi = psi + lift is formed with the field, field_out_kernel).  The charge moves little in one step, so the previous
// potential is a close guess and each sweep gains the FP32 transforms'
// ~1e-6 on a small correction (the tridiagonal solves inside run in FP64:
// in FP32 the lowest modes, conditioned like (nz / pi)^2, would limit a sweep
// to ~1e-3).  Every sweep is launched (a captured step replays the same
// kernels); the kernels of a sweep after convergence return at once on
// ctl[0].  norms[0..1] receive ||r||^2, ||b||^2 of the last residual formed;
// norms[2..] hold 2 partials per residual block: ceil(nx ny / 256) blocks per
// interior plane; ctl as in norm_reduce_kernel.
void launch_solve_refined(const FftPlanHost& P, int nx, int ny, int nz, const double* b,
                          double* psi, double* r, void* work32, const void* tw_x32,
                          const void* tw_y32, const void* inv, RfDrive rf, int sweeps,
                          double tol, double* norms, int* ctl, hipStream_t st, bool have_r0) {
  const long plane = (long)nx * ny;
  const int nb = (int)(nb256(plane) * (nz - 1));
  if (!have_r0)
    hipLaunchKernelGGL(residual_kernel<true>, dim3(nb256(plane), nz - 1), dim3(256), 0, st, psi,
                       b, r, nx, ny, nz - 1, norms + 2, nullptr);
  hipLaunchKernelGGL(norm_reduce_kernel, dim3(1), dim3(1024), 0, st, norms + 2, nb, norms, ctl,
                     tol * tol, 0, 0);
  for (int it = 1; it <= sweeps; ++it) {
    solve_once<float>(P, nx, ny, nz, r, work32, tw_x32, tw_y32, inv, OUT_REAL_ACCUM, psi, rf, st,
                      ctl);
    hipLaunchKernelGGL(residual_kernel<true>, dim3(nb256(plane), nz - 1), dim3(256), 0, st, psi,
                       b, r, nx, ny, nz - 1, norms + 2, ctl);
    hipLaunchKernelGGL(norm_reduce_kernel, dim3(1), dim3(1024), 0, st, norms + 2, nb, norms, ctl,
                       tol * tol, it, it == sweeps ? 1 : 0);
  }
}

void launch_rhs_residual(const long long* rho, double scale, const GrainShare* tab, int ntab,
                         const unsigned long long* counts, int ng, double we, double* Q,
                         double* b, const double* psi, double* r, int nx, int ny, int nz,
                         double* partials, hipStream_t st) {
  const long plane = (long)nx * ny;
  hipLaunchKernelGGL(rhs_residual_kernel, dim3(nb256(plane), nz - 1), dim3(256), 0, st, rho, scale,
                     tab, ntab, counts, ng, we, Q, b, psi, r, nx, ny, nz - 1, partials);
}

void launch_refine_final(int nx, int ny, int nz, const double* b, const double* psi, double* r,
                         int sweeps, double tol, double* norms, int* ctl, hipStream_t st);

// The FP32R field solve from the fixed-point charge: the right-hand side and
// the refinement of launch_rhs_residual + launch_solve_refined(have_r0).
// When two planes fit in LDS the residual before each sweep but the last is
// formed inside the sweep's forward plane transform (the first one also forms
// b), so the sweep runs transform, tridiagonal, inverse transform; the
// residual after the last sweep has its own kernel (launch_refine_final; with
// defer_final the caller launches it, and 1 is returned).  The stopping test
// is the same, with the per-plane partial sums of those fused kernels.
// first_done, when given, is recorded on st after the first kernel (the one
// that reads rho and the grains' counts); -1 if that record fails.
int launch_rhs_solve_refined(const RhsArgs& a, const FftPlanHost& P, int nx, int ny, int nz,
                             double* b, double* psi, double* r, void* work32,
                             const void* tw_x32, const void* tw_y32, const void* inv, RfDrive rf,
                             int sweeps, double tol, double* norms, int* ctl, hipStream_t st,
                             bool defer_final, hipEvent_t first_done) {
  using C = cplx<float>;
  const long plane = (long)nx * ny;
  const int K = nz - 1;
  if (2 * sizeof(C) * (size_t)plane > kPlaneLds) {
    launch_rhs_residual(a.rho, a.scale, a.tab, a.ntab, a.counts, a.ng, a.we, a.Q, b, psi, r, nx,
                        ny, nz, norms + 2, st);
    if (first_done && hipEventRecord(first_done, st) != hipSuccess) return -1;
    launch_solve_refined(P, nx, ny, nz, b, psi, r, work32, tw_x32, tw_y32, inv, rf, sweeps, tol,
                         norms, ctl, st, true);
    return 0;
  }
  Fft2Geom g{};
  g.nx = nx;
  g.ny = ny;
  g.nfx = P.nfac_x;
  g.nfy = P.nfac_y;
  for (int i = 0; i < 12; ++i) {
    g.fx[i] = P.fac_x[i];
    g.fy[i] = P.fac_y[i];
  }
  const size_t lds = 2 * sizeof(C) * (size_t)plane;
  const C* tx = (const C*)tw_x32;
  const C* ty = (const C*)tw_y32;
  C* w = (C*)work32;
  hipLaunchKernelGGL((residual_fft_kernel<float, true>), dim3(K), dim3(kPlaneThreads), lds, st, g,
                     tx, ty, w, psi, b, a, norms + 2, nullptr);
  if (first_done && hipEventRecord(first_done, st) != hipSuccess) return -1;
  hipLaunchKernelGGL(norm_reduce_kernel, dim3(1), dim3(1024), 0, st, norms + 2, K, norms, ctl,
                     tol * tol, 0, 0);
  for (int it = 1; it <= sweeps; ++it) {
    tridiag_launch<float>(work32, inv, K, plane, st, ctl);
    fft_plane_launch<float>(P, nx, ny, K, tw_x32, tw_y32, 0, IN_COMPLEX, OUT_REAL_ACCUM, work32,
                            nullptr, psi, 1.0 / (double)plane, rf, nz, st, ctl);
    if (it < sweeps) {
      hipLaunchKernelGGL((residual_fft_kernel<float, false>), dim3(K), dim3(kPlaneThreads), lds,
                         st, g, tx, ty, w, psi, b, a, norms + 2, ctl);
      hipLaunchKernelGGL(norm_reduce_kernel, dim3(1), dim3(1024), 0, st, norms + 2, K, norms, ctl,
                         tol * tol, it, 0);
    } else if (!defer_final) {
      launch_refine_final(nx, ny, nz, b, psi, r, sweeps, tol, norms, ctl, st);
    }
  }
  return defer_final ? 1 : 0;
}

// the residual after the last sweep and its stopping test (the reported
// residual and the count of solves that ended above the tolerance); psi and b
// stay as the solve left them until the next solve, so this may run on
// another stream beside the work that follows the solve
void launch_refine_final(int nx, int ny, int nz, const double* b, const double* psi, double* r,
                         int sweeps, double tol, double* norms, int* ctl, hipStream_t st) {
  const long plane = (long)nx * ny;
  const int K = nz - 1;
  const int nb = (int)(nb256(plane) * K);
  hipLaunchKernelGGL(residual_kernel<true>, dim3(nb256(plane), K), dim3(256), 0, st, psi, b, r,
                     nx, ny, K, norms + 2, ctl);
  hipLaunchKernelGGL(norm_reduce_kernel, dim3(1), dim3(1024), 0, st, norms + 2, nb, norms, ctl,
                     tol * tol, sweeps, 1);
}

void launch_rhs_f64(const double* rho, double scale, double* b, int nx, int ny, int nz,
                    hipStream_t st) {
  const long plane = (long)nx * ny, n_int = plane * (nz - 1);
  hipLaunchKernelGGL(rhs_f64_kernel, dim3(nb256(n_int)), dim3(256), 0, st, rho, scale, b, plane,
                     n_int);
}

void launch_grain_rhs(const unsigned long long* counts, const double* gpos, int ng, int nx, int ny,
                      int nz, double we, double* Q, double* b, double scale, int mode,
                      long long Qp, hipStream_t st) {
  if (ng <= 0) return;
  if (8 * ng <= kGrainPairs)
    hipLaunchKernelGGL(grain_rhs_par_kernel, dim3(1), dim3(256), 0, st, counts, gpos, ng, nx, ny,
                       nz, we, Q, b, scale, mode, Qp);
  else
    hipLaunchKernelGGL(grain_rhs_kernel, dim3(1), dim3(64), 0, st, counts, gpos, ng, nx, ny, nz,
                       we, Q, b, scale, mode, Qp);
}

void launch_unit_rhs(const double* gpos, int g, int nx, int ny, int nz, double scale, double* b,
                     hipStream_t st) {
  hipLaunchKernelGGL(unit_rhs_kernel, dim3(1), dim3(64), 0, st, gpos, g, nx, ny, nz, scale, b);
}

void launch_extract_cube(const double* E, const int* gcell, int g, int c, int nx, int ny, double* U,
                         hipStream_t st) {
  const long side = 2 * c + 2, cube = side * side * side;
  hipLaunchKernelGGL(extract_cube_kernel, dim3(nb256(cube)), dim3(256), 0, st, (const double2*)E,
                     gcell, g, c, nx, ny, U);
}

void launch_efield_f64(const double* phi, double* E, int nx, int ny, int nz, double dx,
                       hipStream_t st) {
  hipLaunchKernelGGL(efield_kernel<double2>, dim3(nb256((long)nx * ny), nz + 1), dim3(256), 0, st,
                     phi, (double2*)E, nx, ny, nz, dx);
}

void launch_e_out(const double* E64, const float* E32, double* out, long nn, hipStream_t st) {
  hipLaunchKernelGGL(e_out_kernel, dim3(nb256(nn)), dim3(256), 0, st, (const double2*)E64,
                     (const float4*)E32, out, nn);
}

void launch_rho_total(const double* acc64, const long long* accfx, double* tot64,
                      long long* totfx, const unsigned long long* counts, const double* gpos,
                      int ng, int nx, int ny, long nn, long long Qp, hipStream_t st) {
  hipLaunchKernelGGL(rho_out_kernel, dim3(nb256(nn)), dim3(256), 0, st, acc64, accfx, 0.0, tot64,
                     totfx, nn);
  if (ng > 0)
    hipLaunchKernelGGL(rho_grains_kernel, dim3(1), dim3(64), 0, st, counts, gpos, ng, nx, ny,
                       acc64 ? tot64 : nullptr, acc64 ? nullptr : totfx, Qp);
}

void launch_scale(const double* in, const long long* infx, double conv, double* out, long nn,
                  hipStream_t st) {
  hipLaunchKernelGGL(scale_kernel, dim3(nb256(nn)), dim3(256), 0, st, in, infx, conv, out, nn);
}

void launch_avg_phi(const double* phi, double* acc, long nn, const AvgBins& avg,
                    unsigned long long* cnt, hipStream_t st) {
  hipLaunchKernelGGL(avg_phi_kernel, dim3(nb256(nn)), dim3(256), 0, st, phi, acc, nn, avg, cnt);
}

void launch_avg_out(const double* acc, int b0, int b1, long stride, long total, long n_plain,
                    const unsigned long long* cnt, double wv, double* out, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(avg_out_kernel, dim3(nb256(total)), dim3(256), 0, st, acc, b0, b1, stride,
                     total, n_plain, cnt, wv, out);
}

void launch_extract_cube_phi(const double* phi, const int* gcell, int g, int c, int nx, int ny,
                             double* Uphi, hipStream_t st) {
  const long side = 2 * c + 2, cube = side * side * side;
  hipLaunchKernelGGL(extract_cube_phi_kernel, dim3(nb256(cube)), dim3(256), 0, st, phi, gcell, g, c,
                     nx, ny, Uphi);
}

void launch_fine_phi(const double* phi, const MdTables& md, const double* Uphi, const FineBox& fb,
                     int nx, int ny, int nz, double dx, double radius, double* out,
                     const AvgBins& avg, hipStream_t st) {
  if (fb.fn <= 0) return;
  hipLaunchKernelGGL(fine_phi_kernel, dim3(nb256(fb.fn)), dim3(256), 0, st, phi, md, Uphi, fb, nx, ny,
                     nz, dx, radius, out, avg);
}

void launch_zero_f64(double* a, long n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(zero_f64_kernel, dim3(nb256(n)), dim3(256), 0, st, a, n);
}
void launch_zero_i64(long long* a, long n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(zero_i64_kernel, dim3(nb256(n)), dim3(256), 0, st, a, n);
}
void launch_zero_i32(int* a, long n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(zero_i32_kernel, dim3(nb256(n)), dim3(256), 0, st, a, n);
}

}  // namespace pic
