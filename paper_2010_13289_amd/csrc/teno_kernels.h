// Kernels of the TENO-M path and their launchers.
//
//  k_faces         one thread per face of one axis; writes the face fluxes
//                  (and optionally the smoothness flags).  The unit the
//                  reconstruct_faces call exposes.
//  k_sweep_row     sweep along x (unit stride).  A 256-thread workgroup owns
//                  one row segment: each thread computes one face flux into
//                  LDS, then each thread forms one cell's divergence and
//                  applies the epilogue.  A periodic row of <= 256 cells is
//                  one segment, so every face is computed exactly once.
//  k_sweep_march   sweep along y or z (strided).  Each lane owns one x
//                  column (coalesced 512-byte rows per wave) and marches
//                  along the axis over a segment of cells, carrying the
//                  previous face flux in registers; M cells cost M+1 faces
//                  (M faces for a whole periodic line).
//
// Sweep epilogues (divergence -dF/dx of the axis, then):
//  STORE  R = div                      ACCUM  R += div
//  RK     Uout = a U0 + b (Us + dt (R + div))      RK1   Uout = a U0 + b (Us + dt div)
#pragma once

#include "teno_device.h"

namespace tenom {

enum : int { EPI_STORE = 0, EPI_ACCUM = 1, EPI_RK = 2, EPI_RK1 = 3 };

template <int NF>
struct SweepParams {
  const double* U;   // state the stencils read
  double* R;         // divergence accumulator (STORE/ACCUM write, RK reads)
  const double* U0;  // RK: U^n
  const double* Us;  // RK: stage state
  double* Uout;      // RK: output state
  double a, b, dt;   // RK coefficients
  int mode;
  int nx, ny, nz;    // grid extents (1 for unused axes)
  int n;             // cells along the sweep axis
  int bc;            // boundary rule of the sweep axis
  double inv_dx;     // 1 / dx of the sweep axis
  int seg;           // cells per segment
  int nseg;          // segments per line
  int fld[NF];       // rotated component -> storage field
  FaceParams fp;
};

template <int NF>
__device__ __forceinline__ void epilogue(const SweepParams<NF>& p, long N, long cell, const double (&div)[NF]) {
#pragma unroll
  for (int q = 0; q < NF; ++q) {
    const long o = (long)p.fld[q] * N + cell;
    if (p.mode == EPI_STORE) {
      p.R[o] = div[q];
    } else if (p.mode == EPI_ACCUM) {
      p.R[o] = p.R[o] + div[q];
    } else {
      const double rhs = (p.mode == EPI_RK) ? p.R[o] + div[q] : div[q];
      const double us = fma(p.dt, rhs, p.Us[o]);
      p.Uout[o] = (p.a != 0.0) ? fma(p.a, p.U0[o], p.b * us) : p.b * us;
    }
  }
}

// ---------------------------------------------------------------------------
template <int NF, int K, int LIM>
__global__ __launch_bounds__(256) void k_faces(const double* __restrict__ U, double* __restrict__ Fhat,
                                               uint8_t* __restrict__ flags, int axis, int nx, int ny, int nz,
                                               int bc, int fld0, int fld1, int fld2, int fld3, int fld4,
                                               FaceParams fp) {
  const int fnx = nx + (axis == 0), fny = ny + (axis == 1), fnz = nz + (axis == 2);
  const long nfaces = (long)fnx * fny * fnz;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nfaces) return;
  const int fx = (int)(t % fnx);
  const int fy = (int)((t / fnx) % fny);
  const int fz = (int)(t / ((long)fnx * fny));
  const long N = (long)nx * ny * nz;
  Line L;
  int j;
  if (axis == 0) {
    L = Line{(long)nx * (fy + (long)ny * fz), 1, nx, bc};
    j = fx;
  } else if (axis == 1) {
    L = Line{fx + (long)nx * ny * fz, nx, ny, bc};
    j = fy;
  } else {
    L = Line{fx + (long)nx * fy, (long)nx * ny, nz, bc};
    j = fz;
  }
  const int fall[5] = {fld0, fld1, fld2, fld3, fld4};
  int fld[NF];
#pragma unroll
  for (int q = 0; q < NF; ++q) fld[q] = fall[q];
  double F[NF];
  uint32_t bits[2][NF];
  if (flags) {
    face_flux<NF, K, LIM, true>(U, N, fld, L, j, fp, F, bits);
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      flags[(long)q * nfaces + t] = (uint8_t)bits[0][q];
      flags[(long)(NF + q) * nfaces + t] = (uint8_t)bits[1][q];
    }
  } else {
    face_flux<NF, K, LIM, false>(U, N, fld, L, j, fp, F, bits);
  }
#pragma unroll
  for (int q = 0; q < NF; ++q) Fhat[(long)fld[q] * nfaces + t] = F[q];
}

// ---------------------------------------------------------------------------
template <int NF, int K, int LIM>
__global__ __launch_bounds__(256) void k_sweep_row(SweepParams<NF> p) {
  __shared__ double Fs[NF][257];
  const int s = blockIdx.x % p.nseg;
  const long row = blockIdx.x / p.nseg;  // y + ny * z
  const int c_begin = s * p.seg;
  const int ncell = min(p.seg, p.n - c_begin);
  const bool wrap = (p.bc == 0) && (p.seg >= p.n);  // whole periodic row
  const int nface = wrap ? p.n : ncell + 1;
  const long N = (long)p.nx * p.ny * p.nz;
  const Line L{row * p.nx, 1, p.n, p.bc};
  const int t = threadIdx.x;
  if (t < nface) {
    double F[NF];
    uint32_t bits[2][NF];
    face_flux<NF, K, LIM, false>(p.U, N, p.fld, L, c_begin + t, p.fp, F, bits);
#pragma unroll
    for (int q = 0; q < NF; ++q) Fs[q][t] = F[q];
  }
  __syncthreads();
  if (t < ncell) {
    const int r = (wrap && t == p.n - 1) ? 0 : t + 1;
    double div[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) div[q] = (Fs[q][t] - Fs[q][r]) * p.inv_dx;
    epilogue<NF>(p, N, L.base + c_begin + t, div);
  }
}

// ---------------------------------------------------------------------------
// blockDim = (64, 4): x = lane, y = line within the block; axis = 1 or 2
template <int NF, int K, int LIM>
__global__ __launch_bounds__(256) void k_sweep_march(SweepParams<NF> p, int axis) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int n_other = (axis == 1) ? p.nz : p.ny;
  const int o = blockIdx.y * 4 + threadIdx.y;
  if (x >= p.nx || o >= n_other) return;
  const int s = blockIdx.z;
  const long N = (long)p.nx * p.ny * p.nz;
  Line L;
  if (axis == 1)
    L = Line{x + (long)p.nx * p.ny * o, p.nx, p.ny, p.bc};
  else
    L = Line{x + (long)p.nx * o, (long)p.nx * p.ny, p.nz, p.bc};
  const int c_begin = s * p.seg;
  const int ncell = min(p.seg, p.n - c_begin);
  const bool wrap = (p.bc == 0) && (p.seg >= p.n);
  double Fprev[NF], Ffirst[NF];
  for (int t = 0; t <= ncell; ++t) {
    double F[NF];
    if (wrap && t == ncell) {
#pragma unroll
      for (int q = 0; q < NF; ++q) F[q] = Ffirst[q];
    } else {
      uint32_t bits[2][NF];
      face_flux<NF, K, LIM, false>(p.U, N, p.fld, L, c_begin + t, p.fp, F, bits);
      if (wrap && t == 0) {
#pragma unroll
        for (int q = 0; q < NF; ++q) Ffirst[q] = F[q];
      }
    }
    if (t > 0) {
      double div[NF];
#pragma unroll
      for (int q = 0; q < NF; ++q) div[q] = (Fprev[q] - F[q]) * p.inv_dx;
      epilogue<NF>(p, N, L.base + (long)(c_begin + t - 1) * L.stride, div);
    }
#pragma unroll
    for (int q = 0; q < NF; ++q) Fprev[q] = F[q];
  }
}

// ---------------------------------------------------------------------------
// Launch descriptors (host side)
// ---------------------------------------------------------------------------
struct FacesLaunch {
  const double* U;
  double* Fhat;
  uint8_t* flags;
  int axis, nx, ny, nz, bc;
  int fld[5];
  FaceParams fp;
  hipStream_t stream;
};

struct SweepLaunch {
  int axis;
  const double* U;
  double* R;
  const double* U0;
  const double* Us;
  double* Uout;
  double a, b, dt;
  int mode;
  int nx, ny, nz, bc;
  double inv_dx;
  int seg;  // cells per segment along the axis (march sweeps)
  int fld[5];
  FaceParams fp;
  hipStream_t stream;
};

template <int NF, int K, int LIM>
hipError_t launch_faces(const FacesLaunch& a) {
  const long nfaces = (long)(a.nx + (a.axis == 0)) * (a.ny + (a.axis == 1)) * (a.nz + (a.axis == 2));
  const unsigned blocks = (unsigned)((nfaces + 255) / 256);
  hipLaunchKernelGGL((k_faces<NF, K, LIM>), dim3(blocks), dim3(256), 0, a.stream, a.U, a.Fhat, a.flags, a.axis,
                     a.nx, a.ny, a.nz, a.bc, a.fld[0], a.fld[1], a.fld[2], a.fld[3], a.fld[4], a.fp);
  return hipGetLastError();
}

template <int NF, int K, int LIM>
hipError_t launch_sweep(const SweepLaunch& a) {
  SweepParams<NF> p;
  p.U = a.U;
  p.R = a.R;
  p.U0 = a.U0;
  p.Us = a.Us;
  p.Uout = a.Uout;
  p.a = a.a;
  p.b = a.b;
  p.dt = a.dt;
  p.mode = a.mode;
  p.nx = a.nx;
  p.ny = a.ny;
  p.nz = a.nz;
  p.bc = a.bc;
  p.inv_dx = a.inv_dx;
  p.fp = a.fp;
  for (int q = 0; q < NF; ++q) p.fld[q] = a.fld[q];
  if (a.axis == 0) {
    p.n = a.nx;
    p.seg = (a.bc == 0 && a.nx <= 256) ? a.nx : 255;
    p.nseg = (p.n + p.seg - 1) / p.seg;
    const long blocks = (long)p.nseg * a.ny * a.nz;
    hipLaunchKernelGGL((k_sweep_row<NF, K, LIM>), dim3((unsigned)blocks), dim3(256), 0, a.stream, p);
  } else {
    p.n = (a.axis == 1) ? a.ny : a.nz;
    p.seg = a.seg >= p.n ? p.n : a.seg;
    p.nseg = (p.n + p.seg - 1) / p.seg;
    const int n_other = (a.axis == 1) ? a.nz : a.ny;
    dim3 grid((a.nx + 63) / 64, (n_other + 3) / 4, p.nseg);
    hipLaunchKernelGGL((k_sweep_march<NF, K, LIM>), grid, dim3(64, 4), 0, a.stream, p, a.axis);
  }
  return hipGetLastError();
}

}  // namespace tenom
