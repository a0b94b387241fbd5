// Kernels of the TENO-M path and their launchers.
//
//  k_faces         one thread per face of one axis; writes the face fluxes
//                  (and optionally the smoothness flags).  The unit the
//                  reconstruct_faces call exposes.
//  k_sweep_row     sweep along x (unit stride).  A 256-thread workgroup owns
//                  one row segment: the segment's cells are staged in LDS
//                  with their flux, signal speed and Roe inputs, each thread
//                  computes one face flux, the fluxes go back to LDS, then
//                  each thread forms one cell's divergence and applies the
//                  epilogue.  A periodic row of <= 256 cells is one segment,
//                  so every face and every cell is computed exactly once.
//  k_sweep_tile    sweep along y or z (strided) for grids with many lines:
//                  a workgroup takes TX adjacent x columns of one line and
//                  walks it in chunks, each chunk a row sweep of a strided
//                  tile staged in LDS.
//  k_sweep_march   sweep along y or z (strided).  Each lane owns one x
//                  column (coalesced 512-byte rows per wave; the block's
//                  wavefronts take consecutive (line, segment) units) and marches
//                  along the axis over a segment of cells, keeping the face's
//                  K cells in an LDS ring and carrying the previous face
//                  flux in registers.  The next face's new cell and the
//                  epilogue operands of the cell being closed are loaded
//                  before the face is computed, so their latency hides
//                  behind it.  M cells cost M+1 faces.
//
// Sweep epilogues (divergence -dF/dx of the axis, then):
//  STORE  R = div                      ACCUM  R += div
//  RK     Uout = a U0 + b (Us + dt (R + div))      RK1   Uout = a U0 + b (Us + dt div)
// where Us is the stage state the stencils read (p.U); the kernels take it
// from their LDS copy of the cell instead of reading HBM again.
#pragma once

#include "teno_device.h"

namespace tenom {

enum : int { EPI_STORE = 0, EPI_ACCUM = 1, EPI_RK = 2, EPI_RK1 = 3 };

template <int NF>
struct SweepParams {
  const double* U;   // state the stencils read
  double* R;         // divergence accumulator (STORE/ACCUM write, RK reads)
  const double* U0;  // RK: U^n
  double* Uout;      // RK: output state
  double a, b, dt;   // RK coefficients
  const double* dtp; // if not NULL: dt is read from this device address instead
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

// Operands the epilogue reads from HBM: R (ACCUM, RK) and U^n (RK with
// a != 0).  Loaded by epi_load so that a caller can issue them early.
template <int NF>
struct EpiIn {
  double r[NF], u0[NF];
};

template <int NF>
__device__ __forceinline__ void epi_load(const SweepParams<NF>& p, long N, long cell, EpiIn<NF>& in) {
#pragma unroll
  for (int q = 0; q < NF; ++q) {
    const long o = (long)p.fld[q] * N + cell;
    in.r[q] = (p.mode == EPI_ACCUM || p.mode == EPI_RK) ? p.R[o] : 0.0;
    in.u0[q] = (p.mode >= EPI_RK && p.a != 0.0) ? p.U0[o] : 0.0;
  }
}

// The step size of the RK modes, read once per thread.
template <int NF>
__device__ __forceinline__ double epi_dt(const SweepParams<NF>& p) {
  return p.dtp ? *p.dtp : p.dt;
}

// us: the cell's stage state (rotated components), only used by RK modes
template <int NF>
__device__ __forceinline__ void epi_store(const SweepParams<NF>& p, long N, long cell, const double (&div)[NF],
                                          const EpiIn<NF>& in, const double (&us)[NF], double dt) {
#pragma unroll
  for (int q = 0; q < NF; ++q) {
    const long o = (long)p.fld[q] * N + cell;
    if (p.mode == EPI_STORE) {
      p.R[o] = div[q];
    } else if (p.mode == EPI_ACCUM) {
      p.R[o] = in.r[q] + div[q];
    } else {
      const double rhs = (p.mode == EPI_RK) ? in.r[q] + div[q] : div[q];
      const double v = fma(dt, rhs, us[q]);
      p.Uout[o] = (p.a != 0.0) ? fma(p.a, in.u0[q], p.b * v) : p.b * v;
    }
  }
}

// ---------------------------------------------------------------------------
template <int NF, int K, int LIM, bool ADAPT>
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
  GlobalCells<NF, K> prov{U, N, fld, L, j, fp.gamma};
  double F[NF];
  uint32_t bits[2][NF];
  if (flags) {
    face_flux<NF, K, LIM, ADAPT, true>(prov, fp, F, bits);
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      flags[(long)q * nfaces + t] = (uint8_t)bits[0][q];
      flags[(long)(NF + q) * nfaces + t] = (uint8_t)bits[1][q];
    }
  } else {
    face_flux<NF, K, LIM, ADAPT, false>(prov, fp, F, bits);
  }
#pragma unroll
  for (int q = 0; q < NF; ++q) Fhat[(long)fld[q] * nfaces + t] = F[q];
}

// ---------------------------------------------------------------------------
// Row sweep.  Cells of the segment (plus K-1 halo cells) are staged once in
// LDS together with their physical flux, signal speed and Roe inputs, so a
// face reads its K cells instead of recomputing them.
// ---------------------------------------------------------------------------
template <int NF>
struct RowStage {
  static constexpr int NE = (NF == 1) ? 1 : 3 * NF + 1;  // U, F, lambda, Roe input
};

// CS: staging-index step between consecutive cells of the sweep axis (1 in
// the row sweep, the tile width in the tile sweep).  REREAD: the Euler face
// projects its stencil group by group of fields from fresh reads of the
// cells and lets wavefronts whose candidates are all smooth skip the limiter
// (worth it where most wavefronts see only smooth data: the tile sweep's
// 8 x 8 patches of faces, which a discontinuity crosses far less often than
// the row sweep's strips of 64, and the batched 1D problems' constant
// states).
template <int NF, int K, int CS = 1, bool REREAD = false>
struct StagedCells {
  static constexpr bool kReread = REREAD;  // the face reads the cells again per group of fields
  const double* s;  // LDS: [NE][NC]
  int nc;           // row pitch of the staging array
  int c0;           // staging index of window cell 0
  __device__ __forceinline__ double at(int e, int c) const { return s[e * nc + c]; }
  // the same provider, its position hidden from the compiler, so that reads
  // through it are not merged with earlier reads of the same cells
  __device__ __forceinline__ StagedCells fresh() const {
    int c = c0;
    asm volatile("" : "+v"(c));
    return StagedCells<NF, K, CS, REREAD>{s, nc, c};
  }
  __device__ __forceinline__ void state_flux(int m, double (&X)[NF], double (&F)[NF]) const {
    const int c = c0 + m * CS;
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      X[q] = at(q, c);
      F[q] = at(NF + q, c);
    }
  }
  __device__ __forceinline__ double speed(int m) const { return at(2 * NF, c0 + m * CS); }
  __device__ __forceinline__ void cell(int m, double (&X)[NF], double (&F)[NF], double& lam) const {
    const int c = c0 + m * CS;
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      X[q] = at(q, c);
      F[q] = at(NF + q, c);
    }
    lam = at(2 * NF, c);
  }
  __device__ __forceinline__ void roe(int sd, RoeIn<NF>& r) const {
    const int c = c0 + (K / 2 - 1 + sd) * CS;
    r.rs = at(2 * NF + 1, c);
#pragma unroll
    for (int d = 0; d < NF - 2; ++d) r.u[d] = at(2 * NF + 2 + d, c);
    r.H = at(3 * NF, c);
  }
  __device__ __forceinline__ double value(int m) const { return at(0, c0 + m * CS); }
};

// Stage cell `cell` of the grid at staging index c: its state and, for the
// Euler equations, its flux, signal speed and Roe inputs.
template <int NF>
__device__ __forceinline__ void stage_cell(double* stage, int nc, int c, const SweepParams<NF>& p, long N, long cell) {
  double X[NF];
#pragma unroll
  for (int q = 0; q < NF; ++q) X[q] = p.U[p.fld[q] * N + cell];
#pragma unroll
  for (int q = 0; q < NF; ++q) stage[q * nc + c] = X[q];
  if constexpr (NF > 1) {
    double F[NF], lam;
    RoeIn<NF> r;
    cell_physics<NF>(X, p.fp.gamma, F, lam);
    roe_input<NF>(X, p.fp.gamma, r);
#pragma unroll
    for (int q = 0; q < NF; ++q) stage[(NF + q) * nc + c] = F[q];
    stage[(2 * NF) * nc + c] = lam;
    stage[(2 * NF + 1) * nc + c] = r.rs;
#pragma unroll
    for (int d = 0; d < NF - 2; ++d) stage[(2 * NF + 2 + d) * nc + c] = r.u[d];
    stage[(3 * NF) * nc + c] = r.H;
  }
}

// Waves per SIMD the row and tile sweeps are compiled for: three where the
// face fits in 168 VGPRs without spilling (six points), two at eight points
// (at most 256 VGPRs; every eight-point variant fits without spilling).
template <int NF, int K>
struct RowOccupancy {
  static constexpr int WAVES = (K == 6) ? 3 : 2;
};

template <int NF, int K, int LIM, bool ADAPT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RowOccupancy<NF, K>::WAVES)))
void k_sweep_row(SweepParams<NF> p) {
  constexpr int NC = 256 + K - 1;  // staged cells per segment
  constexpr int NE = RowStage<NF>::NE;
  __shared__ double stage[NE * NC];
  const int s = blockIdx.x % p.nseg;
  const long row = blockIdx.x / p.nseg;  // y + ny * z
  const int c_begin = s * p.seg;
  const int ncell = min(p.seg, p.n - c_begin);
  const bool wrap = (p.bc == 0) && (p.seg >= p.n);  // whole periodic row
  const int nface = wrap ? p.n : ncell + 1;
  const int nstage = nface + K - 1;
  const long N = (long)p.nx * p.ny * p.nz;
  const Line L{row * p.nx, 1, p.n, p.bc};
  const int t = threadIdx.x;
  // wave priority: high while the wave issues its global loads and stores
  // (staging, epilogue), normal while it computes faces, so that a block's
  // memory phase is not queued behind other blocks' arithmetic on the SIMD
  __builtin_amdgcn_s_setprio(3);

  // stage cells c_begin - K/2 .. c_begin + nface + K/2 - 2
  for (int c = t; c < nstage; c += 256) stage_cell<NF>(stage, NC, c, p, N, cell_at(L, c_begin - K / 2 + c));
  __syncthreads();

  double F[NF];
  __builtin_amdgcn_s_setprio(0);
  if (t < nface) {
    StagedCells<NF, K> prov{stage, NC, t};
    uint32_t bits[2][NF];
    face_flux<NF, K, LIM, ADAPT, false>(prov, p.fp, F, bits);
  }
  // stage state of this thread's cell (staged at t + K/2), copied before the
  // staging array is reused
  double us[NF];
  if (t < ncell) {
#pragma unroll
    for (int q = 0; q < NF; ++q) us[q] = stage[q * NC + t + K / 2];
  }
  __syncthreads();  // every face has read the staged cells
  double* Fs = stage;  // reuse: [NF][257]
  if (t < nface) {
#pragma unroll
    for (int q = 0; q < NF; ++q) Fs[q * 257 + t] = F[q];
  }
  __syncthreads();
  __builtin_amdgcn_s_setprio(3);
  if (t < ncell) {
    const long cell = L.base + c_begin + t;
    EpiIn<NF> ein;
    epi_load<NF>(p, N, cell, ein);
    const int r = (wrap && t == p.n - 1) ? 0 : t + 1;
    double div[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) div[q] = (Fs[q * 257 + t] - Fs[q * 257 + r]) * p.inv_dx;
    epi_store<NF>(p, N, cell, div, ein, us, epi_dt(p));
  }
}

// ---------------------------------------------------------------------------
// Tile sweep (any axis).  A 256-thread workgroup owns TX adjacent lines
// along the axis (x columns for y and z, y rows for x) and walks them whole
// in chunks of FJ = 256 / TX faces per line.  Each chunk is a row sweep on a
// tile: its cells are staged in LDS (row r of the chunk at staging indices
// r TX .. r TX + TX - 1) with their flux, signal speed and Roe inputs, each
// thread computes one face, the fluxes go through LDS and each thread closes
// the cell left of its face.  The last face of a chunk is handed to the next
// chunk through LDS and face 0 of a periodic line is kept for its last cell,
// so a line of M cells costs M faces (M + 1 when transmissive); only the
// K - 1 halo rows of each chunk are staged twice.  A wavefront's 64 faces
// form an 8 x 8 patch (8 lines by 8 faces), which a discontinuity crosses
// far less often than a strip of 64 faces along one line: most wavefronts
// then skip the limiter (StagedCells with REREAD).
// ---------------------------------------------------------------------------
constexpr int kTileColumns = 8;  // columns (lines side by side) per tile-sweep workgroup

// Workgroups of a tile sweep along `axis`: the lines of the other axis times
// the column groups (x columns for y and z, y rows for x).
inline long tile_count(int axis, int nx, int ny, int nz) {
  const long lines = (axis == 2) ? ny : nz;
  const int across = (axis == 0) ? ny : nx;
  return lines * ((across + kTileColumns - 1) / kTileColumns);
}

template <int NF, int K>
struct SweepTile {
  static constexpr int TX = kTileColumns;
  static constexpr int FJ = 256 / TX;    // faces per column per chunk
  static constexpr int ROWS = FJ + K - 1;  // staged cells per column per chunk
};

template <int NF, int K, int LIM, bool ADAPT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RowOccupancy<NF, K>::WAVES)))
void k_sweep_tile(SweepParams<NF> p, int axis) {
  using S = SweepTile<NF, K>;
  constexpr int TX = S::TX, FJ = S::FJ;
  constexpr int NC = S::ROWS * TX;
  constexpr int NE = RowStage<NF>::NE;
  static_assert(256 % TX == 0, "whole columns per workgroup");
  __shared__ double stage[NE * NC];
  __shared__ double Fb[NF * FJ * TX];  // face f of the chunk at row f
  __shared__ double Fc[2 * NF * TX];   // last face of chunk k at [k mod 2], for the next chunk
  __shared__ double Fw[NF * TX];       // face 0 of a periodic line, the right face of its last cell
  // tiles in XCD order: blocks b, b + 8, ... run on one XCD and take
  // consecutive tiles, so the column groups of a line share that XCD's L2
  const int nb = (int)gridDim.x, b = (int)blockIdx.x;
  const int xcd = b & 7, q8 = nb >> 3, r8 = nb & 7;
  const int tile = xcd * q8 + min(xcd, r8) + (b >> 3);
  // column groups: x columns for y and z, y rows for x
  const int ncg = ((axis == 0 ? p.ny : p.nx) + TX - 1) / TX;
  const int o = tile / ncg;  // z of an x or y line, y of a z line
  const long N = (long)p.nx * p.ny * p.nz;
  const bool wrap = p.bc == 0;
  const int nface = wrap ? p.n : p.n + 1;  // face j lies between cells j - 1 and j
  const int nchunk = (nface + FJ - 1) / FJ;
  // A periodic x line is walked from its cell 1 (cell m of the walk is cell
  // m + 1 of the line, the last one cell 0): a chunk then closes 32
  // consecutive cells that start on a cache-line boundary, and writes them
  // whole.  On a ring every face has the same stencil either way, so the
  // fluxes and the results have the same bits.
  const int rot = (axis == 0 && wrap) ? 1 : 0;
  // Phases of a chunk, each ended by a barrier: staging; faces (their
  // fluxes into LDS); closing the cells, which reads the staged cells and
  // the fluxes from LDS.  No value is held in registers across a barrier.
  // The thread's column and line address are formed anew in each phase from
  // an opaque copy of the thread index: hoisted out of the loop they would
  // hold registers through the face computation.
  struct Where {
    int col, f;
    bool in;
    Line L;
  };
  auto where = [&]() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    Where w;
    w.col = t % TX;
    w.f = t / TX;
    const int c = (tile % ncg) * TX + w.col;
    const int nc = axis == 0 ? p.ny : p.nx;
    w.in = c < nc;
    const int cs = w.in ? c : nc - 1;  // columns beyond the grid stage a real line and store nothing
    if (axis == 0)
      w.L = Line{((long)cs + (long)p.ny * o) * p.nx, 1, p.nx, p.bc};
    else if (axis == 1)
      w.L = Line{cs + (long)p.nx * p.ny * o, p.nx, p.ny, p.bc};
    else
      w.L = Line{cs + (long)p.nx * o, (long)p.nx * p.ny, p.nz, p.bc};
    return w;
  };
  for (int k = 0; k < nchunk; ++k) {
    const int j0 = k * FJ;
    const int nfk = min(FJ, nface - j0);  // faces of this chunk per column
    __builtin_amdgcn_s_setprio(3);
    {
      const Where w = where();
      for (int r = w.f; r < nfk + K - 1; r += FJ)
        stage_cell<NF>(stage, NC, r * TX + w.col, p, N, cell_at(w.L, j0 - K / 2 + r + rot));
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);
    {
      const Where w = where();
      const int f = w.f, col = w.col, j = j0 + f;
      if (f < nfk) {
        double F[NF];
        StagedCells<NF, K, TX, true> prov{stage, NC, f * TX + col};
        uint32_t bits[2][NF];
        face_flux<NF, K, LIM, ADAPT, false>(prov, p.fp, F, bits);
#pragma unroll
        for (int q = 0; q < NF; ++q) Fb[(q * FJ + f) * TX + col] = F[q];
        if (f == FJ - 1) {
#pragma unroll
          for (int q = 0; q < NF; ++q) Fc[((k & 1) * NF + q) * TX + col] = F[q];
        }
        if (wrap && j == 0) {
#pragma unroll
          for (int q = 0; q < NF; ++q) Fw[q * TX + col] = F[q];
        }
      }
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(3);
    {
      // this thread closes cell j - 1 and, on a periodic line, the last cell
      // (right of the last face) with face 0 as its right face.  The
      // epilogue's parameters are read anew through an opaque pointer to the
      // argument: held from the kernel's start they would be spilled across
      // the face and read back lane by lane.
      long off = 0;
      asm volatile("" : "+s"(off));
      const SweepParams<NF>& pe = *(const SweepParams<NF>*)((const char*)&p + off);
      const Where w = where();
      const int f = w.f, col = w.col, j = j0 + f;
      const bool act = f < nfk && w.in;
      if (act && j >= 1) {
        const long cell = w.L.base + (long)(j - 1 + rot) * w.L.stride;
        EpiIn<NF> ein;
        epi_load<NF>(pe, N, cell, ein);
        double us[NF], div[NF];
#pragma unroll
        for (int q = 0; q < NF; ++q) {
          us[q] = stage[q * NC + (f + K / 2 - 1) * TX + col];
          const double fl = f > 0 ? Fb[(q * FJ + f - 1) * TX + col] : Fc[(((k - 1) & 1) * NF + q) * TX + col];
          div[q] = (fl - Fb[(q * FJ + f) * TX + col]) * pe.inv_dx;
        }
        epi_store<NF>(pe, N, cell, div, ein, us, epi_dt(pe));
      }
      if (wrap && act && j == nface - 1) {
        const long cell = w.L.base + (long)(rot ? 0 : j) * w.L.stride;
        EpiIn<NF> ein;
        epi_load<NF>(pe, N, cell, ein);
        double us[NF], div[NF];
#pragma unroll
        for (int q = 0; q < NF; ++q) {
          us[q] = stage[q * NC + (f + K / 2) * TX + col];
          div[q] = (Fb[(q * FJ + f) * TX + col] - Fw[q * TX + col]) * pe.inv_dx;
        }
        epi_store<NF>(pe, N, cell, div, ein, us, epi_dt(pe));
      }
    }
    __syncthreads();  // the next chunk's staging overwrites the cells read here
  }
}

// ---------------------------------------------------------------------------
// March sweep (axis 1 or 2).  blockDim = (64, LINES): x = lane, y = line.
// Each lane keeps the K cell states of its current face in an LDS ring
// (slot of window cell m: (slot0 + m) mod K) and fetches the one new cell of
// the next face while the current face is computed.
// ---------------------------------------------------------------------------
template <int NF>
struct RoeCarry {
  RoeIn<NF> r;
};
template <>
struct RoeCarry<1> {};

template <int NF, int K>
struct RingCells {
  static constexpr bool kReread = false;  // the cell flux is recomputed per read
  // values per ring slot: the cell's state and, for the Euler equations, its
  // signal speed (computed once, when the cell enters the window)
  static constexpr int NR = (NF > 1) ? NF + 1 : NF;
  const double* ring;  // LDS: [K][NR][T] with T threads per block
  int T, tid, slot0;
  double gamma;
  RoeCarry<NF>* carry;  // Roe input of the face's right cell, the next face's left
  __device__ __forceinline__ int slot(int m) const {
    const int sl = slot0 + m;
    return sl >= K ? sl - K : sl;
  }
  __device__ __forceinline__ void load(int m, double (&X)[NF]) const {
    const int sl = slot(m);
#pragma unroll
    for (int q = 0; q < NF; ++q) X[q] = ring[(sl * NR + q) * T + tid];
  }
  __device__ __forceinline__ void cell(int m, double (&X)[NF], double (&F)[NF], double& lam) const {
    load(m, X);
    cell_flux<NF>(X, cell_prim<NF>(X, gamma), gamma, F);
    lam = ring[(slot(m) * NR + NF) * T + tid];
  }
  __device__ __forceinline__ void roe(int s, RoeIn<NF>& r) const {
    if (s == 0) {
      r = carry->r;
    } else {
      double X[NF];
      load(K / 2, X);
      roe_input<NF>(X, gamma, r);
      carry->r = r;
    }
  }
  __device__ __forceinline__ double value(int m) const { return ring[slot(m) * NR * T + tid]; }
};

// Store a cell into ring slot sl (state, and the signal speed for Euler).
template <int NF, int K>
__device__ __forceinline__ void ring_put(double* ring, int T, int tid, int sl, const double (&X)[NF], double gamma) {
  constexpr int NR = RingCells<NF, K>::NR;
#pragma unroll
  for (int q = 0; q < NF; ++q) ring[(sl * NR + q) * T + tid] = X[q];
  if constexpr (NF > 1) ring[(sl * NR + NF) * T + tid] = cell_speed<NF>(cell_prim<NF>(X, gamma), gamma);
}

template <int NF, int K>
struct MarchShape {
  // lines per block: 4, or 2 when the ring of 4 lines would exceed 80 KiB
  // (two blocks per CU must fit in its 160 KiB of LDS)
  static constexpr int LINES = (K * RingCells<NF, K>::NR * 8 * 64 * 4 <= 81920) ? 4 : 2;
};

template <int NF, int K, int LIM, bool ADAPT>
__global__ __launch_bounds__((64 * MarchShape<NF, K>::LINES)) void k_sweep_march(SweepParams<NF> p, int axis) {
  constexpr int LINES = MarchShape<NF, K>::LINES;
  constexpr int T = 64 * LINES;
  __shared__ double ring[K * RingCells<NF, K>::NR * T];
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int n_other = (axis == 1) ? p.nz : p.ny;
  // unit u = (line o of the other axis, segment s), o fastest: a 2D grid
  // (one other line) still fills every wavefront of the block
  const long u = ((long)blockIdx.z * gridDim.y + blockIdx.y) * LINES + threadIdx.y;
  if (x >= p.nx || u >= (long)n_other * p.nseg) return;  // no block-wide barrier follows
  const int o = (int)(u % n_other);
  const int s = (int)(u / n_other);
  const int tid = threadIdx.y * 64 + threadIdx.x;
  const long N = (long)p.nx * p.ny * p.nz;
  Line L;
  if (axis == 1)
    L = Line{x + (long)p.nx * p.ny * o, p.nx, p.ny, p.bc};
  else
    L = Line{x + (long)p.nx * o, (long)p.nx * p.ny, p.nz, p.bc};
  const int c_begin = s * p.seg;
  const int ncell = min(p.seg, p.n - c_begin);
  // faces c_begin .. c_begin + ncell; on a whole periodic line face n reads
  // the same wrapped cells as face 0, so its flux is recomputed bit for bit

  auto fetch = [&](int pos, double (&X)[NF]) {
    const long cell = cell_at(L, pos);
#pragma unroll
    for (int q = 0; q < NF; ++q) X[q] = p.U[p.fld[q] * N + cell];
  };
  // window of the first face
#pragma unroll
  for (int m = 0; m < K; ++m) {
    double X[NF];
    fetch(c_begin - K / 2 + m, X);
    ring_put<NF, K>(ring, T, tid, m, X, p.fp.gamma);
  }
  int slot0 = 0;
  RoeCarry<NF> carry;  // the first face's left cell; then handed on face to face
  if constexpr (NF > 1) {
    double X[NF];
    RingCells<NF, K>{ring, T, tid, 0, p.fp.gamma, nullptr}.load(K / 2 - 1, X);
    roe_input<NF>(X, p.fp.gamma, carry.r);
  }
  // six points: dt read once and held in a vector register.  The loop is
  // short of scalar registers, and a scalar copy spills into lanes that every
  // iteration reads back; the eight-point loop, short of vector registers
  // instead, reads it at each store.
  double dt = epi_dt(p);
  if constexpr (K == 6) asm volatile("" : "+v"(dt));
  double Fprev[NF];
  for (int t = 0; t <= ncell; ++t) {
    const int j = c_begin + t;
    const bool more = (t < ncell);
    double nxt[NF];
    __builtin_amdgcn_s_setprio(3);  // high while loads and stores issue, as in the row sweep
    if (more) fetch(j + K / 2, nxt);  // the new cell of face j + 1
    const long ecell = L.base + (long)(j - 1) * L.stride;  // cell closed by face j
    EpiIn<NF> ein;
    double us[NF];
    if (t > 0) epi_load<NF>(p, N, ecell, ein);
    double F[NF];
    __builtin_amdgcn_s_setprio(0);
    {
      RingCells<NF, K> prov{ring, T, tid, slot0, p.fp.gamma, &carry};
      prov.load(K / 2 - 1, us);  // cell j - 1 is window cell K/2 - 1 of face j
      uint32_t bits[2][NF];
      face_flux<NF, K, LIM, ADAPT, false>(prov, p.fp, F, bits);
    }
    __builtin_amdgcn_s_setprio(3);
    if (more) {
      ring_put<NF, K>(ring, T, tid, slot0, nxt, p.fp.gamma);
      slot0 = (slot0 + 1 == K) ? 0 : slot0 + 1;
    }
    if (t > 0) {
      double div[NF];
#pragma unroll
      for (int q = 0; q < NF; ++q) div[q] = (Fprev[q] - F[q]) * p.inv_dx;
      epi_store<NF>(p, N, ecell, div, ein, us, K == 6 ? dt : epi_dt(p));
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
  double* Uout;
  double a, b, dt;
  const double* dtp;  // device dt (NULL: use dt)
  int mode;
  int nx, ny, nz, bc;
  double inv_dx;
  int seg;  // cells per segment along the axis (march sweeps)
  int fld[5];
  FaceParams fp;
  hipStream_t stream;
};

template <int NF, int K, int LIM, bool ADAPT>
hipError_t launch_faces(const FacesLaunch& a) {
  const long nfaces = (long)(a.nx + (a.axis == 0)) * (a.ny + (a.axis == 1)) * (a.nz + (a.axis == 2));
  const unsigned blocks = (unsigned)((nfaces + 255) / 256);
  hipLaunchKernelGGL((k_faces<NF, K, LIM, ADAPT>), dim3(blocks), dim3(256), 0, a.stream, a.U, a.Fhat, a.flags, a.axis,
                     a.nx, a.ny, a.nz, a.bc, a.fld[0], a.fld[1], a.fld[2], a.fld[3], a.fld[4], a.fp);
  return hipGetLastError();
}

template <int NF, int K, int LIM, bool ADAPT>
hipError_t launch_sweep(const SweepLaunch& a) {
  SweepParams<NF> p;
  p.U = a.U;
  p.R = a.R;
  p.U0 = a.U0;
  p.Uout = a.Uout;
  p.a = a.a;
  p.b = a.b;
  p.dt = a.dt;
  p.dtp = a.dtp;
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
    hipLaunchKernelGGL((k_sweep_row<NF, K, LIM, ADAPT>), dim3((unsigned)blocks), dim3(256), 0, a.stream, p);
  } else {
    p.n = (a.axis == 1) ? a.ny : a.nz;
    p.seg = a.seg >= p.n ? p.n : a.seg;
    p.nseg = (p.n + p.seg - 1) / p.seg;
    const int n_other = (a.axis == 1) ? a.nz : a.ny;
    constexpr int LINES = MarchShape<NF, K>::LINES;
    const long ub = ((long)n_other * p.nseg + LINES - 1) / LINES;  // blocks of units per x group
    const long gy = ub < 65535 ? ub : 65535;
    dim3 grid((a.nx + 63) / 64, (unsigned)gy, (unsigned)((ub + gy - 1) / gy));
    hipLaunchKernelGGL((k_sweep_march<NF, K, LIM, ADAPT>), grid, dim3(64, LINES), 0, a.stream, p, a.axis);
  }
  return hipGetLastError();
}

// Tile sweep of axis 1 or 2: one workgroup per (line, group of TX columns).
template <int NF, int K, int LIM, bool ADAPT>
hipError_t launch_tile(const SweepLaunch& a) {
  SweepParams<NF> p;
  p.U = a.U;
  p.R = a.R;
  p.U0 = a.U0;
  p.Uout = a.Uout;
  p.a = a.a;
  p.b = a.b;
  p.dt = a.dt;
  p.dtp = a.dtp;
  p.mode = a.mode;
  p.nx = a.nx;
  p.ny = a.ny;
  p.nz = a.nz;
  p.bc = a.bc;
  p.inv_dx = a.inv_dx;
  p.fp = a.fp;
  for (int q = 0; q < NF; ++q) p.fld[q] = a.fld[q];
  if (a.axis < 0 || a.axis > 2) return hipErrorInvalidValue;
  p.n = (a.axis == 0) ? a.nx : (a.axis == 1) ? a.ny : a.nz;
  p.seg = p.n;
  p.nseg = 1;
  const long tiles = tile_count(a.axis, a.nx, a.ny, a.nz);
  hipLaunchKernelGGL((k_sweep_tile<NF, K, LIM, ADAPT>), dim3((unsigned)tiles), dim3(256), 0, a.stream, p, a.axis);
  return hipGetLastError();
}

}  // namespace tenom
