// Index geometry of a tile and of the staged streaming kernels, shared by
// the kernels and by the host-side bounds check in the tests.
#pragma once

#include <hip/hip_runtime.h>

namespace fmm {

// A tile of edge E in LDS: its E^3 interior cells inside an (E+2)^3 block
// whose outer layer holds the face halos (the 7-point stencil never reads
// the block's edges and corners).  dom() is the block index of interior
// coordinates (-1 and E address the halo), domp() that of interior index p
// (axis 2 fastest).
template <int E> struct Geo {
    static constexpr int D = E + 2;          // tile plus one-point halo per side
    static constexpr int DV = D * D * D;
    static constexpr int V = E * E * E;      // interior points
    static constexpr int K = (V + 63) / 64;  // interior points per lane in a one-wavefront scan
    static constexpr int FACE = E * E;
    static constexpr int OX = D * D, OY = D, OZ = 1;
    static constexpr int LOG = (E == 4) ? 2 : (E == 8) ? 3 : 4;
    __host__ __device__ static constexpr int dom(int i0, int i1, int i2) { return ((i0 + 1) * D + (i1 + 1)) * D + (i2 + 1); }
    __host__ __device__ static constexpr int domp(int p) { return dom(p >> (2 * LOG), (p >> LOG) & (E - 1), p & (E - 1)); }
    // candidate bytes of a one-wavefront group: one per interior cell, then
    // one spare dword per lane, which a lane that does not mark writes
    // instead (so a mark is a store under no lane mask, in distinct banks)
    static constexpr int CFB = V + 4 * 64;
    __host__ __device__ static constexpr int spare(int lane) { return V + 4 * lane; }
};


// Coordinates of halo cell (face f, in-face position u, w): face f = 2*axis +
// (1 for the + side); the in-face coordinates follow the other two axes in order.
template <int E> __host__ __device__ inline void face_cell(int f, int u, int w, int &c0, int &c1, int &c2)
{
    const int ax = f >> 1;
    const int hc = (f & 1) ? E : -1;
    c0 = ax == 0 ? hc : u;
    c1 = ax == 0 ? u : (ax == 1 ? hc : w);
    c2 = ax == 2 ? hc : w;
}

// The interior cell adjacent to a halo cell of face f.
template <int E> __host__ __device__ inline void face_inner(int f, int &c0, int &c1, int &c2)
{
    const int ax = f >> 1;
    const int ic = (f & 1) ? E - 1 : 0;
    if (ax == 0) c0 = ic;
    else if (ax == 1) c1 = ic;
    else c2 = ic;
}

// LDS-staged conversion between a row-major grid and the tiled layout.  A
// work unit is an E x E bundle of grid rows (one tile row along axes 0 and 1)
// over a chunk of CH consecutive tiles along axis 2.  Those CH tiles are
// consecutive in the tiled layout, so the tiled side of a unit is one
// contiguous run of CH * V values and the row-major side is E * E row pieces
// of CH * E contiguous values: both sides stream in long runs.  Tiles are E
// values apart in LDS beyond their V values, which puts the E row pieces of a
// wavefront's 64 consecutive columns in distinct banks.
constexpr int STAGE_THREADS = 256;
constexpr int STAGE_BATCH = 8;  // loads a thread keeps in flight
template <int E, typename T> struct Stage {
    static constexpr int V = E * E * E;
    static constexpr int CH = E == 16 ? (sizeof(T) == 8 ? 2 : 4) : E == 8 ? (sizeof(T) == 8 ? 8 : 16) : 32;
    static constexpr int W = CH * E;  // columns of a row piece
    static constexpr int R = E * E;   // row pieces of a unit
    static constexpr int TS = V + E;  // LDS stride of one tile
};

}  // namespace fmm
