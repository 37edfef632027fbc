// D3Q19 lattice constants and index geometry shared by the kernels and the
// host runtime of the Shan-Chen evaporation library.
//
// Direction order (the paper fixes only the weights, Sec. II A): 0 rest,
// 1..6 = +x,-x,+y,-y,+z,-z, 7..18 the twelve face diagonals with opposites
// adjacent. Weights w_0 = 1/3, w_1..6 = 1/18, w_7..18 = 1/36; c_s^2 = 1/3.
#pragma once

#include <cstdint>

#ifndef LBSC_HD
#define LBSC_HD __host__ __device__ __forceinline__
#endif

namespace lbsc {

constexpr int kQ = 19;

// Velocity components packed per direction; kept as constexpr functions so
// fully unrolled device loops see compile-time constants.
LBSC_HD constexpr int ex(int i)
{
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
         : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
}
LBSC_HD constexpr int ey(int i)
{
    return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
         : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
}
LBSC_HD constexpr int ez(int i)
{
    return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
         : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
}
LBSC_HD constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
LBSC_HD constexpr double wgt(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

// Sink geometry kinds (mirrors the public enum values).
enum SinkKind : int32_t { kSinkNone = 0, kSinkZmax = 1, kSinkFaces = 2, kSinkSphere = 3 };

struct Sink {
    int32_t kind;
    int32_t no_zlo;   // faces sink without its z = 0 face (a solid wall lies below)
    double rho_h;     // density imposed on component A
    double r2;        // squared radius of a spherical sink
    double cx, cy, cz;
};

LBSC_HD bool in_sink(const Sink& s, int x, int y, int z, int nx, int ny, int nz)
{
    switch (s.kind) {
    case kSinkZmax: return z == nz - 1;
    case kSinkFaces:
        return x == 0 || y == 0 || (z == 0 && !s.no_zlo) || x == nx - 1 || y == ny - 1 || z == nz - 1;
    case kSinkSphere: {
        double dx = x - s.cx, dy = y - s.cy, dz = z - s.cz;
        return dx * dx + dy * dy + dz * dz >= s.r2;
    }
    default: return false;
    }
}

// Fluid z range of the column (x, y): nodes (x, y, z) with lo <= z <= hi lie
// outside the sink, every other node of the column inside it. For all sink
// kinds the fluid part of a column is one interval (for the sphere the
// computed distance is monotone in |z - cz|), found here from a continuous
// estimate and settled with the exact test of in_sink. Packed as
// lo | hi << 16; an all-sink column is lo = 1, hi = 0.
LBSC_HD uint32_t sink_zrange(const Sink& s, int x, int y, int nx, int ny, int nz)
{
    int lo = 0, hi = nz - 1;
    switch (s.kind) {
    case kSinkZmax: hi = nz - 2; break;
    case kSinkFaces:
        lo = s.no_zlo ? 0 : 1;
        hi = nz - 2;
        if (x == 0 || y == 0 || x == nx - 1 || y == ny - 1) hi = lo - 1;
        break;
    case kSinkSphere: {
        const double dx = x - s.cx, dy = y - s.cy;
        const double rem = s.r2 - (dx * dx + dy * dy);
        const double h = rem > 0 ? sqrt(rem) : 0.0;
        double zl = ceil(s.cz - h), zh = floor(s.cz + h);
        zl = zl < 0 ? 0 : (zl > nz - 1 ? nz - 1 : zl);
        zh = zh < 0 ? 0 : (zh > nz - 1 ? nz - 1 : zh);
        lo = (int)zl;
        hi = (int)zh;
        if (lo > hi) {
            double zc = floor(s.cz + 0.5);
            zc = zc < 0 ? 0 : (zc > nz - 1 ? nz - 1 : zc);
            lo = hi = (int)zc;
        }
        while (lo <= hi && in_sink(s, x, y, lo, nx, ny, nz)) ++lo;
        while (hi >= lo && in_sink(s, x, y, hi, nx, ny, nz)) --hi;
        if (lo > hi) {
            lo = 1;
            hi = 0;
            break;
        }
        while (lo > 0 && !in_sink(s, x, y, lo - 1, nx, ny, nz)) --lo;
        while (hi < nz - 1 && !in_sink(s, x, y, hi + 1, nx, ny, nz)) ++hi;
        break;
    }
    default: break;
    }
    // A column with no fluid node (a one-plane lattice under a z-max or
    // face sink) takes the all-sink encoding.
    if (hi < lo) {
        lo = 1;
        hi = 0;
    }
    return (uint32_t)lo | ((uint32_t)hi << 16);
}

LBSC_HD bool in_zrange_sink(uint32_t zr, int z) { return z < (int)(zr & 0xffffu) || z > (int)(zr >> 16); }

// Per-instance description, stored in device memory.
// A lattice with a solid wall of h planes at its bottom is described to the
// kernels by its fluid part alone: nz - h planes starting h slabs into the
// instance's storage, with the seam wall on both ends (below the first fluid
// plane and, through the periodic wrap, above the last) and psi_wall = 1, the
// solid nodes' constant psi in place of the seam's mirror. z_off = h maps its
// planes back to the caller's lattice.
struct Inst {
    int32_t nx, ny, nz, wall_z;
    int32_t psi_exp;       // 0: psi = rho, 1: psi = 1 - exp(-rho)
    int32_t count_reset;   // 0: the next pull-time reset is not booked into E
    int64_t n;             // nodes
    int64_t ps;            // elements per (c, i) plane of one z-slab (nx*ny, padded)
    int64_t slab;          // elements per z-slab: 2*19 planes
    int64_t base;          // element offset of this instance in the arena
    double tau[2];
    double omega[2];       // 1 / tau
    double g;
    // FP32 copies for the FP32-arithmetic kernels, formed on the host in
    // FP32 exactly as the kernels would (they stay in scalar registers):
    float shift_f[2], omega_f[2];
    float ntg_f[2];        // -tau^c * g, one FP32 product
    double shift[2];       // rho0^c of shifted storage (0 for plain FP64)
    double phi_in, phi_out;
    Sink reset;            // sink that formed the stored state (applied on pull)
    Sink cur;              // current sink (its nodes skip collision)
    int32_t item_begin, item_end;   // this instance's work items
    int32_t psi_wall;      // 1: psi beyond the wall is psi_w (solid nodes), 0: mirrored
    int32_t z_off;         // solid planes below the kernels' lattice
    int32_t ncomp;         // components: 2, or 1 (single-component multiphase form)
    int32_t pad2;
    double psi_w[2];       // psi of the solid nodes per component
    float psi_wf[2];
};


// One block's work: an xy tile [x0, x0+tw) x [y0, y0+th) marched over z in
// [z0, z0+nzc), upwards, or downwards when down != 0 (pipelined step only).
struct Item {
    int32_t inst;
    int16_t x0, y0;
    int16_t tw, th;
    int16_t z0, nzc;
    int16_t down, pad;
};

LBSC_HD int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Plane index providing psi for a z outside [0, nz): periodic wrap, or the
// mirror psi(-1) := psi(0), psi(nz) := psi(nz-1) at a wall on the z seam.
// (Behind a solid wall psi is the wall's constant instead: see beyond_wall.)
LBSC_HD int psi_plane(int z, int nz, int wall_z)
{
    if (z >= 0 && z < nz) return z;
    if (wall_z) return z < 0 ? 0 : nz - 1;
    return wrap(z, nz);
}

// Pull source of population i at node (x, y, z): returns the node the value
// comes from and whether it is the reflected population opp(i) of the node
// itself (bounce-back across a wall on the z seam).
struct PullSrc {
    int x, y, z;
    bool reflected;
};

LBSC_HD PullSrc pull_src(int i, int x, int y, int z, int nx, int ny, int nz, int wall_z)
{
    int zs = z - ez(i);
    if (wall_z && (zs < 0 || zs >= nz)) return PullSrc{x, y, z, true};
    return PullSrc{wrap(x - ex(i), nx), wrap(y - ey(i), ny), wrap(zs, nz), false};
}

LBSC_HD int64_t node_of(int x, int y, int z, int nx, int ny) { return ((int64_t)z * ny + y) * nx + x; }

// Plane z lies behind a solid wall, where psi is the wall's constant.
LBSC_HD bool beyond_wall(const Inst& I, int z) { return I.psi_wall && I.wall_z && (z < 0 || z >= I.nz); }

}  // namespace lbsc
