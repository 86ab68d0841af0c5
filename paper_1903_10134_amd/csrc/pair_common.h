// pair_common.h -- device helpers shared by the pair passes (pair.hip) and
// their adjoints (adjoint.hip): list layout, neighbour visiting, lane-group
// sums and the XCD-aware block order.
#pragma once
#include <type_traits>

#include "mdpd_internal.h"

namespace mdpd {
namespace {

constexpr double kSqrt3Scaled = 1.7320508075688772 / 16777216.0;  // sqrt(3) 2^-24
constexpr float kSqrt3ScaledF = 1.7320508075688772f / 16777216.0f;
constexpr uint32_t kNearBit = 0x80000000u;  // list entry flag: r < r_d
constexpr uint32_t kWrapBit = 0x40000000u;  // list entry flag: the pair may need the minimum image
constexpr uint32_t kSlotMask = 0x3fffffffu;
constexpr int kWavesPerBlock = kBlock / 64;

// Element idx of an array addressed with a 32-bit byte offset, so that the
// load can take the array base in scalar registers.
template <typename T>
__device__ __forceinline__ T ld(const T *__restrict__ base, int idx)
{
    return *(const T *)((const char *)base + (uint32_t)idx * (uint32_t)sizeof(T));
}

__device__ __forceinline__ int wrap_index(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// Calls fn(begin, end) for the contiguous slot ranges of the distinct cells
// around the cell of (xi, yi, zi) that can hold a particle closer than r_c;
// the caller takes every difference x_i - x_j through the minimum image (the
// torus distance), which is the pair's difference whichever cell lists it.
// Rows (dy, dz) whose nearest face is already r_c away are skipped, and in
// each row the x-neighbour cells are kept only when their facing side is
// closer than the row's remaining reach sqrt(r_c^2 - dy^2 - dz^2).  The
// particles sit in the cells of the last list build and have moved less than
// half the skin since (g.slack; one may even have crossed a periodic face),
// so every gap is reduced by that much.  The clipping margin (1e-9) is far
// above rounding, so it never drops a pair that the exact test would keep.
// An axis with three cells or more has the neighbour offsets -1, 0, +1 (the
// neighbours of an edge cell wrap); with two cells the other cell is a
// neighbour on both sides (its gap is the nearer face); with one cell the
// cell is all there is.
template <typename Fn>
__device__ __forceinline__ void for_each_row(const Geom &g, double xi, double yi, double zi,
                                             const int *__restrict__ cstart, Fn &&fn)
{
    constexpr double kMargin = 1e-9;
    const int nx = g.nc[0], ny = g.nc[1], nz = g.nc[2];
    const int cx = cell_coord(xi, g.s[0], nx);
    const int cy = cell_coord(yi, g.s[1], ny);
    const int cz = cell_coord(zi, g.s[2], nz);
    const double lox = xi - cx * g.cs[0], hix = (cx + 1) * g.cs[0] - xi;
    const double loy = yi - cy * g.cs[1], hiy = (cy + 1) * g.cs[1] - yi;
    const double loz = zi - cz * g.cs[2], hiz = (cz + 1) * g.cs[2] - zi;
    // gap from x_i to the neighbour on side d of an axis (0 for the own cell)
    auto gap = [&](int d, int n, double lo, double hi) {
        if (d == 0) return 0.0;
        const double f = n == 2 ? fmin(lo, hi) : (d < 0 ? lo : hi);
        return fmax(0.0, f - kMargin - g.slack);
    };
    const int z0 = nz >= 3 ? -1 : 0, z1 = nz >= 2 ? 1 : 0;
    const int y0 = ny >= 3 ? -1 : 0, y1 = ny >= 2 ? 1 : 0;
    for (int dz = z0; dz <= z1; ++dz) {
        const double ez = gap(dz, nz, loz, hiz);
        if (ez >= g.rc) continue;
        const int zz = wrap_index(cz + dz, nz);
        for (int dy = y0; dy <= y1; ++dy) {
            const double ey = gap(dy, ny, loy, hiy);
            const double q = ey * ey + ez * ez;
            if (q >= g.rc2) continue;
            const double reach = __builtin_sqrt(g.rc2 - q) + kMargin + g.slack;
            const int base = nx * (wrap_index(cy + dy, ny) + ny * zz);
            if (nx <= 2) {
                const bool other = nx == 2 && fmin(lox, hix) < reach;
                if (other) fn(cstart[base], cstart[base + 2]);
                else fn(cstart[base + cx], cstart[base + cx + 1]);
                continue;
            }
            const int xa = cx - (lox < reach ? 1 : 0);
            const int xb = cx + (hix < reach ? 1 : 0);
            if (xa >= 0 && xb < nx) {
                fn(cstart[base + xa], cstart[base + xb + 1]);
            } else if (xa < 0) {
                fn(cstart[base + nx - 1], cstart[base + nx]);
                fn(cstart[base], cstart[base + xb + 1]);
            } else {
                fn(cstart[base + xa], cstart[base + nx]);
                fn(cstart[base], cstart[base + 1]);
            }
        }
    }
}

// x_i - x_j through the minimum image on every axis (the direct scans).
__device__ __forceinline__ void min_image3(const Geom &g, double &dx, double &dy, double &dz)
{
    dx = min_image(dx, g.L[0], g.invL[0]);
    dy = min_image(dy, g.L[1], g.invL[1]);
    dz = min_image(dz, g.L[2], g.invL[2]);
}

// Fixed-point coordinate of a 32-byte record: x in [0, L) (s = 2^32 / L) as
// round(x s) mod 2^32 (a coordinate that rounds up to 2^32 wraps to 0, the
// same point of the periodic box).
__device__ __forceinline__ uint32_t qfix(double x, double s)
{
    return (uint32_t)(unsigned long long)(long long)__builtin_rint(x * s);
}

// x_i - x_j of two fixed-point coordinates: the minimum image, in FP32.
__device__ __forceinline__ float qdiff(uint32_t qi, uint32_t qj, float d)
{
    return (float)(int)(qi - qj) * d;
}

// Hardware dispatches workgroups to the 8 XCDs round robin; remap so that
// each XCD (and its L2) works through one contiguous chunk of the sorted
// particles, whose neighbour data it then reuses.
__device__ __forceinline__ int xcd_block()
{
    const int nb = gridDim.x, b = blockIdx.x;
    const int per = nb >> 3, rem = nb & 7, x = b & 7, k = b >> 3;
    return x * per + (x < rem ? x : rem) + k;
}

// Sum over the P lanes of a group (butterfly, fixed order).
template <int P, typename T>
__device__ __forceinline__ T group_sum(T v)
{
#pragma unroll
    for (int m = 1; m < P; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Broadcast of lane u's value (u wave-uniform) through the scalar unit.
__device__ __forceinline__ int bcast_i(int v, int u) { return __builtin_amdgcn_readlane(v, u); }
__device__ __forceinline__ double bcast_d(double v, int u)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, u);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), u);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// base + the number of set bits of m in the lanes below this one
__device__ __forceinline__ int lanes_below(unsigned long long m, int base = 0)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, (unsigned)base));
}

// Pair-list row layout: the kListCap entries of particle i hold its
// neighbours closer than r_c (kNearBit: r < r_d) with no gap; the count
// word packs the two counts (near in bits 0..15, far in bits 16..31).  A row whose counts add up to more
// than kListCap is not valid.
__device__ __forceinline__ int list_near(int packed) { return packed & 0xffff; }
__device__ __forceinline__ int list_total(int packed) { return (packed & 0xffff) + (packed >> 16); }

// Visits every neighbour j (r_ij < r_c, j != i) of slot i: from the list when
// it did not overflow, else by a direct cell scan with the same exact test.
// fn(j, dx, dy, dz, near) receives the minimum-image difference x_i - x_j and
// whether r_ij < r_d.
template <int P, typename Fn>
__device__ __forceinline__ void for_each_neighbor(const PairConst &pc, const Geom &g, int i, int sub,
                                                  double xi, double yi, double zi, Soa3c xs,
                                                  const int *__restrict__ cstart, int packed,
                                                  const uint32_t *__restrict__ lst, Fn &&fn)
{
    const int cnt = list_total(packed);
    if (cnt <= kListCap) {
        for (int k = sub; k < cnt; k += P) {
            const uint32_t e = lst[k];
            const int j = (int)(e & kSlotMask);
            double dx = xi - ld(xs.x, j), dy = yi - ld(xs.y, j), dz = zi - ld(xs.z, j);
            if (e & kWrapBit) {
                dx = min_image(dx, pc.L[0], pc.invL[0]);
                dy = min_image(dy, pc.L[1], pc.invL[1]);
                dz = min_image(dz, pc.L[2], pc.invL[2]);
            }
            fn(j, dx, dy, dz, (e & kNearBit) != 0);
        }
    } else {
        for_each_row(g, xi, yi, zi, cstart, [&](int b, int e) {
            for (int j = b + sub; j < e; j += P) {
                if (j == i) continue;
                double dx = xi - xs.x[j], dy = yi - xs.y[j], dz = zi - xs.z[j];
                min_image3(g, dx, dy, dz);
                const double r2 = exact_r2(dx, dy, dz);
                if (r2 < g.rc2) fn(j, dx, dy, dz, r2 < g.rd2);
            }
        });
    }
}

// The replica of this (replica-aligned) block and the slot range its P-lane
// groups cover: particle i0 + threadIdx.x / P, valid while below i1.
struct BlockRep {
    int r, i0, i1;
};

template <int P>
__device__ __forceinline__ BlockRep block_rep(const Reps &R, int blk)
{
    const int *off = R.blk_off + lanes_index(P) * (R.nrep + 1);
    const int r = block_replica(R, lanes_index(P), off, blk);
    return BlockRep{r, cload(R.part_off, r) + (blk - cload(off, r)) * (kBlock / P), cload(R.part_off, r + 1)};
}

// Host: a type tag for dispatching on the arithmetic type of a pass.
template <typename T>
struct Tid {
    using type = T;
};

// Host: instantiate a launch for the lane count P in {1, 2, 4, 8, 16}.
template <typename K>
void launch_lanes(int lanes, K &&k)
{
    switch (lanes) {
    case 1: k(std::integral_constant<int, 1>{}); break;
    case 2: k(std::integral_constant<int, 2>{}); break;
    case 4: k(std::integral_constant<int, 4>{}); break;
    case 8: k(std::integral_constant<int, 8>{}); break;
    default: k(std::integral_constant<int, 16>{}); break;
    }
}

inline int blocks_for(int64_t threads) { return (int)((threads + kBlock - 1) / kBlock); }

}  // namespace
}  // namespace mdpd
