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
constexpr uint32_t kWrapBit = 0x40000000u;  // list entry flag: pair found through a periodic image
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

// Calls fn(begin, end, sx, sy, sz) for the contiguous slot ranges of the
// cells around the cell of (xi, yi, zi) that can hold a particle closer than
// r_c; (sx, sy, sz) is the periodic shift to add to x_i - x_j for candidates of
// that range.  Rows (dy, dz) whose nearest face is already r_c away are
// skipped, and in each row the x-neighbour cells are kept only when their
// facing side is closer than the row's remaining reach sqrt(r_c^2 - dy^2 -
// dz^2).  The clipping margin (1e-9) is far above rounding, so it never drops
// a pair that the exact test would keep.
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
    for (int dz = -1; dz <= 1; ++dz) {
        const double ez = dz == 0 ? 0.0 : fmax(0.0, (dz < 0 ? loz : hiz) - kMargin);
        if (ez >= g.rc) continue;
        const int zz = wrap_index(cz + dz, nz);
        const double sz = cz + dz < 0 ? g.L[2] : (cz + dz >= nz ? -g.L[2] : 0.0);
        for (int dy = -1; dy <= 1; ++dy) {
            const double ey = dy == 0 ? 0.0 : fmax(0.0, (dy < 0 ? loy : hiy) - kMargin);
            const double q = ey * ey + ez * ez;
            if (q >= g.rc2) continue;
            const double reach = __builtin_sqrt(g.rc2 - q) + kMargin;
            const int yy = wrap_index(cy + dy, ny);
            const double sy = cy + dy < 0 ? g.L[1] : (cy + dy >= ny ? -g.L[1] : 0.0);
            const int base = nx * (yy + ny * zz);
            const int xa = cx - (lox < reach ? 1 : 0);
            const int xb = cx + (hix < reach ? 1 : 0);
            if (xa >= 0 && xb < nx) {
                fn(cstart[base + xa], cstart[base + xb + 1], 0.0, sy, sz);
            } else if (xa < 0) {
                fn(cstart[base + nx - 1], cstart[base + nx], g.L[0], sy, sz);
                fn(cstart[base], cstart[base + xb + 1], 0.0, sy, sz);
            } else {
                fn(cstart[base + xa], cstart[base + nx], 0.0, sy, sz);
                fn(cstart[base], cstart[base + 1], -g.L[0], sy, sz);
            }
        }
    }
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

// List row layout: the kListCap entries of particle i hold its neighbours
// with r < r_d first and then the others, with no gap; the count word packs
// the two counts (near in bits 0..15, far in bits 16..31).  A row whose counts
// add up to more than kListCap is not valid.
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
        for_each_row(g, xi, yi, zi, cstart, [&](int b, int e, double sx, double sy, double sz) {
            for (int j = b + sub; j < e; j += P) {
                if (j == i) continue;
                const double dx = (xi - xs.x[j]) + sx;
                const double dy = (yi - xs.y[j]) + sy;
                const double dz = (zi - xs.z[j]) + sz;
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
    const int r = __builtin_amdgcn_readfirstlane(find_rep(off, R.nrep, blk));
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
