// Device-side types and helpers shared by the libigr kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace igr {

constexpr int G = 3;  // ghost layers (five-point upwind reconstruction)

// bfloat16 storage word.  Values are widened to float for arithmetic and
// rounded back to nearest-even once per store (gfx950's conversion
// instruction, in the default rounding mode).
struct bf16 {
    uint16_t bits;
};

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// Storage type T -> arithmetic type C with load/store conversions.  R is
// the register form of a loaded value before conversion: kernels that load
// ahead keep R in their prefetch registers and convert where the value is
// used, so that the conversion does not wait for the load to arrive.
template <class T>
struct Storage;

template <>
struct Storage<double> {
    using C = double;
    using R = double;
    __device__ __forceinline__ static R load_raw(const double* p) { return *p; }
    __device__ __forceinline__ static C cvt(R r) { return r; }
    __device__ __forceinline__ static double load(const double* p) { return *p; }
    __device__ __forceinline__ static void store(double* p, double v) { *p = v; }
    __device__ __forceinline__ static C stored(C v) { return v; }   // value as read back after a store
};

template <>
struct Storage<float> {
    using C = float;
    using R = float;
    __device__ __forceinline__ static R load_raw(const float* p) { return *p; }
    __device__ __forceinline__ static C cvt(R r) { return r; }
    __device__ __forceinline__ static float load(const float* p) { return *p; }
    __device__ __forceinline__ static void store(float* p, float v) { *p = v; }
    __device__ __forceinline__ static C stored(C v) { return v; }
};

template <>
struct Storage<bf16> {
    using C = float;
    using R = uint32_t;   // the 16 stored bits
    __device__ __forceinline__ static R load_raw(const bf16* p) { return p->bits; }
    __device__ __forceinline__ static C cvt(R r) { return __uint_as_float(r << 16); }
    __device__ __forceinline__ static float load(const bf16* p) { return cvt(load_raw(p)); }
    __device__ __forceinline__ static void store(bf16* p, float v) { p->bits = f32_to_bf16_rne(v); }
    __device__ __forceinline__ static C stored(C v) { return cvt(f32_to_bf16_rne(v)); }
};

// IEEE binary16 storage (the paper's storage precision), float arithmetic;
// conversions round to nearest even.
using f16 = _Float16;

template <>
struct Storage<f16> {
    using C = float;
    using R = uint32_t;   // the 16 stored bits
    __device__ __forceinline__ static R load_raw(const f16* p) {
        return __builtin_bit_cast(uint16_t, *p);
    }
    __device__ __forceinline__ static C cvt(R r) { return float(__builtin_bit_cast(f16, uint16_t(r))); }
    __device__ __forceinline__ static float load(const f16* p) { return float(*p); }
    __device__ __forceinline__ static void store(f16* p, float v) { *p = f16(v); }
    __device__ __forceinline__ static C stored(C v) { return float(f16(v)); }
};

// Element `o` of the x-y plane that starts at `plane`: a uniform base (kept
// in scalar registers) plus a 32-bit byte offset per lane, the addressing
// that global loads and stores take as they are (igr_init keeps a padded
// plane below 2^29 elements, so the byte offset of any element type here
// fits 32 bits).
template <class T>
__device__ __forceinline__ const T* at_plane(const T* plane, uint32_t o) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(plane) + o * uint32_t(sizeof(T)));
}
template <class T>
__device__ __forceinline__ T* at_plane(T* plane, uint32_t o) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(plane) + o * uint32_t(sizeof(T)));
}

// Storage forms: how the kernels read a stage state and Sigma.  A kernel
// reads a state value through load_u (base array plus, with HASD, a
// difference array) and a Sigma value through load_s, keeps the register
// form RU until the value is used and widens it with cvt.
//
// Plain<T>: the state, every RK stage state and Sigma are stored in T (the
// difference array is never read).
template <class T>
struct Plain {
    using S = Storage<T>;
    using C = typename S::C;
    using TB = T;   // the step's state U^n (the caller's U) and rhs
    using TD = T;   // RK stage state buffers
    using TS = T;   // Sigma
    using RU = typename S::R;
    static constexpr bool SPLIT = false;
    // later sweeps read rho and divide (in FP64 a stored 1/rho, the same
    // bytes as rho, measured slower: its store costs the first pass more
    // than the divisions cost the memory-bound later passes)
    static constexpr bool IRS = false;
    template <bool HASD>
    __device__ __forceinline__ static RU load_u(const TB* b, const TD*, long long o) {
        return S::load_raw(b + o);
    }
    __device__ __forceinline__ static RU load_s(const TS* s, long long o) { return S::load_raw(s + o); }
    // field f of (U, Sigma): 0..4 the state, 5 Sigma
    template <bool HASD>
    __device__ __forceinline__ static RU load_field(const TB* b, const TD*, const TS* s, int f, long long fs,
                                                    long long o) {
        return S::load_raw((f < 5 ? b + f * fs : s) + o);
    }
    // the same from plane bases and an in-plane offset (at_plane)
    template <bool HASD>
    __device__ __forceinline__ static RU load_up(const TB* bp, const TD*, uint32_t o) {
        return S::load_raw(at_plane(bp, o));
    }
    __device__ __forceinline__ static RU load_sp(const TS* sp, uint32_t o) { return S::load_raw(at_plane(sp, o)); }
    __device__ __forceinline__ static C cvt(RU r) { return S::cvt(r); }
};

// Split: FP32 arithmetic; the step's state U^n is FP32, each later RK stage
// state is stored as its bfloat16 difference from U^n (the stage value is
// U^n + delta, summed in FP32), Sigma is bfloat16.  Rounding a whole stage
// state to 8 significand bits loses 2^-9 of the state at every stage, and
// that accumulates over the steps; rounding its difference from U^n loses
// 2^-9 of the difference only, and U^n itself is rounded to FP32 once per
// step.  Stage 1 reads U^n alone (HASD false).
struct Split {
    using C = float;
    using TB = float;
    using TD = bf16;
    using TS = bf16;
    struct RU {
        float a;      // base value (0 for Sigma)
        uint32_t d;   // bfloat16 bits of the difference (of Sigma itself)
    };
    static constexpr bool SPLIT = true;
    static constexpr bool IRS = true;
    template <bool HASD>
    __device__ __forceinline__ static RU load_u(const float* b, const bf16* d, long long o) {
        RU r;
        r.a = b[o];
        if constexpr (HASD)
            r.d = d[o].bits;
        else
            r.d = 0u;
        return r;
    }
    __device__ __forceinline__ static RU load_s(const bf16* s, long long o) {
        RU r;
        r.a = 0.0f;
        r.d = s[o].bits;
        return r;
    }
    template <bool HASD>
    __device__ __forceinline__ static RU load_field(const float* b, const bf16* d, const bf16* s, int f, long long fs,
                                                    long long o) {
        RU r;
        r.a = f < 5 ? b[f * fs + o] : 0.0f;
        if constexpr (HASD)
            r.d = (f < 5 ? d + f * fs : s)[o].bits;
        else
            r.d = f < 5 ? 0u : uint32_t(s[o].bits);
        return r;
    }
    template <bool HASD>
    __device__ __forceinline__ static RU load_up(const float* bp, const bf16* dp, uint32_t o) {
        RU r;
        r.a = *at_plane(bp, o);
        if constexpr (HASD)
            r.d = at_plane(dp, o)->bits;
        else
            r.d = 0u;
        return r;
    }
    __device__ __forceinline__ static RU load_sp(const bf16* sp, uint32_t o) {
        RU r;
        r.a = 0.0f;
        r.d = at_plane(sp, o)->bits;
        return r;
    }
    __device__ __forceinline__ static C cvt(RU r) { return r.a + __uint_as_float(r.d << 16); }
};

// Reciprocal for finite positive arguments.  FP64: the hardware estimate
// refined by two Newton steps, within an ulp or two of the correctly
// rounded quotient at a third of the instructions of IEEE division.  FP32
// (the arithmetic of the precision forms, whose kernels are bound by
// instruction issue): the hardware estimate alone, accurate to about one
// ulp (a Newton step measured 1.5-2 % slower per step and changes nothing
// at the forms' error level).  Non-positive or non-finite arguments only
// occur for states the kernels already flag as non-physical.
__device__ __forceinline__ double fast_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Block index -> logical tile index such that consecutive logical tiles run
// on the same XCD (blocks are dealt round-robin to the 8 XCDs), so a tile's
// y-halo rows are usually still in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    constexpr int NX = 8;
    const int full = nb - nb % NX;
    if (b >= full) return b;
    const int per = full / NX;
    return (b % NX) * per + b / NX;
}

// Tile coordinates of a logical block index, x fastest: the blocks resident
// on one XCD cover whole rows of tiles (long contiguous row segments per
// plane).  A y-fastest order, which would let them share y-halo rows
// through L2, measured slower (scattered 512-byte row pieces), and so did
// bands 2 or 4 tiles wide with y fastest inside (1024^3 FP64 step 288 and
// 280 ms against 275; FP32 157 and 145 against 139; 8 wide: equal).
__device__ __forceinline__ void tile_coords(int b, int tiles_x, int tiles_y, int& tx, int& ty, int& tz) {
    tx = b % tiles_x;
    b /= tiles_x;
    ty = b % tiles_y;
    tz = b / tiles_y;
}

// Padded-grid geometry passed by value to every kernel.
struct Geom {
    int n[3];          // interior extents nx, ny, nz
    int st[3];         // strides of x, y, z in a padded field (1, px, px*py)
    long long fs;      // elements per padded field
    double ih[3];      // 1/dx, 1/dy, 1/dz
    double gamma;
    double alpha;
    int periodic[3];
};

// index of the viscous stress component tau_ab (a <= b) among the six
// stored ones: xx 0, xy 1, xz 2, yy 3, yz 4, zz 5
__host__ __device__ constexpr int tau_index(int a, int b) {
    return a <= b ? (a == 0 ? b : (a == 1 ? 2 + b : 5)) : tau_index(b, a);
}

__device__ __forceinline__ long long cell_offset(const Geom& g, int i, int j, int k) {
    return (long long)(k + G) * g.st[2] + (long long)(j + G) * g.st[1] + (i + G);
}

// Offset (relative to the cell) of the axis-d neighbour on side s (+1/-1)
// for a field whose ghosts are NOT filled: periodic wrap or the cell itself
// (zero gradient).
__device__ __forceinline__ int neighbour_no_ghost(const Geom& g, int d, int idx, int s) {
    const int n = g.n[d];
    const int t = idx + s;
    if (t >= 0 && t < n) return s * g.st[d];
    if (g.periodic[d]) return (t < 0 ? (n - 1) : -(n - 1)) * g.st[d];
    return 0;
}

}  // namespace igr
