// pw_march.hip -- x-marching PW advection kernels (columns of any height).
//
// Work decomposition.  A workgroup owns a strip of TY consecutive y-columns
// (contiguous in memory, like the y-batches of the paper's section 3) and a
// segment of LX consecutive x-planes, which it walks in increasing x (the
// x-outer loop order of Listing 4).  Slot c of the strip is y-column
// j0 - 1 + c: slots 1..TY are the strip's columns, slots 0 and TY + 1 its
// y-halo columns.  A wavefront holds one slot, with lane k = level k of that
// column (nz <= 64, so one 64-wide wavefront covers a column and every global
// access of a wave is one contiguous, coalesced run along z; lanes k >= nz
// read zeros and store nothing, as lanes past the end of a 64-level column
// do).  Two ways to carry the halo columns:
//   * halo waves: TY + 2 wavefronts, wave w = slot w; waves 0 and TY + 1
//     only load;
//   * edge waves: TY wavefronts, wave w = slot w + 1, all computing; the
//     first and last wave also load a halo column, through a second register
//     ring.  With TY a multiple of 4 the arithmetic spreads evenly over the
//     four SIMDs of a compute unit, which pays where the arithmetic, not HBM,
//     sets the pace.
// Columns of more than 64 levels are held by ZW = 2, 3 or 4 wavefronts of
// one workgroup (variant 7, the default for them), wave z holding levels
// 64 z .. 64 z + 63.  Their z-neighbours come from the LDS ring instead of
// wavefront shifts: it then holds whole columns, with a zero entry below
// level 0 and above the top, and keeps three planes of every field, so that
// plane p+1 of a neighbouring wave's levels is there when step p needs it.
// Columns of more than 256 levels are cut into z-chunks of 64 ZW - 2 levels,
// one per workgroup, whose first and last lanes hold the neighbouring
// chunks' levels (loaded, never stored).  Variants 0-6 cut every column of
// more than 64 levels into z-chunks of 62 levels, one wavefront each: lane l
// holds level 62 c - 1 + l, lanes 0 and 63 are the chunk's halo levels, so
// the z-neighbours of lanes 1..62 still come from wavefront shifts.
//
// Reuse.  Each field (u, v, w and, for the adjoint, lu, lv, lw) is read from
// HBM once per cell:
//   * x-neighbours stay in a per-lane register ring of planes p-1 .. p+D+1,
//     filled D+1 planes ahead of use (software prefetch);
//   * y-neighbours come from an LDS ring where every wave deposits its
//     column of the planes the strip needs next;
//   * k-neighbours come from the neighbouring lane through DPP wavefront
//     shifts (no memory access);
//   * the diagonal operands are recycled: u(p-1, j+1) is last step's u(p, j+1)
//     read, v(p, j-1) is last step's v(p+1, j-1) read.
// LDS slots.  u- and w-type fields are read only on plane p in step p, so a
// two-plane ring suffices (step p deposits plane p+1).  v-type fields are
// also read on plane p+1 (the v(i+1, j-1) operand of su), so they use a
// three-plane ring (step p deposits plane p+2).  One barrier per step.
//
// Block order.  Consecutive workgroup ids are dispatched round-robin over the
// 8 XCDs (hardware id b runs on XCD b % 8).  The work items (strip fastest,
// then z-chunk, then segment) are dealt to the XCDs in groups of G
// consecutive items, XCDs interleaved group by group:
//   * G = ceil(blocks / 8) ("XCD ranges"): each XCD takes one contiguous
//     range of strips, so halo columns shared by neighbouring strips are
//     read through the same L2, but the 8 XCDs march in 8 different parts
//     of the grid;
//   * G = 1 ("natural"): the workgroups resident at any time are
//     neighbouring strips of the same segments on all XCDs, so the device
//     sweeps the same x-planes together (long runs of neighbouring addresses
//     in flight), but every halo column is read through two L2s;
//   * G in between keeps most halo columns inside one XCD's L2 while the
//     device still sweeps one window of the grid.
// Which is fastest depends on the kernel and on where the arrays lie in HBM.
#include <atomic>
#include <type_traits>

#include "pw_half.h"
#include "pw_internal.h"
#include "pw_stencil.h"

namespace {

constexpr int NZ = 64;   // wavefront width = most levels per column
constexpr int kChunk = NZ - 2;   // levels a z-chunk of a taller column owns

// Lane k receives lane k-1's value (wavefront shift right by one, DPP).
__device__ __forceinline__ int dpp_from_below(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, 0x138, 0xF, 0xF, true);
}
// Lane k receives lane k+1's value (wavefront shift left by one, DPP).
__device__ __forceinline__ int dpp_from_above(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, 0x130, 0xF, 0xF, true);
}

template <bool BELOW>
__device__ __forceinline__ float lane_shift(float x)
{
    const int v = __float_as_int(x);
    return __int_as_float(BELOW ? dpp_from_below(v) : dpp_from_above(v));
}

template <bool BELOW>
__device__ __forceinline__ double lane_shift(double x)
{
    const long long v = __double_as_longlong(x);
    int lo = (int)(v & 0xffffffffLL);
    int hi = (int)(v >> 32);
    lo = BELOW ? dpp_from_below(lo) : dpp_from_above(lo);
    hi = BELOW ? dpp_from_below(hi) : dpp_from_above(hi);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <bool BELOW>
__device__ __forceinline__ _Float16 lane_shift(_Float16 x)
{
    const int v = (int)__builtin_bit_cast(unsigned short, x);
    const int r = BELOW ? dpp_from_below(v) : dpp_from_above(v);
    return __builtin_bit_cast(_Float16, (unsigned short)r);
}

template <bool BELOW>
__device__ __forceinline__ bf16_t lane_shift(bf16_t x)
{
    const int r = BELOW ? dpp_from_below((int)x.bits) : dpp_from_above((int)x.bits);
    bf16_t y;
    y.bits = (unsigned short)r;
    return y;
}

template <typename T>
__device__ __forceinline__ T below(T x) { return lane_shift<true>(x); }   // level k-1
template <typename T>
__device__ __forceinline__ T above(T x) { return lane_shift<false>(x); }  // level k+1

// Raw buffer access to one storage column: the descriptor's base is the
// column start (wave-uniform, scalar registers) and its record count the
// column's byte length, or 0 for a wave that must not touch memory.  Loads
// outside the record range return 0 and stores outside it are dropped, so
// every wave issues the same sequence of memory instructions, with no
// branches around them; that keeps the compiler's wait counts exact, which
// the register prefetch relies on.  Word 3 is the gfx9 raw-buffer format.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;
constexpr unsigned kOutOfRange = 0x40000000u;  // byte offset beyond any column

__device__ __forceinline__ rsrc_t column_rsrc(const void* base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, kRsrcWord3);
}

template <typename T>
__device__ __forceinline__ T buf_load(rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ double buf_load<double>(rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ float buf_load<float>(rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ _Float16 buf_load<_Float16>(rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ bf16_t buf_load<bf16_t>(rsrc_t r, unsigned off)
{
    bf16_t y;
    y.bits = __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
    return y;
}

using u32x2 = unsigned int __attribute__((vector_size(8)));
__device__ __forceinline__ void buf_store(double x, rsrc_t r, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_store(float x, rsrc_t r, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_store(_Float16 x, rsrc_t r, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_store(bf16_t x, rsrc_t r, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b16(x.bits, r, (int)off, 0, 0);
}

// Working type of the register ring, the LDS ring and the DPP shifts: the
// arithmetic type C when the storage type T is narrower (16-bit storage
// works in float, float storage with FP64 arithmetic in double), else T.  A
// narrow load lands in a W-typed register as raw bits (zero-extended) and
// becomes a value where the plane is first used, so the conversion does not
// force a wait on the prefetch; the raw pattern 0 (zero records, masks)
// widens to +0.
template <typename T, typename C>
using work_t = typename std::conditional<(sizeof(T) < sizeof(C)), C, T>::type;

template <typename T, typename W>
__device__ __forceinline__ W ld_raw(rsrc_t r, unsigned off)
{
    if constexpr (sizeof(T) == sizeof(W)) {
        return buf_load<T>(r, off);
    } else if constexpr (sizeof(T) == 2) {
        static_assert(sizeof(W) == 4, "16-bit storage works in float");
        return __builtin_bit_cast(W, (unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0));
    } else {
        static_assert(sizeof(T) == 4 && sizeof(W) == 8, "float storage works in double");
        return __builtin_bit_cast(W, (unsigned long long)__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
    }
}

template <typename T, typename W>
__device__ __forceinline__ W widen(W x)
{
    if constexpr (sizeof(T) == sizeof(W)) {
        return x;
    } else if constexpr (std::is_same<T, bf16_t>::value) {
        return __builtin_bit_cast(float, __builtin_bit_cast(unsigned, x) << 16);
    } else if constexpr (sizeof(T) == 2) {
        return (float)__builtin_bit_cast(_Float16, (unsigned short)__builtin_bit_cast(unsigned, x));
    } else {
        return (double)__builtin_bit_cast(float, (unsigned)__builtin_bit_cast(unsigned long long, x));
    }
}

template <typename T, int NF>
struct MarchArgs {
    const T* in[NF];   // u, v, w [, lu, lv, lw]
    T* s[3];           // su, sv, sw (or unused)
    T* gr[3];          // gu, gv, gw (or unused)
    const T* b[3];     // base arrays of the update form (or unused)
    const double* tzc1;
    const double* tzc2;
    double tcx, tcy, beta;
};

// T: storage type; C: arithmetic type (T, or wider: double for float
// storage, float for 16-bit storage); registers, LDS and DPP shifts work in
// work_t<T, C>.  TY: compute columns per workgroup; D: planes prefetched
// beyond the current xp plane (D >= 2); EH: halo columns carried by the edge
// waves (TY wavefronts) instead of two halo waves (TY + 2 wavefronts).
// UPD (forward only): 0 stores s; 1 stores b + beta * s with the base arrays
// b streamed through the register ring like the fields (b may be the output
// itself: each element is read planes before the same wave writes it); 2 the
// same with b = (u, v, w), whose centre values are already in the ring.
// ZW: wavefronts per column (1, or 2, 3 or 4 for columns of up to 128, 192
// or 256 levels or for chunks of 64 ZW - 2 levels of taller ones, whose
// z-neighbours then come from the LDS ring).
template <typename T, typename C, int NF, bool WS, bool WG, int TY, int D, bool EH, int UPD = 0, int ZW = 1>
__global__ void __launch_bounds__(64 * (EH ? TY : TY + 2) * ZW)
march_kernel(MarchArgs<T, NF> a, Geom g, int LX, int nstrips, int nchunk, int nblocks, int group)
{
    static_assert(D >= 2, "v-type fields deposit plane p+2 from the register ring");
    static_assert(ZW >= 1 && ZW <= 4, "one to four wavefronts per column");
    static_assert(!EH || TY >= 2, "the two halo columns belong to different edge waves");
    static_assert(UPD == 0 || (NF == 3 && WS && !WG), "the update form is a forward-only epilogue");
    constexpr int NCOL = TY + 2;    // LDS slots
    constexpr int NT = NF / 3;      // field triples: 1 (winds) or 2 (winds + multipliers)
    // Register ring length and unroll of the plane loop (D + 3 planes are
    // live).  An unroll of 6, a multiple of both LDS ring lengths, makes every
    // LDS slot index a compile-time constant and saves the address arithmetic:
    // 2-5% for the narrow-storage kernels with halo waves, whose instruction
    // issue sets their pace.  The HBM-bound FP64-storage kernels measured 2%
    // slower with it and the register-bound edge-wave kernels spill, so they
    // keep the unroll of D + 3.
    constexpr int U = (D + 3 <= 6 && sizeof(T) < 8 && !EH) ? 6 : D + 3;
    constexpr int NR = NF + (UPD == 1 ? 3 : 0);   // ring rows: fields, then base arrays
    using W = work_t<T, C>;
    // ZL: z-neighbours from the LDS ring, which then holds whole columns
    // (entry 1 + k for level k, entries 0 and LZ - 1 zero) and three planes of
    // the u- and w-type fields as of the v-type ones
    constexpr bool ZL = ZW > 1;
    constexpr int LZ = ZL ? NZ * ZW + 2 : NZ;
    constexpr int UWS = ZL ? 3 : 2;
    __shared__ W s_uw[2 * NT][UWS][NCOL][LZ];
    __shared__ W s_v[NT][3][NCOL][LZ];

    // the wave index is uniform over a wavefront: keep it (and every address
    // part derived from it) in scalar registers, so that a global access is a
    // scalar base plus the lane offset.  With ZW > 1 the ZW wavefronts of a
    // column are consecutive: level block zw of column wave `wave`.
    const int wave_id = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int zw = ZL ? wave_id % ZW : 0;
    const int wave = ZL ? wave_id / ZW : wave_id;
    const int lane = threadIdx.x & 63;

    // block order (uniform): groups of `group` consecutive work items per XCD,
    // XCDs interleaved group by group (the grid is a multiple of 8 * group,
    // so every item below nblocks is taken exactly once)
    const int xcd = (int)(blockIdx.x & 7), gslot = (int)(blockIdx.x >> 3);
    const int L = ((gslot / group) * 8 + xcd) * group + gslot % group;
    if (L >= nblocks) return;
    const int strip = L % nstrips;
    const int chunk = (L / nstrips) % nchunk;
    const int seg = L / nstrips / nchunk;
    const int j0 = strip * TY;
    const int ncols = min(TY, g.ny - j0);
    const int i0 = seg * LX;
    const int i1 = min(i0 + LX, g.nx);
    const int slot = EH ? wave + 1 : wave;
    const int j = j0 - 1 + slot;
    const bool loads = slot <= ncols + 1;         // column j in [j0-1, j0+ncols]
    const bool comp = slot >= 1 && slot <= ncols; // column j in [j0, j0+ncols)
    // Edge waves: the first wave also carries column j0 - 1, the last wave of
    // a full strip column j0 + TY (in a narrower strip the wave of slot
    // ncols + 1 loads that column as its own).
    const bool halo = EH && (wave == 0 || (wave == TY - 1 && ncols == TY));
    const int hdj = wave == 0 ? -1 : 1;           // halo column relative to j
    const int hslot = wave == 0 ? 0 : TY + 1;
    const long long sx = g.sx;
    const int sy = g.sy;
    const int colbytes = g.Sz * (int)sizeof(T);
    const int ldbytes = loads ? colbytes : 0;     // waves past the strip read zeros
    const int stbytes = comp ? colbytes : 0;      // only computing waves write
    // storage column (plane p, column j + dj), as a pointer to its first level
    auto column = [&](const T* f, int p, int dj) -> const T* {
        const int pc = p < g.nx ? p : g.nx;       // planes past the end are never used
        return f + ((long long)(pc + g.h) * sx + (long long)(j + dj + g.h) * sy);
    };
    // level of this lane; loads at levels outside 0..nz-1 are out of range
    // (read zero), stores only from the lanes the chunk owns.  With ZW > 1 a
    // column taller than NZ * ZW levels is cut into z-chunks of NZ * ZW - 2
    // levels, one per workgroup: the first lane of wave 0 and the last lane
    // of wave ZW - 1 hold the chunk's halo levels (loaded, never stored), so
    // every owned level finds its z-neighbours in the LDS column.
    constexpr int kChunkZ = NZ * ZW - 2;
    const int kl = NZ * zw + lane;      // level within the chunk's window (ZW > 1)
    const int k = ZL ? (nchunk == 1 ? kl : chunk * kChunkZ - 1 + kl)
                     : nchunk == 1 ? lane : chunk * kChunk - 1 + lane;
    const bool own = ZL ? (nchunk == 1 || (kl >= 1 && kl <= kChunkZ))
                        : (nchunk == 1 || (lane >= 1 && lane <= kChunk));
    const int lk = ZL ? 1 + kl : lane;  // this lane's LDS entry
    const unsigned voff = (k >= 0 && k < g.nz) ? (unsigned)(g.h + k) * (unsigned)sizeof(T) : kOutOfRange;
    const unsigned vst = own ? voff : kOutOfRange;
    // z-halo levels of an output column: lanes 0..h-1 bottom (first chunk),
    // h..2h-1 top (last chunk)
    const bool first_z = chunk == 0 && (!ZL || zw == 0);
    const bool last_z = chunk == nchunk - 1 && (!ZL || zw == ZW - 1);
    const unsigned vpad = (lane < g.h && first_z) ? (unsigned)lane * (unsigned)sizeof(T)
                        : (lane >= g.h && lane < 2 * g.h && last_z)
                              ? (unsigned)(g.nz + lane) * (unsigned)sizeof(T) : kOutOfRange;

    // Multipliers are used with their level masks applied (see
    // pw_stencil.h): every operand of the gather is then a masked value, a
    // copy of one, or a DPP shift of one (shifts across the column ends read
    // 0).  The mask is applied where a freshly loaded plane is first used, so
    // that the prefetch is not waited for at the load.
    const bool live_uv = lam_uv_live(k, g.nz), live_w = lam_w_live(k, g.nz);
    auto mask = [&](int f, W x) -> W {
        if (f < 3 || f >= NF) return x;
        return ((f == 5) ? live_w : live_uv) ? x : W(0);
    };
    auto ld = [&](int f, int p, int dj, int bytes) -> W {   // raw for 16-bit storage
        const T* src = f < NF ? a.in[f] : a.b[f - NF];
        return ld_raw<T, W>(column_rsrc(column(src, p, dj), bytes), voff);
    };
    // Planes a segment uses: i0-1 .. i1 of the fields, i0 .. i1-1 of base
    // arrays.  The ring is filled further ahead than that near the segment's
    // end; those loads get a zero record count and read no memory.
    auto ring_bytes = [&](int f, int pl) -> int {
        const bool used = f < NF ? pl <= i1 : (pl >= i0 && pl < i1);
        return used ? ldbytes : 0;
    };
    // the halo ring of an edge wave holds planes i0 .. i1 of the fields, raw
    // until deposited
    auto halo_bytes = [&](int pl) -> int { return pl <= i1 ? colbytes : 0; };

    // Ring planes become values (widened, masked) where they are first used:
    // u/w-type plane q in step q-1 (as x+1 and LDS deposit), v-type plane q in
    // step q-2 (LDS deposit).  The fill does the planes first used before the
    // loop: i0-1, i0 and, for v-type, i0+1.
    W R[NR][U];
#pragma unroll
    for (int f = 0; f < NR; ++f)
#pragma unroll
        for (int t = 0; t < D + 2; ++t) {
            const W x = ld(f, i0 - 1 + t, 0, ring_bytes(f, i0 - 1 + t));
            R[f][t] = (f < NF && t < ((f % 3 == 1 || ZL) ? 3 : 2)) ? mask(f, widen<T, W>(x)) : x;
        }
    W H[NF][U];
    if (halo) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int t = 1; t < D + 2; ++t) H[f][t] = ld(f, i0 - 1 + t, hdj, halo_bytes(i0 - 1 + t));
    }
    W carry[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        if (f % 3 == 0) carry[f] = mask(f, widen<T, W>(ld(f, i0 - 1, 1, stbytes)));   // F(i0-1, j+1)
        else if (f % 3 == 1) carry[f] = mask(f, widen<T, W>(ld(f, i0, -1, stbytes))); // F(i0, j-1)
        else carry[f] = W(0);
    }
    // (lanes outside the column read the nearest level's coefficients: tzc has nz entries)
    const LevelCoef<C> cf = level_coef<C>(a.tzc1, a.tzc2, (C)a.tcx, (C)a.tcy, min(max(k, 0), g.nz - 1), g.nz);

    {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const int t = f / 3;
            if (f % 3 == 0) s_uw[2 * t][0][slot][lk] = R[f][1];
            if (f % 3 == 2) s_uw[2 * t + 1][0][slot][lk] = R[f][1];
            if constexpr (ZL) {
                if (f % 3 == 0) s_uw[2 * t][1][slot][lk] = R[f][2];
                if (f % 3 == 2) s_uw[2 * t + 1][1][slot][lk] = R[f][2];
            }
            if (f % 3 == 1) {
                s_v[t][0][slot][lk] = R[f][1];
                s_v[t][1][slot][lk] = R[f][2];
            }
        }
        if (halo) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const int t = f / 3;
                const W h1 = mask(f, widen<T, W>(H[f][1]));
                const W h2 = mask(f, widen<T, W>(H[f][2]));
                if (f % 3 == 0) s_uw[2 * t][0][hslot][lk] = h1;
                if (f % 3 == 2) s_uw[2 * t + 1][0][hslot][lk] = h1;
                if constexpr (ZL) {
                    if (f % 3 == 0) s_uw[2 * t][1][hslot][lk] = h2;
                    if (f % 3 == 2) s_uw[2 * t + 1][1][hslot][lk] = h2;
                }
                if (f % 3 == 1) {
                    s_v[t][0][hslot][lk] = h1;
                    s_v[t][1][hslot][lk] = h2;
                }
            }
        }
        if constexpr (ZL) {
            // the zero entries below level 0 and above the top of every LDS column
            constexpr int kUwCols = 2 * NT * UWS * NCOL, kCols = kUwCols + NT * 3 * NCOL;
            for (int i = (int)threadIdx.x; i < kCols; i += (int)blockDim.x) {
                W* col = i < kUwCols ? &s_uw[0][0][0][0] + i * LZ : &s_v[0][0][0][0] + (i - kUwCols) * LZ;
                col[0] = W(0);
                col[LZ - 1] = W(0);
            }
        }
    }
    __syncthreads();

    // Operands shared by consecutive steps, so each is shifted once: the
    // u-type F(p-1, j, k+1) is the previous step's F(p, j, k+1) of the centre,
    // the w-type F(p, j, k-1) the previous step's F(p+1, j, k-1).
    W zcar[NF];
    if constexpr (ZL) {
        // F(i0-1, j, k+1) of the u-type fields: that plane is not in the LDS
        // ring, so it is loaded one level up (with that level's mask);
        // F(i0, j, k-1) of the w-type ones from the ring
        const unsigned voff_up = (k + 1 < g.nz) ? (unsigned)(g.h + k + 1) * (unsigned)sizeof(T) : kOutOfRange;
        const bool up_uv = lam_uv_live(k + 1, g.nz);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const int t = f / 3;
            if (f % 3 == 0) {
                const W x = widen<T, W>(ld_raw<T, W>(column_rsrc(column(a.in[f], i0 - 1, 0), ring_bytes(f, i0 - 1)),
                                                     voff_up));
                zcar[f] = (f < 3 || up_uv) ? x : W(0);
            } else if (f % 3 == 2) {
                zcar[f] = s_uw[2 * t + 1][0][slot][lk - 1];
            } else {
                zcar[f] = W(0);
            }
        }
    } else {
#pragma unroll
        for (int f = 0; f < NF; ++f) zcar[f] = f % 3 == 0 ? above(R[f][0]) : f % 3 == 2 ? below(R[f][1]) : W(0);
    }

    // LDS slots count planes from the segment start: u/w-type plane q in slot
    // (q - i0) % 2, v-type in (q - i0) % 3
    for (int pb = i0; pb < i1; pb += U) {
        const int rel = U % 6 == 0 ? 0 : pb - i0;
#pragma unroll
        for (int s = 0; s < U; ++s) {
            const int p = pb + s;
            if (p >= i1) break;  // uniform over the workgroup
            const int rm = s % U, rc = (s + 1) % U, rq0 = (s + 2) % U, rq1 = (s + 3) % U;
            const int rnew = (s + D + 2) % U;
            const int pu = (rel + s) & 1;
            const int v0 = (rel + s) % 3, v1 = (rel + s + 1) % 3, v2 = (rel + s + 2) % 3;
            // u/w-type LDS slots of plane p and of the plane this step deposits
            const int ur = ZL ? v0 : pu, udep = ZL ? v2 : (pu ^ 1);

            // prefetch plane p + D + 1
#pragma unroll
            for (int f = 0; f < NR; ++f) R[f][rnew] = ld(f, p + D + 1, 0, ring_bytes(f, p + D + 1));
            if (halo) {  // only the edge waves spend memory instructions on the halo
#pragma unroll
                for (int f = 0; f < NF; ++f) H[f][rnew] = ld(f, p + D + 1, hdj, halo_bytes(p + D + 1));
            }

            // first use of plane p+1 (u/w-type) and p+2 (v-type deposit)
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                if (f % 3 == 1 || ZL) R[f][rq1] = mask(f, widen<T, W>(R[f][rq1]));
                else R[f][rq0] = mask(f, widen<T, W>(R[f][rq0]));
            }

            C out[6] = {C(0), C(0), C(0), C(0), C(0), C(0)};
            if (comp) {  // arithmetic only: no memory access inside the branch
                Star<W> st[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const int t = f / 3;
                    Star<W>& q = st[f];
                    q.c = R[f][rc];
                    q.xm = R[f][rm];
                    q.xp = R[f][rq0];
                    if constexpr (ZL) {          // z-neighbours: LDS entries lk -+ 1
                        if (f % 3 == 0) {
                            q.zm = s_uw[2 * t][ur][slot][lk - 1];
                            q.zp = s_uw[2 * t][ur][slot][lk + 1];
                        } else if (f % 3 == 1) {
                            q.zm = s_v[t][v0][slot][lk - 1];
                            q.zp = s_v[t][v0][slot][lk + 1];
                        } else {
                            q.zm = zcar[f];
                            q.zp = s_uw[2 * t + 1][ur][slot][lk + 1];
                        }
                    } else {
                        q.zm = f % 3 == 2 ? zcar[f] : below(q.c);
                        q.zp = above(q.c);
                    }
                    if (f % 3 == 0) {            // u-type
                        q.ym = s_uw[2 * t][ur][slot - 1][lk];
                        q.yp = s_uw[2 * t][ur][slot + 1][lk];
                        q.d1 = carry[f];         // F(p-1, j+1)
                        q.d2 = zcar[f];          // F(p-1, j, k+1)
                    } else if (f % 3 == 1) {     // v-type
                        q.ym = carry[f];         // F(p, j-1)
                        q.yp = s_v[t][v0][slot + 1][lk];
                        q.d1 = s_v[t][v1][slot - 1][lk];  // F(p+1, j-1)
                        if constexpr (ZL) q.d2 = s_v[t][v0][slot - 1][lk + 1];
                        else q.d2 = above(q.ym);          // F(p, j-1, k+1)
                    } else {                     // w-type
                        q.ym = s_uw[2 * t + 1][ur][slot - 1][lk];
                        q.yp = s_uw[2 * t + 1][ur][slot + 1][lk];
                        if constexpr (ZL) {
                            q.d1 = s_uw[2 * t + 1][v1][slot][lk - 1];
                            q.d2 = s_uw[2 * t + 1][ur][slot + 1][lk - 1];
                        } else {
                            q.d1 = below(q.xp);  // F(p+1, j, k-1)
                            q.d2 = below(q.yp);  // F(p, j+1, k-1)
                        }
                    }
                }
                Star<C> sc[NF];  // operands in the arithmetic type
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const Star<W>& q = st[f];
                    sc[f] = Star<C>{(C)q.c, (C)q.xm, (C)q.xp, (C)q.ym, (C)q.yp, (C)q.zm, (C)q.zp, (C)q.d1, (C)q.d2};
                }
                if (WS) pw_fwd(sc[0], sc[1], sc[2], cf, k, g.nz, out[0], out[1], out[2]);
                if (WG)
                    pw_adj_cell(sc[0], sc[1], sc[2], sc[NF - 3], sc[NF - 2], sc[NF - 1], cf, k, g.nz,
                                out[3], out[4], out[5]);
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    if (f % 3 == 0) carry[f] = st[f].yp;  // becomes F((p+1)-1, j+1)
                    if (f % 3 == 1) carry[f] = st[f].d1;  // becomes F(p+1, j-1)
                    if (f % 3 == 0) zcar[f] = st[f].zp;   // becomes F((p+1)-1, j, k+1)
                    if (f % 3 == 2) zcar[f] = st[f].d1;   // becomes F(p+1, j, k-1)
                }
            }

            // outputs of plane p: interior levels and zero z-halo levels
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                if ((q < 3 && !WS) || (q >= 3 && !WG)) continue;
                T* const dst = q < 3 ? a.s[q] : a.gr[q - 3];
                const rsrc_t r = column_rsrc(column(dst, p, 0), stbytes);
                C o = out[q];
                if (UPD == 1 && q < 3) o = pw_update((C)widen<T, W>(R[NF + q][rc]), (C)a.beta, o);
                if (UPD == 2 && q < 3) o = pw_update((C)R[q][rc], (C)a.beta, o);
                buf_store(store_round<T>(o), r, vst);
                buf_store(T(0), r, vpad);
            }

            // deposit: u/w-type plane p+1 (p+2 with ZL), v-type plane p+2
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const int t = f / 3;
                const W uw = ZL ? R[f][rq1] : R[f][rq0];
                if (f % 3 == 0) s_uw[2 * t][udep][slot][lk] = uw;
                if (f % 3 == 2) s_uw[2 * t + 1][udep][slot][lk] = uw;
                if (f % 3 == 1) s_v[t][v2][slot][lk] = R[f][rq1];
            }
            if (halo) {
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const int t = f / 3;
                    const W uw = mask(f, widen<T, W>(ZL ? H[f][rq1] : H[f][rq0]));
                    if (f % 3 == 0) s_uw[2 * t][udep][hslot][lk] = uw;
                    if (f % 3 == 2) s_uw[2 * t + 1][udep][hslot][lk] = uw;
                    if (f % 3 == 1) s_v[t][v2][hslot][lk] = mask(f, widen<T, W>(H[f][rq1]));
                }
            }
            __syncthreads();
        }
    }
}

struct Launch {
    int LX, nstrips, nchunk, nblocks, group, grid;
};

// Segment length: the caller's choice (lx > 0), else the length that
// minimises a simple cost model of the launch.  With `slots` workgroups
// resident on the device at once, the segments run in about
// ceil(nblocks / slots) rounds, and a segment of LX planes costs about
// LX + kSegmentCost planes: it reads its two end planes beyond the planes it
// computes and fills its prefetch ring before the first step.  The model,
// fitted to sweeps on MI355X, picks 128-plane segments at 4096 x 4096 x 64
// and 10 to 26 planes at 256 x 256 x 64.  Ties go to the longer segment.
constexpr int kMinLX = 4;
constexpr int kMaxLX = 128;
constexpr int kSegmentCost = 5;

Launch plan(const Geom& g, int TY, int lx, int slots, int order, int zw = 1)
{
    Launch l;
    l.nstrips = (g.ny + TY - 1) / TY;
    const int chunk_levels = zw > 1 ? NZ * zw - 2 : kChunk;
    l.nchunk = g.nz <= NZ * zw ? 1 : (g.nz + chunk_levels - 1) / chunk_levels;
    const long long cols = (long long)l.nstrips * l.nchunk;
    if (lx <= 0) {
        long long best = -1;
        const int hi = g.nx < kMaxLX ? g.nx : kMaxLX;
        const int lo = hi < kMinLX ? hi : kMinLX;
        for (int c = hi; c >= lo; --c) {
            const long long blocks = cols * ((g.nx + c - 1) / c);
            const long long cost = ((blocks + slots - 1) / slots) * (c + kSegmentCost);
            if (best < 0 || cost < best) {
                best = cost;
                lx = c;
            }
        }
    }
    // at most 2^30 work items (a segment length asked for through the tuning
    // knob may be short enough to exceed that only on grids of terabytes):
    // longer segments otherwise
    constexpr long long kMaxItems = 1LL << 30;
    if (cols * (((long long)g.nx + lx - 1) / lx) > kMaxItems) {
        const long long segs = kMaxItems / cols;     // cols < 2^26 for any grid check_shape admits
        lx = (int)(((long long)g.nx + segs - 1) / segs);
    }
    l.LX = lx;
    const int nseg = (g.nx + lx - 1) / lx;
    l.nblocks = (int)(cols * nseg);
    // order > 0: groups of `order` items per XCD; 0: one contiguous range each
    const int per = (l.nblocks + 7) / 8;
    l.group = order > 0 && order < per ? order : per;
    l.grid = ((l.nblocks + 8 * l.group - 1) / (8 * l.group)) * (8 * l.group);
    return l;
}

// Compute units of the current device (cached per device).
int compute_units()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return 256;
    }
    int n = cache[dev].load(std::memory_order_relaxed);
    if (n <= 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) {
            (void)hipGetLastError();
            n = 256;
        }
        cache[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

// Strip width, prefetch depth, halo carriers and LDS cap of each variant.
// Variants 0-3 keep their LDS ring within 64 KiB; variants 4-6 may use up to
// the 160 KiB of a compute unit.  A variant whose ring would exceed its cap
// for a given field count and working type falls back to variant 0.
constexpr int kVariants = 7;
constexpr int kTY[kVariants] = {6, 6, 14, 14, 10, 8, 16};
constexpr int kD[kVariants] = {2, 4, 2, 4, 2, 2, 2};
constexpr bool kEH[kVariants] = {false, false, false, false, false, true, true};
constexpr int kLdsCap[kVariants] = {65536, 65536, 65536, 65536, 163840, 163840, 163840};

template <typename T, typename C, int NF, int TY, int ZW = 1>
constexpr int lds_bytes()
{
    return ZW == 1 ? (int)sizeof(work_t<T, C>) * (2 * (NF / 3) * 2 + (NF / 3) * 3) * (TY + 2) * NZ
                   : (int)sizeof(work_t<T, C>) * (2 * (NF / 3) * 3 + (NF / 3) * 3) * (TY + 2) * (NZ * ZW + 2);
}

// Columns of more than 64 levels (PW_MARCH_VARIANTS - 1, the default there):
// ZW = 2, 3 or 4 wavefronts per column, edge waves, D = 2, 16 (15 with
// ZW = 3) wavefronts per workgroup for the forward and 8 (6) for the
// six-field kernels (whose registers allow 8 per compute unit).  At 2048 x 2048 x 128 FP64 the
// forward takes 4.8 ms and the fused pass 10.1 ms (67% and 64% of 8 TB/s),
// against 7.8 and 17.0 ms for the best z-chunked variant; at 256 levels 9.6
// and 21.3 ms against 15.9 and 32.6 ms.
constexpr int kTallVariant = 7;
template <int NF, int ZW>
constexpr int tall_ty()
{
    return (NF == 6 ? 8 : 16) / ZW;
}
static_assert(lds_bytes<double, double, 6, tall_ty<6, 4>(), 4>() <= 163840, "LDS of one compute unit");
static_assert(lds_bytes<double, double, 3, tall_ty<3, 4>(), 4>() <= 163840, "LDS of one compute unit");
static_assert(lds_bytes<double, double, 6, tall_ty<6, 2>(), 2>() <= 163840, "LDS of one compute unit");
static_assert(lds_bytes<double, double, 6, tall_ty<6, 3>(), 3>() <= 163840, "LDS of one compute unit");
static_assert(lds_bytes<double, double, 3, tall_ty<3, 3>(), 3>() <= 163840, "LDS of one compute unit");

// The LDS ring is static shared memory (no dynamic LDS is ever requested),
// so the compiler sizes each instantiation's group segment; the caps keep it
// within the 160 KiB of a compute unit.
static_assert(kLdsCap[0] <= 163840 && kLdsCap[4] <= 163840 && kLdsCap[6] <= 163840, "LDS of one compute unit");

template <typename T, typename C, int NF, bool WS, bool WG, int V, int UPD>
void go(const MarchArgs<T, NF>& m, const Geom& g, int lx, int order, hipStream_t s)
{
    constexpr int TY = kTY[V], D = kD[V];
    constexpr bool EH = kEH[V];
    if constexpr (lds_bytes<T, C, NF, TY>() <= kLdsCap[V]) {
        constexpr int threads = 64 * (EH ? TY : TY + 2);
        const auto kernel = march_kernel<T, C, NF, WS, WG, TY, D, EH, UPD>;
        // workgroups of this kernel that one compute unit holds at once (its
        // registers and LDS decide), queried once per instantiation
        static const int per_cu = [&] {
            int n = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess || n < 1) {
                (void)hipGetLastError();
                n = 1;
            }
            return n;
        }();
        const Launch l = plan(g, TY, lx, per_cu * compute_units(), order);
        hipLaunchKernelGGL(kernel, dim3(l.grid), dim3(threads), 0, s, m, g, l.LX, l.nstrips, l.nchunk, l.nblocks,
                           l.group);
    } else {
        go<T, C, NF, WS, WG, 0, UPD>(m, g, lx, order, s);
    }
}

template <typename T, typename C, int NF, bool WS, bool WG, int UPD, int ZW>
void go_tall(const MarchArgs<T, NF>& m, const Geom& g, int lx, int order, hipStream_t s)
{
    constexpr int TY = tall_ty<NF, ZW>();
    constexpr int threads = 64 * TY * ZW;
    const auto kernel = march_kernel<T, C, NF, WS, WG, TY, 2, true, UPD, ZW>;
    static const int per_cu = [&] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess || n < 1) {
            (void)hipGetLastError();
            n = 1;
        }
        return n;
    }();
    const Launch l = plan(g, TY, lx, per_cu * compute_units(), order, ZW);
    hipLaunchKernelGGL(kernel, dim3(l.grid), dim3(threads), 0, s, m, g, l.LX, l.nstrips, l.nchunk, l.nblocks,
                       l.group);
}

// Default variant and block order per type pair, field count, output set
// and update form.  Chosen from sweeps of every (variant, order) pair in one
// process on the same arrays on MI355X at 4096 x 4096 x 64, and for the
// close candidates from six re-allocations of the arrays in one process (the
// arrays' placement in HBM moves a kernel by up to 15% between allocations;
// one candidate order can be fast in one placement and slow in the next):
//   * the FP64 and FP32 forward and Euler update: 16-column strips with edge
//     waves in natural order (FP64 9.96 ms mean over six placements, range
//     9.22-10.28, against 10.02 ms for 14-column strips with halo waves in
//     XCD ranges and 10.59 ms, range 9.14-11.48, for those in natural order;
//     FP32 5.01 against 5.13 ms);
//   * the FP64 fused pass: 8-column strips with edge waves, pairs of strips
//     per XCD (natural order: 19.61 ms mean over six placements, against 20.00
//     ms in XCD ranges and 19.95 ms for 6-column strips with halo waves; at
//     256 x 256 x 64 and 512 x 512 x 64 10% faster than the latter, as all 8
//     waves compute); the FP64 adjoint: 10-column strips with halo waves in
//     groups of 8 strips per XCD (12 wavefronts, all that its 151 registers
//     allow per unit; in natural order, over arrays in one allocation,
//     13.87-14.27 ms against 13.95-14.53 ms for 6-column strips in XCD
//     ranges, in four placements on two machines; about even over separately
//     allocated arrays).  Their 150-240 registers allow only 8 or 12
//     wavefronts per unit;
//   * FP32 fused pass and adjoint, and the accumulating update of both: 14
//     columns with halo waves in XCD ranges (the FP32 fused pass runs at the
//     speed of a plain copy of its twelve streams; the FP64 accumulating
//     update spills in 16-column strips with edge waves);
//   * FP32 storage with FP64 arithmetic: the adjoint in 10-column strips (11%
//     faster than 6) and the fused pass in 8-column strips with edge waves
//     (9%: its arithmetic sets the pace, and 8 computing waves keep all four
//     SIMDs equally busy), XCD ranges;
//   * 16-bit storage, XCD ranges: the adjoint and the accumulating update in
//     8-column strips with edge waves (8-10% faster), the bfloat16 fused
//     pass in 16-column strips with edge waves (5%), the rest in 14-column
//     strips with halo waves.
// Deeper prefetch (D = 4) measured no faster.  A thread's tuning state
// (pw_set_tuning) can name another variant or order, for sweeps.
template <typename T, typename C, int NF, bool WS, int UPD>
constexpr bool edge16_natural()
{
    return NF == 3 && UPD != 1 && sizeof(T) == sizeof(C) && sizeof(T) >= 4;
}

// Grids whose six arrays of the forward fit in the 256 MB Infinity Cache
// are not HBM-bound: there the forward kernels that default to 16-column
// strips use 8 computing waves in 8-column strips with edge waves in XCD
// ranges instead (256 x 256 x 64 FP64: 0.0377 against 0.0398 ms).
constexpr long long kCacheResidentBytes = 256LL << 20;

template <typename T>
bool cache_resident(const Geom& g)
{
    return 6LL * g.Sx * g.sx * (long long)sizeof(T) <= kCacheResidentBytes;
}

template <typename T, typename C, int NF, bool WS, int UPD>
int default_variant()
{
    if (edge16_natural<T, C, NF, WS, UPD>()) return 6;
    if (NF == 6 && sizeof(T) == 8) return WS ? 5 : 4;
    if (NF == 6 && sizeof(C) == 8) return WS ? 5 : 4;
    if (sizeof(T) == 2) {
        if (NF == 6 && !WS) return 5;
        if (NF == 3 && UPD == 1) return 5;
        if (NF == 6 && std::is_same<T, bf16_t>::value) return 6;
    }
    return 2;
}

// Default block order of the default variant: 0 for XCD ranges, G > 0 for
// groups of G strips per XCD (1: natural order).  The FP64 fused pass takes
// pairs of strips per XCD and the FP64 adjoint groups of 8: most halo columns
// then stay in one XCD's L2 while the device still sweeps one window of the
// grid (at 4096 x 4096 x 64 over arrays in one allocation, two placements:
// fused 19.16 and 19.34 ms against 19.30 and 20.16 ms in natural order,
// adjoint 14.25 and 14.13 ms against 14.41 and 14.57 ms).
template <typename T, typename C, int NF, bool WS, int UPD>
int default_order()
{
    if (NF == 6 && sizeof(T) == 8) return WS ? 2 : 8;
    // the 16-bit forward and Euler update in groups of 16 strips: 1-1.6%
    // faster than XCD ranges in each of five placements
    if (sizeof(T) == 2 && NF == 3 && UPD != 1) return 16;
    return edge16_natural<T, C, NF, WS, UPD>() ? 1 : 0;
}

template <typename T, typename C, int NF, bool WS, bool WG, int UPD = 0>
void dispatch(const MarchArgs<T, NF>& m, const Geom& g, MarchTune t, hipStream_t s)
{
    if (g.nz > NZ && (t.variant < 0 || t.variant == kTallVariant)) {
        // wavefronts per column: the fewest that hold it (up to 256 levels),
        // else the most whose chunks of NZ * ZW - 2 levels idle at most 10%
        // more lanes than the chunking that idles fewest (longer chunks read
        // longer runs of each column: at 400 levels two chunks of four
        // wavefronts, not four of two)
        int zw = g.nz <= 2 * NZ ? 2 : g.nz <= 3 * NZ ? 3 : 4;
        if (t.tall_waves >= 2 && t.tall_waves <= 4) {
            zw = t.tall_waves;
        } else if (g.nz > 4 * NZ) {
            long long lanes[5] = {0, 0, 0, 0, 0}, fewest = -1;
            for (int z = 2; z <= 4; ++z) {
                const long long per = NZ * z - 2;
                lanes[z] = (g.nz + per - 1) / per * per;
                if (fewest < 0 || lanes[z] < fewest) fewest = lanes[z];
            }
            for (int z = 2; z <= 4; ++z)
                if (lanes[z] * 10 <= fewest * 11) zw = z;
        }
        // natural order for the two-wavefront forward (3-7% faster at 100 and
        // 128 levels, 3-13% in chunks of 126 levels at 300, 400 and 600),
        // XCD ranges for the rest (natural is up to 8% slower for the
        // six-field kernels at 200 and 256 levels)
        const int order = t.order >= 0 ? t.order : (NF == 3 && zw == 2) ? 1 : 0;
        if (zw == 2)
            go_tall<T, C, NF, WS, WG, UPD, 2>(m, g, t.lx, order, s);
        else if (zw == 3)
            go_tall<T, C, NF, WS, WG, UPD, 3>(m, g, t.lx, order, s);
        else
            go_tall<T, C, NF, WS, WG, UPD, 4>(m, g, t.lx, order, s);
        return;
    }
    const bool small = edge16_natural<T, C, NF, WS, UPD>() && cache_resident<T>(g);
    const int v = (t.variant >= 0 && t.variant < kVariants) ? t.variant
                : small ? 5 : default_variant<T, C, NF, WS, UPD>();
    const int order = t.order >= 0 ? t.order : small ? 0 : default_order<T, C, NF, WS, UPD>();
    switch (v) {
    case 1: go<T, C, NF, WS, WG, 1, UPD>(m, g, t.lx, order, s); break;
    case 2: go<T, C, NF, WS, WG, 2, UPD>(m, g, t.lx, order, s); break;
    case 3: go<T, C, NF, WS, WG, 3, UPD>(m, g, t.lx, order, s); break;
    case 4: go<T, C, NF, WS, WG, 4, UPD>(m, g, t.lx, order, s); break;
    case 5: go<T, C, NF, WS, WG, 5, UPD>(m, g, t.lx, order, s); break;
    case 6: go<T, C, NF, WS, WG, 6, UPD>(m, g, t.lx, order, s); break;
    default: go<T, C, NF, WS, WG, 0, UPD>(m, g, t.lx, order, s); break;
    }
}

}  // namespace

// The buffer descriptors address one column with 32-bit byte offsets, and a
// lane that must not store gets the offset kOutOfRange: a column must be
// shorter than that for such stores to fall outside it.
template <typename T>
bool march_supported(const Geom& g)
{
    return g.nz >= 2 && g.h <= 32 && (long long)g.Sz * (long long)sizeof(T) < (long long)kOutOfRange;
}

template <typename T, typename C>
void launch_fwd_march(const FwdArgs<T>& a, const Geom& g, MarchTune t, hipStream_t s)
{
    MarchArgs<T, 3> m;
    m.in[0] = a.u;
    m.in[1] = a.v;
    m.in[2] = a.w;
    m.s[0] = a.su;
    m.s[1] = a.sv;
    m.s[2] = a.sw;
    m.gr[0] = m.gr[1] = m.gr[2] = nullptr;
    for (int q = 0; q < 3; ++q) m.b[q] = a.b[q];
    m.tzc1 = a.tzc1;
    m.tzc2 = a.tzc2;
    m.tcx = a.tcx;
    m.tcy = a.tcy;
    m.beta = a.beta;
    if (a.upd == 1)
        dispatch<T, C, 3, true, false, 1>(m, g, t, s);
    else if (a.upd == 2)
        dispatch<T, C, 3, true, false, 2>(m, g, t, s);
    else
        dispatch<T, C, 3, true, false, 0>(m, g, t, s);
}

template <typename T, typename C>
void launch_adj_march(const AdjArgs<T>& a, const Geom& g, MarchTune t, hipStream_t s)
{
    MarchArgs<T, 6> m;
    m.in[0] = a.u;
    m.in[1] = a.v;
    m.in[2] = a.w;
    m.in[3] = a.lu;
    m.in[4] = a.lv;
    m.in[5] = a.lw;
    m.s[0] = a.su;
    m.s[1] = a.sv;
    m.s[2] = a.sw;
    m.gr[0] = a.gu;
    m.gr[1] = a.gv;
    m.gr[2] = a.gw;
    m.b[0] = m.b[1] = m.b[2] = nullptr;
    m.tzc1 = a.tzc1;
    m.tzc2 = a.tzc2;
    m.tcx = a.tcx;
    m.tcy = a.tcy;
    m.beta = 0.0;
    if (a.su)
        dispatch<T, C, 6, true, true>(m, g, t, s);
    else
        dispatch<T, C, 6, false, true>(m, g, t, s);
}

template bool march_supported<double>(const Geom&);
template bool march_supported<float>(const Geom&);
template bool march_supported<_Float16>(const Geom&);
template bool march_supported<bf16_t>(const Geom&);
template void launch_fwd_march<_Float16, float>(const FwdArgs<_Float16>&, const Geom&, MarchTune, hipStream_t);
template void launch_fwd_march<bf16_t, float>(const FwdArgs<bf16_t>&, const Geom&, MarchTune, hipStream_t);
template void launch_adj_march<_Float16, float>(const AdjArgs<_Float16>&, const Geom&, MarchTune, hipStream_t);
template void launch_adj_march<bf16_t, float>(const AdjArgs<bf16_t>&, const Geom&, MarchTune, hipStream_t);
template void launch_fwd_march<double, double>(const FwdArgs<double>&, const Geom&, MarchTune, hipStream_t);
template void launch_fwd_march<float, float>(const FwdArgs<float>&, const Geom&, MarchTune, hipStream_t);
template void launch_fwd_march<float, double>(const FwdArgs<float>&, const Geom&, MarchTune, hipStream_t);
template void launch_adj_march<double, double>(const AdjArgs<double>&, const Geom&, MarchTune, hipStream_t);
template void launch_adj_march<float, float>(const AdjArgs<float>&, const Geom&, MarchTune, hipStream_t);
template void launch_adj_march<float, double>(const AdjArgs<float>&, const Geom&, MarchTune, hipStream_t);
