// HIP kernels of the two-component D3Q19 Shan-Chen step with the
// mass-conserving evaporation sink (Hessling, Xie and Harting,
// arXiv:1701.03637, Sec. II), written for gfx950 (wave64, no MFMA: the step
// is a memory-bound stencil, not a contraction).
//
// Storage. The populations of one instance live in a z-slab-major arena: the
// populations of one z-plane form a contiguous slab, so a pull needs only the
// three slab bases z-1, z, z+1 plus one 32-bit in-plane offset per lane.
// Within a slab, every two-component form keeps population i of both
// components in one plane of (A, B) pairs: the two values a pull takes from
// the same source node are adjacent and move with one load or store
// instruction. For FP32S that is a b64 access instead of two dword ones, which
// doubles the bytes each outstanding memory instruction carries (512^3 step
// 9.02 -> 8.65 ms; the 128^3 one is 1.5 % slower).
// The stored buffer holds post-collision populations f*(t-1); the state S(t)
// of the method (post-stream, post-sink) is obtained by pulling,
//   f_i(x) = f*_i(x - e_i), or f*_opp(i)(x) across a z-seam wall,
// followed by the sink reset of the sink that was active when S(t) formed.
// Storage forms (policies St* below):
//   FP64    f in 19 planes of (A, B) pairs, FP64 arithmetic;
//   FP32S   f - w_i rho0^c (constant shift) in 19 pair planes, FP32
//           arithmetic;
//   FP16S   the same deviations in FP16, 19 pair planes, FP32 arithmetic;
//   FP16N   per-node shift: the rest deviation d_0 = f_0 - w_0 rho0 in FP32
//           and the 18 moving deviations as h_i = d_i - k_i d_0 of the same
//           node in FP16, k_i = w_i / w_0 (h = 0 at rest equilibrium), FP32
//           arithmetic.
// Register values are always deviations from the constant shift rho0^c
// (rho0 = 0 for FP64).
//
// Fused step (one launch per time step): a block owns an xy tile and marches
// along z with a ring of psi planes (tile plus a one-node halo) in LDS: three
// for the register-keeping step, four for the pipelined one. Each tile node
// is pulled once per step into registers; halo nodes are pulled only to form
// their density. Collision reads the 18 neighbour psi values from LDS and
// writes f* aligned to the other buffer.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "lattice.h"

namespace lbsc {

// Storage policies: element type T of the population planes, arithmetic type
// A, and whether the rest population carries a per-node shift (kNode).
// kPair: (A, B) pair planes rather than one plane per component. kHS (per-node
// forms): the power of two the stored FP16 moving values are scaled by.
struct StF64 { using T = double; using A = double; static constexpr bool kNode = false, kPair = true; };
struct StF32S { using T = float; using A = float; static constexpr bool kNode = false, kPair = true; };
struct StF16S { using T = _Float16; using A = float; static constexpr bool kNode = false, kPair = true; };
struct StF16N {
    using T = _Float16;
    using A = float;
    static constexpr bool kNode = true, kPair = true;
    static constexpr float kHS = 1.0f;
};
// FP16NF: FP16N with the moving values stored as 2^12 (d_i - k_i d_0). In the
// near-uniform regions of a slow diffusion those deviations are of order
// 1e-7, below FP16's smallest normal number (6.1e-5), where FP16 keeps only
// an absolute step of 6e-8 and rounds away most of the diffusive flux they
// carry. Scaled, they keep FP16's 11 significant bits down to 1.5e-8; the
// deviations must stay below 16 in magnitude. Scaling by a power of two is
// exact in FP32; the decode then takes one more operation per value.
struct StF16NF {
    using T = _Float16;
    using A = float;
    static constexpr bool kNode = true, kPair = true;
    static constexpr float kHS = 4096.0f;
};

// Slab elements (of T) per in-plane element: 2 x 19 values, or for FP16N
// 18 planes of FP16 pairs plus one plane of FP32 rest pairs (= 4 FP16
// elements per node).
template <class S> constexpr int kSlabPlanes = S::kNode ? 40 : 2 * kQ;

// FP16N encoding constants: k_i = w_i / w_0 as FP32 and 1/K with
// K = 1 + sum_{i>0} k_i evaluated from those same FP32 values, so decoding
// then summing a node reproduces the encoded density deviation. 1/K is split
// into an FP32 head and tail: the head alone sits 4e-8 (relative) below 1/K,
// and that fixed bias, applied to every stored rest population, drifts the
// mass of each component (the two drifts cancel in the total).
__host__ __device__ constexpr float kRatio(int i) { return (float)(wgt(i) / wgt(0)); }
constexpr double kK = 1.0 + 6.0 * (double)(float)(1.0 / 6.0) + 12.0 * (double)(float)(1.0 / 12.0);
constexpr float kInvK = (float)(1.0 / kK);
constexpr float kInvKLo = (float)(1.0 / kK - (double)kInvK);

// y / K rounded once (to within a tail rounding): head product plus tail.
__device__ __forceinline__ float div_k(float y) { return __builtin_fmaf(y, kInvK, y * kInvKLo); }

// Decode of a per-node form's moving value: d_i = k_i d_0(source) + h_i / kHS,
// rounded once (h_i / kHS is exact). Every decode site computes exactly this.
template <class S> __device__ __forceinline__ float decode_h(float k, float d0, _Float16 h)
{
    if constexpr (S::kHS == 1.0f)
        return __builtin_fmaf(k, d0, (float)h);
    else
        return __builtin_fmaf(k, d0, __builtin_fmaf((float)h, 1.0f / S::kHS, 0.0f));
}

// Narrowing of an arithmetic value to the storage type. An FP32 value bound
// for FP16 is formed in a register first: otherwise the compiler may fuse
// the multiply-add that produces it into a mixed-precision FMA that rounds
// once, straight to FP16, where the source rounds to FP32 and then to FP16.
// It does so at some inlined copies of a store and not at others, which
// would make a node's stored bits depend on which copy stored it.
template <typename T, typename A> __device__ __forceinline__ T narrow(A x)
{
    if constexpr (sizeof(T) < sizeof(A)) asm("" : "+v"(x));
    return (T)x;
}

// Bytes per element of population i.
template <class S> __host__ __device__ constexpr uint32_t elem_bytes(int i)
{
    return (S::kNode && i == 0) ? 4u : (uint32_t)sizeof(typename S::T);
}

// Bytes per node of the pair plane of population i (A then B).
template <class S> __host__ __device__ constexpr uint32_t pair_bytes(int i) { return 2u * elem_bytes<S>(i); }

// Bytes between in-plane neighbours in the plane holding element (c, i).
template <class S> __host__ __device__ constexpr uint32_t node_stride(int i)
{
    return S::kPair ? pair_bytes<S>(i) : elem_bytes<S>(i);
}

// Byte offset of the pair plane of population i within a slab of plane
// stride ps; FP16N puts the FP32 rest pairs after the 18 FP16 pair planes.
template <class S>
__host__ __device__ __forceinline__ uint32_t pair_off(int i, uint32_t ps)
{
    static_assert(S::kPair, "pair planes only");
    if constexpr (S::kNode)
        return i == 0 ? 18u * ps * 4u : (uint32_t)(i - 1) * ps * 4u;
    else
        return (uint32_t)i * ps * pair_bytes<S>(i);
}

// Byte offset of element (c, i) of in-plane node 0; node xy adds
// xy * node_stride(i).
template <class S>
__host__ __device__ __forceinline__ uint32_t plane_off(int c, int i, uint32_t ps)
{
    static_assert(S::kPair || !S::kNode, "per-node encodings use pair planes");
    if constexpr (S::kPair)
        return pair_off<S>(i, ps) + (uint32_t)c * elem_bytes<S>(i);
    else
        return (uint32_t)(c * kQ + i) * ps * elem_bytes<S>(i);
}

template <typename A> __device__ __forceinline__ A psi_of(A rho, int psi_exp);
template <> __device__ __forceinline__ double psi_of<double>(double rho, int psi_exp)
{
    return psi_exp ? 1.0 - exp(-rho) : rho;
}
template <> __device__ __forceinline__ float psi_of<float>(float rho, int psi_exp)
{
    return psi_exp ? -expm1f(-rho) : rho;
}

// ---------------------------------------------------------------------------
// Pull of one node: 2 x 19 populations (delta form) and the sink reset.
// ---------------------------------------------------------------------------

// Per-instance constants in the arithmetic type: FP64 from the table's
// doubles, FP32 from its host-rounded FP32 copies (identical values, but
// scalar operands instead of per-lane conversions).
template <typename A> struct Par;
template <> struct Par<double> {
    static __device__ __forceinline__ double shift(const Inst& I, int c) { return I.shift[c]; }
    static __device__ __forceinline__ double omega(const Inst& I, int c) { return I.omega[c]; }
    static __device__ __forceinline__ double ntg(const Inst& I, int c) { return -I.tau[c] * I.g; }
    static __device__ __forceinline__ double psiw(const Inst& I, int c) { return I.psi_w[c]; }
};
template <> struct Par<float> {
    static __device__ __forceinline__ float shift(const Inst& I, int c) { return I.shift_f[c]; }
    static __device__ __forceinline__ float omega(const Inst& I, int c) { return I.omega_f[c]; }
    static __device__ __forceinline__ float ntg(const Inst& I, int c) { return I.ntg_f[c]; }
    static __device__ __forceinline__ float psiw(const Inst& I, int c) { return I.psi_wf[c]; }
};

template <typename A>
struct NodeVals {
    A f[2][kQ];
    A rho[2];    // rho0 + drho
    A drho[2];   // sum of the stored deviations
};

// Populations are read and written with raw buffer instructions: the
// resource (4 scalar registers) points at one z-slab, the plane offset
// (c*19 + i)*ps*sizeof(T) is a scalar offset and the in-plane offset a single
// vector register shared by both components and all planes. A slab is below
// 4 GiB (checked at create), so no access is clipped.
using Rsrc = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ Rsrc slab_rsrc(const void* p)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, -1, 0x00020000);
}

// live = false: a resource with no records, so every access is out of
// range and loads return zero without touching memory (stores are dropped).
template <typename T> __device__ __forceinline__ T bload(Rsrc r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ float bload<float>(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <> __device__ __forceinline__ double bload<double>(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
template <> __device__ __forceinline__ _Float16 bload<_Float16>(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(_Float16, (unsigned short)__builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0));
}

// Population stores carry the non-temporal cache policy (bit 1 of the
// auxiliary operand): the next step reads them only after the whole lattice
// has been written, so there is no reuse to keep them in cache for.
constexpr int kStorePolicy = 2;

__device__ __forceinline__ void bstore(float v, Rsrc r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)voff, (int)soff, kStorePolicy);
}
__device__ __forceinline__ void bstore(double v, Rsrc r, uint32_t voff, uint32_t soff)
{
    using U2 = unsigned int __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, (int)voff, (int)soff, kStorePolicy);
}
__device__ __forceinline__ void bstore(_Float16 v, Rsrc r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)voff, (int)soff, kStorePolicy);
}

// One (A, B) pair of adjacent elements in one instruction.
template <typename T> struct Pair {
    T a, b;
};
using U2 = unsigned int __attribute__((ext_vector_type(2)));
using U4 = unsigned int __attribute__((ext_vector_type(4)));
using H2 = _Float16 __attribute__((ext_vector_type(2)));
using F2 = float __attribute__((ext_vector_type(2)));
using D2 = double __attribute__((ext_vector_type(2)));

template <typename A> struct Psi2T;
template <> struct Psi2T<float> { using type = F2; };
template <> struct Psi2T<double> { using type = D2; };
template <typename A> using Psi2 = typename Psi2T<A>::type;

// One LDS plane of psi over a tile footprint of FP nodes. PAIR keeps
// (psi^A, psi^B) of a node together, so the force stencil reads both
// components of a neighbour with one instruction; otherwise one plane per
// component. Pairs measured faster for FP32S (134.6 -> 132.9 us on the 128^3
// droplet) and FP16N, slower for FP16S (92.0 -> 95.9 us), and made the FP64
// step spill.
template <typename A, int FP, bool PAIR> struct PsiPlane;
template <typename A, int FP> struct PsiPlane<A, FP, true> {
    static constexpr bool kPair = true;
    Psi2<A> v[FP];
    __device__ __forceinline__ void put(int i, A a, A b) { v[i] = Psi2<A>{a, b}; }
    __device__ __forceinline__ Psi2<A> get(int i) const { return v[i]; }
};
template <typename A, int FP> struct PsiPlane<A, FP, false> {
    static constexpr bool kPair = false;
    A v[2][FP];
    __device__ __forceinline__ void put(int i, A a, A b)
    {
        v[0][i] = a;
        v[1][i] = b;
    }
    __device__ __forceinline__ Psi2<A> get(int i) const { return Psi2<A>{v[0][i], v[1][i]}; }
};
template <class S> constexpr bool kPsiPair = std::is_same_v<S, StF32S> || S::kNode;

template <typename T> __device__ __forceinline__ Pair<T> bload2(Rsrc r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ Pair<float> bload2<float>(Rsrc r, uint32_t voff, uint32_t soff)
{
    const F2 v = __builtin_bit_cast(F2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
    return {v.x, v.y};
}
template <> __device__ __forceinline__ Pair<double> bload2<double>(Rsrc r, uint32_t voff, uint32_t soff)
{
    const D2 v = __builtin_bit_cast(D2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
    return {v.x, v.y};
}
template <> __device__ __forceinline__ Pair<_Float16> bload2<_Float16>(Rsrc r, uint32_t voff, uint32_t soff)
{
    const H2 v = __builtin_bit_cast(H2, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
    return {v.x, v.y};
}

__device__ __forceinline__ void bstore2(float a, float b, Rsrc r, uint32_t voff, uint32_t soff)
{
    // Register operands: built straight from an array element, the pair is
    // widened into a two-element load from the array, which then can no
    // longer live in registers.
    asm("" : "+v"(a), "+v"(b));
    const F2 v = {a, b};
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, (int)voff, (int)soff, kStorePolicy);
}
__device__ __forceinline__ void bstore2(double a, double b, Rsrc r, uint32_t voff, uint32_t soff)
{
    const D2 v = {a, b};
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, v), r, (int)voff, (int)soff, kStorePolicy);
}
__device__ __forceinline__ void bstore2(_Float16 a, _Float16 b, Rsrc r, uint32_t voff, uint32_t soff)
{
    const H2 v = {a, b};
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)voff, (int)soff, kStorePolicy);
}

// One (A, B) pair of FP16 values as loaded: one dword.
__device__ __forceinline__ H2 bload_h2(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(H2, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}

// Raw stored values of one pulled node, as loaded: the loads can be issued
// well before the values are decoded. FP16N carries, per population, the
// moving value h_i and the FP32 rest deviation d_0 of its source node. FP16
// pairs stay one (A, B) dword per population: split into per-component
// arrays, the compiler re-packed the halves of adjacent populations with a
// permute per load.
template <class S> constexpr bool kHalfPair = S::kPair && sizeof(typename S::T) == 2;
template <class S, bool NODE = S::kNode, bool HP = kHalfPair<S>> struct RawNode {
    typename S::T v[2][kQ];
};
template <class S> struct RawNode<S, false, true> {
    H2 v2[kQ];
};
template <class S> struct RawNode<S, true, true> {
    float d0[2][kQ];
    H2 h2[kQ];
};

// Source of each population of the pull of node (x, y, z): population i
// comes from x - e_i, or is the reflected population of the node itself
// across a wall on the z seam. z is block-uniform for every pull, so the
// slab resources and the wall branch are scalar.
template <class S>
struct PullAddr {
    Rsrc sl[3];             // slabs read by e_z = +1, 0, -1
    uint32_t xs[3], ys[3];  // x-1, x, x+1 and (y-1, y, y+1) * nx
    bool wall_lo, wall_hi;
    uint32_t ps;

    __device__ __forceinline__ PullAddr(const typename S::T* __restrict__ src, const Inst& I, int x, int y, int z)
    {
        const int nx = I.nx, ny = I.ny, nz = I.nz;
        xs[0] = (uint32_t)wrap(x - 1, nx); xs[1] = (uint32_t)x; xs[2] = (uint32_t)wrap(x + 1, nx);
        ys[0] = (uint32_t)(wrap(y - 1, ny) * nx); ys[1] = (uint32_t)(y * nx); ys[2] = (uint32_t)(wrap(y + 1, ny) * nx);
        wall_lo = I.wall_z && z == 0;
        wall_hi = I.wall_z && z == nz - 1;
        // Directions with e_z = +1 read slab z-1, or slab z when they reflect
        // off the wall below; e_z = -1 likewise with z+1. Choosing the slab
        // pointer (not the resource) keeps every resource a plain scalar
        // value.
        const typename S::T* pz = src + (int64_t)z * I.slab;
        const typename S::T* pm = wall_lo ? pz : src + (int64_t)wrap(z - 1, nz) * I.slab;
        const typename S::T* pp = wall_hi ? pz : src + (int64_t)wrap(z + 1, nz) * I.slab;
        sl[0] = slab_rsrc(pm);
        sl[1] = slab_rsrc(pz);
        sl[2] = slab_rsrc(pp);
        ps = (uint32_t)I.ps;
    }
    __device__ __forceinline__ bool refl(int i) const { return (ez(i) > 0 && wall_lo) || (ez(i) < 0 && wall_hi); }
    __device__ __forceinline__ int q(int i) const { return refl(i) ? opp(i) : i; }
    __device__ __forceinline__ Rsrc rsrc(int i) const { return sl[1 - ez(i)]; }
    __device__ __forceinline__ uint32_t xy(int i) const
    {
        return refl(i) ? ys[1] + xs[1] : ys[1 - ey(i)] + xs[1 - ex(i)];
    }
};

// Loads of the pull of node (x, y, z) for storage without a per-node rest
// encoding, straight into v.
template <class S>
__device__ __forceinline__ void pull_vals(const typename S::T* __restrict__ src, const Inst& I, int x, int y, int z,
                                          typename S::T (&v)[2][kQ])
{
    using T = typename S::T;
    static_assert(!S::kNode, "per-node encodings load through RawNode");
    const PullAddr<S> a(src, I, x, y, z);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        if constexpr (S::kPair) {
            const Pair<T> p = bload2<T>(a.rsrc(i), a.xy(i) * pair_bytes<S>(i), pair_off<S>(a.q(i), a.ps));
            v[0][i] = p.a;
            v[1][i] = p.b;
        } else {
#pragma unroll
            for (int c = 0; c < 2; ++c)
                v[c][i] = bload<T>(a.rsrc(i), a.xy(i) * (uint32_t)sizeof(T), plane_off<S>(c, a.q(i), a.ps));
        }
    }
}

// Issues the loads of the pull of node (x, y, z) into a raw set.
template <class S>
__device__ __forceinline__ void pull_raw(const typename S::T* __restrict__ src, const Inst& I, int x, int y, int z,
                                         RawNode<S>& w)
{
    using T = typename S::T;
    if constexpr (S::kNode) {
        const PullAddr<S> a(src, I, x, y, z);
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const Pair<float> d = bload2<float>(a.rsrc(i), a.xy(i) * pair_bytes<S>(0), pair_off<S>(0, a.ps));
            w.d0[0][i] = d.a;
            w.d0[1][i] = d.b;
            if (i != 0) w.h2[i] = bload_h2(a.rsrc(i), a.xy(i) * pair_bytes<S>(i), pair_off<S>(a.q(i), a.ps));
        }
    } else if constexpr (kHalfPair<S>) {
        const PullAddr<S> a(src, I, x, y, z);
#pragma unroll
        for (int i = 0; i < kQ; ++i) w.v2[i] = bload_h2(a.rsrc(i), a.xy(i) * pair_bytes<S>(i), pair_off<S>(a.q(i), a.ps));
    } else {
        pull_vals<S>(src, I, x, y, z, w.v);
    }
}

// FP16N moving values alone: the pipelined step takes the rest values of the
// source nodes from an LDS ring rather than with 19 loads per node.
template <class S> struct RawH {
    H2 h2[kQ];
};

// Issues the loads of the moving values of the pull of node (x, y, z).
template <class S>
__device__ __forceinline__ void pull_h(const typename S::T* __restrict__ src, const Inst& I, int x, int y, int z,
                                       RawH<S>& w)
{
    using T = typename S::T;
    static_assert(S::kNode, "per-node rest encodings only");
    const PullAddr<S> a(src, I, x, y, z);
#pragma unroll
    for (int i = 1; i < kQ; ++i) w.h2[i] = bload_h2(a.rsrc(i), a.xy(i) * pair_bytes<S>(i), pair_off<S>(a.q(i), a.ps));
}

// Decodes the raw values into deviations f_i - w_i rho0.
template <class S, typename A = typename S::A>
__device__ __forceinline__ void decode_raw(const RawNode<S>& w, NodeVals<A>& v)
{
#pragma unroll
    for (int i = 0; i < kQ; ++i)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if constexpr (S::kNode) {
                // d_i = k_i d_0(source) + h_i(source) / kHS
                v.f[c][i] = i == 0 ? w.d0[c][0] : decode_h<S>(kRatio(i), w.d0[c][i], w.h2[i][c]);
            } else if constexpr (kHalfPair<S>) {
                v.f[c][i] = (A)w.v2[i][c];
            } else {
                v.f[c][i] = (A)w.v[c][i];
            }
        }
}

template <class S, typename A = typename S::A>
__device__ __forceinline__ void pull_node(const typename S::T* __restrict__ src, const Inst& I, int x, int y, int z,
                                          NodeVals<A>& v)
{
    RawNode<S> w;
    pull_raw<S>(src, I, x, y, z, w);
    decode_raw<S>(w, v);
}

// Stores the node's f* (deviations in v) into slab z of dst.
template <class S, typename A = typename S::A>
__device__ __forceinline__ void store_node(typename S::T* __restrict__ dst, const Inst& I, int z, uint32_t xy,
                                           const NodeVals<A>& v)
{
    using T = typename S::T;
    const Rsrc dz = slab_rsrc(dst + (int64_t)z * I.slab);
    const uint32_t ps = (uint32_t)I.ps;
    if constexpr (S::kNode) {
        // moving deviations relative to k_i d_0 in FP16 (times kHS); the rest
        // deviation takes their rounding so the decoded node sums to drho (up
        // to FP32 rounding).
        float hsum[2] = {0.f, 0.f};
#pragma unroll
        for (int i = 1; i < kQ; ++i) {
            // each value rounds to FP32, is scaled exactly, then rounds to
            // FP16 (one packed conversion of the pair); the running sums read
            // the FP16 halves directly, unscaled exactly
            float a0 = v.f[0][i] - kRatio(i) * v.f[0][0], a1 = v.f[1][i] - kRatio(i) * v.f[1][0];
            if constexpr (S::kHS != 1.0f) {
                a0 *= S::kHS;
                a1 *= S::kHS;
            }
            asm("" : "+v"(a0), "+v"(a1));
            const H2 h = __builtin_convertvector(F2{a0, a1}, H2);
            hsum[0] = __builtin_fmaf((float)h[0], 1.0f / S::kHS, hsum[0]);
            hsum[1] = __builtin_fmaf((float)h[1], 1.0f / S::kHS, hsum[1]);
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, h), dz, (int)(xy * pair_bytes<S>(i)),
                                                  (int)pair_off<S>(i, ps), kStorePolicy);
        }
        bstore2(div_k(v.drho[0] - hsum[0]), div_k(v.drho[1] - hsum[1]), dz, xy * pair_bytes<S>(0),
                pair_off<S>(0, ps));
    } else if constexpr (S::kPair) {
#pragma unroll
        for (int i = 0; i < kQ; ++i)
            bstore2(narrow<T>(v.f[0][i]), narrow<T>(v.f[1][i]), dz, xy * pair_bytes<S>(i), pair_off<S>(i, ps));
    } else {
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int i = 0; i < kQ; ++i)
                bstore(narrow<T>(v.f[c][i]), dz, xy * (uint32_t)sizeof(T), plane_off<S>(c, i, ps));
    }
}

template <typename A>
__device__ __forceinline__ void node_density(const Inst& I, NodeVals<A>& v)
{
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        A r = (A)0;
#pragma unroll
        for (int i = 0; i < kQ; ++i) r += v.f[c][i];
        v.drho[c] = r;
        v.rho[c] = Par<A>::shift(I, c) + r;
    }
}

// FP64 arithmetic follows the plain formulas; FP32 arithmetic moves every
// rounding of a mass-conserving update into the rest population, so that the
// stored deviations of a node sum exactly (up to one rounding) to its density.
template <typename A> constexpr bool kPlain = false;
template <> constexpr bool kPlain<double> = true;

template <typename A>
__device__ __forceinline__ void absorb_rest(A (&f)[kQ], A total)
{
    A moving = (A)0;
#pragma unroll
    for (int i = 1; i < kQ; ++i) moving += f[i];
    f[0] = total - moving;
}

// Mass bookkeeping of FP32 storage (FP32S). Rounding the rest population to
// nearest would change a node's stored mass by up to half an FP32 ulp with
// the same sign at every node of a uniform region, a drift that grows with
// the region's volume and the number of steps. The rest instead takes the
// node's exact residual, rounded stochastically: unbiased, with a draw that
// hashes the node and the value being rounded (deterministic, the same in
// every kernel variant, uncorrelated between nodes), so the stored mass
// changes only by a zero-mean error per node and step.
//  - Collision: the residual is f_0 + sum_{i>0} (f_i - f'_i), the pre-collision
//    rest plus the moving populations' increments. The increments are small
//    near equilibrium, so their FP32 differences and sum carry errors far
//    below the rest's ulp; a TwoSum gives the exact remainder to round. One
//    hash per node draws for both components (16 bits each).
//  - Sink reset: the node's stored mass is summed exactly in FP64 (19 FP32
//    values; their exponents span far less than FP64's extra 29 bits) and E
//    books the exact change of its A mass.
template <class S> constexpr bool kExact = std::is_same_v<S, StF32S>;

template <typename A>
__device__ __forceinline__ double sum64(const A (&f)[kQ], int from = 0)
{
    double m = 0.0;
#pragma unroll
    for (int i = from; i < kQ; ++i) m += (double)f[i];
    return m;
}

// 32-bit avalanche of the MurmurHash3 finaliser (Appleby), public domain.
__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// x rounded to FP32 up or down with probabilities that make the result's
// expectation x, from the draw hash(key, bits of x).
__host__ __device__ __forceinline__ float round_sr(double x, uint32_t key)
{
    const float f = (float)x;
    const double r = x - (double)f;   // exact
    const uint64_t xb = __builtin_bit_cast(uint64_t, x);
    const uint32_t h = fmix32(key ^ fmix32((uint32_t)xb ^ (uint32_t)(xb >> 32)));
    // the FP32 neighbour of f on the side of x
    uint32_t b = __builtin_bit_cast(uint32_t, f);
    if (f == 0.0f) b = r > 0.0 ? 1u : 0x80000001u;
    else b += ((r > 0.0) == (f > 0.0f)) ? 1u : 0xffffffffu;
    const float g = __builtin_bit_cast(float, b);
    const double gap = __builtin_fabs((double)g - (double)f);
    const double u = (double)(h >> 8) * (1.0 / 16777216.0);
    return (r != 0.0 && u * gap < __builtin_fabs(r)) ? g : f;
}

// TwoSum (Knuth): s = fl(a + b) and the exact remainder r = (a + b) - s.
__host__ __device__ __forceinline__ void two_sum(float a, float b, float& s, float& r)
{
    s = a + b;
    const float bb = s - a;
    r = (a - (s - bb)) + (b - bb);
}

// s + r (|r| below half an ulp of s) rounded stochastically: s, or its FP32
// neighbour on the side of r with probability |r| / gap, decided by the
// uniform draw u in [0, 1). The gap is a power of two, so u * gap is exact.
__host__ __device__ __forceinline__ float sr_pick(float s, float r, float u)
{
    uint32_t sb = __builtin_bit_cast(uint32_t, s);
    if (s == 0.0f) sb = r > 0.0f ? 1u : 0x80000001u;
    else sb += ((r > 0.0f) == (s > 0.0f)) ? 1u : 0xffffffffu;
    const float g = __builtin_bit_cast(float, sb);
    const float gap = __builtin_fabsf(g - s);
    return (r != 0.0f && u * gap < __builtin_fabsf(r)) ? g : s;
}

__host__ __device__ __forceinline__ uint32_t rotl32(uint32_t x, int k) { return (x << k) | (x >> (32 - k)); }

// a + b rounded to FP32 stochastically, from a 24-bit draw that hashes the
// key and the bits of the TwoSum pair.
__host__ __device__ __forceinline__ float round_sr_sum(float a, float b, uint32_t key)
{
    float s, r;
    two_sum(a, b, s, r);
    const uint32_t h = fmix32(key ^ fmix32(__builtin_bit_cast(uint32_t, s) ^ (__builtin_bit_cast(uint32_t, r) << 1)));
    return sr_pick(s, r, (float)(h >> 8) * (1.0f / 16777216.0f));
}

// The same for a node's two components at once: one hash of the key and the
// bits of both TwoSum pairs gives each component a 16-bit draw (the rounding
// stays unbiased to 2^-16 of an ulp).
__host__ __device__ __forceinline__ void round_sr_sum2(const float (&a)[2], const float (&b)[2], uint32_t key,
                                                       float (&out)[2])
{
    float s[2], r[2];
    two_sum(a[0], b[0], s[0], r[0]);
    two_sum(a[1], b[1], s[1], r[1]);
    const uint32_t m = (key * 0x9e3779b1u) ^ __builtin_bit_cast(uint32_t, s[0]) ^
                       (__builtin_bit_cast(uint32_t, r[0]) << 1) ^ rotl32(__builtin_bit_cast(uint32_t, s[1]), 16) ^
                       rotl32(__builtin_bit_cast(uint32_t, r[1]), 9);
    const uint32_t h = fmix32(m);
    out[0] = sr_pick(s[0], r[0], (float)(h >> 16) * (1.0f / 65536.0f));
    out[1] = sr_pick(s[1], r[1], (float)(h & 0xffffu) * (1.0f / 65536.0f));
}

// Rest population of an FP32S node whose stored deviations must sum to m
// (exact FP64): m minus the exact sum of the moving ones, rounded
// stochastically.
__device__ __forceinline__ void absorb_rest_exact(float (&f)[kQ], double m, uint32_t key)
{
    f[0] = round_sr(m - sum64(f, 1), key);
}

// Sink reset (Sec. II C): A -> f^eq(rho_H, 0), B -> f^eq(rhoA + rhoB - rho_H, 0)
// from the densities pulled in this step. Returns rhoA_pre - rho_H in FP64:
// for FP32S the exact change of the node's stored A mass (its new stored
// density is rho_H up to the rest's zero-mean rounding), otherwise from the
// exact FP64 sum of the pulled deviations. key: the node's index, for the
// stochastic rounding.
template <typename A, bool EX = false>
__device__ __forceinline__ double sink_reset(const Inst& I, NodeVals<A>& v, uint32_t key)
{
    const double rho_h = I.reset.rho_h;
    const double ma = kPlain<A> ? (double)v.drho[0] : sum64(v.f[0]);
    const double mb = kPlain<A> ? (double)v.drho[1] : sum64(v.f[1]);
    double flux = I.shift[0] + ma - rho_h;
    // rho_H - rho0^A is exact in FP64; the partner deviation
    // rhoB_H - rho0^B = (rho0^A - rho_H) + drho^A + drho^B is formed from
    // small terms, so no O(1) density is rounded.
    A da = (A)(rho_h - I.shift[0]);
    // The A reset is the same at every sink node; kept opaque so that it is
    // formed here, at the (few) sink nodes, not hoisted out of the march
    // into 19 registers.
    asm volatile("" : "+v"(da));
    A db;
    if constexpr (EX) db = (A)(I.shift[0] - rho_h + ma + mb);
    else db = (A)(I.shift[0] - rho_h) + v.drho[0] + v.drho[1];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        v.f[0][i] = (A)wgt(i) * da;
        v.f[1][i] = (A)wgt(i) * db;
    }
    if constexpr (EX) {
        // A takes rho_H exactly up to its rest's rounding; B the rest of
        // the node's stored mass; E books the exact change of A.
        absorb_rest_exact(v.f[0], rho_h - I.shift[0], key * 2u);
        const double ma_new = sum64(v.f[0]);
        absorb_rest_exact(v.f[1], ma + mb - ma_new, key * 2u + 1u);
        flux = ma - ma_new;
    } else if constexpr (!kPlain<A>) {
        // FP32 weights do not sum to 1 exactly; the rest population takes
        // the residual so each component holds exactly its reset density.
        absorb_rest(v.f[0], da);
        absorb_rest(v.f[1], db);
    }
    node_density<A>(I, v);
    return flux;
}

// ---------------------------------------------------------------------------
// Collision of one fluid node (Eqs. (LBM), (eqdis), (sc); Sec. II B shift).
// S[c] = sum_{i>0} w_i psi^{cbar}(x + e_i) e_i, the neighbour sum of Eq. (sc).
// ---------------------------------------------------------------------------

// 1/x: IEEE division in FP64, the hardware reciprocal (1 ulp) in FP32.
template <typename A> __device__ __forceinline__ A recip(A x);
template <> __device__ __forceinline__ double recip<double>(double x) { return 1.0 / x; }
template <> __device__ __forceinline__ float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// RESID: the FP32 rest takes the residual drho - sum of the moving values, so
// the node's FP32 values sum to drho; FP16N skips it, its store encodes the
// rest from drho itself.
template <typename A, bool EX = false, bool RESID = true>
__device__ __forceinline__ void collide_node(const Inst& I, NodeVals<A>& v, const A S[2][3], A psiA, A psiB,
                                             uint32_t key)
{
    A j[2][3];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        A jx = 0, jy = 0, jz = 0;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            if (ex(i)) jx += ex(i) > 0 ? v.f[c][i] : -v.f[c][i];
            if (ey(i)) jy += ey(i) > 0 ? v.f[c][i] : -v.f[c][i];
            if (ez(i)) jz += ez(i) > 0 ? v.f[c][i] : -v.f[c][i];
        }
        j[c][0] = jx; j[c][1] = jy; j[c][2] = jz;
    }
    // u' = sum_c j^c / sum_c rho^c; the force shift tau^c F^c / rho^c with
    // F^c = -psi^c g S^c is applied as u^c = u' + k^c S^c.
    const A inv_rt = recip<A>(v.rho[0] + v.rho[1]);
    const A up[3] = {(j[0][0] + j[1][0]) * inv_rt, (j[0][1] + j[1][1]) * inv_rt, (j[0][2] + j[1][2]) * inv_rt};
    const A psi[2] = {psiA, psiB};
    // FP32S: each component's pre-collision rest and the sum of its moving
    // populations' increments, from which the rest takes the node's exact
    // stored mass
    A f0[2], dsum[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const A rho = v.rho[c];
        // k^c = -tau^c g psi^c / rho^c. In FP32, psi = rho gives psi / rho = 1
        // exactly; for psi = 1 - exp(-rho) the reciprocal overflows below the
        // smallest normal density, where psi / rho takes its limit 1. At
        // rho = 0, f^eq vanishes whatever the velocity.
        A kc;
        if constexpr (kPlain<A>)
            kc = rho != (A)0 ? Par<A>::ntg(I, c) * psi[c] * recip<A>(rho) : (A)0;
        else if (!I.psi_exp)
            kc = Par<A>::ntg(I, c);
        else
            kc = __builtin_fabsf(rho) >= __FLT_MIN__ ? Par<A>::ntg(I, c) * psi[c] * recip<A>(rho)
                                                      : (rho != (A)0 ? Par<A>::ntg(I, c) : (A)0);
        const A u[3] = {up[0] + kc * S[c][0], up[1] + kc * S[c][1], up[2] + kc * S[c][2]};
        const A uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const A drho = v.drho[c];
        const A omega = Par<A>::omega(I, c);
        // Rest: f^eq_0 = w_0 (drho + rho (-1.5 u.u)) in deviation form.
        const A base0 = drho - (A)1.5 * rho * uu;
        f0[c] = v.f[c][0];
        dsum[c] = (A)0;
        v.f[c][0] = v.f[c][0] - (v.f[c][0] - (A)wgt(0) * base0) * omega;
        // Opposite pairs (i, i+1) share w, |e.u| and the even part of q.
#pragma unroll
        for (int i = 1; i < kQ; i += 2) {
            const A eu = (A)ex(i) * u[0] + (A)ey(i) * u[1] + (A)ez(i) * u[2];
            const A even = (A)wgt(i) * (base0 + (A)4.5 * rho * eu * eu);
            const A odd = (A)wgt(i) * (A)3 * rho * eu;
            const A fp = even + odd, fm = even - odd;
            const A a = v.f[c][i], b = v.f[c][i + 1];
            v.f[c][i] = a - (a - fp) * omega;
            v.f[c][i + 1] = b - (b - fm) * omega;
            if constexpr (EX) {
                dsum[c] += a - v.f[c][i];
                dsum[c] += b - v.f[c][i + 1];
            }
        }
        // BGK conserves each component's mass exactly (sum_i f^eq_i = rho).
        if constexpr (!EX && RESID && !kPlain<A>) absorb_rest(v.f[c], drho);
    }
    if constexpr (EX) {
        float r0[2];
        round_sr_sum2(f0, dsum, key, r0);
        v.f[0][0] = r0[0];
        v.f[1][0] = r0[1];
    }
}

// ---------------------------------------------------------------------------
// The fused step kernel.
// ---------------------------------------------------------------------------

// Neighbour sum of Eq. (sc) from the psi planes z-1, z, z+1 held in LDS
// (footprint row stride `row`): S[c] = sum_i w_i psi^{cbar}(x + e_i)
// e_i, taken over opposite pairs as w_i e_i times the difference of psi across
// the node, axis and diagonal classes accumulated separately and weighted
// once. cI[1 + e] / rI[1 + e] are the footprint column / row of the
// neighbour at offset e in x / y.
template <typename A, class P>
__device__ __forceinline__ void force_sum(const P& pm, const P& p0, const P& pp, const int cI[3], const int rI[3],
                                          int row, A S[2][3])
{
    A S1[2][3] = {{0, 0, 0}, {0, 0, 0}}, S2[2][3] = {{0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int i = 1; i < kQ; i += 2) {
        const P& lp = ez(i) < 0 ? pm : (ez(i) > 0 ? pp : p0);
        const P& lm = ez(i) > 0 ? pm : (ez(i) < 0 ? pp : p0);
        const int fp = rI[1 + ey(i)] * row + cI[1 + ex(i)];
        const int fm = rI[1 - ey(i)] * row + cI[1 - ex(i)];
        Psi2<A> qp, qm;
        if constexpr (P::kPair) {
            qp = lp.get(fp);
            qm = lm.get(fm);
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            A dpsi;
            if constexpr (P::kPair)
                dpsi = qp[1 - c] - qm[1 - c];
            else
                dpsi = lp.v[1 - c][fp] - lm.v[1 - c][fm];
            A(&acc)[3] = i < 7 ? S1[c] : S2[c];
            if (ex(i)) acc[0] += ex(i) > 0 ? dpsi : -dpsi;
            if (ey(i)) acc[1] += ey(i) > 0 ? dpsi : -dpsi;
            if (ez(i)) acc[2] += ez(i) > 0 ? dpsi : -dpsi;
        }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) S[c][dd] = (A)wgt(1) * S1[c][dd] + (A)wgt(7) * S2[c][dd];
}

template <int NT> struct Foot {
    // Largest (tw + 2)(th + 2) = tw*th + 2(tw + th) + 4 over tiles with
    // tw*th <= NT and tw, th <= NT: tw + th peaks at the extremes (NT x 1).
    static constexpr int kMax = 3 * NT + 6;
};

__device__ __forceinline__ void ring_coord(int r, int tw, int th, int& fx, int& fy)
{
    const int row = tw + 2;
    if (r < row) { fx = r - 1; fy = -1; return; }
    r -= row;
    if (r < row) { fx = r - 1; fy = th; return; }
    r -= row;
    if (r < th) { fx = -1; fy = r; return; }
    r -= th;
    fx = tw; fy = r;
}

// Index of node (x, y, z) in the kernels' lattice: the key of its rest
// populations' stochastic rounding (FP32S).
__device__ __forceinline__ uint32_t node_key(const Inst& I, int x, int y, int z)
{
    return ((uint32_t)z * (uint32_t)I.ny + (uint32_t)y) * (uint32_t)I.nx + (uint32_t)x;
}

__device__ __forceinline__ int xcd_item(int b, int n_items)
{
    // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous run of items so neighbouring tiles share its L2.
    const int per = (n_items + 7) >> 3;
    return (b & 7) * per + (b >> 3);
}

// Lane 0's value as a wave-uniform (scalar-register) double.
__device__ __forceinline__ double wave_uniform(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <typename A>
__device__ __forceinline__ A block_sum_wave(A v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// KEEP = true: a tile node's pulled populations stay in registers from the
// plane-ahead density pass to its collision (two population sets live).
// KEEP = false: the density pass keeps only the densities and the collision
// pulls the node again (one set live, higher occupancy, second read from L2).
template <class St, int NT, bool KEEP>
__global__ __launch_bounds__(NT) void k_step(const Inst* __restrict__ insts, const Item* __restrict__ items,
                                             int n_items, const typename St::T* __restrict__ src,
                                             typename St::T* __restrict__ dst, double* __restrict__ eacc)
{
    using T = typename St::T;
    using A = typename St::A;
    constexpr int FP = Foot<NT>::kMax;
    __shared__ PsiPlane<A, FP, kPsiPair<St>> psiS[3];
    __shared__ double red[NT / 64];

    const int k = xcd_item(blockIdx.x, n_items);
    if (k >= n_items) return;
    const Item it = items[k];
    if (it.nzc == 0) return;  // padding of an XCD's run of items
    const Inst I = insts[it.inst];
    const T* __restrict__ s = src + I.base;
    T* __restrict__ d = dst + I.base;

    const int t = threadIdx.x;
    const int tw = it.tw, th = it.th;
    const int row = tw + 2;
    const bool own = t < tw * th;
    const int tx = own ? t % tw : 0;
    const int ty = own ? t / tw : 0;
    const int x = wrap(it.x0 + tx, I.nx);
    const int y = wrap(it.y0 + ty, I.ny);
    const int nring = 2 * row + 2 * th;
    const int z0 = it.z0, z1 = it.z0 + it.nzc;
    const bool book = I.count_reset != 0 && I.reset.kind != kSinkNone;
    double eflux = 0.0;

    NodeVals<A> cur, nxt;

    // Pull plane zq (logical z) into LDS slot sl; tile nodes keep their values.
    // Halo nodes first, so only one extra population set is live at a time.
    auto load_plane = [&](int zq, int sl, NodeVals<A>& keep_or_tmp) {
        const int zp = psi_plane(zq, I.nz, I.wall_z);
        const bool wallc = beyond_wall(I, zq);
        for (int r = t; r < nring; r += NT) {
            int fx, fy;
            ring_coord(r, tw, th, fx, fy);
            const int hx = wrap(it.x0 + fx, I.nx), hy = wrap(it.y0 + fy, I.ny);
            NodeVals<A> h;
            pull_node<St>(s, I, hx, hy, zp, h);
            node_density<A>(I, h);
            if (in_sink(I.reset, hx, hy, zp, I.nx, I.ny, I.nz)) sink_reset<A, kExact<St>>(I, h, node_key(I, hx, hy, zp));
            const int fi = (fy + 1) * row + fx + 1;
            if (wallc) psiS[sl].put(fi, Par<A>::psiw(I, 0), Par<A>::psiw(I, 1));
            else psiS[sl].put(fi, psi_of<A>(h.rho[0], I.psi_exp), psi_of<A>(h.rho[1], I.psi_exp));
        }
        if (own) {
            NodeVals<A> tmp;
            NodeVals<A>& keep = KEEP ? keep_or_tmp : tmp;
            pull_node<St>(s, I, x, y, zp, keep);
            node_density<A>(I, keep);
            if (in_sink(I.reset, x, y, zp, I.nx, I.ny, I.nz)) {
                const double fl = sink_reset<A, kExact<St>>(I, keep, node_key(I, x, y, zp));
                if (book && zq >= z0 && zq < z1) eflux += fl;
            }
            const int fi = (ty + 1) * row + tx + 1;
            if (wallc) psiS[sl].put(fi, Par<A>::psiw(I, 0), Par<A>::psiw(I, 1));
            else psiS[sl].put(fi, psi_of<A>(keep.rho[0], I.psi_exp), psi_of<A>(keep.rho[1], I.psi_exp));
        }
    };

    // Collide plane z of the tile node held in v and store f* to dst.
    auto collide_plane = [&](int z, NodeVals<A>& kept) {
        if (!own) return;
        NodeVals<A> tmp;
        NodeVals<A>& v = KEEP ? kept : tmp;
        if constexpr (!KEEP) {
            pull_node<St>(s, I, x, y, z, v);
            node_density<A>(I, v);
            if (in_sink(I.reset, x, y, z, I.nx, I.ny, I.nz)) sink_reset<A, kExact<St>>(I, v, node_key(I, x, y, z));
        }
        const int sm = (z - z0) % 3, s0 = (z - z0 + 1) % 3, sp = (z - z0 + 2) % 3;
        const uint32_t xy = (uint32_t)y * (uint32_t)I.nx + (uint32_t)x;
        if (!in_sink(I.cur, x, y, z, I.nx, I.ny, I.nz)) {
            const int cI[3] = {tx, tx + 1, tx + 2}, rI[3] = {ty, ty + 1, ty + 2};
            A S[2][3];
            force_sum<A>(psiS[sm], psiS[s0], psiS[sp], cI, rI, row, S);
            const int fc = (ty + 1) * row + tx + 1;
            const Psi2<A> pc = psiS[s0].get(fc);
            collide_node<A, kExact<St>, !St::kNode>(I, v, S, pc[0], pc[1], node_key(I, x, y, z));
        }
        store_node<St>(d, I, z, xy, v);
    };

    load_plane(z0 - 1, 0, nxt);
    load_plane(z0, 1, cur);
    for (int z = z0; z < z1; z += 2) {
        load_plane(z + 1, (z - z0 + 2) % 3, nxt);
        __syncthreads();
        collide_plane(z, cur);
        __syncthreads();
        if (z + 1 < z1) {
            load_plane(z + 2, (z - z0 + 3) % 3, cur);
            __syncthreads();
            collide_plane(z + 1, nxt);
            __syncthreads();
        }
    }

    if (book) {
        double e = block_sum_wave(eflux);
        if ((t & 63) == 0) red[t >> 6] = e;
        __syncthreads();
        if (t == 0) {
            double sum = 0.0;
            for (int w = 0; w < NT / 64; ++w) sum += red[w];
            eacc[k] += sum;
        }
    }
}

// ---------------------------------------------------------------------------
// Software-pipelined step (FP64, FP32S and FP16S storage).
//
// Same tiles, arithmetic and results as k_step; the schedule differs:
//  - the loads of plane z+2 (tile node and one halo node per thread) are
//    issued before the barrier and collision of plane z and decoded after
//    it, so their latency hides behind a plane of work;
//  - four psi slots in LDS let a plane's psi be written while the previous
//    plane's stencil is still being read: one barrier per plane;
//  - where the tile spans the whole periodic x (or y) extent, the halo
//    column (row) is the tile's own opposite column (row): the stencil
//    index wraps inside the tile and nothing is pulled for it.
// Every halo node must have its own thread (PipeTile::nring <= NT).
// ---------------------------------------------------------------------------

struct PipeTile {
    int nrow;    // halo nodes in each of the two halo rows (0: y wraps in the tile)
    int ncol;    // halo nodes in each of the two halo columns (0: x wraps in the tile)
    int nring;   // 2 nrow + 2 ncol
};

__host__ __device__ inline PipeTile pipe_tile(int tw, int th, int nx, int ny)
{
    const bool xper = tw == nx, yper = th == ny;
    PipeTile p;
    p.nrow = yper ? 0 : (xper ? tw : tw + 2);
    p.ncol = xper ? 0 : th;
    p.nring = 2 * p.nrow + 2 * p.ncol;
    return p;
}

// Halo node r < nring in tile coordinates (fx, fy): the two halo rows, then
// the two halo columns.
__host__ __device__ inline void pipe_ring_node(int r, const PipeTile& p, int tw, int th, bool xper, int& fx, int& fy)
{
    if (r < 2 * p.nrow) {
        const bool lo = r < p.nrow;
        fy = lo ? -1 : th;
        fx = (lo ? r : r - p.nrow) - (xper ? 0 : 1);
    } else {
        const int q = r - 2 * p.nrow;
        const bool lo = q < p.ncol;
        fx = lo ? -1 : tw;
        fy = lo ? q : q - p.ncol;
    }
}

// Footprint column (row) of the neighbours at offsets -1, 0, +1 of tile
// column (row) a of extent w; `per`: the tile spans the periodic extent.
__host__ __device__ inline void pipe_stencil(int a, int w, bool per, int out[3])
{
    out[0] = per && a == 0 ? w : a;
    out[1] = a + 1;
    out[2] = per && a == w - 1 ? 1 : a + 2;
}

// FP16N in the pipelined step: the rest pairs of the tile plus two halo
// rings ((tw + 4)(th + 4) nodes: every source of a tile or halo node's pull)
// are staged per plane into LDS, at most kRestLoads per thread.
constexpr int kRestLoads = 3;
__host__ __device__ inline bool rest_fits(int tw, int th, int nt) { return (tw + 4) * (th + 4) <= kRestLoads * nt; }

__host__ __device__ inline int mod_n(int a, int n) { return ((a % n) + n) % n; }

// Waves per SIMD the pipelined step is compiled for: two in FP32 arithmetic
// (<= 256 VGPRs); one in FP64, whose three population sets take ~490.
template <class St> constexpr int kPipeWaves = std::is_same_v<typename St::A, double> ? 1 : 2;

template <class St, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(kPipeWaves<St>))) void k_step_pipe(
    const Inst* __restrict__ insts, const Item* __restrict__ items, int n_items, const typename St::T* __restrict__ src,
    typename St::T* __restrict__ dst, double* __restrict__ eacc)
{
    using T = typename St::T;
    using A = typename St::A;
    // Storage in the arithmetic type (FP32S): decoding is the identity, so a
    // plane loads straight into the population set its collision uses, and
    // three sets rotate (collided / decoded / in flight). Otherwise the loads
    // land in a raw set that is decoded into one of two sets.
    constexpr bool kRotate = std::is_same_v<T, A> && !St::kNode;
    // FP16N: the sources' FP32 rest pairs come from a four-plane LDS ring.
    constexpr bool kLdsRest = St::kNode;
    constexpr int FP = Foot<NT>::kMax;
    __shared__ PsiPlane<A, FP, kPsiPair<St>> psiS[4];
    __shared__ double red[NT / 64];
    __shared__ F2 restS[kLdsRest ? 4 : 1][kLdsRest ? kRestLoads * NT : 1];

    const int k = xcd_item(blockIdx.x, n_items);
    if (k >= n_items) return;
    const Item it = items[k];
    if (it.nzc == 0) return;  // padding of an XCD's run of items
    const Inst I = insts[it.inst];
    const T* __restrict__ s = src + I.base;
    T* __restrict__ d = dst + I.base;

    const int t = threadIdx.x;
    const int tw = it.tw, th = it.th;
    const int row = tw + 2;
    const bool xper = tw == I.nx, yper = th == I.ny;
    const PipeTile pt = pipe_tile(tw, th, I.nx, I.ny);
    const bool own = t < tw * th;
    const bool ring = t < pt.nring;
    // Per-thread coordinates and sink intervals live in LDS and are read
    // where they are used: held in registers across the march they would
    // crowd out the population sets, and the compiler would hoist the
    // address arithmetic derived from them out of the march as well.
    __shared__ uint32_t tinfo[kLdsRest ? 8 + kRestLoads : 7][NT];
    {
        const int tx = own ? t % tw : 0, ty = own ? t / tw : 0;
        const int x = wrap(it.x0 + tx, I.nx), y = wrap(it.y0 + ty, I.ny);
        int fx = 0, fy = 0;
        if (ring) pipe_ring_node(t, pt, tw, th, xper, fx, fy);  // this thread's halo node
        const int hx = wrap(it.x0 + fx, I.nx), hy = wrap(it.y0 + fy, I.ny);
        auto pack = [](int a, int b) { return (uint32_t)a | ((uint32_t)b << 16); };
        tinfo[0][t] = pack(x, y);
        tinfo[1][t] = pack(hx, hy);
        tinfo[2][t] = pack((ty + 1) * row + tx + 1, (fy + 1) * row + fx + 1);
        tinfo[3][t] = pack(tx, ty);
        // sink membership along the march: one packed z interval per column
        tinfo[4][t] = sink_zrange(I.reset, x, y, I.nx, I.ny, I.nz);
        tinfo[5][t] = sink_zrange(I.cur, x, y, I.nx, I.ny, I.nz);
        tinfo[6][t] = sink_zrange(I.reset, hx, hy, I.nx, I.ny, I.nz);
        if constexpr (kLdsRest) {
            // rest footprint positions: this thread's tile and halo nodes,
            // and the in-plane index of the nodes it stages. Positions past
            // the footprint stage node 0 into ring entries nothing reads, so
            // the staging runs without divergent branches around its loads
            // (whose joins would make the compiler wait for every load).
            const int W = tw + 4, nfp = W * (th + 4);
            tinfo[7][t] = pack((ty + 2) * W + tx + 2, (fy + 2) * W + fx + 2);
#pragma unroll
            for (int j = 0; j < kRestLoads; ++j) {
                const int p = t + j * NT;
                uint32_t v = 0;
                if (p < nfp) {
                    const int gx = mod_n(it.x0 + p % W - 2, I.nx), gy = mod_n(it.y0 + p / W - 2, I.ny);
                    v = (uint32_t)gy * (uint32_t)I.nx + (uint32_t)gx;
                }
                tinfo[8 + j][t] = v;
            }
        }
    }
    auto lo = [](uint32_t v) { return (int)(v & 0xffffu); };
    auto hi = [](uint32_t v) { return (int)(v >> 16); };

    // The march runs over indices m in [z0, z1) = [0, nzc), plane zs + dz m:
    // upwards from the chunk's bottom, or downwards from its top. Adjacent
    // chunks march in opposite directions, so both reach their shared
    // boundary planes at the same time (both at the start or both at the
    // end) and the second read of each is served by the cache.
    const int dz = it.down ? -1 : 1;
    const int zs = it.down ? it.z0 + it.nzc - 1 : it.z0;
    const int z0 = 0, z1 = it.nzc;
    const bool book = I.count_reset != 0 && I.reset.kind != kSinkNone;
    // Evaporated mass of this wave: each plane's sink fluxes are summed over
    // the wave (fixed tree order) into one wave-uniform double, so no
    // per-lane accumulator occupies registers across the march.
    double ewave = 0.0;

    // Loads of logical plane zq (none past the chunk's halo plane z1): the
    // halo node into wr, the tile node into wo. Every step of the march
    // reduces the plane loaded by the step before, on every path (planes past
    // z1 reduce stale registers into a psi slot nothing reads), so no path
    // carries a load past the point that consumes it and the compiler's
    // memory waits stay exact. Every lane loads and reduces a tile node
    // (lanes past the tile take the tile's first node, whose lines the tile
    // lanes fetch anyway).
    auto issue_ring = [&](int zq, RawNode<St>& wr) {
        const uint32_t h = tinfo[1][t];
        if (zq <= z1 && ring) pull_raw<St>(s, I, lo(h), hi(h), psi_plane(zs + dz * zq, I.nz, I.wall_z), wr);
    };
    auto issue_own = [&](int zq, T (&wo)[2][kQ]) {
        if constexpr (!St::kNode) {
            const uint32_t o = tinfo[0][t];
            if (zq <= z1) pull_vals<St>(s, I, lo(o), hi(o), psi_plane(zs + dz * zq, I.nz, I.wall_z), wo);
        }
    };
    // Densities (with the pull-time sink reset) of logical plane zq: psi of
    // the halo node from wr and of the tile node from v (decoded, reset in
    // place) into the plane's LDS slot; the flux of reset tile nodes is
    // booked.
    auto dens_with = [&](int zq, auto&& ring_decode, NodeVals<A>& v) {
        const int zp = psi_plane(zs + dz * zq, I.nz, I.wall_z);
        // behind a solid wall the plane's psi is the wall's (its loads, of
        // the mirrored plane, are reduced as usual and left unused)
        const bool wallc = beyond_wall(I, zs + dz * zq);
        auto& ps = psiS[(zq - z0 + 1) & 3];
        const uint32_t fi = tinfo[2][t];
        double fl = 0.0;
        if (ring) {
            NodeVals<A> h;
            ring_decode(h);
            node_density<A>(I, h);
            if (in_zrange_sink(tinfo[6][t], zp)) {
                const uint32_t hh = tinfo[1][t];
                sink_reset<A, kExact<St>>(I, h, node_key(I, lo(hh), hi(hh), zp));
            }
            if (wallc) ps.put(hi(fi), Par<A>::psiw(I, 0), Par<A>::psiw(I, 1));
            else ps.put(hi(fi), psi_of<A>(h.rho[0], I.psi_exp), psi_of<A>(h.rho[1], I.psi_exp));
        }
        node_density<A>(I, v);
        if (own && in_zrange_sink(tinfo[4][t], zp)) {
            const uint32_t o = tinfo[0][t];
            fl = sink_reset<A, kExact<St>>(I, v, node_key(I, lo(o), hi(o), zp));
        }
        if (own) {
            if (wallc) ps.put(lo(fi), Par<A>::psiw(I, 0), Par<A>::psiw(I, 1));
            else ps.put(lo(fi), psi_of<A>(v.rho[0], I.psi_exp), psi_of<A>(v.rho[1], I.psi_exp));
        }
        if (book && zq >= z0 && zq < z1 && __builtin_amdgcn_ballot_w64(fl != 0.0))
            ewave = wave_uniform(ewave + block_sum_wave(fl));
    };
    auto dens = [&](int zq, const RawNode<St>& wr, NodeVals<A>& v) {
        dens_with(zq, [&](NodeVals<A>& h) { decode_raw<St>(wr, h); }, v);
    };
    auto collide = [&](int m, NodeVals<A>& v) {
        if (!own) return;
        const int z = zs + dz * m;
        const uint32_t o = tinfo[0][t];
        const uint32_t xy = (uint32_t)hi(o) * (uint32_t)I.nx + (uint32_t)lo(o);
        if (!in_zrange_sink(tinfo[5][t], z)) {
            const uint32_t txy = tinfo[3][t];
            const int fo = lo(tinfo[2][t]);
            int sc[3], sr[3];
            pipe_stencil(lo(txy), tw, xper, sc);
            pipe_stencil(hi(txy), th, yper, sr);
            // psi slots of march indices m-1, m, m+1; planes z-1 / z+1 swap
            // roles on a downward march
            const int sb = m & 3, sc0 = (m + 1) & 3, sa = (m + 2) & 3;
            A S[2][3];
            force_sum<A>(psiS[dz > 0 ? sb : sa], psiS[sc0], psiS[dz > 0 ? sa : sb], sc, sr, row, S);
            const Psi2<A> pc = psiS[sc0].get(fo);
            collide_node<A, kExact<St>, !St::kNode>(I, v, S, pc[0], pc[1],
                                                    xy + (uint32_t)z * (uint32_t)I.nx * (uint32_t)I.ny);
        }
        store_node<St>(d, I, z, xy, v);
    };

    if constexpr (kRotate) {
        NodeVals<A> p0, p1, p2;
        RawNode<St> rr;
        // Prologue: two planes in flight at a time.
        {
            RawNode<St> rr2;
            issue_ring(z0 - 1, rr);
            issue_own(z0 - 1, p2.f);
            issue_ring(z0, rr2);
            issue_own(z0, p0.f);
            dens(z0 - 1, rr, p2);
            issue_ring(z0 + 1, rr);
            issue_own(z0 + 1, p1.f);
            dens(z0, rr2, p0);
        }
        dens(z0 + 1, rr, p1);
        issue_ring(z0 + 2, rr);
        issue_own(z0 + 2, p2.f);
        // Plane z collides from a; plane z+2 (loaded into c) is reduced to
        // densities (past the halo plane: zeros into a psi slot nothing
        // reads); plane z+3 loads into a.
        auto step = [&](int z, NodeVals<A>& a, NodeVals<A>& c) {
            __syncthreads();
            collide(z, a);
            dens(z + 2, rr, c);
            // Keep the next loads after the work that frees their registers:
            // hoisted, they would hold a fourth population set.
            __builtin_amdgcn_sched_barrier(0);
            issue_ring(z + 3, rr);
            issue_own(z + 3, a.f);
        };
        for (int z = z0;; z += 3) {
            step(z, p0, p2);
            if (z + 1 >= z1) break;
            step(z + 1, p1, p0);
            if (z + 2 >= z1) break;
            step(z + 2, p2, p1);
            if (z + 3 >= z1) break;
        }
    } else if constexpr (kLdsRest) {
        // Rest pairs of stored logical plane q (physical plane zs + dz q,
        // wrapped, or clamped at a wall: planes past a wall are never
        // sources) into registers, then into ring slot (q + 2) & 3. Plane q
        // is loaded at the start of the half-step decoding plane q - 2 and
        // written at its end, before the barrier ahead of the decode of plane
        // q - 1, its first reader; the slot it takes last held plane q - 4,
        // whose last reader (the decode of plane q - 3) is behind the barrier
        // that opens the half-step.
        auto stage_issue = [&](int q, F2 (&sv)[kRestLoads]) {
            if (q > z1 + 1) return;
            const int zr = zs + dz * q;
            // the plane is the same on every lane: say so, or the integer
            // modulo (vector-only) makes the resource look divergent
            const int zp = __builtin_amdgcn_readfirstlane(I.wall_z ? min(max(zr, 0), I.nz - 1) : mod_n(zr, I.nz));
            const Rsrc r = slab_rsrc(s + (int64_t)zp * I.slab);
            const uint32_t off = pair_off<St>(0, (uint32_t)I.ps);
#pragma unroll
            for (int j = 0; j < kRestLoads; ++j) {
                const Pair<float> pr = bload2<float>(r, tinfo[8 + j][t] * pair_bytes<St>(0), off);
                sv[j] = F2{pr.a, pr.b};
            }
        };
        auto stage_write = [&](int q, const F2 (&sv)[kRestLoads]) {
            if (q > z1 + 1) return;
            F2* slot = restS[(q + 2) & 3];
#pragma unroll
            for (int j = 0; j < kRestLoads; ++j) slot[t + j * NT] = sv[j];
        };
        auto stage_now = [&](int q) {
            F2 sv[kRestLoads];
            stage_issue(q, sv);
            stage_write(q, sv);
        };
        // Decode of the moving values w of logical plane m at rest footprint
        // position b: each population's source rest value from the ring, the
        // same arithmetic as decode_raw. A halo plane mirrored at a wall pulls
        // exactly like the plane next to it.
        auto decode_lds = [&](int m, uint32_t b, const RawH<St>& w, NodeVals<A>& v) {
            const int zr = zs + dz * m;
            const int me = (I.wall_z && (zr < 0 || zr >= I.nz)) ? (m < z0 ? z0 : z1 - 1) : m;
            const int zp = zs + dz * me;
            const bool wlo = I.wall_z && zp == 0, whi = I.wall_z && zp == I.nz - 1;
            const int W = tw + 4;
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const int e = ez(i);
                const bool refl = (e > 0 && wlo) || (e < 0 && whi);
                const F2 d = (i == 0 || refl) ? restS[(me + 2) & 3][b]
                                              : restS[(me - dz * e + 2) & 3][(int)b - ey(i) * W - ex(i)];
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    v.f[c][i] = i == 0 ? d[c] : decode_h<St>(kRatio(i), d[c], w.h2[i][c]);
            }
        };
        RawH<St> ro, rr;
        NodeVals<A> va, vb;
        auto issue_into = [&](int zq, RawH<St>& wo, RawH<St>& wr) {
            if (zq > z1) return;
            const int zp = psi_plane(zs + dz * zq, I.nz, I.wall_z);
            const uint32_t h = tinfo[1][t], o = tinfo[0][t];
            // the tile node first: the slab pointers it derives (branches on
            // the wall) are then formed outside the halo lanes' divergent
            // region, where the compiler would take them as divergent and
            // wrap every load in a loop over their values
            pull_h<St>(s, I, lo(o), hi(o), zp, wo);
            if (ring) pull_h<St>(s, I, lo(h), hi(h), zp, wr);
        };
        auto dens_from = [&](int zq, NodeVals<A>& keep, const RawH<St>& wo, const RawH<St>& wr) {
            const uint32_t fb = tinfo[7][t];
            decode_lds(zq, lo(fb), wo, keep);
            dens_with(zq, [&](NodeVals<A>& h) { decode_lds(zq, hi(fb), wr, h); }, keep);
        };
        // Prologue: rest planes -2 .. 1, the densities of planes -1 and 0,
        // then rest planes 2 and 3 into the slots of -2 and -1.
        {
            RawH<St> ro2, rr2;
            stage_now(z0 - 2);
            stage_now(z0 - 1);
            stage_now(z0);
            stage_now(z0 + 1);
            __syncthreads();
            issue_into(z0 - 1, ro2, rr2);
            issue_into(z0, ro, rr);
            dens_from(z0 - 1, va, ro2, rr2);
            issue_into(z0 + 1, ro2, rr2);
            dens_from(z0, va, ro, rr);
            __syncthreads();
            stage_now(z0 + 2);
            stage_now(z0 + 3);
            __syncthreads();
            issue_into(z0 + 2, ro, rr);
            dens_from(z0 + 1, vb, ro2, rr2);
        }
        F2 sv[kRestLoads];
        for (int z = z0;; z += 2) {
            __syncthreads();
            stage_issue(z + 4, sv);
            collide(z, va);
            dens_from(z + 2, va, ro, rr);
            stage_write(z + 4, sv);
            __builtin_amdgcn_sched_barrier(0);
            issue_into(z + 3, ro, rr);
            if (z + 1 >= z1) break;
            __syncthreads();
            stage_issue(z + 5, sv);
            collide(z + 1, vb);
            dens_from(z + 3, vb, ro, rr);
            stage_write(z + 5, sv);
            __builtin_amdgcn_sched_barrier(0);
            issue_into(z + 4, ro, rr);
            if (z + 2 >= z1) break;
        }
    } else {
        RawNode<St> ro, rr;
        NodeVals<A> va, vb;
        auto issue_into = [&](int zq, RawNode<St>& wo, RawNode<St>& wr) {
            issue_ring(zq, wr);
            const uint32_t o = tinfo[0][t];
            if (zq <= z1) pull_raw<St>(s, I, lo(o), hi(o), psi_plane(zs + dz * zq, I.nz, I.wall_z), wo);
        };
        auto dens_from = [&](int zq, NodeVals<A>& keep, const RawNode<St>& wo, const RawNode<St>& wr) {
            decode_raw<St>(wo, keep);
            dens(zq, wr, keep);
        };
        // Prologue: two planes in flight at a time (the second pair of raw
        // sets is dead before the loop's working set is live).
        {
            RawNode<St> ro2, rr2;
            issue_into(z0 - 1, ro2, rr2);
            issue_into(z0, ro, rr);
            dens_from(z0 - 1, va, ro2, rr2);
            issue_into(z0 + 1, ro2, rr2);
            dens_from(z0, va, ro, rr);
            issue_into(z0 + 2, ro, rr);
            dens_from(z0 + 1, vb, ro2, rr2);
        }
        for (int z = z0;; z += 2) {
            __syncthreads();
            collide(z, va);
            dens_from(z + 2, va, ro, rr);
            __builtin_amdgcn_sched_barrier(0);
            issue_into(z + 3, ro, rr);
            if (z + 1 >= z1) break;
            __syncthreads();
            collide(z + 1, vb);
            dens_from(z + 3, vb, ro, rr);
            __builtin_amdgcn_sched_barrier(0);
            issue_into(z + 4, ro, rr);
            if (z + 2 >= z1) break;
        }
    }

    if (book) {
        const double e = ewave;
        if ((t & 63) == 0) red[t >> 6] = e;
        __syncthreads();
        if (t == 0) {
            double sum = 0.0;
            for (int w = 0; w < NT / 64; ++w) sum += red[w];
            eacc[k] += sum;
        }
    }
}

// ---------------------------------------------------------------------------
// Initialisation: write the stored buffer so that pulling it yields S(0).
// The slot P_i(y) is read by y + e_i as population i, or, when y + e_i lies
// across a z-seam wall, by y itself as population opp(i).
// ---------------------------------------------------------------------------

// Writes the stored value `val` (a full FP64 population) of plane (c, i) at
// in-plane index xy of slab z; f0 is the slot node's own rest population,
// which FP16N encodes the moving populations against.
template <class S>
__device__ __forceinline__ void put_slot(typename S::T* __restrict__ d, const Inst& I, int c, int i, int z,
                                         int64_t xy, double val, double f0)
{
    using T = typename S::T;
    using A = typename S::A;
    char* slab = reinterpret_cast<char*>(d + (int64_t)z * I.slab);
    const uint32_t off = plane_off<S>(c, i, (uint32_t)I.ps) + (uint32_t)xy * node_stride<S>(i);
    if constexpr (S::kNode) {
        const float d0 = (float)(f0 - wgt(0) * I.shift[c]);
        if (i == 0) *reinterpret_cast<float*>(slab + off) = d0;
        else {
            const float a = (float)(val - wgt(i) * I.shift[c]) - kRatio(i) * d0;
            *reinterpret_cast<T*>(slab + off) = narrow<T>(a * S::kHS);
        }
    } else {
        *reinterpret_cast<T*>(slab + off) = (T)(A)(val - wgt(i) * I.shift[c]);
    }
}

template <class S>
__global__ void k_init_density(Inst I, const double* __restrict__ rhoA, const double* __restrict__ rhoB,
                               typename S::T* __restrict__ dst)
{
    const int64_t n = I.n;
    const double* rho[2] = {rhoA, rhoB};
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(k % I.nx);
        const int y = (int)((k / I.nx) % I.ny);
        const int z = (int)(k / ((int64_t)I.nx * I.ny));
        const int64_t xy = k - (int64_t)z * I.nx * I.ny;
        typename S::T* d = dst + I.base;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int zt = z + ez(i);
            int64_t src;
            if (I.wall_z && (zt < 0 || zt >= I.nz))
                src = k;
            else
                src = node_of(wrap(x + ex(i), I.nx), wrap(y + ey(i), I.ny), wrap(zt, I.nz), I.nx, I.ny);
            for (int c = 0; c < 2; ++c) put_slot<S>(d, I, c, i, z, xy, wgt(i) * rho[c][src], wgt(0) * rho[c][k]);
        }
    }
}

// From full FP64 populations f[(c*19 + i)*fstride + node].
template <class S>
__global__ void k_init_pops(Inst I, const double* __restrict__ f, int64_t fstride, typename S::T* __restrict__ dst)
{
    const int64_t n = I.n;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(k % I.nx);
        const int y = (int)((k / I.nx) % I.ny);
        const int z = (int)(k / ((int64_t)I.nx * I.ny));
        const int64_t xy = k - (int64_t)z * I.nx * I.ny;
        typename S::T* d = dst + I.base;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int zt = z + ez(i);
            int64_t src;
            int q;
            if (I.wall_z && (zt < 0 || zt >= I.nz)) {
                src = k;
                q = opp(i);
            } else {
                src = node_of(wrap(x + ex(i), I.nx), wrap(y + ey(i), I.ny), wrap(zt, I.nz), I.nx, I.ny);
                q = i;
            }
            for (int c = 0; c < 2; ++c)
                put_slot<S>(d, I, c, i, z, xy, f[(int64_t)(c * kQ + q) * fstride + src],
                            f[(int64_t)(c * kQ) * fstride + k]);
        }
    }
}

// ---------------------------------------------------------------------------
// Read-outs of S(t) in FP64.
// ---------------------------------------------------------------------------

template <class S>
__device__ __forceinline__ void state_at(const typename S::T* s, const Inst& I, int x, int y, int z,
                                         NodeVals<typename S::A>& v)
{
    using A = typename S::A;
    pull_node<S>(s, I, x, y, z, v);
    node_density<A>(I, v);
    if (in_sink(I.reset, x, y, z, I.nx, I.ny, I.nz)) sink_reset<A, kExact<S>>(I, v, node_key(I, x, y, z));
}

template <class S>
__global__ void k_read_density(Inst I, const typename S::T* __restrict__ src, double* __restrict__ outA,
                               double* __restrict__ outB)
{
    using A = typename S::A;
    const typename S::T* s = src + I.base;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < I.n; k += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(k % I.nx), y = (int)((k / I.nx) % I.ny), z = (int)(k / ((int64_t)I.nx * I.ny));
        NodeVals<A> v;
        state_at<S>(s, I, x, y, z, v);
        if (outA) outA[k] = I.shift[0] + (double)v.drho[0];
        if (outB) outB[k] = I.shift[1] + (double)v.drho[1];
    }
}

// out[(c*19 + i)*ostride + node].
template <class S>
__global__ void k_read_pops(Inst I, const typename S::T* __restrict__ src, double* __restrict__ out, int64_t ostride)
{
    using A = typename S::A;
    const typename S::T* s = src + I.base;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < I.n; k += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(k % I.nx), y = (int)((k / I.nx) % I.ny), z = (int)(k / ((int64_t)I.nx * I.ny));
        NodeVals<A> v;
        state_at<S>(s, I, x, y, z, v);
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int i = 0; i < kQ; ++i)
                out[(int64_t)(c * kQ + i) * ostride + k] = (double)v.f[c][i] + wgt(i) * I.shift[c];
    }
}

// Barycentric velocity U of Eq. (velw) from S(t) and its densities (already
// written by k_read_density): U = (sum_c j^c + (F^A + F^B)/2) / sum_c rho^c,
// into U[d*ustride + node].
template <class S>
__global__ void k_read_velocity(Inst I, const typename S::T* __restrict__ src, const double* __restrict__ rhoA,
                                const double* __restrict__ rhoB, double* __restrict__ U, int64_t ustride)
{
    using A = typename S::A;
    const typename S::T* s = src + I.base;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < I.n; k += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(k % I.nx), y = (int)((k / I.nx) % I.ny), z = (int)(k / ((int64_t)I.nx * I.ny));
        NodeVals<A> v;
        state_at<S>(s, I, x, y, z, v);
        double num[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                num[0] += (double)v.f[c][i] * ex(i);
                num[1] += (double)v.f[c][i] * ey(i);
                num[2] += (double)v.f[c][i] * ez(i);
            }
        if (!in_sink(I.cur, x, y, z, I.nx, I.ny, I.nz)) {
            const double* rho[2] = {rhoA, rhoB};
            for (int c = 0; c < 2; ++c) {
                double Sv[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int i = 1; i < kQ; ++i) {
                    const int zn = psi_plane(z + ez(i), I.nz, I.wall_z);
                    const int64_t nb = node_of(wrap(x + ex(i), I.nx), wrap(y + ey(i), I.ny), zn, I.nx, I.ny);
                    const double r = rho[1 - c][nb];
                    const double p = beyond_wall(I, z + ez(i)) ? I.psi_w[1 - c] : (I.psi_exp ? 1.0 - exp(-r) : r);
                    Sv[0] += wgt(i) * p * ex(i);
                    Sv[1] += wgt(i) * p * ey(i);
                    Sv[2] += wgt(i) * p * ez(i);
                }
                const double r = rho[c][k];
                const double pc = I.psi_exp ? 1.0 - exp(-r) : r;
                for (int dd = 0; dd < 3; ++dd) num[dd] += 0.5 * (-pc * I.g * Sv[dd]);
            }
        }
        const double rt = rhoA[k] + rhoB[k];
        for (int dd = 0; dd < 3; ++dd) U[(int64_t)dd * ustride + k] = num[dd] / rt;
    }
}

// ---------------------------------------------------------------------------
// FP64 diagnostics: one block per z-plane writes plane partials, then one
// block sums them in a fixed order (deterministic).
// Partial layout per plane: massA, massB, px, py, pz, phi, flux, nonfinite,
// nonpositive.
// ---------------------------------------------------------------------------

constexpr int kDiagVals = 9;

template <typename A>
__device__ __forceinline__ void block_sum_n(A* vals, int nv, A* lds)
{
    // lds: [nv][NT/64]
    const int t = threadIdx.x, nw = blockDim.x >> 6;
    for (int q = 0; q < nv; ++q) {
        A v = block_sum_wave(vals[q]);
        if ((t & 63) == 0) lds[q * nw + (t >> 6)] = v;
    }
    __syncthreads();
    if (t < nv) {
        A s = 0;
        for (int w = 0; w < nw; ++w) s += lds[t * nw + w];
        lds[t * nw] = s;
    }
    __syncthreads();
    for (int q = 0; q < nv; ++q) vals[q] = lds[q * nw];
    __syncthreads();
}

template <class S>
__global__ __launch_bounds__(256) void k_diag_planes(Inst I, const typename S::T* __restrict__ src,
                                                     double* __restrict__ part)
{
    using A = typename S::A;
    __shared__ double lds[kDiagVals * 4];
    const typename S::T* s = src + I.base;
    const int z = blockIdx.x;
    const int area = I.nx * I.ny;
    double acc[kDiagVals] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = threadIdx.x; k < area; k += blockDim.x) {
        const int x = k % I.nx, y = k / I.nx;
        NodeVals<A> v;
        pull_node<S>(s, I, x, y, z, v);
        node_density<A>(I, v);
        if (in_sink(I.reset, x, y, z, I.nx, I.ny, I.nz)) acc[6] += sink_reset<A, kExact<S>>(I, v, node_key(I, x, y, z));
        // masses from the exact FP64 sums of the stored deviations (the FP32
        // sums carry a rounding that repeats at every node of a uniform region)
        const double ra = I.shift[0] + sum64(v.f[0]), rb = I.shift[1] + sum64(v.f[1]);
        acc[0] += ra;
        acc[1] += rb;
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const double fi = (double)v.f[c][i];
                acc[2] += fi * ex(i);
                acc[3] += fi * ey(i);
                acc[4] += fi * ez(i);
            }
        double phi = (ra - rb - I.phi_out) / (I.phi_in - I.phi_out);
        phi = phi < 0.0 ? 0.0 : (phi > 1.0 ? 1.0 : phi);
        acc[5] += phi;
        if (!isfinite(ra) || !isfinite(rb)) acc[7] += 1.0;
        if (ra <= 0.0 || rb <= 0.0) acc[8] += 1.0;
    }
    block_sum_n<double>(acc, kDiagVals, lds);
    if (threadIdx.x < kDiagVals) part[(int64_t)z * kDiagVals + threadIdx.x] = acc[threadIdx.x];
}

// out: [0] massA [1] massB [2..4] momentum [5] phi sum [6] pending flux
//      [7] nonfinite [8] nonpositive [9] booked E [10] z_interface
template <int NT>
__global__ __launch_bounds__(NT) void k_diag_final(Inst I, const double* __restrict__ part,
                                                   const double* __restrict__ eacc, const double* __restrict__ ebase,
                                                   int inst, double* __restrict__ out)
{
    __shared__ double lds[(kDiagVals + 1) * (NT / 64)];
    double acc[kDiagVals + 1];
    for (int q = 0; q <= kDiagVals; ++q) acc[q] = 0.0;
    for (int z = threadIdx.x; z < I.nz; z += NT)
        for (int q = 0; q < kDiagVals; ++q) acc[q] += part[(int64_t)z * kDiagVals + q];
    for (int k = I.item_begin + threadIdx.x; k < I.item_end; k += NT) acc[kDiagVals] += eacc[k];
    block_sum_n<double>(acc, kDiagVals + 1, lds);
    if (threadIdx.x == 0) {
        for (int q = 0; q < kDiagVals; ++q) out[q] = acc[q];
        out[9] = acc[kDiagVals] + ebase[inst];
        double zi = __builtin_nan("");
        const double area = (double)I.nx * I.ny;
        for (int z = 0; z + 1 < I.nz; ++z) {
            const double a = (part[(int64_t)z * kDiagVals] - part[(int64_t)z * kDiagVals + 1]) / area;
            const double b = (part[(int64_t)(z + 1) * kDiagVals] - part[(int64_t)(z + 1) * kDiagVals + 1]) / area;
            if ((a > 0.0 && b <= 0.0) || (a < 0.0 && b >= 0.0)) {
                zi = z + a / (a - b);
                break;
            }
        }
        out[10] = zi;
    }
}

// Folds the per-item evaporation accumulators of each instance into its base
// value (used before the work-item list changes), then clears them.
__global__ void k_fold_eacc(const Inst* __restrict__ insts, int n_inst, double* __restrict__ eacc,
                            double* __restrict__ ebase)
{
    const int inst = blockIdx.x * blockDim.x + threadIdx.x;
    if (inst >= n_inst) return;
    const Inst I = insts[inst];
    double s = 0.0;
    for (int k = I.item_begin; k < I.item_end; ++k) {
        s += eacc[k];
        eacc[k] = 0.0;
    }
    ebase[inst] += s;
}

// Plain streaming copy (16 bytes per lane, grid-stride): the HBM ceiling the
// step kernel is compared with, and the calibration of the byte counters.
__global__ __launch_bounds__(256) void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n16)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n16) dst[k] = src[k];
}

__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

}  // namespace lbsc
