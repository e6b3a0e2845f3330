// Fused iPiano step on the matrix cores (gfx950, FP32 MFMA 16x16x4).
//
// One launch performs one iteration of eq. 2.8 for every tile of every job:
//
//   z_i  = K_i u^n                          forward filter bank  (MFMA)
//   phi_i = z_i / (1 + z_i^2)               influence / (2 alpha_i)  (VALU)
//   g    = sum_i K_i^T (2 alpha_i phi_i)    adjoint filter bank  (MFMA)
//   u^{n+1} = prox(u^n - tau g + gamma (u^n - u^{n-1}))          (VALU)
//
// Tiling.  A workgroup owns an output tile of at most TY x TX pixels.  The
// adjoint at an output pixel needs psi on the tile grown by r, which needs
// u on the tile grown by 2r; both grown regions are computed in the
// workgroup (halo recompute) so that nothing but u^n, u^{n-1} and y crosses
// HBM.  The psi region is processed as "q-rows" of QW = 16 * QB pixels,
// one q-row per wave per step, each q-row as QB blocks of 16 pixels:
//
//   forward  Z^T[16 filters x 16 px] += A[16 filters x 4 taps] B[4 taps x 16 px]
//            A: filter taps (registers), B: u gathered from the LDS tile
//   adjoint  C[16 px x 16 taps] += Phi[16 px x 4 filters] Kt[4 filters x 16 taps]
//            Phi is the forward accumulator itself: the MFMA output layout
//            (lane = px + 16 * (filter/4), item = filter%4) is exactly the A
//            operand layout of the next product with the filter index as
//            the reduction index, so no data moves between the two.
//
// m^2 = 4 k + 1 for odd m, so 4 k taps go through the matrix cores and the
// last tap through VALU FMAs.  C[p][t] is the contribution of psi at pixel p
// to the extended position p + (a - r, b - r), t = (a, b).  It is collapsed
// in two deterministic passes through LDS: horizontally per q-row into
// H[q-row][a][x] = sum_b C[x - b + r][(a, b)], then vertically per output
// row, g(y) = sum_a H[y - a + r][a], adding the ghost rows and columns that
// mirror each border pixel (the transpose of the symmetric extension).
// No atomics: every sum is taken in a fixed order, so results are bitwise
// reproducible and independent of what else is in the batch.
//
// Reduced precision (FE_PREC_BF16 / FE_PREC_FP16): both contractions use
// v_mfma_f32_16x16x32_{bf16,f16} (operands rounded to nearest even, FP32
// accumulation).  K = 32 per instruction, so all m^2 taps of the forward bank
// fit in ceil(m^2 / 32) k-steps (no VALU tap).  The adjoint runs in gather
// form: psi, rounded, goes through a per-wave LDS scratch and one product
// per block yields H directly (see MathP16), replacing the C scratch and the
// horizontal collapse.  The influence, the H and output-row sums, the
// inertial step and the prox stay FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <atomic>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "fe_internal.h"
#include "fe_math.h"
#include "fe_plan.h"

namespace fe {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
// Global-memory float.  Pointers read out of the job table are generic;
// accesses through them would compile to FLAT instructions, which also
// count against the LDS wait counter and would make every LDS wait wait for
// HBM as well.
typedef __attribute__((address_space(1))) float gfloat;
// LDS quad: 16-byte reads through it compile to ds_read_b128.
typedef __attribute__((address_space(3))) f32x4 lquad;
typedef __attribute__((address_space(3))) float lfloat;
typedef __attribute__((address_space(3))) u32x4 lu32x4;
typedef __attribute__((address_space(3))) u32x2 lpair;

// Waves per workgroup: FP32 is built for 8 (every operand in registers,
// two waves per SIMD, u tile rows streamed during the steps) and 12
// (adjoint tables in LDS, three per SIMD, whole u tile in the prologue);
// 12 is the default for launches that fill the GPU (measured 0.9 % faster
// on 4 x 512^2 since its second barrier per step became a ring-slot wait;
// plan_waves), the tuner may pick either.
// BF16/FP16 are built for 12 (three per SIMD).
constexpr int kWavesF32 = 8, kWavesP16 = 12;
constexpr int kDefaultWavesF32 = 12;
constexpr int kMinSteps12 = 6;        // see plan_waves
constexpr int kQB = 4;                // 16-pixel blocks per q-row
constexpr int kQW = 16 * kQB;         // q-row width (pixels)
constexpr int kRingSpins = 1 << 20;   // bound of a ring_wait (polls of ~100 cycles)

// Per-job description the step kernel reads.
struct JobDesc {
    const float *counts;
    float *ua, *ub;     // state planes; u^n is ua on even iterations
    int H, W;
    int ntx, nty;       // tile grid of this job
    int tile_base;      // index of the job's first tile in the launch
    int iters;          // iterations this launch sequence applies
    int it0;            // iterations already applied (parity of the state)
    float tau, gamma, tl;
    float q1;           // 1 / (1 + tl)
    float lambda;       // data-term weight (the gradient modes)
    int data_term;
};

// What a launch of the fused kernel computes per output pixel:
//   kStep:       one iPiano iteration (eq. 2.8), u^{n+1} over u^{n-1};
//   kGrad:       grad E(u) = sum_i alpha_i K_i^T rho'(K_i u) + grad D(u, v)
//                (eq. 3.2 with the data term of eq. 3.4 / 3.6) into ub;
//   kGradEnergy: the same, plus the workgroup's partial sums of the prior
//                energy sum_i alpha_i rho(K_i u) over the pixels its tile
//                owns and of the data energy D(u, v) / lambda (eq. 2.5, 2.6);
//                the gradient store is skipped when ub is NULL.
constexpr int kStep = 0, kGrad = 1, kGradEnergy = 2;

template <int M>
struct Geo {
    static constexpr int R = (M - 1) / 2;
    static constexpr int T = M * M;
    static constexpr int KF = (T - 1) / 4;            // MFMA k-steps (4 taps each)
    static constexpr int NTB = (T - 1 + 15) / 16;     // adjoint tap blocks of 16
    static constexpr int TX = kQW - 2 * R;            // output columns per tile
    static constexpr int UC = kQW + 2 * R;            // u tile columns
    static constexpr int US = UC + 2;                 // u tile row stride (floats)
    static constexpr int UROWS_EXTRA = 1;             // row read (at weight 0) by padded taps
    static constexpr int SROWS = (16 * NTB > T) ? 16 * NTB : T;  // scratch rows = taps
    static constexpr int SPAD = 8;                    // zero columns left of a block
    static constexpr int SW = 36;                     // scratch row stride (floats)
    static constexpr int XSPAN = 16 + 2 * R;          // columns one block reaches
    static constexpr int TASKS = M * XSPAN;           // (a, x) collapse tasks per block
    static constexpr int ROUNDS = (TASKS + 63) / 64;
    static constexpr int LAST_ROW = T - 1;            // scratch row of the last tap
};

// H ring slots: with one barrier per pipeline step the rows being finished
// (2R + NW q-rows) and the NW rows being written coexist; in the TWO form
// (a barrier between a step's q-rows and its output rows, and a wait before
// a q-row's first ring write for the output rows that still read the slot)
// they do not.
template <int M, int NW, bool TWO>
struct Ring {
    static constexpr int HR = TWO ? NW + (M - 1) : 2 * NW + (M - 1);
};

// LDS of one workgroup: the u tile, the per-wave tap scratch, the H ring
// and the policy's operand tables (if it keeps any in LDS).
constexpr int kLdsFloats = 160 * 1024 / 4;

// The energy mode adds the weights alpha_i (64 floats) after the tables.
constexpr int kAlphaFloats = 64;

template <int M, typename Math, int MODE = kStep>
constexpr size_t lds_fixed_floats()
{
    using G = Geo<M>;
    return (size_t)Math::kNW * Math::kScratchFloats +
           (size_t)Ring<M, Math::kNW, Math::kTwo>::HR * M * Math::kHS + Math::kTabFloats +
           (MODE == kGradEnergy ? kAlphaFloats : 0) + (Math::kTwo ? Math::kNW : 0);
}

template <int M, typename Math, int MODE = kStep>
size_t lds_bytes(int ty_max)
{
    using G = Geo<M>;
    return sizeof(float) * ((size_t)(ty_max + 4 * G::R + G::UROWS_EXTRA) * Math::kUS +
                            lds_fixed_floats<M, Math, MODE>());
}

// Tallest tile whose workgroup fits the LDS.
template <int M, typename Math, int MODE = kStep>
constexpr int rows_limit()
{
    using G = Geo<M>;
    const long rows = ((long)kLdsFloats - (long)lds_fixed_floats<M, Math, MODE>()) / Math::kUS -
                      (4 * G::R + G::UROWS_EXTRA);
    return rows < kMaxTileRows ? (int)rows : kMaxTileRows;
}

// Tile of workgroup i of n under the XCD-contiguous order: XCD x = i % 8
// receives workgroups x, x + 8, ... and with them the tiles
// [x q + min(x, r), ...) in order, q = n / 8, r = n % 8 (a bijection of 0..n-1).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int i, int n)
{
    const int x = i % kXcds, k = i / kXcds, q = n / kXcds, r = n % kXcds;
    return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ int sym_clamp(int i, int n)
{
    if (i < 0) i = -1 - i;
    if (i >= n) i = 2 * n - 1 - i;
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Keeps this wave's LDS accesses in program order at compile time.  The LDS
// executes one wave's requests in issue order, so a lane reading what
// another lane of the same wave wrote earlier needs no wait, only that the
// compiler (which reasons per lane) does not move the accesses.
__device__ __forceinline__ void lds_order() { asm volatile("" ::: "memory"); }

// Workgroup barrier that orders LDS only.  __syncthreads() would also wait
// for this wave's outstanding global stores (the finished output rows),
// which nothing in the workgroup reads back during the launch.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Block arithmetic, FP32: forward and adjoint on v_mfma_f32_16x16x4_f32.
// Operand tables (one float per lane per register slot):
//   t0 forward A   [KF][NFB][64]      A[filter 16fb + l%16][tap 4s + l/16]
//   t1 adjoint B   [NFB][4][NTB][64]  B[k: filter 16fb + 4(l/16) + j][tap 16nb + l%16] * 2 alpha
//   t2 last tap    [NFB][4][64]       tap m^2-1 of filter 16fb + 4(l/16) + j
//   t3 last tap    [NFB][4][64]       the same times 2 alpha
// LDS = false: 8 waves per workgroup, every operand in registers (two waves
// per SIMD), one barrier per pipeline step.  LDS = true: 12 waves (three per
// SIMD); the adjoint operands and both last-tap tables live in LDS, one row
// of 16-byte aligned floats per lane (row strides of 4 mod 8 floats keep the
// 16-byte reads of eight consecutive lanes on distinct banks); the TWO form of
// the pipeline (see Ring).
constexpr int odd_quads(int n) { return ((n + 3) / 4) % 2 ? (n + 3) / 4 * 4 : (n + 3) / 4 * 4 + 4; }

template <int M, int NFB, bool LDS>
struct MathF32 {
    using G = Geo<M>;
    static constexpr int kNW = LDS ? 12 : kWavesF32;
    static constexpr bool kTwo = LDS;
    static constexpr int NA = NFB * 4 * G::NTB;          // adjoint operands per lane
    static constexpr int SA = odd_quads(NA), SL = odd_quads(NFB * 4);
    static constexpr int kTabFloats = LDS ? 64 * (SA + 2 * SL) : 0;
    static constexpr bool kPairTile = false;
    static constexpr bool kGather = false;               // scatter form + collapse
    static constexpr int kHS = kQW;                      // H row stride (floats)
    static constexpr int kUS = G::US;                    // u tile row stride (floats)
    // u tile rows streamed during the steps (registers allow it with 8 waves)
    static constexpr bool kStreamU = !LDS;
    static constexpr int kScratchFloats = G::SROWS * G::SW;  // C[px][tap] of one block
    static constexpr int RB = LDS ? 1 : NFB;             // register-resident copies
    float afwd[G::KF][NFB];
    float badj[RB][LDS ? 1 : 4][LDS ? 1 : G::NTB];
    float lastf[RB][LDS ? 1 : 4], lasta[RB][LDS ? 1 : 4];
    const float *tabA, *tabF, *tabL;                     // this lane's LDS rows
    int boff[G::KF], loff, perm16, perm32;
    struct Acc {
        f32x4 z[NFB];
        float ul;
    };

    // LDS copies of the adjoint and last-tap tables (all threads; the
    // caller's barrier publishes them), in two parts: the loads early in
    // the prologue, all in flight at once, the LDS stores later.
    static constexpr int kStA = LDS ? (64 * NA + 64 * kNW - 1) / (64 * kNW) : 1;
    static constexpr int kStL = LDS ? (64 * NFB * 4 + 64 * kNW - 1) / (64 * kNW) : 1;
    struct Staged {
        float a[kStA], f[kStL], l[kStL];
    };
    static __device__ void stage_load(Staged &r, const void *t1, const void *t2, const void *t3,
                                      int tid)
    {
        if constexpr (LDS) {
            const gfloat *adj = (const gfloat *)t1, *lf = (const gfloat *)t2,
                         *la = (const gfloat *)t3;
#pragma unroll
            for (int j = 0; j < kStA; ++j) {
                const int i = tid + j * 64 * kNW;
                r.a[j] = i < 64 * NA ? adj[i] : 0.0f;
            }
#pragma unroll
            for (int j = 0; j < kStL; ++j) {
                const int i = tid + j * 64 * kNW;
                r.f[j] = i < 64 * NFB * 4 ? lf[i] : 0.0f;
                r.l[j] = i < 64 * NFB * 4 ? la[i] : 0.0f;
            }
        }
    }
    static __device__ void stage_store(float *tab, const Staged &r, int tid)
    {
        if constexpr (LDS) {
#pragma unroll
            for (int j = 0; j < kStA; ++j) {
                const int i = tid + j * 64 * kNW;
                if (i < 64 * NA) tab[(i & 63) * SA + (i >> 6)] = r.a[j];
            }
            float *tf = tab + 64 * SA, *tl = tf + 64 * SL;
#pragma unroll
            for (int j = 0; j < kStL; ++j) {
                const int i = tid + j * 64 * kNW;
                if (i < 64 * NFB * 4) {
                    tf[(i & 63) * SL + (i >> 6)] = r.f[j];
                    tl[(i & 63) * SL + (i >> 6)] = r.l[j];
                }
            }
        }
    }

    // 32-bit words of the operand tables t0 .. t3 (the layouts above)
    static constexpr int tab_words(int i)
    {
        return i == 0 ? G::KF * NFB * 64 : i == 1 ? NFB * 4 * G::NTB * 64 : NFB * 4 * 64;
    }
    // FL: the tables are read from an LDS copy (same layout) instead of HBM
    template <bool FL = false>
    __device__ void load(const void *t0, const void *t1, const void *t2, const void *t3,
                         int lane, const float *tab)
    {
        using TP = std::conditional_t<FL, const lfloat *, const float *>;
        const TP fwd_tab = (TP)t0, adj_tab = (TP)t1;
        const TP lastf_tab = (TP)t2, lasta_tab = (TP)t3;
        const int p = lane & 15, g = lane >> 4;
#pragma unroll
        for (int s = 0; s < G::KF; ++s)
#pragma unroll
            for (int fb = 0; fb < NFB; ++fb) afwd[s][fb] = fwd_tab[(s * NFB + fb) * 64 + lane];
        if constexpr (LDS) {
            tabA = tab + lane * SA;
            tabF = tab + 64 * SA + lane * SL;
            tabL = tab + 64 * (SA + SL) + lane * SL;
        } else {
#pragma unroll
            for (int fb = 0; fb < NFB; ++fb)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int nb = 0; nb < G::NTB; ++nb)
                        badj[fb][j][nb] = adj_tab[((fb * 4 + j) * G::NTB + nb) * 64 + lane];
#pragma unroll
            for (int fb = 0; fb < NFB; ++fb)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    lastf[fb][j] = lastf_tab[(fb * 4 + j) * 64 + lane];
                    lasta[fb][j] = lasta_tab[(fb * 4 + j) * 64 + lane];
                }
        }
        // LDS offsets of the forward B operand: tap 4s + g at pixel p
#pragma unroll
        for (int s = 0; s < G::KF; ++s) {
            const int t = 4 * s + g;
            boff[s] = (t / M) * kUS + (t % M) + p;
        }
        loff = (M - 1) * kUS + (M - 1) + p;
        perm16 = (lane ^ 16) << 2;
        perm32 = (lane ^ 32) << 2;
    }

    // Z^T[filter][px] for the block whose top-left u sample is Ub[0].
    __device__ __forceinline__ void forward(const float *Ub, Acc &a) const
    {
#pragma unroll
        for (int fb = 0; fb < NFB; ++fb) a.z[fb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < G::KF; ++s) {
            const float b = Ub[boff[s]];
#pragma unroll
            for (int fb = 0; fb < NFB; ++fb)
                a.z[fb] = __builtin_amdgcn_mfma_f32_16x16x4f32(afwd[s][fb], b, a.z[fb], 0, 0, 0);
        }
        a.ul = Ub[loff];
    }

    // LDS operands of filter block fb: the adjoint B values for (j, nb) as
    // NTB 16-byte quads (element j * NTB + nb) and one quad of each last-tap
    // table (element j).
    struct Ops {
        f32x4 a[LDS ? G::NTB : 1], f, l;
    };
    __device__ __forceinline__ void fetch(int fb, Ops &o) const
    {
        if constexpr (LDS) {
            // one 16-byte LDS read per quad (volatile keeps each read whole)
            const volatile lquad *A = (const volatile lquad *)tabA + fb * G::NTB;
#pragma unroll
            for (int q = 0; q < G::NTB; ++q) o.a[q] = A[q];
            o.f = ((const volatile lquad *)tabF)[fb];
            o.l = ((const volatile lquad *)tabL)[fb];
        }
    }
    __device__ __forceinline__ float adj_op(const Ops &o, int fb, int j, int nb) const
    {
        if constexpr (LDS) {
            const int i = j * G::NTB + nb;
            return o.a[i >> 2][i & 3];
        } else {
            return badj[fb][j][nb];
        }
    }
    __device__ __forceinline__ float last_f(const Ops &o, int fb, int j) const
    {
        if constexpr (LDS) return o.f[j];
        else return lastf[fb][j];
    }
    __device__ __forceinline__ float last_a(const Ops &o, int fb, int j) const
    {
        if constexpr (LDS) return o.l[j];
        else return lasta[fb][j];
    }

    // Influence, adjoint, tap contributions C[px][tap] into the scratch.
    // EN: also adds alpha_f rho(z_f) of the lane's filters (alpha from the
    // LDS table `al`) to `en` when the pixel is one the tile owns.
    template <bool MASK, bool EN = false>
    __device__ __forceinline__ void adjoint(const Acc &a, bool inside, int p, int g,
                                            float *Sw, bool own = false, float *en = nullptr,
                                            const float *al = nullptr) const
    {
        f32x4 c[G::NTB];
#pragma unroll
        for (int nb = 0; nb < G::NTB; ++nb) c[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
        float part = 0.0f;
#pragma unroll
        for (int fb = 0; fb < NFB; ++fb) {
            Ops o;
            fetch(fb, o);
            f32x4 al4 = {0.f, 0.f, 0.f, 0.f};
            if constexpr (EN) al4 = *(const lquad *)(al + 16 * fb + 4 * g);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float zz = fmaf(last_f(o, fb, j), a.ul, a.z[fb][j]);
                if constexpr (EN) *en += own ? al4[j] * student_t_rho(zz) : 0.0f;
                float phi = zz * __builtin_amdgcn_rcpf(fmaf(zz, zz, 1.0f));
                if (MASK) phi = inside ? phi : 0.0f;
#pragma unroll
                for (int nb = 0; nb < G::NTB; ++nb)
                    c[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(phi, adj_op(o, fb, j, nb), c[nb],
                                                                 0, 0, 0);
                part = fmaf(last_a(o, fb, j), phi, part);
            }
        }
        part += __int_as_float(__builtin_amdgcn_ds_bpermute(perm16, __float_as_int(part)));
        part += __int_as_float(__builtin_amdgcn_ds_bpermute(perm32, __float_as_int(part)));
        // C[px = 4g + jj][tap = 16 nb + p] -> scratch row = tap, column = px
#pragma unroll
        for (int nb = 0; nb < G::NTB; ++nb)
            *(f32x4 *)(Sw + (16 * nb + p) * G::SW + G::SPAD + 4 * g) = c[nb];
        if (g == 0) Sw[G::LAST_ROW * G::SW + G::SPAD + p] = part;
    }
};

// ---------------------------------------------------------------------------
// Block arithmetic, BF16 or FP16 operands (P), v_mfma_f32_16x16x32_*:
// lane l supplies A[l % 16][8 (l/16) + e] and B[8 (l/16) + e][l % 16],
// e = 0..7, as 8 packed values; D[i][j] lands at lane j + 16 (i/4), item
// i % 4.
//
// Forward as in FP32 (filters x pixels), all m^2 taps on the matrix cores.
// Adjoint in gather form: psi, rounded to P, is stored per q-row in the
// wave's scratch ([q-position][filter], zero beyond the q-row), and one
// product per 16-pixel block yields the horizontal collapse directly,
//   H[a][x] = sum_{b, f} psi_f(x - b + r) (2 alpha_f k_f(a, b)),
// as D[16 px x 16 (a; only m used)] = A[16 px x K] B[K x 16 a] with
// K = (b, group of 8 filters) slots of 8: the A operand of a lane is 8
// consecutive filters of psi at one shifted pixel (one 16-byte LDS read).
// Tables (8 values of P per lane per slot):
//   t0 forward A   [KS][NFB][64][8]  A[filter 16fb + l%16][tap 32s + 8(l/16) + e]
//   t1 adjoint B   [KG][64][8]       B[slot 4s + l/16 = (b, j), filter 8j + e][a = l%16]
//                                    = 2 alpha_f k_f(a, b), slot = j * M + b
// NWV: waves per workgroup (12 for the step; the energy mode, whose
// log(1 + z^2) terms need more registers, runs 8).
template <int M, int NFB, typename P, int NWV = kWavesP16>
struct MathP16 {
    using G = Geo<M>;
    static constexpr int kNW = NWV;
    static constexpr bool kTwo = true;
    static constexpr bool kGather = true;
    static constexpr int kTabFloats = 0;
    typedef P vec8 __attribute__((ext_vector_type(8)));
    typedef P vec4 __attribute__((ext_vector_type(4)));
    // M = 7: k-step s covers tap rows 4s..4s+3, lane group g row 4s + g,
    // element e column e (8 x 8 padded; row 7 and column 7 weigh zero), so
    // a lane's 8 values are consecutive in the LDS tile.  Otherwise taps are
    // packed densely, 32 per k-step.
    static constexpr bool PAD = (M == 7);
    // M = 7: the LDS u tile holds, at every column c, the packed pair
    // (u[c], u[c + 1]) in P, converted once per launch; a lane's 8 values
    // of a k-step are then 4 aligned 32-bit words.
    static constexpr bool kPairTile = PAD;
    static constexpr int KS = PAD ? 2 : (G::T + 31) / 32;    // forward k-steps
    static constexpr int NJ = 2 * NFB;             // groups of 8 filters
    static constexpr int KG = (NJ * M + 3) / 4;    // adjoint k-steps (4 slots each)
    // psi scratch: q-positions -R .. QW + R - 1 (rows), PS values of P per
    // row (16 NFB filters and 8 unused: a row stride of 8 (2 NFB + 1) bytes
    // mod 32 words keeps the 16-byte reads of 8 consecutive lanes on
    // distinct banks)
    static constexpr int PS = 16 * NFB + 8;
    static constexpr int PROWS = kQW + 2 * G::R;
    static constexpr int kScratchFloats = PROWS * PS / 2;
    // H row stride: 4 floats more than a q-row, so that the 16-byte stores of
    // the m rows a of one block start on distinct banks
    static constexpr int kHS = kQW + 4;
    // u tile row stride: 16 mod 32 floats, so that the 4-byte reads of the
    // four lane groups (tap rows 4s + g) fall on disjoint banks
    static constexpr int kUS = 80;
    static_assert(kUS >= G::UC + 2, "u tile row too short");
    // two forward accumulators in flight (not for 64 filters of 7 x 7,
    // whose operand tables leave no room for them)
    static constexpr bool kTwoAcc = !(M == 7 && NFB == 4);
    static constexpr bool kStreamU = kTwoAcc;   // u tile rows streamed during the steps
    u32x4 afwd[KS][NFB];
    u32x4 bgat[KG];
    int boff[KS][PAD ? 1 : 8];
    int aoff[KG];        // this lane's A operand of k-step s, block 0 (P elements)
    struct Acc {
        f32x4 z[NFB];
    };

    struct Staged {};
    static __device__ void stage_load(Staged &, const void *, const void *, const void *, int) {}
    static __device__ void stage_store(float *, const Staged &, int) {}

    // The pair tile's word: lo = P(a), hi = P(b), each rounded to nearest even.
    static __device__ __forceinline__ float pack_pair(float a, float b)
    {
        const P pa = (P)a, pb = (P)b;
        const unsigned w = (unsigned)__builtin_bit_cast(unsigned short, pa) |
                           ((unsigned)__builtin_bit_cast(unsigned short, pb) << 16);
        return __builtin_bit_cast(float, w);
    }

    // 32-bit words of the operand tables t0, t1 (the layouts above)
    static constexpr int tab_words(int i)
    {
        return i == 0 ? KS * NFB * 64 * 4 : i == 1 ? KG * 64 * 4 : 0;
    }
    // FL: the tables are read from an LDS copy (same layout) instead of HBM
    template <bool FL = false>
    __device__ void load(const void *t0, const void *t1, const void *, const void *, int lane,
                         const float *)
    {
        using TP = std::conditional_t<FL, const lu32x4 *, const u32x4 *>;
        const TP fwd_tab = (TP)t0, adj_tab = (TP)t1;
        const int p = lane & 15, g = lane >> 4;
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int fb = 0; fb < NFB; ++fb) afwd[s][fb] = fwd_tab[(s * NFB + fb) * 64 + lane];
#pragma unroll
        for (int s = 0; s < KG; ++s) bgat[s] = adj_tab[s * 64 + lane];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if constexpr (PAD) {
                boff[s][0] = (4 * s + g) * kUS + p;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int t = 32 * s + 8 * g + e;
                    // padded taps read tap 0 (finite; its weight is zero)
                    boff[s][e] = t < G::T ? (t / M) * kUS + (t % M) + p : p;
                }
            }
        }
        // slot 4s + g = (b, j) = (slot % M, slot / M): psi of filters 8j..
        // at q-position p - b + R (row p - b + 2R); padding slots (zero B)
        // read row p + R.  The four lane groups of a k-step read mostly the
        // same filter group at different shifts (different rows): with the
        // groups reading one row at different filter groups instead, the
        // reads had 3x the bank-conflict cycles (measured).
#pragma unroll
        for (int s = 0; s < KG; ++s) {
            const int sg = 4 * s + g;
            const bool ok = sg < NJ * M;
            const int b = ok ? sg % M : G::R, j = ok ? sg / M : 0;
            aoff[s] = (p - b + 2 * G::R) * PS + 8 * j;
        }
    }

    __device__ __forceinline__ void forward(const float *Ub, Acc &a) const
    {
#pragma unroll
        for (int fb = 0; fb < NFB; ++fb) a.z[fb] = f32x4{0.f, 0.f, 0.f, 0.f};
        // while a wave issues its forward products its issue priority is
        // raised, so that the matrix pipe is fed ahead of the other waves'
        // vector work (BF16 and FP16 products overlap vector instructions of
        // other waves; -1 % per launch, measured; the same around the gather
        // products measured no better)
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            vec8 b;
            if constexpr (PAD) {
                const unsigned *q = (const unsigned *)Ub + boff[s][0];
                const u32x4 w = {q[0], q[2], q[4], q[6]};
                b = __builtin_bit_cast(vec8, w);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) b[e] = (P)Ub[boff[s][e]];
            }
#pragma unroll
            for (int fb = 0; fb < NFB; ++fb)
                a.z[fb] = mfma(__builtin_bit_cast(vec8, afwd[s][fb]), b, a.z[fb]);
        }
        __builtin_amdgcn_s_setprio(0);
    }

    // Influence of block k (FP32), rounded to P, into the psi scratch:
    // filters 16fb + 4g .. + 3 of q-position 16k + p (8 bytes per fb); a
    // q-position outside the image (inside = false) stores zeros.
    // EN: also adds alpha_f rho(z_f) of the lane's filters to `en` when the
    // pixel is one the tile owns (as MathF32::adjoint).
    template <bool EN = false>
    __device__ __forceinline__ void store_psi(const Acc &a, bool inside, int p, int g,
                                              unsigned short *Pw, int k, bool own = false,
                                              float *en = nullptr,
                                              const float *al = nullptr) const
    {
        unsigned short *row = Pw + (16 * k + p + G::R) * PS + 4 * g;
#pragma unroll
        for (int fb = 0; fb < NFB; ++fb) {
            vec4 v;
            f32x4 al4 = {0.f, 0.f, 0.f, 0.f};
            if constexpr (EN) al4 = *(const lquad *)(al + 16 * fb + 4 * g);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float zz = a.z[fb][i];
                if constexpr (EN) *en += own ? al4[i] * student_t_rho(zz) : 0.0f;
                v[i] = (P)(zz * __builtin_amdgcn_rcpf(fmaf(zz, zz, 1.0f)));
            }
            u32x2 w = __builtin_bit_cast(u32x2, v);
            w.x = inside ? w.x : 0u;
            w.y = inside ? w.y : 0u;
            *(volatile lpair *)(row + 16 * fb) = w;
        }
    }

    // H[a][16k + 4g + jj] (a = p < M) of block k from the psi scratch.
    __device__ __forceinline__ void gather(const unsigned short *Pw, float *Hs, int k, int p,
                                           int g) const
    {
        const unsigned short *base = Pw + 16 * k * PS;
        // all A operands are read before the first product (the reads are
        // not volatile, so they may be issued back to back)
        f32x4 w[KG];
#pragma unroll
        for (int s = 0; s < KG; ++s) w[s] = *(const lquad *)(base + aoff[s]);
        f32x4 d = {0.f, 0.f, 0.f, 0.f};

#pragma unroll
        for (int s = 0; s < KG; ++s)
            d = mfma(__builtin_bit_cast(vec8, w[s]), __builtin_bit_cast(vec8, bgat[s]), d);
        // keep the reads ahead of the products (the scheduler would
        // otherwise sink each read to its product and expose its latency)
        __builtin_amdgcn_sched_group_barrier(0x0100, KG, 0);   // LDS reads
        __builtin_amdgcn_sched_group_barrier(0x0008, KG, 0);   // MFMA
        if (p < M) *(f32x4 *)(Hs + p * kHS + 16 * k + 4 * g) = d;
    }

    static __device__ __forceinline__ f32x4 mfma(vec8 a, vec8 b, f32x4 c)
    {
        if constexpr (std::is_same<P, __bf16>::value)
            return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
        else
            return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

template <int M, typename Math, int MODE = kStep>
__global__ __launch_bounds__(64 * Math::kNW)
__attribute__((amdgpu_waves_per_eu(Math::kNW / 4, Math::kNW / 4)))
void fused_step_kernel(const JobDesc *__restrict__ jobs, int njobs,
                       const void *__restrict__ t0, const void *__restrict__ t1,
                       const void *__restrict__ t2, const void *__restrict__ t3,
                       int iter, int ty_max, int tile0, const float *__restrict__ alpha,
                       float *__restrict__ epart)
{
    constexpr bool GRAD = MODE != kStep, EN = MODE == kGradEnergy;
    using G = Geo<M>;
    constexpr int R = G::R;
    constexpr int NW = Math::kNW;
    constexpr int HR = Ring<M, NW, Math::kTwo>::HR;
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int p = lane & 15;   // pixel within a 16-pixel block
    const int g = lane >> 4;   // lane group: k index of the MFMA operands

    // ---- locate the tile: jobs are sorted by tile_base --------------------
    // Launches cover tiles tile0 .. tile0 + gridDim.x - 1.  Workgroups go to
    // the 8 XCDs in turn (workgroup i to XCD i % 8), each XCD with its own
    // L2: XCD x takes one contiguous run of tiles, so that the tiles next to
    // each other in a job (which read each other's halo rows and columns of
    // u) share an L2.
    const int bid = tile0 + xcd_tile((int)blockIdx.x, (int)gridDim.x);
    // 64-way search: each lane reads the tile_base of one sample of the
    // remaining range and a ballot counts the samples at or below the tile
    // (sample 0 always is), so 64 jobs take one round of loads and 4096 two,
    // instead of one dependent load per halving.
    int lo = 0, cnt = njobs;                   // the tile's job lies in [lo, lo + cnt)
    while (cnt > 1) {
        const int step = (cnt + 63) / 64;      // jobs per sample
        const bool le = lane * step < cnt && jobs[lo + lane * step].tile_base <= bid;
        const int k = __popcll(__ballot(le));
        lo += (k - 1) * step;
        cnt = min(step, cnt - (k - 1) * step);
    }
    const JobDesc J = jobs[lo];
    if (iter >= J.iters) return;
    const int local = bid - J.tile_base;
    const int tix = local % J.ntx, tiy = local / J.ntx;
    if (tiy >= J.nty) return;
    const int H = J.H, W = J.W;
    const int x0 = (int)((long)tix * W / J.ntx), x1 = (int)((long)(tix + 1) * W / J.ntx);
    const int y0 = (int)((long)tiy * H / J.nty), y1 = (int)((long)(tiy + 1) * H / J.nty);
    const int tx = x1 - x0, ty = y1 - y0;
    const bool odd = ((J.it0 + iter) & 1) != 0;
    const gfloat *ucur = (const gfloat *)(odd ? J.ub : J.ua);
    gfloat *uprev = (gfloat *)(odd ? J.ua : J.ub);  // u^{n-1} -> u^{n+1}
    const gfloat *counts = (const gfloat *)J.counts;

    float *U = lds;                                        // (ty_max + 4R) x US
    float *S = U + (size_t)(ty_max + 4 * R + G::UROWS_EXTRA) * Math::kUS;  // per-wave scratch
    float *Hr = S + (size_t)NW * Math::kScratchFloats;     // HR x M x QW
    float *Tab = Hr + (size_t)HR * M * Math::kHS;          // the policy's tables
    float *Al = Tab + Math::kTabFloats;                    // alpha_i (energy mode)
    // TWO form of the pipeline: per-wave count of finished output-row phases
    int *fdone = (int *)(Al + (MODE == kGradEnergy ? kAlphaFloats : 0));
    float *Sw = S + (size_t)wave * Math::kScratchFloats;
    unsigned short *Pw = (unsigned short *)Sw;             // psi scratch (gather form)

    // ---- u tile: image rows y0-2R.., cols x0-2R.., symmetric extension ----
    // (one more row and the two padding columns hold finite values that
    // zero-weight taps of the padded BF16/FP16 layout may read).  Step st
    // reads tile rows below (st + 1) NW + 2R + 1.  Where the registers allow
    // (Math::kStreamU), the prologue loads the rows of step 0 and during step
    // st wave w fetches tile row (st + 1) NW + 2R + 1 + w (loads issued at
    // the start of the step, the row stored to LDS before its first
    // barrier); otherwise the prologue loads the whole tile.
    const int urows = ty + 4 * R + G::UROWS_EXTRA;
    constexpr int kURow0 = NW + 2 * R + G::UROWS_EXTRA;   // rows step 0 reads
    const int urows0 = Math::kStreamU ? min(urows, kURow0) : urows;
    // Loads go out kUB per thread before their LDS stores, so that their
    // latencies overlap (a load-store loop waits one latency per element).
    // The first batch (all of it when the rows stream) is issued before the
    // operand tables: the tables' many loads would otherwise queue ahead of
    // it and its latency would follow theirs instead of overlapping them.
    constexpr int kUB = 4;
    const int nu = urows0 * Math::kUS;
    float va[kUB], vb[kUB];
    auto u_load = [&](int i0) {
#pragma unroll
        for (int j = 0; j < kUB; ++j) {
            const int i = i0 + j * 64 * NW;
            va[j] = vb[j] = 0.0f;
            if (i < nu) {
                const int ur = i / Math::kUS, uc = i - ur * Math::kUS;
                const gfloat *row = ucur + (long)sym_clamp(y0 - 2 * R + ur, H) * W;
                va[j] = row[sym_clamp(x0 - 2 * R + uc, W)];
                if constexpr (Math::kPairTile) vb[j] = row[sym_clamp(x0 - 2 * R + uc + 1, W)];
            }
        }
    };
    auto u_put = [&](int i0) {
#pragma unroll
        for (int j = 0; j < kUB; ++j) {
            const int i = i0 + j * 64 * NW;
            if (i < nu) {
                if constexpr (Math::kPairTile) U[i] = Math::pack_pair(va[j], vb[j]);
                else U[i] = va[j];
            }
        }
    };
    u_load(threadIdx.x);
    typename Math::Staged staged;
    Math::stage_load(staged, t1, t2, t3, threadIdx.x);

    // ---- operand tables ----------------------------------------------------
    // Every wave needs the same per-lane tables in registers.  Where they fit
    // the H ring (unused until step 0), the workgroup reads them from HBM
    // once, cooperatively, into the ring, and
    // the waves load their registers from there: one pass through the vector
    // L1 instead of one per wave (the L1 bandwidth bounded the per-wave reads).
    // (a policy that keeps t1 .. t3 in LDS itself stages t0 only)
    constexpr int kTw0 = Math::tab_words(0), kTw1 = Math::tab_words(1),
                  kTw2 = Math::tab_words(2), kTw3 = Math::tab_words(3);
    constexpr bool kOwnTabs = Math::kTabFloats != 0;
    constexpr int kTq = (kOwnTabs ? kTw0 : kTw0 + kTw1 + kTw2 + kTw3) / 4;   // 16-byte quads
    constexpr bool kStageTabs = kTq * 4 <= HR * M * Math::kHS && kTw0 % 4 == 0 &&
                                (kOwnTabs || (kTw1 % 4 == 0 && kTw2 % 4 == 0));
    constexpr int kTqPer = (kTq + 64 * NW - 1) / (64 * NW);
    u32x4 tq[kStageTabs ? kTqPer : 1];
    if constexpr (kStageTabs) {
#pragma unroll
        for (int j = 0; j < kTqPer; ++j) {
            const int q = threadIdx.x + j * 64 * NW;
            if (q < kTq) {
                const u32x4 *src = q < kTw0 / 4 ? (const u32x4 *)t0 + q
                                   : q < (kTw0 + kTw1) / 4 ? (const u32x4 *)t1 + (q - kTw0 / 4)
                                   : q < (kTw0 + kTw1 + kTw2) / 4
                                       ? (const u32x4 *)t2 + (q - (kTw0 + kTw1) / 4)
                                       : (const u32x4 *)t3 + (q - (kTw0 + kTw1 + kTw2) / 4);
                tq[j] = *(const __attribute__((address_space(1))) u32x4 *)src;
            }
        }
    }
    Math mth;
    if constexpr (!kStageTabs) mth.load(t0, t1, t2, t3, lane, Tab);

    // Collapse tasks of this lane, round rr: (a, xr) with task = 64 rr + lane
    // = a * XSPAN + xr + R.  sbase: scratch offset of tap (a, 0) at the
    // block column xr + R; hoff: H offset of (a, xr); xrr: xr, or a value
    // that never lands in the row when the task does not exist (its loads
    // then read a harmless in-range address and its store is skipped).
    int sbase[G::ROUNDS], hoff[G::ROUNDS], xrr[G::ROUNDS];
#pragma unroll
    for (int rr = 0; rr < G::ROUNDS; ++rr) {
        const int task = rr * 64 + lane;
        const bool ok = task < G::TASKS;
        const int a = ok ? task / G::XSPAN : 0;
        const int xr = ok ? task - a * G::XSPAN - R : 0;
        sbase[rr] = (a * M) * G::SW + G::SPAD + xr + R;
        hoff[rr] = a * Math::kHS + xr;
        xrr[rr] = ok ? xr : -1000;
    }

    // ---- zero this wave's scratch (its pad columns / rows stay zero) ------
    for (int i = lane; i < Math::kScratchFloats; i += 64) Sw[i] = 0.0f;

    u_put(threadIdx.x);
    if constexpr (kStageTabs) {
        u32x4 *Hq = (u32x4 *)Hr;
#pragma unroll
        for (int j = 0; j < kTqPer; ++j) {
            const int q = threadIdx.x + j * 64 * NW;
            if (q < kTq) Hq[q] = tq[j];
        }
        lds_barrier();
        mth.template load<true>(Hr, Hr + kTw0, Hr + kTw0 + kTw1, Hr + kTw0 + kTw1 + kTw2, lane,
                                Tab);
    }
    for (int i0 = threadIdx.x + kUB * 64 * NW; i0 < nu; i0 += kUB * 64 * NW) {
        u_load(i0);
        u_put(i0);
    }
    // the wave index as a scalar (the row arithmetic of the steps stays on
    // the scalar unit: -1 % per launch, measured)
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    // the row a wave fetches: columns lane and 64 + lane (lane < US - 64),
    // both values of each pair for the pair tile
    float uf[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    auto u_fetch = [&](int st) {
        const int ur = (st + 1) * NW + 2 * R + G::UROWS_EXTRA + wv;
        if (Math::kStreamU && ur < urows) {
            const gfloat *row = ucur + (long)sym_clamp(y0 - 2 * R + ur, H) * W;
            const int c0 = x0 - 2 * R + lane;
            uf[0] = row[sym_clamp(c0, W)];
            if constexpr (Math::kPairTile) uf[1] = row[sym_clamp(c0 + 1, W)];
            if (lane < Math::kUS - 64) {
                uf[2] = row[sym_clamp(c0 + 64, W)];
                if constexpr (Math::kPairTile) uf[3] = row[sym_clamp(c0 + 65, W)];
            }
        }
    };
    auto u_store = [&](int st) {
        const int ur = (st + 1) * NW + 2 * R + G::UROWS_EXTRA + wv;
        if (Math::kStreamU && ur < urows) {
            float *dst = U + ur * Math::kUS + lane;
            if constexpr (Math::kPairTile) {
                dst[0] = Math::pack_pair(uf[0], uf[1]);
                if (lane < Math::kUS - 64) dst[64] = Math::pack_pair(uf[2], uf[3]);
            } else {
                dst[0] = uf[0];
                if (lane < Math::kUS - 64) dst[64] = uf[2];
            }
        }
    };
    Math::stage_store(Tab, staged, threadIdx.x);
    if constexpr (EN)
        if (threadIdx.x < kAlphaFloats) Al[threadIdx.x] = alpha[threadIdx.x];
    if constexpr (Math::kTwo)
        if (threadIdx.x < NW) fdone[threadIdx.x] = 0;
    // per-lane partial energies of the pixels this tile owns (energy mode)
    float e_prior = 0.0f, e_data = 0.0f;
    // Every global load of the prologue (operand tables, u tile) has landed:
    // said explicitly, so that the compiler's wait counting does not carry
    // them into the step loop, where a conservative wait would also wait
    // for the prefetches issued there.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    const int nq = ty + 2 * R;                 // q-rows of the tile
    const int nsteps = (nq + NW - 1) / NW;

    using Acc = typename Math::Acc;
    // ---- one 16-pixel block: forward bank (matrix cores) ------------------
    auto forward = [&](int qr, int k, Acc &acc) {
        mth.forward(U + qr * Math::kUS + 16 * k, acc);
    };
    // ---- influence, adjoint bank, tap contributions into the scratch ------
    // Pixels of block k outside the image carry psi = 0 (the adjoint's
    // input vanishes off the image); blocks wholly inside skip the mask.
    // Energy mode: a q-row pixel counts towards the energy only in the tile
    // that owns it (rows y0..y1-1, columns x0..x1-1), so that each image
    // pixel is counted once over the tiles.
    auto adjoint = [&](int k, const Acc &acc, bool own_row) {
        const int q0 = x0 - R + 16 * k;
        const int qx = q0 + p;
        const bool own = own_row && qx >= x0 && qx < x1;
        if constexpr (Math::kGather) {
            mth.template store_psi<EN>(acc, qx >= 0 && qx < W, p, g, Pw, k, own, &e_prior, Al);
        } else {
            if (q0 >= 0 && q0 + 15 < W) {
                mth.template adjoint<false, EN>(acc, true, p, g, Sw, own, &e_prior, Al);
            } else {
                mth.template adjoint<true, EN>(acc, qx >= 0 && qx < W, p, g, Sw, own, &e_prior,
                                               Al);
            }
        }
    };
    // ---- horizontal collapse of block k into the q-row's H slot -----------
    //   H[a][16k + xr] (+)= sum_b C[xr + R - b][(a, b)]; the first block to
    //   reach a column writes it, the next one adds.
    auto collapse = [&](float *Hs, int k) {
        // all loads first (no branch between them), then sums and stores
        float v[G::ROUNDS][M], old[G::ROUNDS];
        int hidx[G::ROUNDS];
        bool st[G::ROUNDS], add[G::ROUNDS];
#pragma unroll
        for (int rr = 0; rr < G::ROUNDS; ++rr) {
            const int xr = xrr[rr];
            const int x = 16 * k + xr;
            st[rr] = x >= 0 && x < kQW;
            add[rr] = k > 0 && xr < R;
            hidx[rr] = st[rr] ? hoff[rr] + 16 * k : 0;
            const float *sp = Sw + sbase[rr];
#pragma unroll
            for (int b = 0; b < M; ++b) v[rr][b] = sp[b * (G::SW - 1)];
            old[rr] = Hs[hidx[rr]];
        }
#pragma unroll
        for (int rr = 0; rr < G::ROUNDS; ++rr) {
            float acc = v[rr][0];
#pragma unroll
            for (int b = 1; b < M; ++b) acc += v[rr][b];
            if (st[rr]) Hs[hidx[rr]] = add[rr] ? old[rr] + acc : acc;
        }
    };
    // ---- output rows: g = sum over ghosts and a of H; iPiano update --------
    // Inputs of the row a wave will finish are fetched one step ahead.
    float pf_up = 0.0f, pf_y = 0.0f, pf_u = 0.0f;
    auto prefetch = [&](int st) {
        const int orow = st * NW - 2 * R + wv;
        if (orow >= 0 && orow < ty && lane < tx) {
            const long pix = (long)(y0 + orow) * W + x0 + lane;
            if constexpr (!GRAD) pf_up = uprev[pix];
            pf_y = counts[pix];
            if constexpr (Math::kPairTile) pf_u = ucur[pix];   // the tile holds P pairs
        }
    };
    auto finalize = [&](int st) {
        const int orow = st * NW - 2 * R + wv;
        if (orow < 0 || orow >= ty) return;    // uniform over the wave
        const int y = y0 + orow;
        const int x = x0 + (lane < tx ? lane : tx - 1);
        // the column and, at the left or right border, its ghost columns
        // (both when W < 2R); side: the tile reaches a left or right border
        // (uniform), else no lane has ghost columns and one load per a does
        const int hx = x - (x0 - R);
        const bool gl = x < R, gr = x >= W - R;
        const int hgl = gl ? (-1 - x) - (x0 - R) : hx;
        const int hgr = gr ? (2 * W - 1 - x) - (x0 - R) : hx;
        const bool side = x0 < R || x1 > W - R;
        // sum over a of H[row - a + R][a] for one extended row; every load
        // is issued before the first add (rows off the image weigh zero).
        // The ring slot of tile q-row row + 2R - y0 - a: one modulo for
        // a = 0, then a decrement that wraps.
        auto row_sum = [&](int row) {
            float vh[M], vl[M], vr[M];
            bool ok[M];
            int slot = (row + 2 * R - y0) % HR;   // the index is >= 0
#pragma unroll
            for (int a = 0; a < M; ++a) {
                const int qyy = row - a + R;
                ok[a] = qyy >= 0 && qyy < H;
                const float *h = Hr + (size_t)slot * M * Math::kHS + a * Math::kHS;
                vh[a] = h[hx];
                if (side) {
                    vl[a] = h[hgl];
                    vr[a] = h[hgr];
                }
                slot = slot == 0 ? HR - 1 : slot - 1;
            }
            float sum = 0.0f;
#pragma unroll
            for (int a = 0; a < M; ++a) {
                float t = vh[a];
                if (side) {
                    t += gl ? vl[a] : 0.0f;
                    t += gr ? vr[a] : 0.0f;
                }
                sum += ok[a] ? t : 0.0f;
            }
            return sum;
        };
        // the output row and, at the top or bottom border, its ghost rows
        float gsum = 0.0f;
        if (y < R) gsum += row_sum(-1 - y);
        gsum += row_sum(y);
        if (y >= H - R) gsum += row_sum(2 * H - 1 - y);
        if (lane >= tx) return;
        float uc;
        if constexpr (Math::kPairTile) uc = pf_u;
        else uc = U[(orow + 2 * R) * Math::kUS + lane + 2 * R];
        // the column laundered: its 64-bit address is formed here each step
        // rather than hoisted out of the step loop into a register pair
        int xs = x;
        asm volatile("" : "+v"(xs));
        if constexpr (GRAD) {
            const float v = anscombe_fast(pf_y);
            if constexpr (EN) e_data += data_energy(uc, v, J.data_term);
            if (uprev)
                uprev[(long)y * W + xs] = gsum + J.lambda * data_gradient_fast(uc, v, J.data_term);
        } else {
            const float ut = inertial_step(uc, pf_up, gsum, J.tau, J.gamma);
            uprev[(long)y * W + xs] = prox_fast(ut, anscombe_fast(pf_y), J.tl, J.q1, J.data_term);
        }
    };

    // TWO form of the pipeline: instead of a second barrier per step, a
    // wait, right before a q-row's first write into the H ring, for the
    // output rows that still read the slot it overwrites.  q-row
    // qr = st NW + w takes the slot of q-row qr - (NW + 2R), which only the
    // output rows finished in step st - 1 by waves w - 2R .. w read (older
    // readers finished before the step's first barrier).  A wave's count in
    // fdone is the number of its output-row phases finished.  The waited-for
    // waves belong to the workgroup and reach their release (after their
    // output rows) without waiting on anything but the step's barrier, which
    // this wave has passed, so the wait ends.  The spin is bounded all the
    // same (at ~0.1 s, far beyond any real wait; a wave that gave up would go
    // on with wrong results, but every wave ends).
    auto ring_wait = [&](int st) {
        if constexpr (Math::kTwo) {
            if (st == 0) return;
            for (int spin = 0; spin < kRingSpins; ++spin) {
                int ok = 1;
                if (lane < NW && lane >= wv - 2 * R && lane <= wv)
                    ok = __hip_atomic_load(fdone + lane, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP) >= st;
                if (__all(ok)) break;
                __builtin_amdgcn_s_sleep(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        }
    };
    auto ring_release = [&](int st) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        if (lane == 0)
            __hip_atomic_store(fdone + wv, st + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };

    auto qrow = [&](int st) {
        const int qr = st * NW + wv;
        const int qy = y0 - R + qr;
        const bool own_row = qr >= R && qr < R + ty;
        if (qr < nq && qy >= 0 && qy < H) {
            float *Hs = Hr + (size_t)(qr % HR) * M * Math::kHS;
            Acc acc;
            if constexpr (Math::kGather) {
                // psi of every block into the scratch; block k's H needs psi
                // of blocks k - 1 .. k + 1, so it follows psi of block k + 1.
                // Branch-free, two accumulators: the forward products of
                // block k + 1 are issued before the influence of block k.
                // (one accumulator where two would not fit the registers)
                constexpr bool two = Math::kTwoAcc;
                Acc acc1;
                Acc &accb = two ? acc1 : acc;
                forward(qr, 0, acc);
                if (two) forward(qr, 1, accb);
                adjoint(0, acc, own_row);
                if (!two) forward(qr, 1, accb);
                if (two) forward(qr, 2, acc);
                adjoint(1, accb, own_row);
                ring_wait(st);
                lds_order();
                mth.gather(Pw, Hs, 0, p, g);
                if (!two) forward(qr, 2, acc);
                if (two) forward(qr, 3, accb);
                adjoint(2, acc, own_row);
                lds_order();
                mth.gather(Pw, Hs, 1, p, g);
                if (!two) forward(qr, 3, accb);
                adjoint(3, accb, own_row);
                lds_order();
                mth.gather(Pw, Hs, 2, p, g);
                mth.gather(Pw, Hs, 3, p, g);
                lds_order();
            } else {
                // software pipeline: the collapse of block k - 1 (LDS, VALU)
                // is issued next to the forward MFMAs of block k
                forward(qr, 0, acc);
                adjoint(0, acc, own_row);
#pragma unroll
                for (int k = 1; k < kQB; ++k) {
                    lds_order();
                    forward(qr, k, acc);
                    if (k == 1 && Math::kTwo) ring_wait(st);
                    collapse(Hs, k - 1);
                    lds_order();
                    adjoint(k, acc, own_row);
                }
                lds_order();
                collapse(Hs, kQB - 1);
                lds_order();
            }
        }
    };

    if constexpr (Math::kTwo) {
        // Step st: q-row st * NW + wave, barrier, then the output rows whose
        // q-rows are now complete (the ring needs NW + 2R slots; the next
        // q-row's first ring write waits for the output rows that read the
        // slot it takes: ring_wait).
        for (int st = 0; st < nsteps; ++st) {
            prefetch(st);
            u_fetch(st);
            qrow(st);
            u_store(st);
            lds_barrier();
            // the output rows (vector work that the waves waiting in ring_wait
            // depend on) at the highest issue priority of the step (-1 % per
            // launch, measured)
            __builtin_amdgcn_s_setprio(2);
            finalize(st);
            __builtin_amdgcn_s_setprio(0);
            ring_release(st);
        }
    } else {
        // Step st: finish the output rows of step st - 1, then run q-row
        // st * NW + wave.  One barrier per step; the ring holds 2 NW + 2R
        // q-rows so rows being finished and rows being written never share
        // a slot.
        for (int st = 0; st <= nsteps; ++st) {
            if (st > 0) finalize(st - 1);
            if (st < nsteps) {
                prefetch(st);
                u_fetch(st);
                qrow(st);
                u_store(st);
            }
            lds_barrier();
        }
    }
    if constexpr (EN) {
        // The workgroup's partial energies: lanes, then waves, in a fixed
        // order (after a barrier that retires every LDS read of the steps,
        // the u tile's first floats are free).
        lds_barrier();
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            e_prior += __shfl_xor(e_prior, o);
            e_data += __shfl_xor(e_data, o);
        }
        if (lane == 0) {
            U[2 * wave] = e_prior;
            U[2 * wave + 1] = e_data;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            float sp = 0.0f, sd = 0.0f;
            for (int w = 0; w < NW; ++w) {
                sp += U[2 * w];
                sd += U[2 * w + 1];
            }
            epart[2 * (long)bid] = sp;
            epart[2 * (long)bid + 1] = sd;
        }
    }
}

// Job table upload through kernel arguments (no host-to-device copy, so the
// call stays asynchronous and capturable).
constexpr int kChunk = 32;
constexpr int kMaxLaunchTiles = 1 << 21;   // x 1024 threads at most = 2^31 work-items
struct JobChunk {
    int first, count;
    JobDesc d[kChunk];
};

__global__ void write_jobs_kernel(JobChunk c, JobDesc *dst)
{
    const int i = threadIdx.x;
    if (i < c.count) dst[c.first + i] = c.d[i];
}

int nfb_for(int nf) { return (nf + 15) / 16; }

template <int M, typename Math, int MODE = kStep>
hipError_t launch_step(const void *const *tabs, const JobDesc *jobs, int njobs, int nblocks,
                       int tile0, int iter, int ty_max, hipStream_t s,
                       const float *alpha = nullptr, float *epart = nullptr)
{
    constexpr int NW = Math::kNW;
    if (ty_max > rows_limit<M, Math, MODE>()) return hipErrorInvalidValue;
    const size_t bytes = lds_bytes<M, Math, MODE>(ty_max);
    // the dynamic-LDS limit is raised once per device (any thread)
    static std::atomic<uint64_t> attr_set{0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = dev < 64 ? (uint64_t)1 << dev : 0;
    if (!bit || !(attr_set.load(std::memory_order_acquire) & bit)) {
        e = hipFuncSetAttribute((const void *)fused_step_kernel<M, Math, MODE>,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_bytes<M, Math, MODE>(rows_limit<M, Math, MODE>()));
        if (e != hipSuccess) return e;
        attr_set.fetch_or(bit, std::memory_order_release);
    }
    fused_step_kernel<M, Math, MODE><<<nblocks, 64 * NW, bytes, s>>>(
        jobs, njobs, tabs[0], tabs[1], tabs[2], tabs[3], iter, ty_max, tile0, alpha, epart);
    return hipGetLastError();
}

// Gradient modes: FP32 runs the 8-wave variant (built for every bank),
// BF16 / FP16 their 12-wave variant.
constexpr int kWavesP16Energy = 8;
template <int MODE>
constexpr int p16_waves() { return MODE == kGradEnergy ? kWavesP16Energy : kWavesP16; }

template <int M, int NFB, int MODE>
hipError_t launch_grad_prec(int prec, const FusedBank &b, const JobDesc *jobs, int njobs,
                            int nblocks, int tile0, int ty_max, float *epart, hipStream_t s)
{
    constexpr int NWV = p16_waves<MODE>();
    if (prec == FE_PREC_BF16) {
        const void *t[4] = {b.bf_fwd, b.bf_adj, nullptr, nullptr};
        return launch_step<M, MathP16<M, NFB, __bf16, NWV>, MODE>(t, jobs, njobs, nblocks, tile0, 0,
                                                                   ty_max, s, b.alpha, epart);
    }
    if (prec == FE_PREC_FP16) {
        const void *t[4] = {b.h_fwd, b.h_adj, nullptr, nullptr};
        return launch_step<M, MathP16<M, NFB, _Float16, NWV>, MODE>(t, jobs, njobs, nblocks, tile0,
                                                                     0, ty_max, s, b.alpha, epart);
    }
    const void *t[4] = {b.fwd, b.adj, b.lastf, b.lasta};
    return launch_step<M, MathF32<M, NFB, false>, MODE>(t, jobs, njobs, nblocks, tile0, 0,
                                                         ty_max, s, b.alpha, epart);
}

template <int M, int NFB>
int rows_grad_prec(int prec, bool energy)
{
    constexpr int NWE = p16_waves<kGradEnergy>();
    if (prec == FE_PREC_BF16)
        return energy ? rows_limit<M, MathP16<M, NFB, __bf16, NWE>, kGradEnergy>()
                      : rows_limit<M, MathP16<M, NFB, __bf16>, kGrad>();
    if (prec == FE_PREC_FP16)
        return energy ? rows_limit<M, MathP16<M, NFB, _Float16, NWE>, kGradEnergy>()
                      : rows_limit<M, MathP16<M, NFB, _Float16>, kGrad>();
    return energy ? rows_limit<M, MathF32<M, NFB, false>, kGradEnergy>()
                  : rows_limit<M, MathF32<M, NFB, false>, kGrad>();
}

// The 12-wave FP32 variant is built where its registers fit three waves
// per SIMD (168): 64 filters of 7 x 7 do not.
template <int M, int NFB>
constexpr bool f32_lds_built() { return !(M == 7 && NFB == 4); }

template <int M, int NFB>
hipError_t launch_prec(int prec, int nw, const FusedBank &b, const JobDesc *jobs, int njobs,
                       int nblocks, int tile0, int iter, int ty_max, hipStream_t s)
{
    if (prec == FE_PREC_BF16) {
        const void *t[4] = {b.bf_fwd, b.bf_adj, nullptr, nullptr};
        return launch_step<M, MathP16<M, NFB, __bf16>>(t, jobs, njobs, nblocks, tile0, iter, ty_max, s);
    }
    if (prec == FE_PREC_FP16) {
        const void *t[4] = {b.h_fwd, b.h_adj, nullptr, nullptr};
        return launch_step<M, MathP16<M, NFB, _Float16>>(t, jobs, njobs, nblocks, tile0, iter, ty_max, s);
    }
    const void *t[4] = {b.fwd, b.adj, b.lastf, b.lasta};
    if (nw == 12) {
        if constexpr (f32_lds_built<M, NFB>())
            return launch_step<M, MathF32<M, NFB, true>>(t, jobs, njobs, nblocks, tile0, iter, ty_max, s);
        return hipErrorInvalidValue;
    }
    return launch_step<M, MathF32<M, NFB, false>>(t, jobs, njobs, nblocks, tile0, iter, ty_max, s);
}

// Tallest tile of a variant (0 if the variant is not built).
template <int M, int NFB>
int rows_prec(int prec, int nw)
{
    if (prec == FE_PREC_BF16)
        return nw == kWavesP16 ? rows_limit<M, MathP16<M, NFB, __bf16>>() : 0;
    if (prec == FE_PREC_FP16)
        return nw == kWavesP16 ? rows_limit<M, MathP16<M, NFB, _Float16>>() : 0;
    if (nw == 12) {
        if constexpr (f32_lds_built<M, NFB>()) return rows_limit<M, MathF32<M, NFB, true>>();
        return 0;
    }
    return nw == kWavesF32 ? rows_limit<M, MathF32<M, NFB, false>>() : 0;
}

hipError_t launch_grad_any(int prec, bool energy, const FusedBank &b, const JobDesc *jobs,
                           int njobs, int nblocks, int tile0, int ty_max, float *epart,
                           hipStream_t s)
{
#define FE_GRAD(MM, NB)                                                                       \
    return energy ? launch_grad_prec<MM, NB, kGradEnergy>(prec, b, jobs, njobs, nblocks, tile0, \
                                                          ty_max, epart, s)                   \
                  : launch_grad_prec<MM, NB, kGrad>(prec, b, jobs, njobs, nblocks, tile0,     \
                                                    ty_max, nullptr, s)
    switch (b.m * 10 + b.nfb) {
    case 31: FE_GRAD(3, 1);
    case 32: FE_GRAD(3, 2);
    case 33: FE_GRAD(3, 3);
    case 34: FE_GRAD(3, 4);
    case 51: FE_GRAD(5, 1);
    case 52: FE_GRAD(5, 2);
    case 53: FE_GRAD(5, 3);
    case 54: FE_GRAD(5, 4);
    case 71: FE_GRAD(7, 1);
    case 72: FE_GRAD(7, 2);
    case 73: FE_GRAD(7, 3);
    case 74: FE_GRAD(7, 4);
    default: return hipErrorInvalidValue;
    }
#undef FE_GRAD
}

int rows_grad_any(int m, int nfb, int prec, bool energy)
{
#define FE_ROWS(MM, NB) return rows_grad_prec<MM, NB>(prec, energy)
    switch (m * 10 + nfb) {
    case 31: FE_ROWS(3, 1);
    case 32: FE_ROWS(3, 2);
    case 33: FE_ROWS(3, 3);
    case 34: FE_ROWS(3, 4);
    case 51: FE_ROWS(5, 1);
    case 52: FE_ROWS(5, 2);
    case 53: FE_ROWS(5, 3);
    case 54: FE_ROWS(5, 4);
    case 71: FE_ROWS(7, 1);
    case 72: FE_ROWS(7, 2);
    case 73: FE_ROWS(7, 3);
    case 74: FE_ROWS(7, 4);
    default: return 0;
    }
#undef FE_ROWS
}

hipError_t launch_any(int prec, int nw, const FusedBank &b, const JobDesc *jobs, int njobs,
                      int nblocks, int tile0, int iter, int ty_max, hipStream_t s)
{
#define FE_STEP(MM, NB) \
    return launch_prec<MM, NB>(prec, nw, b, jobs, njobs, nblocks, tile0, iter, ty_max, s)
    switch (b.m * 10 + b.nfb) {
    case 31: FE_STEP(3, 1);
    case 32: FE_STEP(3, 2);
    case 33: FE_STEP(3, 3);
    case 34: FE_STEP(3, 4);
    case 51: FE_STEP(5, 1);
    case 52: FE_STEP(5, 2);
    case 53: FE_STEP(5, 3);
    case 54: FE_STEP(5, 4);
    case 71: FE_STEP(7, 1);
    case 72: FE_STEP(7, 2);
    case 73: FE_STEP(7, 3);
    case 74: FE_STEP(7, 4);
    default: return hipErrorInvalidValue;
    }
#undef FE_STEP
}

// Round to nearest even: float -> bfloat16 bits (finite inputs).
uint16_t bf16_bits(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

uint16_t f16_bits(float x)
{
    _Float16 h = (_Float16)x;  // round to nearest even
    uint16_t b;
    std::memcpy(&b, &h, 2);
    return b;
}

}  // namespace

bool fused_supported(int m, int nf) { return (m == 3 || m == 5 || m == 7) && nf >= 1 && nf <= 64; }

// Host-side construction of the operand tables (lane layouts of
// v_mfma_f32_16x16x4_f32: A[i][k] at lane i + 16k, B[k][j] at lane j + 16k,
// D[i][j] at lane j + 16 (i / 4), item i % 4).
hipError_t fused_upload(const float *taps, const float *alpha, int m, int nf, FusedBank *out)
{
    const int T = m * m, KF = (T - 1) / 4, NTB = (T - 1 + 15) / 16, NFB = nfb_for(nf);
    auto tap = [&](int f, int t) { return (f < nf && t < T) ? taps[f * T + t] : 0.0f; };
    auto a2 = [&](int f) { return f < nf ? 2.0f * alpha[f] : 0.0f; };
    std::vector<float> fwd((size_t)KF * NFB * 64), adj((size_t)NFB * 4 * NTB * 64),
        lastf((size_t)NFB * 4 * 64), lasta((size_t)NFB * 4 * 64);
    for (int s = 0; s < KF; ++s)
        for (int fb = 0; fb < NFB; ++fb)
            for (int l = 0; l < 64; ++l)  // A[filter = l%16][tap = 4s + l/16]
                fwd[(s * NFB + fb) * 64 + l] = tap(fb * 16 + (l & 15), 4 * s + (l >> 4));
    for (int fb = 0; fb < NFB; ++fb)
        for (int j = 0; j < 4; ++j)
            for (int nb = 0; nb < NTB; ++nb)
                for (int l = 0; l < 64; ++l) {  // B[k = filter 4(l/16)+j][tap 16nb + l%16]
                    const int f = fb * 16 + 4 * (l >> 4) + j, t = nb * 16 + (l & 15);
                    adj[((fb * 4 + j) * NTB + nb) * 64 + l] = t < T - 1 ? a2(f) * tap(f, t) : 0.0f;
                }
    for (int fb = 0; fb < NFB; ++fb)
        for (int j = 0; j < 4; ++j)
            for (int l = 0; l < 64; ++l) {
                const int f = fb * 16 + 4 * (l >> 4) + j;
                lastf[(fb * 4 + j) * 64 + l] = tap(f, T - 1);
                lasta[(fb * 4 + j) * 64 + l] = a2(f) * tap(f, T - 1);
            }
    // BF16 / FP16 operands (16x16x32 lane layout; see MathP16)
    const int KS = m == 7 ? 2 : (T + 31) / 32, NJ = 2 * NFB, KG = (NJ * m + 3) / 4;
    std::vector<float> pf((size_t)KS * NFB * 64 * 8), pa((size_t)KG * 64 * 8);
    for (int s = 0; s < KS; ++s)
        for (int fb = 0; fb < NFB; ++fb)
            for (int l = 0; l < 64; ++l)
                for (int e = 0; e < 8; ++e)
                    pf[((s * NFB + fb) * 64 + l) * 8 + e] =
                        m == 7 ? ((4 * s + (l >> 4)) < 7 && e < 7
                                      ? tap(fb * 16 + (l & 15), (4 * s + (l >> 4)) * 7 + e)
                                      : 0.0f)
                               : tap(fb * 16 + (l & 15), 32 * s + 8 * (l >> 4) + e);
    for (int s = 0; s < KG; ++s)
        for (int l = 0; l < 64; ++l)
            for (int e = 0; e < 8; ++e) {
                // B[slot (b, j), filter 8j + e][a]: slot 4s + l/16 = j * m + b
                const int sg = 4 * s + (l >> 4), a = l & 15;
                const int b = sg % m, f = 8 * (sg / m) + e;
                pa[((size_t)s * 64 + l) * 8 + e] =
                    (sg < NJ * m && a < m) ? a2(f) * tap(f, a * m + b) : 0.0f;
            }
    std::vector<uint16_t> bff(pf.size()), bfa(pa.size()), hf(pf.size()), ha(pa.size());
    for (size_t i = 0; i < pf.size(); ++i) {
        bff[i] = bf16_bits(pf[i]);
        hf[i] = f16_bits(pf[i]);
    }
    for (size_t i = 0; i < pa.size(); ++i) {
        bfa[i] = bf16_bits(pa[i]);
        ha[i] = f16_bits(pa[i]);
    }
    out->m = m;
    out->nf = nf;
    out->nfb = NFB;
    auto up16 = [](const std::vector<uint16_t> &h, void **d) {
        hipError_t e = hipMalloc(d, h.size() * 2);
        if (e == hipSuccess) e = hipMemcpy(*d, h.data(), h.size() * 2, hipMemcpyHostToDevice);
        return e;
    };
    // the weights alpha_i, zero-padded to 64 (energy mode)
    std::vector<float> al(kAlphaFloats, 0.0f);
    for (int f = 0; f < nf && f < kAlphaFloats; ++f) al[f] = alpha[f];
    hipError_t ea = hipMalloc((void **)&out->alpha, al.size() * sizeof(float));
    if (ea == hipSuccess)
        ea = hipMemcpy(out->alpha, al.data(), al.size() * sizeof(float), hipMemcpyHostToDevice);
    if (ea != hipSuccess) return ea;
    hipError_t e16 = up16(bff, &out->bf_fwd);
    if (e16 == hipSuccess) e16 = up16(bfa, &out->bf_adj);
    if (e16 == hipSuccess) e16 = up16(hf, &out->h_fwd);
    if (e16 == hipSuccess) e16 = up16(ha, &out->h_adj);
    if (e16 != hipSuccess) return e16;
    hipError_t e = hipMalloc((void **)&out->fwd, fwd.size() * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&out->adj, adj.size() * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&out->lastf, lastf.size() * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&out->lasta, lasta.size() * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(out->fwd, fwd.data(), fwd.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(out->adj, adj.data(), adj.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(out->lastf, lastf.data(), lastf.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(out->lasta, lasta.data(), lasta.size() * 4, hipMemcpyHostToDevice);
    return e;
}

void fused_release(FusedBank *b)
{
    (void)hipFree(b->fwd);
    (void)hipFree(b->adj);
    (void)hipFree(b->lastf);
    (void)hipFree(b->lasta);
    (void)hipFree(b->bf_fwd);
    (void)hipFree(b->bf_adj);
    (void)hipFree(b->h_fwd);
    (void)hipFree(b->h_adj);
    (void)hipFree(b->alpha);
    b->alpha = nullptr;
    b->fwd = b->adj = b->lastf = b->lasta = nullptr;
    b->bf_fwd = b->bf_adj = b->h_fwd = b->h_adj = nullptr;
}

// Tile shape: columns are fixed by the q-row width (TX = 64 - 2r); the row
// count is chosen to fill the chip: the smallest per-CU work over rounds of
// 256 workgroups, each tile costing ceil((ty + 2r) / nw) pipeline steps.
namespace {
// Cost-model estimate of one tile height for a group (lower is better):
// rounds of 256 workgroups times pipeline steps per tile.
double plan_cost(int m, const AdvanceItem *items, int n, int nw, int ty)
{
    const int R = (m - 1) / 2, TX = kQW - 2 * R;
    const int kCUs = 256;
    long tiles = 0;
    int steps = 0;
    for (int i = 0; i < n; ++i) {
        if (items[i].count <= 0) continue;
        const int ntx = (items[i].job->width + TX - 1) / TX;
        const int nty = (items[i].job->height + ty - 1) / ty;
        tiles += (long)ntx * nty;
        const int th = (items[i].job->height + nty - 1) / nty;
        steps = std::max(steps, (th + 2 * R + nw - 1) / nw);
    }
    const long rounds = (tiles + kCUs - 1) / kCUs;
    return (double)rounds * steps;
}

int rows_any(int m, int nfb, int prec, int nw)
{
#define FE_ROWS(MM, NB) return rows_prec<MM, NB>(prec, nw)
    switch (m * 10 + nfb) {
    case 31: FE_ROWS(3, 1);
    case 32: FE_ROWS(3, 2);
    case 33: FE_ROWS(3, 3);
    case 34: FE_ROWS(3, 4);
    case 51: FE_ROWS(5, 1);
    case 52: FE_ROWS(5, 2);
    case 53: FE_ROWS(5, 3);
    case 54: FE_ROWS(5, 4);
    case 71: FE_ROWS(7, 1);
    case 72: FE_ROWS(7, 2);
    case 73: FE_ROWS(7, 3);
    case 74: FE_ROWS(7, 4);
    default: return 0;
    }
#undef FE_ROWS
}
}  // namespace

// FP32: 12 waves with LDS-resident adjoint tables measured faster than 8
// waves with every operand in registers; both remain for the autotuner.
int default_waves(int prec) { return prec == FE_PREC_FP32 ? kDefaultWavesF32 : kWavesP16; }

// The default when its variant exists for this bank, else the other one.
int bank_default_waves(const FusedBank &bank, int prec)
{
    const int nw = default_waves(prec);
    if (max_tile_rows(bank, prec, nw) > 0) return nw;
    for (int w : wave_options(prec))
        if (max_tile_rows(bank, prec, w) > 0) return w;
    return nw;
}

std::vector<int> wave_options(int prec)
{
    if (prec == FE_PREC_FP32) return {kWavesF32, 12};
    return {kWavesP16};
}

int max_tile_rows(const FusedBank &bank, int prec, int nw)
{
    return rows_any(bank.m, bank.nfb, prec, nw);
}

std::string batch_key(int prec, const AdvanceItem *items, int n)
{
    std::vector<std::pair<int, int>> sz;
    for (int i = 0; i < n; ++i)
        if (items[i].count > 0) sz.emplace_back(items[i].job->height, items[i].job->width);
    std::sort(sz.begin(), sz.end());
    std::string k = "p" + std::to_string(prec) + ":";
    for (auto &hw : sz) k += std::to_string(hw.first) + "x" + std::to_string(hw.second) + ",";
    return k;
}

std::vector<int> tile_candidates(const FusedBank &bank, int prec, const AdvanceItem *items,
                                 int n, int nw, int max_n)
{
    const int hi = max_tile_rows(bank, prec, nw);
    std::vector<std::pair<double, int>> c;
    for (int ty = kMinTileRows; ty <= hi; ++ty)
        c.emplace_back(plan_cost(bank.m, items, n, nw, ty), ty);
    std::stable_sort(c.begin(), c.end(),
                     [](const std::pair<double, int> &a, const std::pair<double, int> &b) {
                         return a.first < b.first;
                     });
    std::vector<int> out;
    for (auto &e : c) {
        if ((int)out.size() >= max_n) break;
        out.push_back(e.second);
    }
    return out;
}

// Tile shape: columns are fixed by the q-row width (TX = 64 - 2r); the row
// count comes from the tuning table if measured, else from the cost model
// (fewest rounds of 256 workgroups times pipeline steps per tile), within
// what the variant's LDS allows.
void make_plan(const FusedBank &bank, int prec, const AdvanceItem *items, int n, Plan *plan,
               int nw, int forced_ty)
{
    const int m = bank.m, R = (m - 1) / 2, TX = kQW - 2 * R;
    const int hi = std::max(kMinTileRows, max_tile_rows(bank, prec, nw));
    int best_ty = forced_ty;
    if (best_ty <= 0) {
        double best = 1e300;
        best_ty = kMinTileRows;
        for (int ty = kMinTileRows; ty <= hi; ++ty) {
            const double cost = plan_cost(m, items, n, nw, ty);
            if (cost < best - 1e-9) {
                best = cost;
                best_ty = ty;
            }
        }
    }
    best_ty = std::min(std::max(best_ty, kMinTileRows), hi);
    plan->tile_w = TX;
    plan->tile_h = best_ty;
    plan->waves = nw;
    plan->njobs = n;
    plan->ntiles = 0;
    plan->jobs_ntx.assign(n, 0);
    plan->jobs_nty.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        if (items[i].count <= 0) continue;   // contributes no tiles
        plan->jobs_ntx[i] = (items[i].job->width + TX - 1) / TX;
        plan->jobs_nty[i] = (items[i].job->height + best_ty - 1) / best_ty;
        plan->ntiles += (long)plan->jobs_ntx[i] * plan->jobs_nty[i];
    }
}

// Waves per workgroup when no measured choice exists.  FP32 runs its
// 12-wave variant where its cost-model tiles take at least kMinSteps12
// pipeline steps, else the 8-wave one: on short tiles (small images spread
// over the CUs) the 12-wave prologue (whole u tile, LDS-resident tables) is
// not amortised (measured on single-image serving: 64 vs 62 images/s).
int plan_waves(const FusedBank &bank, int prec, const AdvanceItem *items, int n)
{
    const int nw = bank_default_waves(bank, prec);
    if (prec != FE_PREC_FP32 || nw != 12 || max_tile_rows(bank, prec, 8) <= 0) return nw;
    Plan p;
    make_plan(bank, prec, items, n, &p, 12, 0);
    return (p.tile_h + bank.m - 1 + 11) / 12 >= kMinSteps12 ? 12 : 8;
}

size_t Plan::device_bytes() const { return (size_t)std::max(njobs, 1) * sizeof(JobDesc); }
size_t fused_table_bytes(int n) { return (size_t)std::max(n, 1) * sizeof(JobDesc); }

hipError_t run_fused(const FusedBank &bank, const AdvanceItem *items, int n, void *plan_ws,
                     hipStream_t s, const TuneTable *tune, int only_prec, TileChoice forced)
{
    // Jobs run in groups of equal precision (one kernel per precision); each
    // group has its own slice of the job table and its own plan.
    JobDesc *table = (JobDesc *)plan_ws;
    int slot = 0;
    for (int prec = FE_PREC_FP32; prec <= FE_PREC_FP16; ++prec) {
        if (only_prec >= 0 && prec != only_prec) continue;
        std::vector<AdvanceItem> grp;
        for (int i = 0; i < n; ++i)
            if (items[i].job->precision == prec && items[i].count > 0) grp.push_back(items[i]);
        if (grp.empty()) continue;
        // Jobs in order of decreasing iteration count: at iteration it the
        // jobs still running are a prefix of the table, and the launch covers
        // just their tiles (no workgroups that return at once, and every XCD
        // gets its share of the running tiles).
        std::stable_sort(grp.begin(), grp.end(), [](const AdvanceItem &a, const AdvanceItem &b) {
            return a.count > b.count;
        });
        const int gn = (int)grp.size();
        Plan plan;
        TileChoice ch = forced;
        if (ch.waves <= 0 && ch.ty <= 0 && tune) ch = tune->lookup(batch_key(prec, grp.data(), gn));
        if (ch.waves <= 0 || max_tile_rows(bank, prec, ch.waves) <= 0)
            ch.waves = plan_waves(bank, prec, grp.data(), gn);
        make_plan(bank, prec, grp.data(), gn, &plan, ch.waves, ch.ty);
        if (plan.ntiles > INT_MAX) return hipErrorInvalidValue;   // tile indices are ints
        JobDesc *dj = table + slot;
        slot += gn;
        int max_it = 0, base = 0;
        std::vector<long> first_tile(gn + 1, 0);   // tile_base of job i; [gn] = all tiles
        for (int c0 = 0; c0 < gn; c0 += kChunk) {
            JobChunk jc{};
            jc.first = c0;
            jc.count = std::min(kChunk, gn - c0);
            for (int i = 0; i < jc.count; ++i) {
                const AdvanceItem &it = grp[c0 + i];
                const fe_job &j = *it.job;
                JobDesc &d = jc.d[i];
                const size_t plane = (size_t)j.height * j.width;
                d.counts = j.counts;
                d.ua = it.state;
                d.ub = it.state + plane;
                d.H = j.height;
                d.W = j.width;
                d.ntx = plan.jobs_ntx[c0 + i];
                d.nty = plan.jobs_nty[c0 + i];
                d.tile_base = base;
                base += d.ntx * d.nty;
                first_tile[c0 + i + 1] = base;
                d.iters = it.count;
                d.it0 = it.done;
                d.tau = j.tau;
                d.gamma = j.gamma;
                d.tl = j.tau * j.lambda;
                d.q1 = (float)(1.0 / (1.0 + (double)d.tl));
                d.data_term = j.data_term == FE_DATA_AUTO
                                  ? (j.peak >= 5.0f ? FE_DATA_QUADRATIC : FE_DATA_IDIV)
                                  : j.data_term;
                max_it = std::max(max_it, d.iters);
            }
            write_jobs_kernel<<<1, kChunk, 0, s>>>(jc, dj);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        // Iteration it runs the jobs [0, k) with count > it, tiles
        // [0, first_tile[k]); a launch covers at most kMaxLaunchTiles
        // workgroups (its work-item count stays below 2^31).
        int k = gn;
        for (int it = 0; it < max_it; ++it) {
            while (k > 0 && grp[k - 1].count <= it) --k;
            const long active = first_tile[k];
            for (long t0 = 0; t0 < active; t0 += kMaxLaunchTiles) {
                const int nb = (int)std::min<long>(kMaxLaunchTiles, active - t0);
                hipError_t e = launch_any(prec, plan.waves, bank, dj, gn, nb, (int)t0, it,
                                          plan.tile_h, s);
                if (e != hipSuccess) return e;
            }
        }
    }
    return hipSuccess;
}

// ---- gradient and energy (eq. 3.2, 2.5) ------------------------------------
// One launch of the fused kernel in a gradient mode over every tile of every
// image of a batch.  Workspace: [job table][2 floats per tile][one double
// per image].
namespace {
size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
long grad_tiles_max(const FusedBank &bank, const GradItem *items, int n)
{
    const int R = (bank.m - 1) / 2, TX = kQW - 2 * R;
    long t = 0;
    for (int i = 0; i < n; ++i)
        t += (long)((items[i].width + TX - 1) / TX) *
             ((items[i].height + kMinTileRows - 1) / kMinTileRows);
    return t;
}
size_t grad_part_offset(int n) { return al256(fused_table_bytes(n)); }
size_t grad_energy_offset(const FusedBank &bank, const GradItem *items, int n)
{
    return grad_part_offset(n) + al256(2 * sizeof(float) * (size_t)grad_tiles_max(bank, items, n));
}

// Energy of each image of a gradient-mode launch: block j sums image j's
// workgroup partials, E_j = sum of prior partials + lambda_j * sum of data
// partials, in FP64, every thread over a fixed stride of the image's tiles,
// then a fixed tree (deterministic).
__global__ __launch_bounds__(256) void energy_finish_kernel(const JobDesc *__restrict__ jobs,
                                                            const float *__restrict__ epart,
                                                            double *__restrict__ out)
{
    __shared__ double sp[256], sd[256];
    const JobDesc J = jobs[blockIdx.x];
    const long t0 = J.tile_base, nt = (long)J.ntx * J.nty;
    double a = 0.0, b = 0.0;
    for (long t = threadIdx.x; t < nt; t += 256) {
        a += (double)epart[2 * (t0 + t)];
        b += (double)epart[2 * (t0 + t) + 1];
    }
    sp[threadIdx.x] = a;
    sd[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sp[threadIdx.x] += sp[threadIdx.x + w];
            sd[threadIdx.x] += sd[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sp[0] + (double)J.lambda * sd[0];
}
}  // namespace

size_t grad_workspace_bytes(const FusedBank &bank, const GradItem *items, int n)
{
    return grad_energy_offset(bank, items, n) + al256(sizeof(double) * (size_t)std::max(n, 1));
}

hipError_t run_grad(const FusedBank &bank, const GradItem *items, int n, int prec, bool energy,
                    void *ws, double **energy_dev, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int m = bank.m, R = (m - 1) / 2, TX = kQW - 2 * R;
    const int nw = prec == FE_PREC_FP32 ? kWavesF32
                   : energy               ? kWavesP16Energy
                                          : kWavesP16;
    // tile height: the cost model's choice within the mode's LDS limit
    std::vector<fe_job> jj(n);
    std::vector<AdvanceItem> adv(n);
    for (int i = 0; i < n; ++i) {
        jj[i] = fe_job{};
        jj[i].height = items[i].height;
        jj[i].width = items[i].width;
        jj[i].precision = prec;
        adv[i] = AdvanceItem{&jj[i], nullptr, 0, 1};
    }
    const int hi = std::max(kMinTileRows, rows_grad_any(m, bank.nfb, prec, energy));
    int ty = kMinTileRows;
    double best = 1e300;
    for (int t = kMinTileRows; t <= hi; ++t) {
        const double c = plan_cost(m, adv.data(), n, nw, t);
        if (c < best - 1e-9) {
            best = c;
            ty = t;
        }
    }
    char *w = (char *)ws;
    JobDesc *table = (JobDesc *)w;
    float *epart = (float *)(w + grad_part_offset(n));
    double *edev = (double *)(w + grad_energy_offset(bank, items, n));
    long base = 0;
    for (int c0 = 0; c0 < n; c0 += kChunk) {
        JobChunk jc{};
        jc.first = c0;
        jc.count = std::min(kChunk, n - c0);
        for (int i = 0; i < jc.count; ++i) {
            const GradItem &it = items[c0 + i];
            JobDesc &d = jc.d[i];
            d.counts = it.counts;
            d.ua = const_cast<float *>(it.u);   // read only: the gradient modes write ub
            d.ub = it.grad;
            d.H = it.height;
            d.W = it.width;
            d.ntx = (it.width + TX - 1) / TX;
            d.nty = (it.height + ty - 1) / ty;
            d.tile_base = (int)base;
            base += (long)d.ntx * d.nty;
            d.iters = 1;
            d.it0 = 0;
            d.lambda = it.lambda;
            d.data_term = it.data_term;
            if (base > INT_MAX) return hipErrorInvalidValue;   // tile indices are ints
        }
        write_jobs_kernel<<<1, kChunk, 0, s>>>(jc, table);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (base > grad_tiles_max(bank, items, n)) return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    for (long t0 = 0; t0 < base && e == hipSuccess; t0 += kMaxLaunchTiles) {
        const int nb = (int)std::min<long>(kMaxLaunchTiles, base - t0);
        e = launch_grad_any(prec, energy, bank, table, n, nb, (int)t0, ty, epart, s);
    }
    if (e == hipSuccess && energy) {
        energy_finish_kernel<<<n, 256, 0, s>>>(table, epart, edev);
        e = hipGetLastError();
    }
    if (energy_dev) *energy_dev = edev;
    return e;
}

}  // namespace fe
