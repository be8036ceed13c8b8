// HIP kernels (gfx950) for the matrix-free product H(t)|psi> of Sec. II.A and
// the integrator stages of Sec. II.B, with float64 reductions.
//
// Tile passes.  A workgroup holds a tile of 2^tb amplitudes of the source
// vector u in LDS: `lbits` contiguous low bits (coalesced 16-byte loads) plus
// the high bits in `hmask`.  Every flip pattern x whose bits all lie in the
// tile is applied from LDS: (H u)[g] += c_x(g) u[g ^ x].  Flip patterns with
// bits above the last pass's tile are handled by earlier passes (register
// hypercube passes for single-qubit flips, tile passes whose tiles include the
// pattern's bits) that write a partial product the last pass reads, or by the
// last pass itself reading the partner u[g ^ x] from memory (stream groups).
// The last pass tiles the low tb bits contiguously, adds the diagonal from
// split tables (popcount parity folded per tile), and fuses the integrator's
// stage update (a fixed linear combination of H u with up to four streamed
// vectors and u itself).
#include <hip/hip_runtime.h>


#include "aqc_internal.h"

namespace aqc {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// Streaming (non-temporal) access for vectors that are touched once per pass.
// a * b + c with one rounding
__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ float2 ldnt(const float2* p) {
  const f32x2 e = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(p));
  return float2{e.x, e.y};
}
__device__ __forceinline__ double2 ldnt(const double2* p) {
  const f64x2 e = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p));
  return double2{e.x, e.y};
}
__device__ __forceinline__ void stnt(float2* p, float2 v) {
  __builtin_nontemporal_store(f32x2{v.x, v.y}, reinterpret_cast<f32x2*>(p));
}
__device__ __forceinline__ void stnt(double2* p, double2 v) {
  __builtin_nontemporal_store(f64x2{v.x, v.y}, reinterpret_cast<f64x2*>(p));
}

// The low part of a compensated complex64 state is stored as a pair of
// bfloat16 (4 bytes per amplitude): it is the rounding residual of the float32
// high part, so 8 mantissa bits leave an error of 2^-9 of a residual per step.
__device__ __forceinline__ uint32_t bf16_bits(float f) {  // round to nearest even
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ uint32_t pack_bf16x2(float re, float im) {
  return bf16_bits(re) | (bf16_bits(im) << 16);
}
__device__ __forceinline__ float bf16_lo(uint32_t p) { return __uint_as_float(p << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t p) { return __uint_as_float(p & 0xFFFF0000u); }

template <typename R> struct CT2;
template <> struct CT2<float> { using V = float2; };
template <> struct CT2<double> { using V = double2; };

// Deposit the low bits of v into the set bits of mask (ascending order).
__device__ __forceinline__ uint64_t pdep64(uint64_t v, uint64_t mask) {
  uint64_t r = 0;
  while (mask) {
    const uint64_t low = mask & (~mask + 1ull);
    if (v & 1ull) r |= low;
    v >>= 1;
    mask &= mask - 1ull;
  }
  return r;
}

// The bits of mask above its k lowest set bits.
__device__ __forceinline__ uint64_t mask_above(uint64_t mask, int k) {
  for (int i = 0; i < k && mask; ++i) mask &= mask - 1ull;
  return mask;
}

// Successor of x among the subsets of m in increasing order: pdep(j + 1, m)
// from pdep(j, m) in three operations.
__device__ __forceinline__ uint64_t next_subset(uint64_t x, uint64_t m) {
  return ((x | ~m) + 1ull) & m;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order block reduction of up to 3 values; thread 0 writes parts.
template <int NT>
__device__ __forceinline__ void block_reduce3(double r0, double r1, double r2, int flags,
                                              double* sbuf, double* parts, int64_t nblocks,
                                              int64_t bid) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  constexpr int NW = NT / 64;
  if (flags & 1) r0 = wave_sum(r0);
  if (flags & 2) r1 = wave_sum(r1);
  if (flags & 4) r2 = wave_sum(r2);
  if (lane == 0) {
    sbuf[0 * NW + wv] = r0;
    sbuf[1 * NW + wv] = r1;
    sbuf[2 * NW + wv] = r2;
  }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int w = 0; w < NW; ++w) {
      s0 += sbuf[0 * NW + w];
      s1 += sbuf[1 * NW + w];
      s2 += sbuf[2 * NW + w];
    }
    if (flags & 1) parts[0 * nblocks + bid] = s0;
    if (flags & 2) parts[1 * nblocks + bid] = s1;
    if (flags & 4) parts[2 * nblocks + bid] = s2;
  }
}

// LDS layout of a tile workgroup (offsets in bytes, 16-byte aligned pieces).
struct Lds {
  static constexpr int kF = 0;                                   // double f[kMaxSched]
  static constexpr int kLin = kF + 8 * kMaxSched;                // double lin[16]
  static constexpr int kC = kLin + 8 * 16;                       // double C'
  static constexpr int kRed = kC + 16;                           // double [3][NW]
  static constexpr int kLA = kRed + 8 * 3 * (kThreads / 64);     // double LA[128]
  static constexpr int kLB = kLA + 8 * 128;                      // double LB[128]
  static constexpr int kGco = kLB + 8 * 128;                     // R gco[kMaxPassGroups]
  static constexpr int kGxl = kGco + 8 * kMaxPassGroups;         // u32 gxl[kMaxPassGroups]
  static constexpr int kGfl = kGxl + 4 * kMaxPassGroups;         // u32 gfl[kMaxPassGroups]
  static constexpr int kTm = kGfl + 4 * kMaxPassGroups;          // R tm[kMaxPassTerms]
  static constexpr int kTmd = kTm + 8 * kMaxPassTerms;           // double tmd[kMaxPassTerms]
  static constexpr int kTile = kTmd + 8 * kMaxPassTerms;         // V tile[2^tb]
};

size_t pass_lds_bytes(int tb, int dtype) {
  const size_t es = dtype == 0 ? 8 : 16;
  return (size_t)Lds::kTile + (es << tb);
}

// Per-tile diagonal set-up (hi = the tile's high bits): C' and the linear
// coefficients, then the two sign tables LA (bits 0..6) and LB (bits 7..tb-1).
template <typename R>
__device__ __forceinline__ void diag_setup_a(const PassArgs& a, uint64_t hi, const double* fsh,
                                             double* lin, double* cp) {
  const int tid = threadIdx.x;
  const int tb = a.tb;
  const int64_t nhi = (int64_t)1 << (a.n - tb);
  // the first four schedules unrolled (their loads issued together); more
  // schedules (a clause-by-clause path has one per clause) in a loop
  constexpr int kUnrolled = 4;
  if (tid < tb) {
    double v = 0.0;
#pragma unroll
    for (int s = 0; s < kUnrolled; ++s) {
      if (s < a.dg.nsd) v += fsh[a.dg.sd_sid[s]] * a.dg.LT[((int64_t)s * nhi + (int64_t)hi) * tb + tid];
    }
    for (int s = kUnrolled; s < a.dg.nsd; ++s)
      v += fsh[a.dg.sd_sid[s]] * a.dg.LT[((int64_t)s * nhi + (int64_t)hi) * tb + tid];
    lin[tid] = v;
  }
  if (tid == 64) {
    double c = a.dconst;
#pragma unroll
    for (int s = 0; s < kUnrolled; ++s) {
      if (s < a.dg.nsd) c += fsh[a.dg.sd_sid[s]] * a.dg.CT[(int64_t)s * nhi + (int64_t)hi];
    }
    for (int s = kUnrolled; s < a.dg.nsd; ++s)
      c += fsh[a.dg.sd_sid[s]] * a.dg.CT[(int64_t)s * nhi + (int64_t)hi];
    *cp = c;
  }
}

__device__ __forceinline__ void diag_setup_b(const PassArgs& a, const double* lin, double* LA, double* LB) {
  const int tid = threadIdx.x;
  const int tb = a.tb;
  const int na = tb < 7 ? tb : 7;
  const int nb = tb > 7 ? tb - 7 : 0;
  if (tid < 128) {
    double v = 0.0;
    if (tid < (1 << na)) {
      for (int i = 0; i < na; ++i) v += ((tid >> i) & 1) ? -lin[i] : lin[i];
    }
    LA[tid] = v;
  } else if (tid < 256) {
    const int b = tid - 128;
    double v = 0.0;
    if (b < (1 << nb)) {
      for (int i = 0; i < nb; ++i) v += ((b >> i) & 1) ? -lin[7 + i] : lin[7 + i];
    }
    LB[b] = v;
  }
}

// Diagonal energy of the tile element with low bits lo and global index g,
// always in float64 (a handful of adds per amplitude): the per-tile constant
// and the sign tables nearly cancel for a centred shift, so summing them in
// float32 would put a rounding error of the size of the spectrum into every
// diagonal value.
__device__ __forceinline__ double diag_value(const PassArgs& a, uint32_t lo, uint64_t g, double cprime,
                                             const double* LA, const double* LB, const double* fsh) {
  double d = cprime + LA[lo & 127u] + LB[lo >> 7];
  const int64_t ntile = (int64_t)1 << a.tb;
  // one table read per schedule: the first few unrolled, the rest (a path
  // with a schedule per clause) in a loop
  constexpr int kTabUnrolled = 4;
#pragma unroll
  for (int s = 0; s < kTabUnrolled; ++s) {
    if (s < a.dg.ntab) d += fsh[a.dg.tab_sid[s]] * a.dg.TAB64[(int64_t)s * ntile + lo];
  }
#pragma unroll 1
  for (int s = kTabUnrolled; s < a.dg.ntab; ++s) {
    const double* tab = a.dg.TAB64 + (int64_t)s * ntile;   // uniform
    d += fsh[a.dg.tab_sid[s]] * tab[lo];
  }
  for (int k = 0; k < a.dg.nres; ++k) {
    const DevTerm t = a.dg.res[k];
    const double m = t.w * fsh[t.sid];
    d += (__popcll(g & t.z) & 1) ? -m : m;
  }
  return d;
}

template <typename R, bool FINAL>
__device__ __forceinline__ void pass_body(const PassArgs& a, const int64_t bid, const int64_t nblocks,
                                          unsigned char* smem) {
  using V = typename CT2<R>::V;
  double* fsh = reinterpret_cast<double*>(smem + Lds::kF);
  double* lin = reinterpret_cast<double*>(smem + Lds::kLin);
  double* cps = reinterpret_cast<double*>(smem + Lds::kC);
  double* rbuf = reinterpret_cast<double*>(smem + Lds::kRed);
  double* LA = reinterpret_cast<double*>(smem + Lds::kLA);
  double* LB = reinterpret_cast<double*>(smem + Lds::kLB);
  R* gco = reinterpret_cast<R*>(smem + Lds::kGco);
  uint32_t* gxl = reinterpret_cast<uint32_t*>(smem + Lds::kGxl);
  // per group: fslot + 1 (0: not a fast group) | li << 8 | lj << 16, so that
  // the product loop finds a fast group's table without reading its
  // descriptor from memory (a vector load, whose wait would also wait for
  // the stores the pass has issued: one counter covers both)
  uint32_t* gfl = reinterpret_cast<uint32_t*>(smem + Lds::kGfl);
  R* tm = reinterpret_cast<R*>(smem + Lds::kTm);
  V* tile = reinterpret_cast<V*>(smem + Lds::kTile);

  double* tmd = reinterpret_cast<double*>(smem + Lds::kTmd);
  static_assert(kMaxPassGroups <= kThreads && kMaxPassTerms <= kThreads,
                "one group and one term per thread in the set-up");

  const int tid = threadIdx.x;
  const int tb = a.tb;
  const uint32_t ntile = 1u << tb;
  const uint64_t lowmask = (1ull << a.lbits) - 1ull;
  const uint64_t tmask = lowmask | a.hmask;
  const uint64_t base = FINAL ? ((uint64_t)bid << tb) : pdep64((uint64_t)bid, a.cmask);
  const uint32_t E = ntile >= (uint32_t)kThreads ? ntile / kThreads : 1u;
  const uint64_t edep_tid = FINAL ? (uint64_t)tid : pdep64((uint64_t)tid, tmask);
  const V* accin = reinterpret_cast<const V*>(a.acc_in);
  V* accout = reinterpret_cast<V*>(a.acc_out);

  // ---- 1. every global read of the set-up is issued before the first wait:
  // the tile (16-byte chunks), the high pass's partial product, the group and
  // term descriptors and the diagonal's per-tile tables, so their latencies
  // overlap instead of adding up
  constexpr int VEC = 16 / (int)sizeof(V);            // elements per chunk
  constexpr int LOGV = VEC == 2 ? 1 : 0;
  // chunks per thread held in registers: all of a 2^14 complex64 tile, half of
  // a 2^13 complex128 tile (the rest is loaded after the first commit)
  constexpr int MAXC = sizeof(R) == 4 ? 16 : 8;
  const uint32_t nchunks = ntile / VEC;
  const int cpt = (int)(nchunks / kThreads);          // 0: tile smaller than one chunk per thread
  const V* src = reinterpret_cast<const V*>(a.src);
  // local element l = q*VEC with q = tid + kThreads*j: the tid part and the j
  // part occupy disjoint bits of l, so their deposits can be OR-ed.
  const uint64_t dep_tid = FINAL ? ((uint64_t)tid << LOGV) : pdep64((uint64_t)tid << LOGV, tmask);
  // chunk j sits at pdep((kThreads j) << LOGV, tmask), element j at
  // pdep(kThreads j, tmask): successive subsets of the tile mask above its
  // lowest 9 + LOGV (9) bits, enumerated incrementally (uniform, scalar)
  static_assert(kThreads == 512, "offset enumeration assumes 2^9 threads");
  const uint64_t cmask_hi = mask_above(tmask, 9 + LOGV);
  const uint64_t emask_hi = mask_above(tmask, 9);
  // (the last pass's tile is contiguous: constant offsets)
  u32x4 tv[MAXC];
  uint64_t co = 0;
#pragma unroll
  for (int j = 0; j < MAXC; ++j) {
    if (j < cpt) {
      if constexpr (FINAL) {
        const uint64_t jpart = (uint64_t)(kThreads * j) << LOGV;
        tv[j] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(src + (base | dep_tid | jpart)));
      } else {
        tv[j] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(src + (base | dep_tid | co)));
        co = next_subset(co, cmask_hi);
      }
    }
  }
  if (cpt == 0 && (uint32_t)tid < nchunks) tv[0] = *reinterpret_cast<const u32x4*>(src + (base | dep_tid));
  // high passes: the partial product of the first elements, all of them
  // for a complex64 tile of 2^13, so no load waits behind the pass's stores
  // (loads and stores share one counter); complex128 half a block
  constexpr int PF = FINAL ? 1 : (sizeof(R) == 4 ? 16 : 4);
  V apf[PF];
  {
    uint64_t eo = 0;
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      apf[j] = V{0, 0};
      if (!FINAL && accin && (uint32_t)j < E && tid + kThreads * j < ntile)
        apf[j] = ldnt(accin + (base | edep_tid | eo));
      eo = next_subset(eo, emask_hi);
    }
  }
  const bool hasg = tid < a.ng, hast = tid < a.nterms;
  DevGroup gr{};
  DevTerm tt{};
  if (hasg) gr = a.groups[tid];
  if (hast) tt = a.terms[tid];
  if (FINAL) diag_setup_a<R>(a, (uint64_t)bid, a.f, lin, cps);

  // ---- 2. the tile into LDS; per-workgroup coefficients --------------------
#pragma unroll
  for (int j = 0; j < MAXC; ++j)
    if (j < cpt) *reinterpret_cast<u32x4*>(tile + (tid + kThreads * j) * VEC) = tv[j];
  if (cpt == 0 && (uint32_t)tid < nchunks) *reinterpret_cast<u32x4*>(tile + tid * VEC) = tv[0];
  for (int j = MAXC; j < cpt; ++j) {
    const uint64_t off = FINAL ? ((uint64_t)(kThreads * j) << LOGV) : co;
    *reinterpret_cast<u32x4*>(tile + (tid + kThreads * j) * VEC) =
        __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(src + (base | dep_tid | off)));
    co = next_subset(co, cmask_hi);
  }
  if (tid < kMaxSched) fsh[tid] = a.f[tid];
  __syncthreads();
  if (hast) {
    const double v = tt.w * fsh[tt.sid];
    tmd[tid] = v;
    tm[tid] = (R)v;
  }
  __syncthreads();
  // fast groups: c_x as a function of the source's bits (bi, bj), entry
  // sb_i + 2 sb_j, from the per-term values (written over them below)
  double fv[8];
  const bool isfast = hasg && gr.fslot >= 0;
  if (hasg) {
    double c = 0.0;
    if (gr.plain)
      for (int t = 0; t < gr.nt; ++t) c += tmd[gr.t0 + t];
    gco[tid] = (R)c;
    // tile-local flip mask; bit 31 marks a group whose coefficient depends on
    // g, bit 30 one whose partner lies outside the tile (read from memory)
    gxl[tid] = gr.xl | (gr.plain ? 0u : 0x80000000u) | ((gr.x & ~tmask) ? 0x40000000u : 0u);
    gfl[tid] = (uint32_t)(gr.fslot + 1) | ((uint32_t)gr.lij << 8);
  }
  if (isfast) {
    const int bi = gr.bij & 255, bj = gr.bij >> 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) fv[q] = 0.0;
    for (int t = 0; t < gr.nt; ++t) {
      const DevTerm ft = a.terms[gr.t0 + t];
      const double m = tmd[gr.t0 + t];
      const int hi_ = (int)((ft.z >> bi) & 1ull), hj = bj != bi ? (int)((ft.z >> bj) & 1ull) : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int par = ((q & 1) & hi_) ^ ((q >> 1) & hj);
        const double v = par ? -m : m;
        switch (ft.p & 3) {
          case 0: fv[2 * q] += v; break;
          case 1: fv[2 * q + 1] += v; break;
          case 2: fv[2 * q] -= v; break;
          default: fv[2 * q + 1] -= v; break;
        }
      }
    }
  }
  if (FINAL) diag_setup_b(a, lin, LA, LB);
  __syncthreads();
  R* ftab = reinterpret_cast<R*>(tmd);   // per-term float64 values are dead now
  if (isfast) {
#pragma unroll
    for (int q = 0; q < 8; ++q) ftab[8 * gr.fslot + q] = (R)fv[q];
  }
  __syncthreads();

  // ---- 3. products and epilogue --------------------------------------------
  // a tile smaller than the workgroup: the threads past it stand in for one
  // inside (their results are dropped)
  const uint32_t tidc = ntile >= (uint32_t)kThreads ? (uint32_t)tid : ((uint32_t)tid & (ntile - 1u));
  const double cprime = FINAL ? cps[0] : 0.0;
  const EpiDesc& e = a.epi;
  const bool has_comp = FINAL && e.comp != nullptr;
  uint32_t* compv = reinterpret_cast<uint32_t*>(e.comp);   // bfloat16 pairs
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;
  // Elements are processed in blocks of EB: H u for the whole block is kept in
  // registers while the flip groups are walked once (group-outer order), then
  // the stage update streams the block's other vectors in batches of U.
  // High passes (E <= 32) unroll their NJB blocks so the prefetched partial
  // product is indexed at compile time.
  constexpr int EB = FINAL ? 4 : 8;
  constexpr int NJB = FINAL ? 1 : 4;
  // elements per batch of the stage update (streamed loads in flight)
  constexpr int U = sizeof(R) == 4 ? 4 : 2;
  uint64_t eo_run = 0;   // offset of element jb (blocks run in ascending order)
  for (uint32_t jb0 = 0; jb0 < E; jb0 += EB * NJB) {
#pragma unroll
  for (int qb = 0; qb < NJB; ++qb) {
    const uint32_t jb = jb0 + qb * EB;
    if (jb >= E) break;
    // high passes: offsets of the block's elements, enumerated in order
    uint64_t eou[FINAL ? 1 : EB];
    if constexpr (!FINAL) {
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        eou[u] = eo_run;
        eo_run = next_subset(eo_run, emask_hi);
      }
    }
    // complex64: hr/hi sum the flip groups only; their terms are small next
    // to the diagonal term, which the last pass adds in float64 at the end, so
    // the float32 partial sums never carry the diagonal's magnitude.
    // complex128 starts the sums with the diagonal term.
    constexpr bool kDiagLate = sizeof(R) == 4;
    // element u of the block: tile index tid + kThreads (jb + u); its global
    // index and tile value are recomputed / re-read from LDS where needed
    // rather than held in registers.  An element past the tile (small tiles
    // only: ok[u] false) is computed as element min(jb + u, E - 1) of thread
    // tidc, so that the products run without per-element branches and every
    // index they read lies inside the tile and the state; its results are
    // dropped.
    auto jc_of = [&](int u) -> uint32_t { return min(jb + (uint32_t)u, E - 1u); };
    auto gidx_of = [&](int u) -> uint64_t {
      if constexpr (FINAL) return base | (uint64_t)tidc | ((uint64_t)kThreads * jc_of(u));
      else return base | edep_tid | eou[u];
    };
    auto tile_of = [&](int u) -> V { return tile[tidc + kThreads * jc_of(u)]; };
    R hr[EB], hi[EB];
    bool ok[EB];
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const uint32_t j = jb + u;
      const uint32_t l = tid + kThreads * j;
      ok[u] = (j < E) && (l < ntile);
      hr[u] = 0;
      hi[u] = 0;
      if (!FINAL && ok[u] && accin) {
        // jb0 == 0 whenever E <= EB * NJB, so qb * EB + u is the element index
        const int jc = qb * EB + u;
        const V av = (jc < PF && jb0 == 0) ? apf[jc < PF ? jc : 0] : ldnt(accin + gidx_of(u));
        hr[u] = av.x;
        hi[u] = av.y;
      }
    }
    if (FINAL && !kDiagLate) {
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        if (!ok[u]) continue;
        const uint32_t l = tid + kThreads * (jb + u);
        const double d = diag_value(a, l, gidx_of(u), cprime, LA, LB, fsh);
        const V uu = tile_of(u);
        hr[u] = (R)(d * (double)uu.x);
        hi[u] = (R)(d * (double)uu.y);
      }
    }
    for (int k = 0; k < a.ng; ++k) {
      const uint32_t gx = gxl[k];
      if (gx & 0x40000000u) {
        // partner outside the tile: a second coalesced stream of the source
        // (the tiles of other workgroups, mostly served from cache)
        const DevGroup gr = a.groups[k];
        V pv[EB];
#pragma unroll
        for (int u = 0; u < EB; ++u) pv[u] = src[gidx_of(u) ^ gr.x];
        if (!(gx >> 31)) {
          const R c = gco[k];
#pragma unroll
          for (int u = 0; u < EB; ++u) {
            hr[u] += c * pv[u].x;
            hi[u] += c * pv[u].y;
          }
        } else if (gr.fslot >= 0) {
          const int bi = gr.bij & 255, bj = gr.bij >> 8;
          const R* fc = ftab + 8 * gr.fslot;
#pragma unroll
          for (int u = 0; u < EB; ++u) {
            const uint64_t src_idx = gidx_of(u) ^ gr.x;
            const int q = 2 * ((int)((src_idx >> bi) & 1ull) | ((int)((src_idx >> bj) & 1ull) << 1));
            const R cr = fc[q], ci = fc[q + 1];
            hr[u] = fma_r(cr, pv[u].x, fma_r(-ci, pv[u].y, hr[u]));
            hi[u] = fma_r(cr, pv[u].y, fma_r(ci, pv[u].x, hi[u]));
          }
        } else {
#pragma unroll
          for (int u = 0; u < EB; ++u) {
            const uint64_t src_idx = gidx_of(u) ^ gr.x;
            R cr = 0, ci = 0;
            for (int t = 0; t < gr.nt; ++t) {
              const DevTerm tt = a.terms[gr.t0 + t];
              R m = tm[gr.t0 + t];
              if (__popcll(src_idx & tt.z) & 1) m = -m;
              switch (tt.p & 3) {
                case 0: cr += m; break;
                case 1: ci += m; break;
                case 2: cr -= m; break;
                default: ci -= m; break;
              }
            }
            hr[u] = fma_r(cr, pv[u].x, fma_r(-ci, pv[u].y, hr[u]));
            hi[u] = fma_r(cr, pv[u].y, fma_r(ci, pv[u].x, hi[u]));
          }
        }
        continue;
      }
      // The tile index of element u is l = tid | (jb + u) << 9 (2^9 threads),
      // so its partner's, l ^ xl, splits into a part fixed per thread, tid ^
      // (xl's low 9 bits), and a part shared by the wave, (jb + u) ^ (xl >> 9):
      // per element one OR forms the address.
      constexpr int kTidBits = 9;
      if (!(gx >> 31)) {
        const R c = gco[k];
        const uint32_t at = tidc ^ (gx & (kThreads - 1u));
#pragma unroll
        for (int u = 0; u < EB; ++u) {
          const uint32_t jx = jc_of(u) ^ (gx >> kTidBits);
          const V v = tile[at | (jx << kTidBits)];
          hr[u] += c * v.x;
          hi[u] += c * v.y;
        }
      } else {
        const uint32_t fl = gfl[k];
        if (fl & 255u) {
          // the table entry is 2 (s_i + 2 s_j) for the source's bits s_i, s_j,
          // bits li, lj of the partner's tile index
          const uint32_t li = (fl >> 8) & 255u, lj = (fl >> 16) & 255u;
          const uint32_t xl = gx & 0x3fffffffu;
          const uint32_t at = tidc ^ (xl & (kThreads - 1u));
          const R* fc = ftab + 8 * (int)((fl & 255u) - 1u);
#pragma unroll
          for (int u = 0; u < EB; ++u) {
            const uint32_t sl = at | ((jc_of(u) ^ (xl >> kTidBits)) << kTidBits);
            const uint32_t q = 2u * (__builtin_amdgcn_ubfe(sl, li, 1) | (__builtin_amdgcn_ubfe(sl, lj, 1) << 1));
            const R cr = fc[q], ci = fc[q + 1];
            const V v = tile[sl];
            hr[u] = fma_r(cr, v.x, fma_r(-ci, v.y, hr[u]));
            hi[u] = fma_r(cr, v.y, fma_r(ci, v.x, hi[u]));
          }
          continue;
        }
        const DevGroup gr = a.groups[k];   // a group whose terms are summed per element
#pragma unroll
        for (int u = 0; u < EB; ++u) {
          const uint32_t l = tidc + kThreads * jc_of(u);
          const uint64_t src_idx = gidx_of(u) ^ gr.x;
          R cr = 0, ci = 0;
          for (int t = 0; t < gr.nt; ++t) {
            const DevTerm tt = a.terms[gr.t0 + t];
            R m = tm[gr.t0 + t];
            if (__popcll(src_idx & tt.z) & 1) m = -m;
            switch (tt.p & 3) {
              case 0: cr += m; break;
              case 1: ci += m; break;
              case 2: cr -= m; break;
              default: ci -= m; break;
            }
          }
          const V v = tile[l ^ gr.xl];
          hr[u] = fma_r(cr, v.x, fma_r(-ci, v.y, hr[u]));
          hi[u] = fma_r(cr, v.y, fma_r(ci, v.x, hi[u]));
        }
      }
    }
    if (!FINAL) {
#pragma unroll
      for (int u = 0; u < EB; ++u)
        if (ok[u]) stnt(accout + gidx_of(u), V{hr[u], hi[u]});
      continue;
    }
#pragma unroll
    for (int u0 = 0; u0 < EB; u0 += U) {
      // every element's loads are issued before any is used (an element past
      // the tile reads its stand-in's values, which are inside the state; its
      // results are dropped), and the low part is unpacked where it is used,
      // so that no element's loads wait for an earlier element's
      V ain[U], xin[U][4];
      uint32_t lop[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint64_t gq = gidx_of(u0 + u);
        ain[u] = accin ? ldnt(accin + gq) : V{0, 0};
#pragma unroll
        for (int i = 0; i < 4; ++i)
          xin[u][i] = e.in[i] ? ldnt(reinterpret_cast<const V*>(e.in[i]) + gq) : V{0, 0};
        lop[u] = has_comp ? __builtin_nontemporal_load(compv + gq) : 0u;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = u0 + u;
        if (!ok[q]) continue;
        const V lo_u = V{(R)bf16_lo(lop[u]), (R)bf16_hi(lop[u])};
        const uint64_t g = gidx_of(q);
        const V uq = tile_of(q);
        // H u = diagonal term + flip sum + partial product of the high passes,
        // the (large) diagonal term added in float64 with one rounding
        R hrr = hr[q] + ain[u].x, hii = hi[q] + ain[u].y;
        if (kDiagLate) {
          const uint32_t l = tid + kThreads * (jb + q);
          const double d = diag_value(a, l, g, cprime, LA, LB, fsh);
          hrr = (R)(d * (double)uq.x + (double)hrr);
          hii = (R)(d * (double)uq.y + (double)hii);
        }
#pragma unroll
        for (int o = 0; o < 3; ++o) {
          if (!e.out[o]) continue;
          R ir = (R)e.br[o] * hrr - (R)e.bi[o] * hii;
          R ii = (R)e.br[o] * hii + (R)e.bi[o] * hrr;
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            ir += (R)e.a[o][i] * xin[u][i + 1].x;
            ii += (R)e.a[o][i] * xin[u][i + 1].y;
          }
          // increment: scale * (sum a x + b Hv), scale as a float-float pair
          const R shh = (R)e.scale[o], sll = (R)(e.scale[o] - (double)shh);
          R vr = shh * ir + sll * ir;
          R vi = shh * ii + sll * ii;
          if (e.comp_flags & (1 << o)) {
            vr += lo_u.x;
            vi += lo_u.y;
          }
          const R bre = (R)e.c0[o] * xin[u][0].x + (R)e.cu[o] * uq.x;
          const R bim = (R)e.c0[o] * xin[u][0].y + (R)e.cu[o] * uq.y;
          const R sr = bre + vr, si = bim + vi;
          if (o == 0 && (e.comp_flags & 8)) {
            // two-sum: the rounding error of bre + vr goes to the low part
            const R tr = sr - bre, ti = si - bim;
            const R er = (bre - (sr - tr)) + (vr - tr);
            const R ei = (bim - (si - ti)) + (vi - ti);
            __builtin_nontemporal_store(pack_bf16x2((float)er, (float)ei), compv + g);
          }
          stnt(reinterpret_cast<V*>(e.out[o]) + g, V{sr, si});
          if (o == 0) {
            if (e.red_flags & 1) r0 += (double)sr * (double)sr + (double)si * (double)si;
            if (e.red_flags & 2) {
              const double dr = (double)sr - (double)uq.x, di = (double)si - (double)uq.y;
              r1 += dr * dr + di * di;
            }
          }
        }
        if (e.red_flags & 4) r2 += (double)uq.x * (double)hrr + (double)uq.y * (double)hii;
      }
    }
  }
  }
  if (FINAL && e.red_flags) block_reduce3<kThreads>(r0, r1, r2, e.red_flags, rbuf, e.red, nblocks, bid);
}

template <typename R, bool FINAL>
__global__ __launch_bounds__(kThreads) void k_pass(const PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  pass_body<R, FINAL>(a, blockIdx.x, gridDim.x, smem);
}

// Many solves in one launch: block b works on tile bmap[b].y of the solve whose
// arguments are args[bmap[b].x] (x < 0: nothing to do).
template <typename R, bool FINAL>
__global__ __launch_bounds__(kThreads) void k_pass_batch(const PassArgs* __restrict__ args,
                                                         const int2* __restrict__ bmap) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int2 m = bmap[blockIdx.x];
  if (m.x < 0) return;
  const PassArgs& a = args[m.x];
  pass_body<R, FINAL>(a, m.y, (int64_t)1 << (a.n - a.tb), smem);
}

// The complex64 high pass of the batch, held to 128 VGPRs (two workgroups of
// 512 threads per CU).
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_pass_batch_high_c64(
    const PassArgs* __restrict__ args, const int2* __restrict__ bmap) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int2 m = bmap[blockIdx.x];
  if (m.x < 0) return;
  const PassArgs& a = args[m.x];
  pass_body<float, false>(a, m.y, (int64_t)1 << (a.n - a.tb), smem);
}

// High-qubit flips on a hypercube held in registers: lane = bits 0..5 (64
// contiguous amplitudes per load instruction), registers = the 2^RB vertices of
// the hypercube over bits [hb, hb + RB).  A flip of bit hb + b pairs vertex v
// with v ^ 2^b inside the same lane's registers.
//
// WB = 0: every wave is independent (four per workgroup, no LDS, no barriers).
// WB > 0: the 2^WB waves of a workgroup are the values of the next WB bits
// [hb + RB, hb + RB + WB), so one pass covers RB + WB bits.  A flip of one of
// those bits pairs a wave with wave ^ 2^j; the partner's vertices are passed
// through LDS in chunks of CV vertices (double-buffered, one barrier a chunk).
template <int WB> struct RegShape {
  static constexpr int threads = WB == 0 ? 256 : (64 << WB);
};

// ACC: the pass adds the partial product of earlier passes (acc_in).  It is a
// template parameter so that the pass without it has no loads inside its
// store loop: loads and stores share one in-order counter on this GPU, so a
// wait for a load issued after a store also waits for that store.
template <typename R, int RB, int WB, bool ACC>
__device__ __forceinline__ void regpass_body(const RegPassArgs& a, const uint64_t blk,
                                             typename CT2<R>::V* ex) {
  using V = typename CT2<R>::V;
  constexpr int NV = 1 << RB;
  constexpr int NT = RegShape<WB>::threads;
  const int lane = threadIdx.x & 63;
  const int hb = a.hb;
  // the wave index is uniform: keep the row bases in scalar registers and add
  // only the lane offset per thread
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint64_t ubase;
  if constexpr (WB == 0) {
    const uint64_t wave = blk * 4 + (uint64_t)wv;
    if (wave >= (1ull << (a.n - 6 - RB))) return;
    const int lowcnt = hb - 6;
    ubase = ((wave & ((1ull << lowcnt) - 1ull)) << 6) | ((wave >> lowcnt) << (hb + RB));
  } else {
    const int lowcnt = hb - 6;
    ubase = ((blk & ((1ull << lowcnt) - 1ull)) << 6) | ((blk >> lowcnt) << (hb + RB + WB)) |
            ((uint64_t)wv << (hb + RB));
  }
  const V* src = reinterpret_cast<const V*>(a.src);
  const V* accin = reinterpret_cast<const V*>(a.acc_in);
  V* accout = reinterpret_cast<V*>(a.acc_out);
  auto at = [&](int v) -> uint64_t { return (ubase + ((uint64_t)v << hb)) + lane; };
  V x[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) x[v] = ldnt(src + at(v));
  R c[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) c[b] = (R)a.cb[b];
  if constexpr (WB == 0) {
    // blocks of VB vertices; with ACC the partial product of block k + 1 is
    // requested before block k is stored
    constexpr int VB = 8;
    V ain[2][VB];
    if constexpr (ACC) {
#pragma unroll
      for (int u = 0; u < VB; ++u) ain[0][u] = ldnt(accin + at(u));
    }
#pragma unroll
    for (int v0 = 0; v0 < NV; v0 += VB) {
      const int cb_ = (v0 / VB) & 1;
      if constexpr (ACC) {
        if (v0 + VB < NV) {
#pragma unroll
          for (int u = 0; u < VB; ++u) ain[cb_ ^ 1][u] = ldnt(accin + at(v0 + VB + u));
        }
      }
#pragma unroll
      for (int u = 0; u < VB; ++u) {
        const int v = v0 + u;
        R hr = 0, hi = 0;
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          hr += c[b] * x[v ^ (1 << b)].x;
          hi += c[b] * x[v ^ (1 << b)].y;
        }
        if constexpr (ACC) {
          hr += ain[cb_][u].x;
          hi += ain[cb_][u].y;
        }
        stnt(accout + at(v), V{hr, hi});
      }
    }
  } else {
    constexpr int CV = sizeof(R) == 4 ? 4 : 2;   // vertices per exchange chunk
    R cw[WB];
#pragma unroll
    for (int j = 0; j < WB; ++j) cw[j] = (R)a.cb[RB + j];
    const int tid = threadIdx.x;
    V ain[2][CV];
    if constexpr (ACC) {
#pragma unroll
      for (int u = 0; u < CV; ++u) ain[0][u] = ldnt(accin + at(u));
    }
#pragma unroll
    for (int v0 = 0; v0 < NV; v0 += CV) {
      const int cb_ = (v0 / CV) & 1;
      V* buf = ex + cb_ * (CV * NT);
#pragma unroll
      for (int u = 0; u < CV; ++u) buf[u * NT + tid] = x[v0 + u];
      // the next chunk's partial product is requested one chunk ahead
      if constexpr (ACC) {
        if (v0 + CV < NV) {
#pragma unroll
          for (int u = 0; u < CV; ++u) ain[cb_ ^ 1][u] = ldnt(accin + at(v0 + CV + u));
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < CV; ++u) {
        const int v = v0 + u;
        R hr = 0, hi = 0;
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          hr += c[b] * x[v ^ (1 << b)].x;
          hi += c[b] * x[v ^ (1 << b)].y;
        }
#pragma unroll
        for (int j = 0; j < WB; ++j) {
          const V p = buf[u * NT + (tid ^ (64 << j))];
          hr += cw[j] * p.x;
          hi += cw[j] * p.y;
        }
        if constexpr (ACC) {
          hr += ain[cb_][u].x;
          hi += ain[cb_][u].y;
        }
        stnt(accout + at(v), V{hr, hi});
      }
    }
  }
}

// LDS of the wide form: two chunk buffers of CV vertices for every thread
template <typename R, int WB> struct RegLds {
  static constexpr int CV = sizeof(R) == 4 ? 4 : 2;
  static constexpr int count = WB == 0 ? 1 : 2 * CV * RegShape<WB>::threads;
};

template <typename R, int RB, int WB, bool ACC>
__global__ __launch_bounds__(RegShape<WB>::threads) void k_regpass(const RegPassArgs a) {
  __shared__ typename CT2<R>::V ex[RegLds<R, WB>::count];
  regpass_body<R, RB, WB, ACC>(a, blockIdx.x, ex);
}

template <typename R, int RB, int WB>
__global__ __launch_bounds__(RegShape<WB>::threads) void k_regpass_batch(
    const RegPassArgs* __restrict__ args, const int2* __restrict__ bmap) {
  __shared__ typename CT2<R>::V ex[RegLds<R, WB>::count];
  const int2 m = bmap[blockIdx.x];
  if (m.x < 0) return;   // uniform over the workgroup
  const RegPassArgs& a = args[m.x];
  if (a.acc_in) regpass_body<R, RB, WB, true>(a, (uint64_t)m.y, ex);
  else regpass_body<R, RB, WB, false>(a, (uint64_t)m.y, ex);
}

int64_t regpass_blocks(int n, int wb, int dtype) {
  const int rb = dtype == 0 ? kRegBitsC64 : kRegBitsC128;
  if (wb == 0) return (((int64_t)1 << (n - 6 - rb)) + 3) / 4;
  return (int64_t)1 << (n - 6 - rb - wb);
}

hipError_t launch_regpass_batch(const RegPassArgs* args, const int2* bmap, int64_t nblocks, int wb,
                                int dtype, hipStream_t s) {
  const dim3 grid((unsigned)nblocks);
  if (wb != 0 && wb != kWaveBits) return hipErrorInvalidValue;
  if (dtype == 0) {
    if (wb == 0)
      hipLaunchKernelGGL((k_regpass_batch<float, kRegBitsC64, 0>), grid, dim3(RegShape<0>::threads), 0,
                         s, args, bmap);
    else
      hipLaunchKernelGGL((k_regpass_batch<float, kRegBitsC64, kWaveBits>), grid,
                         dim3(RegShape<kWaveBits>::threads), 0, s, args, bmap);
  } else {
    if (wb == 0)
      hipLaunchKernelGGL((k_regpass_batch<double, kRegBitsC128, 0>), grid, dim3(RegShape<0>::threads),
                         0, s, args, bmap);
    else
      hipLaunchKernelGGL((k_regpass_batch<double, kRegBitsC128, kWaveBits>), grid,
                         dim3(RegShape<kWaveBits>::threads), 0, s, args, bmap);
  }
  return hipGetLastError();
}

hipError_t launch_pass_batch(const PassArgs* args, const int2* bmap, int64_t nblocks, int final_pass,
                             int max_tb, int dtype, hipStream_t s) {
  const size_t lds = pass_lds_bytes(max_tb, dtype);
  dim3 grid((unsigned)nblocks), block(kThreads);
  if (dtype == 0) {
    if (final_pass) hipLaunchKernelGGL((k_pass_batch<float, true>), grid, block, lds, s, args, bmap);
    else hipLaunchKernelGGL(k_pass_batch_high_c64, grid, block, lds, s, args, bmap);
  } else {
    if (final_pass) hipLaunchKernelGGL((k_pass_batch<double, true>), grid, block, lds, s, args, bmap);
    else hipLaunchKernelGGL((k_pass_batch<double, false>), grid, block, lds, s, args, bmap);
  }
  return hipGetLastError();
}

// Graph nodes of the batched kernels (graphs are built node by node, not by
// stream capture, so other threads may use the device meanwhile).
static hipError_t add_kernel_node(hipGraph_t g, hipGraphNode_t* node, hipGraphNode_t dep,
                                  const void* fn, dim3 grid, dim3 block, size_t lds, void** params) {
  hipKernelNodeParams p{};
  p.func = const_cast<void*>(fn);
  p.gridDim = grid;
  p.blockDim = block;
  p.sharedMemBytes = (unsigned int)lds;
  p.kernelParams = params;
  p.extra = nullptr;
  return hipGraphAddKernelNode(node, g, dep ? &dep : nullptr, dep ? 1 : 0, &p);
}

hipError_t add_regpass_batch_node(hipGraph_t g, hipGraphNode_t* node, hipGraphNode_t dep,
                                  const RegPassArgs* args, const int2* bmap, int64_t nblocks, int wb,
                                  int dtype) {
  if (wb != 0 && wb != kWaveBits) return hipErrorInvalidValue;
  void* prm[] = {(void*)&args, (void*)&bmap};
  const void* fn;
  if (dtype == 0)
    fn = wb ? reinterpret_cast<const void*>(&k_regpass_batch<float, kRegBitsC64, kWaveBits>)
            : reinterpret_cast<const void*>(&k_regpass_batch<float, kRegBitsC64, 0>);
  else
    fn = wb ? reinterpret_cast<const void*>(&k_regpass_batch<double, kRegBitsC128, kWaveBits>)
            : reinterpret_cast<const void*>(&k_regpass_batch<double, kRegBitsC128, 0>);
  const int threads = wb ? RegShape<kWaveBits>::threads : RegShape<0>::threads;
  return add_kernel_node(g, node, dep, fn, dim3((unsigned)nblocks), dim3(threads), 0, prm);
}

hipError_t add_pass_batch_node(hipGraph_t g, hipGraphNode_t* node, hipGraphNode_t dep,
                               const PassArgs* args, const int2* bmap, int64_t nblocks, int final_pass,
                               int max_tb, int dtype) {
  void* prm[] = {(void*)&args, (void*)&bmap};
  const void* fn;
  if (dtype == 0)
    fn = final_pass ? reinterpret_cast<const void*>(&k_pass_batch<float, true>)
                    : reinterpret_cast<const void*>(&k_pass_batch_high_c64);
  else
    fn = final_pass ? reinterpret_cast<const void*>(&k_pass_batch<double, true>)
                    : reinterpret_cast<const void*>(&k_pass_batch<double, false>);
  return add_kernel_node(g, node, dep, fn, dim3((unsigned)nblocks), dim3(kThreads),
                         pass_lds_bytes(max_tb, dtype), prm);
}

template <typename R, int RB, int WB>
static void launch_regpass_t(const RegPassArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)regpass_blocks(a.n, WB, sizeof(R) == 4 ? 0 : 1));
  const dim3 block(RegShape<WB>::threads);
  if (a.acc_in) hipLaunchKernelGGL((k_regpass<R, RB, WB, true>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_regpass<R, RB, WB, false>), grid, block, 0, s, a);
}

hipError_t launch_regpass(const RegPassArgs& a, int dtype, hipStream_t s) {
  if (a.wb != 0 && a.wb != kWaveBits) return hipErrorInvalidValue;
  if (dtype == 0) {
    if (a.wb == 0) launch_regpass_t<float, kRegBitsC64, 0>(a, s);
    else launch_regpass_t<float, kRegBitsC64, kWaveBits>(a, s);
  } else {
    if (a.wb == 0) launch_regpass_t<double, kRegBitsC128, 0>(a, s);
    else launch_regpass_t<double, kRegBitsC128, kWaveBits>(a, s);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Resident solves of a batch: workgroup b runs solves[b] from start to end.
// Thread 0 walks the segment stepper and writes each pass's arguments into
// LDS; all threads evaluate the passes (tile passes only) tile by tile,
// separated by workgroup barriers, so no other workgroup is ever waited for.
// The shift's phase is applied at the end.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kThreads) void k_resident(const ResidentSolve* __restrict__ solves) {
  using V = typename CT2<R>::V;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ PassArgs pa;
  __shared__ EpiDesc epi;
  __shared__ double fs[kMaxSched];
  __shared__ double stage_t;
  __shared__ const void* stage_src;
  const ResidentSolve& S = solves[blockIdx.x];
  const int tid = threadIdx.x;
  SegStepper sg;
  sg.method = AQC_METHOD_PC4;
  sg.ts = S.t0;
  sg.h = S.h;
  sg.k_end = S.K;
  sg.more_after = false;
  sg.dbl = S.dbl != 0;
  const int64_t total = pc4_matvecs(S.K);
  for (int64_t m = 0; m < total; ++m) {
    if (tid == 0) {
      const MatvecStage st = sg.next(S.v);
      stage_t = st.t;
      stage_src = st.src;
      epi = st.e;
    }
    if (tid == 0) sg.advance();
    __syncthreads();
    if (tid < kMaxSched) fs[tid] = tid < S.nsched ? sched_value(S.sched[tid], S.path, stage_t) : 0.0;
    __syncthreads();
    for (int p = 0; p < S.npass; ++p) {
      const ResPass& P = S.pass[p];
      const bool last = p + 1 == S.npass;
      const uint64_t* from = reinterpret_cast<const uint64_t*>(&P.pa);
      uint64_t* to = reinterpret_cast<uint64_t*>(&pa);
      for (int i = tid; i < (int)(sizeof(PassArgs) / 8); i += kThreads) to[i] = from[i];
      __syncthreads();
      if (tid == 0) {
        double ident = 0.0;
        for (int q = 0; q < S.nsched; ++q) ident += S.ident_w[q] * fs[q];
        for (int q = 0; q < kMaxSched; ++q) pa.f[q] = fs[q];
        pa.dconst = ident - S.shift;
        pa.src = stage_src;
        if (!last) {
          pa.acc_in = p > 0 ? S.v.hbuf : nullptr;
          pa.acc_out = S.v.hbuf;
        } else {
          pa.acc_in = S.npass > 1 ? S.v.hbuf : nullptr;
          pa.epi = epi;
        }
      }
      __syncthreads();
      for (int64_t b = 0; b < P.nblocks; ++b) {
        if (last) pass_body<R, true>(pa, b, P.nblocks, smem);
        else pass_body<R, false>(pa, b, P.nblocks, smem);
        __syncthreads();
      }
    }
  }
  const double ph = -S.shift * (S.t1 - S.t0);
  const R cr = (R)cos(ph), ci = (R)sin(ph);
  V* y = reinterpret_cast<V*>(S.v.y);
  const int64_t N = (int64_t)1 << S.n;
  for (int64_t i = tid; i < N; i += kThreads) {
    const V v = y[i];
    y[i] = V{cr * v.x - ci * v.y, cr * v.y + ci * v.x};
  }
}

hipError_t launch_resident(const ResidentSolve* solves, int count, int max_tb, int dtype, hipStream_t s) {
  if (count < 1) return hipSuccess;
  const size_t lds = pass_lds_bytes(max_tb, dtype);
  if (dtype == 0)
    hipLaunchKernelGGL(k_resident<float>, dim3((unsigned)count), dim3(kThreads), lds, s, solves);
  else
    hipLaunchKernelGGL(k_resident<double>, dim3((unsigned)count), dim3(kThreads), lds, s, solves);
  return hipGetLastError();
}

template <typename R, bool FINAL>
static hipError_t set_lds_attr() {
  const int bytes = (int)pass_lds_bytes(sizeof(R) == 4 ? 14 : 13, sizeof(R) == 4 ? 0 : 1);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pass<R, FINAL>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pass_batch<R, FINAL>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess || sizeof(R) != 4 || FINAL) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pass_batch_high_c64),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

static hipError_t set_sector_lds_attr();

hipError_t prepare_kernels() {
  hipError_t e;
  if ((e = set_sector_lds_attr()) != hipSuccess) return e;
  if ((e = set_lds_attr<float, false>()) != hipSuccess) return e;
  if ((e = set_lds_attr<float, true>()) != hipSuccess) return e;
  if ((e = set_lds_attr<double, false>()) != hipSuccess) return e;
  if ((e = set_lds_attr<double, true>()) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_resident<float>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pass_lds_bytes(14, 0))) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_resident<double>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)pass_lds_bytes(13, 1))) != hipSuccess)
    return e;
  return hipSuccess;
}

hipError_t launch_pass(const PassArgs& a, int dtype, int64_t nblocks, hipStream_t s) {
  const size_t lds = pass_lds_bytes(a.tb, dtype);
  dim3 grid((unsigned)nblocks), block(kThreads);
  if (dtype == 0) {
    if (a.final_pass) hipLaunchKernelGGL((k_pass<float, true>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((k_pass<float, false>), grid, block, lds, s, a);
  } else {
    if (a.final_pass) hipLaunchKernelGGL((k_pass<double, true>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((k_pass<double, false>), grid, block, lds, s, a);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed scratch of the allocation-free entry point.  Host code must not pass
// `scratch` itself to a kernel (in host code the name is a host-side stand-in);
// it takes the device address from scratch_address once per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void** p) {
  return hipGetSymbolAddress(p, HIP_SYMBOL(scratch));
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kRedThreads) void k_reduce_sum(const double* parts, int64_t nb, int nk,
                                                            double* out) {
  __shared__ double sb[kRedThreads];
  for (int k = 0; k < nk; ++k) {
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += kRedThreads) v += parts[k * nb + i];
    sb[threadIdx.x] = v;
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sb[threadIdx.x] += sb[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sb[0];
    __syncthreads();
  }
}

hipError_t launch_reduce_sum(const double* parts, int64_t nblocks, int nk, double* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(kRedThreads), 0, s, parts, nblocks, nk, out);
  return hipGetLastError();
}

static int64_t red_blocks(int64_t N) {
  int64_t nb = (N + (int64_t)kRedThreads * 16 - 1) / ((int64_t)kRedThreads * 16);
  if (nb > 16384) nb = 16384;
  if (nb < 1) nb = 1;
  return nb;
}

template <typename V>
__global__ __launch_bounds__(kRedThreads) void k_norm2(const V* psi, int64_t N, double* parts) {
  __shared__ double sb[3 * (kRedThreads / 64)];
  double r = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kRedThreads) {
    const V v = psi[i];
    r += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
  }
  block_reduce3<kRedThreads>(r, 0.0, 0.0, 1, sb, parts, gridDim.x, blockIdx.x);
}

hipError_t launch_norm2(const void* psi, int dtype, int64_t N, double* parts, int64_t* nb,
                        hipStream_t s) {
  *nb = red_blocks(N);
  if (dtype == 0)
    hipLaunchKernelGGL(k_norm2<float2>, dim3((unsigned)*nb), dim3(kRedThreads), 0, s,
                       (const float2*)psi, N, parts);
  else
    hipLaunchKernelGGL(k_norm2<double2>, dim3((unsigned)*nb), dim3(kRedThreads), 0, s,
                       (const double2*)psi, N, parts);
  return hipGetLastError();
}

template <typename V>
__global__ __launch_bounds__(kRedThreads) void k_overlap(const V* phi, const V* psi, int64_t N,
                                                         double* parts) {
  __shared__ double sb[3 * (kRedThreads / 64)];
  double re = 0.0, im = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kRedThreads) {
    const V a = phi[i], b = psi[i];
    re += (double)a.x * (double)b.x + (double)a.y * (double)b.y;
    im += (double)a.x * (double)b.y - (double)a.y * (double)b.x;
  }
  block_reduce3<kRedThreads>(re, im, 0.0, 3, sb, parts, gridDim.x, blockIdx.x);
}

hipError_t launch_overlap(const void* phi, const void* psi, int dtype, int64_t N, double* parts,
                          int64_t* nb, hipStream_t s) {
  *nb = red_blocks(N);
  if (dtype == 0)
    hipLaunchKernelGGL(k_overlap<float2>, dim3((unsigned)*nb), dim3(kRedThreads), 0, s,
                       (const float2*)phi, (const float2*)psi, N, parts);
  else
    hipLaunchKernelGGL(k_overlap<double2>, dim3((unsigned)*nb), dim3(kRedThreads), 0, s,
                       (const double2*)phi, (const double2*)psi, N, parts);
  return hipGetLastError();
}

template <typename V>
__global__ __launch_bounds__(kRedThreads) void k_gather_mass(const V* psi, const int64_t* idx,
                                                             int64_t m, double* parts) {
  __shared__ double sb[3 * (kRedThreads / 64)];
  double r = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * kRedThreads) {
    const V v = psi[idx[i]];
    r += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
  }
  block_reduce3<kRedThreads>(r, 0.0, 0.0, 1, sb, parts, gridDim.x, blockIdx.x);
}

hipError_t launch_gather_mass(const void* psi, int dtype, const int64_t* idx, int64_t m,
                              double* parts, int64_t* nb, hipStream_t s) {
  *nb = red_blocks(m);
  if (dtype == 0)
    hipLaunchKernelGGL(k_gather_mass<float2>, dim3((unsigned)*nb), dim3(kRedThreads), 0, s,
                       (const float2*)psi, idx, m, parts);
  else
    hipLaunchKernelGGL(k_gather_mass<double2>, dim3((unsigned)*nb), dim3(kRedThreads), 0, s,
                       (const double2*)psi, idx, m, parts);
  return hipGetLastError();
}

// Diagonal over one tile of the last pass's geometry (always float64).
__device__ __forceinline__ void diag_tile_setup(const PassArgs& a, double* fsh, double* lin,
                                                double* cps, double* LA, double* LB) {
  if (threadIdx.x < kMaxSched) fsh[threadIdx.x] = a.f[threadIdx.x];
  __syncthreads();
  diag_setup_a<double>(a, (uint64_t)blockIdx.x, fsh, lin, cps);
  __syncthreads();
  diag_setup_b(a, lin, LA, LB);
  __syncthreads();
}

__global__ __launch_bounds__(kThreads) void k_diag_minmax(const PassArgs a, double* parts) {
  __shared__ double fsh[kMaxSched], lin[16], cps[1], LA[128], LB[128];
  __shared__ double sb[2 * (kThreads / 64)];
  diag_tile_setup(a, fsh, lin, cps, LA, LB);
  const uint32_t ntile = 1u << a.tb;
  const uint64_t base = (uint64_t)blockIdx.x << a.tb;
  double mn = INFINITY, mx = -INFINITY;
  for (uint32_t l = threadIdx.x; l < ntile; l += kThreads) {
    const double d = diag_value(a, l, base + l, cps[0], LA, LB, fsh);
    mn = fmin(mn, d);
    mx = fmax(mx, d);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o, 64));
    mx = fmax(mx, __shfl_xor(mx, o, 64));
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sb[wv] = mn;
    sb[kThreads / 64 + wv] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / 64; ++w) {
      mn = fmin(mn, sb[w]);
      mx = fmax(mx, sb[kThreads / 64 + w]);
    }
    mn = fmin(mn, sb[0]);
    mx = fmax(mx, sb[kThreads / 64]);
    parts[blockIdx.x] = mn;
    parts[gridDim.x + blockIdx.x] = mx;
  }
}

hipError_t launch_diag_minmax(const PassArgs& a, int64_t nblocks, double* parts, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_minmax, dim3((unsigned)nblocks), dim3(kThreads), 0, s, a, parts);
  return hipGetLastError();
}

template <typename V>
__global__ __launch_bounds__(kThreads) void k_diag_mass(const PassArgs a, const V* psi, double thr,
                                                        double* parts) {
  __shared__ double fsh[kMaxSched], lin[16], cps[1], LA[128], LB[128];
  __shared__ double sb[3 * (kThreads / 64)];
  diag_tile_setup(a, fsh, lin, cps, LA, LB);
  const uint32_t ntile = 1u << a.tb;
  const uint64_t base = (uint64_t)blockIdx.x << a.tb;
  double r = 0.0;
  for (uint32_t l = threadIdx.x; l < ntile; l += kThreads) {
    const double d = diag_value(a, l, base + l, cps[0], LA, LB, fsh);
    if (d <= thr) {
      const V v = psi[base + l];
      r += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
    }
  }
  block_reduce3<kThreads>(r, 0.0, 0.0, 1, sb, parts, gridDim.x, blockIdx.x);
}

hipError_t launch_diag_mass(const PassArgs& a, int dtype, int64_t nblocks, double thr,
                            double* parts, hipStream_t s) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_diag_mass<float2>, dim3((unsigned)nblocks), dim3(kThreads), 0, s, a,
                       (const float2*)a.src, thr, parts);
  else
    hipLaunchKernelGGL(k_diag_mass<double2>, dim3((unsigned)nblocks), dim3(kThreads), 0, s, a,
                       (const double2*)a.src, thr, parts);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Elementwise
// ---------------------------------------------------------------------------

static unsigned ew_blocks(int64_t N) {
  int64_t nb = (N + 255) / 256;
  if (nb > 65536) nb = 65536;
  return (unsigned)(nb < 1 ? 1 : nb);
}

template <typename V, typename R>
__global__ void k_scale(V* y, int64_t N, R re, R im) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    const V v = y[i];
    y[i] = V{re * v.x - im * v.y, re * v.y + im * v.x};
  }
}

hipError_t launch_scale(void* y, int dtype, int64_t N, double re, double im, hipStream_t s) {
  if (dtype == 0)
    hipLaunchKernelGGL((k_scale<float2, float>), dim3(ew_blocks(N)), dim3(256), 0, s, (float2*)y, N,
                       (float)re, (float)im);
  else
    hipLaunchKernelGGL((k_scale<double2, double>), dim3(ew_blocks(N)), dim3(256), 0, s,
                       (double2*)y, N, re, im);
  return hipGetLastError();
}


__global__ void k_zero(uint4* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = uint4{0u, 0u, 0u, 0u};
}

hipError_t launch_zero(void* dst, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 16);
  hipLaunchKernelGGL(k_zero, dim3(ew_blocks(n)), dim3(256), 0, s, (uint4*)dst, n);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, int dtype, int64_t N, hipStream_t s) {
  return hipMemcpyAsync(dst, src, (size_t)N * (dtype == 0 ? 8 : 16), hipMemcpyDeviceToDevice, s);
}

// ---------------------------------------------------------------------------
// Hamming-weight sector (Sec. III.A.2-3): H^xy, H^xyz and a diagonal H_f keep
// the number of 1-bits, so a state of weight w lives on C(n, w) amplitudes
// stored by rank.  A workgroup walks chunks of kSecThreads * kSecEPT
// consecutive ranks; each thread unranks its first rank once and steps to the
// next states of the same weight with Gosper's successor.  A weight-preserving
// hop of two differing bits reaches the partner at rank r(z ^ x), read from
// the 6-bit chunk table; the diagonal is summed over the set bits (or the
// zero bits, whichever are fewer) from per-bit and pairwise coefficients.
// ---------------------------------------------------------------------------
struct SecLds {
  uint32_t binom[kSecBinom * kSecBinom];
  double hsh[kSecMaxN];      // one-bit coefficients h_p (sigma^z_p)
  double rsh[kSecMaxN];      // R_p = sum_q J_pq
  double a[kSecMaxN];        // per-bit part of the diagonal
  double J[kSecMaxN * kSecMaxN];
  uint64_t nbr[kSecMaxN];    // bits q < p with J_pq != 0
  double fsh[kMaxSched];
  double c0;
  double red[3 * (kSecThreads / 64)];
};

// Coefficients at this time: with s_q = 1 - 2 b_q the diagonal
//   D(z) = dconst + sum_q h_q s_q + sum_{p<q} J_pq s_p s_q + (3+ bit terms)
// becomes c0 + sum_{p in S} a_p + 4 sum_{q<p in S} J_pq over the set S of the
// one-bits (a_p = -2 (h_p + R_p), c0 = dconst + sum h + sum_{p<q} J) or of the
// zero bits (a_p = 2 (h_p - R_p), c0 = dconst - sum h + sum_{p<q} J).
__device__ void sector_setup(const SectorArgs& a, SecLds& L) {
  const int tid = threadIdx.x;
  const SectorDev& s = a.s;
  const int n = s.n;
  if (tid < kMaxSched) L.fsh[tid] = a.f[tid];
  for (int i = tid; i < kSecBinom * kSecBinom; i += kSecThreads) L.binom[i] = s.binom[i];
  for (int i = tid; i < n * n; i += kSecThreads) L.J[i] = 0.0;
  if (tid < n) L.hsh[tid] = 0.0;
  __syncthreads();
  for (int k = tid; k < s.nmasks; k += kSecThreads) {
    const SecMask m = s.masks[k];
    double c = 0.0;
    for (int t = 0; t < m.nt; ++t) {
      const DevTerm tt = s.mterms[m.t0 + t];
      c += tt.w * L.fsh[tt.sid];
    }
    if (m.q < 0) {
      L.hsh[m.p] = c;
    } else {
      L.J[m.p * n + m.q] = c;
      L.J[m.q * n + m.p] = c;
    }
  }
  __syncthreads();
  if (tid < n) {
    double r = 0.0;
    uint64_t nb = 0;
    for (int q = 0; q < n; ++q) {
      const double j = L.J[tid * n + q];
      r += j;
      if (q < tid && j != 0.0) nb |= 1ull << q;
    }
    L.rsh[tid] = r;
    L.nbr[tid] = nb;
    L.a[tid] = s.zero_bits ? 2.0 * (L.hsh[tid] - r) : -2.0 * (L.hsh[tid] + r);
  }
  __syncthreads();
  if (tid == 0) {
    double hs = 0.0, js = 0.0;
    for (int p = 0; p < n; ++p) {
      hs += L.hsh[p];
      js += L.rsh[p];
    }
    L.c0 = a.dconst + (s.zero_bits ? -hs : hs) + 0.5 * js;
  }
  __syncthreads();
}

// number of trailing zeros, count of 1-bits and a chunk of a state word
__device__ __forceinline__ int sw_ctz(uint32_t v) { return __builtin_ctz(v); }
__device__ __forceinline__ int sw_ctz(uint64_t v) { return __builtin_ctzll(v); }
__device__ __forceinline__ uint32_t sw_popc(uint32_t v) { return __builtin_popcount(v); }
__device__ __forceinline__ uint32_t sw_popc(uint64_t v) { return __builtin_popcountll(v); }
__device__ __forceinline__ uint32_t sw_nib(uint32_t v, int c) {
  return __builtin_amdgcn_ubfe(v, kSecChunkBits * c, kSecChunkBits);
}
__device__ __forceinline__ uint32_t sw_nib(uint64_t v, int c) {
  return (uint32_t)(v >> (kSecChunkBits * c)) & ((1u << kSecChunkBits) - 1u);
}

template <typename W>
__device__ __forceinline__ double sector_diag(const SectorArgs& a, const SecLds& L, W z) {
  const SectorDev& s = a.s;
  const W full = s.n >= (int)(8 * sizeof(W)) ? ~W(0) : (W(1) << s.n) - W(1);
  const W S = s.zero_bits ? (~z & full) : z;
  double d = L.c0, pj = 0.0;
  W m = S;
  while (m) {
    const int p = sw_ctz(m);
    m &= m - W(1);
    d += L.a[p];
    W nb = (W)L.nbr[p] & S;
    while (nb) {
      const int q = sw_ctz(nb);
      nb &= nb - W(1);
      pj += L.J[p * s.n + q];
    }
  }
  d += 4.0 * pj;
  for (int k = 0; k < s.nres; ++k) {
    const DevTerm t = s.res[k];
    const double mm = t.w * L.fsh[t.sid];
    d += (__popcll((uint64_t)z & t.z) & 1) ? -mm : mm;
  }
  return d;
}

// the basis state of weight w at rank r (largest C(p, k) <= r, bit by bit)
template <typename W = uint64_t>
__device__ __forceinline__ W sector_unrank(const uint32_t* binom, int n, int w, int64_t r) {
  W z = 0;
  int p = n - 1;
  uint32_t rr = (uint32_t)r;
  for (int k = w; k >= 1; --k) {
    // stops at p >= k - 1, where C(k - 1, k) = 0
    while (binom[p * kSecBinom + k] > rr) --p;
    z |= W(1) << p;
    rr -= binom[p * kSecBinom + k];
    --p;
  }
  return z;
}

// the next larger integer with the same number of 1-bits (Gosper)
template <typename W>
__device__ __forceinline__ W next_same_weight(W z) {
  const W c = z & (W(0) - z);
  const W r = z + c;
  return (((r ^ z) >> 2) >> sw_ctz(c)) | r;
}

int64_t sector_blocks(int64_t dim) {
  const int64_t per = (int64_t)kSecThreads * kSecEPT;
  const int64_t nb = (dim + per - 1) / per;
  return nb < 1 ? 1 : (nb > kSecGrid ? kSecGrid : nb);
}

// Coefficients of the pair hops at this time: for a "fast" hop (every Z
// string inside its two bits) the coefficient of a state whose two bits
// differ depends only on the partner's bit bi: hc[4k..4k+1] for partner bit 0,
// hc[4k+2..4k+3] for 1 (re, im).  Other hops keep per-term values in tm.
template <typename R>
__device__ __forceinline__ void sector_hop_setup(const SectorDev& s, const SecLds& L, R* tm, R* hc) {
  for (int k = threadIdx.x; k < s.nhterms; k += kSecThreads) {
    const DevTerm t = s.hterms[k];
    tm[k] = (R)(t.w * L.fsh[t.sid]);
  }
  for (int k = threadIdx.x; k < s.nhops; k += kSecThreads) {
    const SecHop hp = s.hops[k];
    if (!hp.fast) continue;
    double c[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = 0; t < hp.nt; ++t) {
      const DevTerm tt = s.hterms[hp.t0 + t];
      const double m = tt.w * L.fsh[tt.sid];
      const int zi = (int)((tt.z >> hp.bi) & 1ull), zj = (int)((tt.z >> hp.bj) & 1ull);
      for (int b = 0; b < 2; ++b) {
        // the partner's bits are (bi, bj) = (b, 1 - b)
        const double v = (((zi & b) ^ (zj & (1 - b))) & 1) ? -m : m;
        switch (tt.p & 3) {
          case 0: c[2 * b] += v; break;
          case 1: c[2 * b + 1] += v; break;
          case 2: c[2 * b] -= v; break;
          default: c[2 * b + 1] -= v; break;
        }
      }
    }
    for (int q = 0; q < 4; ++q) hc[4 * k + q] = (R)c[q];
  }
}

// the rank table's share of k_sector's dynamic LDS, padded to 16 bytes
__host__ __device__ __forceinline__ size_t sector_rtab_lds_bytes(const SectorDev& sd) {
  return ((size_t)sd.rwords * sizeof(uint32_t) + 15) & ~(size_t)15;
}

// A hop's gathered partners and coefficients, added to the product one hop
// that needs partners later
template <typename R>
struct SecPend {
  typename CT2<R>::V v[kSecEPT];
  R cr[kSecEPT], ci[kSecEPT];
};

// hr + i hi += (cr + i ci) * pv for each state
template <typename R>
__device__ __forceinline__ void sector_hop_fma(R (&hr)[kSecEPT], R (&hi)[kSecEPT], const typename CT2<R>::V (&pv)[kSecEPT],
                                               const R (&cr)[kSecEPT], const R (&ci)[kSecEPT]) {
#pragma unroll
  for (int u = 0; u < kSecEPT; ++u) {
    hr[u] = hr[u] + cr[u] * pv[u].x;
    hr[u] = hr[u] - ci[u] * pv[u].y;
    hi[u] = hi[u] + cr[u] * pv[u].y;
    hi[u] = hi[u] + ci[u] * pv[u].x;
  }
}

// The off-diagonal sum over one run of pair hops that share their chunk pair
// (ca, cb) of the rank table, for kSecEPT states per lane.  The partner z ^ x
// of a state z (x = bits bi < bj, which differ in z) differs from z in the
// patterns of chunks ca and cb only; the chunks in between keep their pattern
// but see one 1-bit more (z_bi = 0) or one less (z_bi = 1) below them, so
// their table row moves by +-1.  Its rank is therefore
//   r + T_ca[k_a][np_a] - T_ca[k_a][nz_a] + M(+-1) + T_cb[k_b +- 1][np_b] - T_cb[k_b][nz_b]
// where only the two partner patterns depend on the hop: everything else is
// computed once per run and state.  Every lane runs the same instructions
// whether or not its states' bits differ: a lane whose state has no partner
// gathers its own state (in bounds, and in the lines the stage update reads
// anyway) with coefficient zero, and a hop that no state of the wave needs is
// skipped.  A hop's term is added one hop later, from one of two buffers
// taken in turn (pa, pb; par names the next one to fill), so that its gathers
// overlap the next hop's rank arithmetic.  (With a single buffer, the compiler
// copied each gathered value into it at the end of the hop, which waits for
// the gathers there.  With two it still copies those gathered into pb, not
// knowing that the buffers alternate: half of the hops overlap.)
template <typename R, typename W>
__device__ __forceinline__ void sector_group(const SectorDev& s, const uint32_t* rtab, const uint32_t* hrec,
                                             int g0, int gn, const W (&zs)[kSecEPT], const bool (&ok)[kSecEPT],
                                             uint32_t r0, uint32_t last, const R* hc, const R* tm,
                                             const typename CT2<R>::V* __restrict__ src,
                                             const typename CT2<R>::V* __restrict__ srcb,
                                             R (&hr)[kSecEPT], R (&hi)[kSecEPT], SecPend<R>& pa, SecPend<R>& pb,
                                             int& par) {
  using V = typename CT2<R>::V;
  constexpr uint32_t CW = 1u << kSecChunkBits;     // words per table row
  const uint32_t rec0 = __builtin_amdgcn_readfirstlane(hrec[g0]);
  const int ca = (int)((rec0 >> 12) & 7u), cb = (int)((rec0 >> 15) & 7u);
  // per state: table rows (word offsets) at ca and cb, the patterns there, and
  // the hop-independent part of the partner rank for z_bi = 0 / 1
  uint32_t ra[kSecEPT], rb[kSecEPT], na[kSecEPT], nb[kSecEPT], cp[kSecEPT], cm[kSecEPT];
  const W below = (W(1) << (kSecChunkBits * ca)) - W(1);
#pragma unroll
  for (int u = 0; u < kSecEPT; ++u) {
    const uint32_t ka = sw_popc(zs[u] & below);
    na[u] = sw_nib(zs[u], ca);
    ra[u] = (uint32_t)s.cbase[ca] + ka * CW;
    cp[u] = r0 + (uint32_t)u - rtab[ra[u] + na[u]];
    rb[u] = ka + sw_popc(na[u]);                  // 1-bits below the next chunk
  }
  if (cb > ca) {
#pragma unroll
    for (int u = 0; u < kSecEPT; ++u) cm[u] = cp[u];
    for (int c = ca + 1; c < cb; ++c) {
#pragma unroll
      for (int u = 0; u < kSecEPT; ++u) {
        const uint32_t m = sw_nib(zs[u], c);
        // a lane whose partner goes one row down has a 1-bit below, so the row
        // above zero is never needed by it; its index is in range regardless
        const uint32_t* rw = rtab + ((uint32_t)s.cbase[c] + rb[u] * CW + m);
        const uint32_t t = rw[0];
        cp[u] += rw[CW] - t;
        cm[u] += rw[-(int)CW] - t;
        rb[u] += sw_popc(m);
      }
    }
#pragma unroll
    for (int u = 0; u < kSecEPT; ++u) {
      nb[u] = sw_nib(zs[u], cb);
      const uint32_t row = (uint32_t)s.cbase[cb] + rb[u] * CW;
      const uint32_t t = rtab[row + nb[u]];
      cp[u] -= t;
      cm[u] -= t;
      rb[u] = row;
    }
  }
  for (int k = g0; k < g0 + gn; ++k) {
    const uint32_t rec = __builtin_amdgcn_readfirstlane(hrec[k]);
    const int bi = (int)(rec & 63u), bj = (int)((rec >> 6) & 63u);
    const bool fast = ((rec >> 18) & 1u) != 0u;
    const W x = (W(1) << bi) | (W(1) << bj);
    bool act[kSecEPT], z1[kSecEPT];
    bool any = false;
#pragma unroll
    for (int u = 0; u < kSecEPT; ++u) {
      const W t = zs[u] & x;
      act[u] = ok[u] && t != W(0) && t != x;
      z1[u] = ((t >> bi) & W(1)) != W(0);
      any = any || act[u];
    }
    // consecutive ranks share their high bits, so for a hop between two of
    // them no state of the wave may need a partner
    if (!__any(any)) continue;
    uint32_t rp[kSecEPT];
    if (cb == ca) {
      const uint32_t fa = (1u << (bi - kSecChunkBits * ca)) | (1u << (bj - kSecChunkBits * ca));
#pragma unroll
      for (int u = 0; u < kSecEPT; ++u) rp[u] = cp[u] + rtab[ra[u] + (na[u] ^ fa)];
    } else {
      const uint32_t fa = 1u << (bi - kSecChunkBits * ca), fb = 1u << (bj - kSecChunkBits * cb);
#pragma unroll
      for (int u = 0; u < kSecEPT; ++u) {
        const uint32_t rbp = z1[u] ? rb[u] - CW : rb[u] + CW;
        rp[u] = (z1[u] ? cm[u] : cp[u]) + rtab[ra[u] + (na[u] ^ fa)] + rtab[rbp + (nb[u] ^ fb)];
      }
    }
    // a weight-w state has a rank below dim; the clamp only guards the read
    uint32_t gi[kSecEPT];
#pragma unroll
    for (int u = 0; u < kSecEPT; ++u) gi[u] = act[u] ? min(rp[u], last) : min(r0 + (uint32_t)u, last);
    R cr[kSecEPT], ci[kSecEPT];
    if (fast) {
      // the coefficient depends only on the partner's bit bi (= 1 - z_bi)
      const R* hk = hc + 4 * k;
      const R a0 = hk[0], a1 = hk[1], b0 = hk[2], b1 = hk[3];
#pragma unroll
      for (int u = 0; u < kSecEPT; ++u) {
        cr[u] = z1[u] ? a0 : b0;
        ci[u] = z1[u] ? a1 : b1;
      }
    } else {
      // Z strings reach outside the two bits: sum the terms with the partner's signs
      const int t0 = s.hops[k].t0, nt = s.hops[k].nt;
#pragma unroll
      for (int u = 0; u < kSecEPT; ++u) cr[u] = ci[u] = 0;
      for (int t = 0; t < nt; ++t) {
        const DevTerm tt = s.hterms[t0 + t];
        const R m0 = tm[t0 + t];
#pragma unroll
        for (int u = 0; u < kSecEPT; ++u) {
          const R m = (sw_popc((zs[u] ^ x) & (W)tt.z) & 1u) ? -m0 : m0;
          switch (tt.p & 3) {
            case 0: cr[u] += m; break;
            case 1: ci[u] += m; break;
            case 2: cr[u] -= m; break;
            default: ci[u] -= m; break;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kSecEPT; ++u) {
      cr[u] = act[u] ? cr[u] : R(0);
      ci[u] = act[u] ? ci[u] : R(0);
    }
    // gather into one buffer, then add the previous hop's term from the other,
    // whose gathers have had this hop's work to land
    if (par == 0) {
#pragma unroll
      for (int u = 0; u < kSecEPT; ++u) {
        pa.v[u] = src[gi[u]];
        pa.cr[u] = cr[u];
        pa.ci[u] = ci[u];
      }
      sector_hop_fma<R>(hr, hi, pb.v, pb.cr, pb.ci);
    } else {
#pragma unroll
      for (int u = 0; u < kSecEPT; ++u) {
        pb.v[u] = srcb[gi[u]];
        pb.cr[u] = cr[u];
        pb.ci[u] = ci[u];
      }
      sector_hop_fma<R>(hr, hi, pa.v, pa.cr, pa.ci);
    }
    par ^= 1;
  }
}

// five waves per SIMD where the registers allow it (complex64, 32-bit
// states), four otherwise, so that nothing spills
// DS: the diagonal is read from the sector's per-schedule parts (dstore >= 0)
// instead of summed from the terms
template <typename R, typename W, bool DS>
__global__ __launch_bounds__(kSecThreads) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 && sizeof(W) == 4 ? 5 : 4)))
void k_sector(const SectorArgs a) {
  using V = typename CT2<R>::V;
  __shared__ SecLds L;
  // the rank table, the hop coefficients (4 per hop), per-term values of the
  // other hops and one word per hop (bi | bj << 6 | chunk of bi << 12 | chunk
  // of bj << 15 | fast << 18 | run length << 19), sized to this sector at
  // launch (sector_dyn_lds_bytes) so that more workgroups share a compute unit
  extern __shared__ __align__(16) unsigned char smem[];
  const SectorDev& s = a.s;
  const int nrt = s.rwords;
  uint32_t* rtab = reinterpret_cast<uint32_t*>(smem);
  R* hc = reinterpret_cast<R*>(smem + sector_rtab_lds_bytes(s));
  R* tm = hc + 4 * s.nhops;
  uint32_t* hrec = reinterpret_cast<uint32_t*>(tm + s.nhterms);
  for (int i = threadIdx.x; i < nrt; i += kSecThreads) rtab[i] = s.rtab[i];
  for (int k = threadIdx.x; k < s.nhops; k += kSecThreads) {
    const SecHop hp = s.hops[k];
    hrec[k] = (uint32_t)hp.bi | ((uint32_t)hp.bj << 6) | ((uint32_t)(hp.bi / kSecChunkBits) << 12) |
              ((uint32_t)(hp.bj / kSecChunkBits) << 15) | ((uint32_t)(hp.fast != 0) << 18) |
              ((uint32_t)hp.group << 19);
  }
  sector_setup(a, L);
  sector_hop_setup<R>(s, L, tm, hc);
  __syncthreads();
  const V* __restrict__ src = reinterpret_cast<const V*>(a.src);
  // the same address, opaque to the compiler: the two pending buffers gather
  // through different pointers, so that their loads stay apart (merged into
  // one load, each would be copied into its buffer, waiting for the gather)
  const __attribute__((address_space(1))) V* srcg = (const __attribute__((address_space(1))) V*)src;
  asm("" : "+s"(srcg));
  const V* srcb = (const V*)srcg;
  const EpiDesc& e = a.epi;
  const bool has_comp = e.comp != nullptr;
  uint32_t* __restrict__ compv = reinterpret_cast<uint32_t*>(e.comp);
  const uint32_t last = (uint32_t)(s.dim - 1);
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;
  const int64_t per = (int64_t)kSecThreads * kSecEPT;
  for (int64_t base = (int64_t)blockIdx.x * per; base < s.dim; base += (int64_t)gridDim.x * per) {
    const int64_t rf = base + (int64_t)threadIdx.x * kSecEPT;
    W zs[kSecEPT];
    bool ok[kSecEPT];
    {
      // past the end a lane walks the last state (its results are dropped),
      // so that every table row it reads is one a weight-w state can reach
      W z = sector_unrank<W>(L.binom, s.n, s.w, min(rf, s.dim - 1));
#pragma unroll
      for (int u = 0; u < kSecEPT; ++u) {
        ok[u] = rf + u < s.dim;
        zs[u] = z;
        if (u + 1 < kSecEPT && rf + u + 1 < s.dim) z = next_same_weight(z);
      }
    }
    R hr[kSecEPT], hi[kSecEPT];
    SecPend<R> pa, pb;
    int par = 0;
#pragma unroll
    for (int u = 0; u < kSecEPT; ++u) {
      hr[u] = hi[u] = 0;
      pa.cr[u] = pa.ci[u] = pb.cr[u] = pb.ci[u] = 0;
      pa.v[u] = pb.v[u] = V{0, 0};
    }
    for (int g0 = 0; g0 < s.nhops;) {
      // the run length (host-built) is at least 1 and ends at the last hop; the
      // clamps keep the loop finite and the reads inside the hop table
      const int gn = min(s.nhops - g0, max(1, (int)(__builtin_amdgcn_readfirstlane(hrec[g0]) >> 19)));
      sector_group<R, W>(s, rtab, hrec, g0, gn, zs, ok, (uint32_t)rf, last, hc, tm, src, srcb, hr, hi, pa, pb,
                         par);
      g0 += gn;
    }
    // the last filled buffer
    if (par) sector_hop_fma<R>(hr, hi, pa.v, pa.cr, pa.ci);
    else sector_hop_fma<R>(hr, hi, pb.v, pb.cr, pb.ci);
    // epilogue: the same update as the last tile pass (see EpiDesc).  With
    // the diagonal kept per state, the streamed values of all the lane's
    // states are loaded before any is used (a state past the end reads the
    // last one; its results are dropped), so that no state's loads wait for
    // another's; with the summed diagonal, whose loop needs the registers,
    // state by state.  The low part is unpacked where it is used.
    // (load_state is the first form's; its diagonal parts are read there.)
    V uqv[kSecEPT], xinv[kSecEPT][4];
    uint32_t lop[kSecEPT];
    double dd[kSecEPT];
    auto load_state = [&](int u) {
      const int64_t g = min(rf + u, s.dim - 1);
      uqv[u] = src[g];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        xinv[u][i] = e.in[i] ? ldnt(reinterpret_cast<const V*>(e.in[i]) + g) : V{0, 0};
      lop[u] = has_comp ? __builtin_nontemporal_load(compv + g) : 0u;
      if constexpr (DS) {
        dd[u] = a.dconst;
#pragma unroll
        for (int k = 0; k < kSecDiagStore; ++k)
          if (k < s.dstore) dd[u] += a.dstore_f[k] * __builtin_nontemporal_load(s.dtab + k * s.dim + g);
      }
    };
    auto update_state = [&](int u) {
      const int64_t g = rf + u;
      const V uq = uqv[u];
      const double d = dd[u];
      const R hrr = (R)(d * (double)uq.x + (double)hr[u]);
      const R hii = (R)(d * (double)uq.y + (double)hi[u]);
      const V (&xin)[4] = xinv[u];
      const V lo = V{(R)bf16_lo(lop[u]), (R)bf16_hi(lop[u])};
#pragma unroll
      for (int o = 0; o < 3; ++o) {
        if (!e.out[o]) continue;
        R ir = (R)e.br[o] * hrr - (R)e.bi[o] * hii;
        R ii = (R)e.br[o] * hii + (R)e.bi[o] * hrr;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          ir += (R)e.a[o][i] * xin[i + 1].x;
          ii += (R)e.a[o][i] * xin[i + 1].y;
        }
        const R shh = (R)e.scale[o], sll = (R)(e.scale[o] - (double)shh);
        R vr = shh * ir + sll * ir;
        R vi = shh * ii + sll * ii;
        if (e.comp_flags & (1 << o)) {
          vr += lo.x;
          vi += lo.y;
        }
        const R bre = (R)e.c0[o] * xin[0].x + (R)e.cu[o] * uq.x;
        const R bim = (R)e.c0[o] * xin[0].y + (R)e.cu[o] * uq.y;
        const R sr = bre + vr, si = bim + vi;
        if (o == 0 && (e.comp_flags & 8)) {
          const R tr = sr - bre, ti = si - bim;
          const R er = (bre - (sr - tr)) + (vr - tr);
          const R ei = (bim - (si - ti)) + (vi - ti);
          __builtin_nontemporal_store(pack_bf16x2((float)er, (float)ei), compv + g);
        }
        stnt(reinterpret_cast<V*>(e.out[o]) + g, V{sr, si});
        if (o == 0) {
          if (e.red_flags & 1) r0 += (double)sr * (double)sr + (double)si * (double)si;
          if (e.red_flags & 2) {
            const double dr = (double)sr - (double)uq.x, di = (double)si - (double)uq.y;
            r1 += dr * dr + di * di;
          }
        }
      }
      if (e.red_flags & 4) r2 += (double)uq.x * (double)hrr + (double)uq.y * (double)hii;
    };
    if constexpr (DS) {
#pragma unroll
      for (int u = 0; u < kSecEPT; ++u) load_state(u);
#pragma unroll
      for (int u = 0; u < kSecEPT; ++u)
        if (ok[u]) update_state(u);
    } else {
#pragma unroll
      for (int u = 0; u < kSecEPT; ++u) {
        if (!ok[u]) continue;
        // the summed diagonal between the first load and the others, as its
        // loop needs the registers
        const int64_t g = rf + u;
        uqv[u] = src[g];
        dd[u] = sector_diag<W>(a, L, zs[u]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          xinv[u][i] = e.in[i] ? ldnt(reinterpret_cast<const V*>(e.in[i]) + g) : V{0, 0};
        lop[u] = has_comp ? __builtin_nontemporal_load(compv + g) : 0u;
        update_state(u);
      }
    }
  }
  if (e.red_flags) block_reduce3<kSecThreads>(r0, r1, r2, e.red_flags, L.red, e.red, gridDim.x, blockIdx.x);
}

// dynamic LDS of k_sector: the rank table, then 4 coefficients per hop, one
// value per hop term and one word per hop
static size_t sector_dyn_lds_bytes(const SectorDev& sd, int dtype) {
  return sector_rtab_lds_bytes(sd) +
         (size_t)(4 * sd.nhops + sd.nhterms) * (dtype == 0 ? sizeof(float) : sizeof(double)) +
         (size_t)sd.nhops * sizeof(uint32_t);
}

// the largest dynamic LDS of k_sector (34 qubits, weight 17, complex128, the
// most hops and hop terms) exceeds the default limit together with SecLds
static hipError_t set_sector_lds_attr() {
  SectorDev big{};
  big.n = kSecMaxN;
  big.w = kSecMaxN / 2;
  big.nch = kSecMaxChunks;
  big.rwords = kSecMaxChunks * (kSecMaxN + 3) << kSecChunkBits;
  big.nhops = kSecMaxHops;
  big.nhterms = kSecMaxHopTerms;
  const int dyn = (int)sector_dyn_lds_bytes(big, 1);
  const void* fns[8] = {reinterpret_cast<const void*>(&k_sector<float, uint32_t, false>),
                        reinterpret_cast<const void*>(&k_sector<float, uint64_t, false>),
                        reinterpret_cast<const void*>(&k_sector<double, uint32_t, false>),
                        reinterpret_cast<const void*>(&k_sector<double, uint64_t, false>),
                        reinterpret_cast<const void*>(&k_sector<float, uint32_t, true>),
                        reinterpret_cast<const void*>(&k_sector<float, uint64_t, true>),
                        reinterpret_cast<const void*>(&k_sector<double, uint32_t, true>),
                        reinterpret_cast<const void*>(&k_sector<double, uint64_t, true>)};
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_sector_matvec(const SectorArgs& a, int dtype, hipStream_t s) {
  if (a.s.nhops < 0 || a.s.nhops > kSecMaxHops || a.s.nhterms < 0 || a.s.nhterms > kSecMaxHopTerms ||
      a.s.nch < 1 || a.s.nch > kSecMaxChunks || a.s.w < 0 || a.s.w > kSecMaxN || a.s.rwords < 1 ||
      a.s.rwords > (kSecMaxChunks * (kSecMaxN + 3) << kSecChunkBits))
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)sector_blocks(a.s.dim)), block(kSecThreads);
  const size_t dyn = sector_dyn_lds_bytes(a.s, dtype);
  if (a.s.dstore > kSecDiagStore || (a.s.dstore > 0 && !a.s.dtab)) return hipErrorInvalidValue;
  // states of at most 32 qubits fit a 32-bit word
  const bool w32 = a.s.n <= 32;
  const bool ds = a.s.dstore >= 0;
  if (dtype == 0) {
    if (w32) {
      if (ds) hipLaunchKernelGGL((k_sector<float, uint32_t, true>), grid, block, dyn, s, a);
      else hipLaunchKernelGGL((k_sector<float, uint32_t, false>), grid, block, dyn, s, a);
    } else {
      if (ds) hipLaunchKernelGGL((k_sector<float, uint64_t, true>), grid, block, dyn, s, a);
      else hipLaunchKernelGGL((k_sector<float, uint64_t, false>), grid, block, dyn, s, a);
    }
  } else {
    if (w32) {
      if (ds) hipLaunchKernelGGL((k_sector<double, uint32_t, true>), grid, block, dyn, s, a);
      else hipLaunchKernelGGL((k_sector<double, uint32_t, false>), grid, block, dyn, s, a);
    } else {
      if (ds) hipLaunchKernelGGL((k_sector<double, uint64_t, true>), grid, block, dyn, s, a);
      else hipLaunchKernelGGL((k_sector<double, uint64_t, false>), grid, block, dyn, s, a);
    }
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(kSecThreads) void k_sector_dtab(const SectorArgs a, double* out) {
  __shared__ SecLds L;
  sector_setup(a, L);
  const SectorDev& s = a.s;
  const int64_t per = (int64_t)kSecThreads * kSecEPT;
  for (int64_t base = (int64_t)blockIdx.x * per; base < s.dim; base += (int64_t)gridDim.x * per) {
    const int64_t rf = base + (int64_t)threadIdx.x * kSecEPT;
    if (rf >= s.dim) continue;
    uint64_t z = sector_unrank(L.binom, s.n, s.w, rf);
    for (int u = 0; u < kSecEPT && rf + u < s.dim; ++u) {
      if (u > 0) z = next_same_weight(z);
      out[rf + u] = sector_diag(a, L, z);
    }
  }
}

hipError_t launch_sector_dtab(const SectorArgs& a, double* out, hipStream_t s) {
  const dim3 grid((unsigned)sector_blocks(a.s.dim)), block(kSecThreads);
  hipLaunchKernelGGL(k_sector_dtab, grid, block, 0, s, a, out);
  return hipGetLastError();
}

template <typename V>
__global__ __launch_bounds__(kSecThreads) void k_sector_diag(const SectorArgs a, int mode, double thr,
                                                             const V* psi, double* parts) {
  __shared__ SecLds L;
  sector_setup(a, L);
  const SectorDev& s = a.s;
  double mn = INFINITY, mx = -INFINITY, ms = 0.0;
  const int64_t per = (int64_t)kSecThreads * kSecEPT;
  for (int64_t base = (int64_t)blockIdx.x * per; base < s.dim; base += (int64_t)gridDim.x * per) {
    const int64_t rf = base + (int64_t)threadIdx.x * kSecEPT;
    if (rf >= s.dim) continue;
    uint64_t z = sector_unrank(L.binom, s.n, s.w, rf);
    for (int u = 0; u < kSecEPT && rf + u < s.dim; ++u) {
      if (u > 0) z = next_same_weight(z);
      const double d = sector_diag(a, L, z);
      if (mode == 0) {
        mn = fmin(mn, d);
        mx = fmax(mx, d);
      } else if (d <= thr) {
        const V v = psi[rf + u];
        ms += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
      }
    }
  }
  if (mode == 1) {
    block_reduce3<kSecThreads>(ms, 0.0, 0.0, 1, L.red, parts, gridDim.x, blockIdx.x);
    return;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o, 64));
    mx = fmax(mx, __shfl_xor(mx, o, 64));
  }
  constexpr int NW = kSecThreads / 64;
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    L.red[wv] = mn;
    L.red[NW + wv] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < NW; ++k) {
      mn = fmin(mn, L.red[k]);
      mx = fmax(mx, L.red[NW + k]);
    }
    parts[blockIdx.x] = mn;
    parts[gridDim.x + blockIdx.x] = mx;
  }
}

hipError_t launch_sector_diag(const SectorArgs& a, int mode, double thr, const void* psi, int dtype,
                              double* parts, hipStream_t s) {
  const dim3 grid((unsigned)sector_blocks(a.s.dim)), block(kSecThreads);
  if (dtype == 0)
    hipLaunchKernelGGL(k_sector_diag<float2>, grid, block, 0, s, a, mode, thr, (const float2*)psi,
                       parts);
  else
    hipLaunchKernelGGL(k_sector_diag<double2>, grid, block, 0, s, a, mode, thr, (const double2*)psi,
                       parts);
  return hipGetLastError();
}

template <typename V>
__global__ __launch_bounds__(kSecThreads) void k_sector_expand(const SectorDev s, const V* sec, V* full) {
  __shared__ uint32_t binom[kSecBinom * kSecBinom];
  for (int i = threadIdx.x; i < kSecBinom * kSecBinom; i += kSecThreads) binom[i] = s.binom[i];
  __syncthreads();
  for (int64_t r = (int64_t)blockIdx.x * kSecThreads + threadIdx.x; r < s.dim;
       r += (int64_t)gridDim.x * kSecThreads)
    full[sector_unrank(binom, s.n, s.w, r)] = sec[r];
}

hipError_t launch_sector_expand(const SectorDev& sd, const void* sec, void* full, int dtype,
                                hipStream_t s) {
  int64_t nb = (sd.dim + kSecThreads - 1) / kSecThreads;
  if (nb > 65536) nb = 65536;
  if (dtype == 0)
    hipLaunchKernelGGL(k_sector_expand<float2>, dim3((unsigned)nb), dim3(kSecThreads), 0, s, sd,
                       (const float2*)sec, (float2*)full);
  else
    hipLaunchKernelGGL(k_sector_expand<double2>, dim3((unsigned)nb), dim3(kSecThreads), 0, s, sd,
                       (const double2*)sec, (double2*)full);
  return hipGetLastError();
}

template <typename V>
__global__ void k_fill(V* y, int64_t N, V v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}

hipError_t launch_fill(void* y, int dtype, int64_t N, double re, double im, hipStream_t s) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_fill<float2>, dim3(ew_blocks(N)), dim3(256), 0, s, (float2*)y, N,
                       float2{(float)re, (float)im});
  else
    hipLaunchKernelGGL(k_fill<double2>, dim3(ew_blocks(N)), dim3(256), 0, s, (double2*)y, N,
                       double2{re, im});
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Lanczos basis operations (lowest eigenvalues of H(t), Sec. IV.B).  Every
// sum is formed in float64; the basis vectors keep the state's type.
// ---------------------------------------------------------------------------
int64_t lz_blocks(int64_t N) {
  int64_t nb = (N + (int64_t)kRedThreads * 8 - 1) / ((int64_t)kRedThreads * 8);
  return nb < 1 ? 1 : (nb > 4096 ? 4096 : nb);
}

// blockIdx.y picks a group of kLzGroup basis vectors
template <typename V>
__global__ __launch_bounds__(kRedThreads) void k_multidot(const V* base, int64_t stride, int64_t N, int k,
                                                          const V* w, double* parts) {
  __shared__ double sb[2 * kLzGroup * (kRedThreads / 64)];
  const int j0 = blockIdx.y * kLzGroup;
  const int ng = min(kLzGroup, k - j0);
  double re[kLzGroup], im[kLzGroup];
#pragma unroll
  for (int j = 0; j < kLzGroup; ++j) re[j] = im[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kRedThreads) {
    const V b = w[i];
#pragma unroll
    for (int j = 0; j < kLzGroup; ++j) {
      if (j < ng) {
        const V a = base[(int64_t)(j0 + j) * stride + i];
        re[j] += (double)a.x * (double)b.x + (double)a.y * (double)b.y;
        im[j] += (double)a.x * (double)b.y - (double)a.y * (double)b.x;
      }
    }
  }
  constexpr int NW = kRedThreads / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kLzGroup; ++j) {
    const double r = wave_sum(re[j]), q = wave_sum(im[j]);
    if (lane == 0) {
      sb[(2 * j) * NW + wv] = r;
      sb[(2 * j + 1) * NW + wv] = q;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * ng) {
    double acc = 0.0;
    for (int v = 0; v < NW; ++v) acc += sb[threadIdx.x * NW + v];
    parts[(int64_t)(2 * j0 + threadIdx.x) * gridDim.x + blockIdx.x] = acc;
  }
}

hipError_t launch_multidot(const void* base, int64_t stride, int64_t N, int k, const void* w, int dtype,
                           double* parts, hipStream_t s) {
  const dim3 grid((unsigned)lz_blocks(N), (unsigned)((k + kLzGroup - 1) / kLzGroup));
  if (dtype == 0)
    hipLaunchKernelGGL(k_multidot<float2>, grid, dim3(kRedThreads), 0, s, (const float2*)base, stride, N,
                       k, (const float2*)w, parts);
  else
    hipLaunchKernelGGL(k_multidot<double2>, grid, dim3(kRedThreads), 0, s, (const double2*)base, stride,
                       N, k, (const double2*)w, parts);
  return hipGetLastError();
}

template <typename V>
__global__ __launch_bounds__(kRedThreads) void k_multiaxpy(const V* base, int64_t stride, int64_t N,
                                                           int k, const double* c, V* w, double* parts) {
  __shared__ double cs[2 * kLzMaxBasis];
  __shared__ double sb[3 * (kRedThreads / 64)];
  if (threadIdx.x < 2 * k) cs[threadIdx.x] = c[threadIdx.x];
  __syncthreads();
  double nrm = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kRedThreads) {
    const V b = w[i];
    double xr = (double)b.x, xi = (double)b.y;
    for (int j = 0; j < k; ++j) {
      const V a = base[(int64_t)j * stride + i];
      const double cr = cs[2 * j], ci = cs[2 * j + 1];
      xr -= cr * (double)a.x - ci * (double)a.y;
      xi -= cr * (double)a.y + ci * (double)a.x;
    }
    const V o{(decltype(b.x))xr, (decltype(b.x))xi};
    w[i] = o;
    nrm += (double)o.x * (double)o.x + (double)o.y * (double)o.y;
  }
  block_reduce3<kRedThreads>(nrm, 0.0, 0.0, 1, sb, parts, gridDim.x, blockIdx.x);
}

hipError_t launch_multiaxpy(const void* base, int64_t stride, int64_t N, int k, const double* c, void* w,
                            int dtype, double* parts, hipStream_t s) {
  const dim3 grid((unsigned)lz_blocks(N));
  if (dtype == 0)
    hipLaunchKernelGGL(k_multiaxpy<float2>, grid, dim3(kRedThreads), 0, s, (const float2*)base, stride, N,
                       k, c, (float2*)w, parts);
  else
    hipLaunchKernelGGL(k_multiaxpy<double2>, grid, dim3(kRedThreads), 0, s, (const double2*)base, stride,
                       N, k, c, (double2*)w, parts);
  return hipGetLastError();
}

template <typename V, typename R>
__global__ void k_scale_copy(V* dst, const V* src, int64_t N, double a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    const V v = src[i];
    dst[i] = V{(R)((double)v.x * a), (R)((double)v.y * a)};
  }
}

hipError_t launch_scale_copy(void* dst, const void* src, int dtype, int64_t N, double a, hipStream_t s) {
  if (dtype == 0)
    hipLaunchKernelGGL((k_scale_copy<float2, float>), dim3(ew_blocks(N)), dim3(256), 0, s, (float2*)dst,
                       (const float2*)src, N, a);
  else
    hipLaunchKernelGGL((k_scale_copy<double2, double>), dim3(ew_blocks(N)), dim3(256), 0, s,
                       (double2*)dst, (const double2*)src, N, a);
  return hipGetLastError();
}

// One wave per workgroup; a lane stages the m components of its row in LDS,
// then writes the kk combinations over the first kk vectors (each row is read
// completely before any of its outputs is written).
constexpr int kLzTfThreads = 64;
template <typename V>
__global__ __launch_bounds__(kLzTfThreads) void k_basis_transform(V* base, int64_t stride, int64_t N, int m,
                                                                  int kk, const double* Y) {
  __shared__ V row[kLzMaxBasis * kLzTfThreads];
  __shared__ double ys[2 * kLzMaxBasis * kLzMaxKeep];
  for (int i = threadIdx.x; i < 2 * m * kk; i += kLzTfThreads) ys[i] = Y[i];
  __syncthreads();
  for (int64_t r = (int64_t)blockIdx.x * kLzTfThreads + threadIdx.x; r < N;
       r += (int64_t)gridDim.x * kLzTfThreads) {
    for (int j = 0; j < m; ++j) row[j * kLzTfThreads + threadIdx.x] = base[(int64_t)j * stride + r];
    for (int i = 0; i < kk; ++i) {
      double xr = 0.0, xi = 0.0;
      for (int j = 0; j < m; ++j) {
        const V a = row[j * kLzTfThreads + threadIdx.x];
        const double yr = ys[2 * (j * kk + i)], yi = ys[2 * (j * kk + i) + 1];
        xr += (double)a.x * yr - (double)a.y * yi;
        xi += (double)a.x * yi + (double)a.y * yr;
      }
      base[(int64_t)i * stride + r] = V{(decltype(V{}.x))xr, (decltype(V{}.x))xi};
    }
  }
}

hipError_t launch_basis_transform(void* base, int64_t stride, int64_t N, int m, int kk, const double* Y,
                                  int dtype, hipStream_t s) {
  int64_t nb = (N + kLzTfThreads - 1) / kLzTfThreads;
  if (nb > 8192) nb = 8192;
  if (dtype == 0)
    hipLaunchKernelGGL(k_basis_transform<float2>, dim3((unsigned)nb), dim3(kLzTfThreads), 0, s,
                       (float2*)base, stride, N, m, kk, Y);
  else
    hipLaunchKernelGGL(k_basis_transform<double2>, dim3((unsigned)nb), dim3(kLzTfThreads), 0, s,
                       (double2*)base, stride, N, m, kk, Y);
  return hipGetLastError();
}

// splitmix64 (Steele, Lea and Flood 2014) of the element index
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

template <typename V, typename R>
__global__ void k_random_fill(V* y, int64_t N, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t a = splitmix64(seed ^ (2ull * (uint64_t)i));
    const uint64_t b = splitmix64(seed ^ (2ull * (uint64_t)i + 1ull));
    const double ur = (double)(a >> 11) * (1.0 / 9007199254740992.0);
    const double ui = (double)(b >> 11) * (1.0 / 9007199254740992.0);
    y[i] = V{(R)(2.0 * ur - 1.0), (R)(2.0 * ui - 1.0)};
  }
}

hipError_t launch_random_fill(void* y, int dtype, int64_t N, uint64_t seed, hipStream_t s) {
  if (dtype == 0)
    hipLaunchKernelGGL((k_random_fill<float2, float>), dim3(ew_blocks(N)), dim3(256), 0, s, (float2*)y, N,
                       seed);
  else
    hipLaunchKernelGGL((k_random_fill<double2, double>), dim3(ew_blocks(N)), dim3(256), 0, s,
                       (double2*)y, N, seed);
  return hipGetLastError();
}

}  // namespace aqc
