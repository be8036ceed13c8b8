// Internal interface between the host runtime (aqc_host.cpp) and the HIP
// kernels (aqc_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/aqc.h"

namespace aqc {

constexpr int kMaxSched = 32;       // schedules per Hamiltonian
constexpr int kMaxDiagSched = kMaxSched;  // schedules with split diagonal tables
constexpr int kMaxTabSched = kMaxSched;  // schedules with a low-bit diagonal table
constexpr int kMaxPassGroups = 256;
constexpr int kMaxPassTerms = 512;
constexpr int kThreads = 512;       // threads per tile workgroup
constexpr int kRedThreads = 256;    // threads per reduction workgroup

// One Pauli term inside a flip group or the residual diagonal list.
// The operator is w * f_sid(t) * i^p * X^x Z^z with p = popc(x & z) mod 4
// (sigma^y = i sigma^x sigma^z on each qubit that carries it).
struct DevTerm {
  uint64_t z;
  double w;
  int32_t sid;
  int32_t p;
};

// All terms sharing one flip pattern x.  (H psi)[g] gets
// c_x(g) psi[g ^ x] with c_x(g) = sum_t m_t i^{p_t} (-1)^{popc((g ^ x) & z_t)}.
struct DevGroup {
  uint64_t x;      // global flip mask
  uint32_t xl;     // the same mask in tile-local coordinates
  int32_t t0;      // first term (index into the pass's term array)
  int32_t nt;      // number of terms
  int32_t plain;   // 1: all z_t = 0 and p_t = 0, so c_x is one real number
  int32_t fslot;   // >= 0: x flips one or two bits bi <= bj and every z_t lies
                   // inside x, so c_x depends only on the source's bits bi,
                   // bj: a 4-entry table, slot fslot of the pass (else -1)
  int32_t bij;     // bi | bj << 8 (fast groups)
  int32_t lij;     // li | lj << 8: the tile-local positions of bi and bj (fast
                   // groups inside the tile)
};
// fast-group tables per pass: 4 complex values each, in the LDS bytes of the
// per-term float64 coefficients (free once the set-up has used them)
constexpr int kFastSlotsC64 = 128;
constexpr int kFastSlotsC128 = 64;

// Diagonal part split for a tile of `tb` low bits ("lo") and the remaining
// high bits ("hi"): E_s(g) = CT_s[hi] + sum_{i<tb} LT_s[hi][i] (-1)^{lo_i}
//                           + TAB_s[lo] + (residual terms, evaluated directly).
struct DiagDev {
  int32_t nsd;                  // schedules with CT/LT tables
  int32_t sd_sid[kMaxDiagSched];
  int32_t ntab;                 // schedules with a TAB table
  int32_t tab_sid[kMaxTabSched];
  int32_t nres;                 // residual terms
  int32_t pad;
  const double* CT;             // [nsd][2^(n-tb)]
  const double* LT;             // [nsd][2^(n-tb)][tb]
  const double* TAB64;          // [ntab][2^tb]
  const DevTerm* res;           // [nres]
};

// Epilogue of the last pass.  With Hv = ((H - c) u)[g], u the tile value and
// in_1..in_3 streamed inputs, output j is
//   out_j = c0_j in_0 + cu_j u + scale_j (sum_i a_j[i] in_{i+1} + (br_j + i bi_j) Hv)
// The weights c0, cu, a, br, bi are small integers (exact in float32); the
// step-size factor scale_j is applied as a float-float pair in complex64
// kernels, so the integrator's weights carry no float32 rounding.
// Compensated state (complex64): `comp` holds the low part y_lo of in_0 = y.
// Bit j of comp_flags (j < 3) adds y_lo to out_j's increment; bit 3 makes
// out_0 = in_0 + increment an exact two-sum whose error is written back to
// comp.  Reductions (float64, per workgroup):
//   red0 = sum |out_0|^2, red1 = sum |out_0 - u|^2, red2 = sum Re(conj(u) Hv).
struct EpiDesc {
  const void* in[4];
  void* out[3];
  void* comp;
  double c0[3];
  double cu[3];
  double a[3][3];
  double br[3];
  double bi[3];
  double scale[3];
  double* red;        // [3][nblocks] partial sums or nullptr
  int32_t red_flags;  // bit0 red0, bit1 red1, bit2 red2
  int32_t comp_flags;
};

struct PassArgs {
  int32_t n;          // qubits
  int32_t tb;         // tile bits
  int32_t lbits;      // contiguous low bits of the tile
  int32_t final_pass; // 1: add the diagonal, read acc_in, run the epilogue
  uint64_t hmask;     // high bits of the tile (outside [0, lbits))
  uint64_t cmask;     // bits outside the tile (enumerate the workgroups)
  const void* src;    // tile source vector u
  const DevGroup* groups;
  const DevTerm* terms;
  int32_t ng;
  int32_t nterms;
  double f[kMaxSched];   // schedule values at this time
  double dconst;         // constant added to the diagonal (identity terms - shift)
  DiagDev dg;
  const void* acc_in;    // partial H u from earlier passes (or nullptr)
  void* acc_out;         // high passes: partial H u written here
  EpiDesc epi;
};

// Register hypercube pass: single-qubit flips (real coefficients) on the bits
// [hb, hb + RB + wb), with RB = kRegBitsC64 / kRegBitsC128 and wb = 0 or
// kWaveBits.  A wave owns 64 contiguous amplitudes (one per lane) at each
// vertex of the hypercube over [hb, hb + RB); with wb > 0 the 2^wb waves of a
// workgroup span the next wb bits and exchange vertices through LDS.
constexpr int kRegBitsC64 = 6;
constexpr int kRegBitsC128 = 5;
constexpr int kWaveBits = 3;
struct RegPassArgs {
  int32_t n;
  int32_t hb;
  int32_t wb;
  int32_t pad;
  const void* src;
  const void* acc_in;
  void* acc_out;
  double cb[12];      // coefficient of the flip of bit hb + b
};

// ---- Hamming-weight sector ---------------------------------------------------
// A state of the sector of weight w holds the C(n, w) amplitudes of the basis
// states with w one-bits, at the rank r(z) = sum_k C(p_k, k + 1) over the set
// bits p_0 < p_1 < ... of z (increasing order of z).  Ranks fit in 32 bits for
// n <= 34.
constexpr int kSecThreads = 256;
constexpr int kSecEPT = 2;          // consecutive ranks per thread and chunk
constexpr int kSecMaxN = 34;
constexpr int kSecBinom = 35;       // binomial table C(p, k), p, k <= 34
constexpr int kSecChunkBits = 6;    // bits per chunk of the rank table
constexpr int kSecMaxChunks = 6;    // chunks of at most kSecMaxN bits
constexpr int kSecMaxHopTerms = 1024;
constexpr int kSecGrid = 3840;      // at most this many workgroups per launch: three rounds of
                                     // 256 compute units x 5 resident workgroups of k_sector

// A weight-preserving flip of two bits and its terms (as DevGroup).
struct SecHop {
  uint64_t x;
  int32_t t0, nt;
  int32_t bi, bj;  // the two flipped bits, bi < bj
  int32_t fast;    // 1: every Z string lies inside x, so the coefficient of
                   // a state with differing bits depends only on bit bi
  int32_t group;   // hops are sorted by their chunks (bi / 6, bj / 6); the
                   // first hop of each run of equal chunk pairs holds the
                   // run's length, the others 0
};
constexpr int kSecMaxHops = 600;
// A sector whose diagonal terms use at most this many schedules keeps its
// diagonal per state, split by schedule, when that takes at most
// kSecDiagStoreBytes of device memory.
constexpr int kSecDiagStore = 2;
constexpr size_t kSecDiagStoreBytes = size_t(16) << 30;
// The diagonal terms sharing one mask of one or two bits (q < 0: one bit p).
struct SecMask {
  int32_t p, q;
  int32_t t0, nt;
};
struct SectorDev {
  int32_t n, w;
  int32_t zero_bits;   // 1: the diagonal is summed over the 0-bits of z
  int32_t nch;         // 6-bit chunks of n
  int32_t rwords;      // words of the rank table
  int32_t cbase[kSecMaxChunks];  // word offset of chunk c's row for 0 1-bits below it
  int32_t nhops, nhterms;
  int32_t nmasks, nres;
  int64_t dim;         // C(n, w)
  const uint32_t* binom;   // [kSecBinom][kSecBinom]
  const uint32_t* rtab;    // per chunk, rows of 64 words (one per 6-bit pattern) for the counts of
                           // 1-bits below it that a weight-w state can have, plus one spare row
                           // on each side: the rank part of the chunk's pattern given that count
  const SecHop* hops;
  const DevTerm* hterms;
  const SecMask* masks;
  const DevTerm* mterms;
  const DevTerm* res;      // diagonal terms with three or more bits
  // the diagonal kept per state: -1 not kept (summed from the terms per
  // state), else the number of schedules of the diagonal terms (0: none)
  int32_t dstore;
  int32_t dstore_sid[kSecDiagStore];
  const double* dtab;      // [dstore][dim]: the part under schedule dstore_sid[k]
};
struct SectorArgs {
  SectorDev s;
  const void* src;
  double f[kMaxSched];
  double dconst;       // identity terms minus the shift
  double dstore_f[kSecDiagStore];   // f[dstore_sid[k]]
  EpiDesc epi;
};

// ---- schedules and the segment stepper (shared by host and device) ---------
// Coefficient schedules (end of Sec. II.A) evaluated at time t, and the walk
// over the H|psi> evaluations of a fixed-step segment (Sec. II.B).  The host
// runs them for aqc_evolve and the batch engine's ticks; the resident batch
// kernel runs the same code on the device.
__host__ __device__ inline double path_s(const aqc_path& p, double t) {
  if (p.kind == AQC_PATH_LINEAR) return t / p.T;
  const double v = sin(3.14159265358979323846 * t / (2.0 * p.T));
  return v * v;
}

__host__ __device__ inline double sched_value(const aqc_sched& s, const aqc_path& p, double t) {
  switch (s.kind) {
    case AQC_SCHED_CONST:
      return 1.0;
    case AQC_SCHED_POLY_S: {
      const double x = path_s(p, t);
      const bool inside = x >= s.s_lo && (s.hi_closed ? x <= s.s_hi : x < s.s_hi);
      if (!inside) return 0.0;
      double v = 0.0, pw = 1.0;
      for (int d = 0; d <= s.degree; ++d) {
        v += s.coef[d] * pw;
        pw *= x;
      }
      return v;
    }
    case AQC_SCHED_PWL_S: {
      const double x = path_s(p, t);
      const double* k = s.coef;   // (s_i, v_i) pairs
      if (x < k[0]) return k[1];
      for (int i = 0; i < s.degree; ++i) {
        // here x >= s_i; the first knot above x bounds its segment
        if (x < k[2 * i + 2])
          return k[2 * i + 1] + (k[2 * i + 3] - k[2 * i + 1]) * (x - k[2 * i]) / (k[2 * i + 2] - k[2 * i]);
      }
      return k[2 * s.degree + 1];
    }
    default:
      return s.amp * cos(s.omega * t + s.phase);
  }
}


// Vectors of one running solve (device pointers; see aqc_evolve's workspace).
struct SolveVecs {
  void* y;       // the caller's state
  void* yp;      // y^p (pc4) or the RK4 stage input u
  void* yp2;     // second y^p buffer when the last pass reads other tiles of
                 // its source (stream groups), so no stage updates it in place
  void* B[4];    // f history (pc4, rotating); RK4 accumulator: B[3] (pc4 bootstrap) or B[0]
  void* hbuf;    // partial product of the high passes
  void* ycomp;   // complex64 compensated state: low part of y, or nullptr
};

// One H|psi> of a fixed-step segment: time, tile source and stage update.
struct MatvecStage {
  double t;
  const void* src;
  EpiDesc e;
  bool ends_step;  // completes an integration step
  bool pc4;        // a predictor-corrector step (Milne estimate defined)
};

// Walks the matvecs of a segment on the grid t_s + k h.  pc4: RK4 steps for
// k = 0, 1, 2 (their first stages are f_0..f_2), then one evaluation at t_3 that
// also forms the first prediction y^p_4, then one H|psi> per step.  The same
// sequence serves aqc_evolve and the batch engine, so a solve performs the
// same launches alone and in a batch.
struct SegStepper {
  int method = AQC_METHOD_PC4;
  double ts = 0, h = 0;
  int64_t k = 0;      // steps done
  int sub = 0;        // RK4 stage 0..3; 4 = evaluation at t_3 pending (pc4)
  int64_t k_end = 0;  // stop when k reaches this
  bool more_after = false;  // the segment continues after k_end
  bool dbl = false;   // y^p alternates between yp and yp2
  int ypc = 0;        // which buffer holds the current y^p

  __host__ __device__ bool rk_phase() const { return method == AQC_METHOD_RK4 || (k < 3 && sub < 4); }
  __host__ __device__ void* yp_cur(const SolveVecs& v) const { return (dbl && ypc) ? v.yp2 : v.yp; }
  __host__ __device__ void* yp_next(const SolveVecs& v) const { return dbl ? (ypc ? v.yp : v.yp2) : v.yp; }
  // the stage next() describes reads y^p and writes its successor
  __host__ __device__ bool swaps_yp() const {
    if (rk_phase()) return sub == 1 || sub == 2;
    if (sub == 4) return false;
    return k + 1 < k_end || more_after;
  }

  __host__ __device__ MatvecStage next(const SolveVecs& v) const {
    MatvecStage m;
    m.e = EpiDesc{};
    m.ends_step = false;
    m.pc4 = false;
    const int lo_in = v.ycomp ? 1 : 0;
    EpiDesc& e = m.e;
    e.comp = v.ycomp;
    const double tk = ts + (double)k * h;
    if (rk_phase()) {
      void* fk = method == AQC_METHOD_PC4 ? v.B[k & 3] : nullptr;
      void* acc = method == AQC_METHOD_PC4 ? v.B[3] : v.B[0];
      if (sub == 0) {  // acc (or f_k) = F, u = y + h/2 F
        m.t = tk;
        m.src = v.y;
        e.out[0] = fk ? fk : acc;
        e.scale[0] = 1.0;
        e.bi[0] = -1.0;
        e.out[1] = yp_cur(v);
        e.cu[1] = 1.0;
        e.scale[1] = 0.5 * h;
        e.bi[1] = -1.0;
        e.comp_flags = lo_in << 1;
      } else if (sub <= 2) {  // acc = acc_in + 2F, u = y + c h F
        m.t = tk + 0.5 * h;
        m.src = yp_cur(v);
        e.in[0] = v.y;
        e.in[1] = (sub == 1 && fk) ? fk : acc;
        e.out[0] = acc;
        e.scale[0] = 1.0;
        e.a[0][0] = 1.0;
        e.bi[0] = -2.0;
        e.out[1] = yp_next(v);
        e.c0[1] = 1.0;
        e.scale[1] = sub == 1 ? 0.5 * h : h;
        e.bi[1] = -1.0;
        e.comp_flags = lo_in << 1;
      } else {  // y = y + h/6 (acc + F)
        m.t = tk + h;
        m.src = yp_cur(v);
        e.in[0] = v.y;
        e.in[1] = acc;
        e.out[0] = v.y;
        e.c0[0] = 1.0;
        e.scale[0] = h / 6.0;
        e.a[0][0] = 1.0;
        e.bi[0] = -1.0;
        e.comp_flags = v.ycomp ? (1 | 8) : 0;
        m.ends_step = true;
      }
      return m;
    }
    if (sub == 4) {
      // f_3 = F(t_3, y_3) and y^p_4 = y_3 + h/24 (55 f_3 - 59 f_2 + 37 f_1 - 9 f_0)
      m.t = ts + 3.0 * h;
      m.src = v.y;
      e.out[0] = v.B[3];
      e.scale[0] = 1.0;
      e.bi[0] = -1.0;
      e.in[0] = v.y;
      e.in[1] = v.B[2];
      e.in[2] = v.B[1];
      e.in[3] = v.B[0];
      e.out[1] = yp_cur(v);
      e.c0[1] = 1.0;
      e.scale[1] = h / 24.0;
      e.a[1][0] = -59.0;
      e.a[1][1] = 37.0;
      e.a[1][2] = -9.0;
      e.bi[1] = -55.0;
      e.comp_flags = lo_in << 1;
      return m;
    }
    // predictor-corrector step k -> k+1: one H|psi> at t_{k+1} on y^p_{k+1}
    const double c = h / 24.0;
    m.t = ts + (double)(k + 1) * h;
    m.src = yp_cur(v);
    m.ends_step = true;
    m.pc4 = true;
    e.in[0] = v.y;
    e.in[1] = v.B[k & 3];        // f_k
    e.in[2] = v.B[(k - 1) & 3];  // f_{k-1}
    e.in[3] = v.B[(k - 2) & 3];  // f_{k-2}
    e.out[0] = v.y;              // y_{k+1} = y_k + h/24 (9 F + 19 f_k - 5 f_{k-1} + f_{k-2})
    e.c0[0] = 1.0;
    e.scale[0] = c;
    e.a[0][0] = 19.0;
    e.a[0][1] = -5.0;
    e.a[0][2] = 1.0;
    e.bi[0] = -9.0;
    e.out[1] = v.B[(k + 1) & 3];  // f_{k+1} = F over f_{k-3}
    e.scale[1] = 1.0;
    e.bi[1] = -1.0;
    if (k + 1 < k_end || more_after) {
      e.out[2] = yp_next(v);  // y^p_{k+2} = y_k + h/24 (64 F - 40 f_k + 32 f_{k-1} - 8 f_{k-2})
      e.c0[2] = 1.0;
      e.scale[2] = c;
      e.a[2][0] = -40.0;
      e.a[2][1] = 32.0;
      e.a[2][2] = -8.0;
      e.bi[2] = -64.0;
    }
    e.comp_flags = v.ycomp ? (1 | 8 | 4) : 0;
    return m;
  }

  __host__ __device__ void advance() {
    if (dbl && swaps_yp()) ypc ^= 1;
    if (rk_phase()) {
      if (sub < 3) {
        ++sub;
        return;
      }
      sub = 0;
      ++k;
      // the pc4 bootstrap ends with the evaluation at t_3 when a pc4 step follows
      if (method == AQC_METHOD_PC4 && k == 3 && (k < k_end || more_after)) sub = 4;
      return;
    }
    if (sub == 4) {
      sub = 0;
      return;
    }
    ++k;
  }
};


// H|psi> evaluations a fixed-step pc4 solve of K steps takes
__host__ __device__ inline int64_t pc4_matvecs(int64_t K) { return K <= 3 ? 4 * K : 12 + 1 + (K - 3); }

// ---- resident solves of a batch (one workgroup runs a whole solve) ---------
// A small solve is run start to end by one workgroup of one launch: the
// workgroup walks the segment stepper, evaluates the schedules at each
// stage's time and applies every tile pass of its plan tile by tile, with
// workgroup barriers only (no other workgroup touches its vectors).
constexpr int kResMaxPass = 4;
struct ResPass {
  int64_t nblocks;    // tiles of the pass
  PassArgs pa;        // every field that does not depend on the stage
};
struct ResidentSolve {
  int32_t n, npass, nsched, dbl;
  aqc_path path;
  double shift, t0, t1, h;
  int64_t K;
  double ident_w[kMaxSched];   // identity terms: weight per schedule
  aqc_sched sched[kMaxSched];
  SolveVecs v;
  ResPass pass[kResMaxPass];
};

// ---- fixed device scratch (allocation-free entry point) ----------------------
// A file-scope device array in aqc_kernels.hip, one copy per GPU, held until
// the process ends.  aqc_energy_noalloc keeps the partial product of the high
// passes in the first kScratchVecBytes (a state of up to 2^22 complex64 or
// 2^21 complex128 amplitudes) and the per-workgroup reduction partials in the
// remaining kScratchPartBytes.
constexpr size_t kScratchVecBytes = (size_t)32 << 20;
constexpr size_t kScratchPartBytes = (size_t)1 << 20;
constexpr size_t kScratchBytes = kScratchVecBytes + kScratchPartBytes;
// device address of the scratch array on the current device
hipError_t scratch_address(void** p);

// ---- launchers (aqc_kernels.hip) -------------------------------------------
hipError_t launch_regpass(const RegPassArgs& a, int dtype, hipStream_t s);
// workgroups of a register pass over n qubits
int64_t regpass_blocks(int n, int wb, int dtype);
// batched forms: block b serves args[bmap[b].x] at local block bmap[b].y
hipError_t launch_regpass_batch(const RegPassArgs* args, const int2* bmap, int64_t nblocks, int wb,
                                int dtype, hipStream_t s);
hipError_t launch_pass_batch(const PassArgs* args, const int2* bmap, int64_t nblocks, int final_pass,
                             int max_tb, int dtype, hipStream_t s);
hipError_t launch_pass(const PassArgs& a, int dtype, int64_t nblocks, hipStream_t s);
// the batched launches as graph nodes after `dep` (nullptr: a root node)
hipError_t add_regpass_batch_node(hipGraph_t g, hipGraphNode_t* node, hipGraphNode_t dep,
                                  const RegPassArgs* args, const int2* bmap, int64_t nblocks, int wb,
                                  int dtype);
hipError_t add_pass_batch_node(hipGraph_t g, hipGraphNode_t* node, hipGraphNode_t dep,
                               const PassArgs* args, const int2* bmap, int64_t nblocks, int final_pass,
                               int max_tb, int dtype);
size_t pass_lds_bytes(int tb, int dtype);
hipError_t prepare_kernels();
// resident solves: workgroup b runs solves[b] to its end (max_tb: largest
// tile of their tile passes, which sizes the dynamic LDS)
hipError_t launch_resident(const ResidentSolve* solves, int count, int max_tb, int dtype, hipStream_t s);

// red: per-block partials [k][nblocks] -> out[k] (k < nk), fixed-order sum
hipError_t launch_reduce_sum(const double* parts, int64_t nblocks, int nk, double* out,
                             hipStream_t s);
// sum |psi|^2 -> parts[nblocks]; returns nblocks via *nb
hipError_t launch_norm2(const void* psi, int dtype, int64_t N, double* parts, int64_t* nb,
                        hipStream_t s);
// sum conj(phi) psi -> parts[2][nb]
hipError_t launch_overlap(const void* phi, const void* psi, int dtype, int64_t N, double* parts,
                          int64_t* nb, hipStream_t s);
// sum of |psi_z|^2 over a device list of indices -> parts[nb]
hipError_t launch_gather_mass(const void* psi, int dtype, const int64_t* idx, int64_t m,
                              double* parts, int64_t* nb, hipStream_t s);
// per tile minimum and maximum of the diagonal part (float64 tables):
// minmax[2][nblocks]; each schedule separately when sid_only >= 0
hipError_t launch_diag_minmax(const PassArgs& a, int64_t nblocks, double* parts, hipStream_t s);
// mass of psi where diag(g) <= thr -> parts[nblocks]
hipError_t launch_diag_mass(const PassArgs& a, int dtype, int64_t nblocks, double thr,
                            double* parts, hipStream_t s);
// y *= (re + i im)
hipError_t launch_scale(void* y, int dtype, int64_t N, double re, double im, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, int dtype, int64_t N, hipStream_t s);
// zero `bytes` (a multiple of 16) with a fill kernel
hipError_t launch_zero(void* dst, size_t bytes, hipStream_t s);
// sector: (H - c) u with the last pass's epilogue (a.epi), per-block
// reductions into a.epi.red over sector_blocks() blocks
int64_t sector_blocks(int64_t dim);
hipError_t launch_sector_matvec(const SectorArgs& a, int dtype, hipStream_t s);
// out[r] = the diagonal at the state of rank r for the coefficients of `a`
// (used with one schedule set to 1, the others 0, and dconst 0)
hipError_t launch_sector_dtab(const SectorArgs& a, double* out, hipStream_t s);
// sector diagonal: mode 0 per-block min and max -> parts[2][nb]; mode 1
// mass of psi where the diagonal is <= thr -> parts[nb]
hipError_t launch_sector_diag(const SectorArgs& a, int mode, double thr, const void* psi, int dtype,
                              double* parts, hipStream_t s);
// sector <-> full space: full[z(r)] = sec[r] (full zeroed elsewhere by the caller)
hipError_t launch_sector_expand(const SectorDev& sd, const void* sec, void* full, int dtype,
                                hipStream_t s);
// y[i] = v for i < N
hipError_t launch_fill(void* y, int dtype, int64_t N, double re, double im, hipStream_t s);

// ---- Lanczos basis operations (lowest eigenvalues) -----------------------------
// The basis holds vectors V_j = base + j * stride (N <= stride amplitudes each).
constexpr int kLzMaxBasis = 48;
constexpr int kLzMaxKeep = 16;
constexpr int kLzGroup = 8;          // vectors per dot-product pass
// c_j = <V_j, w>, j < k: partials parts[2j][nb] (re), parts[2j+1][nb] (im)
int64_t lz_blocks(int64_t N);
hipError_t launch_multidot(const void* base, int64_t stride, int64_t N, int k, const void* w, int dtype,
                           double* parts, hipStream_t s);
// w -= sum_{j<k} c_j V_j (c: device double2[k]) and |w|^2 partials -> parts[nb]
hipError_t launch_multiaxpy(const void* base, int64_t stride, int64_t N, int k, const double* c, void* w,
                            int dtype, double* parts, hipStream_t s);
// dst = src * a (real)
hipError_t launch_scale_copy(void* dst, const void* src, int dtype, int64_t N, double a, hipStream_t s);
// V_i <- sum_{j<m} V_j Y[j][i] for i < kk, in place (Y: device double2[m][kk])
hipError_t launch_basis_transform(void* base, int64_t stride, int64_t N, int m, int kk, const double* Y,
                                  int dtype, hipStream_t s);
// a fixed pseudo-random state: components uniform in [-1, 1) from a counter hash
hipError_t launch_random_fill(void* y, int dtype, int64_t N, uint64_t seed, hipStream_t s);

}  // namespace aqc
