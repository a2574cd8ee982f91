// Unpivoted blocked Householder QR with explicit Q and a non-negative
// diagonal of R -- the "Qpos" of the PowerURV iteration (Section 3, eqs.
// power and powerqr) and of DDH-URV (Section 2.2).  Following Section 2.2,
// reflectors are accumulated per block of kPanelNB columns and applied to the
// trailing matrix with matrix-matrix products (compact WY form
// H_1 ... H_b = I - Y T Y^T, Schreiber & Van Loan 1989).
//
// Per block:
//   panel_kernel     Householder vectors of an (m-j0) x b panel, column by
//                    column.  The panel is spread over P workgroups by rows;
//                    each holds its rows in registers (one column per lane).
//                    One column needs one device-wide reduction: the partial
//                    inner products of the pivot column with every column of
//                    the panel, from which the norm, the reflector and its
//                    action follow.  Workgroups meet at a counter barrier;
//                    partial sums are added in a fixed order, so every
//                    workgroup derives bitwise-identical reflectors.
//                    The same reductions carry the Gram matrix S = Y^T Y,
//                    from which workgroup 0 forms T (upper triangular).
//   trailing update  C <- (I - Y T^T Y^T) C by three GEMMs.
// Q is formed afterwards from the stored blocks, last block first, starting
// from [D; 0] with D = sign(diag R), which makes diag(R) >= 0 at no cost.
#include "common.hpp"

#include <cstdlib>

namespace urv {
namespace {

constexpr int NB = kPanelNB;        // columns per panel (one lane per column)
constexpr int PANEL_WAVES = 8;      // row groups (waves) per workgroup
constexpr int RPT = 32;             // rows per lane
constexpr int RPW = PANEL_WAVES * RPT;  // rows per workgroup
constexpr int PANEL_THREADS = 64 * PANEL_WAVES;
constexpr int kMaxPanelWgs = static_cast<int>(kMaxRows / 256);  // all panel workgroups co-resident
constexpr long kSpinLimit = 1L << 23;   // bounded wait: ~seconds, then give up

// How the panel's waits end.  Normal runs: the spin limit above, tags as
// published.  Failure tests: a short limit and an expected tag that is never
// published, so every wait expires (and every kernel still returns).
struct PanelWait {
  long spin_limit = kSpinLimit;
  uint32_t skew = 0;  // added to every expected tag
};

// Cross-workgroup exchange of the panel.  An FP64 value is published as two
// 64-bit words (tag << 32 | high half) and (tag << 32 | low half), an FP32
// value as one word (tag << 32 | bits), with agent-scope atomic stores, which
// bypass the per-XCD caches; a reader polls with agent-scope atomic loads
// until every word carries the tag it expects.  Each word is self-validating,
// so no fences or counters are needed, and a round costs one trip to the
// coherence point.  Tags (block * 64 + column + 1) grow through a
// factorisation, and the buffer is zeroed when it starts.  A slot is two
// words for either type.
__device__ inline void tagged_store(uint64_t* p, uint32_t tag, double v) {
  const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(v));
  const uint64_t t = static_cast<uint64_t>(tag) << 32;
  __hip_atomic_store(p, t | (bits >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + 1, t | (bits & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void tagged_store(uint64_t* p, uint32_t tag, float v) {
  const uint64_t bits = static_cast<uint64_t>(__float_as_uint(v));
  __hip_atomic_store(p, (static_cast<uint64_t>(tag) << 32) | bits, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// Waits for K tagged values and returns them in out[].  Gives up (returns
// false, raises *err) after a bounded number of polls, or as soon as another
// workgroup has raised *err.
template <class T, int K>
__device__ inline bool tagged_load_all(const uint64_t* const* ptr, int count, uint32_t tag,
                                       T* out, unsigned* err, long spin_limit) {
  constexpr bool kTwo = sizeof(T) == 8;
  long spins = 0;
  for (;;) {
    uint64_t w0[K], w1[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k < count) {
        w0[k] = __hip_atomic_load(ptr[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        w1[k] = kTwo ? __hip_atomic_load(ptr[k] + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     : w0[k];
      }
    }
    bool ready = true;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < count) ready = ready && (w0[k] >> 32) == tag && (w1[k] >> 32) == tag;
    if (ready) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (k < count) {
          if constexpr (kTwo)
            out[k] = __longlong_as_double(static_cast<long long>((w0[k] << 32) | (w1[k] & 0xffffffffull)));
          else
            out[k] = __uint_as_float(static_cast<unsigned>(w0[k] & 0xffffffffull));
        }
      }
      return true;
    }
    // the error flag is looked at every 64th poll only: each look is a round trip
    if ((++spins & 63) == 0 &&
        (spins > spin_limit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
      __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// A load that sees stores made by other kernels after this one started (an
// agent-scope atomic load, as the exchange uses): for data that a kernel
// waited for with a flag rather than by stream order.
__device__ inline double load_coherent(const double* p) {
  return __longlong_as_double(static_cast<long long>(
      __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
}
__device__ inline float load_coherent(const float* p) {
  return __uint_as_float(
      __hip_atomic_load(reinterpret_cast<const unsigned*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Waits until *flag >= value (one lane of the workgroup polls); false, with
// *err raised, when the bounded wait expires or another workgroup gave up.
__device__ inline bool wait_flag_geq(const unsigned* flag, unsigned value, unsigned* err, long spin_limit) {
  long spins = 0;
  while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < value) {
    if ((++spins & 63) == 0 &&
        (spins > spin_limit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
      __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

// Raises a flag for a kernel that is already running: launched after the work
// the flag stands for, on the same stream.
__global__ void signal_kernel(unsigned* flag, unsigned value) {
  if (threadIdx.x == 0) __hip_atomic_store(flag, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
struct Vec2;
template <>
struct Vec2<double> {
  using type = double2;
  static __device__ inline double2 make(double a, double b) { return make_double2(a, b); }
};
template <>
struct Vec2<float> {
  using type = float2;
  static __device__ inline float2 make(float a, float b) { return make_float2(a, b); }
};

// One 16x16x4 matrix-core step: D = a b + C with operand a given by lane l as
// element (i = l % 16, k = l / 16), operand b as (k = l / 16, j = l % 16), and
// entry v of the result held by lane l being D(row(l / 16, v), l % 16).
template <class T>
struct PanelMma;
template <>
struct PanelMma<double> {
  typedef double acc __attribute__((ext_vector_type(4)));
  static __device__ inline acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct PanelMma<float> {
  typedef float acc __attribute__((ext_vector_type(4)));
  static __device__ inline acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int v) { return 4 * lk + v; }
};

// Makes one lane's LDS writes visible to the other lanes of its wave: the
// lanes run in lockstep, so only the compiler must be kept from moving LDS
// accesses across this point (and the LDS queue drained).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// sum over the waves of a workgroup, in a fixed order
template <class T, int W>
__device__ __forceinline__ T sum_waves(const T (*red)[W], int c) {
  T a = 0, b = 0;
#pragma unroll
  for (int w = 0; w < PANEL_WAVES; w += 2) {
    a += red[w][c];
    b += red[w + 1][c];
  }
  return a + b;
}

// Column jj of T (lane i computes T(i, jj)):
// T(jj,jj) = tau_jj,  T(i,jj) = -tau_jj sum_{k<jj} T(i,k) S(k,jj) for i < jj (T(i,k) = 0 for k < i).
template <class T>
__device__ inline void t_column(T (*Tsh)[NB + 2], const T (*Ssh)[NB + 2], const T* tau_sh,
                                int jj, int i) {
  using V2 = typename Vec2<T>::type;
  T acc[4] = {0, 0, 0, 0};
  int k = 0;
  for (; k + 1 < jj; k += 2) {
    const V2 tk = *reinterpret_cast<const V2*>(&Tsh[i][k]);
    const V2 sk = *reinterpret_cast<const V2*>(&Ssh[jj][k]);
    acc[k & 2] += tk.x * sk.x;
    acc[(k & 2) + 1] += tk.y * sk.y;
  }
  if (k < jj) acc[0] += Tsh[i][k] * Ssh[jj][k];
  const T tj = tau_sh[jj];
  const T sum = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  Tsh[i][jj] = (i < jj) ? -tj * sum : (i == jj ? tj : T(0));
}

// Second panel of a 128-column sub-block, joined with the first: the panel
// also forms S12 = Y1^T Y2 (a device-wide reduction of 64 x 64 partial sums
// in two tagged rounds) and workgroup 0 writes T12 = -T1 S12 T2 and the zero
// lower-left block, so that the sub-block's T is complete when it returns.
template <class T>
struct PanelJoin {
  const T* Y1 = nullptr;    // first panel's reflectors at this panel's first row (ld ldy1); null: no join
  int64_t ldy1 = 0;
  T* T1 = nullptr;          // first panel's T (ld ldt); this panel's T is at T1 + jb1 (1 + ldt)
  int jb1 = 0;
  uint64_t* ps = nullptr;   // P x 4096 tagged partial sums
  uint64_t* sums = nullptr; // 4096 tagged sums
};
constexpr int kJoinEntries = NB * NB;

// ---------------------------------------------------------------------------
// Tall-skinny QR of a panel with Householder reconstruction.
//
// The loop above needs one device-wide reduction per column.  The TSQR form
// needs three exchanges per panel:
//  1. Leaf.  Each workgroup factors its own rows alone (registers, lane =
//     column, one workgroup barrier per column): R_w (64 x 64 upper), its
//     reflectors (written to the Y rows it owns) and T_w (from the Gram
//     entries).
//  2. Tree.  The R factors of up to 8 workgroups are stacked and factored by
//     every member of the group (each gets bitwise the same result); with more
//     than 8 workgroups a second node combines the group factors likewise.  In
//     a stack of upper-triangular factors the reflector of column j touches
//     row j of the top factor and rows 0..j of the others, a pattern the steps
//     keep, so the top block of the node's reflector matrix is I and the
//     node's Q is [I; 0] - Yc Tc.
//  3. Each workgroup forms its rows of the panel's Q (orthonormal columns),
//     Q_w = Q_leaf M_w with M_w its 64 x 64 block of the tree's Q.
//  4. Householder vectors are rebuilt from Q (Ballard, Demmel, Grigori,
//     Jacquelin, Knight, Nguyen, "Reconstructing Householder vectors from
//     tall-skinny QR", 2015): with S diagonal (+-1, chosen during the
//     elimination so that every pivot has modulus >= 1), S - Q1 = L U (Q1 the
//     panel's top 64 rows of Q, no pivoting) gives Y = [L; -Q2 U^-1],
//     T = U S L^-T and R = S R_tree; then H_1 ... H_64 = I - Y T Y^T with
//     H[:, 0:64] = Q S.  Workgroup 0 factors S - Q1 and sends U^-1 and T.
// Every sum runs in a fixed order, so results are bitwise reproducible.
constexpr int kTriEntries = NB * (NB + 1) / 2;  // packed upper triangle, column by column
constexpr int kTsqrFan = 4;                     // factors per tree node (two waves each)
static_assert(2 * kTsqrFan == PANEL_WAVES, "two waves per stacked factor");
__host__ __device__ __forceinline__ int tri_index(int i, int c) { return c * (c + 1) / 2 + i; }  // i <= c

// Exchange areas of the TSQR panel: values (one 8-byte word each) and the flags
// that announce them.
struct TsqrXch {
  uint64_t* tri = nullptr;    // 2 P x kTriEntries: the R of every unit of every tree level
  uint64_t* recon = nullptr;  // 2 NB^2: U^-1 and T from workgroup 0
  uint64_t* gram = nullptr;   // (P + 1) x NB^2: partial sums of the 64 x 64 reductions, then the sums
  uint64_t* flags = nullptr;  // one per unit, one for the reconstruction, two per workgroup for the sums
  uint64_t* upd = nullptr;    // (P + 1) x 4 NB^2: partial sums of the previous block's update, then the sums
  uint64_t* uflags = nullptr; // two per workgroup, for that sum
  int chol = 1;               // try CholeskyQR2 first
};
// The streaming panel: 128 rows per workgroup (two 64-row chunks), so that
// more compute units share each pass over the panel.
constexpr int CQR_RPW = 128;
constexpr int CQR_CHUNKS = CQR_RPW / 64;
constexpr int CQR_RPT = CQR_RPW / PANEL_WAVES;  // rows per wave in its tall-skinny leaf
// (+1: the rows above a panel that first applies the previous block's reflectors)
constexpr int kMaxCqrWgs = static_cast<int>(kMaxRows / CQR_RPW) + 1;
constexpr int kTsqrUnits = 2 * kMaxCqrWgs;  // P + P/4 + P/16 + ... < 2 P
constexpr int kTsqrFlags = kTsqrUnits + 1 + 2 * kMaxCqrWgs;

// Announced exchange: every thread writes its values with agent-scope stores
// (write-through), waits for them to complete (s_waitcnt vmcnt(0)), and after a
// workgroup barrier one thread raises the flag to the tag; a reader waits for
// the tag, then reads the values with agent-scope loads.  One flag per block of
// values, so the values travel as plain words (no tag in each).
constexpr unsigned kWaitStores = 0x0F70;  // s_waitcnt vmcnt(0) expcnt(7) lgkmcnt(15)
__device__ __forceinline__ void store_agent(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), static_cast<uint64_t>(__double_as_longlong(v)),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(float* p, float v) {
  __hip_atomic_store(reinterpret_cast<unsigned*>(p), __float_as_uint(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void raise_flag(uint64_t* flag, uint32_t tag) {
  __builtin_amdgcn_s_waitcnt(kWaitStores);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, static_cast<uint64_t>(tag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Bounded wait until *flag == tag (every calling lane polls the same word).
__device__ __forceinline__ bool await_flag(const uint64_t* flag, uint32_t tag, unsigned* err, long spin_limit) {
  long spins = 0;
  while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != static_cast<uint64_t>(tag)) {
    if ((++spins & 63) == 0 &&
        (spins > spin_limit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
      __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // the value loads stay after the wait
  return true;
}

// A 64 x 64 matrix on the matrix cores: wave g holds rows ib = 16 (g >> 1) ..
// +16 and columns cb0 = 32 (g & 1) .. +32 as two 16 x 16 accumulators.
template <class T>
struct Frag {
  typename PanelMma<T>::acc a0, a1;
};

struct FragPos {
  int ib, cb0, l16, lk;
};

template <class T>
__device__ __forceinline__ void frag_zero(Frag<T>& f) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    f.a0[v] = T(0);
    f.a1[v] = T(0);
  }
}

// f = diag * I - f
template <class T>
__device__ __forceinline__ void frag_negate_plus_identity(Frag<T>& f, const FragPos& p, bool identity) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = p.ib + PanelMma<T>::row(p.lk, v);
    f.a0[v] = ((identity && i == p.cb0 + p.l16) ? T(1) : T(0)) - f.a0[v];
    f.a1[v] = ((identity && i == p.cb0 + 16 + p.l16) ? T(1) : T(0)) - f.a1[v];
  }
}

template <class T>
__device__ __forceinline__ void frag_identity(Frag<T>& f, const FragPos& p) {
  frag_zero(f);
  frag_negate_plus_identity(f, p, true);
}

template <class T>
__device__ __forceinline__ void frag_to_lds(const Frag<T>& f, T (*M)[NB + 2], const FragPos& p) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = p.ib + PanelMma<T>::row(p.lk, v);
    M[i][p.cb0 + p.l16] = f.a0[v];
    M[i][p.cb0 + 16 + p.l16] = f.a1[v];
  }
}

template <class T>
__device__ __forceinline__ void frag_from_lds(Frag<T>& f, const T (*M)[NB + 2], const FragPos& p) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = p.ib + PanelMma<T>::row(p.lk, v);
    f.a0[v] = M[i][p.cb0 + p.l16];
    f.a1[v] = M[i][p.cb0 + 16 + p.l16];
  }
}

// f += op(A) op(B) for 64 x 64 A, B in LDS; op(A)(i, k) = A[i][k] (A[k][i] when
// TA), op(B)(k, j) = B[k][j] (B[j][k] when TB).
template <class T, bool TA, bool TB = false>
__device__ __forceinline__ void frag_mma(Frag<T>& f, const T (*A)[NB + 2], const T (*B)[NB + 2], const FragPos& p) {
#pragma unroll 4
  for (int ks = 0; ks < NB / 4; ++ks) {
    const int kk = 4 * ks + p.lk;
    const T a = TA ? A[kk][p.ib + p.l16] : A[p.ib + p.l16][kk];
    const T b0 = TB ? B[p.cb0 + p.l16][kk] : B[kk][p.cb0 + p.l16];
    const T b1 = TB ? B[p.cb0 + 16 + p.l16][kk] : B[kk][p.cb0 + 16 + p.l16];
    f.a0 = PanelMma<T>::run(a, b0, f.a0);
    f.a1 = PanelMma<T>::run(a, b1, f.a1);
  }
}

// f += sum over k in [k0, k1) of a(i, k) b(k, j), the operands given by
// functors (an LDS read, with masking); k0, k1 multiples of 16.
template <class T, class FA, class FB>
__device__ __forceinline__ void frag_mma_f(Frag<T>& f, FA a, FB b, const FragPos& p, int k0, int k1) {
  for (int k = k0; k < k1; k += 16) {  // k0, k1 multiples of 16: four steps with their loads in flight
    T av[4], b0[4], b1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k + 4 * u + p.lk;
      av[u] = a(p.ib + p.l16, kk);
      b0[u] = b(kk, p.cb0 + p.l16);
      b1[u] = b(kk, p.cb0 + 16 + p.l16);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      f.a0 = PanelMma<T>::run(av[u], b0[u], f.a0);
      f.a1 = PanelMma<T>::run(av[u], b1[u], f.a1);
    }
  }
}

// fn(i, j, value) for the 8 entries of f this lane holds.
template <class T, class F>
__device__ __forceinline__ void frag_each(Frag<T>& f, const FragPos& p, F fn) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = p.ib + PanelMma<T>::row(p.lk, v);
    fn(i, p.cb0 + p.l16, f.a0[v]);
    fn(i, p.cb0 + 16 + p.l16, f.a1[v]);
  }
}

// ---- 64 x 64 triangular algebra in one workgroup, in 16 x 16 blocks
constexpr int BS = 16;

// A double or float of lane `lane` to every lane (through scalar registers).
__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffff), lane);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
__device__ __forceinline__ float lane_value(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// 1 / u: the hardware estimate refined by Newton's iteration r <- r + r (1 - u r)
// (two steps in double precision, one in single), within an ulp or two of the
// quotient.  u = 0 gives NaN (callers reject such pivots).
__device__ __forceinline__ double recip(double u) {
  double r = __builtin_amdgcn_rcp(u);
  r = fma(r, fma(-u, r, 1.0), r);
  r = fma(r, fma(-u, r, 1.0), r);
  return r;
}
__device__ __forceinline__ float recip(float u) {
  float r = __builtin_amdgcn_rcpf(u);
  r = fmaf(r, fmaf(-u, r, 1.0f), r);
  return r;
}

// One wave: LU without pivoting of the 16 x 16 block of M at (b0, b0), in
// place (multipliers below the diagonal, U on and above it).  With signs, the
// pivot of step j is u = m_jj + s, s = sgn(m_jj) (sgn(0) = +1, so |u| >= 1);
// without, u = m_jj.  u, 1/u and s go to ubuf, ubuf + NB and sgnb at b0 + j.
// Lane r < 16 holds row r; the pivot row reaches the other lanes through
// scalar registers, and every step is free of branches.
template <class T>
__device__ __forceinline__ void base16_lu(T (*M)[NB + 2], int b0, bool signs, T* ubuf, T* sgnb, int c) {
  const bool act = c < BS;
  T m[BS];
#pragma unroll
  for (int k = 0; k < BS; ++k) m[k] = act ? M[b0 + c][b0 + k] : T(0);
  T myrinv = T(0), mys = T(0);
#pragma unroll
  for (int j = 0; j < BS; ++j) {
    const T d = lane_value(m[j], j);
    const T sj = signs ? (d >= T(0) ? T(1) : T(-1)) : T(0);
    const T u = d + sj;
    const T rinv = recip(u);
    const T l = m[j] * rinv;  // this row's multiplier (rows below j)
    const T coef = c > j ? l : T(0);
#pragma unroll
    for (int k = j + 1; k < BS; ++k) m[k] = fma(-coef, lane_value(m[k], j), m[k]);
    m[j] = c > j ? l : (c == j ? u : m[j]);
    myrinv = c == j ? rinv : myrinv;
    mys = c == j ? sj : mys;
  }
  if (act) {
#pragma unroll
    for (int k = 0; k < BS; ++k) M[b0 + c][b0 + k] = m[k];
    ubuf[b0 + c] = m[c];
    ubuf[NB + b0 + c] = myrinv;
    sgnb[b0 + c] = mys;
  }
}

// Inverse of the 16 x 16 diagonal block of a triangular factor held in M
// (upper: U on and above the diagonal, rdiag the reciprocals of its diagonal;
// lower: unit L below it) into Z's same block, one column per lane c < 16, by
// column-oriented substitution (the updates of one step are independent).
template <class T, bool kUpper>
__device__ __forceinline__ void base16_inv(const T (*M)[NB + 2], int b0, const T* rdiag, T (*Z)[NB + 2], int c) {
  if (c >= BS) return;
  T z[BS];
#pragma unroll
  for (int r = 0; r < BS; ++r) z[r] = r == c ? T(1) : T(0);
  if constexpr (kUpper) {
#pragma unroll
    for (int r = BS - 1; r >= 0; --r) {
      z[r] *= rdiag[b0 + r];
#pragma unroll
      for (int i = 0; i < r; ++i) z[i] = fma(-M[b0 + i][b0 + r], z[r], z[i]);
    }
  } else {
#pragma unroll
    for (int r = 0; r < BS; ++r) {
#pragma unroll
      for (int i = r + 1; i < BS; ++i) z[i] = fma(-M[b0 + i][b0 + r], z[r], z[i]);
    }
  }
#pragma unroll
  for (int r = 0; r < BS; ++r) Z[b0 + r][b0 + c] = z[r];
}

// One wave's 16 x 16 tile on the matrix cores: acc += sum over k in [k0, k0 + nk)
// of a(i0 + i, k) b(k, j0 + j), nk a multiple of 16, the operands given by
// functors (LDS reads); four k-steps have their loads in flight together.
template <class T>
using TileAcc = typename PanelMma<T>::acc;
template <class T>
__device__ __forceinline__ void tile_zero(TileAcc<T>& a) {
#pragma unroll
  for (int v = 0; v < 4; ++v) a[v] = T(0);
}
template <class T, class FA, class FB>
__device__ __forceinline__ void tile_mm(TileAcc<T>& acc, FA a, FB b, int i0, int j0, int k0, int nk, int c) {
  const int l16 = c & 15, lk = c >> 4;
  for (int k = k0; k < k0 + nk; k += 16) {
    T av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k + 4 * u + lk;
      av[u] = a(i0 + l16, kk);
      bv[u] = b(kk, j0 + l16);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = PanelMma<T>::run(av[u], bv[u], acc);
  }
}
// fn(i, j, value) for the 4 entries of the tile at (i0, j0) this lane holds.
template <class T, class F>
__device__ __forceinline__ void tile_each(const TileAcc<T>& acc, int i0, int j0, int c, F fn) {
#pragma unroll
  for (int v = 0; v < 4; ++v) fn(i0 + PanelMma<T>::row(c >> 4, v), j0 + (c & 15), acc[v]);
}

// LU without pivoting of the 64 x 64 M in place, in 16-column blocks: the
// diagonal block (base16_lu, wave 0), its inverses (waves 0 and 1, into the
// diagonal blocks of Ui and Li, zero elsewhere), then the tiles of U's block
// row L_kk^-1 M_k* and of L's block column M_*k U_kk^-1, and the Schur update,
// one 16 x 16 tile per wave.  ubuf receives the pivots and, at ubuf + NB,
// their reciprocals.
template <class T>
__device__ __forceinline__ void blocked_lu(T (*M)[NB + 2], bool signs, T* ubuf, T* sgnb, T (*Ui)[NB + 2],
                                           T (*Li)[NB + 2], int g, int c) {
  for (int e = threadIdx.x; e < NB * (NB + 2); e += PANEL_THREADS) {
    (&Ui[0][0])[e] = T(0);
    (&Li[0][0])[e] = T(0);
  }
  for (int kb = 0; kb < NB / BS; ++kb) {
    const int b0 = kb * BS, b1 = b0 + BS;
    __syncthreads();
    if (g == 0) base16_lu(M, b0, signs, ubuf, sgnb, c);
    __syncthreads();
    if (g == 0) base16_inv<T, true>(M, b0, ubuf + NB, Ui, c);
    if (g == 1) base16_inv<T, false>(M, b0, ubuf + NB, Li, c);
    __syncthreads();
    const int nt = (NB - b1) / BS;
    if (nt == 0) break;
    if (g < 2 * nt) {  // wave g < nt: U's tile (kb, kb + 1 + g); else L's tile (kb + 1 + g - nt, kb)
      TileAcc<T> a;
      tile_zero<T>(a);
      if (g < nt) {
        const int j0 = b1 + BS * g;
        tile_mm<T>(a, [&](int i, int k) { return Li[i][k]; }, [&](int k, int j) { return M[k][j]; }, b0, j0, b0, BS, c);
        tile_each<T>(a, b0, j0, c, [&](int i, int j, T v) { M[i][j] = v; });
      } else {
        const int i0 = b1 + BS * (g - nt);
        tile_mm<T>(a, [&](int i, int k) { return M[i][k]; }, [&](int k, int j) { return Ui[k][j]; }, i0, b0, b0, BS, c);
        tile_each<T>(a, i0, b0, c, [&](int i, int j, T v) { M[i][j] = v; });
      }
    }
    __syncthreads();
    for (int t = g; t < nt * nt; t += PANEL_WAVES) {
      const int i0 = b1 + BS * (t / nt), j0 = b1 + BS * (t % nt);
      TileAcc<T> a;
      tile_zero<T>(a);
      tile_mm<T>(a, [&](int i, int k) { return M[i][k]; }, [&](int k, int j) { return M[k][j]; }, i0, j0, b0, BS, c);
      tile_each<T>(a, i0, j0, c, [&](int i, int j, T v) { M[i][j] -= v; });
    }
  }
  __syncthreads();
}

// Z triangular 64 x 64 with its 16 x 16 diagonal blocks in place and zero
// elsewhere: the off-diagonal blocks are filled by joining pairs of 16-, then
// 32-blocks, Z_AB = -Z_A C_AB Z_B (upper) or Z_BA = -Z_B C_BA Z_A (lower),
// C(a, b) = cf(a, b) the coupling.  This gives the inverse of a triangular
// matrix C from the inverses of its diagonal blocks, and T of a compact WY form
// from the Gram entries.  One phase of one level: wave w < 4 takes every fourth
// 16 x 16 tile; phase 0 forms X = C_AB Z_B (C_BA Z_A) into W, phase 1
// Z_AB = -Z_A X (Z_BA = -Z_B X).  W is used in its strictly upper (upper) or
// strictly lower (lower) part only, so an upper and a lower join may share it.
template <class T, bool kUpper, class CF>
__device__ __forceinline__ void tri_join_phase(T (*Z)[NB + 2], CF cf, T (*W)[NB + 2], int half, int phase, int w,
                                               int c) {
  const int side = half / BS, per = side * side, tiles = (NB / (2 * half)) * per;
  for (int t = w; t < tiles; t += 4) {
    const int p0 = (t / per) * 2 * half, ti = BS * ((t % per) / side), tj = BS * ((t % per) % side);
    TileAcc<T> a;
    tile_zero<T>(a);
    if (phase == 0) {
      if constexpr (kUpper) {  // rows of A, columns of B; Z_B upper: k up to tj + 16
        tile_mm<T>(a, cf, [&](int k, int j) { return Z[k][j]; }, p0 + ti, p0 + half + tj, p0 + half, tj + BS, c);
        tile_each<T>(a, p0 + ti, p0 + half + tj, c, [&](int i, int j, T v) { W[i][j] = v; });
      } else {  // rows of B, columns of A; Z_A lower: k from tj
        tile_mm<T>(a, cf, [&](int k, int j) { return Z[k][j]; }, p0 + half + ti, p0 + tj, p0 + tj, half - tj, c);
        tile_each<T>(a, p0 + half + ti, p0 + tj, c, [&](int i, int j, T v) { W[i][j] = v; });
      }
    } else {
      if constexpr (kUpper) {  // Z_A upper: k from ti
        tile_mm<T>(a, [&](int i, int k) { return Z[i][k]; }, [&](int k, int j) { return W[k][j]; }, p0 + ti,
                   p0 + half + tj, p0 + ti, half - ti, c);
        tile_each<T>(a, p0 + ti, p0 + half + tj, c, [&](int i, int j, T v) { Z[i][j] = -v; });
      } else {  // Z_B lower: k up to ti + 16
        tile_mm<T>(a, [&](int i, int k) { return Z[i][k]; }, [&](int k, int j) { return W[k][j]; }, p0 + half + ti,
                   p0 + tj, p0 + half, ti + BS, c);
        tile_each<T>(a, p0 + half + ti, p0 + tj, c, [&](int i, int j, T v) { Z[i][j] = -v; });
      }
    }
  }
}
// The join on waves 0..3 (every wave of the workgroup calls: barriers inside).
template <class T, bool kUpper, class CF>
__device__ __forceinline__ void tri_join(T (*Z)[NB + 2], CF cf, T (*W)[NB + 2], int g, int c) {
  for (int half = BS; half < NB; half *= 2)
    for (int phase = 0; phase < 2; ++phase) {
      if (g < 4) tri_join_phase<T, kUpper>(Z, cf, W, half, phase, g, c);
      __syncthreads();
    }
}
// An upper join on waves 0..3 beside a lower one on waves 4..7, sharing W.
template <class T, class CFU, class CFL>
__device__ __forceinline__ void tri_join_both(T (*Zu)[NB + 2], CFU cfu, T (*Zl)[NB + 2], CFL cfl, T (*W)[NB + 2],
                                              int g, int c) {
  for (int half = BS; half < NB; half *= 2)
    for (int phase = 0; phase < 2; ++phase) {
      if (g < 4)
        tri_join_phase<T, true>(Zu, cfu, W, half, phase, g, c);
      else
        tri_join_phase<T, false>(Zl, cfl, W, half, phase, g - 4, c);
      __syncthreads();
    }
}

// v unchanged, through a step the compiler cannot see into: LDS addresses
// derived from it are then formed in the phase that uses them instead of being
// hoisted to the kernel's entry and held in registers across every phase.
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// LDS of the TSQR steps.
template <class T>
struct TsqrLds {
  T (*S1)[NB + 2];           // R of the leaf, then of a tree node
  T (*S2)[NB + 2];           // work matrices
  T (*S3)[NB + 2];           // Gram entries (S3[j][c] = y_c^T y_j, c < j), work matrix
  T (*S4)[NB + 2];           // T of the leaf / node, then of the panel
  T (*cb)[NB];               // pivot column of each wave's rows
  T (*red0)[NB];             // partial sums of even steps, per wave
  T (*red1)[NB];             // partial sums of odd steps
  T (*piv)[NB];              // [2][NB]: pivot row by step parity
  T* tau;                    // [NB]
  T* aux;                    // [8][NB]: elimination buffers, pivots, signs
};

// One reflector: x_j = (alpha; x_below) with sigma2 = ||x_below||^2 gives
// beta = -sgn(alpha) ||x_j|| (sgn(0) = +1), tau = (beta - alpha) / beta and
// v = x_j / (alpha - beta) with v_1 = 1 (LAPACK's convention); H = I when
// sigma2 = 0.
template <class T>
__device__ __forceinline__ void reflector(T alpha, T sigma2, T& t, T& beta, T& rinv) {
  t = T(0);
  beta = alpha;
  rinv = T(0);
  if (sigma2 != T(0)) {
    const T norm = sqrt(alpha * alpha + sigma2);
    beta = (alpha >= T(0)) ? -norm : norm;
    rinv = T(1) / (alpha - beta);
    t = (beta - alpha) / beta;
  }
}

// T (upper triangular, 64 x 64, into Tm) of H_0 ... H_{jb-1} = I - Y T Y^T from
// tau and the Gram entries G[j][c] = y_c^T y_j (c < j), Schreiber and Van Loan's
// recurrence taken in blocks: the four 16 x 16 diagonal blocks column by column
// (waves 0..3, lane l < 16 holding row l of its block in registers), then the
// blocks joined, T_AB = -T_A (Y_A^T Y_B) T_B (tri_join).  Columns from jb on are
// zero.  W is scratch.
template <class T>
__device__ __forceinline__ void tsqr_build_t(T (*Tm)[NB + 2], const T (*G)[NB + 2], const T* tau, int jb,
                                             T (*W)[NB + 2], int g, int c, const FragPos& fp) {
  for (int e = threadIdx.x; e < NB * (NB + 2); e += PANEL_THREADS) (&Tm[0][0])[e] = T(0);
  __syncthreads();
  if (g < NB / BS && c < BS) {
    const int b0 = g * BS, il = c;
    T tr[BS];
#pragma unroll
    for (int jj = 0; jj < BS; ++jj) {
      const int col = b0 + jj;
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < jj; ++k) acc = fma(tr[k], G[col][b0 + k], acc);
      const T tc = col < jb ? tau[col] : T(0);
      tr[jj] = col >= jb ? T(0) : (il == jj ? tc : (il < jj ? -tc * acc : T(0)));
    }
#pragma unroll
    for (int jj = 0; jj < BS; ++jj) Tm[b0 + il][b0 + jj] = tr[jj];
  }
  __syncthreads();
  tri_join<T, true>(Tm, [&](int a, int b) { return b < jb ? G[b][a] : T(0); }, W, g, c);
}

// Leaf: Householder QR of this workgroup's rows alone.  Column j's pivot is
// block row lbase + j; rows above lbase are outside the leaf and untouched.
// On return x holds the reflectors, scaled (y_c below the pivot of lane c's
// column), L.S1 the leaf's R (S1[i][c], i <= c, zero elsewhere), L.S4 its T
// and L.tau its tau.  Wave 0 builds T column by column, one step behind; its
// own rows leave the leaf first.
template <class T, int R>
__device__ __forceinline__ void tsqr_leaf(T (&x)[R], int jbp, int lbase, int myrow0i, int g, int c,
                                 const TsqrLds<T>& L) {
  using V2 = typename Vec2<T>::type;
  c = opaque(c);
  for (int e = threadIdx.x; e < NB * (NB + 2); e += PANEL_THREADS) {
    (&L.S1[0][0])[e] = T(0);
    (&L.S4[0][0])[e] = T(0);
  }
  __syncthreads();
  T my_rinv = T(0);
  constexpr int OWN_LD = R + 2;
  T* const own = &L.S2[0][0];
  for (int j = 0; j < jbp; ++j) {
    const int par = j & 1;
    T (*red)[NB] = par ? L.red1 : L.red0;
    const int lo = min(max(lbase + j - myrow0i, -1), R);  // wave-uniform
    const bool owner = lo >= 0 && lo < R;
    const bool below = lo < R;
    const T* colp = &L.cb[g][0];
    if (lo < 0) {
      if (c == j) {
#pragma unroll
        for (int r = 0; r < R; r += 2) *reinterpret_cast<V2*>(&L.cb[g][r]) = Vec2<T>::make(x[r], x[r + 1]);
      }
    } else if (owner) {
      T* mine_t = own + c * OWN_LD;
#pragma unroll
      for (int r = 0; r < R; r += 2) *reinterpret_cast<V2*>(mine_t + r) = Vec2<T>::make(x[r], x[r + 1]);
      L.piv[par][c] = mine_t[lo];
      if (c == j)
        for (int r = 0; r <= lo; ++r) mine_t[r] = T(0);
      colp = own + j * OWN_LD;
    }
    wave_lds_sync();
    T qa[4] = {T(0), T(0), T(0), T(0)};
    if (below) {
#pragma unroll
      for (int r = 0; r < R; r += 2) {
        const V2 xj = *reinterpret_cast<const V2*>(colp + r);
        qa[r & 2] += xj.x * x[r];
        qa[(r & 2) + 1] += xj.y * x[r + 1];
      }
    }
    red[g][c] = (qa[0] + qa[1]) + (qa[2] + qa[3]);
    __syncthreads();
    const T xcj = L.piv[par][c];
    const T alpha = L.piv[par][j];
    const T qc = sum_waves(red, c);
    const T sigma2 = sum_waves(red, j);
    T t, beta, rinv;
    reflector(alpha, sigma2, t, beta, rinv);
    if (c == j) my_rinv = rinv;
    const T w = xcj + qc * rinv;  // v^T x_c
    if (g == 0) {
      if (c < j) L.S3[j][c] = my_rinv * w;
      if (c == 0) L.tau[j] = t;
      L.S1[j][c] = (c == j) ? beta : (c > j ? xcj - t * w : T(0));
    }
    const T coef = (c > j && t != T(0)) ? t * w * rinv : T(0);
    if (below) {
#pragma unroll
      for (int r = 0; r < R; r += 2) {
        const V2 xj = *reinterpret_cast<const V2*>(colp + r);
        x[r] = fma(-coef, xj.x, x[r]);
        x[r + 1] = fma(-coef, xj.y, x[r + 1]);
      }
    }
  }
  __syncthreads();
  const FragPos fp{(g >> 1) * 16, (g & 1) * 32, c & 15, c >> 4};
  tsqr_build_t(L.S4, L.S3, L.tau, jbp, L.S2, g, c, fp);
  const int loc = lbase + c - myrow0i;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (c < jbp && r > loc) x[r] *= my_rinv;
  __syncthreads();
}

// A packed upper-triangular 64 x 64 factor (S1) published, then announced.
template <class T>
__device__ __forceinline__ void tsqr_publish_tri(const T (*S1)[NB + 2], uint64_t* dst, uint64_t* flag, uint32_t tag) {
  T* d = reinterpret_cast<T*>(dst);
  for (int e = threadIdx.x; e < NB * NB; e += PANEL_THREADS) {
    const int i = e & (NB - 1), c = e / NB;
    if (i <= c) store_agent(d + tri_index(i, c), S1[i][c]);
  }
  raise_flag(flag, tag);
}

// One tree node: the QR of K (2..4) stacked upper-triangular factors taken from
// `src` (packed) once their flags carry the tag.  The top factor goes to L.S2,
// where row j is read at step j only (no step before touches it); factor t >=
// 1 lives in the registers of waves 2t (rows 0..31) and 2t + 1 (rows 32..63),
// lane c holding column c (rows 0..c).  On return tri holds this wave's half of
// its factor's block of the scaled reflectors, L.S1 the node's R, L.S4 its T;
// false if a wait expired.
template <class T>
__device__ __forceinline__ bool tsqr_node(T (&tri)[RPT], const uint64_t* src, const uint64_t* flags, int K, uint32_t tag,
                                 int jbp, int g, int c, const TsqrLds<T>& L, unsigned* err, const PanelWait& pw) {
  static_assert(2 * RPT == NB, "a factor spans two waves");
  c = opaque(c);
  for (int e = threadIdx.x; e < NB * (NB + 2); e += PANEL_THREADS) {
    (&L.S1[0][0])[e] = T(0);
    (&L.S4[0][0])[e] = T(0);
  }
  const int t = g >> 1, h0 = (g & 1) * RPT;  // this wave's factor and first row
  bool ok = true;
#pragma unroll
  for (int r = 0; r < RPT; ++r) tri[r] = T(0);
  if (t < K) {
    // rows h0 .. h0 + 31 of column c (those on or above the diagonal), all in flight at once
    ok = await_flag(flags + t, tag + pw.skew, err, pw.spin_limit);
    // (each unit's area is kTriEntries 8-byte words, whatever T is)
    const T* colp = reinterpret_cast<const T*>(src + static_cast<int64_t>(t) * kTriEntries) + tri_index(h0, c);
#pragma unroll
    for (int r = 0; r < RPT; ++r) tri[r] = (ok && h0 + r <= c) ? load_coherent(colp + r) : T(0);
  }
  if (t == 0) {
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      L.S2[h0 + r][c] = tri[r];
      tri[r] = T(0);
    }
  }
  if (__syncthreads_or(ok ? 0 : 1)) return false;

  T my_rinv = T(0);
  const bool act = t >= 1 && t < K;  // wave-uniform
  for (int j = 0; j < jbp; ++j) {
    const int par = j & 1;
    T (*red)[NB] = par ? L.red1 : L.red0;
    if (act && h0 <= j) {
      // rows h0 + 8 rb .. of column j that lie on or above its diagonal (the rest are zero)
      if (c == j) {
#pragma unroll
        for (int rb = 0; rb < RPT; rb += 8)
          if (h0 + rb <= j) {
#pragma unroll
            for (int u = 0; u < 8; ++u) L.cb[g][rb + u] = tri[rb + u];
          }
      }
      wave_lds_sync();
      T qa[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int rb = 0; rb < RPT; rb += 8)
        if (h0 + rb <= j) {
#pragma unroll
          for (int u = 0; u < 8; ++u) qa[u & 3] += L.cb[g][rb + u] * tri[rb + u];
        }
      red[g][c] = (qa[0] + qa[1]) + (qa[2] + qa[3]);
    } else {
      red[g][c] = T(0);
    }
    __syncthreads();
    const T xcj = L.S2[j][c];
    const T alpha = L.S2[j][j];
    const T qc = sum_waves(red, c);
    const T sigma2 = sum_waves(red, j);
    T tt, beta, rinv;
    reflector(alpha, sigma2, tt, beta, rinv);
    if (c == j) my_rinv = rinv;
    const T w = xcj + qc * rinv;
    if (g == 0) {
      if (c < j) L.S3[j][c] = my_rinv * w;
      if (c == 0) L.tau[j] = tt;
      L.S1[j][c] = (c == j) ? beta : (c > j ? xcj - tt * w : T(0));
    }
    const T coef = (c > j && tt != T(0)) ? tt * w * rinv : T(0);
    if (act && h0 <= j) {
#pragma unroll
      for (int rb = 0; rb < RPT; rb += 8)
        if (h0 + rb <= j) {
#pragma unroll
          for (int u = 0; u < 8; ++u) tri[rb + u] = fma(-coef, L.cb[g][rb + u], tri[rb + u]);
        }
    }
  }
  __syncthreads();
  const FragPos fp{(g >> 1) * 16, (g & 1) * 32, c & 15, c >> 4};
  tsqr_build_t(L.S4, L.S3, L.tau, jbp, L.S2, g, c, fp);  // Rtop in S2 is no longer needed
#pragma unroll
  for (int r = 0; r < RPT; ++r) tri[r] *= my_rinv;
  __syncthreads();
  return true;
}

// Block s of a node's Q, [I; 0] - Yc Tc (Tc in L.S4): I - Tc for s = 0, whose
// reflector block is I; -Yc_s Tc otherwise, Yc_s held by waves 2s and 2s + 1.
template <class T>
__device__ __forceinline__ void tsqr_node_q(const T (&tri)[RPT], int s, int g, int c, const TsqrLds<T>& L, const FragPos& p,
                                   Frag<T>& f) {
  c = opaque(c);
  if (s > 0 && (g >> 1) == s) {
    const int h0 = (g & 1) * RPT;
#pragma unroll
    for (int r = 0; r < RPT; ++r) L.S2[h0 + r][c] = tri[r];
  }
  __syncthreads();
  frag_zero(f);
  if (s == 0) {
    frag_from_lds(f, L.S4, p);
    frag_negate_plus_identity(f, p, true);
  } else {
    frag_mma<T, false>(f, L.S2, L.S4, p);
    frag_negate_plus_identity(f, p, false);
  }
  __syncthreads();
}


// Householder panel.  Rows [0, mp) x columns [0, jb) at X (ld ldx); the
// panel's first row is the diagonal row of its first column.  Writes back in
// place (R above the diagonal, beta on it, v below), the explicit unit-lower
// reflector block to Y (ld ldy), tau[0..jb), and from workgroup 0 the
// triangular factor T (ld ldt) of H_0 ... H_{jb-1} = I - Y T Y^T.
//
// Layout: workgroup w owns panel rows [w*RPW, (w+1)*RPW); wave g of it owns
// RPT consecutive rows of those, lane c holds column c of them in registers.
//
// Column j takes one device-wide reduction of q_c = sum_{rows > j} x_j x_c
// for every column c (x_j before the step).  For c >= j these give the norm
// of the pivot column and v^T x_c; for c < j, where x_c already holds the
// reflector y_c, they give the Gram entries S(c,j) = y_c^T y_j =
// x_c(j) + q_c / (alpha - beta), from which T is built column by column
// (T(j,j) = tau_j, T(0:j,j) = -tau_j T(0:j,0:j) S(0:j,j)).
// Partial sums of a round are added over workgroups in one fixed order, so
// every workgroup derives bitwise-identical reflectors.
//
// Second part (jb2 > 0): the launch also factors the jb2 columns to the right
// (columns NB.., diagonal rows NB..), on the same rows per workgroup.  While
// the first part is stored, each workgroup forms its share of
// W = Y1^T C2 (C2: the second part's columns); W is summed device-wide in
// three tagged rounds, and each workgroup applies C2 -= Y1 (T1^T W) to its own
// rows, which stay in registers for the second part.  That part's store forms
// S12 = Y1^T Y2 and the joined T (as with `join`), so one launch factors a
// 2 NB-column block: no second launch and no separate update between them.
template <class T>
__global__ __launch_bounds__(PANEL_THREADS) void panel_kernel(T* __restrict__ X, int64_t ldx,
                                                     int64_t mp, int jb, T* __restrict__ Y,
                                                     int64_t ldy, T* __restrict__ tau,
                                                     T* __restrict__ Tout, int ldt,
                                                     uint64_t* __restrict__ xch, uint32_t tag0,
                                                     unsigned* __restrict__ err, int zero_above,
                                                     PanelJoin<T> join, PanelWait pw, int jb2,
                                                     const unsigned* __restrict__ wait_flag) {
  using V2 = typename Vec2<T>::type;
  __shared__ T stage[64][NB + 1];
  __shared__ __attribute__((aligned(16))) T Ys[64][NB + 2];  // Y1 / C2 rows of a chunk; W or S12 sums
  __shared__ __attribute__((aligned(16))) T bc[PANEL_WAVES][RPT];  // pivot column, per wave
  __shared__ T red[PANEL_WAVES][NB];   // partial q of this workgroup, per wave
  __shared__ T red2[PANEL_WAVES][NB];  // gathered partial sums, per wave
  __shared__ T pivrow[NB];
  __shared__ __attribute__((aligned(16))) T Ssh[NB][NB + 2];  // Ssh[j][c] = S(c, j), c < j
  __shared__ __attribute__((aligned(16))) T Tsh[NB][NB + 2];  // Tsh[i][k] = T(i, k)
  __shared__ T tau_sh[NB];

  const int P = gridDim.x;
  const int wg = blockIdx.x;
  const int c = threadIdx.x & 63;                                   // column of this lane
  const int g = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // row group (wave)
  const int64_t row0 = static_cast<int64_t>(wg) * RPW;
  const int64_t myrow0 = row0 + static_cast<int64_t>(g) * RPT;     // first panel row of the wave
  const int myrow0i = static_cast<int>(myrow0);                      // panels have < 2^31 rows
  // exchange slots: [parity][P + 1][NB][2 words]; slot P carries the pivot row
  auto slot = [&](int par, int w, int col) {
    return xch + ((static_cast<int64_t>(par) * (P + 1) + w) * NB + col) * 2;
  };
  const bool two = jb2 > 0;
  // every workgroup builds T when the second part needs T1 (W -> T1^T W)
  const bool build_t = two || wg == 0;

  // ---- launched ahead of the update of its columns: wait for that update's flag,
  // then read X with loads that see it
  bool ok = true;
  const bool waited = wait_flag != nullptr;
  if (waited) {
    if (threadIdx.x == 0) ok = wait_flag_geq(wait_flag, 1u, err, pw.spin_limit);
    ok = !__syncthreads_or(ok ? 0 : 1);
  }
  auto load_x = [&](const T* p) -> T { return waited ? load_coherent(p) : *p; };

  // ---- load through LDS, 64 rows at a time (coalesced along columns)
  constexpr int WAVES_PER_CHUNK = 64 / RPT;
  T x[RPT];
  for (int k = 0; k < RPW / 64; ++k) {
    for (int e = threadIdx.x; e < 64 * NB; e += PANEL_THREADS) {
      const int r = e & 63, col = e >> 6;
      const int64_t gi = row0 + k * 64 + r;
      stage[r][col] = (gi < mp && col < jb) ? load_x(X + gi + col * ldx) : T(0);
    }
    __syncthreads();
    if (g / WAVES_PER_CHUNK == k) {
      const int r0 = (g % WAVES_PER_CHUNK) * RPT;
#pragma unroll
      for (int r = 0; r < RPT; ++r) x[r] = stage[r0 + r][c];
    }
    __syncthreads();
  }

  // a 64 x NB chunk of a column-major matrix, one chunk ahead in registers:
  // thread t holds row t & 63 of columns (t >> 6) + 8u
  constexpr int YPT = 64 * NB / PANEL_THREADS;
  static_assert(PANEL_THREADS % 64 == 0 && YPT * (PANEL_THREADS / 64) == NB, "chunk layout");
  const int ch_r = threadIdx.x & 63, ch_i = threadIdx.x >> 6;
  T yv[YPT];
  auto load_chunk = [&](const T* src, int64_t lds, int ncols, int k, bool coherent) {
    const int64_t gi = row0 + k * 64 + ch_r;
    const T* p = src + gi + ch_i * lds;
    const int64_t step = static_cast<int64_t>(PANEL_THREADS / 64) * lds;
#pragma unroll
    for (int u = 0; u < YPT; ++u)
      yv[u] = (gi < mp && ch_i + u * (PANEL_THREADS / 64) < ncols)
                  ? (coherent ? load_coherent(p + u * step) : p[u * step])
                  : T(0);
  };
  auto chunk_to_lds = [&](T (*dst)[NB + 2]) {
#pragma unroll
    for (int u = 0; u < YPT; ++u) dst[ch_r][ch_i + u * (PANEL_THREADS / 64)] = yv[u];
  };

  // the rows of the wave that holds the pivot row, transposed (the column loop
  // does not use Ys otherwise)
  constexpr int OWN_LD = RPT + 2;
  static_assert(64 * OWN_LD <= 64 * (NB + 2), "transposed rows fit in Ys");
  T* const own = &Ys[0][0];

#pragma unroll
  for (int part = 0; part < 2; ++part) {
    if (part == 1 && !two) break;
    const int p0 = part * NB;              // the part's first column and first pivot row
    const int jbp = part ? jb2 : jb;
    const uint32_t tagp = tag0 + static_cast<uint32_t>(part * NB);
    T* Xp = X + static_cast<int64_t>(p0) * ldx;
    T* Yp = Y + static_cast<int64_t>(p0) * ldy;
    T* Tp = Tout + p0 + static_cast<int64_t>(p0) * ldt;
    // S12 with an earlier panel: the first part of this launch, or the caller's
    const bool fuse = part == 1 || join.Y1 != nullptr;
    const T* jY1 = part == 1 ? Y : join.Y1;
    const int64_t jld = part == 1 ? ldy : join.ldy1;
    T* jT1 = part == 1 ? Tout : join.T1;
    const int jjb1 = part == 1 ? NB : join.jb1;

    if (build_t)
      for (int e = threadIdx.x; e < NB * (NB + 2); e += PANEL_THREADS) (&Tsh[0][0])[e] = T(0);
    __syncthreads();  // stage is reused below for the rows of R
    // Column c keeps its reflector unscaled (u_c = (alpha_c - beta_c) y_c below the
    // pivot) until the panel is done; my_rinv = 1 / (alpha_c - beta_c).
    T my_rinv = T(0);
    constexpr int TW = PANEL_WAVES - 1;  // the wave that builds T

    for (int j = 0; j < jbp && ok; ++j) {
      const int par = j & 1;
      const int pr = p0 + j;  // pivot row
      const uint32_t tag = tagp + static_cast<uint32_t>(j) + 1u;
      // lo: local index of the pivot row in this wave (uniform); rows r > lo lie below it
      const int lo = min(max(pr - myrow0i, -1), RPT);  // 32-bit, wave-uniform
      const bool owner = lo >= 0 && lo < RPT;

      // 1. the pivot column of this wave's rows, zeroed on and above the pivot
      //    row, into LDS.  Below the pivot, lane j copies it to bc[g].  The wave
      //    holding the pivot row stores all its rows transposed (lane c at
      //    own[c * OWN_LD ..]), takes the pivot row entry of every column from
      //    there, and lane j zeroes its own copy down to the pivot.  A wave above
      //    the pivot has nothing below it and skips the products.
      const bool below = lo < RPT;  // wave-uniform: some of its rows lie below the pivot
      const T* colp = &bc[g][0];
      if (lo < 0) {
        if (c == j) {
#pragma unroll
          for (int r = 0; r < RPT; r += 2) *reinterpret_cast<V2*>(&bc[g][r]) = Vec2<T>::make(x[r], x[r + 1]);
        }
      } else if (owner) {
        T* mine_t = own + c * OWN_LD;
#pragma unroll
        for (int r = 0; r < RPT; r += 2) *reinterpret_cast<V2*>(mine_t + r) = Vec2<T>::make(x[r], x[r + 1]);
        pivrow[c] = mine_t[lo];
        if (c == j)
          for (int r = 0; r <= lo; ++r) mine_t[r] = T(0);
        colp = own + j * OWN_LD;
      }
      wave_lds_sync();
      // 2. q_c over this wave's rows below the pivot
      T qa[4] = {T(0), T(0), T(0), T(0)};
      if (below) {
#pragma unroll
        for (int r = 0; r < RPT; r += 2) {
          const V2 xj = *reinterpret_cast<const V2*>(colp + r);
          qa[r & 2] += xj.x * x[r];
          qa[(r & 2) + 1] += xj.y * x[r + 1];
        }
      }
      red[g][c] = (qa[0] + qa[1]) + (qa[2] + qa[3]);
      __syncthreads();
      if (g == 0) {
        tagged_store(slot(par, wg, c), tag, sum_waves(red, c));
        if (pr >= row0 && pr < row0 + RPW) tagged_store(slot(par, P, c), tag, pivrow[c]);
      }
      // one wave finishes column j-1 of T while the exchange is in flight
      if (build_t && g == TW && j > 0) t_column(Tsh, Ssh, tau_sh, j - 1, c);
      // 3. gather, in one batch where possible: pivot row entries c and j, and this
      //    wave's share (w = g, g + PANEL_WAVES, ...) of the partial sums
      T piv[2];
      T sacc = T(0);
      {
        const uint64_t* ptrs[6] = {slot(par, P, c), slot(par, P, j)};
        int cnt = 2;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int w = g + PANEL_WAVES * u;
          ptrs[2 + u] = slot(par, w < P ? w : 0, c);
          cnt += (w < P) ? 1 : 0;
        }
        T vals[6];
        ok = tagged_load_all<T, 6>(ptrs, cnt, tag + pw.skew, vals, err, pw.spin_limit);
        piv[0] = vals[0];
        piv[1] = vals[1];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (2 + u < cnt) sacc += vals[2 + u];
      }
      for (int w0 = g + 4 * PANEL_WAVES; w0 < P && ok; w0 += 4 * PANEL_WAVES) {
        const uint64_t* ptrs[4];
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int w = w0 + PANEL_WAVES * u;
          ptrs[u] = slot(par, w < P ? w : 0, c);
          cnt += (w < P) ? 1 : 0;
        }
        T vals[4];
        ok = tagged_load_all<T, 4>(ptrs, cnt, tag + pw.skew, vals, err, pw.spin_limit);
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (u < cnt) sacc += vals[u];
      }
      red2[g][c] = sacc;
      // every wave failing to gather gives up together
      if (__syncthreads_or(ok ? 0 : 1)) {
        ok = false;
        break;
      }
      const T xcj = piv[0];
      const T alpha = piv[1];
      const T qc = sum_waves(red2, c);
      const T sigma2 = sum_waves(red2, j);
      // 4. reflector of column j
      T t = T(0), beta = alpha, rinv = T(0);
      if (sigma2 != T(0)) {
        const T norm = sqrt(alpha * alpha + sigma2);
        beta = (alpha >= T(0)) ? -norm : norm;
        rinv = T(1) / (alpha - beta);
        t = (beta - alpha) / beta;
      }
      if (c == j) my_rinv = rinv;
      if (g == 0) {
        // S(c,j) = y_c^T y_j with y_c = my_rinv u_c
        if (c < j) Ssh[j][c] = my_rinv * (xcj + qc * rinv);
        if (c == 0) tau_sh[j] = t;
        // row j of R is final after this step: R(j,c) for c >= j, kept for the end
        if (wg == 0) stage[j][c] = (c == j) ? beta : xcj - t * (xcj + qc * rinv);
      }
      // its action on the columns right of j, below the pivot:
      //   x_c -= tau (v^T x_c) v  with v = u_j / (alpha - beta),
      // one FMA per element for every lane: the broadcast column is zero on and
      // above the pivot row, and coef is zero for c <= j.
      const bool upd = c > j && t != T(0);
      const T coef = upd ? t * (xcj + qc * rinv) * rinv : T(0);
      if (below) {
#pragma unroll
        for (int r = 0; r < RPT; r += 2) {
          const V2 xj = *reinterpret_cast<const V2*>(colp + r);
          x[r] = fma(-coef, xj.x, x[r]);
          x[r + 1] = fma(-coef, xj.y, x[r + 1]);
        }
      }
    }
    __syncthreads();

    if (ok) {
      // scale each reflector below its pivot, and put the rows of R (kept in
      // stage) back on and above the diagonal
      const int loc = p0 + c - myrow0i;
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (c < jbp && r > loc) x[r] *= my_rinv;
      if (wg == 0 && myrow0i < p0 + jbp && myrow0i + RPT > p0) {
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
          const int row = myrow0i + r - p0;
          if (row >= 0 && row < jbp && c >= row) x[r] = stage[row][c];
        }
      }
    } else {
      // A device-side wait gave up: poison the outputs so the failure is visible.
      const T nan = static_cast<T>(__builtin_nan(""));
#pragma unroll
      for (int r = 0; r < RPT; ++r) x[r] = nan;
      if (g == 0) tau_sh[c] = nan;
    }
    __syncthreads();

    // ---- last column of T, then T and tau out
    if (build_t) {
      if (ok && g == TW && jbp > 0) t_column(Tsh, Ssh, tau_sh, jbp - 1, c);
      __syncthreads();
    }
    if (wg == 0) {
      for (int e = threadIdx.x; e < NB * NB; e += PANEL_THREADS) {
        const int i = e % NB, k = e / NB;
        if (i < jbp && k < jbp)
          Tp[i + static_cast<int64_t>(k) * ldt] = ok ? Tsh[i][k] : static_cast<T>(__builtin_nan(""));
      }
      if (threadIdx.x < jbp) tau[p0 + threadIdx.x] = tau_sh[threadIdx.x];
      // Y is zero in the zero_above rows above the panel (an earlier panel of the same block)
      for (int e = threadIdx.x; e < zero_above * jbp; e += PANEL_THREADS)
        Yp[(e % zero_above) - zero_above + static_cast<int64_t>(e / zero_above) * ldy] = T(0);
    }

    // ---- store: the part in place, and explicit Y (0 above, 1 on the diagonal).
    // With S12 to form, the partial S12(i, c) = sum over this workgroup's rows of
    // Y1(r, i) Y2(r, c); before a second part, the partial W(i, c) = sum of
    // Y1(r, i) C2(r, c), and the rows of C2 are taken into registers.  Thread
    // (wave g, lane c) holds entries i = 8g .. 8g+7.
    const bool form_w = part == 0 && two;
    // 64 x 64 products on the matrix cores: wave g owns rows ib .. ib+15 and the
    // two 16-column blocks at cb0 and cb0 + 16 of the result
    using Mma = PanelMma<T>;
    const int l16 = c & 15, lk = c >> 4;
    const int ib = (g >> 1) * 16, cb0 = (g & 1) * 32;
    typename Mma::acc acc0 = {T(0), T(0), T(0), T(0)}, acc1 = {T(0), T(0), T(0), T(0)};
    if (fuse) load_chunk(jY1, jld, jjb1, 0, false);
    if (form_w) load_chunk(X + static_cast<int64_t>(NB) * ldx, ldx, jb2, 0, waited);
    for (int k = 0; k < RPW / 64; ++k) {
      const bool mine = g / WAVES_PER_CHUNK == k;
      const int r0 = (g % WAVES_PER_CHUNK) * RPT;
      if (mine) {
#pragma unroll
        for (int r = 0; r < RPT; ++r) stage[r0 + r][c] = x[r];
      }
      if (fuse) {
        chunk_to_lds(Ys);
        if (k + 1 < RPW / 64) load_chunk(jY1, jld, jjb1, k + 1, false);
      }
      if (form_w) {
        chunk_to_lds(Ys);
        if (k + 1 < RPW / 64) load_chunk(X + static_cast<int64_t>(NB) * ldx, ldx, jb2, k + 1, waited);
      }
      __syncthreads();
      for (int e = threadIdx.x; e < 64 * NB; e += PANEL_THREADS) {
        const int r = e & 63, col = e >> 6;
        const int64_t gi = row0 + k * 64 + r, dg = p0 + col;
        if (gi < mp && col < jbp) {
          const T v = stage[r][col];
          Xp[gi + col * ldx] = v;
          Yp[gi + col * ldy] = (gi > dg) ? v : (gi == dg ? T(1) : T(0));
        }
      }
      if (fuse) {
        // S12(i, c) += sum over the chunk of Y1(r, i) Y2(r, c); Y2 from the staged
        // part (v below its diagonal, 1 on it, 0 above and in unused columns)
#pragma unroll 4
        for (int ks = 0; ks < 16; ++ks) {
          const int r = 4 * ks + lk;
          const int64_t gi = row0 + k * 64 + r;
          const T a = Ys[r][ib + l16];
          const int c0 = cb0 + l16, c1 = c0 + 16;
          const T s0 = stage[r][c0], s1 = stage[r][c1];
          const T b0 = c0 < jbp ? ((gi > p0 + c0) ? s0 : (gi == p0 + c0 ? T(1) : T(0))) : T(0);
          const T b1 = c1 < jbp ? ((gi > p0 + c1) ? s1 : (gi == p0 + c1 ? T(1) : T(0))) : T(0);
          acc0 = Mma::run(a, b0, acc0);
          acc1 = Mma::run(a, b1, acc1);
        }
      }
      if (form_w) {
        // W(i, c) += sum over the chunk of Y1(r, i) C2(r, c); Y1 from the staged
        // part (v below the diagonal, 1 on it, 0 above)
#pragma unroll 4
        for (int ks = 0; ks < 16; ++ks) {
          const int r = 4 * ks + lk;
          const int64_t gi = row0 + k * 64 + r;
          const int i = ib + l16;
          const T sv = stage[r][i];
          const T a = (gi > i) ? sv : (gi == i ? T(1) : T(0));
          acc0 = Mma::run(a, Ys[r][cb0 + l16], acc0);
          acc1 = Mma::run(a, Ys[r][cb0 + 16 + l16], acc1);
        }
        if (mine) {
#pragma unroll
          for (int r = 0; r < RPT; ++r) x[r] = Ys[r0 + r][c];
        }
      }
      __syncthreads();
    }
    if (!fuse && !form_w) return;

    // ---- device-wide sum of the 64 x 64 partials (W, or S12)
    // round A: publish this workgroup's partial sums
    const uint32_t tagS = tagp + static_cast<uint32_t>(NB) + 1u;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ib + Mma::row(lk, v);
      uint64_t* pw0 = join.ps + (static_cast<int64_t>(wg) * kJoinEntries + i * NB + cb0 + l16) * 2;
      tagged_store(pw0, tagS, ok ? acc0[v] : static_cast<T>(__builtin_nan("")));
      tagged_store(pw0 + 32, tagS, ok ? acc1[v] : static_cast<T>(__builtin_nan("")));
    }
    // round B: this workgroup sums its share of the entries over all workgroups.
    // With few entries per workgroup, `parts` threads share an entry, each adding
    // the partials of workgroups part, part + parts, ...; the parts are then added
    // in order (a fixed order, so every run gives the same sums).
    {
      const int per = (kJoinEntries + P - 1) / P;
      const int e_end = min(kJoinEntries, (wg + 1) * per);
      const int parts = max(1, min(PANEL_THREADS / per, 8));
      T* red_b = &red[0][0];  // PANEL_WAVES * NB = 512 values
      for (int base = wg * per; base < e_end; base += PANEL_THREADS / parts) {
        const int slot_e = threadIdx.x % (PANEL_THREADS / parts), sub = threadIdx.x / (PANEL_THREADS / parts);
        const int e = base + slot_e;
        T total = T(0);
        if (e < e_end && sub < parts) {
          for (int p1 = sub; p1 < P && ok; p1 += 8 * parts) {
            const uint64_t* ptrs[8];
            int cnt = 0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int src = p1 + u * parts;
              ptrs[u] = join.ps + (static_cast<int64_t>(src < P ? src : 0) * kJoinEntries + e) * 2;
              cnt += (src < P) ? 1 : 0;
            }
            T vals[8];
            ok = tagged_load_all<T, 8>(ptrs, cnt, tagS + pw.skew, vals, err, pw.spin_limit);
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (u < cnt) total += vals[u];
          }
        }
        __syncthreads();
        if (sub < parts) red_b[sub * (PANEL_THREADS / parts) + slot_e] = total;
        __syncthreads();
        if (sub == 0 && e < e_end) {
          T sum = T(0);
          for (int q = 0; q < parts; ++q) sum += red_b[q * (PANEL_THREADS / parts) + slot_e];
          tagged_store(join.sums + static_cast<int64_t>(e) * 2, tagS, ok ? sum : static_cast<T>(__builtin_nan("")));
        }
      }
    }
    // round C: the sums into Ys[i][c] (every workgroup for W, workgroup 0 for S12)
    if (fuse && wg != 0) return;
    static_assert(kJoinEntries == 8 * PANEL_THREADS, "round C loads eight sums per thread");
    if (ok) {
      const uint64_t* ptrs[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) ptrs[u] = join.sums + static_cast<int64_t>(threadIdx.x + u * PANEL_THREADS) * 2;
      T v[8];
      ok = tagged_load_all<T, 8>(ptrs, 8, tagS + pw.skew, v, err, pw.spin_limit);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = threadIdx.x + u * PANEL_THREADS;
        Ys[e / NB][e % NB] = v[u];
      }
    }

    if (form_w) {
      ok = !__syncthreads_or(ok ? 0 : 1);
      // W' = T1^T W into Ssh (Ssh[i][c] = W'(i, c)): a(i, k) = T1(k, i)
      typename Mma::acc w0 = {T(0), T(0), T(0), T(0)}, w1 = {T(0), T(0), T(0), T(0)};
#pragma unroll 4
      for (int ks = 0; ks < 16; ++ks) {
        const int kk = 4 * ks + lk;
        const T a = Tsh[kk][ib + l16];
        w0 = Mma::run(a, Ys[kk][cb0 + l16], w0);
        w1 = Mma::run(a, Ys[kk][cb0 + 16 + l16], w1);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = ib + Mma::row(lk, v);
        Ssh[i][cb0 + l16] = w0[v];
        Ssh[i][cb0 + 16 + l16] = w1[v];
      }
      __syncthreads();  // W read from Ys by every wave; W' complete in Ssh
      // C2 -= Y1 W' on this workgroup's rows, 64 rows at a time: the owners put
      // their rows of C2 into Ys, each wave updates a 16 x 32 block of the chunk
      // on the matrix cores, the owners take the rows back
      load_chunk(Y, ldy, NB, 0, false);
      for (int k = 0; k < RPW / 64; ++k) {
        const bool mine = g / WAVES_PER_CHUNK == k;
        const int r0 = (g % WAVES_PER_CHUNK) * RPT;
        if (mine) {
#pragma unroll
          for (int r = 0; r < RPT; ++r) Ys[r0 + r][c] = x[r];
        }
#pragma unroll
        for (int u = 0; u < YPT; ++u) stage[ch_r][ch_i + u * (PANEL_THREADS / 64)] = yv[u];
        if (k + 1 < RPW / 64) load_chunk(Y, ldy, NB, k + 1, false);
        __syncthreads();
        typename Mma::acc u0, u1;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = ib + Mma::row(lk, v);
          u0[v] = Ys[r][cb0 + l16];
          u1[v] = Ys[r][cb0 + 16 + l16];
        }
#pragma unroll 4
        for (int ks = 0; ks < 16; ++ks) {
          const int kk = 4 * ks + lk;
          const T a = -stage[ib + l16][kk];  // a(r, k) = -Y1(r, k)
          u0 = Mma::run(a, Ssh[kk][cb0 + l16], u0);
          u1 = Mma::run(a, Ssh[kk][cb0 + 16 + l16], u1);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = ib + Mma::row(lk, v);
          Ys[r][cb0 + l16] = u0[v];
          Ys[r][cb0 + 16 + l16] = u1[v];
        }
        __syncthreads();
        if (mine) {
#pragma unroll
          for (int r = 0; r < RPT; ++r) x[r] = ok ? Ys[r0 + r][c] : static_cast<T>(__builtin_nan(""));
        }
        __syncthreads();
      }
      continue;
    }

    // ---- workgroup 0 joins T: T12 = -T1 (S12 T2) with T2 in Tsh
    for (int e = threadIdx.x; e < NB * NB; e += PANEL_THREADS) {
      const int i = e % NB, kk = e / NB;
      Ssh[i][kk] = (i < jjb1 && kk < jjb1) ? jT1[i + static_cast<int64_t>(kk) * ldt] : T(0);
    }
    ok = !__syncthreads_or(ok ? 0 : 1);
    constexpr int PER = NB * NB / PANEL_THREADS;
    T uacc[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = threadIdx.x + r * PANEL_THREADS, i = e % NB, j = e / NB;
      T a = 0;
      if (j < jbp)
        for (int kk = 0; kk <= j; ++kk) a += Ys[i][kk] * Tsh[kk][j];
      uacc[r] = a;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = threadIdx.x + r * PANEL_THREADS;
      Ys[e % NB][e / NB] = uacc[r];
    }
    __syncthreads();
    const T nan = static_cast<T>(__builtin_nan(""));
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = threadIdx.x + r * PANEL_THREADS, i = e % NB, j = e / NB;
      T a = 0;
      for (int kk = i; kk < jjb1; ++kk) a += Ssh[i][kk] * Ys[kk][j];
      if (i < jjb1 && j < jbp) jT1[i + static_cast<int64_t>(jjb1 + j) * ldt] = ok ? -a : nan;
      if (i < jbp && j < jjb1) jT1[jjb1 + i + static_cast<int64_t>(j) * ldt] = T(0);
    }
    return;
  }
}

// ---------------------------------------------------------------------------
// The panel kernel the QR uses: one launch per block of up to 128 columns, two
// 64-column parts, each factored without a device-wide step per column
// (CholeskyQR2, or the tall-skinny QR when that is refused, then the rebuilt
// Householder vectors).  The panel never lives in registers: each pass streams
// this workgroup's rows (CQR_RPW of them) through LDS 64 rows at a time, the
// next chunk's loads in flight while the matrix cores work on the current one.

// Sum of N 64 x 64 matrices over the P workgroups of the launch, every
// workgroup getting bitwise the same sums (one fixed order): this workgroup's
// terms are in M[0..N) (LDS) on entry, the sums on return.  Each workgroup adds
// up a slice of the entries over all terms (staged in M, which is free once the
// terms are published: its N 64 x 66 arrays hold any slice's P terms for
// P <= 128 N), then every workgroup gathers the slices: two announced
// exchanges through part (P x N NB^2 words) and sum (N NB^2), flagged in fa and
// fb.  False if a wait expired.
template <class T, int N>
__device__ __forceinline__ bool allreduce_n(T (*const (&M)[N])[NB + 2], int P, int wg, T* part, T* sum, uint64_t* fa,
                                            uint64_t* fb, uint32_t tag, unsigned* err, const PanelWait& pw) {
  if (P == 1) return true;
  constexpr int E = N * NB * NB, BLK = NB * (NB + 2);
  const int tid = opaque(static_cast<int>(threadIdx.x));
  T* const mine = part + static_cast<int64_t>(wg) * E;
  for (int e = tid; e < E; e += PANEL_THREADS) {
    const int b = e / (NB * NB), r = e % (NB * NB);
    store_agent(mine + e, M[b][r & (NB - 1)][r / NB]);
  }
  raise_flag(fa + wg, tag);
  bool ok = tid >= P || await_flag(fa + tid, tag + pw.skew, err, pw.spin_limit);
  if (__syncthreads_or(ok ? 0 : 1)) return false;
  // this workgroup's slice [e0, e1): every term of it into M, entry (e - e0) P + q, with the
  // loads of a thread all in flight; then each sum in the order q = 0, 1, ...
  const int e0 = E * wg / P, e1 = E * (wg + 1) / P, ne = e1 - e0, nt = ne * P;
  auto flat = [&](int f) -> T& { return (&M[f / BLK][0][0])[f % BLK]; };
  constexpr int U = 8;
  for (int i0 = tid; i0 < nt; i0 += U * PANEL_THREADS) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * PANEL_THREADS;
      v[u] = i < nt ? load_coherent(part + static_cast<int64_t>(i % P) * E + e0 + i / P) : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * PANEL_THREADS;
      if (i < nt) flat(i) = v[u];
    }
  }
  __syncthreads();
  for (int t = tid; t < ne; t += PANEL_THREADS) {
    T a = T(0);
    for (int q = 0; q < P; ++q) a += flat(t * P + q);
    store_agent(sum + e0 + t, a);
  }
  raise_flag(fb + wg, tag);
  ok = tid >= P || await_flag(fb + tid, tag + pw.skew, err, pw.spin_limit);
  if (__syncthreads_or(ok ? 0 : 1)) return false;
  for (int e00 = 0; e00 < E; e00 += NB * NB) {
    T v[NB * NB / PANEL_THREADS];
#pragma unroll
    for (int u = 0; u < NB * NB / PANEL_THREADS; ++u) v[u] = load_coherent(sum + e00 + tid + u * PANEL_THREADS);
#pragma unroll
    for (int u = 0; u < NB * NB / PANEL_THREADS; ++u) {
      const int r = tid + u * PANEL_THREADS;
      M[e00 / (NB * NB)][r & (NB - 1)][r / NB] = v[u];
    }
  }
  __syncthreads();
  return true;
}

// One 64 x 64 matrix summed over the workgroups (the factorisation's exchanges).
template <class T>
__device__ __forceinline__ bool allreduce64(T (*M)[NB + 2], int P, int wg, const TsqrXch& xt, uint32_t tag,
                                            unsigned* err, const PanelWait& pw) {
  T (*const blocks[1])[NB + 2] = {M};
  uint64_t* const fa = xt.flags + kTsqrUnits + 1;
  return allreduce_n<T, 1>(blocks, P, wg, reinterpret_cast<T*>(xt.gram),
                           reinterpret_cast<T*>(xt.gram + static_cast<int64_t>(P) * NB * NB), fa, fa + kMaxCqrWgs, tag,
                           err, pw);
}

// A 64-row chunk of a column-major matrix in registers: thread t holds row
// t & 63 of columns (t >> 6) + 8u.
template <class T>
struct ChunkRegs {
  T v[64 * NB / PANEL_THREADS];
};

// Where this workgroup's rows of one part are and how to move them.
template <class T>
struct CqrRows {
  int64_t row0, mp;  // first block row of the workgroup; rows of the block
  int lbase;         // first row of the part this workgroup holds (p0 in workgroup 0)
  int p0, jbp;       // the part's first pivot row and width
  int kc;            // first chunk holding part rows (the pivot rows in workgroup 0)
  // rows row0 + 64k .. of a column-major matrix (ld lds) into registers; 0 outside
  // the part (lane indices through opaque(): the addresses are formed at each
  // call, not hoisted out of the phases and held in registers or scratch)
  __device__ __forceinline__ void load(ChunkRegs<T>& R, const T* src, int64_t lds, int k, bool coherent) const {
    const int r = opaque(threadIdx.x & 63), i0 = opaque(threadIdx.x >> 6);
    const int64_t gi = row0 + k * 64 + r;
    const bool rowok = gi < mp && gi >= lbase;
#pragma unroll
    for (int u = 0; u < 64 * NB / PANEL_THREADS; ++u) {
      const int col = i0 + u * (PANEL_THREADS / 64);
      const T* p = src + gi + static_cast<int64_t>(col) * lds;
      R.v[u] = (rowok && col < jbp) ? (coherent ? load_coherent(p) : *p) : T(0);
    }
  }
  __device__ __forceinline__ void put(T (*dst)[NB + 2], const ChunkRegs<T>& R) const {
    const int r = threadIdx.x & 63, i0 = threadIdx.x >> 6;
#pragma unroll
    for (int u = 0; u < 64 * NB / PANEL_THREADS; ++u) dst[r][i0 + u * (PANEL_THREADS / 64)] = R.v[u];
  }
  __device__ __forceinline__ void out(const T (*sr)[NB + 2], T* dst, int64_t ldd, int k) const {
    const int r = opaque(threadIdx.x & 63), i0 = opaque(threadIdx.x >> 6);
    const int64_t gi = row0 + k * 64 + r;
    if (!(gi < mp && gi >= lbase)) return;
#pragma unroll
    for (int u = 0; u < 64 * NB / PANEL_THREADS; ++u) {
      const int col = i0 + u * (PANEL_THREADS / 64);
      if (col < jbp) dst[gi + static_cast<int64_t>(col) * ldd] = sr[r][col];
    }
  }
};

// Z <- Z B for this workgroup's rows of Z (ld ldz), B in LDS; S is the chunk buffer.
template <class T>
__device__ __forceinline__ void cqr_rows_times(const CqrRows<T>& rw, T* Z, int64_t ldz, const T (*B)[NB + 2],
                                               T (*S)[NB + 2], const FragPos& fp) {
  ChunkRegs<T> cur;
  rw.load(cur, Z, ldz, rw.kc, false);
  for (int k = rw.kc; k < CQR_CHUNKS; ++k) {
    rw.put(S, cur);
    __syncthreads();
    if (k + 1 < CQR_CHUNKS) rw.load(cur, Z, ldz, k + 1, false);
    Frag<T> f;
    frag_zero(f);
    frag_mma<T, false>(f, S, B, fp);
    __syncthreads();
    frag_to_lds(f, S, fp);
    __syncthreads();
    rw.out(S, Z, ldz, k);
    __syncthreads();
  }
}

// M (LDS) <- its upper triangle mirrored below the diagonal, identity outside
// [0, jbp)^2.
template <class T>
__device__ __forceinline__ void sym_pad(T (*M)[NB + 2], int jbp) {
  for (int e = opaque(static_cast<int>(threadIdx.x)); e < NB * NB; e += PANEL_THREADS) {
    const int i = e & (NB - 1), j = e / NB;
    if (i >= jbp || j >= jbp)
      M[i][j] = (i == j) ? T(1) : T(0);
    else if (i > j)
      M[i][j] = M[j][i];
  }
  __syncthreads();
}

// One 64-column part.  On entry the part's columns are in Xp (rows of the
// block, ld ldx; `coherent` when another kernel may have written them after
// this one started).  On return Yp holds the explicit reflectors of this
// workgroup's rows (1 on the diagonal, 0 above), Xp R on and above the
// diagonal of the pivot rows and the reflectors below it, L.S4 the part's T
// (workgroup 0, and every workgroup when all_t) and L.tau its tau.
//
// CholeskyQR2 (Yamamoto, Nakatsukasa, Yanagisawa, Fukaya 2015): G1 = X^T X
// summed over the workgroups, G1 = R1^T R1, Q1 = X R1^-1 (into the Y rows) with
// G2 = Q1^T Q1 formed in the same pass, G2 = R2^T R2, R = R2 R1; Q = Q1 R2^-1
// is never stored: the reconstruction needs only its top rows, and the
// reflectors below them are -Q U^-1 = -Q1 (R2^-1 U^-1).  Taken when both
// factorizations have positive pivots, G2 is within 0.1 of I entrywise (the
// first pass left Q1 well conditioned, the second restores orthogonality to
// rounding level) and the part is not already upper triangular (where the
// Householder form is exact).  Otherwise the tall-skinny QR: a Householder QR
// of each workgroup's rows, a tree that stacks the R factors of up to 4 units
// per level and factors the stack in every workgroup of the group, and
// Q_w = Q_leaf M_w.  Either way workgroup 0 then factors S - Q_top = L U and
// sends R2^-1 U^-1 (or U^-1) and T.
template <class T>
__device__ __forceinline__ bool cqr_part(const CqrRows<T>& rw, int P, int wg, int g, int c, T* __restrict__ Xp,
                                         int64_t ldx, T* __restrict__ Yp, int64_t ldy, bool coherent,
                                         const TsqrXch& xt, uint32_t tagp, unsigned* err, const PanelWait& pw,
                                         bool all_t, bool use_chol, const TsqrLds<T>& L) {
  const uint32_t tagR = tagp + 1, tagU = tagp + 2, tagG = tagp + 3;
  FragPos fp{(g >> 1) * 16, (g & 1) * 32, c & 15, c >> 4};
  auto phase = [&]() {
    c = opaque(c);
    fp.l16 = c & 15;
    fp.lk = c >> 4;
  };
  const int jbp = rw.jbp, p0 = rw.p0, kc = rw.kc;
  T* const ubuf = L.aux;          // pivots, then (at + NB) their reciprocals
  T* const sgn = L.aux + 2 * NB;  // signs of the reconstruction
  T* const dsq = L.aux + 3 * NB;  // square roots of the Cholesky pivots
  Frag<T> f;
  bool chol = use_chol;

  // ---- G1 = X^T X over this workgroup's rows; is the part upper triangular already?
  if (chol) {
    phase();
    frag_zero(f);
    int below_nz = 0;
    ChunkRegs<T> cur;
    rw.load(cur, Xp, ldx, kc, coherent);
    for (int k = kc; k < CQR_CHUNKS; ++k) {
      {
        const int r = threadIdx.x & 63, i0 = threadIdx.x >> 6;
        const int64_t gi = rw.row0 + k * 64 + r;
#pragma unroll
        for (int u = 0; u < 64 * NB / PANEL_THREADS; ++u)
          below_nz |= (gi > p0 + i0 + u * (PANEL_THREADS / 64) && cur.v[u] != T(0)) ? 1 : 0;
      }
      rw.put(L.S1, cur);
      __syncthreads();
      if (k + 1 < CQR_CHUNKS) rw.load(cur, Xp, ldx, k + 1, coherent);
      frag_mma<T, true>(f, L.S1, L.S1, fp);
      __syncthreads();
    }
    frag_to_lds(f, L.S3, fp);
    // the triangular test rides in entry (63, 0), below the diagonal (mirrored over afterwards)
    const int any = __syncthreads_or(below_nz);
    if (threadIdx.x == 0) L.S3[NB - 1][0] = any ? T(1) : T(0);
    __syncthreads();
    if (!allreduce64(L.S3, P, wg, xt, tagG, err, pw)) return false;
    chol = L.S3[NB - 1][0] != T(0);  // some workgroup holds a nonzero below the diagonal
    __syncthreads();
    sym_pad(L.S3, jbp);
  }
  // ---- G1 = L U, U = D R1 (no pivoting; every pivot must be positive)
  if (chol) {
    phase();
    blocked_lu(L.S3, false, ubuf, sgn, L.S2, L.S1, g, c);
    int bad = 0;
    if (threadIdx.x < NB) {
      const T u = ubuf[threadIdx.x];
      bad = !(u > T(0)) ? 1 : 0;
      dsq[threadIdx.x] = sqrt(u);
    }
    chol = !__syncthreads_or(bad);
  }
  if (chol) {
    phase();
    // R1^-1 = U^-1 diag(sqrt u) into S2 (S1 scratch); R1 = diag(sqrt u)^-1 U into S4
    tri_join<T, true>(L.S2, [&](int a, int b) { return L.S3[a][b]; }, L.S1, g, c);
    for (int e = opaque(static_cast<int>(threadIdx.x)); e < NB * NB; e += PANEL_THREADS) {
      const int i = e & (NB - 1), j = e / NB;
      L.S2[i][j] *= dsq[j];
      L.S4[i][j] = i <= j ? L.S3[i][j] / dsq[i] : T(0);
    }
    __syncthreads();
    // ---- Q1 = X R1^-1 into the Y rows, and G2 = Q1^T Q1
    phase();
    Frag<T> g2;
    frag_zero(g2);
    ChunkRegs<T> cur;
    rw.load(cur, Xp, ldx, kc, coherent);
    for (int k = kc; k < CQR_CHUNKS; ++k) {
      rw.put(L.S1, cur);
      __syncthreads();
      if (k + 1 < CQR_CHUNKS) rw.load(cur, Xp, ldx, k + 1, coherent);
      frag_zero(f);
      frag_mma<T, false>(f, L.S1, L.S2, fp);
      __syncthreads();
      frag_to_lds(f, L.S1, fp);
      __syncthreads();
      frag_mma<T, true>(g2, L.S1, L.S1, fp);
      rw.out(L.S1, Yp, ldy, k);
      __syncthreads();
    }
    frag_to_lds(g2, L.S3, fp);
    __syncthreads();
    if (!allreduce64(L.S3, P, wg, xt, tagG + 1, err, pw)) return false;
    sym_pad(L.S3, jbp);
    // the first pass must have left Q1 nearly orthonormal
    int far = 0;
    for (int e = opaque(static_cast<int>(threadIdx.x)); e < NB * NB; e += PANEL_THREADS) {
      const T d = L.S3[e & (NB - 1)][e / NB] - ((e & (NB - 1)) == e / NB ? T(1) : T(0));
      far |= !(d <= T(0.1) && d >= T(-0.1)) ? 1 : 0;  // also NaN
    }
    chol = !__syncthreads_or(far);
  }
  if (chol) {
    phase();
    blocked_lu(L.S3, false, ubuf, sgn, L.S2, L.S1, g, c);  // G2 = L U, U = D R2
    int bad = 0;
    if (threadIdx.x < NB) {
      const T u = ubuf[threadIdx.x];
      bad = !(u > T(0)) ? 1 : 0;
      dsq[threadIdx.x] = sqrt(u);
    }
    chol = !__syncthreads_or(bad);
  }
  if (chol) {
    phase();
    // R2^-1 into S2; R = R2 R1 into S3
    tri_join<T, true>(L.S2, [&](int a, int b) { return L.S3[a][b]; }, L.S1, g, c);
    for (int e = opaque(static_cast<int>(threadIdx.x)); e < NB * NB; e += PANEL_THREADS) L.S2[e & (NB - 1)][e / NB] *= dsq[e / NB];
    frag_zero(f);
    frag_mma_f(f, [&](int i, int k) { return k >= i ? L.S3[i][k] / dsq[i] : T(0); },
               [&](int k, int j) { return L.S4[k][j]; }, fp, 0, NB);
    __syncthreads();
    frag_to_lds(f, L.S3, fp);
    __syncthreads();
  } else {
    // ---- tall-skinny QR: the leaf needs the rows in registers (every row, from X)
    phase();
    const int myrow0i = static_cast<int>(rw.row0) + g * CQR_RPT;
    constexpr int WAVES_PER_CHUNK = 64 / CQR_RPT;
    const int kw = g / WAVES_PER_CHUNK, r0w = (g % WAVES_PER_CHUNK) * CQR_RPT;
    {
      T x[CQR_RPT];
#pragma unroll
      for (int r = 0; r < CQR_RPT; ++r) {
        const int64_t gi = myrow0i + r;
        const T* p = Xp + gi + static_cast<int64_t>(c) * ldx;
        x[r] = (gi < rw.mp && gi >= rw.lbase && c < jbp) ? (coherent ? load_coherent(p) : *p) : T(0);
      }
      tsqr_leaf<T, CQR_RPT>(x, jbp, rw.lbase, myrow0i, g, c, L);
      const int loc = rw.lbase + c - myrow0i;  // local row of lane c's pivot in this wave
      if (P == 1) {
        // one leaf: its reflectors are the part's; Y explicit, R onto the pivot rows of X
        for (int k = kc; k < CQR_CHUNKS; ++k) {
          if (kw == k) {
#pragma unroll
            for (int r = 0; r < CQR_RPT; ++r) {
              L.S2[r0w + r][c] = c < jbp ? (r > loc ? x[r] : (r == loc ? T(1) : T(0))) : T(0);
              const int row = myrow0i + r - p0;
              L.S3[r0w + r][c] = (row >= 0 && row < jbp && c >= row) ? L.S1[row][c] : x[r];
            }
          }
          __syncthreads();
          rw.out(L.S2, Yp, ldy, k);
          rw.out(L.S3, Xp, ldx, k);
          __syncthreads();
        }
        return true;
      }
      phase();
      tsqr_publish_tri(L.S1, xt.tri + static_cast<int64_t>(wg) * kTriEntries, xt.flags + wg, tagR);
      // the leaf's explicit Q, Qt = [I; 0] - Y_w (T_w Y_w0^T), into the Y rows
      if (kw == kc) {
#pragma unroll
        for (int r = 0; r < CQR_RPT; ++r)
          L.S2[r0w + r][c] = c < jbp ? (r > loc ? x[r] : (r == loc ? T(1) : T(0))) : T(0);
      }
      __syncthreads();
      frag_zero(f);
      frag_mma<T, false, true>(f, L.S4, L.S2, fp);  // T_w Y_w0^T
      frag_to_lds(f, L.S3, fp);
      for (int k = kc; k < CQR_CHUNKS; ++k) {
        __syncthreads();
        if (kw == k) {
#pragma unroll
          for (int r = 0; r < CQR_RPT; ++r)
            L.S2[r0w + r][c] = c < jbp ? (r > loc ? x[r] : (r == loc ? T(1) : T(0))) : T(0);
        }
        __syncthreads();
        frag_zero(f);
        frag_mma<T, false>(f, L.S2, L.S3, fp);
        frag_negate_plus_identity(f, fp, k == kc);
        __syncthreads();
        frag_to_lds(f, L.S2, fp);
        __syncthreads();
        rw.out(L.S2, Yp, ldy, k);
      }
      __syncthreads();
    }
    // tree
    Frag<T> fM;
    frag_identity(fM, fp);
    {
      T tri[RPT];
      int units = P, off = 0, span = 1;  // units of the current level, their first slot, workgroups per unit
      while (units > 1) {
        phase();
        const int unit = wg / span, grp = unit / kTsqrFan, s = unit % kTsqrFan;
        const int K = min(kTsqrFan, units - grp * kTsqrFan);
        if (span > 1 && wg % span == 0)  // the unit's first workgroup publishes its R (level 0 did above)
          tsqr_publish_tri(L.S1, xt.tri + static_cast<int64_t>(off + unit) * kTriEntries, xt.flags + off + unit,
                           tagR);
        if (K >= 2) {
          __syncthreads();
          const int first = off + grp * kTsqrFan;
          if (!tsqr_node(tri, xt.tri + static_cast<int64_t>(first) * kTriEntries, xt.flags + first, K, tagR, jbp, g,
                         c, L, err, pw))
            return false;
          Frag<T> fb;
          tsqr_node_q(tri, s, g, c, L, fp, fb);
          frag_to_lds(fM, L.S3, fp);
          frag_to_lds(fb, L.S2, fp);
          __syncthreads();
          frag_zero(fM);
          frag_mma<T, false>(fM, L.S3, L.S2, fp);  // M <- M B
          __syncthreads();
        }
        off += units;
        units = (units + kTsqrFan - 1) / kTsqrFan;
        span *= kTsqrFan;
      }
    }
    // Q_w = Qt M into the Y rows; the root's R from S1 into S3
    phase();
    frag_to_lds(fM, L.S2, fp);
    for (int e = opaque(static_cast<int>(threadIdx.x)); e < NB * NB; e += PANEL_THREADS) L.S3[e & (NB - 1)][e / NB] = L.S1[e & (NB - 1)][e / NB];
    __syncthreads();
    cqr_rows_times(rw, Yp, ldy, L.S2, L.S1, fp);
  }
  // The Y rows hold Q1 (Q = Q1 R2^-1, R2^-1 in S2) or Q itself; R is in S3 (up to the signs S).

  // ---- reconstruction: workgroup 0 factors S - Q_top = L U, sends M = R2^-1 U^-1 (U^-1) and T
  phase();
  const int tid = opaque(static_cast<int>(threadIdx.x));
  T* const xu = reinterpret_cast<T*>(xt.recon);  // M (NB^2), then T (NB^2), entry i + NB c
  uint64_t* const rflag = xt.flags + kTsqrUnits;
  if (wg == 0) {
    Frag<T> fR2;
    frag_zero(fR2);
    {
      ChunkRegs<T> cur;
      rw.load(cur, Yp, ldy, kc, false);
      rw.put(L.S4, cur);
    }
    __syncthreads();
    frag_zero(f);
    if (chol) {
      frag_mma<T, false>(f, L.S4, L.S2, fp);  // Q_top = Q1_top R2^-1
      frag_from_lds(fR2, L.S2, fp);
    } else {
      frag_from_lds(f, L.S4, fp);
    }
    frag_negate_plus_identity(f, fp, false);
    __syncthreads();
    frag_to_lds(f, L.S1, fp);
    // S - Q_top = L U in S1 (S diagonal, chosen during the elimination); inverses of
    // the diagonal blocks of U and L in S2, S4
    blocked_lu(L.S1, true, ubuf, sgn, L.S2, L.S4, g, c);
    phase();
    // the pivot rows: Y = L (unit lower), X = L below the diagonal and S R on and above it
    for (int e = tid; e < NB * NB; e += PANEL_THREADS) {
      const int i = e & (NB - 1), j = e / NB;
      const int64_t gi = p0 + i;
      if (gi < rw.mp && j < jbp) {
        const T lij = L.S1[i][j];
        Yp[gi + static_cast<int64_t>(j) * ldy] = i > j ? lij : (i == j ? T(1) : T(0));
        Xp[gi + static_cast<int64_t>(j) * ldx] = i > j ? lij : sgn[i] * L.S3[i][j];
      }
    }
    __syncthreads();
    // U^-1 (S2) and L^-1 (S4) side by side; S3 is free: scratch
    tri_join_both<T>(L.S2, [&](int a, int b) { return L.S1[a][b]; }, L.S4, [&](int a, int b) { return L.S1[a][b]; },
                     L.S3, g, c);
    phase();
    if (chol) frag_to_lds(fR2, L.S3, fp);
    __syncthreads();
    // T = (U S) L^-T and M = R2^-1 U^-1
    frag_zero(f);
    frag_mma_f(f, [&](int i, int k) { return k >= i ? L.S1[i][k] * sgn[k] : T(0); },
               [&](int k, int j) { return L.S4[j][k]; }, fp, 0, NB);
    Frag<T> fm;
    if (chol) {
      frag_zero(fm);
      frag_mma<T, false>(fm, L.S3, L.S2, fp);
    }
    __syncthreads();
    frag_to_lds(f, L.S4, fp);
    if (chol) frag_to_lds(fm, L.S2, fp);
    __syncthreads();
    for (int e = tid; e < NB * NB; e += PANEL_THREADS) {
      store_agent(xu + e, L.S2[e & (NB - 1)][e / NB]);
      store_agent(xu + NB * NB + e, L.S4[e & (NB - 1)][e / NB]);
    }
    raise_flag(rflag, tagU);
  } else {
    // M into S2, and T into S4 when every workgroup needs it
    const bool ok = await_flag(rflag, tagU + pw.skew, err, pw.spin_limit);
    const int nget = all_t ? 2 : 1;
    for (int hh = 0; hh < nget && ok; ++hh) {
      T (*dst)[NB + 2] = hh ? L.S4 : L.S2;
      T v[NB * NB / PANEL_THREADS];
#pragma unroll
      for (int u = 0; u < NB * NB / PANEL_THREADS; ++u) v[u] = load_coherent(xu + hh * NB * NB + tid + u * PANEL_THREADS);
#pragma unroll
      for (int u = 0; u < NB * NB / PANEL_THREADS; ++u) {
        const int e = tid + u * PANEL_THREADS;
        dst[e & (NB - 1)][e / NB] = v[u];
      }
    }
    if (__syncthreads_or(ok ? 0 : 1)) return false;
  }
  if (threadIdx.x < NB && (wg == 0 || all_t)) L.tau[threadIdx.x] = L.S4[threadIdx.x][threadIdx.x];

  // ---- Y2 = -Q1 M below the pivot rows, into the Y rows and X
  phase();
  const int k1 = wg == 0 ? kc + 1 : kc;  // workgroup 0's chunk kc holds the pivot rows
  if (k1 < CQR_CHUNKS) {
    ChunkRegs<T> cur;
    rw.load(cur, Yp, ldy, k1, false);
    for (int k = k1; k < CQR_CHUNKS; ++k) {
      rw.put(L.S1, cur);
      __syncthreads();
      if (k + 1 < CQR_CHUNKS) rw.load(cur, Yp, ldy, k + 1, false);
      frag_zero(f);
      frag_mma<T, false>(f, L.S1, L.S2, fp);
      frag_negate_plus_identity(f, fp, false);
      __syncthreads();
      frag_to_lds(f, L.S1, fp);
      __syncthreads();
      rw.out(L.S1, Yp, ldy, k);
      rw.out(L.S1, Xp, ldx, k);
      __syncthreads();
    }
  }
  return true;
}

// f <-> rows [r0, r0 + 64) of a column-major matrix (ld ld), in the fragment
// layout; entries at rows >= mrows or columns >= ncols read as 0 and are not
// written.  Each wave's 16 x 32 block covers whole 128-byte lines of 16 rows.
template <class T>
__device__ __forceinline__ void frag_load_global(Frag<T>& f, const T* src, int64_t ld, int64_t r0, int64_t mrows,
                                                 int ncols, const FragPos& p, bool coherent) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t gi = r0 + p.ib + PanelMma<T>::row(p.lk, v);
    const int j0 = p.cb0 + p.l16, j1 = j0 + 16;
    const T* q0 = src + gi + static_cast<int64_t>(j0) * ld;
    const T* q1 = src + gi + static_cast<int64_t>(j1) * ld;
    f.a0[v] = (gi < mrows && j0 < ncols) ? (coherent ? load_coherent(q0) : *q0) : T(0);
    f.a1[v] = (gi < mrows && j1 < ncols) ? (coherent ? load_coherent(q1) : *q1) : T(0);
  }
}
template <class T>
__device__ __forceinline__ void frag_store_global(const Frag<T>& f, T* dst, int64_t ld, int64_t r0, int64_t mrows,
                                                  int ncols, const FragPos& p) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t gi = r0 + p.ib + PanelMma<T>::row(p.lk, v);
    const int j0 = p.cb0 + p.l16, j1 = j0 + 16;
    if (gi < mrows && j0 < ncols) dst[gi + static_cast<int64_t>(j0) * ld] = f.a0[v];
    if (gi < mrows && j1 < ncols) dst[gi + static_cast<int64_t>(j1) * ld] = f.a1[v];
  }
}
// S = the 64 x 64 block of a column-major matrix at src (ld ld).
template <class T>
__device__ __forceinline__ void block_to_lds(T (*S)[NB + 2], const T* src, int64_t ld) {
  const int tid = opaque(static_cast<int>(threadIdx.x));
  T v[NB * NB / PANEL_THREADS];
#pragma unroll
  for (int u = 0; u < NB * NB / PANEL_THREADS; ++u) {
    const int e = tid + u * PANEL_THREADS;
    v[u] = src[(e & (NB - 1)) + static_cast<int64_t>(e / NB) * ld];
  }
#pragma unroll
  for (int u = 0; u < NB * NB / PANEL_THREADS; ++u) {
    const int e = tid + u * PANEL_THREADS;
    S[e & (NB - 1)][e / NB] = v[u];
  }
}

// The previous 128-column block's reflectors applied to this launch's columns
// (the look-ahead update of the blocked QR, Section 2.2), by every workgroup on
// its own rows: C <- (I - Yp Tp Yp^T)^T C = C - Yp (Tp^T (Yp^T C)), with
// W = Yp^T C (128 x 128) summed over the workgroups.  C is X's columns [0, nc1)
// and [NB, NB + nc2) over rows [0, mp) (kernel rows: row 0 is the previous
// block's first pivot row); Yp the previous block's explicit reflectors at the
// same rows (ld ldy, 128 columns), Tp its 128 x 128 T (ld ldt).  False if a
// wait expired.
template <class T>
__device__ __forceinline__ bool prev_update(T* __restrict__ X, int64_t ldx, int64_t mp, int nc1, int nc2,
                                            const T* __restrict__ Yp, int64_t ldy, const T* __restrict__ Tp, int ldt,
                                            int P, int wg, int g, int c, const TsqrXch& xt, uint32_t tag,
                                            unsigned* err, const PanelWait& pw, bool coherent, const TsqrLds<T>& L) {
  FragPos fp{(g >> 1) * 16, (g & 1) * 32, c & 15, c >> 4};
  const int64_t row0 = static_cast<int64_t>(wg) * CQR_RPW;
  CqrRows<T> yr;
  yr.row0 = row0;
  yr.mp = mp;
  yr.lbase = static_cast<int>(row0);
  yr.p0 = 0;
  yr.jbp = NB;
  yr.kc = 0;
  CqrRows<T> c1 = yr, c2 = yr;
  c1.jbp = nc1;
  c2.jbp = nc2;
  const T* Yh = Yp + static_cast<int64_t>(NB) * ldy;
  T* X2 = X + static_cast<int64_t>(NB) * ldx;
  // ---- W = Yp^T C over this workgroup's rows, four 64 x 64 blocks W_ab = Yp_a^T C_b
  {
    Frag<T> w00, w01, w10, w11;
    frag_zero(w00);
    frag_zero(w01);
    frag_zero(w10);
    frag_zero(w11);
    ChunkRegs<T> ya, yb, ca, cb;
    yr.load(ya, Yp, ldy, 0, false);
    yr.load(yb, Yh, ldy, 0, false);
    c1.load(ca, X, ldx, 0, coherent);
    c2.load(cb, X2, ldx, 0, coherent);
    for (int k = 0; k < CQR_CHUNKS; ++k) {
      yr.put(L.S1, ya);
      yr.put(L.S2, yb);
      yr.put(L.S3, ca);
      yr.put(L.S4, cb);
      __syncthreads();
      if (k + 1 < CQR_CHUNKS) {
        yr.load(ya, Yp, ldy, k + 1, false);
        yr.load(yb, Yh, ldy, k + 1, false);
        c1.load(ca, X, ldx, k + 1, coherent);
        c2.load(cb, X2, ldx, k + 1, coherent);
      }
      frag_mma<T, true>(w00, L.S1, L.S3, fp);
      frag_mma<T, true>(w01, L.S1, L.S4, fp);
      frag_mma<T, true>(w10, L.S2, L.S3, fp);
      frag_mma<T, true>(w11, L.S2, L.S4, fp);
      __syncthreads();
    }
    frag_to_lds(w00, L.S1, fp);
    frag_to_lds(w01, L.S2, fp);
    frag_to_lds(w10, L.S3, fp);
    frag_to_lds(w11, L.S4, fp);
    __syncthreads();
  }
  {
    T (*const blocks[4])[NB + 2] = {L.S1, L.S2, L.S3, L.S4};
    T* const part = reinterpret_cast<T*>(xt.upd);
    if (!allreduce_n<T, 4>(blocks, P, wg, part, part + static_cast<int64_t>(P) * 4 * NB * NB, xt.uflags,
                           xt.uflags + kMaxCqrWgs, tag, err, pw))
      return false;
  }
  // ---- W' = Tp^T W: W'_0b = T00^T W_0b, W'_1b = T01^T W_0b + T11^T W_1b (S1 = W00, S2 = W01,
  // S3 = W10, S4 = W11 on entry; the T blocks pass through S2 and S4)
  Frag<T> f00, f01, f10, f11, g01, g11;
  frag_from_lds(g01, L.S2, fp);
  frag_from_lds(g11, L.S4, fp);
  __syncthreads();
  const T* T00 = Tp;
  const T* T01 = Tp + static_cast<int64_t>(NB) * ldt;
  const T* T11 = Tp + NB + static_cast<int64_t>(NB) * ldt;
  block_to_lds(L.S2, T01, ldt);
  block_to_lds(L.S4, T11, ldt);
  __syncthreads();
  frag_zero(f10);
  frag_mma<T, true>(f10, L.S2, L.S1, fp);
  frag_mma<T, true>(f10, L.S4, L.S3, fp);
  __syncthreads();
  block_to_lds(L.S2, T00, ldt);
  __syncthreads();
  frag_zero(f00);
  frag_mma<T, true>(f00, L.S2, L.S1, fp);
  __syncthreads();
  frag_to_lds(g01, L.S1, fp);
  frag_to_lds(g11, L.S3, fp);
  block_to_lds(L.S2, T01, ldt);
  block_to_lds(L.S4, T11, ldt);
  __syncthreads();
  frag_zero(f11);
  frag_mma<T, true>(f11, L.S2, L.S1, fp);
  frag_mma<T, true>(f11, L.S4, L.S3, fp);
  __syncthreads();
  block_to_lds(L.S2, T00, ldt);
  __syncthreads();
  frag_zero(f01);
  frag_mma<T, true>(f01, L.S2, L.S1, fp);
  __syncthreads();
  // ---- C_b -= Yp_0 W'_0b + Yp_1 W'_1b, one half of C at a time (W' in S1, S2; Yp chunks in S3, S4)
  for (int b = 0; b < 2; ++b) {
    const int ncb = b ? nc2 : nc1;
    T* Cb = b ? X2 : X;
    frag_to_lds(b ? f01 : f00, L.S1, fp);
    frag_to_lds(b ? f11 : f10, L.S2, fp);
    ChunkRegs<T> ya, yb;
    yr.load(ya, Yp, ldy, 0, false);
    yr.load(yb, Yh, ldy, 0, false);
    for (int k = 0; k < CQR_CHUNKS; ++k) {
      yr.put(L.S3, ya);
      yr.put(L.S4, yb);
      __syncthreads();
      if (k + 1 < CQR_CHUNKS) {
        yr.load(ya, Yp, ldy, k + 1, false);
        yr.load(yb, Yh, ldy, k + 1, false);
      }
      Frag<T> fc, fy;
      frag_load_global(fc, Cb, ldx, row0 + 64 * k, mp, ncb, fp, coherent);
      frag_zero(fy);
      frag_mma<T, false>(fy, L.S3, L.S1, fp);
      frag_mma<T, false>(fy, L.S4, L.S2, fp);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        fc.a0[v] -= fy.a0[v];
        fc.a1[v] -= fy.a1[v];
      }
      frag_store_global(fc, Cb, ldx, row0 + 64 * k, mp, ncb, fp);
      __syncthreads();
    }
  }
  return true;
}

// The block of columns [0, jb + jb2) (jb2 > 0: a second part of jb2 columns,
// with the first part's reflectors applied to it in between and the joined T)
// of rows [ext, mp) at X: Householder vectors (explicit, into Y), T (into Tout,
// ld ldt, from the workgroup holding the pivot rows), tau; R in place in X.
// Rows are kernel rows: with ext = CQR_RPW, rows [0, ext) are the previous
// block's pivot rows, and the launch first applies that block's reflectors
// (Yprev, Tprev) to its columns over rows [0, mp); workgroup 0 holds those
// rows and leaves after that update.  P = ceil(mp / CQR_RPW) co-resident
// workgroups.  With wait_flag, the launch waits (bounded) for that flag before
// reading its columns, which another stream updates.
template <class T>
__global__ __launch_bounds__(PANEL_THREADS) void cqr_panel_kernel(T* __restrict__ X, int64_t ldx, int64_t mp, int jb,
                                                                 T* __restrict__ Y, int64_t ldy, T* __restrict__ tau,
                                                                 T* __restrict__ Tout, int ldt, uint32_t tag0,
                                                                 unsigned* __restrict__ err, int zero_above,
                                                                 PanelWait pw, int jb2,
                                                                 const unsigned* __restrict__ wait_flag, TsqrXch xt,
                                                                 const T* __restrict__ Yprev,
                                                                 const T* __restrict__ Tprev, int ext) {
  __shared__ __attribute__((aligned(16))) T S1[NB][NB + 2];
  __shared__ __attribute__((aligned(16))) T S2[NB][NB + 2];
  __shared__ __attribute__((aligned(16))) T S3[NB][NB + 2];
  __shared__ __attribute__((aligned(16))) T S4[NB][NB + 2];
  __shared__ __attribute__((aligned(16))) T cb[PANEL_WAVES][NB];
  __shared__ T red0[PANEL_WAVES][NB];
  __shared__ T red1[PANEL_WAVES][NB];
  __shared__ T piv[2][NB];
  __shared__ T aux[8 * NB];
  __shared__ T tau_sh[NB];
  const TsqrLds<T> L{S1, S2, S3, S4, cb, red0, red1, piv, tau_sh, aux};

  const int P = gridDim.x, wg = blockIdx.x;
  int c = threadIdx.x & 63;
  const int g = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t row0 = static_cast<int64_t>(wg) * CQR_RPW;
  const bool two = jb2 > 0;
  const int pwg = ext / CQR_RPW;  // the workgroup of the pivot rows
  FragPos fp{(g >> 1) * 16, (g & 1) * 32, c & 15, c >> 4};
  auto phase = [&]() {
    c = opaque(c);
    fp.l16 = c & 15;
    fp.lk = c >> 4;
  };

  bool ok = true;
  const bool waited = wait_flag != nullptr;
  if (waited) {
    if (threadIdx.x == 0) ok = wait_flag_geq(wait_flag, 1u, err, pw.spin_limit);
    ok = !__syncthreads_or(ok ? 0 : 1);
  }
  if (ext > 0 && ok) {
    ok = prev_update(X, ldx, mp, jb, jb2, Yprev, ldy, Tprev, ldt, P, wg, g, c, xt, tag0 + 7, err, pw, waited, L);
    phase();
  }
  if (wg < pwg) return;  // rows above the block: only the previous block's update
  for (int part = 0; part < (two ? 2 : 1); ++part) {
    phase();
    const int p0 = part * NB;
    const int jbp = part ? jb2 : jb;
    const uint32_t tagp = tag0 + static_cast<uint32_t>(part * NB);
    T* Xp = X + static_cast<int64_t>(p0) * ldx;
    T* Yp = Y + static_cast<int64_t>(p0) * ldy;
    T* Tp = Tout + p0 + static_cast<int64_t>(p0) * ldt;
    CqrRows<T> rw;
    rw.row0 = row0;
    rw.mp = mp;
    rw.lbase = wg == pwg ? ext + p0 : static_cast<int>(row0);
    rw.p0 = ext + p0;
    rw.jbp = jbp;
    rw.kc = (rw.lbase - static_cast<int>(row0)) / 64;
    // part 0 reads columns another kernel may have just written; part 1 reads this kernel's own
    ok = ok && cqr_part(rw, P - pwg, wg - pwg, g, c, Xp, ldx, Yp, ldy, waited && part == 0, xt, tagp, err, pw, two,
                        xt.chol != 0, L);
    if (!ok) {
      // A device-side wait gave up: poison T and tau so that the failure is visible.
      if (threadIdx.x < NB) tau_sh[threadIdx.x] = static_cast<T>(__builtin_nan(""));
      for (int e = threadIdx.x; e < NB * NB; e += PANEL_THREADS) S4[e & (NB - 1)][e / NB] = static_cast<T>(__builtin_nan(""));
    }
    __syncthreads();
    if (wg == pwg) {
      for (int e = threadIdx.x; e < NB * NB; e += PANEL_THREADS) {
        const int i = e % NB, k = e / NB;
        if (i < jbp && k < jbp) Tp[i + static_cast<int64_t>(k) * ldt] = S4[i][k];
      }
      if (threadIdx.x < jbp) tau[p0 + threadIdx.x] = tau_sh[threadIdx.x];
      // Y is zero in the zero_above rows above the block's first pivot row (an earlier
      // panel of the same block pair)
      T* Yf = Yp + ext;
      for (int e = threadIdx.x; e < zero_above * jbp; e += PANEL_THREADS)
        Yf[(e % zero_above) - zero_above + static_cast<int64_t>(e / zero_above) * ldy] = T(0);
      // and in the rows of the first part above the second
      if (part == 1)
        for (int e = threadIdx.x; e < NB * jbp; e += PANEL_THREADS)
          Yf[(e % NB) + static_cast<int64_t>(e / NB) * ldy] = T(0);
    }
    if (!two || !ok) break;
    phase();
    CqrRows<T> all = rw;  // every row of the block that this workgroup holds
    all.lbase = static_cast<int>(row0);
    all.jbp = NB;
    all.kc = 0;
    CqrRows<T> rw2 = all;
    rw2.jbp = jb2;
    T* X2 = X + static_cast<int64_t>(NB) * ldx;
    T* Y2 = Y + static_cast<int64_t>(NB) * ldy;
    if (part == 0) {
      // ---- the second part's columns C2 <- (I - Y1 T1^T Y1^T) C2: W = Y1^T C2 summed over the workgroups
      Frag<T> f;
      frag_zero(f);
      {
        ChunkRegs<T> ya, ca;
        all.load(ya, Y, ldy, 0, false);
        rw2.load(ca, X2, ldx, 0, waited);
        for (int k = 0; k < CQR_CHUNKS; ++k) {
          all.put(S1, ya);
          rw2.put(S2, ca);
          __syncthreads();
          if (k + 1 < CQR_CHUNKS) {
            all.load(ya, Y, ldy, k + 1, false);
            rw2.load(ca, X2, ldx, k + 1, waited);
          }
          frag_mma<T, true>(f, S1, S2, fp);
          __syncthreads();
        }
      }
      frag_to_lds(f, S3, fp);
      __syncthreads();
      ok = allreduce64(S3, P - pwg, wg - pwg, xt, tagp + 5, err, pw);
      if (!ok) break;
      phase();
      // W' = T1^T W (T1 in S4, every workgroup) into S2
      frag_zero(f);
      frag_mma<T, true>(f, S4, S3, fp);
      __syncthreads();
      frag_to_lds(f, S2, fp);
      __syncthreads();
      // C2 -= Y1 W', chunk by chunk, back into X
      {
        ChunkRegs<T> ya, ca;
        all.load(ya, Y, ldy, 0, false);
        rw2.load(ca, X2, ldx, 0, waited);
        for (int k = 0; k < CQR_CHUNKS; ++k) {
          all.put(S1, ya);
          rw2.put(S3, ca);
          __syncthreads();
          if (k + 1 < CQR_CHUNKS) {
            all.load(ya, Y, ldy, k + 1, false);
            rw2.load(ca, X2, ldx, k + 1, waited);
          }
          frag_from_lds(f, S3, fp);
          Frag<T> g1;
          frag_zero(g1);
          frag_mma<T, false>(g1, S1, S2, fp);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            f.a0[v] -= g1.a0[v];
            f.a1[v] -= g1.a1[v];
          }
          __syncthreads();
          frag_to_lds(f, S3, fp);
          __syncthreads();
          rw2.out(S3, X2, ldx, k);
          __syncthreads();
        }
      }
    } else {
      // ---- T of the whole block: T12 = -T1 (Y1^T Y2) T2, S12 = Y1^T Y2 summed over the
      // workgroups (Y2 is zero above its part: rows from the part's first pivot row on)
      Frag<T> f;
      frag_zero(f);
      {
        ChunkRegs<T> ya, yb;
        all.load(ya, Y, ldy, rw.kc, false);
        rw.load(yb, Y2, ldy, rw.kc, false);
        for (int k = rw.kc; k < CQR_CHUNKS; ++k) {
          all.put(S1, ya);
          rw.put(S2, yb);
          __syncthreads();
          if (k + 1 < CQR_CHUNKS) {
            all.load(ya, Y, ldy, k + 1, false);
            rw.load(yb, Y2, ldy, k + 1, false);
          }
          frag_mma<T, true>(f, S1, S2, fp);
          __syncthreads();
        }
      }
      frag_to_lds(f, S3, fp);
      __syncthreads();
      ok = allreduce64(S3, P - pwg, wg - pwg, xt, tagp + 6, err, pw);
      if (!ok) break;
      if (wg == pwg) {
        phase();
        // S12 T2 (T2 in S4) into S2, T1 (from Tout) into S1, T12 = -T1 (S12 T2)
        frag_zero(f);
        frag_mma<T, false>(f, S3, S4, fp);
        for (int e = threadIdx.x; e < NB * NB; e += PANEL_THREADS) {
          const int i = e & (NB - 1), k = e / NB;
          S1[i][k] = (i < jb && k < jb) ? Tout[i + static_cast<int64_t>(k) * ldt] : T(0);
        }
        __syncthreads();
        frag_to_lds(f, S2, fp);
        __syncthreads();
        frag_zero(f);
        frag_mma<T, false>(f, S1, S2, fp);
        frag_each(f, fp, [&](int i, int j, T v) {
          if (i < jb && j < jb2) Tout[i + static_cast<int64_t>(NB + j) * ldt] = -v;
        });
        for (int e = threadIdx.x; e < NB * NB; e += PANEL_THREADS) {
          const int i = e & (NB - 1), j = e / NB;
          if (i < jb2 && j < jb) Tout[NB + i + static_cast<int64_t>(j) * ldt] = T(0);
        }
      }
    }
  }
}

// R(i,c) = d_i X(i,c) for i <= c, 0 below; d_i = sign(X(i,i)), sign(0) = +1.
template <class T>
__global__ void extract_r_kernel(const T* __restrict__ X, int64_t ldx, int64_t n,
                                 T* __restrict__ R, int64_t ldr) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx % n, c = idx / n;
  T v = 0;
  if (i <= c) {
    const T d = (X[i + i * ldx] < T(0)) ? T(-1) : T(1);
    v = d * X[i + c * ldx];
  }
  R[i + c * ldr] = v;
}

// Q = [D; 0], D = diag(sign(X(c,c))).
template <class T>
__global__ void init_q_kernel(const T* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                              T* __restrict__ Q, int64_t ldq) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t i = idx % m, c = idx / m;
  T v = 0;
  if (i == c) v = (X[c + c * ldx] < T(0)) ? T(-1) : T(1);
  Q[i + c * ldq] = v;
}

__global__ void fill_u64_kernel(uint64_t* p, int64_t count) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx < count) p[idx] = 0;
}

// Sum of `splits` partial values spaced `slice` apart, in ascending order
// (four independent loads in flight, added in the same order as one loop).
template <class T>
__device__ inline T sum_splits(const T* __restrict__ src, int splits, int64_t slice) {
  T a = 0;
  int z = 0;
  for (; z + 4 <= splits; z += 4) {
    const T v0 = src[z * slice], v1 = src[(z + 1) * slice], v2 = src[(z + 2) * slice], v3 = src[(z + 3) * slice];
    a += v0;
    a += v1;
    a += v2;
    a += v3;
  }
  for (; z < splits; ++z) a += src[z * slice];
  return a;
}

// Joins the T factors of two consecutive panels into the T of their union:
// for H = (I - Y1 T1 Y1^T)(I - Y2 T2 Y2^T) = I - [Y1 Y2] T [Y1 Y2]^T,
// T = [[T1, -T1 (Y1^T Y2) T2], [0, T2]].  T1 and T2 are already in place in
// the (ld ldt) block at Tb; S12 = Y1^T Y2 (jb1 x jb2, ld lds).  One workgroup.
template <class T>
__global__ __launch_bounds__(1024) void t_join_kernel(T* __restrict__ Tb, int ldt, int jb1, int jb2,
                                                      const T* __restrict__ S12, int lds) {
  __shared__ T t1[NB][NB + 1];
  __shared__ T t2[NB][NB + 1];
  __shared__ T u[NB][NB + 1];
  constexpr int PER = NB * NB / 1024;
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
    const int i = e % NB, j = e / NB;
    t1[i][j] = (i < jb1 && j < jb1) ? Tb[i + static_cast<int64_t>(j) * ldt] : T(0);
    t2[i][j] = (i < jb2 && j < jb2) ? Tb[jb1 + i + static_cast<int64_t>(jb1 + j) * ldt] : T(0);
    u[i][j] = (i < jb1 && j < jb2) ? S12[i + static_cast<int64_t>(j) * lds] : T(0);
  }
  __syncthreads();
  // u <- S12 T2 (T2 upper triangular: only k <= j contributes)
  T acc[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int e = threadIdx.x + r * 1024, i = e % NB, j = e / NB;
    T a = 0;
    for (int k = 0; k <= j; ++k) a += u[i][k] * t2[k][j];
    acc[r] = a;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int e = threadIdx.x + r * 1024;
    u[e % NB][e / NB] = acc[r];
  }
  __syncthreads();
  // T12 = -T1 u (T1 upper triangular: only k >= i contributes); lower-left block is zero
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int e = threadIdx.x + r * 1024, i = e % NB, j = e / NB;
    T a = 0;
    for (int k = i; k < NB; ++k) a += t1[i][k] * u[k][j];
    if (i < jb1 && j < jb2) Tb[i + static_cast<int64_t>(jb1 + j) * ldt] = -a;
    if (i < jb2 && j < jb1) Tb[jb1 + i + static_cast<int64_t>(j) * ldt] = T(0);
  }
}

// W2 = T^T W1 with W1 = sum_z P[z] (jb x N each, packed, z ascending) and T
// upper triangular (ld ldt; entries below its diagonal are not read): the
// middle factor of (I - Y T^T Y^T) C, fused with the split-K reduction of
// W1 = Y^T C.  A workgroup takes RT_CW columns: their W1 into LDS (each entry
// summed over the splits in ascending order, a thread's entries of two splits
// loaded together), then T^T W1 on the matrix cores, T staged through LDS
// RT_KC rows at a time; row blocks of T^T past a chunk's diagonal skip it.
// jb <= RJB (128, or 256 for the widest outer block).
constexpr int RT_CW = 32, RT_KC = 32;
template <class T, int RJB>
__global__ __launch_bounds__(256) void reduce_tmul_kernel(int jb, int64_t N, int splits, const T* __restrict__ P,
                                                          const T* __restrict__ Tm, int ldt, T* __restrict__ W2,
                                                          int64_t ldw2) {
  __shared__ T w1[RJB][RT_CW + 1];  // W1(k, j)
  __shared__ T ts[RT_KC][RJB + 1];  // T(k0 + r, i)
  const int tid = threadIdx.x, c = tid & 63, g = tid >> 6;
  const int64_t c0 = static_cast<int64_t>(blockIdx.x) * RT_CW;
  const int cols = static_cast<int>(min<int64_t>(RT_CW, N - c0));
  const int jb16 = (jb + 15) & ~15;
  const int64_t slice = static_cast<int64_t>(jb) * N;
  constexpr int EPT = RJB * RT_CW / 256;  // entries of W1 per thread
  int64_t off[EPT];
  bool live[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = tid + 256 * u, k = e % jb16, jj = e / jb16;
    live[u] = e < jb16 * RT_CW && k < jb && jj < cols;
    off[u] = (c0 + jj) * jb + k;
  }
  T sum[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) sum[u] = T(0);
  int z = 0;
  for (; z + 2 <= splits; z += 2) {
    T v0[EPT], v1[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      v0[u] = live[u] ? P[z * slice + off[u]] : T(0);
      v1[u] = live[u] ? P[(z + 1) * slice + off[u]] : T(0);
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      sum[u] += v0[u];
      sum[u] += v1[u];
    }
  }
  if (z < splits) {
#pragma unroll
    for (int u = 0; u < EPT; ++u) sum[u] += live[u] ? P[z * slice + off[u]] : T(0);
  }
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = tid + 256 * u;
    if (e < jb16 * RT_CW) w1[e % jb16][e / jb16] = live[u] ? sum[u] : T(0);
  }
  // tiles of the jb16 x RT_CW result: t = 2 (row block) + (column block), wave g takes t = g + 4q
  constexpr int QMAX = 2 * RJB / 16 / 4;
  const int ntiles = 2 * (jb16 / 16);
  TileAcc<T> acc[QMAX];
#pragma unroll
  for (int q = 0; q < QMAX; ++q) tile_zero<T>(acc[q]);
  for (int kc = 0; kc < jb16; kc += RT_KC) {
    const int nk = min(RT_KC, jb16 - kc);
    __syncthreads();  // w1 written (first chunk), or the previous chunk's products done
    for (int e = tid; e < RT_KC * jb16; e += 256) {
      const int r = e % RT_KC, i = e / RT_KC, k = kc + r;
      ts[r][i] = (r < nk && k < jb && i < jb && k <= i) ? Tm[k + static_cast<int64_t>(i) * ldt] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int t = g + 4 * q;
      const int i0 = (t >> 1) * 16, j0 = (t & 1) * 16;
      if (t < ntiles && kc <= i0 + 15)
        tile_mm<T>(acc[q], [&](int i, int k) { return ts[k - kc][i]; }, [&](int k, int j) { return w1[k][j]; }, i0,
                   j0, kc, nk, c);
    }
  }
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    const int t = g + 4 * q;
    if (t < ntiles)
      tile_each<T>(acc[q], (t >> 1) * 16, (t & 1) * 16, c, [&](int i, int j, T v) {
        if (i < jb && j < cols) W2[i + (c0 + j) * ldw2] = v;
      });
  }
}

template <class T>
void launch_reduce_tmul(int jb, int64_t N, int splits, const T* P, const T* Tm, int ldt, T* W2, int64_t ldw2,
                        hipStream_t s) {
  const unsigned grid = static_cast<unsigned>(ceil_div(N, RT_CW));
  if (jb <= 128)
    reduce_tmul_kernel<T, 128><<<grid, 256, 0, s>>>(jb, N, splits, P, Tm, ldt, W2, ldw2);
  else
    reduce_tmul_kernel<T, 256><<<grid, 256, 0, s>>>(jb, N, splits, P, Tm, ldt, W2, ldw2);
}

// dst (rows x cols, ld ldd) = src (ld lds).
template <class T>
__global__ void copy_block_kernel(const T* __restrict__ src, int64_t lds, T* __restrict__ dst, int64_t ldd,
                                  int64_t rows, int64_t cols) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= rows * cols) return;
  dst[idx % rows + (idx / rows) * ldd] = src[idx % rows + (idx / rows) * lds];
}

__global__ void fill_u32_kernel(unsigned* p, int64_t count, unsigned v) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx < count) p[idx] = v;
}

int64_t panel_wgs(int64_t mp) { return ceil_div(mp, RPW); }

// Sub-block: two consecutive panels joined (NB2 columns).  Outer block: two
// sub-blocks joined (NBO columns); the trailing matrix and the targets are
// updated once per outer block, so their GEMMs have k = NBO.
constexpr int NB2 = 2 * NB;
constexpr int NBO = 4 * NB;  // widest outer block; T is stored with this leading dimension

// Whether the second panel of a sub-block forms S12 and the joined T itself
// (URV_PANEL_JOIN=0 uses a GEMM and t_join_kernel instead, for tuning).
bool panel_join() {
  const char* e = std::getenv("URV_PANEL_JOIN");
  return !(e && std::atoi(e) == 0);
}

// Whether the two panels of a 128-column sub-block are factored by one launch
// (URV_PANEL_FUSED=0 launches them separately with an update in between, for tuning).
bool panel_fused() {
  const char* e = std::getenv("URV_PANEL_FUSED");
  return !(e && std::atoi(e) == 0);
}

// Whether a block's factorisation is queued ahead of the update of its columns
// and waits for it on the device (URV_PANEL_EARLY=0 orders them through the
// streams, for tuning).  `fallback` when the variable is unset.
bool panel_early(bool fallback) {
  const char* e = std::getenv("URV_PANEL_EARLY");
  return e ? std::atoi(e) != 0 : fallback;
}

// Whether a block's panel launch applies the previous block's reflectors to its
// columns first (URV_PANEL_PREV=0 leaves that to an update on the caller's stream).
bool panel_prev() {
  const char* e = std::getenv("URV_PANEL_PREV");
  return !(e && std::atoi(e) == 0);
}

// Whether panels are factored by the tall-skinny QR with reconstructed
// reflectors (URV_PANEL_TSQR=0 selects the loop with one device-wide reduction
// per column, for comparison).
bool panel_tsqr() {
  const char* e = std::getenv("URV_PANEL_TSQR");
  return !(e && std::atoi(e) == 0);
}

// Whether the panels try CholeskyQR2 before the tall-skinny QR
// (URV_PANEL_CHOL=0 goes straight to the tall-skinny QR, for comparison).
bool panel_chol() {
  const char* e = std::getenv("URV_PANEL_CHOL");
  return !(e && std::atoi(e) == 0);
}

// Whether the trailing updates apply pairs of 128-column blocks at once (k = 256) once
// the pair's second block is factored (URV_BULK_PAIRS=1, for tuning).  Off: the pair's
// update of the rest starts a block later and the chain waits for it (measured on
// MI355X at n = 8000, q = 2: FULL 288 ms with pairs against 271, HALF 222 against 213).
bool bulk_pairs() {
  const char* e = std::getenv("URV_BULK_PAIRS");
  return e && std::atoi(e) == 1;
}

// Column blocks updated on the caller's stream ahead of the bulk update (URV_LOOKAHEAD
// 1 to 3, for tuning).  Measured on MI355X at n = 8000, q = 2 (FULL / HALF): one block
// 266.1 / 210.6 ms, two 264.0 / 209.5 (later, with V formed beside the final QR:
// 253.1 / 199.0), three 263.1-263.7 / 204.5 - the near updates on the caller's stream
// then hold the chain back more than the bulk updates did.
int lookahead() {
  const char* e = std::getenv("URV_LOOKAHEAD");
  return e ? std::min(3, std::max(1, std::atoi(e))) : 2;
}

// Whether targets take pairs of 128-column blocks (URV_TARGET_PAIRS=0 turns it off, for tuning).
bool target_pairs() {
  const char* e = std::getenv("URV_TARGET_PAIRS");
  return !(e && std::atoi(e) == 0);
}

// How many blocks the targets trail the factorisation by (URV_TARGET_LAG
// overrides it, for tuning).  The targets only have to be done when the QR
// returns, while the trailing updates of the first blocks gate the chain: held
// back, the target products leave the CUs to those updates while the trailing
// matrix is large and run beside the later, lighter blocks.  Measured on
// MI355X at n = 8000, q = 2 (FP64 FULL / HALF, V formed beside the final QR):
// lag 6: 261.0 / 204.0 ms, 12: 257.0 / 201.9, 18: 253.4-254.5 / 198.5-200.5,
// 21: 254.2, 24: 256.1 / 200.1, 30: 262.6 / 203.8.  Targets with more rows than the QR
// has columns hold proportionally more work per block, and a tall QR's trailing matrix
// stays tall to its last block, leaving little idle time to fill there: the lag shrinks
// by n / target_rows and by n / m.  Measured on MI355X (alternating runs), FP64 FULL
// q = 2 of a 4000 x 8000 A (its transpose factored): 120.1-120.2 ms against 124.7-125.1
// with the first factor alone, which gave 124.8-125.3 against 128.7-128.8 with 18 on
// another box; 8000 x 8000 unchanged, 16000 x 8000 within the noise (URV_TARGET_LAG=-1
// keeps 18).
int target_lag(int64_t m, int64_t n, int64_t target_rows) {
  const char* e = std::getenv("URV_TARGET_LAG");
  const int v = e ? std::atoi(e) : -2;
  if (v >= 0) return v;
  if (v == -1) return 18;
  double lag = 18.0;
  if (target_rows > n) lag *= static_cast<double>(n) / target_rows;
  if (m > n) lag *= static_cast<double>(n) / m;
  return std::max(4, static_cast<int>(lag + 0.5));
}

// Outer block width used by qr_pos: NB2 or NBO (URV_QR_BLOCK, for tuning).
int outer_block() {
  const char* e = std::getenv("URV_QR_BLOCK");
  return (e && std::atoi(e) == NBO) ? NBO : NB2;
}

// URV_PANEL_EXPIRE_TEST=1 makes every panel wait expire (tests of the failure path).
PanelWait panel_wait() {
  PanelWait pw;
  const char* e = std::getenv("URV_PANEL_EXPIRE_TEST");
  if (e && std::atoi(e) == 1) {
    pw.spin_limit = 256;
    pw.skew = 1;
  }
  return pw;
}

struct QrSizes {
  size_t y, t, tau, w, xch, sync, gemm_work, wb, gemm_work_b, wf, gemm_work_f, wn, gemm_work_n, tp, tq, jxch, txch;
};

// Words of the exchange of the streaming panel: the units' R, U^-1 and T, the 64 x 64 sums, the flags.
int cqr_wgs(int64_t m) { return static_cast<int>(ceil_div(m, CQR_RPW)); }
size_t tsqr_tri_words(int64_t m) { return static_cast<size_t>(2) * cqr_wgs(m) * kTriEntries; }
size_t tsqr_recon_words() { return static_cast<size_t>(2) * NB * NB; }
size_t tsqr_gram_words(int64_t m) { return (static_cast<size_t>(cqr_wgs(m)) + 1) * NB * NB; }
// the previous block's update: rows from one block above the panel
size_t tsqr_upd_words(int64_t m) { return (static_cast<size_t>(cqr_wgs(m + NB2)) + 1) * 4 * NB * NB; }

QrSizes qr_sizes(int64_t m, int64_t n, int64_t target_rows) {
  QrSizes z;
  const int64_t nblocks = ceil_div(n, NB);
  z.y = static_cast<size_t>(m) * n;
  z.t = static_cast<size_t>(NBO) * n;
  z.tau = n;
  z.w = static_cast<size_t>(NBO) * n;
  z.xch = 2 * (static_cast<size_t>(panel_wgs(m)) + 1) * NB * 2;
  z.jxch = (static_cast<size_t>(panel_wgs(m)) + 1) * kJoinEntries * 2;
  z.txch = tsqr_tri_words(m + NB2) + tsqr_recon_words() + tsqr_gram_words(m + NB2) + kTsqrFlags + tsqr_upd_words(m) +
           2 * kMaxCqrWgs;
  z.sync = nblocks + 2;
  size_t gw = 0, gwb = 0, gwf = 0, gwn = 0;
  for (const int64_t nbo : {static_cast<int64_t>(NB2), static_cast<int64_t>(NBO)}) {
    for (int64_t j0 = 0; j0 < n; j0 += nbo) {
      const int64_t jb = std::min<int64_t>(nbo, n - j0), mp = m - j0;
      const int64_t ja = std::min<int64_t>(NB2, jb), jbb = jb - ja;
      const int64_t nc = n - j0 - jb, nn = std::min<int64_t>(nbo, nc);
      // the block factorisation (side stream): panel pairs, A applied to B, S_AB, the next block
      for (int64_t r0 = j0; r0 < j0 + jb; r0 += NB2) {
        const int64_t js = std::min<int64_t>(NB2, j0 + jb - r0);
        const int64_t jb1 = std::min<int64_t>(NB, js), jb2 = js - jb1;
        gwb = std::max(gwb, gemm_partials_elems(jb1, jb2, m - r0));
      }
      gwb = std::max(gwb, gemm_partials_elems(ja, jbb, mp));
      gwb = std::max(gwb, gemm_work_elems(ja, jbb, mp));
      gwb = std::max(gwb, gemm_partials_elems(jb, nn, mp));
      const int64_t nn2 = std::min<int64_t>(nbo, std::max<int64_t>(nc - nn, 0));
      gwn = std::max(gwn, gemm_partials_elems(jb, nn, mp));
      gwn = std::max(gwn, gemm_partials_elems(jb, nn2, mp));
      gw = std::max(gw, gemm_partials_elems(jb, std::max<int64_t>(nc - nn - nn2, 0), mp));
      // two look-ahead blocks: the third column block on the caller's stream, the rest after it
      const int64_t nn3 = std::min<int64_t>(nbo, std::max<int64_t>(nc - nn - nn2, 0));
      gwn = std::max(gwn, gemm_partials_elems(jb, nn3, mp));
      gw = std::max(gw, gemm_partials_elems(jb, std::max<int64_t>(nc - nn - nn2 - nn3, 0), mp));
      gw = std::max(gw, gemm_work_elems(jb, nc - nn, mp));
      gw = std::max(gw, gemm_work_elems(jb, n - j0, mp));
      if (nbo == NB2 && j0 >= NB2) {
        // block j0 closes the pair that starts one block earlier: its joined T (S of the
        // pair), the pair on block j0 + 2 (caller's stream) and on the rest (fourth stream)
        const int64_t mpp = m - (j0 - NB2);
        gwn = std::max(gwn, gemm_work_elems(NB2, NB2, mpp));
        gwn = std::max(gwn, gemm_partials_elems(2 * NB2, nn2, mpp));
        gw = std::max(gw, gemm_partials_elems(2 * NB2, std::max<int64_t>(nc - nn - nn2, 0), mpp));
      }
      if (target_rows > 0) {
        gwf = std::max(gwf, gemm_work_elems(target_rows, jb, mp));
        gwf = std::max(gwf, gemm_work_elems(NB2, NB2, mp));  // S of a block pair
      }
    }
  }
  z.gemm_work = gw;
  z.wb = static_cast<size_t>(NBO) * NBO;
  z.gemm_work_b = gwb;
  z.wf = static_cast<size_t>(std::max<int64_t>(target_rows, 0)) * NBO;
  z.gemm_work_f = gwf;
  z.tp = target_rows > 0 ? static_cast<size_t>(NBO) * n : 0;
  z.wn = static_cast<size_t>(NBO) * NBO;
  z.tq = static_cast<size_t>(NBO) * NBO;
  z.gemm_work_n = gwn;
  return z;
}

}  // namespace

template <class T>
size_t qr_work_bytes(int64_t m, int64_t n, int64_t target_rows) {
  Arena a;
  QrWorkT<T> w;
  qr_work_carve(a, m, n, w, target_rows);
  return a.used;
}

template <class T>
void qr_work_carve(Arena& a, int64_t m, int64_t n, QrWorkT<T>& w, int64_t target_rows) {
  const QrSizes z = qr_sizes(m, n, target_rows);
  w.Y = a.take<T>(z.y);
  w.Tm = a.take<T>(z.t);
  w.tau = a.take<T>(z.tau);
  w.W1 = a.take<T>(z.w);
  w.W2 = a.take<T>(z.w);
  w.xch = a.take<uint64_t>(z.xch);
  w.xch_words = z.xch;
  w.jxch = a.take<uint64_t>(z.jxch);
  w.jxch_words = z.jxch;
  w.txch = a.take<uint64_t>(z.txch);
  w.txch_words = z.txch;
  w.sync = a.take<unsigned>(z.sync);
  w.gemm_work = a.take<T>(z.gemm_work);
  w.gemm_work_elems = z.gemm_work;
  w.W1b = a.take<T>(z.wb);
  w.W2b = a.take<T>(z.wb);
  w.gemm_work_b = a.take<T>(z.gemm_work_b);
  w.gemm_work_b_elems = z.gemm_work_b;
  w.target_rows = std::max<int64_t>(target_rows, 0);
  w.W1f = a.take<T>(z.wf);
  w.W2f = a.take<T>(z.wf);
  w.gemm_work_f = a.take<T>(z.gemm_work_f);
  w.gemm_work_f_elems = z.gemm_work_f;
  w.Tp = a.take<T>(z.tp);
  w.W1n = a.take<T>(z.wn);
  w.W2n = a.take<T>(z.wn);
  w.Tq = a.take<T>(z.tq);
  w.gemm_work_n = a.take<T>(z.gemm_work_n);
  w.gemm_work_n_elems = z.gemm_work_n;
}

template <class T>
int qr_pos(T* X, int64_t m, int64_t n, int64_t ldx, T* Q, int64_t ldq, T* R, int64_t ldr,
           const QrWorkT<T>& w, hipStream_t s, const QrTarget<T>* targets, int ntargets) {
  if (n == 0) return URV_OK;
  for (int i = 0; i < ntargets; ++i) {
    if (targets[i].rows > w.target_rows || targets[i].ldz < targets[i].rows) {
      set_last_error("qr_pos: target larger than the workspace covers");
      return URV_EINVAL;
    }
  }
  const int64_t nblocks = ceil_div(n, NB);
  if (panel_wgs(m) > kMaxPanelWgs) {
    set_last_error("qr_pos: too many rows for the panel kernel");
    return URV_ENOTSUP;
  }
  SideStream side;
  URV_TRY(side_stream(&side));
  std::lock_guard<std::mutex> side_lock(*side.mu);

  // the error flag is cleared by the caller of a whole computation, not here, so
  // that an expired wait in one QR is still reported after the QRs that follow
  unsigned* err = w.sync + nblocks;
  fill_u64_kernel<<<static_cast<unsigned>(ceil_div(static_cast<int64_t>(w.xch_words), 256)), 256, 0, s>>>(
      w.xch, static_cast<int64_t>(w.xch_words));
  URV_LAUNCHED("fill_u64_kernel");
  fill_u64_kernel<<<static_cast<unsigned>(ceil_div(static_cast<int64_t>(w.jxch_words), 256)), 256, 0, s>>>(
      w.jxch, static_cast<int64_t>(w.jxch_words));
  URV_LAUNCHED("fill_u64_kernel");
  const bool tsqr = panel_tsqr();
  if (tsqr) {
    fill_u64_kernel<<<static_cast<unsigned>(ceil_div(static_cast<int64_t>(w.txch_words), 256)), 256, 0, s>>>(
        w.txch, static_cast<int64_t>(w.txch_words));
    URV_LAUNCHED("fill_u64_kernel");
  }
  TsqrXch txch;
  txch.tri = w.txch;
  txch.recon = txch.tri + tsqr_tri_words(m + NB2);
  txch.gram = txch.recon + tsqr_recon_words();
  txch.chol = panel_chol() ? 1 : 0;
  txch.flags = txch.gram + tsqr_gram_words(m + NB2);
  txch.upd = txch.flags + kTsqrFlags;
  txch.uflags = txch.upd + tsqr_upd_words(m);
  // per-block flags: "the columns of the block at column b * NB are up to date"
  unsigned* ready = w.sync;
  fill_u32_kernel<<<static_cast<unsigned>(ceil_div(nblocks, 256)), 256, 0, s>>>(ready, nblocks, 0u);
  URV_LAUNCHED("fill_u32_kernel");

  // Look-ahead: 128-column blocks are factored on a second stream while the
  // other streams apply the previous blocks to the rest of the matrix.
  // The panels occupy a few dozen CUs; the trailing update fills the others.
  const hipStream_t s2 = side.stream;
  const int nbo = outer_block();
  const PanelWait pwait = panel_wait();
  const bool fused = panel_fused();

  uint32_t panels = 0;  // panel launches so far: exchange tags stay distinct
  // prev_j0 >= 0: the launch first applies the 128-column block at prev_j0
  // (= r0 - NB2) to its columns (the streaming panel only).
  auto panel = [&](int64_t r0, int jbp, T* Tp, int zero_above, const PanelJoin<T>& join, int jb2,
                   const unsigned* wf, int64_t prev_j0 = -1) -> int {
    const int64_t mp = m - r0;
    const unsigned P = static_cast<unsigned>(panel_wgs(mp));
    if (tsqr && join.Y1 == nullptr) {
      const int ext = prev_j0 >= 0 ? static_cast<int>(r0 - prev_j0) : 0;
      const int64_t k0 = r0 - ext;  // the launch's kernel row 0
      const T* Yprev = prev_j0 >= 0 ? w.Y + prev_j0 + prev_j0 * m : nullptr;
      const T* Tprev = prev_j0 >= 0 ? w.Tm + prev_j0 * NBO : nullptr;
      const int tok = sizeof(T) == 8 ? timing_begin(s2) : -1;
      cqr_panel_kernel<T><<<static_cast<unsigned>(cqr_wgs(mp + ext)), PANEL_THREADS, 0, s2>>>(
          X + k0 + r0 * ldx, ldx, mp + ext, jbp, w.Y + k0 + r0 * m, m, w.tau + r0, Tp, NBO, panels * NB, err,
          zero_above, pwait, jb2, wf, txch, Yprev, Tprev, ext);
      URV_LAUNCHED("cqr_panel_kernel");
      // algorithmic flops: Householder QR of the mp x jt panel, and the previous block's
      // W = Yp^T C and C -= Yp W' over its mp + ext rows
      const double jt = jbp + jb2, mr = static_cast<double>(mp);
      timing_end(tok, kTimedPanel,
                 2.0 * mr * jt * jt - 2.0 / 3.0 * jt * jt * jt + (ext ? 4.0 * (mr + ext) * NB2 * jt : 0.0), s2);
    } else {
      panel_kernel<T><<<P, PANEL_THREADS, 0, s2>>>(X + r0 + r0 * ldx, ldx, mp, jbp, w.Y + r0 + r0 * m, m,
                                                   w.tau + r0, Tp, NBO, w.xch, panels * NB, err, zero_above, join,
                                                   pwait, jb2, wf);
      URV_LAUNCHED("panel_kernel");
    }
    panels += jb2 > 0 ? 2 : 1;
    return URV_OK;
  };
  // Householder vectors, tau and T (at Tp, ld NBO) of the sub-block of width
  // jbs at row/column r0 of the outer block starting at j0, on the side stream;
  // with wf, its first launch waits for that flag before reading its columns.
  auto factor_sub = [&](int64_t j0, int64_t r0, int jbs, T* Tp, const unsigned* wf, int64_t prev_j0 = -1) -> int {
    const int jb1 = std::min(jbs, NB), jb2 = jbs - jb1;
    const int64_t mp = m - r0;
    T* Yb = w.Y + r0 + r0 * m;
    if (jb2 > 0 && fused) {
      // both panels in one launch; its exchange of W = Y1^T C2 and S12 uses the join buffers
      PanelJoin<T> bufs;
      bufs.ps = w.jxch;
      bufs.sums = w.jxch + w.jxch_words - 2 * kJoinEntries;
      return panel(r0, jb1, Tp, static_cast<int>(r0 - j0), bufs, jb2, wf, prev_j0);
    }
    URV_TRY(panel(r0, jb1, Tp, static_cast<int>(r0 - j0), PanelJoin<T>{}, 0, wf, jb2 > 0 ? -1 : prev_j0));
    if (jb2 > 0) {
      // first panel's reflectors applied to the second panel's columns:
      // C2 -= Y1 (T1^T (Y1^T C2)), the reduction of Y1^T C2 fused with T1^T
      T* C2 = X + r0 + (r0 + jb1) * ldx;
      int splits = 0;
      URV_TRY(gemm_partials<T>(true, false, jb1, jb2, mp, Yb, m, C2, ldx, w.gemm_work_b, w.gemm_work_b_elems,
                               &splits, s2));
      launch_reduce_tmul<T>(jb1, jb2, splits, w.gemm_work_b, Tp, NBO, w.W2b, NBO, s2);
      URV_LAUNCHED("reduce_tmul_kernel");
      URV_TRY(gemm<T>(false, false, mp, jb2, jb1, T(-1), Yb, m, w.W2b, NBO, T(1), C2, ldx, nullptr, 0, s2));
      // the second panel (Y2 zero above it), then the joined T from S12 = Y1^T Y2:
      // formed by the panel itself, or by a GEMM and t_join_kernel
      T* T2p = Tp + jb1 + static_cast<int64_t>(jb1) * NBO;
      if (panel_join()) {
        PanelJoin<T> join;
        join.Y1 = Yb + jb1;  // rows from the second panel's first row, columns of the first
        join.ldy1 = m;
        join.T1 = Tp;
        join.jb1 = jb1;
        join.ps = w.jxch;
        join.sums = w.jxch + w.jxch_words - 2 * kJoinEntries;
        URV_TRY(panel(r0 + jb1, jb2, T2p, static_cast<int>(r0 + jb1 - j0), join, 0, nullptr));
      } else {
        URV_TRY(panel(r0 + jb1, jb2, T2p, static_cast<int>(r0 + jb1 - j0), PanelJoin<T>{}, 0, nullptr));
        URV_TRY(gemm<T>(true, false, jb1, jb2, mp, T(1), Yb, m, Yb + static_cast<int64_t>(jb1) * m, m, T(0),
                        w.W1b, NBO, w.gemm_work_b, w.gemm_work_b_elems, s2));
        t_join_kernel<T><<<1, 1024, 0, s2>>>(Tp, NBO, jb1, jb2, w.W1b, NBO);
        URV_LAUNCHED("t_join_kernel");
      }
    }
    return URV_OK;
  };
  // The outer block at column j0: sub-blocks A and B, B updated by A in
  // between, and T = [[T_A, -T_A (Y_A^T Y_B) T_B], [0, T_B]].
  auto factor_block = [&](int64_t j0, const unsigned* wf, int64_t prev_j0 = -1) -> int {
    const int jbo = static_cast<int>(std::min<int64_t>(nbo, n - j0));
    const int ja = std::min(jbo, NB2), jbb = jbo - ja;
    const int64_t mp = m - j0;
    T* Tb = w.Tm + j0 * NBO;
    // Y is kept zero above the diagonal back to the start of the pair of
    // 128-column blocks, so that the targets can take a pair at once
    const int64_t jz = j0 - (j0 / NB2 % 2) * NB2;
    URV_TRY(factor_sub(jz, j0, ja, Tb, wf, prev_j0));
    if (jbb > 0) {
      const T* Ya = w.Y + j0 + j0 * m;
      T* CB = X + j0 + (j0 + ja) * ldx;
      int splits = 0;
      URV_TRY(gemm_partials<T>(true, false, ja, jbb, mp, Ya, m, CB, ldx, w.gemm_work_b, w.gemm_work_b_elems,
                               &splits, s2));
      launch_reduce_tmul<T>(ja, jbb, splits, w.gemm_work_b, Tb, NBO, w.W2b, NBO, s2);
      URV_LAUNCHED("reduce_tmul_kernel");
      URV_TRY(gemm<T>(false, false, mp, jbb, ja, T(-1), Ya, m, w.W2b, NBO, T(1), CB, ldx, nullptr, 0, s2));
      T* TB = Tb + ja + static_cast<int64_t>(ja) * NBO;
      URV_TRY(factor_sub(jz, j0 + ja, jbb, TB, nullptr));
      // Y_B is zero in the rows of A, so S_AB = Y_A^T Y_B over all mp rows
      URV_TRY(gemm<T>(true, false, ja, jbb, mp, T(1), Ya, m, Ya + static_cast<int64_t>(ja) * m, m, T(0),
                      w.W1b, NBO, w.gemm_work_b, w.gemm_work_b_elems, s2));
      URV_TRY(gemm<T>(false, false, ja, jbb, jbb, T(1), w.W1b, NBO, TB, NBO, T(0), w.W2b, NBO, nullptr, 0, s2));
      URV_TRY(gemm<T>(false, false, ja, jbb, ja, T(-1), Tb, NBO, w.W2b, NBO, T(0), Tb + static_cast<int64_t>(ja) * NBO,
                      NBO, nullptr, 0, s2));
      URV_TRY(gemm<T>(false, false, jbb, ja, 0, T(0), Tb, NBO, Tb, NBO, T(0), Tb + ja, NBO, nullptr, 0, s2));
    }
    return URV_OK;
  };
  // C <- (I - Y T^T Y^T) C for the block at j0 and columns [c0, c0 + nc): the next two
  // column blocks on the caller's stream, the bulk on the fourth stream (own scratch each).
  const hipStream_t s4 = side.stream4;
  enum { kOnPanelStream, kOnCallerStream, kOnBulkStream };
  // With jbo > 0 the reflectors are the jbo columns from j0 with T at Tbo (ld NBO): a block pair.
  auto apply_block = [&](int64_t j0, int64_t c0, int64_t nc, int where, int jbo = 0, const T* Tbo = nullptr) -> int {
    if (nc <= 0) return URV_OK;
    const int jb = jbo > 0 ? jbo : static_cast<int>(std::min<int64_t>(nbo, n - j0));
    const int64_t mp = m - j0;
    const T* Yb = w.Y + j0 + j0 * m;
    const T* Tb = Tbo ? Tbo : w.Tm + j0 * NBO;
    T* Cb = X + j0 + c0 * ldx;
    const bool bulk = where == kOnBulkStream, panel_side = where == kOnPanelStream;
    const hipStream_t st = bulk ? s4 : (panel_side ? s2 : s);
    T* W1 = bulk ? w.W1 : (panel_side ? w.W1b : w.W1n);
    T* W2 = bulk ? w.W2 : (panel_side ? w.W2b : w.W2n);
    T* gw = bulk ? w.gemm_work : (panel_side ? w.gemm_work_b : w.gemm_work_n);
    const size_t gwe = bulk ? w.gemm_work_elems : (panel_side ? w.gemm_work_b_elems : w.gemm_work_n_elems);
    (void)W1;
    int splits = 0;
    URV_TRY(gemm_partials<T>(true, false, jb, nc, mp, Yb, m, Cb, ldx, gw, gwe, &splits, st));   // Y^T C
    launch_reduce_tmul<T>(jb, nc, splits, gw, Tb, NBO, W2, NBO, st);  // T^T (Y^T C)
    URV_LAUNCHED("reduce_tmul_kernel");
    URV_TRY(gemm<T>(false, false, mp, nc, jb, T(-1), Yb, m, W2, NBO, T(1), Cb, ldx, nullptr, 0, st));
    return URV_OK;
  };

  // Joined T of the 128-column blocks A at j0 and B at j0 + NB2 (B may be narrower):
  // P = [[T_A, -T_A (Y_A^T Y_B) T_B], [0, T_B]] (ld NBO), on stream st with its own scratch.
  // Y_B is zero in the rows of A, so S = Y_A^T Y_B runs over all rows from j0.
  auto pair_t = [&](int64_t j0, T* P, T* W1, T* W2, T* gw, size_t gwe, hipStream_t st) -> int {
    const int64_t jblk = j0 + NB2;
    const int jbb = static_cast<int>(std::min<int64_t>(NB2, n - jblk));
    const int64_t mp = m - j0;
    const T* TA = w.Tm + j0 * NBO;
    const T* TB = w.Tm + jblk * NBO;
    const T* Ya = w.Y + j0 + j0 * m;
    copy_block_kernel<T><<<static_cast<unsigned>(ceil_div(NB2 * NB2, 256)), 256, 0, st>>>(TA, NBO, P, NBO, NB2, NB2);
    URV_LAUNCHED("copy_block_kernel");
    copy_block_kernel<T><<<static_cast<unsigned>(ceil_div(static_cast<int64_t>(jbb) * jbb, 256)), 256, 0, st>>>(
        TB, NBO, P + NB2 + static_cast<int64_t>(NB2) * NBO, NBO, jbb, jbb);
    URV_LAUNCHED("copy_block_kernel");
    URV_TRY(gemm<T>(false, false, jbb, NB2, 0, T(0), P, NBO, P, NBO, T(0), P + NB2, NBO, nullptr, 0, st));
    URV_TRY(gemm<T>(true, false, NB2, jbb, mp, T(1), Ya, m, Ya + static_cast<int64_t>(NB2) * m, m, T(0), W1, NB2,
                    gw, gwe, st));                                                             // S = Y_A^T Y_B
    URV_TRY(gemm<T>(false, false, NB2, jbb, jbb, T(1), W1, NB2, TB, NBO, T(0), W2, NB2, nullptr, 0, st));  // S T_B
    return gemm<T>(false, false, NB2, jbb, NB2, T(-1), TA, NBO, W2, NB2, T(0), P + static_cast<int64_t>(NB2) * NBO,
                   NBO, nullptr, 0, st);                                                       // -T_A S T_B
  };

  // Z <- Z (I - Y T Y^T) for the block at j0 and every target, on the third stream.
  const hipStream_t s3 = side.stream3;
  // With 128-column blocks the targets take pairs of blocks (k = 256): for a
  // pair (A, B) the joined T = [[T_A, -T_A (Y_A^T Y_B) T_B], [0, T_B]] is
  // formed here, off the factorisation chain.
  auto apply_targets = [&](int64_t jblk) -> int {
    int64_t j0 = jblk;
    int jb = static_cast<int>(std::min<int64_t>(nbo, n - j0));
    const T* Tb = w.Tm + j0 * NBO;
    if (nbo == NB2 && target_pairs()) {
      const bool second = (jblk / NB2) % 2 == 1;
      if (!second && jblk + NB2 < n) return URV_OK;  // wait for the pair's second block
      if (second) {
        j0 = jblk - NB2;
        jb = NB2 + static_cast<int>(std::min<int64_t>(NB2, n - jblk));
        T* P = w.Tp + j0 * NBO;
        URV_TRY(pair_t(j0, P, w.W1f, w.W2f, w.gemm_work_f, w.gemm_work_f_elems, s3));
        Tb = P;
      }
    }
    const int64_t mp = m - j0;
    const T* Yb = w.Y + j0 + j0 * m;
    for (int i = 0; i < ntargets; ++i) {
      const QrTarget<T>& z = targets[i];
      T* Zb = z.Z + j0 * z.ldz;
      URV_TRY(gemm<T>(false, false, z.rows, jb, mp, T(1), Zb, z.ldz, Yb, m, T(0), w.W1f, z.rows,
                      w.gemm_work_f, w.gemm_work_f_elems, s3));               // Z Y
      URV_TRY(gemm<T>(false, false, z.rows, jb, jb, T(1), w.W1f, z.rows, Tb, NBO, T(0), w.W2f, z.rows,
                      nullptr, 0, s3));                                       // (Z Y) T
      URV_TRY(gemm<T>(false, true, z.rows, mp, jb, T(-1), w.W2f, z.rows, Yb, m, T(1), Zb, z.ldz, nullptr,
                      0, s3));                                                // Z -= (Z Y T) Y^T
    }
    return URV_OK;
  };

  // Streams: s2 factors the blocks, one after the other (the critical chain);
  // s updates the next block's columns once block k is factored, raises that
  // block's flag, and updates the block after next; s4 updates the rest; s3
  // applies block k to the targets.  The factorisation of block k+1 is queued
  // on s2 right behind block k's and waits for its flag on the device, so its
  // workgroups take their CUs while the update runs.  The flag is always
  // queued before the factorisation that waits for it, so the two can share a
  // hardware queue.  With URV_PANEL_EARLY=0, s2 updates the next block's
  // columns itself, between the factorisations.
  // each block's factorisation applies the previous block to its own columns (the
  // streaming panel with both parts in one launch; URV_PANEL_PREV=0 turns it off)
  const bool prev_fused = tsqr && fused && nbo == NB2 && panel_prev();
  // Queued early, a launch would hold its compute units spinning while the updates it
  // waits for still run (measured slower with the previous block fused); the separate
  // near update is faster queued early.
  const bool early = panel_early(!prev_fused);
  const bool pair_bulk = nbo == NB2 && bulk_pairs();
  const int ahead = pair_bulk ? 1 : lookahead();
  const bool ahead2 = ahead >= 2;
  int64_t target_rows_max = 0;
  for (int i = 0; i < ntargets; ++i) target_rows_max = std::max<int64_t>(target_rows_max, targets[i].rows);
  const int64_t lag = target_lag(m, n, target_rows_max);
  int64_t tgt_next = 0;  // first block whose targets are not yet queued
  URV_HIP(hipEventRecord(side.ev_next, s));      // the cleared flags and slots
  URV_HIP(hipStreamWaitEvent(s2, side.ev_next, 0));
  if (ntargets > 0) URV_HIP(hipStreamWaitEvent(s3, side.ev_next, 0));  // targets written before the call
  // "block j is factored": two events, by the parity of j, so that block j's event is
  // still the one recorded for it while block j + 1 is queued
  const hipEvent_t ev_fact[2] = {side.ev_fact, side.ev_fact2};
  URV_TRY(factor_block(0, nullptr));
  URV_HIP(hipEventRecord(ev_fact[0], s2));
  bool near_pending = false, bulk_pending = false;
  for (int64_t j0 = 0; j0 < n; j0 += nbo) {
    const int par = static_cast<int>((j0 / nbo) & 1);
    URV_HIP(hipStreamWaitEvent(s, ev_fact[par], 0));  // block j0 is factored
    const int64_t j1 = j0 + nbo;
    if (ntargets > 0) {
      // blocks up to j0 - lag now; at the last block, all that are left
      const int64_t upto = j1 >= n ? j0 : j0 - lag * nbo;
      if (tgt_next <= upto) URV_HIP(hipStreamWaitEvent(s3, ev_fact[par], 0));
      for (; tgt_next <= upto; tgt_next += nbo) URV_TRY(apply_targets(tgt_next));
    }
    if (j1 >= n) break;
    const int64_t nn = std::min<int64_t>(nbo, n - j1);
    if (prev_fused) {
      // block j1's factorisation applies block j0 to its columns itself; the earlier blocks'
      // shares came from s and s4, announced by block j1's flag (none before block 2), or,
      // with URV_PANEL_EARLY=0, by the event after them on s (the launch then takes its
      // compute units only once its columns are ready)
      if (early || j0 == 0) {
        URV_TRY(factor_block(j1, j0 > 0 ? ready + j1 / NB : nullptr, j0));
      } else {
        URV_HIP(hipStreamWaitEvent(s2, side.ev_near, 0));
        URV_TRY(factor_block(j1, nullptr, j0));
      }
    } else if (early) {
      // block j1's columns on s (after the previous block's share, also on s), its flag,
      // then its factorisation on s2
      URV_TRY(apply_block(j0, j1, nn, kOnCallerStream));
      signal_kernel<<<1, 64, 0, s>>>(ready + j1 / NB, 1u);
      URV_LAUNCHED("signal_kernel");
      URV_TRY(factor_block(j1, ready + j1 / NB));
    } else {
      // the chain: block j1's columns (the previous block's share came from s), then its factorisation
      if (near_pending) URV_HIP(hipStreamWaitEvent(s2, side.ev_near, 0));
      URV_TRY(apply_block(j0, j1, nn, kOnPanelStream));
      URV_TRY(factor_block(j1, nullptr));
    }
    URV_HIP(hipEventRecord(ev_fact[par ^ 1], s2));
    const int64_t j2 = j1 + nn;
    if (j2 >= n) continue;
    // the block after next, which needs the previous bulk update first
    const int64_t nn2 = std::min<int64_t>(nbo, n - j2);
    // With block pairs, block j0 closes a pair when its index is odd: the pair (k = 256)
    // goes to block j2 and, below, to the rest; a block that opens a pair updates only
    // block j2 (it reaches the columns beyond with its pair).  Block j2 still gets the
    // blocks in order: the previous pair's bulk update covers it and comes first.
    const bool closes = pair_bulk && (j0 / NB2) % 2 == 1;
    // With two look-ahead blocks, block j2's columns already waited for the bulk update
    // that covers them, before block j0 - 1's update of them (stream order on s).
    if (bulk_pending && !ahead2) URV_HIP(hipStreamWaitEvent(s, side.ev_bulk, 0));
    if (closes) {
      // the pair's T (into Tq, which the previous pair's bulk update has finished reading)
      URV_TRY(pair_t(j0 - NB2, w.Tq, w.W1n, w.W2n, w.gemm_work_n, w.gemm_work_n_elems, s));
      URV_HIP(hipEventRecord(side.ev_pair, s));
      URV_TRY(apply_block(j0 - NB2, j2, nn2, kOnCallerStream, 2 * NB2, w.Tq));
    } else {
      URV_TRY(apply_block(j0, j2, nn2, kOnCallerStream));
    }
    if (prev_fused) {
      // block j2's columns now hold every share but block j1's, which its factorisation applies
      signal_kernel<<<1, 64, 0, s>>>(ready + j2 / NB, 1u);
      URV_LAUNCHED("signal_kernel");
    }
    URV_HIP(hipEventRecord(side.ev_near, s));
    near_pending = true;
    const int64_t j3 = j2 + nn2;
    if (j3 >= n) continue;
    if (ahead2) {
      // the next ahead - 1 column blocks too on s, the farthest after block j0 - 1's bulk
      // update (which covers it; the nearer ones had that wait in earlier iterations), and
      // the rest on s4: a block's columns wait for the bulk update ahead + 2 blocks back
      int64_t jc = j3;
      for (int e = 0; e < ahead - 1 && jc < n; ++e) {
        const int64_t nc = std::min<int64_t>(nbo, n - jc);
        if (e == ahead - 2 && bulk_pending) URV_HIP(hipStreamWaitEvent(s, side.ev_bulk, 0));
        URV_TRY(apply_block(j0, jc, nc, kOnCallerStream));
        jc += nc;
      }
      if (jc >= n) continue;
      URV_HIP(hipStreamWaitEvent(s4, ev_fact[par], 0));
      URV_TRY(apply_block(j0, jc, n - jc, kOnBulkStream));
      URV_HIP(hipEventRecord(side.ev_bulk, s4));
      bulk_pending = true;
      continue;
    }
    if (pair_bulk && !closes) continue;  // block j1 closes the pair and has j2 + nn2 < n too
    // the rest, beside the chain: needs block j0's reflectors only (its columns are not the
    // near updates', and the previous bulk update is ahead of it on s4), or the pair's T
    if (closes) {
      URV_HIP(hipStreamWaitEvent(s4, side.ev_pair, 0));
      URV_TRY(apply_block(j0 - NB2, j3, n - j3, kOnBulkStream, 2 * NB2, w.Tq));
    } else {
      URV_HIP(hipStreamWaitEvent(s4, ev_fact[par], 0));
      URV_TRY(apply_block(j0, j3, n - j3, kOnBulkStream));
    }
    URV_HIP(hipEventRecord(side.ev_bulk, s4));
    bulk_pending = true;
  }
  if (bulk_pending) URV_HIP(hipStreamWaitEvent(s, side.ev_bulk, 0));
  if (ntargets > 0) {
    // Q = H_1 ... H_n [D; 0]: the sign fix D on the first n columns, then join
    for (int i = 0; i < ntargets; ++i)
      URV_TRY(scale_cols_sign<T>(targets[i].Z, targets[i].rows, n, targets[i].ldz, X, ldx, s3));
    URV_HIP(hipEventRecord(side.ev_tgt, s3));
    URV_HIP(hipStreamWaitEvent(s, side.ev_tgt, 0));
  }

  if (R) {
    extract_r_kernel<T><<<static_cast<unsigned>(ceil_div(n * n, 256)), 256, 0, s>>>(X, ldx, n, R, ldr);
    URV_LAUNCHED("extract_r_kernel");
  }
  if (Q) URV_TRY(form_q<T>(X, ldx, m, n, Q, ldq, w, s, false));
  return URV_OK;
}

template <class T>
int form_q(const T* X, int64_t ldx, int64_t m, int64_t n, T* Q, int64_t ldq, const QrWorkT<T>& w, hipStream_t s,
           bool pairs) {
  if (n == 0) return URV_OK;
  init_q_kernel<T><<<static_cast<unsigned>(ceil_div(m * n, 256)), 256, 0, s>>>(X, ldx, m, n, Q, ldq);
  URV_LAUNCHED("init_q_kernel");
  const int nbo = outer_block();
  // pairs of 128-column blocks with the joined T the target products formed (a lone last
  // block keeps its own T)
  const int64_t step = (pairs && nbo == NB2 && target_pairs()) ? 2 * NB2 : nbo;
  const int64_t nouter = ceil_div(n, step);
  for (int64_t blk = nouter - 1; blk >= 0; --blk) {
    const int64_t j0 = blk * step;
    const int jb = static_cast<int>(std::min<int64_t>(step, n - j0));
    const int64_t mp = m - j0, nq = n - j0;
    const T* Yb = w.Y + j0 + j0 * m;
    const T* Tb = (step > nbo && jb > NB2) ? w.Tp + j0 * NBO : w.Tm + j0 * NBO;
    T* Qb = Q + j0 + j0 * ldq;
    URV_TRY(gemm<T>(true, false, jb, nq, mp, T(1), Yb, m, Qb, ldq, T(0), w.W1, NBO, w.gemm_work,
                    w.gemm_work_elems, s));
    URV_TRY(gemm<T>(false, false, jb, nq, jb, T(1), Tb, NBO, w.W1, NBO, T(0), w.W2, NBO, nullptr, 0, s));
    URV_TRY(gemm<T>(false, false, mp, nq, jb, T(-1), Yb, m, w.W2, NBO, T(1), Qb, ldq, nullptr, 0, s));
  }
  return URV_OK;
}

template <class T>
unsigned* qr_error_flag(const QrWorkT<T>& w, int64_t n) {
  return w.sync + ceil_div(n, NB);
}

template <class T>
int qr_clear_error_flag(const QrWorkT<T>& w, int64_t n, hipStream_t s) {
  fill_u32_kernel<<<1, 64, 0, s>>>(qr_error_flag(w, n), 1, 0u);
  URV_LAUNCHED("fill_u32_kernel");
  return URV_OK;
}

#define URV_QR_INSTANTIATE(T)                                                                 \
  template size_t qr_work_bytes<T>(int64_t, int64_t, int64_t);                                \
  template void qr_work_carve<T>(Arena&, int64_t, int64_t, QrWorkT<T>&, int64_t);            \
  template int qr_pos<T>(T*, int64_t, int64_t, int64_t, T*, int64_t, T*, int64_t,             \
                         const QrWorkT<T>&, hipStream_t, const QrTarget<T>*, int);            \
  template int form_q<T>(const T*, int64_t, int64_t, int64_t, T*, int64_t, const QrWorkT<T>&, hipStream_t, \
                         bool);                                                                \
  template unsigned* qr_error_flag<T>(const QrWorkT<T>&, int64_t);                          \
  template int qr_clear_error_flag<T>(const QrWorkT<T>&, int64_t, hipStream_t);
URV_QR_INSTANTIATE(double)
URV_QR_INSTANTIATE(float)
#undef URV_QR_INSTANTIATE

}  // namespace urv
