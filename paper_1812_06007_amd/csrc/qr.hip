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
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// sum over the waves of a workgroup, in a fixed order
template <class T, int W>
__device__ inline T sum_waves(const T (*red)[W], int c) {
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
// upper triangular (ld ldt): the middle factor of (I - Y T^T Y^T) C, fused with
// the split-K reduction of W1 = Y^T C.  Four columns per workgroup.
template <class T>
__global__ __launch_bounds__(256) void reduce_tmul_kernel(int jb, int64_t N, int splits, const T* __restrict__ P,
                                                          const T* __restrict__ Tm, int ldt, T* __restrict__ W2,
                                                          int64_t ldw2) {
  constexpr int CW = 4;
  __shared__ T w1[CW][4 * NB + 1];
  const int64_t c0 = static_cast<int64_t>(blockIdx.x) * CW;
  const int cols = static_cast<int>(min<int64_t>(CW, N - c0));
  const int64_t slice = static_cast<int64_t>(jb) * N;
  for (int e = threadIdx.x; e < jb * cols; e += blockDim.x) {
    const int k = e % jb, jj = e / jb;
    w1[jj][k] = sum_splits(P + (c0 + jj) * jb + k, splits, slice);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < jb * cols; e += blockDim.x) {
    const int i = e % jb, jj = e / jb;
    const T* tcol = Tm + static_cast<int64_t>(i) * ldt;
    T a0 = 0, a1 = 0;
    int k = 0;
    for (; k + 1 <= i; k += 2) {
      a0 += tcol[k] * w1[jj][k];
      a1 += tcol[k + 1] * w1[jj][k + 1];
    }
    if (k <= i) a0 += tcol[k] * w1[jj][k];
    W2[i + (c0 + jj) * ldw2] = a0 + a1;
  }
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
// and waits for it on the device (URV_PANEL_EARLY=0 orders them on one stream, for tuning).
bool panel_early() {
  const char* e = std::getenv("URV_PANEL_EARLY");
  return !(e && std::atoi(e) == 0);
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
// MI355X at n = 8000, q = 2: 343 ms with no lag, 335-334 ms with 10-14
// blocks, 338 ms with 20 (the held-back products then outlast the chain).
int target_lag() {
  const char* e = std::getenv("URV_TARGET_LAG");
  return e ? std::max(0, std::atoi(e)) : 12;
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
  size_t y, t, tau, w, xch, sync, gemm_work, wb, gemm_work_b, wf, gemm_work_f, wn, gemm_work_n, tp, jxch;
};

QrSizes qr_sizes(int64_t m, int64_t n, int64_t target_rows) {
  QrSizes z;
  const int64_t nblocks = ceil_div(n, NB);
  z.y = static_cast<size_t>(m) * n;
  z.t = static_cast<size_t>(NBO) * n;
  z.tau = n;
  z.w = static_cast<size_t>(NBO) * n;
  z.xch = 2 * (static_cast<size_t>(panel_wgs(m)) + 1) * NB * 2;
  z.jxch = (static_cast<size_t>(panel_wgs(m)) + 1) * kJoinEntries * 2;
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
      gw = std::max(gw, gemm_work_elems(jb, nc - nn, mp));
      gw = std::max(gw, gemm_work_elems(jb, n - j0, mp));
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
  auto panel = [&](int64_t r0, int jbp, T* Tp, int zero_above, const PanelJoin<T>& join, int jb2,
                   const unsigned* wf) -> int {
    const int64_t mp = m - r0;
    const unsigned P = static_cast<unsigned>(panel_wgs(mp));
    panel_kernel<T><<<P, PANEL_THREADS, 0, s2>>>(X + r0 + r0 * ldx, ldx, mp, jbp, w.Y + r0 + r0 * m, m,
                                                 w.tau + r0, Tp, NBO, w.xch, panels * NB, err, zero_above, join,
                                                 pwait, jb2, wf);
    panels += jb2 > 0 ? 2 : 1;
    URV_LAUNCHED("panel_kernel");
    return URV_OK;
  };
  // Householder vectors, tau and T (at Tp, ld NBO) of the sub-block of width
  // jbs at row/column r0 of the outer block starting at j0, on the side stream;
  // with wf, its first launch waits for that flag before reading its columns.
  auto factor_sub = [&](int64_t j0, int64_t r0, int jbs, T* Tp, const unsigned* wf) -> int {
    const int jb1 = std::min(jbs, NB), jb2 = jbs - jb1;
    const int64_t mp = m - r0;
    T* Yb = w.Y + r0 + r0 * m;
    if (jb2 > 0 && fused) {
      // both panels in one launch; its exchange of W = Y1^T C2 and S12 uses the join buffers
      PanelJoin<T> bufs;
      bufs.ps = w.jxch;
      bufs.sums = w.jxch + w.jxch_words - 2 * kJoinEntries;
      return panel(r0, jb1, Tp, static_cast<int>(r0 - j0), bufs, jb2, wf);
    }
    URV_TRY(panel(r0, jb1, Tp, static_cast<int>(r0 - j0), PanelJoin<T>{}, 0, wf));
    if (jb2 > 0) {
      // first panel's reflectors applied to the second panel's columns:
      // C2 -= Y1 (T1^T (Y1^T C2)), the reduction of Y1^T C2 fused with T1^T
      T* C2 = X + r0 + (r0 + jb1) * ldx;
      int splits = 0;
      URV_TRY(gemm_partials<T>(true, false, jb1, jb2, mp, Yb, m, C2, ldx, w.gemm_work_b, w.gemm_work_b_elems,
                               &splits, s2));
      reduce_tmul_kernel<T><<<static_cast<unsigned>(ceil_div(jb2, 4)), 256, 0, s2>>>(
          jb1, jb2, splits, w.gemm_work_b, Tp, NBO, w.W2b, NBO);
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
  auto factor_block = [&](int64_t j0, const unsigned* wf) -> int {
    const int jbo = static_cast<int>(std::min<int64_t>(nbo, n - j0));
    const int ja = std::min(jbo, NB2), jbb = jbo - ja;
    const int64_t mp = m - j0;
    T* Tb = w.Tm + j0 * NBO;
    // Y is kept zero above the diagonal back to the start of the pair of
    // 128-column blocks, so that the targets can take a pair at once
    const int64_t jz = j0 - (j0 / NB2 % 2) * NB2;
    URV_TRY(factor_sub(jz, j0, ja, Tb, wf));
    if (jbb > 0) {
      const T* Ya = w.Y + j0 + j0 * m;
      T* CB = X + j0 + (j0 + ja) * ldx;
      int splits = 0;
      URV_TRY(gemm_partials<T>(true, false, ja, jbb, mp, Ya, m, CB, ldx, w.gemm_work_b, w.gemm_work_b_elems,
                               &splits, s2));
      reduce_tmul_kernel<T><<<static_cast<unsigned>(ceil_div(jbb, 4)), 256, 0, s2>>>(
          ja, jbb, splits, w.gemm_work_b, Tb, NBO, w.W2b, NBO);
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
  auto apply_block = [&](int64_t j0, int64_t c0, int64_t nc, int where) -> int {
    if (nc <= 0) return URV_OK;
    const int jb = static_cast<int>(std::min<int64_t>(nbo, n - j0));
    const int64_t mp = m - j0;
    const T* Yb = w.Y + j0 + j0 * m;
    const T* Tb = w.Tm + j0 * NBO;
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
    reduce_tmul_kernel<T><<<static_cast<unsigned>(ceil_div(nc, 4)), 256, 0, st>>>(jb, nc, splits, gw, Tb, NBO,
                                                                                   W2, NBO);  // T^T (Y^T C)
    URV_LAUNCHED("reduce_tmul_kernel");
    URV_TRY(gemm<T>(false, false, mp, nc, jb, T(-1), Yb, m, W2, NBO, T(1), Cb, ldx, nullptr, 0, st));
    return URV_OK;
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
        const int jbb = static_cast<int>(std::min<int64_t>(NB2, n - jblk));
        jb = NB2 + jbb;
        const int64_t mp = m - j0;
        T* P = w.Tp + j0 * NBO;
        const T* TA = w.Tm + j0 * NBO;
        const T* TB = w.Tm + jblk * NBO;
        const T* Ya = w.Y + j0 + j0 * m;
        copy_block_kernel<T><<<static_cast<unsigned>(ceil_div(NB2 * NB2, 256)), 256, 0, s3>>>(TA, NBO, P, NBO, NB2,
                                                                                             NB2);
        URV_LAUNCHED("copy_block_kernel");
        copy_block_kernel<T><<<static_cast<unsigned>(ceil_div(static_cast<int64_t>(jbb) * jbb, 256)), 256, 0, s3>>>(
            TB, NBO, P + NB2 + static_cast<int64_t>(NB2) * NBO, NBO, jbb, jbb);
        URV_LAUNCHED("copy_block_kernel");
        URV_TRY(gemm<T>(false, false, jbb, NB2, 0, T(0), P, NBO, P, NBO, T(0), P + NB2, NBO, nullptr, 0, s3));
        URV_TRY(gemm<T>(true, false, NB2, jbb, mp, T(1), Ya, m, Ya + static_cast<int64_t>(NB2) * m, m, T(0), w.W1f,
                        NB2, w.gemm_work_f, w.gemm_work_f_elems, s3));                           // S = Y_A^T Y_B
        URV_TRY(gemm<T>(false, false, NB2, jbb, jbb, T(1), w.W1f, NB2, TB, NBO, T(0), w.W2f, NB2, nullptr, 0,
                        s3));                                                                     // S T_B
        URV_TRY(gemm<T>(false, false, NB2, jbb, NB2, T(-1), TA, NBO, w.W2f, NB2, T(0),
                        P + static_cast<int64_t>(NB2) * NBO, NBO, nullptr, 0, s3));               // -T_A S T_B
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
  const bool early = panel_early();
  const int64_t lag = target_lag();
  int64_t tgt_next = 0;  // first block whose targets are not yet queued
  URV_HIP(hipEventRecord(side.ev_next, s));      // the cleared flags and slots
  URV_HIP(hipStreamWaitEvent(s2, side.ev_next, 0));
  if (ntargets > 0) URV_HIP(hipStreamWaitEvent(s3, side.ev_next, 0));  // targets written before the call
  URV_TRY(factor_block(0, nullptr));
  URV_HIP(hipEventRecord(side.ev_fact, s2));
  bool near_pending = false, bulk_pending = false;
  for (int64_t j0 = 0; j0 < n; j0 += nbo) {
    URV_HIP(hipStreamWaitEvent(s, side.ev_fact, 0));  // block j0 is factored
    const int64_t j1 = j0 + nbo;
    if (ntargets > 0) {
      // blocks up to j0 - lag now; at the last block, all that are left
      const int64_t upto = j1 >= n ? j0 : j0 - lag * nbo;
      if (tgt_next <= upto) URV_HIP(hipStreamWaitEvent(s3, side.ev_fact, 0));
      for (; tgt_next <= upto; tgt_next += nbo) URV_TRY(apply_targets(tgt_next));
    }
    if (j1 >= n) break;
    const int64_t nn = std::min<int64_t>(nbo, n - j1);
    if (early) {
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
    URV_HIP(hipEventRecord(side.ev_fact, s2));
    const int64_t j2 = j1 + nn;
    if (j2 >= n) continue;
    // the block after next, which needs the previous bulk update first
    const int64_t nn2 = std::min<int64_t>(nbo, n - j2);
    if (bulk_pending) URV_HIP(hipStreamWaitEvent(s, side.ev_bulk, 0));
    URV_TRY(apply_block(j0, j2, nn2, kOnCallerStream));
    URV_HIP(hipEventRecord(side.ev_near, s));
    near_pending = true;
    const int64_t j3 = j2 + nn2;
    if (j3 >= n) continue;
    URV_HIP(hipStreamWaitEvent(s4, side.ev_near, 0));
    URV_TRY(apply_block(j0, j3, n - j3, kOnBulkStream));  // the rest, beside the chain
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
  if (Q) {
    init_q_kernel<T><<<static_cast<unsigned>(ceil_div(m * n, 256)), 256, 0, s>>>(X, ldx, m, n, Q, ldq);
    URV_LAUNCHED("init_q_kernel");
    const int64_t nouter = ceil_div(n, nbo);
    for (int64_t blk = nouter - 1; blk >= 0; --blk) {
      const int64_t j0 = blk * nbo;
      const int jb = static_cast<int>(std::min<int64_t>(nbo, n - j0));
      const int64_t mp = m - j0, nq = n - j0;
      const T* Yb = w.Y + j0 + j0 * m;
      const T* Tb = w.Tm + j0 * NBO;
      T* Qb = Q + j0 + j0 * ldq;
      URV_TRY(gemm<T>(true, false, jb, nq, mp, T(1), Yb, m, Qb, ldq, T(0), w.W1, NBO, w.gemm_work,
                      w.gemm_work_elems, s));
      URV_TRY(gemm<T>(false, false, jb, nq, jb, T(1), Tb, NBO, w.W1, NBO, T(0), w.W2, NBO, nullptr, 0, s));
      URV_TRY(gemm<T>(false, false, mp, nq, jb, T(-1), Yb, m, w.W2, NBO, T(1), Qb, ldq, nullptr, 0, s));
    }
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
  template unsigned* qr_error_flag<T>(const QrWorkT<T>&, int64_t);                          \
  template int qr_clear_error_flag<T>(const QrWorkT<T>&, int64_t, hipStream_t);
URV_QR_INSTANTIATE(double)
URV_QR_INSTANTIATE(float)
#undef URV_QR_INSTANTIATE

}  // namespace urv
