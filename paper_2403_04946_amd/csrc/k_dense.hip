// Small dense factorisation used once per TT bond.
//
// jacobi_svd: one-sided (Hestenes) Jacobi SVD of the small square factor of
// a truncation step (the "SVD of the R factor" of App. A.4): columns are
// rotated pairwise until orthogonal; their norms are the singular values
// and the normalised columns the left singular vectors.  The columns are
// cut into blocks of 8.  One sweep runs every block on its own (all pairs
// inside a block, circle ordering) and then the rounds of a round-robin
// tournament over the blocks, one workgroup per block pair meeting all 64
// pairs between the two blocks.  A column pair is held in registers by a
// group of 32 lanes (a whole wavefront beyond 320 rows); columns move
// between groups through LDS.  Every column pair meets once per sweep, so
// this is a cyclic Jacobi method with a block ordering; the iteration stops
// when a sweep would rotate no pair, found by one launch that applies the
// rotation test to every pair at once (or by a sweep without a rotation).
#include <mutex>
#include <string>

#include "common.hpp"
#include "dpp.hpp"
#include "recip.hpp"

namespace ttf {

constexpr int JB_NORMS = 1536;  // columns of the finishing kernel

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

// ------------------------------------------------------------ Jacobi SVD
constexpr int JAC_THREADS = 1024;
constexpr int JAC_GROUPS = JAC_THREADS / 16;
constexpr int JAC_MAX_SWEEPS = 60;
constexpr int JB_COLS = 8;     // columns per block
constexpr int JB_MAXM = 1536;  // rows supported by the register-resident form
constexpr int JB_MAXK = 1536;  // columns
constexpr int JB_XCHUNK = 8;   // rows per lane moved through LDS at a time
constexpr int JB_MAXS = 64;    // sweep counters
// counters of one SVD: JB_MAXS + 2 ints, |B|_F^2 (a double), then the
// arrival count and give-up flag of the fused sweeps' barrier
constexpr int JB_BAR = JB_MAXS + 4;
constexpr size_t JB_ROT_BYTES = sizeof(int) * (JB_MAXS + 2) + 64;
static_assert(sizeof(int) * (JB_BAR + 2) <= JB_ROT_BYTES, "barrier words beyond the counters");
// workgroups of a fused launch (P / 2) up to which the sweeps run fused:
// all of them must be resident at once, which this many are on any
// MI355X even beside other work
constexpr int JB_FUSED_MAX_WG = 64;
// rows up to which the sweeps run fused (beyond, the columns held in
// registers by both phases would spill)
constexpr int JB_FUSED_MAXM = 640;

// round-robin pairing of players 0..P-1 (P even) in round r
__device__ inline void rr_pair(int P, int r, int i, int& a, int& b) {
  const int M = P - 1;
  if (i == 0) {
    a = 0;
    b = 1 + (r % M);
  } else {
    a = 1 + ((r + i) % M);
    b = 1 + ((r - i + M) % M);
  }
}

void jacobi_blocked(tt_ctx* ctx, int m, int k, zc* B, zc* U, double* sigma, int* sweeps, int* rot_ext = nullptr);

void jacobi_svd(tt_ctx* ctx, int m, int k, zc* B, zc* U, double* sigma, int* sweeps) {
  if (k <= 0) return;
  if (k > JB_MAXK || m > JB_MAXM || m < 1) fail(TT_EINVAL, "jacobi_svd: sizes above the supported maximum of 1536");
  std::string shape;
  if (ctx->profile_shapes) shape = "jacobi:" + std::to_string(m) + "x" + std::to_string(k);
  KTimer kt2(ctx->profile_shapes ? ctx : nullptr, shape.c_str(), 0.0, 0.0);
  KTimer kt(ctx, "jacobi_svd", 0.0, 0.0);
  jacobi_blocked(ctx, m, k, B, U, sigma, sweeps);
}

// ------------------------------------------ allocation-free variant
// The counters of jacobi_svd_noalloc live in a file-scope device array, one
// copy per GPU, whose address is looked up once per device (the host-side
// name is not a device address); NOALLOC_BYTES bytes, held until the
// process ends.  Every call on a GPU uses that GPU's copy.
constexpr size_t NOALLOC_BYTES = 1024;
static_assert(JB_ROT_BYTES + sizeof(int) <= NOALLOC_BYTES, "counters exceed the static scratch");
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex noalloc_mu;
static void* noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

void noalloc_scratch_init(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) fail(TT_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(noalloc_mu);
  if (noalloc_ptr[device]) return;
  void* p = nullptr;
  hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
  if (!p) fail(TT_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
  noalloc_ptr[device] = p;
}

void jacobi_svd_noalloc(tt_ctx* ctx, int m, int k, zc* B, zc* U, double* sigma, int* sweeps_host) {
  if (k > JB_MAXK || m > JB_MAXM || m < 1 || k < 1)
    fail(TT_EINVAL, "tt_svd_small_noalloc: sizes outside 1..1536");
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (ctx->device >= 0 && ctx->device < NOALLOC_MAX_DEVICES) base = noalloc_ptr[ctx->device];
  }
  if (!base) fail(TT_EHIP, "tt_svd_small_noalloc: the scratch of this device was not set up");
  int* rot = (int*)base;
  int* sw = (int*)((char*)base + JB_ROT_BYTES);
  jacobi_blocked(ctx, m, k, B, U, sigma, sw, rot);
  int h = 0;
  TTF_HIP(hipMemcpyAsync(&h, sw, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  TTF_HIP(hipStreamSynchronize(ctx->stream));
  *sweeps_host = h;
}

// ------------------------------------------------ block-parallel Jacobi
// A column pair is held by a group of GS lanes (16: one DPP row, 32: half a
// wavefront, 64: a whole wavefront), lane l owning rows l + GS j, j < RPL.
template <int GS>
__device__ inline double group_sum(double x) {
  x = row16_sum(x);
  if (GS >= 32) x = row_pair_sum(x);
  if (GS == 64) x = half_pair_sum(x);
  return x;
}

// Rotate the column pair (x, y) so that x^H y = 0 unless they already are
// to the tolerance; returns 1 when a rotation was applied.
// Squared norms al, be of the columns x, y of a pair and g = x^H y (gr +
// i gi), summed over the GS lanes of the group: each lane adds its RPL rows
// in order, then the lane sums are combined in a fixed tree, so every
// kernel that calls this sees the same bits for the same columns.
template <int RPL, int GS>
__device__ inline void jacobi_pair_sums(const zc (&x)[RPL], const zc (&y)[RPL], double& al, double& be, double& gr,
                                        double& gi) {
  al = 0, be = 0, gr = 0, gi = 0;
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    const zc a = x[j], c = y[j];
    al += a.x * a.x + a.y * a.y;
    be += c.x * c.x + c.y * c.y;
    gr += a.x * c.x + a.y * c.y;  // conj(x) * y
    gi += a.x * c.y - a.y * c.x;
  }
  al = group_sum<GS>(al);
  be = group_sum<GS>(be);
  gr = group_sum<GS>(gr);
  gi = group_sum<GS>(gi);
}

// The rotation test: |g| above tol times the geometric mean of the column
// norms; pairs with a negligible column (squared norm below abs2) are left
// alone.
__device__ inline bool jacobi_needs_rotation(double al, double be, double g2, double tol, double abs2) {
  return g2 > tol * tol * al * be && g2 != 0.0 && al >= abs2 && be >= abs2;
}

template <int RPL, int GS>
__device__ inline int jacobi_rotate(zc (&x)[RPL], zc (&y)[RPL], double tol, double abs2) {
  double al, be, gr, gi;
  jacobi_pair_sums<RPL, GS>(x, y, al, be, gr, gi);
  const double g2 = gr * gr + gi * gi;
  if (!jacobi_needs_rotation(al, be, g2, tol, abs2)) return 0;
  double ig, tt, cs;
  if (g2 >= 0x1p-900 && g2 <= 0x1p900) {
    // one dependent chain of reciprocal square roots and one reciprocal
    ig = rsqrt_newton(g2);  // 1 / |g|
    const double zeta = (be - al) * (0.5 * ig);
    const double q = fma(zeta, zeta, 1.0);  // |zeta| < 1e30: al, be lie within 1e30 of each other
    const double t = rcp_newton(fabs(zeta) + q * rsqrt_newton(q));
    tt = zeta >= 0 ? t : -t;
    cs = rsqrt_newton(fma(tt, tt, 1.0));
  } else {  // |g| outside [2^-450, 2^450]: Frobenius norm below 1e-45 or above 3e67
    ig = 1.0 / sqrt(g2);
    const double zeta = (be - al) * (0.5 * ig);
    tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    cs = 1.0 / sqrt(1.0 + tt * tt);
  }
  const double sn = cs * tt;
  const double er = gr * ig, ei = gi * ig;  // e^{i phi}
  const double ser = sn * er, sei = sn * ei;
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    const zc a = x[j], c = y[j];
    // x' = cs x - sn e^{-i phi} y ; y' = sn e^{i phi} x + cs y
    x[j] = make_double2(cs * a.x - (ser * c.x + sei * c.y), cs * a.y - (ser * c.y - sei * c.x));
    y[j] = make_double2((ser * a.x - sei * a.y) + cs * c.x, (ser * a.y + sei * a.x) + cs * c.y);
  }
  return 1;
}

// add the workgroup's rotation count to rot[idx]; returns it to every thread
__device__ inline int jacobi_count(int nrot, int* wg_rot, int* rot, int idx) {
  __syncthreads();
  if (threadIdx.x == 0) *wg_rot = 0;
  __syncthreads();
  if (nrot && (threadIdx.x & 15) == 0) atomicAdd(wg_rot, nrot);
  __syncthreads();
  const int tot = *wg_rot;
  if (threadIdx.x == 0 && tot) atomicAdd(&rot[idx], tot);
  return tot;
}

// Cyclic one-sided Jacobi over the 2W columns c0 .. c0 + 2W - 1 (those >= k
// are absent) with W lane groups.  Circle ordering: group w holds positions
// w and 2W-1-w; after each of the 2W-1 rounds positions 1..2W-1 shift by
// one, so every pair meets once per sweep and after the sweep every column
// is back in place.  Workgroup g handles the columns starting at 2W g.  Up
// to inner_max sweeps (counts in rot[sweep ..]); a launch of sweep > 0
// returns at once when sweep - 1 rotated nothing.
template <int RPL, int W, int GS>
__global__ __launch_bounds__(GS * W) void jacobi_circle_kernel(zc* __restrict__ B, int m, int k, int inner_max,
                                                               int sweep, int* __restrict__ rot, double tol,
                                                               const double* __restrict__ fro2) {
  extern __shared__ double2 xch[];  // W slots of GS XC rows
  __shared__ int wg_rot;
  constexpr int NP = 2 * W - 1;
  constexpr int XC = RPL < JB_XCHUNK ? RPL : JB_XCHUNK;  // rows per lane per exchange
  constexpr int LD = GS * XC;
  const int c0 = blockIdx.x * 2 * W;
  const int w = threadIdx.x / GS, lane = threadIdx.x % GS;
  zc xt[RPL], xb[RPL];
  // columns requested before the convergence flag is read (overlapping loads)
  {
    const int ct = c0 + w, cb = c0 + 2 * W - 1 - w;
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      const int row = lane + GS * j;
      xt[j] = (ct < k && row < m) ? B[row + (long)m * ct] : make_double2(0.0, 0.0);
      xb[j] = (cb < k && row < m) ? B[row + (long)m * cb] : make_double2(0.0, 0.0);
    }
  }
  const double f2 = fro2[0];
  if (sweep > 0 && rot[sweep - 1] == 0) return;
  const double abs2 = 1e-30 * f2;  // (1e-15 |B|_F)^2
  zc* mine = xch + (long)LD * w;
  for (int it = 0; it < inner_max; ++it) {
    int nrot = 0;
    for (int r = 0; r < NP; ++r) {
      // positions w and 2W-1-w after r shifts
      const int pt = (w == 0) ? 0 : ((w - 1 - r) % NP + NP) % NP + 1;
      const int pb = ((2 * W - 2 - w - r) % NP + NP) % NP + 1;
      if (c0 + pt < k && c0 + pb < k) nrot += jacobi_rotate<RPL, GS>(xt, xb, tol, abs2);
      // shift: bottoms move to the previous group (the last one takes its
      // own top), then tops to the next one (group 1 takes group 0's old
      // bottom, left in slot 0 by the first phase)
      // (the rows go through LDS XC per lane at a time)
#pragma unroll
      for (int c = 0; c < RPL; c += XC) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < XC; ++j)
          if (c + j < RPL) mine[lane + GS * j] = xb[c + j];
        __syncthreads();
        if (w <= W - 2) {
          const zc* src = mine + LD;
#pragma unroll
          for (int j = 0; j < XC; ++j)
            if (c + j < RPL) xb[c + j] = src[lane + GS * j];
        } else {
#pragma unroll
          for (int j = 0; j < XC; ++j)
            if (c + j < RPL) xb[c + j] = xt[c + j];
        }
        __syncthreads();
        if (w >= 1 && w <= W - 2) {
#pragma unroll
          for (int j = 0; j < XC; ++j)
            if (c + j < RPL) mine[lane + GS * j] = xt[c + j];
        }
        __syncthreads();
        if (w >= 1) {
          const zc* src = mine - LD;
#pragma unroll
          for (int j = 0; j < XC; ++j)
            if (c + j < RPL) xt[c + j] = src[lane + GS * j];
        }
      }
    }
    const int tot = jacobi_count(nrot, &wg_rot, rot, sweep + it);
    if (tot == 0) break;
  }
  const int ct = c0 + w, cb = c0 + 2 * W - 1 - w;
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    const int row = lane + GS * j;
    if (row < m) {
      if (ct < k) B[row + (long)m * ct] = xt[j];
      if (cb < k) B[row + (long)m * cb] = xb[j];
    }
  }
}

// rows per lane per exchange of the cross kernel: its two sets of slots
// stay within 64 KB of LDS
constexpr int cross_chunk(int rpl, int gs) {
  const int c = gs == 64 ? JB_XCHUNK / 2 : JB_XCHUNK;
  return rpl < c ? rpl : c;
}

// All BC x BC column pairs between blocks a and b (BC columns each; the
// pair of workgroup g in round `round` of a round-robin over P blocks):
// group w keeps column BC a + w and meets column BC b + (w + s) mod BC in
// step s; between steps the b columns move to the previous group.
template <int RPL, int GS, int BC>
__global__ __launch_bounds__(BC * GS) void jacobi_cross_kernel(zc* __restrict__ B, int m, int k, int P, int round,
                                                               int sweep, int* __restrict__ rot, double tol,
                                                               const double* __restrict__ fro2) {
  extern __shared__ double2 xch[];  // two sets of BC slots of GS XC rows
  __shared__ int wg_rot;
  constexpr int XC = cross_chunk(RPL, GS);  // rows per lane per exchange
  constexpr int LD = GS * XC;
  int ba, bb;
  rr_pair(P, round, blockIdx.x, ba, bb);
  const int w = threadIdx.x / GS, lane = threadIdx.x % GS;
  const int ca = ba * BC + w;
  zc xa[RPL], xb[RPL];
  // the columns are requested before the convergence flag is read, so the
  // two memory latencies overlap
  {
    const int cb = bb * BC + w;
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      const int row = lane + GS * j;
      xa[j] = (ca < k && row < m) ? B[row + (long)m * ca] : make_double2(0.0, 0.0);
      xb[j] = (cb < k && row < m) ? B[row + (long)m * cb] : make_double2(0.0, 0.0);
    }
  }
  const double f2 = fro2[0];
  if (sweep > 0 && rot[sweep - 1] == 0) return;
  const double abs2 = 1e-30 * f2;  // (1e-15 |B|_F)^2
  // two sets of exchange slots used alternately: a slot is written again
  // only two exchanges later, after a barrier that follows every read of
  // it, so one barrier per exchange suffices
  zc* mine = xch + (long)LD * w;
  const zc* next = xch + (long)LD * ((w + 1) % BC);
  int nrot = 0, set = 0;
  for (int st = 0; st < BC; ++st) {
    const int cb = bb * BC + (w + st) % BC;
    if (ca < k && cb < k) nrot += jacobi_rotate<RPL, GS>(xa, xb, tol, abs2);
    if (st == BC - 1) break;
#pragma unroll
    for (int c = 0; c < RPL; c += XC) {
      const long off = set ? (long)LD * BC : 0;
      set ^= 1;
#pragma unroll
      for (int j = 0; j < XC; ++j)
        if (c + j < RPL) mine[off + lane + GS * j] = xb[c + j];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < XC; ++j)
        if (c + j < RPL) xb[c + j] = next[off + lane + GS * j];
    }
  }
  jacobi_count(nrot, &wg_rot, rot, sweep);
  const int cb = bb * BC + (w + BC - 1) % BC;
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    const int row = lane + GS * j;
    if (row < m) {
      if (ca < k) B[row + (long)m * ca] = xa[j];
      if (cb < k) B[row + (long)m * cb] = xb[j];
    }
  }
}

__global__ void zero_ints_kernel(int* x, int n) {
  for (int e = threadIdx.x; e < n; e += blockDim.x) x[e] = 0;
}

void zero_ints(tt_ctx* ctx, int* x, int n) {
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(256), 0, ctx->stream, x, n);
  TTF_HIP(hipGetLastError());
}

// singular values (column norms) sorted decreasingly, ties by index; U =
// normalised columns in that order; sweeps = first sweep without rotation
// + 1, or nsweeps when the all-pairs test labelled nsweeps ran (checked) and
// passed, else -1: the iteration stopped at its sweep limit unconverged
__global__ __launch_bounds__(1024) void jacobi_finish_kernel(int m, int k, const zc* __restrict__ B,
                                                             zc* __restrict__ U, double* __restrict__ sigma,
                                                             const int* __restrict__ rot, int nsweeps,
                                                             int checked, int* __restrict__ sweeps_out) {
  __shared__ double norms[JB_NORMS];
  const int t = threadIdx.x, g = t >> 4, l16 = t & 15;
  for (int c = g; c < k; c += JAC_GROUPS) {
    double sq = 0;
    for (int row = l16; row < m; row += 16) {
      const zc a = B[row + (long)m * c];
      sq += a.x * a.x + a.y * a.y;
    }
    sq = row16_sum(sq);
    if (l16 == 0) norms[c] = sqrt(sq);
  }
  __syncthreads();
  for (int c = g; c < k; c += JAC_GROUPS) {
    const double v = norms[c];
    int pos = 0;
    for (int o = 0; o < k; ++o) {
      const double w = norms[o];
      pos += (w > v) || (w == v && o < c);
    }
    const double inv = v > 0 ? 1.0 / v : 0.0;
    for (int row = l16; row < m; row += 16) {
      const zc a = B[row + (long)m * c];
      U[row + (long)m * pos] = make_double2(a.x * inv, a.y * inv);
    }
    if (l16 == 0) sigma[pos] = v;
  }
  if (t == 0) {
    int s = 0;
    while (s < nsweeps && rot[s] != 0) ++s;
    if (s < nsweeps)
      *sweeps_out = s + 1;
    else
      *sweeps_out = (checked && rot[JB_MAXS] < nsweeps) ? nsweeps : -1;
  }
}

// Convergence test over every column pair at once: workgroup t takes the
// t-th pair of blocks (a <= b) in the order (0,0), (0,1), (1,1), (0,2), ...
// and meets the pairs between them in the layout of the cross kernel
// (within one block, each unordered pair once), applying the rotation
// test to the same sums a sweep would compute, without rotating.  A pair
// that would be rotated raises *failed to `label` (atomic maximum, so the
// host reads whether the test labelled `label` failed without clearing).
template <int RPL, int GS, int BC>
__global__ __launch_bounds__(BC * GS) void jacobi_check_kernel(const zc* __restrict__ B, int m, int k, double tol,
                                                               const double* __restrict__ fro2,
                                                               int* __restrict__ failed, int label) {
  extern __shared__ double2 xch[];  // two sets of BC slots of GS XC rows
  constexpr int XC = cross_chunk(RPL, GS);
  constexpr int LD = GS * XC;
  int bb = 0, t = blockIdx.x;
  while (t > bb) t -= ++bb;  // t-th pair: block bb, block ba = t <= bb
  const int ba = t;
  const int w = threadIdx.x / GS, lane = threadIdx.x % GS;
  const int ca = ba * BC + w;
  zc xa[RPL], xb[RPL];
  {
    const int cb = bb * BC + w;
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      const int row = lane + GS * j;
      xa[j] = (ca < k && row < m) ? B[row + (long)m * ca] : make_double2(0.0, 0.0);
      xb[j] = (cb < k && row < m) ? B[row + (long)m * cb] : make_double2(0.0, 0.0);
    }
  }
  const double abs2 = 1e-30 * fro2[0];
  zc* mine = xch + (long)LD * w;
  const zc* next = xch + (long)LD * ((w + 1) % BC);
  int bad = 0, set = 0;
  for (int st = 0; st < BC; ++st) {
    const int cb = bb * BC + (w + st) % BC;
    if (ca < k && cb < k && (ba != bb || ca < cb)) {
      double al, be, gr, gi;
      jacobi_pair_sums<RPL, GS>(xa, xb, al, be, gr, gi);
      bad |= jacobi_needs_rotation(al, be, gr * gr + gi * gi, tol, abs2) ? 1 : 0;
    }
    if (st == BC - 1) break;
#pragma unroll
    for (int c = 0; c < RPL; c += XC) {
      const long off = set ? (long)LD * BC : 0;
      set ^= 1;
#pragma unroll
      for (int j = 0; j < XC; ++j)
        if (c + j < RPL) mine[off + lane + GS * j] = xb[c + j];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < XC; ++j)
        if (c + j < RPL) xb[c + j] = next[off + lane + GS * j];
    }
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicMax(failed, label);
}

// ------------------------------------------ one launch per batch of sweeps
// Grid-wide barrier of the fused sweeps.  Every workgroup adds one arrival
// to bar[0] and waits until `target` arrivals are counted.  The wait is
// bounded: after `limit` polls, or once another workgroup has given up
// (bar[1] set), it gives up and sets bar[1]; the workgroups then return and
// the host reports the SVD as unconverged.  Device-scope fences publish the
// columns written before the barrier and drop stale cached copies after it
// (the L2 caches of the chiplets are not coherent with each other).
__device__ inline bool fused_barrier(int* bar, int target, long limit, int* gave_up_lds) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    __hip_atomic_fetch_add(bar, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int gave_up = 0;
    long polls = 0;
    while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (polls >= limit || __hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        gave_up = 1;
        __hip_atomic_store(bar + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      ++polls;
      __builtin_amdgcn_s_sleep(2);
    }
    *gave_up_lds = gave_up;
  }
  __syncthreads();
  __threadfence();
  return *gave_up_lds != 0;
}

// Sweeps sweep0 .. sweep0 + nsw - 1 of the block Jacobi in one launch of
// P/2 workgroups: per sweep, the within-block phase (workgroup g runs blocks
// 2g and 2g + 1, four lane groups each, as the circle kernel with W = 4),
// then the P - 1 rounds of the round-robin (as the cross kernel), with a
// grid barrier after every phase.  The rotations, their order and the
// counts are those of the one-launch-per-phase form, so the results are
// bitwise the same.  A sweep starts only when the previous one rotated.
template <int RPL, int GS, int BC>
__global__ __launch_bounds__(BC * GS) void jacobi_fused_kernel(zc* __restrict__ B, int m, int k, int P, int sweep0,
                                                               int nsw, int* __restrict__ rot, double tol,
                                                               const double* __restrict__ fro2, int* __restrict__ bar,
                                                               long limit) {
  extern __shared__ double2 xch[];
  __shared__ int wg_rot, prev_rot, gave_up;
  constexpr int W = BC / 2;  // lane groups per block in the within-block phase
  constexpr int NP = 2 * W - 1;
  constexpr int XCC = RPL < JB_XCHUNK ? RPL : JB_XCHUNK;
  constexpr int LDC = GS * XCC;
  constexpr int XC = cross_chunk(RPL, GS);
  constexpr int LD = GS * XC;
  const int w = threadIdx.x / GS, lane = threadIdx.x % GS;
  const double abs2 = 1e-30 * fro2[0];  // (1e-15 |B|_F)^2
  const int nwg = gridDim.x;
  int arrivals = 0;
  for (int s = sweep0; s < sweep0 + nsw; ++s) {
    if (s > 0) {
      if (threadIdx.x == 0) prev_rot = __hip_atomic_load(&rot[s - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      if (prev_rot == 0) return;
    }
    {  // within-block phase
      const int wl = w % W;
      const int c0 = (2 * (int)blockIdx.x + w / W) * BC;
      const int ct = c0 + wl, cb = c0 + 2 * W - 1 - wl;
      zc xt[RPL], xb[RPL];
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        const int row = lane + GS * j;
        xt[j] = (ct < k && row < m) ? B[row + (long)m * ct] : make_double2(0.0, 0.0);
        xb[j] = (cb < k && row < m) ? B[row + (long)m * cb] : make_double2(0.0, 0.0);
      }
      zc* mine = xch + (long)LDC * w;
      int nrot = 0;
      for (int r = 0; r < NP; ++r) {
        const int pt = (wl == 0) ? 0 : ((wl - 1 - r) % NP + NP) % NP + 1;
        const int pb = ((2 * W - 2 - wl - r) % NP + NP) % NP + 1;
        if (c0 + pt < k && c0 + pb < k) nrot += jacobi_rotate<RPL, GS>(xt, xb, tol, abs2);
#pragma unroll
        for (int c = 0; c < RPL; c += XCC) {
          __syncthreads();
#pragma unroll
          for (int j = 0; j < XCC; ++j)
            if (c + j < RPL) mine[lane + GS * j] = xb[c + j];
          __syncthreads();
          if (wl <= W - 2) {
            const zc* src = mine + LDC;
#pragma unroll
            for (int j = 0; j < XCC; ++j)
              if (c + j < RPL) xb[c + j] = src[lane + GS * j];
          } else {
#pragma unroll
            for (int j = 0; j < XCC; ++j)
              if (c + j < RPL) xb[c + j] = xt[c + j];
          }
          __syncthreads();
          if (wl >= 1 && wl <= W - 2) {
#pragma unroll
            for (int j = 0; j < XCC; ++j)
              if (c + j < RPL) mine[lane + GS * j] = xt[c + j];
          }
          __syncthreads();
          if (wl >= 1) {
            const zc* src = mine - LDC;
#pragma unroll
            for (int j = 0; j < XCC; ++j)
              if (c + j < RPL) xt[c + j] = src[lane + GS * j];
          }
        }
      }
      jacobi_count(nrot, &wg_rot, rot, s);
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        const int row = lane + GS * j;
        if (row < m) {
          if (ct < k) B[row + (long)m * ct] = xt[j];
          if (cb < k) B[row + (long)m * cb] = xb[j];
        }
      }
    }
    arrivals += nwg;
    if (fused_barrier(bar, arrivals, limit, &gave_up)) return;
    for (int round = 0; round < P - 1; ++round) {
      int ba, bb;
      rr_pair(P, round, blockIdx.x, ba, bb);
      const int ca = ba * BC + w;
      zc xa[RPL], xb[RPL];
      {
        const int cb = bb * BC + w;
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          const int row = lane + GS * j;
          xa[j] = (ca < k && row < m) ? B[row + (long)m * ca] : make_double2(0.0, 0.0);
          xb[j] = (cb < k && row < m) ? B[row + (long)m * cb] : make_double2(0.0, 0.0);
        }
      }
      zc* mine = xch + (long)LD * w;
      const zc* next = xch + (long)LD * ((w + 1) % BC);
      int nrot = 0, set = 0;
      for (int st = 0; st < BC; ++st) {
        const int cb = bb * BC + (w + st) % BC;
        if (ca < k && cb < k) nrot += jacobi_rotate<RPL, GS>(xa, xb, tol, abs2);
        if (st == BC - 1) break;
#pragma unroll
        for (int c = 0; c < RPL; c += XC) {
          const long off = set ? (long)LD * BC : 0;
          set ^= 1;
#pragma unroll
          for (int j = 0; j < XC; ++j)
            if (c + j < RPL) mine[off + lane + GS * j] = xb[c + j];
          __syncthreads();
#pragma unroll
          for (int j = 0; j < XC; ++j)
            if (c + j < RPL) xb[c + j] = next[off + lane + GS * j];
        }
      }
      jacobi_count(nrot, &wg_rot, rot, s);
      {
        const int cb = bb * BC + (w + BC - 1) % BC;
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          const int row = lane + GS * j;
          if (row < m) {
            if (ca < k) B[row + (long)m * ca] = xa[j];
            if (cb < k) B[row + (long)m * cb] = xb[j];
          }
        }
      }
      arrivals += nwg;
      if (fused_barrier(bar, arrivals, limit, &gave_up)) return;
    }
  }
}

template <int RPL, int GS>
void jacobi_launch_rpl(tt_ctx* ctx, int kind, int m, int k, zc* B, int P, int round, int inner_max, int sweep,
                       int* rot, double tol, const double* fro2) {
  const size_t slot = sizeof(zc) * GS * (RPL < JB_XCHUNK ? RPL : JB_XCHUNK);
  // algorithmic work: a column pair that meets costs 16 m flops for its
  // three inner products and 24 m for the rotation (counted as applied);
  // bytes: the columns read and written once
  const double pair = 40.0 * m;
  double pairs, cols;
  if (kind == 0) {
    pairs = 0.5 * k * (k - 1) * inner_max;
    cols = k;
  } else if (kind == 1) {
    pairs = 0.5 * JB_COLS * (JB_COLS - 1) * ((k + JB_COLS - 1) / JB_COLS);
    cols = k;
  } else {
    pairs = (double)JB_COLS * JB_COLS * (P / 2);
    cols = 2.0 * JB_COLS * (P / 2);
  }
  if (kind == 4) {  // inner_max sweeps from `sweep` in one launch
    if constexpr (RPL * GS > JB_FUSED_MAXM) {
      fail(TT_EINVAL, "jacobi_svd: the fused form takes at most 640 rows");
    } else {
    constexpr int XCC = RPL < JB_XCHUNK ? RPL : JB_XCHUNK;
    const size_t lds = std::max(sizeof(zc) * JB_COLS * GS * XCC, 2 * JB_COLS * sizeof(zc) * GS * cross_chunk(RPL, GS));
    const double sweep_pairs = 0.5 * (double)k * (k - 1.0);
    KTimer kf(ctx, "jacobi_fused", pair * sweep_pairs * inner_max, 2.0 * 16.0 * m * (double)k * P * inner_max, true);
    TTF_LAUNCH(kf, (jacobi_fused_kernel<RPL, GS, JB_COLS>), dim3(P / 2), dim3(JB_COLS * GS), lds, ctx->stream, B, m,
               k, P, sweep, inner_max, rot, tol, fro2, rot + JB_BAR, ctx->jacobi_wait_limit);
    TTF_HIP(hipGetLastError());
    }
    return;
  }
  if (kind == 3) {  // the all-pairs convergence test (P = number of blocks, inner_max = label)
    const int nb = P;
    KTimer kc(ctx, "jacobi_check", 16.0 * m * 0.5 * k * (k - 1.0), 16.0 * m * k * (nb + 1.0), true);
    TTF_LAUNCH(kc, (jacobi_check_kernel<RPL, GS, JB_COLS>), dim3(nb * (nb + 1) / 2), dim3(JB_COLS * GS),
               2 * JB_COLS * sizeof(zc) * GS * cross_chunk(RPL, GS), ctx->stream, B, m, k, tol, fro2, rot + JB_MAXS,
               inner_max);
    TTF_HIP(hipGetLastError());
    return;
  }
  KTimer kt(ctx, kind == 2 ? "jacobi_cross" : "jacobi_circle", pair * pairs, 2.0 * 16.0 * m * cols, true);
  if (kind == 0) {  // whole matrix (k <= 32, at most 320 rows) in one workgroup
    if constexpr (GS == 32)
      TTF_LAUNCH(kt, (jacobi_circle_kernel<RPL, 16, GS>), dim3(1), dim3(16 * GS), 16 * slot, ctx->stream, B, m, k,
                 inner_max, sweep, rot, tol, fro2);
    else
      fail(TT_EINVAL, "jacobi_svd: single-workgroup form needs at most 320 rows");
  } else if (kind == 1)  // every block of JB_COLS columns on its own
    TTF_LAUNCH(kt, (jacobi_circle_kernel<RPL, JB_COLS / 2, GS>), dim3((k + JB_COLS - 1) / JB_COLS),
               dim3(JB_COLS / 2 * GS), JB_COLS / 2 * slot, ctx->stream, B, m, k, 1, sweep, rot, tol, fro2);
  else
    TTF_LAUNCH(kt, (jacobi_cross_kernel<RPL, GS, JB_COLS>), dim3(P / 2), dim3(JB_COLS * GS),
               2 * JB_COLS * sizeof(zc) * GS * cross_chunk(RPL, GS),
               ctx->stream, B, m, k, P, round, sweep, rot, tol, fro2);
  TTF_HIP(hipGetLastError());
}

// Blocks of JB_COLS columns; one sweep = every block on its own (all pairs
// inside a block) followed by the P - 1 rounds of a round-robin over the
// blocks (all pairs between two blocks), so each column pair meets once.
// rot_ext: caller-provided counters (JB_ROT_BYTES of device memory); the
// run then allocates nothing and records nothing in the context
void jacobi_blocked(tt_ctx* ctx, int m, int k, zc* B, zc* U, double* sigma, int* sweeps, int* rot_ext) {
  // rot[0 .. JB_MAXS): rotations per sweep; rot[JB_MAXS]: the last
  // orthogonality check that failed; then |B|_F^2 (8-byte aligned)
  int* rot = rot_ext ? rot_ext : (int*)ctx->get_ws("jac_rot", JB_ROT_BYTES);
  double* fro2 = (double*)(rot + JB_MAXS + 2);
  frob_norm2(ctx, B, (long)m * k, fro2);
  // a 32-lane group per column pair up to 320 rows (at most 10 rows per
  // lane), a whole wavefront beyond (up to 16 rows per lane)
  auto launch = [&](int kind, int P, int round, int inner_max, int sweep, int* rot, double tol) {
    const double* f2 = fro2;
    if (m <= 64)
      jacobi_launch_rpl<2, 32>(ctx, kind, m, k, B, P, round, inner_max, sweep, rot, tol, f2);
    else if (m <= 128)
      jacobi_launch_rpl<4, 32>(ctx, kind, m, k, B, P, round, inner_max, sweep, rot, tol, f2);
    else if (m <= 192)
      jacobi_launch_rpl<6, 32>(ctx, kind, m, k, B, P, round, inner_max, sweep, rot, tol, f2);
    else if (m <= 256)
      jacobi_launch_rpl<8, 32>(ctx, kind, m, k, B, P, round, inner_max, sweep, rot, tol, f2);
    else if (m <= 320)
      jacobi_launch_rpl<10, 32>(ctx, kind, m, k, B, P, round, inner_max, sweep, rot, tol, f2);
    else if (m <= 512)
      jacobi_launch_rpl<8, 64>(ctx, kind, m, k, B, P, round, inner_max, sweep, rot, tol, f2);
    else if (m <= 640)
      jacobi_launch_rpl<10, 64>(ctx, kind, m, k, B, P, round, inner_max, sweep, rot, tol, f2);
    else if (m <= 1024)
      jacobi_launch_rpl<16, 64>(ctx, kind, m, k, B, P, round, inner_max, sweep, rot, tol, f2);
    else
      jacobi_launch_rpl<24, 64>(ctx, kind, m, k, B, P, round, inner_max, sweep, rot, tol, f2);
  };
  const double tol = 1e-15 * sqrt((double)m);
  const int nblk = (k + JB_COLS - 1) / JB_COLS;
  const int P = nblk + (nblk & 1);
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, ctx->stream, rot, JB_MAXS + 1);
  TTF_HIP(hipGetLastError());
  int nsweeps = 0, checked = 0;
  const int max_sweeps = std::max(1, std::min(JAC_MAX_SWEEPS, ctx->jacobi_max_sweeps));
  if (k <= 32 && m <= 320) {
    launch(0, 2, 0, max_sweeps, 0, rot, tol);
    nsweeps = max_sweeps;
  } else {
    // Sweeps are launched in batches between host checks.  After a batch
    // one launch applies the rotation test to every column pair at once
    // (the same sums a sweep computes): when no pair would be rotated, the
    // next sweep would rotate nothing, and the iteration ends without it.
    // A sweep without rotations also ends the iteration.  A sweep launched
    // after convergence returns at once but still costs its launches, so
    // the first batch is as long as the last SVD of this size needed (5 for
    // a new size), the later ones one sweep.  The launched count does not
    // change the result.
    int hbuf[JB_BAR + 2];
    int* h = rot_ext ? hbuf : (int*)ctx->host_scratch(sizeof(int) * (JB_BAR + 2));
    const bool fused = ctx->jacobi_fused && P / 2 <= JB_FUSED_MAX_WG && m <= JB_FUSED_MAXM;
    auto seen = ctx->jacobi_sweeps_seen.find({m, k});
    const bool known = seen != ctx->jacobi_sweeps_seen.end();
    int batch = known ? std::max(1, seen->second) : 5;
    bool done = false;
    int converged = 0, rotating = 0;  // sweeps until converged; of them with rotations
    while (!done && nsweeps < max_sweeps) {
      if (fused) {
        const int nsw = std::min(batch, max_sweeps - nsweeps);
        hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, ctx->stream, rot + JB_BAR, 2);
        TTF_HIP(hipGetLastError());
        launch(4, P, 0, nsw, nsweeps, rot, tol);
        nsweeps += nsw;
      } else {
        for (int b = 0; b < batch && nsweeps < max_sweeps; ++b, ++nsweeps) {
          launch(1, P, 0, 1, nsweeps, rot, tol);
          for (int r = 0; r < P - 1; ++r) launch(2, P, r, 1, nsweeps, rot, tol);
        }
      }
      launch(3, nblk, 0, nsweeps, 0, rot, tol);  // the test labelled nsweeps
      checked = 1;
      TTF_HIP(hipMemcpyAsync(h, rot, sizeof(int) * (JB_BAR + 2), hipMemcpyDeviceToHost, ctx->stream));
      TTF_HIP(hipStreamSynchronize(ctx->stream));
      if (fused && h[JB_BAR + 1] != 0)
        fail(TT_ENOCONV, "jacobi_svd: a workgroup of the fused sweeps gave up waiting at a grid barrier");
      for (int s = 0; s < nsweeps && !done; ++s)
        if (h[s] == 0) {
          done = true;
          converged = s + 1;
          rotating = s;
        }
      if (!done && h[JB_MAXS] < nsweeps) {
        done = true;
        converged = rotating = nsweeps;
        ctx->jacobi_check_passed += 1;
      }
      batch = 1;
    }
    // the next SVD of this size starts with as many sweeps as this one
    // rotated in: after them the test would have ended this one
    if (done && !rot_ext) ctx->jacobi_sweeps_seen[{m, k}] = std::max(1, rotating);
    ctx->jacobi_svds += 1;
    ctx->jacobi_sweeps_launched += nsweeps;
    ctx->jacobi_sweeps_needed += converged;
  }
  hipLaunchKernelGGL(jacobi_finish_kernel, dim3(1), dim3(1024), 0, ctx->stream, m, k, B, U, sigma, rot, nsweeps,
                     checked, sweeps);
  TTF_HIP(hipGetLastError());
}

// ------------------------------------------------------------- helpers
__global__ void set_identity_kernel(zc* A, int m, int k, long lda) {
  const long total = (long)m * k;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int r = (int)(e % m), c = (int)(e / m);
    A[r + lda * c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
}

void set_identity(tt_ctx* ctx, zc* A, int m, int k, long lda) {
  const long total = (long)m * k;
  if (total <= 0) return;
  const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(set_identity_kernel, dim3(blocks), dim3(256), 0, ctx->stream, A, m, k, lda);
  TTF_HIP(hipGetLastError());
}

__global__ void copy_matrix_kernel(const zc* src, long lds_, zc* dst, long ldd, int m, int k) {
  const long total = (long)m * k;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int r = (int)(e % m), c = (int)(e / m);
    dst[r + ldd * c] = src[r + lds_ * c];
  }
}

void copy_matrix(tt_ctx* ctx, const zc* src, long lds_, zc* dst, long ldd, int m, int k) {
  const long total = (long)m * k;
  if (total <= 0) return;
  const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(copy_matrix_kernel, dim3(blocks), dim3(256), 0, ctx->stream, src, lds_, dst, ldd, m, k);
  TTF_HIP(hipGetLastError());
}

__global__ __launch_bounds__(1024) void frob_norm2_kernel(const zc* x, long n, double* out) {
  __shared__ double red[16];
  double s = 0;
  for (long e = threadIdx.x; e < n; e += blockDim.x) s += x[e].x * x[e].x + x[e].y * x[e].y;
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = s;
}

void frob_norm2(tt_ctx* ctx, const zc* x, long n, double* out_dev) {
  hipLaunchKernelGGL(frob_norm2_kernel, dim3(1), dim3(1024), 0, ctx->stream, x, n, out_dev);
  TTF_HIP(hipGetLastError());
}

}  // namespace ttf
