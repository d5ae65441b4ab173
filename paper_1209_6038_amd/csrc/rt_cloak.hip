// rt_cloak.hip -- kernels and C ABI of the cloak ray tracer (gfx950).
//
// Pipeline of one call (all launches on the caller's stream):
//   1. entry kernel   vacuum ray -> cloak intersection -> Sect. 3 refraction;
//                     rays that miss (or reflect at the entry) are finished
//                     here, rays that enter get a slot in the work table,
//                     grouped by branch, with a difficulty key
//   2. sort           counting sort of the slots, hardest rays first
//   3. integrator     persistent kernel: one ray per lane, FP64 state in
//                     registers, refilled from the queue in wave-private
//                     chunks every `refill_period` steps; boundary crossings,
//                     exit refraction, total internal reflection and the
//                     inner metal mirror are handled in line (k_transit)
//   4. finish kernel  vacuum leg to r_out (trace) or to the room (render)
//   5. resolve        (render) per-pixel mean of the sample colours
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/rt.h"
#include "device.h"
#include "internal.h"

using namespace rtk;

struct rt_cloak_s {
  rt_cloak_desc d;
};

struct rt_plan_s;

namespace {

// segments of the work table: one per (cloak, branch) of a call, each of
// `cap` slots; the integrator's waves stay on one segment at a time
constexpr int NSEG = 4;

// counters in device memory
enum {
  // the per-segment counters sit on separate 128-byte lines: the atomics of
  // different segments then go to different L2 channels instead of
  // serializing on one line
  C_LINE = 32,
  C_NBASE = 0,               // C_N(s): slots used in segment s
  C_FBASE = NSEG * C_LINE,   // C_FETCH(s): integrator work counter of segment s
  C_SUR = 2 * NSEG * C_LINE,        // surrogate render: side entries offered to the network
  C_ACC = C_SUR + C_LINE,            // surrogate render: entries whose prediction was accepted
  C_COUNT = C_ACC + C_LINE
};
constexpr int MAX_BOUNCES = 64;
constexpr long long REFL_CHUNK = 1LL << 22;  // samples per chunk with first-order reflections
constexpr unsigned int FETCH_CHUNK = 64;  // rays claimed per wave per atomic
constexpr int LONG_RAY_ATTEMPTS = 64;      // see the issue priority in k_transit
constexpr int NBUCKET = 16;               // difficulty buckets
constexpr int NBIN = NBUCKET * NSEG;       // sort keys: (segment, difficulty bucket)
// the counting sort runs a fixed grid; each block owns one contiguous range of
// the queue, and the table keeps one count (then one offset) per (key, block)
constexpr int SORT_BLOCKS = 1024;
constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 8;              // keys per thread per tile
static_assert(NBIN <= SORT_THREADS, "the scatter gives one thread to each key");
__host__ __device__ constexpr int C_N(int s) { return C_NBASE + s * C_LINE; }
__host__ __device__ constexpr int C_FETCH(int s) { return C_FBASE + s * C_LINE; }

struct Table {
  double *px, *py, *pz, *vx, *vy, *vz;
  double *t, *opl0, *hres;  // t and hres, like nsteps, bounces and status, are written when the ray stops
  double *wt;  // Eq. (12) weight carried along the ray (rt_trace_batch with trans)
  int *nsteps, *bounces, *status, *kind;
  long long *key;
  int *order;   // integrator queue: slots sorted hardest first
  int *key0;    // sort key of each slot
  unsigned int *ctr;
  unsigned int *bh;  // sort: NBIN x SORT_BLOCKS counts, key-major, then their offsets
  long long cap;  // capacity of one segment; segment s starts at s * cap
};

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long lanemask_lt() {
  unsigned int lane = __lane_id();
  return lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
}

// Block-aggregated append: this thread's index in the counter's range
// (valid where `want`), with one global atomic per block instead of one per
// wave. Every thread of the block must call it (it synchronizes); `sh` is
// block-shared scratch of at least 2 * (blockDim.x / 64) + 1 words.
__device__ __forceinline__ unsigned int block_append(unsigned int *counter, bool want, unsigned int *sh) {
  const unsigned long long m = __ballot(want);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (__lane_id() == 0) sh[w] = (unsigned int)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int tot = 0;
    for (int k = 0; k < nw; ++k) { sh[nw + k] = tot; tot += sh[k]; }
    sh[2 * nw] = tot ? atomicAdd(counter, tot) : 0u;
  }
  __syncthreads();
  const unsigned int idx = sh[2 * nw] + sh[nw + w] + (unsigned int)__popcll(m & lanemask_lt());
  __syncthreads();  // scratch free for the next call
  return idx;
}

__device__ __forceinline__ bool finite6(const double x[3], const double v[3]) {
  return isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) && isfinite(v[0]) &&
         isfinite(v[1]) && isfinite(v[2]);
}

// queue position -> (segment, slot) over the concatenation of the used
// parts of the segments
struct SegMap {
  unsigned int off[NSEG + 1];
};

__device__ __forceinline__ SegMap seg_map(const Table &T) {
  SegMap m;
  m.off[0] = 0;
#pragma unroll
  for (int q = 0; q < NSEG; ++q) m.off[q + 1] = m.off[q] + T.ctr[C_N(q)];
  return m;
}

__device__ __forceinline__ int seg_of(const SegMap &m, unsigned int idx) {
  int q = 0;
#pragma unroll
  for (int k = 1; k < NSEG; ++k) q += idx >= m.off[k] ? 1 : 0;
  return q;
}

// m.off[q] for a run-time q without dynamic indexing (keeps SegMap in registers)
__device__ __forceinline__ unsigned int off_of(const SegMap &m, int q) {
  unsigned int r = 0;
#pragma unroll
  for (int k = 0; k <= NSEG; ++k) r = (k == q) ? m.off[k] : r;
  return r;
}

__device__ __forceinline__ int slot_at(const Table &T, const SegMap &m, unsigned int idx, int &seg) {
  seg = seg_of(m, idx);
  return (int)(seg * T.cap + (idx - off_of(m, seg)));
}

// Sort key of an entering ray: rays whose conserved angular momentum p_theta
// (and axial wave number p_z, for the branches whose metric is singular in
// both) is small pass close to r = a, where the adaptive step shrinks; they
// take the most steps and are integrated first so that a launch ends on
// short rays. key = NBUCKET-1 - bucket with bucket = -log2(p).
__device__ __forceinline__ int sort_key(const CloakP &c, int kind, const double x[3],
                                        const double d[3]) {
  int bucket = 0;
  if (kind != K_RO) {
    double pth = fabs(x[0] * d[1] - x[1] * d[0]) / c.b;
    double p = kind == K_AE ? pth : sqrt(fma(pth, pth, d[2] * d[2]));
    int e = 0;
    (void)frexp(p, &e);  // p = f 2^e, f in [0.5, 1)
    bucket = min(max(1 - e, 0), NBUCKET - 1);
  }
  return NBUCKET - 1 - bucket;
}

__device__ __forceinline__ void load_state(const Table &T, int s, double x[3], double v[3]) {
  x[0] = T.px[s]; x[1] = T.py[s]; x[2] = T.pz[s];
  v[0] = T.vx[s]; v[1] = T.vy[s]; v[2] = T.vz[s];
}

__device__ __forceinline__ void store_state(const Table &T, int s, const double x[3],
                                            const double v[3]) {
  T.px[s] = x[0]; T.py[s] = x[1]; T.pz[s] = x[2];
  T.vx[s] = v[0]; T.vy[s] = v[1]; T.vz[s] = v[2];
}

// a new slot: entry state, sort key, vacuum path so far, branch and output
// index. The integrator starts every slot with t = 0, step h0, no steps and
// no bounces, and writes the rest when the ray stops.
__device__ __forceinline__ void put_slot(const Table &T, int s, const double x[3], const double v[3],
                                         int kind, long long key, double opl0, int skey) {
  store_state(T, s, x, v);
  T.key0[s] = skey;
  T.opl0[s] = opl0;
  T.kind[s] = kind;
  T.key[s] = key;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ void k_zero(unsigned int *p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// rt_trace_batch entry: one thread per input ray
__global__ void __launch_bounds__(256) k_tb_entry(CloakP c, OptsP o, Table T, int kind, long long n,
                                                  const double *__restrict__ in6,
                                                  double *__restrict__ out6, double *__restrict__ opl,
                                                  int *__restrict__ status, double *__restrict__ hres,
                                                  int *__restrict__ nsteps, double *__restrict__ trans) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  bool enter = false, disk = false;
  double x[3], v[3], s = 0.0, w_in = 0.0;
  int skey = 0;
  if (i < n) {
    double org[3], d[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) { org[j] = in6[j * n + i]; d[j] = in6[(3 + j) * n + i]; }
    double dl = sqrt(fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2])));
    bool ok = isfinite(org[0]) && isfinite(org[1]) && isfinite(org[2]) && isfinite(dl) && dl > 0.0;
    if (ok) {
#pragma unroll
      for (int j = 0; j < 3; ++j) d[j] /= dl;
      double r2 = fma(org[0], org[0], org[1] * org[1]);
      ok = !(r2 < c.b2 && org[2] > c.z0 && org[2] < c.z1);
    }
    int st = RT_RAY_INVALID;
    double p[3] = {org[0], org[1], org[2]}, L = 0.0;
    if (ok) {
      int surf;
      st = RT_RAY_MISSED;
      if (vacuum_entry(c, org, d, s, surf)) {
#pragma unroll
        for (int j = 0; j < 3; ++j) x[j] = fma(s, d[j], org[j]);
        if (surf == B_TOP) x[2] = c.z1;
        if (surf == B_BOTTOM) x[2] = c.z0;
        double r2 = fma(x[0], x[0], x[1] * x[1]);
        double nrm[3];
        boundary_normal(surf, x, nrm);
        if (surf != B_SIDE && r2 <= c.a2) {
          p[0] = x[0]; p[1] = x[1]; p[2] = x[2];
          L = s;
          if (c.mirror) { reflect3(d, nrm); st = RT_RAY_REFLECTED; disk = true; }
          else st = RT_RAY_ABSORBED;
        } else if (refract_in(c, kind, surf, x, d, v)) {
          enter = true;
          skey = sort_key(c, kind, x, d);
          if (trans) {
            double eo, ee, cax[3];
            material_axis(c, kind >> 1, x, eo, ee, cax);
            w_in = fresnel_in_dev(eo, ee, cax, nrm, d, kind & 1);
          }
        } else {
          p[0] = x[0]; p[1] = x[1]; p[2] = x[2];
          L = s;
          reflect3(d, nrm);
          st = RT_RAY_REFLECTED;
        }
      }
      if (!enter && st != RT_RAY_ABSORBED) {
        double sl = leave_radius(p, d, o.r_out);
#pragma unroll
        for (int j = 0; j < 3; ++j) p[j] = fma(sl, d[j], p[j]);
        L += sl;
      }
    }
    if (!enter) {
#pragma unroll
      for (int j = 0; j < 3; ++j) { out6[j * n + i] = p[j]; out6[(3 + j) * n + i] = d[j]; }
      opl[i] = L;
      status[i] = st;
      if (hres) hres[i] = __builtin_nan("");
      if (nsteps) nsteps[i] = 0;
      // a miss keeps all of its light, and so does a reflection off the
      // perfect metal end disk
      if (trans) trans[i] = (st == RT_RAY_MISSED || disk) ? 1.0 : 0.0;
    }
  }
  __shared__ unsigned int sh[16];
  unsigned int sl = block_append(T.ctr + C_N(0), enter, sh);
  if (enter) {
    put_slot(T, (int)sl, x, v, kind, i, s, skey);
    if (trans) T.wt[sl] = w_in;
  }
}

// Counting sort of the entered slots by key, stable in queue order. The
// queue is cut into SORT_BLOCKS contiguous ranges, one per block of the
// histogram and scatter passes (both launched with SORT_BLOCKS x
// SORT_THREADS), so no pass needs a global atomic.

// queue range [lo, hi) of sort block b
__device__ __forceinline__ void sort_range(unsigned int n, unsigned int b, unsigned int &lo, unsigned int &hi) {
  const unsigned int chunk = (n + SORT_BLOCKS - 1) / SORT_BLOCKS;
  lo = min(n, b * chunk);
  hi = min(n, lo + chunk);
}

// lanes of the wave whose key equals this lane's (0 where !active); every
// lane of the wave must call it
__device__ __forceinline__ unsigned long long same_key_lanes(int key, bool active) {
  unsigned long long left = __ballot(active), mine = 0;
  while (left) {
    const int k = __shfl(key, __ffsll((long long)left) - 1);
    const unsigned long long m = __ballot(active && key == k);
    if (active && key == k) mine = m;
    left &= ~m;
  }
  return mine;
}

// pass 1: the block's count of each key, into bh[key * SORT_BLOCKS + block]
__global__ void __launch_bounds__(SORT_THREADS) k_sort_hist(Table T) {
  __shared__ unsigned int lh[NBIN];
  for (int i = threadIdx.x; i < NBIN; i += blockDim.x) lh[i] = 0;
  __syncthreads();
  const SegMap m = seg_map(T);
  unsigned int lo, hi;
  sort_range(m.off[NSEG], blockIdx.x, lo, hi);
  for (unsigned int base = lo; base < hi; base += SORT_ITEMS * SORT_THREADS) {
    int key[SORT_ITEMS];
    bool active[SORT_ITEMS];
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; ++j) {
      const unsigned int idx = base + j * SORT_THREADS + threadIdx.x;
      active[j] = idx < hi;
      key[j] = 0;
      if (active[j]) {
        int seg;
        const int slot = slot_at(T, m, idx, seg);
        key[j] = seg * NBUCKET + T.key0[slot];
      }
    }
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; ++j) {
      const unsigned long long same = same_key_lanes(key[j], active[j]);
      if (active[j] && (same & lanemask_lt()) == 0) atomicAdd(&lh[key[j]], (unsigned int)__popcll(same));
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NBIN; i += blockDim.x) T.bh[i * SORT_BLOCKS + blockIdx.x] = lh[i];
}

// pass 2: exclusive scan of bh in place by one block of SORT_THREADS threads,
// each summing a run of E consecutive entries. A small block: it starts on a
// CU that integrator waves of another stream still occupy, instead of waiting
// for a whole CU to drain.
__global__ void __launch_bounds__(SORT_THREADS) k_sort_scan(Table T) {
  constexpr int E = NBIN * SORT_BLOCKS / SORT_THREADS, NW = SORT_THREADS / 64;
  static_assert(E % 4 == 0, "runs are read as uint4");
  __shared__ unsigned int ws[NW];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  uint4 *p = (uint4 *)(T.bh + t * E);  // the table is 256-byte aligned
  unsigned int sum = 0;
#pragma unroll 8
  for (int i = 0; i < E / 4; ++i) { const uint4 c = p[i]; sum += c.x + c.y + c.z + c.w; }
  // inclusive scan of the 64 lane sums, then across the waves
  unsigned int inc = sum;
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned int u = __shfl_up(inc, d);
    if (lane >= d) inc += u;
  }
  if (lane == 63) ws[w] = inc;
  __syncthreads();
  if (t == 0) {
    unsigned int acc = 0;
    for (int k = 0; k < NW; ++k) { const unsigned int c = ws[k]; ws[k] = acc; acc += c; }
  }
  __syncthreads();
  unsigned int acc = ws[w] + inc - sum;
#pragma unroll 8
  for (int i = 0; i < E / 4; ++i) {
    const uint4 c = p[i];
    uint4 o;
    o.x = acc; acc += c.x;
    o.y = acc; acc += c.y;
    o.z = acc; acc += c.z;
    o.w = acc; acc += c.w;
    p[i] = o;
  }
}

// pass 3: place the block's range tile by tile. The keys of one tile are
// ranked among equal keys of their wave with ballots; a per-key scan over the
// tile's (item, wave) groups, added to the block's running offset of the
// key, orders the groups. Every slot lands after the slots of its key that
// precede it in the queue.
__global__ void __launch_bounds__(SORT_THREADS) k_sort_scatter(Table T) {
  constexpr int NW = SORT_THREADS / 64, NG = SORT_ITEMS * NW;
  __shared__ unsigned int run[NBIN];
  __shared__ unsigned int gc[NG * NBIN];  // per (group, key): count, then offset
  const SegMap m = seg_map(T);
  unsigned int lo, hi;
  sort_range(m.off[NSEG], blockIdx.x, lo, hi);
  for (int i = threadIdx.x; i < NBIN; i += blockDim.x) run[i] = T.bh[i * SORT_BLOCKS + blockIdx.x];
  const int w = threadIdx.x >> 6;
  const unsigned long long lt = lanemask_lt();
  for (unsigned int base = lo; base < hi; base += SORT_ITEMS * SORT_THREADS) {
    for (int i = threadIdx.x; i < NG * NBIN; i += blockDim.x) gc[i] = 0;
    int key[SORT_ITEMS], slot[SORT_ITEMS];
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; ++j) {
      const unsigned int idx = base + j * SORT_THREADS + threadIdx.x;
      slot[j] = -1;
      key[j] = 0;
      if (idx < hi) {
        int seg;
        slot[j] = slot_at(T, m, idx, seg);
        key[j] = seg * NBUCKET + T.key0[slot[j]];
      }
    }
    __syncthreads();  // gc cleared (and the previous tile's reads done)
    unsigned int rank[SORT_ITEMS];
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; ++j) {
      const bool active = slot[j] >= 0;
      const unsigned long long same = same_key_lanes(key[j], active);
      rank[j] = (unsigned int)__popcll(same & lt);
      if (active && rank[j] == 0) gc[(j * NW + w) * NBIN + key[j]] = (unsigned int)__popcll(same);
    }
    __syncthreads();
    if (threadIdx.x < NBIN) {
      unsigned int acc = run[threadIdx.x];
      for (int g = 0; g < NG; ++g) {
        const unsigned int c = gc[g * NBIN + threadIdx.x];
        gc[g * NBIN + threadIdx.x] = acc;
        acc += c;
      }
      run[threadIdx.x] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; ++j)
      if (slot[j] >= 0) T.order[gc[(j * NW + w) * NBIN + key[j]] + rank[j]] = slot[j];
    __syncthreads();  // gc read before the next tile clears it
  }
}

// integrator state of one lane (lives in registers)
struct Lane {
  double x[3], v[3], A1[3];  // base state and its acceleration
  double h, t;               // next step length, optical path so far
  double lo, hi, ht;         // boundary search: bracket and trial length
  int ns, bounces, rid, riter;
  bool after_reject;
  double wt;  // Eq. (12) weight (FRES only)
};

// One iteration of a lane of branch KIND: one attempt of the scheme from the
// base state, then either the step controller (stepping) or one safeguarded
// Newton update of the crossing length (rid >= 0: locating the crossing of
// boundary rid). Returns the final status when the ray stops, else -1.
// Eq. (12) at an interface event of branch KIND: the wave k = M v meets
// boundary rid at x; transmitted fraction (.x) and same-type reflected
// fraction (.y). Kept out of line, with scalar arguments: the events are rare
// and their complex arithmetic would otherwise set the register allocation
// of the whole integration loop.
template <int KIND>
__device__ __noinline__ double2 fresnel_event(double kappa, double a, int rid, double x0, double x1,
                                              double x2, double v0, double v1, double v2) {
  CloakP c{};
  c.kappa = kappa;
  c.a = a;
  const double x[3] = {x0, x1, x2};
  double eo, ee, cax[3], nrm[3], k[3];
  material_axis(c, KIND >> 1, x, eo, ee, cax);
  boundary_normal(rid, x, nrm);
  double rh[2], th[2], w;
  local_frame(x, rh, th, w);
  double mr, mt, mz;
  metric_diag(KIND, kappa, a, w, mr, mt, mz);
  const double vr = v0 * rh[0] + v1 * rh[1], vt = v0 * th[0] + v1 * th[1];
  k[0] = mr * vr * rh[0] + mt * vt * th[0];
  k[1] = mr * vr * rh[1] + mt * vt * th[1];
  k[2] = mz * v2;
  double Tt, Rr;
  fresnel_out_dev(eo, ee, cax, nrm, k, KIND & 1, Tt, Rr);
  return make_double2(Tt, Rr);
}

template <int KIND, bool HAM, bool FRES>
__device__ __forceinline__ int iterate(Lane &L, const CloakP &c, const OptsP &o,
                                       double tol, double &hr) {
  if (L.rid < 0 && L.ns >= o.max_steps) return RT_RAY_MAXSTEPS;
  const double hs = L.rid < 0 ? L.h : L.ht;
  double xn[3], vn[3];
  double A[7][3];
  double sum = 0.0;
  double dts = hs;  // optical path of the attempt: its length but in the Hamiltonian form
  if constexpr (HAM) {
    // state (x, k); the step is in the ray parameter tau of the polynomial
    // or (RT_SCHEME_RK4_HAMC) the canonically normalized Hamiltonian
    if (o.scheme == RT_SCHEME_RK4_HAMC) rk4_ham_step<KIND, true>(c.a, c.kappa, L.x, L.v, hs, xn, vn, dts);
    else rk4_ham_step<KIND, false>(c.a, c.kappa, L.x, L.v, hs, xn, vn, dts);
  } else if (o.scheme == RT_SCHEME_RK4) {
    rk4_step<KIND>(c.a, L.x, L.v, L.A1, hs, xn, vn);
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i) A[0][i] = L.A1[i];
    sum = dp45_attempt<KIND>(c.a, L.x, L.v, A, hs, o.rtol, o.atol, xn, vn);
  }
  if (L.rid < 0) {
    // ---- stepping ----
    ++L.ns;
    if (o.scheme == RT_SCHEME_DP45) {
      if (!(sum <= 6.0)) {
        L.h *= dp45_factor(sum, false);
        L.after_reject = true;
        return (L.h >= 1e-12) ? -1 : RT_RAY_DIVERGED;
      }
      L.h = fmin(L.h * dp45_factor(sum, L.after_reject), o.hmax);
      L.after_reject = false;
    }
    if (!finite6(xn, vn)) return RT_RAY_DIVERGED;
    if (inside_open(c, xn)) {
      if constexpr (KIND == K_RO) {
        // homogeneous medium (Eq. (14): eps_o = kappa): the step is a
        // straight chord, which can dip into r < a and come back out
        // within one step. If its closest approach to the axis lies inside,
        // search the crossing before that point, starting from the chord's
        // first root of |x + tau (xn - x)|_xy = a.
        const double dx = xn[0] - L.x[0], dy = xn[1] - L.x[1];
        const double dd = fma(dx, dx, dy * dy);
        if (dd > 0.0) {
          const double f = -fma(L.x[0], dx, L.x[1] * dy) / dd;
          const double px = fma(f, dx, L.x[0]), py = fma(f, dy, L.x[1]);
          const double pc2 = fma(px, px, py * py);
          if (f > 0.0 && f < 1.0 && pc2 < c.a2) {
            const double tau = f - sqrt((c.a2 - pc2) / dd);
            L.rid = B_INNER;
            L.lo = 0.0;
            L.hi = f * hs;
            L.ht = hs * fmin(fmax(tau, 1e-3 * f), (1.0 - 1e-3) * f);
            L.riter = 0;
            return -1;
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) { L.x[i] = xn[i]; L.v[i] = vn[i]; }
      L.t += dts;
      if constexpr (!HAM) {
        if (o.scheme == RT_SCHEME_RK4) {
          accel<KIND>(c.a, L.x[0], L.x[1], L.v[0], L.v[1], L.v[2], L.A1[0], L.A1[1], L.A1[2]);
        } else {
#pragma unroll
          for (int i = 0; i < 3; ++i) L.A1[i] = A[6][i];
        }
      }
      return -1;
    }
    // the step left the material: search the earliest crossing, starting
    // from the boundary with the smallest linearly interpolated fraction
    // -g0 / (g1 - g0) (compared as num * den' < num' * den, denominators
    // positive; one reciprocal for the winner: the fraction only seeds the
    // search)
    double bn = 2.0, bd = 1.0;
    int rid = B_SIDE;
#pragma unroll
    for (int id = 0; id < 4; ++id) {
      double g1 = gsq(c, id, xn);
      if (g1 >= 0.0) {
        double g0 = fmin(gsq(c, id, L.x), -1e-300);
        double num = -g0, den = g1 - g0;
        if (num * bd < bn * den) { bn = num; bd = den; rid = id; }
      }
    }
    const double best = bn * rcp64_1(bd);
    L.rid = rid;
    L.lo = 0.0;
    L.hi = hs;
    L.ht = hs * fmin(fmax(best, 1e-3), 1.0 - 1e-3);
    L.riter = 0;
    return -1;
  }
  // ---- locating the crossing of boundary rid ----
  if (!finite6(xn, vn)) return RT_RAY_DIVERGED;
  double f = gsq(c, L.rid, xn);
  ++L.riter;
  if (!(fabs(f) <= tol || L.riter >= 100 || !(L.hi - L.lo > 1e-300))) {
    if (f < 0.0) L.lo = L.ht; else L.hi = L.ht;
    double slope;
    if constexpr (HAM) {
      // dg/dtau along dx/dtau at the trial point
      double dx[3], dk[3], dt_;
      if (o.scheme == RT_SCHEME_RK4_HAMC) ham_rhs_canon<KIND>(c.a, c.kappa, xn, vn, dx, dk, dt_);
      else ham_rhs<KIND>(c.a, c.kappa, xn, vn, dx, dk, dt_);
      slope = gsq_slope(c, L.rid, xn, dx);
    } else {
      slope = gsq_slope(c, L.rid, xn, vn);
    }
    double hn = L.ht - f * rcp64_1(slope);
    if (!(hn > L.lo && hn < L.hi)) hn = 0.5 * (L.lo + L.hi);
    L.ht = hn;
    return -1;
  }
  // an earlier crossing of another boundary takes precedence
  int other = -1;
#pragma unroll
  for (int id = 0; id < 4; ++id)
    if (id != L.rid && gsq(c, id, xn) > tol) other = id;
  if (other >= 0) {
    L.rid = other;
    L.lo = 0.0;
    L.hi = L.ht;
    L.ht = 0.5 * L.ht;
    L.riter = 0;
    return -1;
  }
  // the ray is on boundary rid at (xn, vn)
  L.t += dts;
#pragma unroll
  for (int i = 0; i < 3; ++i) { L.x[i] = xn[i]; L.v[i] = vn[i]; }
  if constexpr (HAM) ham_convert<KIND>(c.a, c.kappa, L.x, L.v, false);  // k -> v
  const int rid = L.rid;
  L.rid = -1;
  if (rid == B_INNER) {
    // optic axis along the mirror normal (radial cloak): one reflected ray
    if (!(c.mirror && (KIND == K_RO || KIND == K_RE) && L.bounces < o.max_bounces))
      return RT_RAY_ABSORBED;
    reflect_inside(B_INNER, L.x, L.v);
  } else {
    double d[3];
    const bool leaves = refract_out(c, KIND, rid, L.x, L.v, d, hr);
    // |v^T M v - 1| > 1e-3 at an outer interface: the state no longer
    // satisfies the dispersion relation, so it is not a ray of the medium
    if (!(hr <= 1e-3)) {
      if constexpr (HAM) ham_convert<KIND>(c.a, c.kappa, L.x, L.v, true);  // the stop path converts back
      return RT_RAY_DIVERGED;
    }
    if (leaves) {
#pragma unroll
      for (int i = 0; i < 3; ++i) L.v[i] = d[i];
      L.rid = rid;  // the exit boundary, kept with the finished ray
      return RT_RAY_EXITED;  // the exit transmission is applied by the finish kernel
    }
    if (L.bounces >= o.max_bounces) return RT_RAY_TIR;
    if constexpr (FRES) {
      const double2 tr = fresnel_event<KIND>(c.kappa, c.a, rid, L.x[0], L.x[1], L.x[2], L.v[0], L.v[1], L.v[2]);
      L.wt *= tr.y;
    }
    reflect_inside(rid, L.x, L.v);
  }
  // continue from the boundary point after the reflection
  ++L.bounces;
  L.h = o.h0;
  L.after_reject = false;
  if constexpr (HAM) ham_convert<KIND>(c.a, c.kappa, L.x, L.v, true);  // v -> k
  else accel<KIND>(c.a, L.x[0], L.x[1], L.v[0], L.v[1], L.v[2], L.A1[0], L.A1[1], L.A1[2]);
  return -1;
}

// Persistent integrator with in-line boundary events.
// Every iteration each active lane makes one attempt of the scheme from its
// base state (x, v). A lane is either stepping (accept/reject by the error
// controller) or locating a boundary crossing: after an accepted step that
// ends outside the material, the step is re-taken from the same base state
// with lengths chosen by a safeguarded Newton iteration on the boundary
// function g until |g| <= 1e-13 b. The crossing then goes through the
// interface: exit refraction (the ray stops), same-mode total internal
// reflection or the inner metal mirror (the ray continues from the boundary
// point with the step controller restarted). Only this bookkeeping diverges;
// the attempt itself is the same code for every lane of a branch.
// Integrate the rays of segment `seg` (all of one branch, KIND) with the
// calling wave until the segment's queue is drained and every lane of the
// wave is idle. The wave claims chunks of FETCH_CHUNK queue positions with
// one atomic each and refills its idle lanes every `refill` attempts. The
// lane state lives here, specialized for the branch, so no code of another
// branch is interleaved with the step loop.
template <int KIND, bool HAM, bool FRES>
__device__ __forceinline__ void run_segment(const CloakP &c, const OptsP &o, const Table &T, const SegMap &sm,
                                            int seg, double tol, int refill,
                                            unsigned int &drained) {
  int slot = -1;
  Lane L;
  L.h = 0.0; L.t = 0.0; L.lo = 0.0; L.hi = 0.0; L.ht = 0.0;
  L.x[0] = L.x[1] = L.x[2] = 0.0; L.v[0] = L.v[1] = L.v[2] = 0.0; L.A1[0] = L.A1[1] = L.A1[2] = 0.0;
  L.ns = 0; L.bounces = 0; L.rid = -1; L.riter = 0; L.after_reject = false;
  // wave-private chunk [cur, end) of the queue; cur, end and drained are wave-uniform
  unsigned int cur = 0, end = 0;
  const unsigned int off = off_of(sm, seg), len = off_of(sm, seg + 1) - off;
  for (;;) {
    unsigned long long m = __ballot(slot < 0);
    while (m != 0ull) {
      if (cur >= end) {
        if (drained >> seg & 1u) break;
        unsigned int base = 0;
        if (__lane_id() == 0) base = atomicAdd(T.ctr + C_FETCH(seg), FETCH_CHUNK);
        base = __shfl(base, 0);
        if (base + FETCH_CHUNK >= len) drained |= 1u << seg;
        cur = off + min(base, len);
        end = off + min(base + FETCH_CHUNK, len);
        continue;
      }
      const unsigned int idx = cur + (unsigned int)__popcll(m & lanemask_lt());
      if (slot < 0 && idx < end) {
        slot = T.order[idx];
        load_state(T, slot, L.x, L.v);
        L.t = 0.0;
        L.h = o.h0;
        L.ns = 0;
        L.bounces = 0;
        L.after_reject = false;
        L.rid = -1;
        if constexpr (HAM) ham_convert<KIND>(c.a, c.kappa, L.x, L.v, true);  // v -> k
        else accel<KIND>(c.a, L.x[0], L.x[1], L.v[0], L.v[1], L.v[2], L.A1[0], L.A1[1], L.A1[2]);
        if constexpr (FRES) L.wt = T.wt[slot];
      }
      cur = min(cur + (unsigned int)__popcll(m), end);
      m = __ballot(slot < 0);
    }
    if (__ballot(slot >= 0) == 0ull) return;

    // A wave that holds a ray past LONG_RAY_ATTEMPTS attempts is on the
    // launch's critical path (the longest rays take ~1500 attempts where the
    // mean is ~40): give it issue priority over the waves that share its
    // SIMD, which fill the remaining issue slots.
    if (__ballot(slot >= 0 && L.ns > LONG_RAY_ATTEMPTS) != 0ull) __builtin_amdgcn_s_setprio(3);
    else __builtin_amdgcn_s_setprio(0);

    for (int it = 0; it < refill; ++it) {
      if (slot >= 0) {
        double hr = __builtin_nan("");
        const int stop = iterate<KIND, HAM, FRES>(L, c, o, tol, hr);
        if (stop >= 0) {
          // the Hamiltonian form holds k until an interface: report v
          if constexpr (HAM)
            if (stop == RT_RAY_MAXSTEPS || stop == RT_RAY_DIVERGED) ham_convert<KIND>(c.a, c.kappa, L.x, L.v, false);
          store_state(T, slot, L.x, L.v);
          T.t[slot] = L.t;
          T.nsteps[slot] = L.ns;
          // bits 8..: the boundary an exited ray left through
          T.bounces[slot] = L.bounces | (stop == RT_RAY_EXITED ? L.rid << 8 : 0);
          T.status[slot] = stop;
          T.hres[slot] = hr;
          if constexpr (FRES) T.wt[slot] = L.wt;
          slot = -1;
        }
      }
    }
  }
}

template <bool HAM, bool FRES>
__global__ void __launch_bounds__(256) k_transit(CloakP c, OptsP o, Table T, int refill) {
  // the queue holds the used parts of the segments one after the other,
  // each sorted hardest first and holding one branch (every entry kernel
  // fills segment q with one (cloak, branch) pair); a wave integrates one
  // segment at a time and moves on to the next one that still has rays
  const SegMap sm = seg_map(T);
  const double tol = 1e-13 * c.b;
  unsigned int drained = 0;  // bit q: this wave found segment q's queue exhausted
  int nused = 0;
#pragma unroll
  for (int q = 0; q < NSEG; ++q) {
    if (sm.off[q + 1] == sm.off[q]) drained |= 1u << q;
    else ++nused;
  }
  if (nused == 0) return;
  // start on the (wave mod nused)-th used segment
  const unsigned int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int seg = 0;
  {
    int k = (int)(wave % (unsigned int)nused);
    for (int q = 0; q < NSEG; ++q)
      if (!(drained >> q & 1u)) {
        if (k == 0) { seg = q; break; }
        --k;
      }
  }
  while (drained != (1u << NSEG) - 1u) {
    while (drained >> seg & 1u) seg = (seg + 1) % NSEG;
    const int kind = __builtin_amdgcn_readfirstlane(T.kind[(long long)seg * T.cap]);
    switch (kind) {
      case K_RE: run_segment<K_RE, HAM, FRES>(c, o, T, sm, seg, tol, refill, drained); break;
      case K_AO: run_segment<K_AO, HAM, FRES>(c, o, T, sm, seg, tol, refill, drained); break;
      case K_AE: run_segment<K_AE, HAM, FRES>(c, o, T, sm, seg, tol, refill, drained); break;
      default: run_segment<K_RO, HAM, FRES>(c, o, T, sm, seg, tol, refill, drained); break;
    }
  }
}

// rt_trace_batch finish: vacuum leg of the entered rays to r_out
__global__ void __launch_bounds__(256) k_tb_finish(CloakP c, OptsP o, Table T, long long n,
                                                   double *__restrict__ out6, double *__restrict__ opl,
                                                   int *__restrict__ status, double *__restrict__ hres,
                                                   int *__restrict__ nsteps, double *__restrict__ trans) {
  unsigned int n0 = T.ctr[C_N(0)];
  unsigned int stride = gridDim.x * blockDim.x;
  for (unsigned int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n0; idx += stride) {
    int s = (int)idx;
    long long i = T.key[s];
    double x[3], v[3];
    load_state(T, s, x, v);
    int st = T.status[s];
    int kind = T.kind[s];
    double L = T.opl0[s] + T.t[s];
    double hr = T.hres[s];
    double wt = 0.0;
    if (trans && st == RT_RAY_EXITED) wt = T.wt[s] * exit_transmission(c, kind, T.bounces[s] >> 8, x, v);
    if (st == RT_RAY_EXITED) {
      double sl = leave_radius(x, v, o.r_out);
#pragma unroll
      for (int j = 0; j < 3; ++j) x[j] = fma(sl, v[j], x[j]);
      L += sl;
    } else {
      hr = hamiltonian_res(c, kind, x, v);
      double w = rsq64(fma(v[0], v[0], fma(v[1], v[1], v[2] * v[2])));
#pragma unroll
      for (int j = 0; j < 3; ++j) v[j] *= w;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) { out6[j * n + i] = x[j]; out6[(3 + j) * n + i] = v[j]; }
    opl[i] = L;
    status[i] = st;
    if (hres) hres[i] = hr;
    if (nsteps) nsteps[i] = T.nsteps[s];
    if (trans) trans[i] = wt;
  }
}

// rt_transit_exact entry: ray i enters through the side r = b at azimuth
// phi, height z, with horizontal angle alpha to the inward normal and
// elevation beta; its (cloak axis, branch) pair picks segment and metric.
// Rays outside the mask are skipped; invalid rays are finished at once.
__global__ void __launch_bounds__(256) k_sx_entry(CloakP c, OptsP o, Table T, long long n, long long ld,
                                                  const float *__restrict__ x6,
                                                  const unsigned char *__restrict__ mask, int have_axes,
                                                  float *__restrict__ y5, int *__restrict__ status,
                                                  float *__restrict__ hres, int *__restrict__ nsteps) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  bool entered = false;
  double x[3], v[3];
  int kind = 0, skey = 0;
  if (i < n && (!mask || mask[i])) {
    const double phi = x6[i], z = x6[ld + i], al = x6[2 * ld + i], be = x6[3 * ld + i];
    const float pol = x6[4 * ld + i], axis = x6[5 * ld + i];
    bool ok = isfinite(phi) && isfinite(z) && fabs(al) < 0.5 * M_PI && fabs(be) < 0.5 * M_PI &&
              z >= c.z0 && z <= c.z1 && (pol == 0.0f || pol == 1.0f) && (axis == 0.0f || axis == 1.0f);
    if (ok) {
      kind = (axis == 0.0f ? 0 : 2) + (pol == 0.0f ? 0 : 1);
      ok = (have_axes >> (kind >> 1)) & 1;
    }
    int st = RT_RAY_INVALID;
    if (ok) {
      double sp, cp, sa, ca, sb, cb;
      sincos(phi, &sp, &cp);
      sincos(al, &sa, &ca);
      sincos(be, &sb, &cb);
      x[0] = c.b * cp; x[1] = c.b * sp; x[2] = z;
      // d = cos(beta) (cos(alpha) (-r) + sin(alpha) theta) + sin(beta) z
      const double d[3] = {cb * (-ca * cp - sa * sp), cb * (-ca * sp + sa * cp), sb};
      if (refract_in(c, kind, B_SIDE, x, d, v)) {
        entered = true;
        skey = sort_key(c, kind, x, d);
      } else {
        st = RT_RAY_REFLECTED;
      }
    }
    if (!entered) {
      for (int j = 0; j < 5; ++j) y5[j * ld + i] = __builtin_nanf("");
      status[i] = st;
      if (hres) hres[i] = __builtin_nanf("");
      if (nsteps) nsteps[i] = 0;
    }
  }
  __shared__ unsigned int sh[16];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const bool want = entered && kind == q;
    unsigned int sl = block_append(T.ctr + C_N(q), want, sh);
    if (want) put_slot(T, (int)(q * T.cap + sl), x, v, q, i, 0.0, skey);
  }
}

// rt_transit_exact finish: vacuum leg of the outgoing ray back to r = b
// (zero for side exits) and its exit parameters
__global__ void __launch_bounds__(256) k_sx_finish(CloakP c, Table T, long long ld, float *__restrict__ y5,
                                                   int *__restrict__ status, float *__restrict__ hres,
                                                   int *__restrict__ nsteps) {
  const SegMap m = seg_map(T);
  const unsigned int n = m.off[NSEG];
  unsigned int stride = gridDim.x * blockDim.x;
  for (unsigned int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += stride) {
    int seg;
    int s = slot_at(T, m, idx, seg);
    long long i = T.key[s];
    int st = T.status[s];
    float out[5];
    if (st == RT_RAY_EXITED) {
      double x[3], v[3];
      load_state(T, s, x, v);
      double w = rsq64(fma(v[0], v[0], fma(v[1], v[1], v[2] * v[2])));
#pragma unroll
      for (int j = 0; j < 3; ++j) v[j] *= w;
      double sl = leave_radius(x, v, c.b);
#pragma unroll
      for (int j = 0; j < 3; ++j) x[j] = fma(sl, v[j], x[j]);
      double phi = atan2(x[1], x[0]);
      if (phi < 0.0) phi += 2.0 * M_PI;
      double rl = rsq64(fma(x[0], x[0], x[1] * x[1]));
      double vr = (x[0] * v[0] + x[1] * v[1]) * rl, vt = (x[0] * v[1] - x[1] * v[0]) * rl;
      out[0] = (float)phi;
      out[1] = (float)x[2];
      out[2] = (float)atan2(vt, vr);
      out[3] = (float)asin(fmin(1.0, fmax(-1.0, v[2])));
      out[4] = (float)(T.opl0[s] + T.t[s] + sl);
    } else {
#pragma unroll
      for (int j = 0; j < 5; ++j) out[j] = __builtin_nanf("");
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) y5[j * ld + i] = out[j];
    status[i] = st;
    if (hres) hres[i] = (float)T.hres[s];
    if (nsteps) nsteps[i] = T.nsteps[s];
  }
}

// ---------------------------------------------------------------------------
// render kernels
// ---------------------------------------------------------------------------
struct RenderP {
  long long g0, g1;   // chunk of the flattened (camera, pixel, sample) index
  long long ns_img;   // samples per image = w*h*spp
  int n_cams, ncl, npol, spp;
  int axis[2];        // optic axis of each cloak
  int pol[2];         // branch of each traced polarization
  int has_cloak, idx32;  // idx32: every flattened sample index < 2^32
  int sur_min;           // surrogate render: side entries of difficulty bucket >= sur_min are candidates
  double edge_tol;       // surrogate render: exit-error bound of an accepted prediction (tile-edge gate)
  unsigned char *codes;  // chunk-local codes [segment][g1-g0]
  float *topl;           // chunk-local optical path to the room [segment][g1-g0] (NaN: no room point); NULL unless tof
  double *rec;           // aux (may be NULL)
  int *st;
  unsigned char *code;
  int *nsteps;
  float *tof;            // aux per-pixel time of flight (may be NULL)
  float *twt;            // chunk-local Eq. (12) image weight [segment][g1-g0]; NULL unless unpol or goggles
  float *unpol;          // aux per-pixel unpolarized image, per (cloak, camera) (may be NULL)
  // chunk-local [segment][g1-g0]: the entry transmission of the in-plane
  // goggle's field over the unpolarized one (1 for a sample that stays in
  // vacuum); NULL unless goggle images
  float *grho;
  float *gog[2];         // aux per-pixel goggle images (in-plane, axial), per (cloak, camera) (may be NULL)
  // first-order reflections (with refl set), chunk-local: per [segment][g1-g0]
  // the entry's reflected vacuum ray, its unpolarized image weight (R / 2),
  // the in-plane goggle's weight (R_in / 4; NULL without goggles) and its
  // room code; per [segment][child mode][g1-g0] the weight and room code of
  // the wave reflected at the exit into that mode, followed to its own exit
  int refl;
  float *rext, *rgin, *cw;
  unsigned char *rcode, *ccode;
};

// Surrogate render: the side entries of a chunk that go to the network
// first (candidates), one row each.
struct CandP {
  float *x6;          // SoA 6 x ld: phi, z, alpha, beta, branch bit, axis bit (the surrogate's inputs)
  long long ld;       // rows allocated
  long long *key;     // flattened sample index * NSEG + segment
  float *s_in;        // vacuum distance from the eye to the entry
  float *y5;          // SoA 5 x ld: predicted exit (phi', z', alpha', beta', T) of accepted rows
  unsigned char *fb;  // 1 where the gate rejected the prediction
  int *st;            // gate status (RT_RAY_EXITED where accepted)
};

// flattened sample index -> (camera, sample within the image), in 32-bit
// arithmetic when every index fits (64-bit division is a long sequence)
__device__ __forceinline__ void split_index(const RenderP &R, long long gidx, long long &cam, long long &loc) {
  if (R.idx32) {
    const unsigned int g = (unsigned int)gidx, ns = (unsigned int)R.ns_img, c32 = g / ns;
    cam = c32;
    loc = g - c32 * ns;
  } else {
    cam = gidx / R.ns_img;
    loc = gidx - cam * R.ns_img;
  }
}

// segment q = cloak * npol + polarization; images are laid out
// [cloak][camera][polarization]. OUT = false: the caller guarantees that no
// optional output (weights, optical paths, per-sample records) is asked
// for, and only the colour code is written.
template <bool OUT = true>
__device__ __forceinline__ void rd_write(const RenderP &R, int q, long long gidx, int code,
                                         int st, const double p[3], const double d[3], double L,
                                         int nsteps, float wt = 0.f) {
  R.codes[(long long)q * (R.g1 - R.g0) + (gidx - R.g0)] = (unsigned char)code;
  if constexpr (!OUT) return;
  if (R.twt) R.twt[(long long)q * (R.g1 - R.g0) + (gidx - R.g0)] = wt;
  if (R.topl) R.topl[(long long)q * (R.g1 - R.g0) + (gidx - R.g0)] = code < 12 ? (float)L : __builtin_nanf("");
  long long cam, loc;
  split_index(R, gidx, cam, loc);
  int ci = q / R.npol, pi = q - ci * R.npol;
  long long img = ((long long)ci * R.n_cams + cam) * R.npol + pi;
  if (R.st) R.st[img * R.ns_img + loc] = st;
  if (R.code) R.code[img * R.ns_img + loc] = (unsigned char)code;
  if (R.nsteps) R.nsteps[img * R.ns_img + loc] = nsteps;
  if (R.rec) {
    double *r = R.rec + img * 7 * R.ns_img + loc;
#pragma unroll
    for (int j = 0; j < 3; ++j) { r[j * R.ns_img] = p[j]; r[(3 + j) * R.ns_img] = d[j]; }
    r[6 * R.ns_img] = L;
  }
}

// a side entry as surrogate input: azimuth and height of the entry point,
// horizontal angle of the incident direction to the inward normal (positive
// towards +theta), elevation, and the (branch, axis) bits of `kind`
__device__ __forceinline__ void put_candidate(const CandP &C, unsigned int i, const double x[3], const double d[3],
                                              int kind, long long gidx, int q, double s) {
  double phi = atan2(x[1], x[0]);
  if (phi < 0.0) phi += 2.0 * M_PI;
  const double rl = rsq64(fma(x[0], x[0], x[1] * x[1]));
  const double dr = (x[0] * d[0] + x[1] * d[1]) * rl, dt = (x[0] * d[1] - x[1] * d[0]) * rl;
  float *X = C.x6 + i;
  X[0] = (float)phi;
  X[C.ld] = (float)x[2];
  X[2 * C.ld] = (float)atan2(dt, -dr);
  X[3 * C.ld] = (float)asin(fmin(1.0, fmax(-1.0, d[2])));
  X[4 * C.ld] = (float)(kind & 1);
  X[5 * C.ld] = (float)(kind >> 1);
  C.key[i] = gidx * NSEG + q;
  C.s_in[i] = (float)s;
}

// Eq. (12) at a camera sample's entry into the cloak of axis kind >> 1
// through boundary surf at x, direction d: the unpolarized transmission
// into branch kind & 1 (.x), with goggle the ratio to it of the
// transmission of the in-plane goggle's field (.y, else 1), and the
// reflected fractions of unpolarized light (.z) and of the goggle's field
// (.w, with goggle), 1 - T_o - T_e. The goggle's field is the camera's
// horizontal axis r made transverse to the ray (Figs. 1d and 2d); the axial
// goggle's is d x it, and the two transmissions add up to twice the
// unpolarized one. Out of line with scalar arguments, like fresnel_event:
// the complex solves would otherwise set the register allocation of the
// whole generation kernel.
__device__ __noinline__ double4 entry_weight(double kappa, double a, int kind, int surf, double x0, double x1,
                                             double x2, double d0, double d1, double d2, double r0, double r1,
                                             double r2, int goggle) {
  CloakP c{};
  c.kappa = kappa;
  c.a = a;
  const double x[3] = {x0, x1, x2}, d[3] = {d0, d1, d2};
  double eo, ee, cax[3], nrm[3];
  boundary_normal(surf, x, nrm);
  material_axis(c, kind >> 1, x, eo, ee, cax);
  double To, Te;
  fresnel_in2_dev(eo, ee, cax, nrm, d, To, Te);
  const double w = (kind & 1) ? Te : To;
  if (!goggle) return make_double4(w, 1.0, 1.0 - To - Te, 0.0);
  const double rd = r0 * d0 + r1 * d1 + r2 * d2;
  double e[3] = {r0 - rd * d0, r1 - rd * d1, r2 - rd * d2};
  const double ie = 1.0 / sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
  e[0] *= ie; e[1] *= ie; e[2] *= ie;
  double go, ge, uo, ue;
  fresnel_in_pol_dev(eo, ee, cax, nrm, d, e, go, ge, uo, ue);
  const double tg = (kind & 1) ? ge : go, tun = (kind & 1) ? ue : uo;
  return make_double4(w, tun > 0.0 ? tg / tun : 1.0, 1.0 - To - Te, 1.0 - go - ge);
}

// camera rays of a chunk; one thread per sample, every (cloak, branch).
// SUR: side entries become surrogate candidates instead of work-table slots.
// WM: Eq. (12) weights at the entry, 0 none, 1 unpolarized, 2 with the
// goggle ratio (separate instantiations: the entry solves are large, and a
// render without weights should not carry their registers). Without weights
// the kernel is held to 128 VGPRs (4 waves per SIMD instead of 3): its
// barriers and table stores then hide better. OUT: per-sample outputs
// (records, optical paths) are asked for; without them and without weights
// the kernel writes colour codes and work-table slots only, and holds fewer
// uniform pointers.
template <bool SUR, int WM, bool OUT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WM == 0 ? 4 : 1))) k_rd_gen(CloakP c, OptsP o, RoomP rm,
                                                const CamP *__restrict__ cams, Table T, RenderP R, CandP Cd) {
  long long gidx = R.g0 + (long long)blockIdx.x * blockDim.x + threadIdx.x;
  bool valid = gidx < R.g1;
  double org[3] = {0, 0, 0}, d[3] = {0, 0, 1}, x[3] = {0, 0, 0}, s = 0.0, cr[3] = {1, 0, 0};
  int surf = 0;
  bool hitc = false, disk = false;
  if (valid) {
    long long cam, loc;
    split_index(R, gidx, cam, loc);
    const unsigned int l32 = (unsigned int)loc, sp = (unsigned int)R.spp;  // loc < ns_img <= 2^30
    const long long pix = l32 / sp;
    const int smp = (int)(l32 - (unsigned int)pix * sp);
    const CamP &C = cams[cam];
    org[0] = C.eye[0]; org[1] = C.eye[1]; org[2] = C.eye[2];
    cr[0] = C.R[0]; cr[1] = C.R[1]; cr[2] = C.R[2];
    camera_ray(C, (int)cam, pix, smp, d);
    if (R.has_cloak) hitc = vacuum_entry(c, org, d, s, surf);
    if (hitc) {
#pragma unroll
      for (int j = 0; j < 3; ++j) x[j] = fma(s, d[j], org[j]);
      if (surf == B_TOP) x[2] = c.z1;
      if (surf == B_BOTTOM) x[2] = c.z0;
      disk = surf != B_SIDE && fma(x[0], x[0], x[1] * x[1]) <= c.a2;
    }
  }
  // rays that miss the cloak or hit the metal end disk see the same room
  // point for every (cloak, branch): shade them once
  int vcode = 12, vst = RT_RAY_MISSED;
  double vp[3] = {org[0], org[1], org[2]}, vd[3] = {d[0], d[1], d[2]}, vL = 0.0;
  if (valid && (!hitc || disk)) {
    if (disk) {
      double nrm[3];
      boundary_normal(surf, x, nrm);
      vp[0] = x[0]; vp[1] = x[1]; vp[2] = x[2];
      vL = s;
      if (c.mirror) { reflect3(vd, nrm); vst = RT_RAY_REFLECTED; }
      else vst = RT_RAY_ABSORBED;
    }
    if (vst != RT_RAY_ABSORBED) {
      double sh;
      vcode = room_code(rm, vp, vd, sh);
      vL += sh;
    }
  }
  __shared__ unsigned int sh[16];
  for (int q = 0; q < R.ncl * R.npol; ++q) {
    int ci = q / R.npol, pi = q - ci * R.npol;
    int kind = (ci == 0 ? R.axis[0] : R.axis[1]) * 2 + (pi == 0 ? R.pol[0] : R.pol[1]);
    bool enter = false, cand = false;
    double v[3] = {0, 0, 0}, w_in = 0.0;
    const long long li = (long long)q * (R.g1 - R.g0) + (gidx - R.g0);  // chunk-local index
    int skey = 0;
    // goggles and reflections need the Eq. (12) weights (WM > 0)
    if (WM > 0 && valid) {
      // goggle ratio 1 and no reflected light unless the sample meets the
      // crystal (set below)
      if (R.grho) R.grho[li] = 1.0f;
      if (R.refl) {
        R.rext[li] = 0.0f;
        if (R.rgin) R.rgin[li] = 0.0f;
        R.rcode[li] = 12;
#pragma unroll
        for (int bp = 0; bp < 2; ++bp) {
          R.cw[(2 * q + bp) * (R.g1 - R.g0) + (gidx - R.g0)] = 0.0f;
          R.ccode[(2 * q + bp) * (R.g1 - R.g0) + (gidx - R.g0)] = 12;
        }
      }
    }
    double4 ew = make_double4(0.0, 1.0, 0.0, 0.0);
    if (WM > 0 && valid && hitc && !disk) {
      ew = entry_weight(c.kappa, c.a, kind, surf, x[0], x[1], x[2], d[0], d[1], d[2], cr[0], cr[1], cr[2],
                        WM == 2);
      if (R.refl) {
        // the vacuum ray reflected at the entry (a convex body: it leaves)
        double nrm[3], dd[3] = {d[0], d[1], d[2]}, sh;
        boundary_normal(surf, x, nrm);
        reflect3(dd, nrm);
        R.rext[li] = (float)(0.5 * ew.z);
        if (R.rgin) R.rgin[li] = (float)(0.25 * ew.w);
        R.rcode[li] = (unsigned char)room_code(rm, x, dd, sh);
      }
    }
    if (valid) {
      if (!hitc || disk) {
        rd_write<(OUT || WM > 0)>(R, q, gidx, vcode, vst, vp, vd, vL, 0, 0.5f);  // vacuum light splits evenly
      } else if (refract_in(c, kind, surf, x, d, v)) {
        skey = sort_key(c, kind, x, d);
        if (SUR && surf == B_SIDE && NBUCKET - 1 - skey >= R.sur_min) cand = true;
        else enter = true;
        if (WM > 0) {
          w_in = ew.x;
          if (WM == 2) R.grho[li] = (float)ew.y;
        }
      } else {
        // evanescent transmission into this branch: reflected at the entry
        double nrm[3], dd[3] = {d[0], d[1], d[2]}, sh;
        boundary_normal(surf, x, nrm);
        reflect3(dd, nrm);
        int code = room_code(rm, x, dd, sh);
        rd_write<(OUT || WM > 0)>(R, q, gidx, code, RT_RAY_REFLECTED, x, dd, s + sh, 0);
      }
    }
    unsigned int sl = block_append(T.ctr + C_N(q), enter, sh);
    if (enter) put_slot(T, (int)(q * T.cap + sl), x, v, kind, gidx, s, skey);
    if (WM > 0 && enter) T.wt[q * T.cap + sl] = w_in;
    if constexpr (SUR) {
      const unsigned int ci2 = block_append(T.ctr + C_SUR, cand, sh);
      if (cand) put_candidate(Cd, ci2, x, d, kind, gidx, q, s);
    }
  }
}

// Surrogate render, after the gate: an accepted candidate's predicted exit
// ray (on r = b, alpha' to the outward normal) takes its vacuum leg to the
// room (its record: that point, or for an exit beyond a cap the cap point on
// the same line); a rejected one is generated again from its camera sample
// exactly as k_rd_gen does and queued for the integrator in its segment.
__global__ void __launch_bounds__(256) k_rd_sur_apply(CloakP c, OptsP o, RoomP rm, const CamP *__restrict__ cams,
                                                      Table T, RenderP R, CandP Cd, unsigned int n) {
  const unsigned int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  const long long key = valid ? Cd.key[i] : 0;
  const int q = (int)(key & (NSEG - 1));
  const long long gidx = key >> 2;
  static_assert(NSEG == 4, "key packing assumes 4 segments");
  bool rej = valid && Cd.fb[i] != 0;
  if (valid && !rej) {
    const double ph = Cd.y5[i], ze = Cd.y5[Cd.ld + i], al = Cd.y5[2 * Cd.ld + i];
    const double be = Cd.y5[3 * Cd.ld + i], Tt = Cd.y5[4 * Cd.ld + i];
    const double cp = cos(ph), sp = sin(ph), cb = cos(be);
    const double ca = cos(al), sa = sin(al);
    double p[3] = {c.b * cp, c.b * sp, ze};
    double dd[3] = {cb * (ca * cp - sa * sp), cb * (ca * sp + sa * cp), sin(be)};
    // an exit beyond a cap (a chained cap model's prediction) left the
    // crystal at its cap point, on the same line, where the vacuum leg to
    // the room starts (the point on r = b can lie above the room)
    double tb = 0.0;
    if (ze > c.z1 || ze < c.z0) {
      tb = (ze - (ze > c.z1 ? c.z1 : c.z0)) / dd[2];
#pragma unroll
      for (int j = 0; j < 3; ++j) p[j] = fma(-tb, dd[j], p[j]);
    }
    double sh0;
    const int code = room_code(rm, p, dd, sh0);
    // tile-edge gate: the accepted exit errs by at most edge_tol in
    // position (units of r2) and direction (rad) on r = b, which moves the
    // room point along the face by at most edge_tol (r2 + distance) /
    // cosine, the distance counted from r = b (the vacuum leg back to a cap
    // point included); a point closer than twice that to a tile edge could
    // take the other colour, so the sample goes to the integrator
    double cosn = 1.0;
    const double dist = code < 12 ? tile_edge_distance(rm, p, dd, sh0, code >> 1, cosn) : 0.0;
    if (!(dist * cosn > 2.0 * R.edge_tol * (c.b + tb + sh0))) rej = true;
    else rd_write(R, q, gidx, code, RT_RAY_EXITED, p, dd, (double)Cd.s_in[i] + (Tt - tb) + sh0, 0);
  }
  double x[3] = {0, 0, 0}, v[3] = {0, 0, 0}, d[3] = {0, 0, 1}, s = 0.0;
  int kind = 0;
  bool enter = false;
  if (rej) {
    long long cam, loc;
    split_index(R, gidx, cam, loc);
    const unsigned int l32 = (unsigned int)loc, sp32 = (unsigned int)R.spp;
    const long long pix = l32 / sp32;
    const int smp = (int)(l32 - (unsigned int)pix * sp32);
    const CamP &C = cams[cam];
    const double org[3] = {C.eye[0], C.eye[1], C.eye[2]};
    camera_ray(C, (int)cam, pix, smp, d);
    int surf = 0;
    const bool hitc = vacuum_entry(c, org, d, s, surf);
#pragma unroll
    for (int j = 0; j < 3; ++j) x[j] = fma(s, d[j], org[j]);
    const int ci = q / R.npol, pi = q - ci * R.npol;
    kind = (ci == 0 ? R.axis[0] : R.axis[1]) * 2 + (pi == 0 ? R.pol[0] : R.pol[1]);
    enter = hitc && surf == B_SIDE && refract_in(c, kind, surf, x, d, v);
    if (!enter) rd_write(R, q, gidx, 12, RT_RAY_INVALID, x, d, s, 0);  // not reached: k_rd_gen made it a candidate
  }
  __shared__ unsigned int sh[16];
  for (int qq = 0; qq < R.ncl * R.npol; ++qq) {
    const bool put = enter && q == qq;
    const unsigned int sl = block_append(T.ctr + C_N(qq), put, sh);
    if (put) put_slot(T, (int)(qq * T.cap + sl), x, v, kind, gidx, s, sort_key(c, kind, x, d));
  }
  (void)block_append(T.ctr + C_ACC, valid && !rej, sh);
}

// OUT: per-sample outputs are asked for (sample_outputs); without them a
// ray's colour code needs only its status and, if it exited, its exit ray
template <bool OUT>
__global__ void __launch_bounds__(256) k_rd_finish(CloakP c, RoomP rm, Table T, RenderP R) {
  const SegMap m = seg_map(T);
  const unsigned int n = m.off[NSEG];
  unsigned int stride = gridDim.x * blockDim.x;
  for (unsigned int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += stride) {
    int q;
    int s = slot_at(T, m, idx, q);
    if constexpr (!OUT) {
      int code = 12;
      if (T.status[s] == RT_RAY_EXITED) {
        double x[3], v[3], sh;
        load_state(T, s, x, v);
        code = room_code(rm, x, v, sh);
      }
      rd_write<false>(R, q, T.key[s], code, 0, nullptr, nullptr, 0.0, 0);
      continue;
    }
    double x[3], v[3];
    load_state(T, s, x, v);
    int st = T.status[s];
    double L = T.opl0[s] + T.t[s];
    int code = 12;
    if (st == RT_RAY_EXITED) {
      double sh;
      code = room_code(rm, x, v, sh);
      L += sh;
    } else {
      double w = rsq64(fma(v[0], v[0], fma(v[1], v[1], v[2] * v[2])));
#pragma unroll
      for (int j = 0; j < 3; ++j) v[j] *= w;
    }
    const double wt = (R.twt && st == RT_RAY_EXITED)
                          ? T.wt[s] * exit_transmission(c, T.kind[s], T.bounces[s] >> 8, x, v) : 0.0;
    rd_write(R, q, T.key[s], code, st, x, v, L, T.nsteps[s], (float)wt);
  }
}

// First-order reflections, after k_rd_finish: every primary that left the
// crystal spawns the two waves its exit reflects into the ordinary and the
// extraordinary mode (fractions Ro, Re of the exit solve) as slots of the
// child table Tc, in the segment of that mode. A reflected wave has the
// tangential wave vector of the wave met and the normal component of its
// own mode's dispersion relation, pointing back in: that is the refraction
// of the vacuum ray mirrored about the surface, whose tangential part is
// the exit ray's. A child carries the primary's weight before the exit
// transmission times its reflectance, and its key the sample and the
// primary's branch (bits 56+). The loop runs in whole blocks, so that
// every thread of a block takes part in each append.
constexpr int CHILD_SHIFT = 56;
__global__ void __launch_bounds__(256) k_rd_spawn(CloakP c, OptsP o, Table T, Table Tc, RenderP R) {
  const SegMap m = seg_map(T);
  const unsigned int n = m.off[NSEG];
  __shared__ unsigned int sh[16];
  for (unsigned int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const unsigned int idx = base + threadIdx.x;
    bool have = false;
    int q = 0, kind = 0, rid = 0;
    double x[3] = {0, 0, 0}, d[3] = {0, 0, 1}, wpre = 0.0, Rr[2] = {0.0, 0.0};
    long long key = 0;
    if (idx < n) {
      const int sl = slot_at(T, m, idx, q);
      if (T.status[sl] == RT_RAY_EXITED) {
        load_state(T, sl, x, d);
        kind = T.kind[sl];
        rid = T.bounces[sl] >> 8;
        double Tt;
        exit_fresnel(c, kind, rid, x, d, Tt, Rr[0], Rr[1]);
        wpre = T.wt[sl];
        key = T.key[sl] | ((long long)(q % R.npol) << CHILD_SHIFT);
        have = true;
      }
    }
#pragma unroll
    for (int bp = 0; bp < 2; ++bp) {
      double vc[3], dm[3] = {d[0], d[1], d[2]};
      const int kc = (kind & ~1) | bp, qc = (q / R.npol) * R.npol + bp;
      bool put = false;
      if (have && Rr[bp] > 0.0) {
        double nrm[3];
        boundary_normal(rid, x, nrm);
        reflect3(dm, nrm);
        put = refract_in(c, kc, rid, x, dm, vc);
      }
      for (int qq = 0; qq < R.ncl * R.npol; ++qq) {
        const bool p2 = put && qc == qq;
        const unsigned int cs = block_append(Tc.ctr + C_N(qq), p2, sh);
        if (p2) {
          const int slot = (int)(qq * Tc.cap + cs);
          put_slot(Tc, slot, x, vc, kc, key, 0.0, sort_key(c, kc, x, dm));
          Tc.wt[slot] = wpre * Rr[bp];
        }
      }
    }
  }
}

// The children's exits: room code and weight (x the exit transmission) into
// the chunk-local arrays of their primary's segment and their mode; a child
// that does not leave keeps weight 0.
__global__ void __launch_bounds__(256) k_rd_cfinish(CloakP c, RoomP rm, Table Tc, RenderP R) {
  const SegMap m = seg_map(Tc);
  const unsigned int n = m.off[NSEG];
  const long long chunk = R.g1 - R.g0;
  for (unsigned int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += gridDim.x * blockDim.x) {
    int qc;
    const int s = slot_at(Tc, m, idx, qc);
    if (Tc.status[s] != RT_RAY_EXITED) continue;
    double x[3], d[3], sh;
    load_state(Tc, s, x, d);
    const int code = room_code(rm, x, d, sh);
    const double w = Tc.wt[s] * exit_transmission(c, Tc.kind[s], Tc.bounces[s] >> 8, x, d);
    const long long key = Tc.key[s];
    const int pi = (int)(key >> CHILD_SHIFT), bp = qc % R.npol;
    const long long gidx = key & ((1LL << CHILD_SHIFT) - 1);
    const int qp = (qc / R.npol) * R.npol + pi;
    const long long o = (2LL * qp + bp) * chunk + (gidx - R.g0);
    R.cw[o] = (float)w;
    R.ccode[o] = (unsigned char)code;
  }
}

// per-pixel mean colour; the 13-entry colour table is staged in LDS
// (segment, pixel) entry i of a chunk -> segment q, chunk-local pixel lp,
// camera and the float index of the pixel's RGB in the [cloak][camera]
// [branch][pixel][3] images
__device__ __forceinline__ long long resolve_index(const RenderP &R, long long npix, long long pix_in_chunk,
                                                   long long i, int &q, long long &lp, long long &cam) {
  if (R.idx32) {  // every index below fits 32 bits
    const unsigned int i32 = (unsigned int)i, pc = (unsigned int)pix_in_chunk;
    q = (int)(i32 / pc);
    lp = i32 - (unsigned int)q * pc;
  } else {
    q = (int)(i / pix_in_chunk);
    lp = i - q * pix_in_chunk;
  }
  const long long gpix = R.g0 / R.spp + lp;  // flattened (camera, pixel)
  long long pix;
  if (R.idx32) {
    const unsigned int g32 = (unsigned int)gpix, np = (unsigned int)npix, c32 = g32 / np;
    cam = c32;
    pix = g32 - c32 * np;
  } else {
    cam = gpix / npix;
    pix = gpix - cam * npix;
  }
  const int ci = q / R.npol, pi = q - ci * R.npol;
  return ((((long long)ci * R.n_cams + cam) * R.npol + pi) * npix + pix) * 3;
}

// Pixel means of a render that asks for no other per-pixel image (no time of
// flight, unpolarized or goggle image): tiles of 256 entries, in the order of
// k_rd_resolve, taken by a fixed grid of blocks in turn. A tile whose entries
// form one run of the output (one segment and camera, 16-byte aligned) is
// staged in LDS and stored as 192 float4; any other tile stores each pixel's
// three floats.
__global__ void __launch_bounds__(256) k_rd_resolve_plain(RenderP R, const float *__restrict__ table39,
                                                          float *__restrict__ rgb, long long npix) {
  __shared__ float tab[39];
  __shared__ float4 buf4[192];
  __shared__ long long run0;
  if (threadIdx.x < 39) tab[threadIdx.x] = table39[threadIdx.x];
  const long long chunk = R.g1 - R.g0, pix_in_chunk = chunk / R.spp;
  const long long total = pix_in_chunk * R.ncl * R.npol;
  const long long ntiles = (total + 255) / 256;
  const float inv = 1.0f / (float)R.spp;
  for (long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const long long i0 = t * 256, i = i0 + threadIdx.x;
    const bool valid = i < total;
    if (threadIdx.x == 0) {
      long long r = -1;
      if (i0 + 255 < total) {
        int qa, qb;
        long long la, lb, ca, cb;
        const long long oa = resolve_index(R, npix, pix_in_chunk, i0, qa, la, ca);
        (void)resolve_index(R, npix, pix_in_chunk, i0 + 255, qb, lb, cb);
        if (qa == qb && ca == cb && ((uintptr_t)(rgb + oa) & 15) == 0) r = oa;
      }
      run0 = r;
    }
    __syncthreads();  // tab (first tile) and run0 set; the previous tile's buf4 read
    float c[3] = {0.f, 0.f, 0.f};
    long long o = 0;
    if (valid) {
      int q;
      long long lp, cam;
      o = resolve_index(R, npix, pix_in_chunk, i, q, lp, cam);
      const unsigned char *cd = R.codes + q * chunk + lp * R.spp;
      if (R.spp == 4) {  // chunk and codes are 4-byte aligned
        const unsigned int c4 = *(const unsigned int *)cd;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int cc = (c4 >> (8 * k)) & 0xff;
          c[0] += tab[3 * cc]; c[1] += tab[3 * cc + 1]; c[2] += tab[3 * cc + 2];
        }
      } else {
        for (int k = 0; k < R.spp; ++k) {
          const int cc = cd[k];
          c[0] += tab[3 * cc]; c[1] += tab[3 * cc + 1]; c[2] += tab[3 * cc + 2];
        }
      }
      c[0] *= inv; c[1] *= inv; c[2] *= inv;
    }
    const long long base = run0;
    if (base >= 0) {  // block-uniform
      float *b = (float *)buf4;
      b[3 * threadIdx.x] = c[0];
      b[3 * threadIdx.x + 1] = c[1];
      b[3 * threadIdx.x + 2] = c[2];
      __syncthreads();
      if (threadIdx.x < 192) ((float4 *)(rgb + base))[threadIdx.x] = buf4[threadIdx.x];
    } else if (valid) {
      rgb[o] = c[0];
      rgb[o + 1] = c[1];
      rgb[o + 2] = c[2];
    }
    __syncthreads();  // run0 and buf4 read before the next tile writes them
  }
}

__global__ void __launch_bounds__(256) k_rd_resolve(RenderP R, const float *__restrict__ table39,
                                                    float *__restrict__ rgb, long long npix) {
  __shared__ float tab[39];
  if (threadIdx.x < 39) tab[threadIdx.x] = table39[threadIdx.x];
  __syncthreads();
  long long chunk = R.g1 - R.g0;
  long long pix_in_chunk = chunk / R.spp;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pix_in_chunk * R.ncl * R.npol) return;
  int q;
  long long lp;
  if (R.idx32) {  // every index below fits 32 bits
    const unsigned int i32 = (unsigned int)i, pc = (unsigned int)pix_in_chunk;
    q = (int)(i32 / pc);
    lp = i32 - (unsigned int)q * pc;
  } else {
    q = (int)(i / pix_in_chunk);
    lp = i - q * pix_in_chunk;
  }
  const unsigned char *cd = R.codes + q * chunk + lp * R.spp;
  float r = 0.f, g = 0.f, b = 0.f;
  for (int k = 0; k < R.spp; ++k) {
    int cc = cd[k];
    r += tab[3 * cc];
    g += tab[3 * cc + 1];
    b += tab[3 * cc + 2];
  }
  float inv = 1.0f / (float)R.spp;
  double tsum = 0.0;
  int tn = 0;
  if (R.tof) {
    const float *tl = R.topl + q * chunk + lp * R.spp;
    for (int k = 0; k < R.spp; ++k)
      if (isfinite(tl[k])) { tsum += tl[k]; ++tn; }
  }
  long long gpix = R.g0 / R.spp + lp;  // flattened (camera, pixel)
  long long cam, pix;
  if (R.idx32) {
    const unsigned int g32 = (unsigned int)gpix, np = (unsigned int)npix, c32 = g32 / np;
    cam = c32;
    pix = g32 - c32 * np;
  } else {
    cam = gpix / npix;
    pix = gpix - cam * npix;
  }
  int ci = q / R.npol, pi = q - ci * R.npol;
  const long long img = ((long long)ci * R.n_cams + cam) * R.npol + pi;
  float *o = rgb + (img * npix + pix) * 3;
  o[0] = r * inv;
  o[1] = g * inv;
  o[2] = b * inv;
  if (R.tof) R.tof[img * npix + pix] = tn ? (float)(tsum / tn) : __builtin_nanf("");
  if ((R.unpol || R.grho) && pi == 0) {
    // both branches of this cloak (segments q, q + 1), each sample's colour
    // times the share of its light the branch carries; the goggles take half
    // of that share times the ratio of the goggle field's entry transmission
    // to the unpolarized one, rho for the in-plane goggle and 2 - rho for
    // the axial; with first-order reflections, the entry's reflected ray
    // (R / 2 per branch, R_in / 4 through the in-plane goggle) and the two
    // reflected waves of each branch's exit (entry shared with the branch)
    float u[3] = {0.f, 0.f, 0.f}, gr[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    for (int b = 0; b < 2; ++b) {
      const long long o = (q + b) * chunk + lp * R.spp;
      const unsigned char *cb = R.codes + o;
      const float *wb = R.twt + o;
      for (int k = 0; k < R.spp; ++k) {
        const int cc = cb[k];
        const float wk = wb[k], rk = R.grho ? R.grho[o + k] : 1.0f;
        const float w0 = 0.5f * wk * rk, w1 = wk - w0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          u[j] = fmaf(wk, tab[3 * cc + j], u[j]);
          gr[0][j] = fmaf(w0, tab[3 * cc + j], gr[0][j]);
          gr[1][j] = fmaf(w1, tab[3 * cc + j], gr[1][j]);
        }
        if (R.refl) {
          const int ce = R.rcode[o + k];
          const float we = R.rext[o + k], wi = R.rgin ? R.rgin[o + k] : 0.f;
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            u[j] = fmaf(we, tab[3 * ce + j], u[j]);
            gr[0][j] = fmaf(wi, tab[3 * ce + j], gr[0][j]);
            gr[1][j] = fmaf(we - wi, tab[3 * ce + j], gr[1][j]);
          }
#pragma unroll
          for (int bp = 0; bp < 2; ++bp) {
            const long long oc = (2 * (q + b) + bp) * chunk + lp * R.spp + k;
            const int c2 = R.ccode[oc];
            const float wc = R.cw[oc], c0 = 0.5f * wc * rk, c1 = wc - c0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              u[j] = fmaf(wc, tab[3 * c2 + j], u[j]);
              gr[0][j] = fmaf(c0, tab[3 * c2 + j], gr[0][j]);
              gr[1][j] = fmaf(c1, tab[3 * c2 + j], gr[1][j]);
            }
          }
        }
      }
    }
    const long long po = (((long long)ci * R.n_cams + cam) * npix + pix) * 3;
    if (R.unpol) {
#pragma unroll
      for (int j = 0; j < 3; ++j) R.unpol[po + j] = u[j] * inv;
    }
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      if (!R.gog[g]) continue;
#pragma unroll
      for (int j = 0; j < 3; ++j) R.gog[g][po + j] = gr[g][j] * inv;
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// Device workspace: the work table (NSEG segments of `cap` slots), the colour
// codes and optical paths of one render chunk, camera records and the colour
// table. The direct
// calls share one (g_ws); every render plan owns its own.
struct Workspace {
  void *base = nullptr;
  size_t bytes = 0;
  long long cap = 0;
  long long codes_len = 0;
  int cams_cap = 0;
  int device = -1;
  Table T{};
  unsigned char *codes = nullptr;
  float *topl = nullptr;  // per-sample optical path of a chunk (time-of-flight images)
  float *twt = nullptr;   // per-sample Eq. (12) image weight of a chunk (unpolarized and goggle images)
  float *grho = nullptr;  // per-sample goggle ratio of a chunk (goggle images)
  CamP *cams = nullptr;
  float *table = nullptr;
};

std::mutex g_ws_mu;
Workspace g_ws;
// The direct calls' shared workspaces. Every call waits on its stream for
// the previous use of the workspace it takes (which may have been enqueued
// on another stream) and marks its own use with an event, so calls on
// several streams are ordered where they share memory. rt_render_multi
// keeps up to NWS workspaces, one per stream it sees (a new stream takes the
// workspace used longest ago): renders on several streams then run side by
// side, one's camera rays and sort next to another's integrator and its
// drain. The other direct calls, the surrogate and reflection buffers use
// the first.
constexpr int NWS = 4;
Workspace g_wsx[NWS - 1];  // workspaces 1..NWS-1 (workspace 0 is g_ws)
hipEvent_t g_ws_ev[NWS] = {nullptr, nullptr, nullptr, nullptr};
int g_ws_evdev[NWS] = {-1, -1, -1, -1};
hipStream_t g_ws_stream[NWS] = {nullptr, nullptr, nullptr, nullptr};
unsigned long long g_ws_last[NWS] = {0, 0, 0, 0};  // call counter at the last use
unsigned long long g_ws_calls = 0;

Workspace &ws_at(int k) { return k ? g_wsx[k - 1] : g_ws; }

int ws_order(int k, hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RT_E_DEVICE, "hipGetDevice failed");
  if (g_ws_ev[k] && g_ws_evdev[k] != dev) {
    // the previous use was on another device: a workspace is reallocated on
    // the device of its next use, which synchronizes first
    (void)hipEventDestroy(g_ws_ev[k]);
    g_ws_ev[k] = nullptr;
  }
  if (!g_ws_ev[k]) {
    if (hipEventCreateWithFlags(&g_ws_ev[k], hipEventDisableTiming) != hipSuccess)
      return fail(RT_E_DEVICE, "event creation failed");
    g_ws_evdev[k] = dev;
    return RT_OK;
  }
  if (hipStreamWaitEvent(s, g_ws_ev[k], 0) != hipSuccess) return fail(RT_E_DEVICE, "stream wait failed");
  return RT_OK;
}

void ws_done(int k, hipStream_t s) { (void)hipEventRecord(g_ws_ev[k], s); }
int g_num_cu = 0;

// integrator timing (rt_profile_*): event pairs around every transit launch
struct ProfEvent {
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfEvent> g_prof;

void prof_begin(hipStream_t s, ProfEvent &pe, bool &on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  on = g_prof_on;
  if (!on) return;
  if (hipEventCreate(&pe.a) != hipSuccess || hipEventCreate(&pe.b) != hipSuccess) {
    on = false;
    return;
  }
  (void)hipEventRecord(pe.a, s);
}

void prof_end(hipStream_t s, ProfEvent &pe, bool on) {
  if (!on) return;
  (void)hipEventRecord(pe.b, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.push_back(pe);
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Work table of NSEG segments of `cap` slots at the start of a device
// buffer: SoA doubles (x, v, t, opl0, hres, wt), ints (nsteps, bounces,
// status, kind), the 64-bit sample keys, the queue and sort keys, the
// counters and the sort's per-(key, block) counts. table_bytes(cap) is its
// size.
constexpr size_t table_bytes(long long cap) {
  return ((sizeof(double) * 10 * NSEG * cap + 255) & ~(size_t)255) +
         ((sizeof(int) * 4 * NSEG * cap + 255) & ~(size_t)255) +
         ((sizeof(long long) * NSEG * cap + 255) & ~(size_t)255) +
         ((sizeof(int) * 2 * NSEG * cap + 255) & ~(size_t)255) +
         ((sizeof(unsigned int) * C_COUNT + 255) & ~(size_t)255) +
         ((sizeof(unsigned int) * NBIN * SORT_BLOCKS + 255) & ~(size_t)255);
}

Table table_at(char *b, long long cap) {
  const long long ns = (long long)NSEG * cap;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  const size_t o_d = take(sizeof(double) * 10 * ns);
  const size_t o_i = take(sizeof(int) * 4 * ns);
  const size_t o_k = take(sizeof(long long) * ns);
  const size_t o_q = take(sizeof(int) * 2 * ns);
  const size_t o_c = take(sizeof(unsigned int) * C_COUNT);
  const size_t o_b = take(sizeof(unsigned int) * NBIN * SORT_BLOCKS);
  Table T{};
  double *D = (double *)(b + o_d);
  T.px = D; T.py = D + ns; T.pz = D + 2 * ns; T.vx = D + 3 * ns; T.vy = D + 4 * ns; T.vz = D + 5 * ns;
  T.t = D + 6 * ns; T.opl0 = D + 7 * ns; T.hres = D + 8 * ns; T.wt = D + 9 * ns;
  int *I = (int *)(b + o_i);
  T.nsteps = I; T.bounces = I + ns; T.status = I + 2 * ns; T.kind = I + 3 * ns;
  T.key = (long long *)(b + o_k);
  T.order = (int *)(b + o_q);
  T.key0 = T.order + ns;
  T.ctr = (unsigned int *)(b + o_c);
  T.bh = (unsigned int *)(b + o_b);
  T.cap = cap;
  return T;
}

void ws_free(Workspace &ws) {
  if (ws.base) {
    (void)hipDeviceSynchronize();
    (void)hipFree(ws.base);
  }
  ws = Workspace{};
}

// Make `ws` hold NSEG segments of `cap` slots, `codes_len` code bytes and
// `ncam` camera records (grows, never shrinks; synchronous hipMalloc).
int ws_reserve(Workspace &ws, long long cap, long long codes_len, int ncam) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RT_E_DEVICE, "hipGetDevice failed");
  if (ws.base && ws.device == dev && ws.cap >= cap && ws.codes_len >= codes_len && ws.cams_cap >= ncam)
    return RT_OK;
  if (ws.device == dev) {
    cap = std::max(cap, ws.cap);
    codes_len = std::max(codes_len, ws.codes_len);
    ncam = std::max(ncam, ws.cams_cap);
  }
  cap = std::max(cap, 1024LL);
  codes_len = std::max(codes_len, 1024LL);
  ncam = std::max(ncam, 16);
  ws_free(ws);
  size_t off = table_bytes(cap);
  auto take = [&](size_t b) { size_t o = off; off = align_up(off + b); return o; };
  size_t o_codes = take((size_t)codes_len);
  size_t o_topl = take(sizeof(float) * (size_t)codes_len);
  size_t o_twt = take(sizeof(float) * (size_t)codes_len);
  size_t o_grho = take(sizeof(float) * (size_t)codes_len);
  size_t o_cams = take(sizeof(CamP) * ncam);
  size_t o_tab = take(sizeof(float) * 64);
  void *p = nullptr;
  if (hipMalloc(&p, off) != hipSuccess) {
    (void)hipGetLastError();
    return fail(RT_E_NOMEM, "hipMalloc of %zu bytes for the workspace failed", off);
  }
  char *b = (char *)p;
  ws.T = table_at(b, cap);
  ws.base = p;
  ws.bytes = off;
  ws.cap = cap;
  ws.codes = (unsigned char *)(b + o_codes);
  ws.topl = (float *)(b + o_topl);
  ws.twt = (float *)(b + o_twt);
  ws.grho = (float *)(b + o_grho);
  ws.codes_len = codes_len;
  ws.cams = (CamP *)(b + o_cams);
  ws.cams_cap = ncam;
  ws.table = (float *)(b + o_tab);
  ws.device = dev;
  return RT_OK;
}

int num_cu() {
  if (g_num_cu == 0) {
    int dev = 0, n = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    g_num_cu = n;
  }
  return g_num_cu;
}

int check_desc(const rt_cloak_desc *d) {
  if (!d) return fail(RT_E_INVALID, "cloak description is NULL");
  if (!(d->r1 > 0.0) || !(d->r2 > d->r1) || !std::isfinite(d->r2))
    return fail(RT_E_INVALID, "need 0 < r1 < r2 < inf (got r1=%g r2=%g)", d->r1, d->r2);
  if (!(d->z1 > d->z0)) return fail(RT_E_INVALID, "need z0 < z1 (got %g, %g)", d->z0, d->z1);
  if (d->axis != RT_AXIS_RADIAL && d->axis != RT_AXIS_AZIMUTHAL)
    return fail(RT_E_INVALID, "axis must be RT_AXIS_RADIAL or RT_AXIS_AZIMUTHAL (got %d)", d->axis);
  if (d->inner_mirror != 0 && d->inner_mirror != 1)
    return fail(RT_E_INVALID, "inner_mirror must be 0 or 1");
  return RT_OK;
}

CloakP make_cloak(const rt_cloak_desc &d) {
  CloakP c;
  c.a = d.r1; c.b = d.r2; c.z0 = d.z0; c.z1 = d.z1;
  double q = d.r2 / (d.r2 - d.r1);
  c.kappa = q * q;
  c.a2 = d.r1 * d.r1; c.b2 = d.r2 * d.r2;
  c.inv_a = 1.0 / d.r1; c.inv_b = 1.0 / d.r2;
  c.axis = d.axis; c.mirror = d.inner_mirror;
  return c;
}

int check_opts(const rt_trace_opts *o, double r2, bool need_rout) {
  if (!o) return fail(RT_E_INVALID, "options are NULL");
  if (o->scheme != RT_SCHEME_RK4 && o->scheme != RT_SCHEME_DP45 && o->scheme != RT_SCHEME_RK4_HAM &&
      o->scheme != RT_SCHEME_RK4_HAMC)
    return fail(RT_E_INVALID, "scheme must be RT_SCHEME_RK4, RT_SCHEME_DP45, RT_SCHEME_RK4_HAM or RT_SCHEME_RK4_HAMC");
  if (o->precision != RT_PREC_FP64 && o->precision != RT_PREC_MIXED)
    return fail(RT_E_INVALID, "precision must be RT_PREC_FP64 or RT_PREC_MIXED");
  if (o->precision == RT_PREC_MIXED)
    return fail(RT_E_UNSUPPORTED, "RT_PREC_MIXED is not supported: an FP32 derivative misses the 1e-6 exit bar "
                                  "and issues no faster than FP64 on this GPU; use RT_PREC_FP64");
  if (!(o->h > 0.0) || !std::isfinite(o->h)) return fail(RT_E_INVALID, "h must be > 0");
  if (o->scheme == RT_SCHEME_DP45) {
    if (!(o->rtol > 0.0) || !(o->atol > 0.0)) return fail(RT_E_INVALID, "rtol and atol must be > 0");
    if (!(o->hmax >= o->h)) return fail(RT_E_INVALID, "hmax must be >= h");
  }
  if (need_rout && !(o->r_out >= r2)) return fail(RT_E_INVALID, "r_out (%g) must be >= r2 (%g)", o->r_out, r2);
  if (o->max_steps < 1) return fail(RT_E_INVALID, "max_steps must be >= 1");
  if (o->max_bounces < 0 || o->max_bounces > MAX_BOUNCES)
    return fail(RT_E_INVALID, "max_bounces must be in [0, %d]", MAX_BOUNCES);
  if (o->block != 0 && (o->block < 64 || o->block > 256 || o->block % 64))
    return fail(RT_E_INVALID, "block must be 0 or a multiple of 64 in [64, 256]");
  if (o->refill_period < 0 || o->refill_period > 1024)
    return fail(RT_E_INVALID, "refill_period must be in [0, 1024]");
  if (o->max_chunk < 0 || o->max_chunk > (1 << 28)) return fail(RT_E_INVALID, "max_chunk must be in [0, 2^28]");
  return RT_OK;
}

OptsP make_opts(const rt_trace_opts &o) {
  OptsP p;
  p.h0 = o.h; p.rtol = o.rtol; p.atol = o.atol; p.hmax = o.scheme == RT_SCHEME_DP45 ? o.hmax : o.h;
  p.r_out = o.r_out;
  p.max_steps = o.max_steps;
  p.scheme = o.scheme; p.precision = o.precision; p.max_bounces = o.max_bounces; p.pad = 0;
  return p;
}

int launch_err(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return RT_OK;
}

unsigned int grid_for(long long n, int block) {
  long long g = (n + block - 1) / block;
  return (unsigned int)std::max(1LL, g);
}

template <bool HAM, bool FRES>
unsigned int transit_grid_t(int block) {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_transit<HAM, FRES>, block, 0) != hipSuccess || occ <= 0)
    occ = 1;
  return (unsigned int)(num_cu() * occ);
}

// the integrator variant the options select: Eq. (8) in (x, v) or the
// Hamiltonian form, with or without the Eq. (12) weights
unsigned int transit_grid(const OptsP &o, int block, bool fres = false) {
  if (o.scheme == RT_SCHEME_RK4_HAM || o.scheme == RT_SCHEME_RK4_HAMC)
    return fres ? transit_grid_t<true, true>(block) : transit_grid_t<true, false>(block);
  return fres ? transit_grid_t<false, true>(block) : transit_grid_t<false, false>(block);
}

// integrate the slots already placed in the table: order them hardest
// first, then one persistent integrator launch (kernel launches only)
void run_transit(const CloakP &c, const OptsP &o, const Table &T, int block, int refill,
                 unsigned int grid, hipStream_t s, bool profile, bool fres = false) {
  hipLaunchKernelGGL(k_sort_hist, dim3(SORT_BLOCKS), dim3(SORT_THREADS), 0, s, T);
  hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(SORT_THREADS), 0, s, T);
  hipLaunchKernelGGL(k_sort_scatter, dim3(SORT_BLOCKS), dim3(SORT_THREADS), 0, s, T);
  ProfEvent pe;
  bool on = false;
  if (profile) prof_begin(s, pe, on);
  const bool ham = o.scheme == RT_SCHEME_RK4_HAM || o.scheme == RT_SCHEME_RK4_HAMC;
  if (ham && fres)
    hipLaunchKernelGGL((k_transit<true, true>), dim3(grid), dim3(block), 0, s, c, o, T, refill);
  else if (ham)
    hipLaunchKernelGGL((k_transit<true, false>), dim3(grid), dim3(block), 0, s, c, o, T, refill);
  else if (fres)
    hipLaunchKernelGGL((k_transit<false, true>), dim3(grid), dim3(block), 0, s, c, o, T, refill);
  else
    hipLaunchKernelGGL((k_transit<false, false>), dim3(grid), dim3(block), 0, s, c, o, T, refill);
  if (profile) prof_end(s, pe, on);
}

// launch shapes chosen by rt_autotune_render, keyed by the batch's shape
struct TuneKey {
  int n_cloaks, n_cams, w, h, spp, pol_mask, scheme, precision;
  bool operator<(const TuneKey &k) const {
    return std::tie(n_cloaks, n_cams, w, h, spp, pol_mask, scheme, precision) <
           std::tie(k.n_cloaks, k.n_cams, k.w, k.h, k.spp, k.pol_mask, k.scheme, k.precision);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tuned;

// A render call prepared on the host: validated inputs, camera bases, colour
// table and launch shape. enqueue_render only launches kernels (no
// allocation, no synchronization), so it can be captured into a HIP graph.
struct RenderJob {
  CloakP c{};
  OptsP o{};
  RoomP rm{};
  RenderP R{};
  std::vector<CamP> cams;
  float table[64] = {0};
  long long total = 0, chunk = 0, npix = 0;
  int n_cloaks = 0, block = 256, refill = 2;
  unsigned int grid = 0;
  TuneKey key{};
};

}  // namespace

struct rt_plan_s {
  RenderJob J;
  Workspace ws;
  float *rgb = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

int prepare_render(const rt_cloak *cloaks, int32_t n_cloaks, const rt_trace_opts *opts,
                   const rt_room *room, const rt_camera *cams, int32_t n_cams, int32_t pol_mask,
                   const rt_render_aux *aux, RenderJob &J) {
  if (n_cloaks < 0 || n_cloaks > 2) return fail(RT_E_INVALID, "n_cloaks must be 0, 1 or 2");
  if (n_cloaks > 0 && !cloaks) return fail(RT_E_INVALID, "cloaks is NULL");
  for (int k = 0; k < n_cloaks; ++k)
    if (!cloaks[k]) return fail(RT_E_INVALID, "cloak handle %d is NULL", k);
  for (int k = 1; k < n_cloaks; ++k) {
    const rt_cloak_desc &a = cloaks[0]->d, &b = cloaks[k]->d;
    if (a.r1 != b.r1 || a.r2 != b.r2 || a.z0 != b.z0 || a.z1 != b.z1 || a.inner_mirror != b.inner_mirror)
      return fail(RT_E_INVALID, "cloaks of one call must share r1, r2, z0, z1 and inner_mirror");
  }
  double r2 = n_cloaks ? cloaks[0]->d.r2 : 0.0;
  int e = check_opts(opts, r2, false);
  if (e) return e;
  if (!room || !cams) return fail(RT_E_INVALID, "room and cams are required");
  if (n_cams < 1) return fail(RT_E_INVALID, "n_cams must be >= 1");
  if (pol_mask < 1 || pol_mask > 3) return fail(RT_E_INVALID, "pol_mask must be 1, 2 or 3");
  if (!(room->tile > 0.0)) return fail(RT_E_INVALID, "room tile must be > 0");
  for (int k = 0; k < 3; ++k)
    if (!(room->hi[k] > room->lo[k])) return fail(RT_E_INVALID, "room needs lo < hi");
  const int w = cams[0].w, h = cams[0].h, spp = cams[0].spp;
  int m = (int)std::lround(std::sqrt((double)spp));
  if (w < 1 || h < 1 || spp < 1 || m * m != spp || spp > 256)
    return fail(RT_E_INVALID, "camera needs w, h >= 1 and spp a perfect square <= 256");
  for (int k = 1; k < n_cams; ++k)
    if (cams[k].w != w || cams[k].h != h || cams[k].spp != spp)
      return fail(RT_E_INVALID, "all cameras must share w, h and spp");
  const long long npix = (long long)w * h;
  const long long ns_img = npix * spp;
  if (ns_img > (1LL << 30)) return fail(RT_E_INVALID, "w*h*spp must be <= 2^30");
  const int npol = (pol_mask == 3) ? 2 : 1;
  const int ncl = n_cloaks > 0 ? n_cloaks : 1;  // the empty room renders as one image set

  J.cams.resize(n_cams);
  for (int k = 0; k < n_cams; ++k) {
    const rt_camera &C = cams[k];
    double F[3], R[3], U[3];
    for (int j = 0; j < 3; ++j) F[j] = C.look[j] - C.eye[j];
    double fl = std::sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
    if (!(fl > 0.0) || !(C.fov_deg > 0.0 && C.fov_deg < 180.0))
      return fail(RT_E_INVALID, "camera %d: eye == look or fov outside (0, 180)", k);
    for (int j = 0; j < 3; ++j) F[j] /= fl;
    R[0] = F[1] * C.up[2] - F[2] * C.up[1];
    R[1] = F[2] * C.up[0] - F[0] * C.up[2];
    R[2] = F[0] * C.up[1] - F[1] * C.up[0];
    double rl = std::sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    if (!(rl > 0.0)) return fail(RT_E_INVALID, "camera %d: up is parallel to the view direction", k);
    for (int j = 0; j < 3; ++j) R[j] /= rl;
    U[0] = R[1] * F[2] - R[2] * F[1];
    U[1] = R[2] * F[0] - R[0] * F[2];
    U[2] = R[0] * F[1] - R[1] * F[0];
    CamP &P = J.cams[k];
    for (int j = 0; j < 3; ++j) { P.eye[j] = C.eye[j]; P.F[j] = F[j]; P.R[j] = R[j]; P.U[j] = U[j]; }
    P.tan_half = std::tan(0.5 * C.fov_deg * M_PI / 180.0);
    P.aspect = (double)w / (double)h;
    P.inv_w = (w & (w - 1)) == 0 ? 1.0 / w : 0.0;
    P.inv_h = (h & (h - 1)) == 0 ? 1.0 / h : 0.0;
    P.w = w; P.h = h; P.spp = spp; P.m = m;
    P.seed = C.seed;
  }
  if (n_cloaks) J.c = make_cloak(cloaks[0]->d);
  J.o = make_opts(*opts);
  for (int j = 0; j < 3; ++j) { J.rm.lo[j] = room->lo[j]; J.rm.hi[j] = room->hi[j]; }
  J.rm.tile = room->tile;
  J.rm.inv_tile = 1.0 / room->tile;
  {
    int ex = 0;
    J.rm.tile_pow2 = std::frexp(room->tile, &ex) == 0.5 ? 1 : 0;  // tile = 2^(ex-1)
    J.rm.pad = 0;
  }
  for (int f = 0; f < 6; ++f)
    for (int q = 0; q < 2; ++q)
      for (int j = 0; j < 3; ++j) J.table[(f * 2 + q) * 3 + j] = room->rgb[f][q][j];
  J.total = ns_img * n_cams;
  // samples per chunk: one integrator launch each. Rays whose paths pass
  // very close to r = a take tens of thousands of attempts; they are sorted
  // first and run alongside the rest of their launch, so fewer, larger
  // launches hide them (a 4096^2 x 4 spp frame is one chunk; the work table
  // then takes ~0.5 KB per sample, ~31 GB)
  const long long chunk_max = (opts->max_chunk > 0 ? (long long)opts->max_chunk : (1LL << 26)) / spp * spp;
  J.chunk = std::min(J.total, std::max(chunk_max, (long long)spp));
  J.npix = npix;
  J.n_cloaks = n_cloaks;
  J.key = TuneKey{n_cloaks, n_cams, w, h, spp, pol_mask, opts->scheme, opts->precision};
  J.block = opts->block ? opts->block : 256;
  J.refill = opts->refill_period ? opts->refill_period : 2;
  if (!opts->block && !opts->refill_period) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(J.key);
    if (it != g_tuned.end()) { J.block = it->second.first; J.refill = it->second.second; }
  }
  const bool unpol = aux && aux->unpol;
  const bool goggles = aux && (aux->goggle_inplane || aux->goggle_axial);
  const bool weights = unpol || goggles;  // the Eq. (12) weights ride in the integrator
  J.grid = transit_grid(J.o, J.block, weights);
  RenderP &R = J.R;
  R.ns_img = ns_img; R.n_cams = n_cams; R.ncl = ncl; R.npol = npol; R.spp = spp;
  R.axis[0] = n_cloaks > 0 ? cloaks[0]->d.axis : 0;
  R.axis[1] = n_cloaks > 1 ? cloaks[1]->d.axis : 0;
  R.pol[0] = (pol_mask & 1) ? RT_POL_ORDINARY : RT_POL_EXTRAORDINARY;
  R.pol[1] = RT_POL_EXTRAORDINARY;
  R.has_cloak = n_cloaks > 0 ? 1 : 0;
  R.idx32 = ns_img * n_cams <= 0xffffffffLL ? 1 : 0;
  R.codes = nullptr;
  R.rec = aux ? aux->rec : nullptr;
  R.st = aux ? aux->status : nullptr;
  R.code = aux ? aux->code : nullptr;
  R.nsteps = aux ? aux->nsteps : nullptr;
  R.tof = aux ? aux->tof : nullptr;
  R.topl = nullptr;
  R.unpol = unpol ? aux->unpol : nullptr;
  R.gog[0] = goggles ? aux->goggle_inplane : nullptr;
  R.gog[1] = goggles ? aux->goggle_axial : nullptr;
  R.twt = nullptr;
  R.grho = nullptr;
  if (weights && npol != 2)
    return fail(RT_E_UNSUPPORTED, "the unpolarized and goggle images need both branches (pol_mask = 3)");
  if (weights && opts->precision != RT_PREC_FP64)
    return fail(RT_E_UNSUPPORTED, "the Eq. (12) weights are computed in FP64 only");
  R.refl = aux && aux->reflections ? 1 : 0;
  R.rext = R.rgin = R.cw = nullptr;
  R.rcode = R.ccode = nullptr;
  if (R.refl && !weights)
    return fail(RT_E_INVALID, "first-order reflections need the unpolarized or a goggle image");
  // the reflected waves' table holds up to two children per primary and
  // segment: chunks of at most 2^22 samples keep it near 4 GB
  if (R.refl) J.chunk = std::min(J.chunk, std::max((long long)spp, REFL_CHUNK / spp * spp));
  return RT_OK;
}

int ws_reserve_for(Workspace &ws, const RenderJob &J) {
  return ws_reserve(ws, J.chunk, J.chunk * J.R.ncl * J.R.npol, (int)J.cams.size());
}

// copy the job's camera records and colour table into the workspace
// (synchronous: the host vectors may be freed afterwards)
int upload_job(const RenderJob &J, const Workspace &ws, hipStream_t s) {
  if (hipMemcpyAsync(ws.cams, J.cams.data(), sizeof(CamP) * J.cams.size(), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemcpyAsync(ws.table, J.table, sizeof(float) * 39, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(RT_E_DEVICE, "upload of camera records failed");
  return RT_OK;
}

// First-order reflections: the child table (two children per primary and
// segment at most) and the chunk-local reflection arrays (grows, never
// shrinks)
struct ReflWs {
  void *base = nullptr;
  long long chunk = 0, len = 0;
  int device = -1;
  Table Tc{};
  float *rext = nullptr, *rgin = nullptr, *cw = nullptr;
  unsigned char *rcode = nullptr, *ccode = nullptr;
};
ReflWs g_rws;

int rws_reserve(ReflWs &w, long long chunk, long long len) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RT_E_DEVICE, "hipGetDevice failed");
  if (w.base && w.device == dev && w.chunk >= chunk && w.len >= len) return RT_OK;
  if (w.base) {
    (void)hipDeviceSynchronize();
    (void)hipFree(w.base);
    w = ReflWs{};
  }
  size_t off = table_bytes(2 * chunk);
  auto take = [&](size_t b) { size_t o = off; off = align_up(off + b); return o; };
  const size_t o_re = take(sizeof(float) * len), o_ri = take(sizeof(float) * len);
  const size_t o_cw = take(sizeof(float) * 2 * len), o_rc = take((size_t)len), o_cc = take((size_t)(2 * len));
  void *p = nullptr;
  if (hipMalloc(&p, off) != hipSuccess) {
    (void)hipGetLastError();
    return fail(RT_E_NOMEM, "hipMalloc of %zu bytes for the reflected waves failed", off);
  }
  char *b = (char *)p;
  w.base = p;
  w.chunk = chunk;
  w.len = len;
  w.device = dev;
  w.Tc = table_at(b, 2 * chunk);
  w.rext = (float *)(b + o_re);
  w.rgin = (float *)(b + o_ri);
  w.cw = (float *)(b + o_cw);
  w.rcode = (unsigned char *)(b + o_rc);
  w.ccode = (unsigned char *)(b + o_cc);
  return RT_OK;
}

// any per-sample output of the camera-ray and finish kernels besides the
// colour codes (selects the instantiations that write them)
bool sample_outputs(const RenderP &R) {
  return R.twt || R.topl || R.st || R.code || R.nsteps || R.rec;
}

// fixed grid of the grid-stride plain resolve kernel: a few times the
// blocks the chip holds at once, fewer when the chunk is small
unsigned int resolve_grid(long long nres) {
  return std::min(grid_for(nres, 256), (unsigned int)num_cu() * 16);
}

// any per-pixel image besides the colour image (time of flight,
// unpolarized, goggles): the general resolve kernel makes them
bool pixel_images(const RenderP &R) {
  return R.tof || R.unpol || R.grho || R.gog[0] || R.gog[1];
}

void enqueue_render(const RenderJob &J, const Workspace &ws, float *rgb, hipStream_t s, bool profile,
                    const ReflWs *rw = nullptr) {
  const Table &T = ws.T;
  RenderP R = J.R;
  R.codes = ws.codes;
  R.topl = R.tof ? ws.topl : nullptr;
  const bool goggles = R.gog[0] || R.gog[1];
  R.twt = R.unpol || goggles ? ws.twt : nullptr;
  R.grho = goggles ? ws.grho : nullptr;
  R.refl = R.refl && rw ? 1 : 0;
  if (R.refl) {
    R.rext = rw->rext;
    R.rgin = goggles ? rw->rgin : nullptr;
    R.cw = rw->cw;
    R.rcode = rw->rcode;
    R.ccode = rw->ccode;
  }
  for (long long g0 = 0; g0 < J.total; g0 += J.chunk) {
    R.g0 = g0;
    R.g1 = std::min(J.total, g0 + J.chunk);
    hipLaunchKernelGGL(k_zero, dim3((C_COUNT + 255) / 256), dim3(256), 0, s, T.ctr, (int)C_COUNT);
    if (R.grho)
      hipLaunchKernelGGL((k_rd_gen<false, 2, true>), dim3(grid_for(R.g1 - R.g0, 256)), dim3(256), 0, s, J.c, J.o,
                         J.rm, ws.cams, T, R, CandP{});
    else if (R.twt || R.refl)
      hipLaunchKernelGGL((k_rd_gen<false, 1, true>), dim3(grid_for(R.g1 - R.g0, 256)), dim3(256), 0, s, J.c, J.o,
                         J.rm, ws.cams, T, R, CandP{});
    else if (sample_outputs(R))
      hipLaunchKernelGGL((k_rd_gen<false, 0, true>), dim3(grid_for(R.g1 - R.g0, 256)), dim3(256), 0, s, J.c, J.o,
                         J.rm, ws.cams, T, R, CandP{});
    else
      hipLaunchKernelGGL((k_rd_gen<false, 0, false>), dim3(grid_for(R.g1 - R.g0, 256)), dim3(256), 0, s, J.c, J.o,
                         J.rm, ws.cams, T, R, CandP{});
    if (J.n_cloaks) {
      run_transit(J.c, J.o, T, J.block, J.refill, J.grid, s, profile, R.twt != nullptr);
      if (sample_outputs(R))
        hipLaunchKernelGGL(k_rd_finish<true>, dim3(num_cu() * 8), dim3(256), 0, s, J.c, J.rm, T, R);
      else
        hipLaunchKernelGGL(k_rd_finish<false>, dim3(num_cu() * 8), dim3(256), 0, s, J.c, J.rm, T, R);
      if (R.refl) {
        // the waves reflected at the exits, integrated as a second batch
        const Table &Tc = rw->Tc;
        hipLaunchKernelGGL(k_zero, dim3((C_COUNT + 255) / 256), dim3(256), 0, s, Tc.ctr, (int)C_COUNT);
        hipLaunchKernelGGL(k_rd_spawn, dim3(num_cu() * 8), dim3(256), 0, s, J.c, J.o, T, Tc, R);
        run_transit(J.c, J.o, Tc, J.block, J.refill, J.grid, s, profile, true);
        hipLaunchKernelGGL(k_rd_cfinish, dim3(num_cu() * 8), dim3(256), 0, s, J.c, J.rm, Tc, R);
      }
    }
    long long nres = (R.g1 - R.g0) / R.spp * R.ncl * R.npol;
    if (pixel_images(R))
      hipLaunchKernelGGL(k_rd_resolve, dim3(grid_for(nres, 256)), dim3(256), 0, s, R, ws.table, rgb,
                         J.npix);
    else
      hipLaunchKernelGGL(k_rd_resolve_plain, dim3(resolve_grid(nres)), dim3(256), 0, s, R, ws.table, rgb,
                         J.npix);
  }
}

// candidate rows of the surrogate render (grows, never shrinks)
struct CandWs {
  void *base = nullptr;
  long long cap = 0;
  int device = -1;
  CandP P{};
};
CandWs g_cws;

int cws_reserve(CandWs &w, long long cap) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RT_E_DEVICE, "hipGetDevice failed");
  if (w.base && w.device == dev && w.cap >= cap) return RT_OK;
  if (w.base) {
    (void)hipDeviceSynchronize();
    (void)hipFree(w.base);
    w = CandWs{};
  }
  cap = std::max(cap, 1024LL);
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off = align_up(off + b); return o; };
  const size_t o_x = take(sizeof(float) * 6 * cap), o_k = take(sizeof(long long) * cap);
  const size_t o_s = take(sizeof(float) * cap), o_y = take(sizeof(float) * 5 * cap);
  const size_t o_f = take((size_t)cap), o_t = take(sizeof(int) * cap);
  void *p = nullptr;
  if (hipMalloc(&p, off) != hipSuccess) {
    (void)hipGetLastError();
    return fail(RT_E_NOMEM, "hipMalloc of %zu bytes for the surrogate candidates failed", off);
  }
  char *b = (char *)p;
  w.base = p;
  w.cap = cap;
  w.device = dev;
  w.P.x6 = (float *)(b + o_x);
  w.P.ld = cap;
  w.P.key = (long long *)(b + o_k);
  w.P.s_in = (float *)(b + o_s);
  w.P.y5 = (float *)(b + o_y);
  w.P.fb = (unsigned char *)(b + o_f);
  w.P.st = (int *)(b + o_t);
  return RT_OK;
}

// One render with the surrogate: per chunk, generation (side entries become
// candidates), the network and its gate on the candidates, shading of the
// accepted ones and re-queueing of the rejected ones, then the integrator
// on the cap entries and the rejected side entries, shading and resolve as
// in enqueue_render. The candidate count is read back once per chunk (the
// network's launch is sized by it). counts[0] += candidates, counts[1] +=
// accepted.
int render_surrogate(rt_model model, const rt_cloak_desc &desc, const RenderJob &J, const Workspace &ws,
                     const CandWs &cw, int min_difficulty, float *rgb, hipStream_t s, long long counts[2]) {
  if (J.R.unpol || J.R.gog[0] || J.R.gog[1])
    return fail(RT_E_UNSUPPORTED, "the surrogate render makes no unpolarized or goggle image");
  const Table &T = ws.T;
  RenderP R = J.R;
  R.sur_min = min_difficulty;
  R.edge_tol = surrogate_exit_tolerance(model);
  R.codes = ws.codes;
  R.topl = R.tof ? ws.topl : nullptr;
  for (long long g0 = 0; g0 < J.total; g0 += J.chunk) {
    R.g0 = g0;
    R.g1 = std::min(J.total, g0 + J.chunk);
    hipLaunchKernelGGL(k_zero, dim3((C_COUNT + 255) / 256), dim3(256), 0, s, T.ctr, (int)C_COUNT);
    if (sample_outputs(R))
      hipLaunchKernelGGL((k_rd_gen<true, 0, true>), dim3(grid_for(R.g1 - R.g0, 256)), dim3(256), 0, s, J.c, J.o,
                         J.rm, ws.cams, T, R, cw.P);
    else
      hipLaunchKernelGGL((k_rd_gen<true, 0, false>), dim3(grid_for(R.g1 - R.g0, 256)), dim3(256), 0, s, J.c, J.o,
                         J.rm, ws.cams, T, R, cw.P);
    unsigned int nc = 0;
    if (hipMemcpyAsync(&nc, T.ctr + C_SUR, sizeof(nc), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(RT_E_DEVICE, "surrogate render: candidate count read-back failed");
    if ((long long)nc > cw.cap) return fail(RT_E_DEVICE, "surrogate render: candidate overflow");
    if (nc > 0) {
      int e = surrogate_predict_gated(model, desc, nc, cw.P.ld, cw.P.x6, cw.P.y5, cw.P.fb, cw.P.st, s);
      if (e) return e;
      hipLaunchKernelGGL(k_rd_sur_apply, dim3(grid_for(nc, 256)), dim3(256), 0, s, J.c, J.o, J.rm, ws.cams, T, R,
                         cw.P, nc);
    }
    run_transit(J.c, J.o, T, J.block, J.refill, J.grid, s, true);
    if (sample_outputs(R))
      hipLaunchKernelGGL(k_rd_finish<true>, dim3(num_cu() * 8), dim3(256), 0, s, J.c, J.rm, T, R);
    else
      hipLaunchKernelGGL(k_rd_finish<false>, dim3(num_cu() * 8), dim3(256), 0, s, J.c, J.rm, T, R);
    long long nres = (R.g1 - R.g0) / R.spp * R.ncl * R.npol;
    if (pixel_images(R))
      hipLaunchKernelGGL(k_rd_resolve, dim3(grid_for(nres, 256)), dim3(256), 0, s, R, ws.table, rgb, J.npix);
    else
      hipLaunchKernelGGL(k_rd_resolve_plain, dim3(resolve_grid(nres)), dim3(256), 0, s, R, ws.table, rgb,
                         J.npix);
    if (counts) {
      unsigned int na = 0;
      if (hipMemcpyAsync(&na, T.ctr + C_ACC, sizeof(na), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(RT_E_DEVICE, "surrogate render: accepted count read-back failed");
      counts[0] += nc;
      counts[1] += na;
    }
  }
  return RT_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free tracing: the work table of rt_trace_batch_noalloc lives in
// a file-scope device array instead of the library workspace. Host code may
// not use the array's name as a device address (it is a host-side stand-in);
// its address on each device comes from hipGetSymbolAddress, taken once per
// device with that device current and kept here.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_BYTES = table_bytes(RT_NOALLOC_MAX_RAYS);
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[MAX_DEVICES] = {nullptr};

int noalloc_scratch(char **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RT_E_DEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= MAX_DEVICES) return fail(RT_E_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(RT_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = (char *)p;
  }
  *out = g_scratch_ptr[dev];
  return RT_OK;
}

int check_trace_args(rt_cloak cloak, const rt_trace_opts *opts, int32_t pol, int64_t n, const double *in6,
                     const double *out6, const double *opl, const int32_t *status, const double *trans);
int enqueue_trace(rt_cloak cloak, const rt_trace_opts *opts, int32_t pol, int64_t n, const double *in6,
                  double *out6, double *opl, int32_t *status, double *hres, int32_t *nsteps, double *trans,
                  const Table &T, hipStream_t s, bool profile);

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
void rt_set_error_message(const char *msg) { g_err = msg; }

extern "C" {

const char *rt_last_error(void) { return g_err.c_str(); }

int rt_build_cloak(const rt_cloak_desc *desc, rt_cloak *out) {
  if (!out) return fail(RT_E_INVALID, "out is NULL");
  *out = nullptr;
  int e = check_desc(desc);
  if (e) return e;
  rt_cloak h = new (std::nothrow) rt_cloak_s;
  if (!h) return fail(RT_E_NOMEM, "host allocation failed");
  h->d = *desc;
  *out = h;
  return RT_OK;
}

int rt_cloak_get_desc(rt_cloak cloak, rt_cloak_desc *out) {
  if (!cloak || !out) return fail(RT_E_INVALID, "cloak and out are required");
  *out = cloak->d;
  return RT_OK;
}

int rt_free_cloak(rt_cloak cloak) {
  delete cloak;
  return RT_OK;
}

int rt_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return RT_OK;
}

int rt_profile_read(double *transit_ms, int64_t *launches) {
  if (!transit_ms || !launches) return fail(RT_E_INVALID, "outputs are NULL");
  std::vector<ProfEvent> ev;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    ev.swap(g_prof);
  }
  double tot = 0.0;
  int err = RT_OK;
  for (auto &pe : ev) {
    float ms = 0.f;
    if (hipEventSynchronize(pe.b) != hipSuccess || hipEventElapsedTime(&ms, pe.a, pe.b) != hipSuccess)
      err = fail(RT_E_DEVICE, "event timing failed");
    tot += ms;
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
  *transit_ms = tot;
  *launches = (int64_t)ev.size();
  return err;
}

int rt_release_workspace(void) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  ws_free(g_ws);
  for (int j = 0; j < NWS - 1; ++j) ws_free(g_wsx[j]);
  if (g_rws.base) {
    (void)hipDeviceSynchronize();
    (void)hipFree(g_rws.base);
    g_rws = ReflWs{};
  }
  if (g_cws.base) {
    (void)hipDeviceSynchronize();
    (void)hipFree(g_cws.base);
    g_cws = CandWs{};
  }
  return RT_OK;
}

int rt_trace_batch(rt_cloak cloak, const rt_trace_opts *opts, int32_t pol, int64_t n,
                   const double *in6, double *out6, double *opl, int32_t *status, double *hres,
                   int32_t *nsteps, double *trans, void *stream) {
  int e = check_trace_args(cloak, opts, pol, n, in6, out6, opl, status, trans);
  if (e || n == 0) return e;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  e = ws_order(0, (hipStream_t)stream);
  if (!e) e = ws_reserve(g_ws, n, 0, 0);
  if (e) return e;
  e = enqueue_trace(cloak, opts, pol, n, in6, out6, opl, status, hres, nsteps, trans, g_ws.T,
                    (hipStream_t)stream, true);
  ws_done(0, (hipStream_t)stream);
  return e;
}

int rt_trace_batch_noalloc(rt_cloak cloak, const rt_trace_opts *opts, int32_t pol, int64_t n,
                           const double *in6, double *out6, double *opl, int32_t *status, double *hres,
                           int32_t *nsteps, double *trans, void *stream) {
  int e = check_trace_args(cloak, opts, pol, n, in6, out6, opl, status, trans);
  if (e || n == 0) return e;
  if (n > RT_NOALLOC_MAX_RAYS)
    return fail(RT_E_INVALID, "rt_trace_batch_noalloc takes at most %d rays per call (got %lld)",
                RT_NOALLOC_MAX_RAYS, (long long)n);
  char *base = nullptr;
  e = noalloc_scratch(&base);
  if (e) return e;
  return enqueue_trace(cloak, opts, pol, n, in6, out6, opl, status, hres, nsteps, trans,
                       table_at(base, RT_NOALLOC_MAX_RAYS), (hipStream_t)stream, false);
}

}  // extern "C"

namespace {

int check_trace_args(rt_cloak cloak, const rt_trace_opts *opts, int32_t pol, int64_t n, const double *in6,
                     const double *out6, const double *opl, const int32_t *status, const double *trans) {
  if (!cloak) return fail(RT_E_INVALID, "cloak handle is NULL");
  int e = check_opts(opts, cloak->d.r2, true);
  if (e) return e;
  if (pol != RT_POL_ORDINARY && pol != RT_POL_EXTRAORDINARY)
    return fail(RT_E_INVALID, "pol must be RT_POL_ORDINARY or RT_POL_EXTRAORDINARY");
  if (n < 0) return fail(RT_E_INVALID, "n must be >= 0");
  if (n == 0) return RT_OK;
  if (n > (1LL << 30)) return fail(RT_E_INVALID, "n must be <= 2^30 per call");
  if (!in6 || !out6 || !opl || !status) return fail(RT_E_INVALID, "in6, out6, opl and status are required");
  if (trans && opts->precision != RT_PREC_FP64)
    return fail(RT_E_UNSUPPORTED, "the Eq. (12) weights are computed in FP64 only");
  return RT_OK;
}

// the rt_trace_batch pipeline on a work table of at least n slots per
// segment (kernel launches only: no allocation, no synchronization)
int enqueue_trace(rt_cloak cloak, const rt_trace_opts *opts, int32_t pol, int64_t n, const double *in6,
                  double *out6, double *opl, int32_t *status, double *hres, int32_t *nsteps, double *trans,
                  const Table &T, hipStream_t s, bool profile) {
  int e = RT_OK;
  CloakP c = make_cloak(cloak->d);
  OptsP o = make_opts(*opts);
  int block = opts->block ? opts->block : 256;
  int refill = opts->refill_period ? opts->refill_period : 2;
  int kind = c.axis * 2 + pol;
  const bool fres = trans != nullptr;
  unsigned int grid = transit_grid(o, block, fres);
  hipLaunchKernelGGL(k_zero, dim3((C_COUNT + 255) / 256), dim3(256), 0, s, T.ctr, (int)C_COUNT);
  hipLaunchKernelGGL(k_tb_entry, dim3(grid_for(n, 256)), dim3(256), 0, s, c, o, T, kind, (long long)n,
                     in6, out6, opl, status, hres, nsteps, trans);
  e = launch_err("entry launch");
  if (e) return e;
  run_transit(c, o, T, block, refill, grid, s, profile, fres);
  e = launch_err("transit launch");
  if (e) return e;
  hipLaunchKernelGGL(k_tb_finish, dim3(num_cu() * 8), dim3(256), 0, s, c, o, T, (long long)n, out6,
                     opl, status, hres, nsteps, trans);
  return launch_err("finish launch");
}

}  // namespace

extern "C" {

int rt_transit_exact(const rt_cloak *cloaks, int32_t n_cloaks, const rt_trace_opts *opts, int64_t n,
                     int64_t ld, const float *x6, const uint8_t *mask, float *y5, int32_t *status,
                     float *hres, int32_t *nsteps, void *stream) {
  if (n_cloaks < 1 || n_cloaks > 2 || !cloaks) return fail(RT_E_INVALID, "need 1 or 2 cloak handles");
  for (int k = 0; k < n_cloaks; ++k)
    if (!cloaks[k]) return fail(RT_E_INVALID, "cloak handle %d is NULL", k);
  int have_axes = 0;
  for (int k = 0; k < n_cloaks; ++k) {
    const rt_cloak_desc &a = cloaks[0]->d, &b = cloaks[k]->d;
    if (a.r1 != b.r1 || a.r2 != b.r2 || a.z0 != b.z0 || a.z1 != b.z1 || a.inner_mirror != b.inner_mirror)
      return fail(RT_E_INVALID, "cloaks of one call must share r1, r2, z0, z1 and inner_mirror");
    if (have_axes & (1 << b.axis)) return fail(RT_E_INVALID, "two cloaks with the same optic axis");
    have_axes |= 1 << b.axis;
  }
  int e = check_opts(opts, cloaks[0]->d.r2, false);
  if (e) return e;
  if (n < 0) return fail(RT_E_INVALID, "n must be >= 0");
  if (n == 0) return RT_OK;
  if (n > (1LL << 28)) return fail(RT_E_INVALID, "n must be <= 2^28 per call");
  if (ld < n) return fail(RT_E_INVALID, "ld must be >= n");
  if (!x6 || !y5 || !status) return fail(RT_E_INVALID, "x6, y5 and status are required");
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  e = ws_order(0, s);
  if (!e) e = ws_reserve(g_ws, n, 0, 0);
  if (e) return e;
  const Table &T = g_ws.T;
  CloakP c = make_cloak(cloaks[0]->d);
  OptsP o = make_opts(*opts);
  int block = opts->block ? opts->block : 256;
  int refill = opts->refill_period ? opts->refill_period : 2;
  unsigned int grid = transit_grid(o, block);
  hipLaunchKernelGGL(k_zero, dim3((C_COUNT + 255) / 256), dim3(256), 0, s, T.ctr, (int)C_COUNT);
  hipLaunchKernelGGL(k_sx_entry, dim3(grid_for(n, 256)), dim3(256), 0, s, c, o, T, (long long)n,
                     (long long)ld, x6, mask, have_axes, y5, status, hres, nsteps);
  e = launch_err("entry launch");
  if (!e) {
    run_transit(c, o, T, block, refill, grid, s, true);
    e = launch_err("transit launch");
  }
  if (!e) {
    hipLaunchKernelGGL(k_sx_finish, dim3(num_cu() * 8), dim3(256), 0, s, c, T, (long long)ld, y5, status,
                       hres, nsteps);
    e = launch_err("finish launch");
  }
  ws_done(0, s);
  return e;
}

int rt_render_multi(const rt_cloak *cloaks, int32_t n_cloaks, const rt_trace_opts *opts,
                    const rt_room *room, const rt_camera *cams, int32_t n_cams, int32_t pol_mask,
                    float *rgb, const rt_render_aux *aux, void *stream) {
  if (!rgb) return fail(RT_E_INVALID, "rgb is required");
  RenderJob J;
  int e = prepare_render(cloaks, n_cloaks, opts, room, cams, n_cams, pol_mask, aux, J);
  if (e) return e;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  // the workspace this stream used last, else the one used longest ago
  // (renders with reflections stay on the first, beside their buffers)
  int k = 0;
  if (!J.R.refl) {
    k = -1;
    for (int j = 0; j < NWS && k < 0; ++j)
      if (g_ws_last[j] && g_ws_stream[j] == s) k = j;
    if (k < 0) {
      k = 0;
      for (int j = 1; j < NWS; ++j)
        if (g_ws_last[j] < g_ws_last[k]) k = j;
    }
  }
  g_ws_stream[k] = s;
  g_ws_last[k] = ++g_ws_calls;
  Workspace &ws = ws_at(k);
  e = ws_order(k, s);
  if (!e) e = ws_reserve_for(ws, J);
  if (!e && J.R.refl) e = rws_reserve(g_rws, J.chunk, J.chunk * J.R.ncl * J.R.npol);
  if (!e) e = upload_job(J, ws, s);
  if (e) return e;
  enqueue_render(J, ws, rgb, s, true, J.R.refl ? &g_rws : nullptr);
  ws_done(k, s);
  return launch_err("render launch");
}

int rt_render_surrogate(rt_model model, const rt_cloak *cloaks, int32_t n_cloaks, const rt_trace_opts *opts,
                        const rt_room *room, const rt_camera *cams, int32_t n_cams, int32_t pol_mask,
                        int32_t min_difficulty, float *rgb, const rt_render_aux *aux, int64_t *counts,
                        void *stream) {
  if (!model) return fail(RT_E_INVALID, "model is NULL");
  if (min_difficulty < 0 || min_difficulty > NBUCKET)
    return fail(RT_E_INVALID, "min_difficulty must be in [0, %d]", NBUCKET);
  if (n_cloaks < 1) return fail(RT_E_INVALID, "the surrogate render needs at least one cloak");
  if (!rgb) return fail(RT_E_INVALID, "rgb is required");
  int e = surrogate_check_ready(model);
  if (e) return e;
  RenderJob J;
  e = prepare_render(cloaks, n_cloaks, opts, room, cams, n_cams, pol_mask, aux, J);
  if (e) return e;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  e = ws_order(0, s);
  if (!e) e = ws_reserve_for(g_ws, J);
  if (!e) e = cws_reserve(g_cws, J.chunk * J.R.ncl * J.R.npol);
  if (!e) e = upload_job(J, g_ws, s);
  if (e) return e;
  long long c2[2] = {0, 0};
  e = render_surrogate(model, cloaks[0]->d, J, g_ws, g_cws, min_difficulty, rgb, s, counts ? c2 : nullptr);
  ws_done(0, s);
  if (e) return e;
  if (counts) { counts[0] = c2[0]; counts[1] = c2[1]; }
  return launch_err("surrogate render launch");
}

int rt_render(rt_cloak cloak, const rt_trace_opts *opts, const rt_room *room, const rt_camera *cams,
              int32_t n_cams, int32_t pol_mask, float *rgb, const rt_render_aux *aux, void *stream) {
  return rt_render_multi(cloak ? &cloak : nullptr, cloak ? 1 : 0, opts, room, cams, n_cams, pol_mask,
                         rgb, aux, stream);
}

int rt_render_plan_create(const rt_cloak *cloaks, int32_t n_cloaks, const rt_trace_opts *opts,
                          const rt_room *room, const rt_camera *cams, int32_t n_cams,
                          int32_t pol_mask, float *rgb, const rt_render_aux *aux, rt_plan *out) {
  if (!out) return fail(RT_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!rgb) return fail(RT_E_INVALID, "rgb is required");
  rt_plan p = new (std::nothrow) rt_plan_s;
  if (!p) return fail(RT_E_NOMEM, "host allocation failed");
  int e = prepare_render(cloaks, n_cloaks, opts, room, cams, n_cams, pol_mask, aux, p->J);
  if (!e && p->J.R.refl) e = fail(RT_E_UNSUPPORTED, "render plans do not take first-order reflections");
  if (!e) e = ws_reserve_for(p->ws, p->J);
  hipStream_t cs = nullptr;
  if (!e && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    e = fail(RT_E_DEVICE, "stream creation failed");
  if (!e) e = upload_job(p->J, p->ws, cs);
  if (!e) {
    p->rgb = rgb;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      e = fail(RT_E_DEVICE, "stream capture failed to start");
    } else {
      enqueue_render(p->J, p->ws, rgb, cs, false);
      hipGraph_t g = nullptr;
      if (hipStreamEndCapture(cs, &g) != hipSuccess || !g) {
        e = fail(RT_E_DEVICE, "stream capture failed");
      } else {
        p->graph = g;
        if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess)
          e = fail(RT_E_DEVICE, "graph instantiation failed");
      }
    }
  }
  if (cs) (void)hipStreamDestroy(cs);
  if (e) {
    rt_render_plan_destroy(p);
    return e;
  }
  *out = p;
  return RT_OK;
}

int rt_render_plan_launch(rt_plan plan, void *stream) {
  if (!plan || !plan->exec) return fail(RT_E_INVALID, "plan is NULL");
  if (hipGraphLaunch(plan->exec, (hipStream_t)stream) != hipSuccess)
    return fail(RT_E_DEVICE, "graph launch failed: %s", hipGetErrorString(hipGetLastError()));
  return RT_OK;
}

int rt_render_plan_destroy(rt_plan plan) {
  if (!plan) return RT_OK;
  (void)hipDeviceSynchronize();
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  ws_free(plan->ws);
  delete plan;
  return RT_OK;
}

int rt_autotune_render(const rt_cloak *cloaks, int32_t n_cloaks, const rt_trace_opts *opts,
                       const rt_room *room, const rt_camera *cams, int32_t n_cams, int32_t pol_mask,
                       float *rgb, rt_trace_opts *tuned, double *best_ms) {
  if (!rgb || !tuned) return fail(RT_E_INVALID, "rgb and tuned are required");
  RenderJob J;
  int e = prepare_render(cloaks, n_cloaks, opts, room, cams, n_cams, pol_mask, nullptr, J);
  if (e) return e;
  static const int blocks[] = {64, 128, 256};
  static const int refills[] = {1, 2, 4, 8, 12, 16};
  hipStream_t s = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&a) != hipSuccess ||
      hipEventCreate(&b) != hipSuccess)
    return fail(RT_E_DEVICE, "stream/event creation failed");
  double best = 1e300;
  int bb = J.block, br = J.refill;
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    e = ws_order(0, s);
    if (!e) e = ws_reserve_for(g_ws, J);
    if (!e) e = upload_job(J, g_ws, s);
    for (int bi = 0; !e && bi < 3; ++bi)
      for (int ri = 0; !e && ri < 6; ++ri) {
        J.block = blocks[bi];
        J.refill = refills[ri];
        J.grid = transit_grid(J.o, J.block);
        enqueue_render(J, g_ws, rgb, s, false);  // warm-up
        (void)hipEventRecord(a, s);
        for (int rep = 0; rep < 2; ++rep) enqueue_render(J, g_ws, rgb, s, false);
        (void)hipEventRecord(b, s);
        float ms = 0.f;
        if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) {
          e = fail(RT_E_DEVICE, "timing failed");
          break;
        }
        if (ms * 0.5 < best) { best = ms * 0.5; bb = J.block; br = J.refill; }
      }
    ws_done(0, s);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipStreamDestroy(s);
  if (e) return e;
  *tuned = *opts;
  tuned->block = bb;
  tuned->refill_period = br;
  if (best_ms) *best_ms = best;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[J.key] = {bb, br};
  return RT_OK;
}

}  // extern "C"
