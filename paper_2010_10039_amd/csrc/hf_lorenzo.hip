// hf_lorenzo.hip -- fused front end: error-bounded prequantization, 3D
// Lorenzo prediction and histogramming in one pass over a float32 field.
//
// The paper's multi-byte input (Sec. 5.1.3) is the code stream an SZ-style
// compressor makes from a float field: every value times r = 1 / (2 eb) is
// rounded to an integer d, the Lorenzo predictor's residual e of those
// integers is offset by a radius, and residuals outside the code range become
// code 0 (an outlier).  Making the codes and counting them in one kernel
// saves the histogram's own pass over the codes.
//
// Work split: one workgroup per slab of the encoder's block partition, so the
// per-slab counts the encoder wants come out directly.  In flat C order,
// f = (i * ny + j) * nx + k, the residual is taken as three first
// differences (P = ny * nx):
//   u(f) = d(f) - [i > 0] d(f - P)
//   t(f) = u(f) - [k > 0] u(f - 1)
//   e(f) = t(f) - [j > 0] t(f - nx)
// u reads the field twice: at f (streamed from HBM once) and one plane back
// (read by the workgroup two slabs earlier at about the same time, so mostly
// a cache hit).  The fastest-axis neighbour comes from the next-lower lane.
// t one row back comes from a ring of t values in LDS that the workgroup
// itself wrote (a prologue fills it with the row just before the slab).
#include <math.h>

#include <algorithm>

#include "hf_device.h"
#include "hf_kernels.h"

namespace hf {

namespace {

constexpr int kLzThreads = 256;
constexpr int kLzVec = 8;                          // consecutive elements per lane and step
constexpr uint32_t kLzStep = kLzThreads * kLzVec;  // elements per workgroup and step
constexpr float kLzClamp = 16777216.0f;            // |d| <= 2^24 keeps every residual in int32

// n / d for every 32-bit n with one multiply-high (Granlund and Montgomery,
// "Division by invariant integers using multiplication", PLDI 1994, Sec. 4):
// l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1, n / d = (mulhi(m, n) + n) >> l
// evaluated in 64 bits.
struct FastDiv {
  uint32_t d;
  uint32_t m;
  uint32_t l;
};

FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  const uint64_t m = (((1ull << l) - d) << 32) / d + 1;
  return FastDiv{d, (uint32_t)m, l};
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return (uint32_t)(((uint64_t)__umulhi(n, f.m) + n) >> f.l);
}

__device__ __forceinline__ uint32_t fmod_(uint32_t n, const FastDiv& f) { return n - fdiv(n, f) * f.d; }

struct LzArgs {
  const float* x;
  uint16_t* codes;
  uint32_t* hist;       // zeroed by workgroup 0 when slab_hist is set (hist_reduce adds), else beforehand
  uint32_t* slab_hist;  // [nslabs][A] or null
  uint32_t n;
  uint32_t nx;
  uint32_t plane;  // ny * nx
  FastDiv div_nx;
  FastDiv div_plane;
  float r;
  int radius;
  uint32_t A;          // 2 * radius
  uint32_t rep_shift;  // log2 of the LDS histogram replicas
  uint32_t ring_mask;  // ring words - 1; 0 when ny == 1 (no row above ever exists)
  uint32_t nslabs;
  uint32_t nblocks;
  uint32_t* status;    // HF_ERR_VALUE when a value of the field is NaN or infinite
};

// Prequantization of a finite value: x * r rounded to the nearest integer,
// ties to even, clamped to [-2^24, 2^24] (a product that overflows to an
// infinity clamps too).  Non-finite values are outside the quantizer's
// domain: the steps below flag them with nonfinite() and the call fails.
__device__ __forceinline__ int prequant(float x, float r) {
  return (int)fminf(fmaxf(rintf(x * r), -kLzClamp), kLzClamp);
}

// 1 if x is NaN or an infinity (all exponent bits set).
__device__ __forceinline__ uint32_t nonfinite(float x) {
  return (__float_as_uint(x) & 0x7f800000u) == 0x7f800000u ? 1u : 0u;
}

// u(f) = d(f) - [f >= P] d(f - P)
__device__ __forceinline__ int u_at(const LzArgs& a, uint32_t f) {
  const int own = prequant(a.x[f], a.r);
  return f >= a.plane ? own - prequant(a.x[f - a.plane], a.r) : own;
}

// t(f) = u(f) - [k > 0] u(f - 1)
__device__ __forceinline__ int t_at(const LzArgs& a, uint32_t f) {
  const int u = u_at(a, f);
  return fmod_(f, a.div_nx) ? u - u_at(a, f - 1) : u;
}

// j > 0: the row above f exists inside its plane.
__device__ __forceinline__ bool row_above(const LzArgs& a, uint32_t f) { return fmod_(f, a.div_plane) >= a.nx; }

__device__ __forceinline__ uint32_t code_of(int e, int radius) {
  const int q = e + radius;
  return (uint32_t)(q - 1) < (uint32_t)(2 * radius - 1) ? (uint32_t)q : 0u;
}

__device__ __forceinline__ void load8(const float* p, float v[kLzVec]) {
  const float4 a = *(const float4*)p;
  const float4 b = *(const float4*)(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

// Loads of one vector step, issued one step ahead: the lane's 8 values, the
// 8 one plane back, the value just before the group and its plane-back
// value (lane 0 of a wave uses the last two; the other lanes get that u from
// their lower neighbour).  All six loads are always issued, so the wait for
// a step's data is a fixed count behind the next step's loads: an index with
// nothing to read (no plane back, no value before, a group past the end)
// reads a valid address instead and its value is masked off.
struct LzFetch {
  float o[kLzVec];
  float b[kLzVec];
  float lo;
  float lb;
};

__device__ __forceinline__ void fetch_step(const LzArgs& a, uint64_t f, uint64_t s_hi, LzFetch& v) {
  const uint32_t fo = f + kLzVec <= s_hi ? (uint32_t)f : 0u;
  const uint32_t fl = fo > 0 ? fo - 1 : 0u;
  load8(a.x + (fo >= a.plane ? fo - a.plane : fo), v.b);
  load8(a.x + fo, v.o);
  v.lb = a.x[fl >= a.plane ? fl - a.plane : fl];
  v.lo = a.x[fl];
}

// Codes of one lane's group from t and the row-above values: the 16-byte
// store on the vector path, one store per element otherwise; LDS counts.
__device__ __forceinline__ uint32_t lz_code(const LzArgs& a, int t, int prev) { return code_of(t - prev, a.radius); }

// One whole step on the vector path: group f = base + 8 tid, every lane's
// group inside the slab.  Uses `cur`, fetches the step after into `nxt`,
// writes t to the ring, reads the row above after a barrier, and stores
// codes and counts.
__device__ __forceinline__ void vec_step(const LzArgs& a, uint64_t base, uint64_t s_hi, int* ring, char* subr,
                                         uint32_t hshift, bool lane0, const LzFetch& cur, LzFetch& nxt,
                                         uint32_t& bad) {
  const uint32_t f = (uint32_t)(base + threadIdx.x * kLzVec);
  fetch_step(a, (uint64_t)f + kLzStep, s_hi, nxt);
  // Take all of `cur` here, on every path: the compiler then knows those
  // registers are written before the step after reloads them, and waits
  // only for this step's data, never for the loads just issued.
  asm volatile("" ::"v"(cur.o[0]), "v"(cur.o[1]), "v"(cur.o[2]), "v"(cur.o[3]), "v"(cur.o[4]), "v"(cur.o[5]),
               "v"(cur.o[6]), "v"(cur.o[7]), "v"(cur.b[0]), "v"(cur.b[1]), "v"(cur.b[2]), "v"(cur.b[3]),
               "v"(cur.b[4]), "v"(cur.b[5]), "v"(cur.b[6]), "v"(cur.b[7]), "v"(cur.lo), "v"(cur.lb));
  const int mb = f >= a.plane ? -1 : 0;
  int u[kLzVec];
#pragma unroll
  for (int e = 0; e < kLzVec; ++e) {
    bad |= nonfinite(cur.o[e]);  // the lane's own values (every group of this step is inside the slab)
    u[e] = prequant(cur.o[e], a.r) - (prequant(cur.b[e], a.r) & mb);
  }
  const int up = __shfl_up(u[kLzVec - 1], 1, 64);
  const int own_left = prequant(cur.lo, a.r) - (prequant(cur.lb, a.r) & (f - 1 >= a.plane ? -1 : 0));
  const int left = lane0 ? own_left : up;
  const bool k0 = fmod_(f, a.div_nx) == 0;
  int t[kLzVec];
  t[0] = u[0] - (k0 ? 0 : left);
#pragma unroll
  for (int e = 1; e < kLzVec; ++e) t[e] = u[e] - u[e - 1];
  if (a.ring_mask) {
    int4* w = (int4*)(ring + (f & a.ring_mask));
    w[0] = make_int4(t[0], t[1], t[2], t[3]);
    w[1] = make_int4(t[4], t[5], t[6], t[7]);
  }
  __syncthreads();
  int prev[kLzVec];
  if (a.ring_mask && row_above(a, f)) {
    const int4* rd = (const int4*)(ring + ((f - a.nx) & a.ring_mask));
    const int4 p0 = rd[0];
    const int4 p1 = rd[1];
    prev[0] = p0.x; prev[1] = p0.y; prev[2] = p0.z; prev[3] = p0.w;
    prev[4] = p1.x; prev[5] = p1.y; prev[6] = p1.z; prev[7] = p1.w;
  } else {
#pragma unroll
    for (int e = 0; e < kLzVec; ++e) prev[e] = 0;
  }
  __syncthreads();  // the next step rewrites ring slots read above
  uint32_t q[kLzVec];
#pragma unroll
  for (int e = 0; e < kLzVec; ++e) q[e] = lz_code(a, t[e], prev[e]);
  *(uint4*)(a.codes + f) = make_uint4(q[0] | (q[1] << 16), q[2] | (q[3] << 16), q[4] | (q[5] << 16),
                                      q[6] | (q[7] << 16));
#pragma unroll
  for (int e = 0; e < kLzVec; ++e) atomicAdd((uint32_t*)(subr + (q[e] << hshift)), 1u);
}

// One step element by element (groups that are not whole, unaligned
// fields): the same three differences from direct loads.
__device__ __forceinline__ void elem_step(const LzArgs& a, uint64_t base, uint64_t s_hi, int* ring, char* subr,
                                          uint32_t hshift, uint32_t& bad) {
  const uint64_t f64 = base + threadIdx.x * kLzVec;
  const uint32_t f = (uint32_t)f64;  // meaningful only while f64 < s_hi
  int t[kLzVec];
#pragma unroll
  for (int e = 0; e < kLzVec; ++e) {
    const bool in = f64 + e < s_hi;
    const uint32_t fe = f + e;
    t[e] = in ? t_at(a, fe) : 0;
    if (in) bad |= nonfinite(a.x[fe]);
    if (a.ring_mask && in) ring[fe & a.ring_mask] = t[e];
  }
  __syncthreads();
  int prev[kLzVec];
#pragma unroll
  for (int e = 0; e < kLzVec; ++e) {
    const uint32_t fe = f + e;
    prev[e] = (a.ring_mask && f64 + e < s_hi && row_above(a, fe)) ? ring[(fe - a.nx) & a.ring_mask] : 0;
  }
  __syncthreads();  // the next step rewrites ring slots read above
#pragma unroll
  for (int e = 0; e < kLzVec; ++e) {
    if (f64 + e < s_hi) {
      const uint32_t q = lz_code(a, t[e], prev[e]);
      a.codes[f + e] = (uint16_t)q;
      atomicAdd((uint32_t*)(subr + (q << hshift)), 1u);
    }
  }
}

// kVec: nx % 8 == 0 and both arrays 16-byte aligned, so a lane's 8
// elements share one row and move as two 16-byte vectors, fetched one step
// ahead (two register sets, alternating).  The whole steps of a slab run
// on that path; a last partial step (and every step when !kVec) runs
// element by element.
template <bool kVec>
__global__ __launch_bounds__(kLzThreads) void lorenzo_hist_kernel(LzArgs a) {
  extern __shared__ __align__(16) uint32_t lds[];
  const uint32_t tid = threadIdx.x;
  const uint32_t reps = 1u << a.rep_shift;
  uint32_t* sub = lds;
  int* ring = (int*)(lds + ((a.A * reps + 3) & ~3u));
  for (uint32_t i = tid; i < a.A * reps; i += kLzThreads) sub[i] = 0;
  if (a.slab_hist && blockIdx.x == 0)
    for (uint32_t b = tid; b < a.A; b += kLzThreads) a.hist[b] = 0;

  const uint32_t g = blockIdx.x;
  const uint64_t s_lo = slab_begin(g, a.nblocks, a.nslabs, a.n);
  const uint64_t s_hi = slab_begin(g + 1, a.nblocks, a.nslabs, a.n);
  if (a.ring_mask) {
    const uint32_t p_lo = s_lo > a.nx ? (uint32_t)s_lo - a.nx : 0;
    for (uint32_t f = p_lo + tid; f < s_lo; f += kLzThreads) ring[f & a.ring_mask] = t_at(a, f);
  }
  __syncthreads();

  char* const subr = (char*)(sub + (tid & (reps - 1)));
  const uint32_t hshift = a.rep_shift + 2;
  uint64_t base = s_lo;
  uint32_t bad = 0;
  if (kVec) {
    const uint64_t v_end = s_lo + (s_hi - s_lo) / kLzStep * kLzStep;
    const bool lane0 = (tid & 63) == 0;
    LzFetch va, vb;
    fetch_step(a, s_lo + tid * kLzVec, s_hi, va);
    for (; base + 2 * kLzStep <= v_end; base += 2 * kLzStep) {
      vec_step(a, base, s_hi, ring, subr, hshift, lane0, va, vb, bad);
      vec_step(a, base + kLzStep, s_hi, ring, subr, hshift, lane0, vb, va, bad);
    }
    if (base < v_end) {
      vec_step(a, base, s_hi, ring, subr, hshift, lane0, va, vb, bad);
      base += kLzStep;
    }
  }
  for (; base < s_hi; base += kLzStep) elem_step(a, base, s_hi, ring, subr, hshift, bad);
  if (bad) raise_status(a.status, HF_ERR_VALUE);
  __syncthreads();
  if (a.slab_hist) {
    uint32_t* row = a.slab_hist + (uint64_t)g * a.A;
    for (uint32_t b = tid; b < a.A; b += kLzThreads) {
      uint32_t c = 0;
      for (uint32_t rr = 0; rr < reps; ++rr) c += sub[(b << a.rep_shift) + rr];
      row[b] = c;
    }
  } else {
    for (uint32_t b = tid; b < a.A; b += kLzThreads) {
      uint32_t c = 0;
      for (uint32_t rr = 0; rr < reps; ++rr) c += sub[(b << a.rep_shift) + rr];
      if (c) atomicAdd(a.hist + b, c);
    }
  }
}

// ---------------------------------------------------------------------------
// Chained slabs.  When every slab has the same length L, L is a whole number
// of steps and a plane is D = P / L slabs, slab g's values one plane back
// are exactly slab g - D.  A workgroup of kChain sub-groups (256 threads
// each) then runs the slabs of kChain consecutive planes that sit at the
// same place in their planes, in lockstep: sub-group k publishes its
// prequantized d in LDS, and sub-group k + 1 takes its plane-back values
// from there instead of reading the field again.  Only sub-group 0 reads
// the plane before the chain from memory, so the field is read
// (kChain + 1) / kChain times instead of twice.

constexpr int kChain = 4;
constexpr int kChainThreads = kChain * kLzThreads;

// As fetch_step; the plane-back vector is real only for sub-group 0 (the
// others read their own values a second time, a cache hit, so the load
// count stays fixed), and the plane-back value before the group only for
// lane 0.
__device__ __forceinline__ void fetch_chain(const LzArgs& a, uint64_t f, uint64_t s_hi, bool first_sub, bool lane0,
                                            LzFetch& v) {
  const uint32_t fo = f + kLzVec <= s_hi ? (uint32_t)f : 0u;
  const uint32_t fl = fo > 0 ? fo - 1 : 0u;
  load8(a.x + (first_sub && fo >= a.plane ? fo - a.plane : fo), v.b);
  load8(a.x + fo, v.o);
  v.lb = a.x[lane0 && fl >= a.plane ? fl - a.plane : fl];
  v.lo = a.x[fl];
}

struct ChainLane {
  bool active;     // this sub-group has a slab (the last chain may be short)
  bool first_sub;  // sub-group 0: plane-back values come from memory
  bool publish;    // the next sub-group has a slab and reads d from here
  bool lane0;
  uint32_t lt;     // thread index inside the sub-group
  uint64_t s_hi;   // end of the slab (0 when inactive: fetches read index 0)
  int* ring;
  char* subr;
  uint32_t hshift;
  int* xb_out;
  const int* xb_in;
};

// One step of sub-group k at group f64: uses `cur` (fetched two steps
// earlier) and fetches the step two ahead into `ahead`.
__device__ __forceinline__ void chain_step(const LzArgs& a, const ChainLane& c, uint64_t f64, const LzFetch& cur,
                                           LzFetch& ahead, uint32_t& bad) {
  const uint32_t f = (uint32_t)f64;
  fetch_chain(a, f64 + 2 * kLzStep, c.s_hi, c.first_sub, c.lane0, ahead);
  asm volatile("" ::"v"(cur.o[0]), "v"(cur.o[1]), "v"(cur.o[2]), "v"(cur.o[3]), "v"(cur.o[4]), "v"(cur.o[5]),
               "v"(cur.o[6]), "v"(cur.o[7]), "v"(cur.b[0]), "v"(cur.b[1]), "v"(cur.b[2]), "v"(cur.b[3]),
               "v"(cur.b[4]), "v"(cur.b[5]), "v"(cur.b[6]), "v"(cur.b[7]), "v"(cur.lo), "v"(cur.lb));
  int d[kLzVec];
#pragma unroll
  for (int e = 0; e < kLzVec; ++e) {
    bad |= c.active ? nonfinite(cur.o[e]) : 0u;  // an inactive sub-group reads index 0, not values of its own
    d[e] = prequant(cur.o[e], a.r);
  }
  if (c.publish) {
    int4* w = (int4*)(c.xb_out + c.lt * kLzVec);
    w[0] = make_int4(d[0], d[1], d[2], d[3]);
    w[1] = make_int4(d[4], d[5], d[6], d[7]);
  }
  int db[kLzVec];
  if (c.first_sub) {  // uniform per wave
    const int mb = f >= a.plane ? -1 : 0;
#pragma unroll
    for (int e = 0; e < kLzVec; ++e) db[e] = prequant(cur.b[e], a.r) & mb;
  }
  __syncthreads();  // d published; the last step's ring reads are done
  if (!c.first_sub) {
    const int4* rd = (const int4*)(c.xb_in + c.lt * kLzVec);
    const int4 p0 = rd[0];
    const int4 p1 = rd[1];
    db[0] = p0.x; db[1] = p0.y; db[2] = p0.z; db[3] = p0.w;
    db[4] = p1.x; db[5] = p1.y; db[6] = p1.z; db[7] = p1.w;
  }
  int u[kLzVec];
#pragma unroll
  for (int e = 0; e < kLzVec; ++e) u[e] = d[e] - db[e];
  const int up = __shfl_up(u[kLzVec - 1], 1, 64);
  const int own_left = prequant(cur.lo, a.r) - (prequant(cur.lb, a.r) & (f - 1 >= a.plane ? -1 : 0));
  const int left = c.lane0 ? own_left : up;
  const bool k0 = fmod_(f, a.div_nx) == 0;
  int t[kLzVec];
  t[0] = u[0] - (k0 ? 0 : left);
#pragma unroll
  for (int e = 1; e < kLzVec; ++e) t[e] = u[e] - u[e - 1];
  if (c.active && a.ring_mask) {
    int4* w = (int4*)(c.ring + (f & a.ring_mask));
    w[0] = make_int4(t[0], t[1], t[2], t[3]);
    w[1] = make_int4(t[4], t[5], t[6], t[7]);
  }
  __syncthreads();  // t in the ring; the published d has been read
  if (!c.active) return;
  int prev[kLzVec];
  if (a.ring_mask && row_above(a, f)) {
    const int4* rd = (const int4*)(c.ring + ((f - a.nx) & a.ring_mask));
    const int4 p0 = rd[0];
    const int4 p1 = rd[1];
    prev[0] = p0.x; prev[1] = p0.y; prev[2] = p0.z; prev[3] = p0.w;
    prev[4] = p1.x; prev[5] = p1.y; prev[6] = p1.z; prev[7] = p1.w;
  } else {
#pragma unroll
    for (int e = 0; e < kLzVec; ++e) prev[e] = 0;
  }
  uint32_t q[kLzVec];
#pragma unroll
  for (int e = 0; e < kLzVec; ++e) q[e] = lz_code(a, t[e], prev[e]);
  *(uint4*)(a.codes + f) = make_uint4(q[0] | (q[1] << 16), q[2] | (q[3] << 16), q[4] | (q[5] << 16),
                                      q[6] | (q[7] << 16));
#pragma unroll
  for (int e = 0; e < kLzVec; ++e) atomicAdd((uint32_t*)(c.subr + (q[e] << c.hshift)), 1u);
}

// Workgroup w runs chain (plane group w / D, place w % D): sub-group k takes
// slab (plane group * kChain + k) * D + w % D.  L is the slab length in
// values, nz the number of planes.
__global__ __launch_bounds__(kChainThreads) void lorenzo_chain_kernel(LzArgs a, uint32_t D, uint32_t L, uint32_t nz) {
  extern __shared__ __align__(16) uint32_t lds[];
  const uint32_t k = threadIdx.x / kLzThreads;
  const uint32_t lt = threadIdx.x % kLzThreads;
  const uint32_t reps = 1u << a.rep_shift;
  const uint32_t hist_words = (a.A * reps + 3) & ~3u;
  const uint32_t ring_words = a.ring_mask ? a.ring_mask + 1 : 0;
  for (uint32_t i = threadIdx.x; i < kChain * hist_words; i += kChainThreads) lds[i] = 0;
  if (a.slab_hist && blockIdx.x == 0)
    for (uint32_t b = threadIdx.x; b < a.A; b += kChainThreads) a.hist[b] = 0;

  const uint32_t plane = (blockIdx.x / D) * kChain + k;
  const uint32_t g = plane * D + blockIdx.x % D;
  ChainLane c;
  c.active = plane < nz;
  c.first_sub = k == 0;
  c.publish = k + 1 < kChain && plane + 1 < nz;
  c.lane0 = (lt & 63) == 0;
  c.lt = lt;
  const uint64_t s_lo = c.active ? (uint64_t)g * L : 0;
  c.s_hi = c.active ? s_lo + L : 0;
  uint32_t* sub = lds + k * hist_words;
  c.ring = (int*)(lds + kChain * hist_words) + k * ring_words;
  c.subr = (char*)(sub + (lt & (reps - 1)));
  c.hshift = a.rep_shift + 2;
  int* xb = (int*)(lds + kChain * (hist_words + ring_words));
  c.xb_out = xb + k * kLzStep;
  c.xb_in = xb + (k > 0 ? k - 1 : 0) * kLzStep;
  if (c.active && a.ring_mask) {
    const uint32_t p_lo = s_lo > a.nx ? (uint32_t)s_lo - a.nx : 0;
    for (uint32_t f = p_lo + lt; f < s_lo; f += kLzThreads) c.ring[f & a.ring_mask] = t_at(a, f);
  }
  __syncthreads();

  // Two steps in flight: with one 16-wave workgroup per CU, a single step
  // ahead keeps too few bytes in flight to cover the memory latency.  Three
  // register sets rotate (step s uses set s % 3 and fills set (s + 2) % 3).
  const uint32_t steps = L / kLzStep;
  const uint64_t f0 = s_lo + lt * kLzVec;
  LzFetch va, vb, vc;
  fetch_chain(a, f0, c.s_hi, c.first_sub, c.lane0, va);
  fetch_chain(a, f0 + kLzStep, c.s_hi, c.first_sub, c.lane0, vb);
  uint32_t st = 0;
  uint32_t bad = 0;
  for (; st + 3 <= steps; st += 3) {
    chain_step(a, c, f0 + (uint64_t)st * kLzStep, va, vc, bad);
    chain_step(a, c, f0 + (uint64_t)(st + 1) * kLzStep, vb, va, bad);
    chain_step(a, c, f0 + (uint64_t)(st + 2) * kLzStep, vc, vb, bad);
  }
  if (st < steps) chain_step(a, c, f0 + (uint64_t)st * kLzStep, va, vc, bad);
  if (st + 1 < steps) chain_step(a, c, f0 + (uint64_t)(st + 1) * kLzStep, vb, va, bad);
  if (bad) raise_status(a.status, HF_ERR_VALUE);
  __syncthreads();
  if (!c.active) return;
  if (a.slab_hist) {
    uint32_t* row = a.slab_hist + (uint64_t)g * a.A;
    for (uint32_t b = lt; b < a.A; b += kLzThreads) {
      uint32_t cnt = 0;
      for (uint32_t rr = 0; rr < reps; ++rr) cnt += sub[(b << a.rep_shift) + rr];
      row[b] = cnt;
    }
  } else {
    for (uint32_t b = lt; b < a.A; b += kLzThreads) {
      uint32_t cnt = 0;
      for (uint32_t rr = 0; rr < reps; ++rr) cnt += sub[(b << a.rep_shift) + rr];
      if (cnt) atomicAdd(a.hist + b, cnt);
    }
  }
}

uint32_t pow2_at_least(uint32_t v) {
  uint32_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

}  // namespace

size_t lorenzo_lds_bytes(uint32_t ny, uint32_t nx, uint32_t radius) {
  const uint32_t A = 2 * radius;
  uint32_t shift = 0;
  while (shift < 4 && A * (2u << shift) * 4u <= (16u << 10)) ++shift;
  const uint32_t hist_words = (A * (1u << shift) + 3) & ~3u;
  const uint32_t ring_words = ny > 1 ? pow2_at_least(kLzStep + nx) : 0;
  return (size_t)(hist_words + ring_words) * 4;
}

hipError_t launch_lorenzo_histogram(const float* x, uint32_t nz, uint32_t ny, uint32_t nx, float r, uint32_t radius,
                                    uint16_t* codes, uint32_t* hist, uint32_t nslabs, uint32_t* slab_hist,
                                    uint32_t* status, int num_cus, hipStream_t stream, const KernelTimer& timer) {
  const uint64_t n = (uint64_t)nz * ny * nx;
  const uint32_t A = 2 * radius;
  hipError_t e;
  if (n == 0) return launch_fill_u32(hist, A, 0u, stream);
  LzArgs a;
  a.x = x;
  a.codes = codes;
  a.hist = hist;
  a.slab_hist = slab_hist;
  a.status = status;
  a.n = (uint32_t)n;
  a.nx = nx;
  a.plane = ny * nx;
  a.div_nx = make_fastdiv(nx);
  a.div_plane = make_fastdiv(ny * nx);
  a.r = r;
  a.radius = (int)radius;
  a.A = A;
  a.rep_shift = 0;
  while (a.rep_shift < 4 && A * (2u << a.rep_shift) * 4u <= (16u << 10)) ++a.rep_shift;
  a.ring_mask = ny > 1 ? pow2_at_least(kLzStep + nx) - 1 : 0;
  a.nblocks = (uint32_t)((n + kSlabBlock - 1) / kSlabBlock);
  if (slab_hist) {
    a.nslabs = nslabs;
  } else {
    e = launch_fill_u32(hist, A, 0u, stream);
    if (e != hipSuccess) return e;
    a.nslabs = (uint32_t)std::min<uint64_t>((uint64_t)num_cus * 4, a.nblocks);
  }
  const bool vec = nx % kLzVec == 0 && ((uintptr_t)x & 15) == 0 && ((uintptr_t)codes & 15) == 0;
  // chained slabs: equal slabs of whole steps, a whole number of slabs per plane
  const uint64_t slab_len = a.nblocks % a.nslabs == 0 ? (uint64_t)(a.nblocks / a.nslabs) * kSlabBlock : 0;
  if (vec && nz >= 2 && n % kSlabBlock == 0 && slab_len && slab_len % kLzStep == 0 && a.plane % slab_len == 0) {
    LzArgs c = a;
    c.rep_shift = 0;  // a 16 KiB window per sub-group, as the plain kernel's
    while (c.rep_shift < 4 && A * (2u << c.rep_shift) * 4u <= (16u << 10)) ++c.rep_shift;
    const size_t hist_words = (A * (1u << c.rep_shift) + 3) & ~3u;
    const size_t ring_words = c.ring_mask ? c.ring_mask + 1 : 0;
    const size_t lds_chain = (kChain * (hist_words + ring_words) + (kChain - 1) * (size_t)kLzStep) * 4;
    if (lds_chain <= (160u << 10)) {
      const uint32_t D = (uint32_t)(a.plane / slab_len);
      const uint32_t grid = D * ((nz + kChain - 1) / kChain);
      (void)hipFuncSetAttribute((const void*)lorenzo_chain_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_chain);
      timer.before(stream);
      lorenzo_chain_kernel<<<grid, kChainThreads, lds_chain, stream>>>(c, D, (uint32_t)slab_len, nz);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      timer.after(stream);
      if (slab_hist) return launch_slab_hist_reduce(slab_hist, nslabs, A, hist, stream);
      return hipSuccess;
    }
  }
  const size_t lds = lorenzo_lds_bytes(ny, nx, radius);
  const void* fn = vec ? (const void*)lorenzo_hist_kernel<true> : (const void*)lorenzo_hist_kernel<false>;
  if (lds > (64u << 10)) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  timer.before(stream);
  if (vec)
    lorenzo_hist_kernel<true><<<a.nslabs, kLzThreads, lds, stream>>>(a);
  else
    lorenzo_hist_kernel<false><<<a.nslabs, kLzThreads, lds, stream>>>(a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  timer.after(stream);
  if (slab_hist) return launch_slab_hist_reduce(slab_hist, nslabs, A, hist, stream);
  return hipSuccess;
}

}  // namespace hf
