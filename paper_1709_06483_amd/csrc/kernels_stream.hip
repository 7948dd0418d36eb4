// Two-term CSR Leja iteration (Section 3's recurrence on a1 H1 + a2 H2), the
// streaming wave-tile variant; the first of the two passes of a Method M4
// iteration with the commutator applied matrix-free; and the three-term
// iteration of Method M4 with the commutator assembled.
//
// Every wave walks 8 tiles of 8 consecutive rows.  A tile's column indices and
// values (term 1's entries of its rows, then term 2's) travel from HBM
// straight into a wave-private LDS buffer with global_load_lds (no VGPRs held
// while in flight), one chunk of 256 entries ahead of the chunk being
// processed.  Per chunk the wave waits at the top: the copy of the chunk,
// issued during the previous one, and the row pointers two tiles ahead have
// arrived; it then reads its entries' columns, issues the gathers, issues the
// copy of the next chunk behind them, and waits for both before it
// multiplies.  Lanes are laid out row-fastest
// (lane = g * 8 + r) and each row's 8 groups are summed with shuffles in a
// fixed order, the same order and chunking as the 8-row wave-tile kernel.
//
// The LDS reads of staged entries are inline ds_read instructions followed by
// their own lgkmcnt wait: the compiler would otherwise make every LDS read wait
// for all outstanding copies into LDS (it cannot tell the two buffers apart),
// which would serialise the copy of the next chunk with the current one.  The
// explicit vmcnt(0) at the top of each chunk is what orders the copy of a
// chunk before its reads.
#include <algorithm>
#include <cstdint>

#include "device_common.h"

namespace magnus {
namespace {

using namespace dev;

typedef __attribute__((address_space(3))) void lds_void;

constexpr int kSW = kThreads / 64;  // waves per workgroup
constexpr int kSR = 8;              // rows per tile
constexpr int kSG = 64 / kSR;       // lanes per row
constexpr int kSCap = 256;          // entries per LDS buffer
constexpr int kSU = kSCap / 64;     // copy instructions per buffer and array
constexpr int kNB = 3;              // entries per lane and term in one gather round
constexpr int kTPW = kSG;           // tiles per wave: one per lane slot g
constexpr unsigned kNonTemporal = 2;  // cache policy of the matrix stream (nt)
// The matrix is read again by every iteration.  Copied with non-temporal
// loads it never stays in the 256 MiB memory-side cache (MALL) of MI355X,
// and copied with normal loads it evicts itself before it is read again; so
// the tiles at the front of the matrix, up to what the MALL holds besides the
// vectors an iteration touches (about 80 bytes per row: x, w and p read, w
// and p written), use normal loads and stay resident from one iteration to
// the next, and the rest stream through.  Measured on spin chains (us per
// iteration, none / 96 / 160 / 224 MB kept): n = 20 168 / 164 / 158 / 161,
// n = 19 84 / 77 / 76 / 74.
constexpr long long kMallKeepBytes = 240LL << 20;

// Wave-private double buffers: 2 x (256 values + 256 column indices) per wave,
// 40 KiB per workgroup, so four workgroups (16 waves) share a CU's LDS.
struct StreamLds {
  d2 val[kSW][2][kSCap];
  int col[kSW][2][kSCap];
};

__device__ __forceinline__ unsigned lds_offset(const void* p) {
  return (unsigned)(uintptr_t)(const lds_void*)p;
}

__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

// LDS reads of staged entries: the column indices of three entries of each
// term, and (separately, once the gathers are in flight) their values.  Each
// statement waits for its own reads, so no instruction sees the registers
// before the data has arrived.
__device__ __forceinline__ void lds_read_cols(const unsigned (&ca1)[kNB], const unsigned (&ca2)[kNB],
                                              int (&c1)[kNB], int (&c2)[kNB]) {
  asm volatile(
      "ds_read_b32 %0, %6\n\t"
      "ds_read_b32 %1, %7\n\t"
      "ds_read_b32 %2, %8\n\t"
      "ds_read_b32 %3, %9\n\t"
      "ds_read_b32 %4, %10\n\t"
      "ds_read_b32 %5, %11\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(c1[0]), "=&v"(c1[1]), "=&v"(c1[2]), "=&v"(c2[0]), "=&v"(c2[1]), "=&v"(c2[2])
      : "v"(ca1[0]), "v"(ca1[1]), "v"(ca1[2]), "v"(ca2[0]), "v"(ca2[1]), "v"(ca2[2]));
}

__device__ __forceinline__ void lds_read_vals(const unsigned (&va1)[kNB], const unsigned (&va2)[kNB],
                                              d2 (&h1)[kNB], d2 (&h2)[kNB]) {
  asm volatile(
      "ds_read_b128 %0, %6\n\t"
      "ds_read_b128 %1, %7\n\t"
      "ds_read_b128 %2, %8\n\t"
      "ds_read_b128 %3, %9\n\t"
      "ds_read_b128 %4, %10\n\t"
      "ds_read_b128 %5, %11\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(h1[0]), "=&v"(h1[1]), "=&v"(h1[2]), "=&v"(h2[0]), "=&v"(h2[1]), "=&v"(h2[2])
      : "v"(va1[0]), "v"(va1[1]), "v"(va1[2]), "v"(va2[0]), "v"(va2[1]), "v"(va2[2]));
}

struct Tile {
  int nr;     // rows of the tile inside the matrix (0: past the end)
  int base1;  // first entry of term 1
  int n1;     // entries of term 1
  int base2;  // first entry of term 2
  int total;  // entries of both terms
};

// Workgroup L owns 32 consecutive tiles; its wave w takes tiles L * 32 + w + 4 j,
// j < 8 (the four waves stream neighbouring rows).  After the shuffle sum
// every lane of a row holds that row's total, so lane g * 8 + r keeps the
// own-row operands and results of row r of the wave's tile g: they are loaded
// once when the wave starts and stored once when it ends, and no store is
// outstanding inside the tile loop (a pending store would make every wait on
// a gather wait for all outstanding loads, the next chunk's copy included).
//
// MODE kLeja: y = a1 H1 x1 + a2 H2 x2, then the Leja update and norm partials.
// MODE kSplitComm (x1 = x2 = wcur = w): wout = a1 w + i k H2 w and
// pacc = a2 w - i k H1 w, so that the kLeja pass H1 wout + H2 pacc (a1 = a2 = 1)
// is a1 H1 w + a2 H2 w + k i[H1, H2] w.
template <int MODE>
__global__ __launch_bounds__(kThreads, 4) void csr2_stream_kernel(CsrDev t1, CsrDev t2, int dim, IterArgs a_in,
                                                                  int keep_entries) {
  static_assert(MODE == kLeja || MODE == kSplitComm, "streamed modes");
  const IterArgs a = resolve_args(a_in);
  __shared__ StreamLds sh;
  // the stop flag is the same for every wave; it is tested once the first
  // row pointers are in flight (the fused test reduces the partials first,
  // in LDS that the copies reuse afterwards)
  const bool stopped = iteration_stopped(a, reinterpret_cast<double*>(&sh.val[0][0][0]));
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int r = lane % kSR, g = lane / kSR;
  const d2* v1 = reinterpret_cast<const d2*>(t1.val);
  const d2* v2 = reinterpret_cast<const d2*>(t2.val);
  const d2* x1 = reinterpret_cast<const d2*>(a.x1);
  const d2* x2 = reinterpret_cast<const d2*>(a.x2);

  auto tile_row0 = [&](int j) { return (L * kSW * kTPW + wv + j * kSW) * kSR; };
  auto tile_rows = [&](int j) { return j < kTPW ? max(0, min(kSR, dim - tile_row0(j))) : 0; };
  // row pointers of tile j: lanes 0..nr hold term 1's, lanes 32..32+nr term
  // 2's; one unconditional load per lane (other lanes and tiles past the end
  // read an entry that exists), so no copy has to wait for it
  auto load_rp = [&](int j) {
    const int nr = tile_rows(j);
    const int idx = nr > 0 ? tile_row0(j) + min(lane & 31, nr) : 0;
    const int* rp = lane < 32 ? t1.rp : t2.rp;
    return rp[idx];
  };
  auto tile_of = [&](int j, int v) {
    Tile T{tile_rows(j), 0, 0, 0, 0};
    if (T.nr > 0) {
      T.base1 = __builtin_amdgcn_readlane(v, 0);
      T.n1 = __builtin_amdgcn_readlane(v, T.nr) - T.base1;
      T.base2 = __builtin_amdgcn_readlane(v, 32);
      T.total = T.n1 + __builtin_amdgcn_readlane(v, 32 + T.nr) - T.base2;
    }
    return T;
  };
  // copy entries [c0, c0 + 256) of tile T into buffer b; lanes past the end
  // of the chunk re-read its first entry (always present) and are ignored.
  // Tiles whose entries start within the first keep_entries of the two
  // terms together are copied with normal loads, the others non-temporal.
  auto issue = [&](const Tile& T, int c0, int b) {
    const int cn = min(kSCap, T.total - c0);
    const bool keep = (long long)T.base1 + T.base2 < keep_entries;  // no int overflow
#pragma unroll 1
    for (int u = 0; u < kSU; ++u) {
      if (u * 64 < cn) {
        const int k = u * 64 + lane;
        const int gk = c0 + (k < cn ? k : 0);
        const bool first = gk < T.n1;
        const int e = first ? T.base1 + gk : T.base2 + (gk - T.n1);
        const d2* vp = (first ? v1 : v2) + e;
        const int* cp = (first ? t1.ci : t2.ci) + e;
        if (keep) {
          __builtin_amdgcn_global_load_lds(vp, (lds_void*)&sh.val[wv][b][u * 64], 16, 0, 0);
          __builtin_amdgcn_global_load_lds(cp, (lds_void*)&sh.col[wv][b][u * 64], 4, 0, 0);
        } else {
          __builtin_amdgcn_global_load_lds(vp, (lds_void*)&sh.val[wv][b][u * 64], 16, 0, kNonTemporal);
          __builtin_amdgcn_global_load_lds(cp, (lds_void*)&sh.col[wv][b][u * 64], 4, 0, kNonTemporal);
        }
      }
    }
  };

  int rp_cur = load_rp(0);
  int rp_nxt = load_rp(1);
  // own-row operands of row r of tile g (rows past the end read row 0)
  const int my_row = tile_row0(g) + r;
  const bool my_valid = my_row < dim;
  const int my_ld = my_valid ? my_row : 0;
  const d2 w_old = tod2(a.wcur[my_ld]);
  d2 p_old = {0.0, 0.0};
  if (MODE == kLeja && !a.first) p_old = tod2(a.pacc[my_ld]);
  if (stopped) return;  // uniform over the workgroup

  Tile T = tile_of(0, rp_cur);
  int buf = 0;
  if (T.total > 0) issue(T, 0, 0);
  double pw = 0.0, pv = 0.0;
  d2 res_w = {0.0, 0.0}, res_p = {0.0, 0.0};

  for (int j = 0; j < kTPW && T.nr > 0; ++j) {
    const Tile Tn = tile_of(j + 1, rp_nxt);
    // this lane's entry ranges in the tile's entry stream
    int s1 = 0, e1 = 0, s2 = 0, e2 = 0;
    {
      const int q0 = __shfl(rp_cur, r, 64), q1 = __shfl(rp_cur, r + 1, 64);
      const int q2 = __shfl(rp_cur, 32 + r, 64), q3 = __shfl(rp_cur, 33 + r, 64);
      if (r < T.nr) {
        s1 = q0 - T.base1;
        e1 = q1 - T.base1;
        s2 = T.n1 + q2 - T.base2;
        e2 = T.n1 + q3 - T.base2;
      }
    }
    int rp_after = 0;
    d2 acc1 = {0.0, 0.0}, acc2 = {0.0, 0.0};
    int c0 = 0;
    do {
      const bool has = c0 < T.total;  // false only for a tile without entries
      const int hi = min(T.total, c0 + kSCap);
      const int nb = has ? buf ^ 1 : buf;  // where the next chunk goes
      wait_vmem();  // this chunk is in LDS; every earlier access has completed
      if (c0 == 0) rp_after = load_rp(j + 2);
      // the next chunk: the rest of this tile, or the next tile's first
      const bool more = has && hi < T.total;
      bool issued = false;
      auto issue_next = [&]() {
        if (more) issue(T, hi, nb);
        else if (Tn.total > 0) issue(Tn, 0, nb);
        issued = true;
      };
      if (has) {
        const int lo1 = max(s1, c0) + g, end1 = min(e1, hi);
        const int lo2 = max(s2, c0) + g, end2 = min(e2, hi);
        const unsigned vbase = lds_offset(&sh.val[wv][buf][0]), cbase = lds_offset(&sh.col[wv][buf][0]);
        for (int q = 0;; ++q) {
          const int b1 = lo1 + q * kNB * kSG, b2 = lo2 + q * kNB * kSG;
          if (!__any(b1 < end1 || b2 < end2)) break;
          // entry positions in the buffer, clamped into it for the lanes
          // whose slots run past their row (those values are not used)
          int k1[kNB], k2[kNB];
#pragma unroll
          for (int i = 0; i < kNB; ++i) {
            k1[i] = min(b1 + i * kSG - c0, kSCap - 1);
            k2[i] = min(b2 + i * kSG - c0, kSCap - 1);
          }
          int c1[kNB], c2[kNB];
          {
            unsigned ca1[kNB], ca2[kNB];
#pragma unroll
            for (int i = 0; i < kNB; ++i) {
              ca1[i] = cbase + 4u * (unsigned)k1[i];
              ca2[i] = cbase + 4u * (unsigned)k2[i];
            }
            lds_read_cols(ca1, ca2, c1, c2);
          }
          d2 g1[kNB], g2[kNB];
#pragma unroll
          for (int i = 0; i < kNB; ++i) {
            g1[i] = x1[b1 + i * kSG < end1 ? c1[i] : 0];
            g2[i] = x2[b2 + i * kSG < end2 ? c2[i] : 0];
          }
          // the next chunk's copy goes out behind this round's gathers.  The
          // compiler's wait for the gathers waits for it too (it does not count
          // copies into LDS apart from other loads), but in this order the
          // gathers are served first; issued before them, the copy delays the
          // gathers (n = 20: 200 us per iteration against 148)
          if (!issued) issue_next();
          d2 h1[kNB], h2[kNB];
          {
            unsigned va1[kNB], va2[kNB];
#pragma unroll
            for (int i = 0; i < kNB; ++i) {
              va1[i] = vbase + 16u * (unsigned)k1[i];
              va2[i] = vbase + 16u * (unsigned)k2[i];
            }
            lds_read_vals(va1, va2, h1, h2);
          }
#pragma unroll
          for (int i = 0; i < kNB; ++i)
            if (b1 + i * kSG < end1) acc1 += cmul(h1[i], g1[i]);
#pragma unroll
          for (int i = 0; i < kNB; ++i)
            if (b2 + i * kSG < end2) acc2 += cmul(h2[i], g2[i]);
        }
        buf = nb;
      }
      if (!issued) issue_next();
      c0 += kSCap;
    } while (c0 < T.total);
#pragma unroll
    for (int off = 32; off >= kSR; off >>= 1) {
      acc1.x += __shfl_xor(acc1.x, off, 64);
      acc1.y += __shfl_xor(acc1.y, off, 64);
      acc2.x += __shfl_xor(acc2.x, off, 64);
      acc2.y += __shfl_xor(acc2.y, off, 64);
    }
    // the lanes of slot j hold this tile's rows: the Leja update
    if (MODE == kSplitComm && g == j && r < T.nr) {
      res_w = rmul(a.a1, w_old) + rmul(a.kap, d2{-acc2.y, acc2.x});
      res_p = rmul(a.a2, w_old) - rmul(a.kap, d2{-acc1.y, acc1.x});
    }
    if (MODE == kLeja && g == j && r < T.nr) {
      const d2 y = rmul(a.a1, acc1) + rmul(a.a2, acc2);
      const d2 wn = y - rmul(a.sigma, w_old);
      if (a.first) {
        res_p = cmul(tod2(a.d0), w_old) + cmul(tod2(a.d), wn);
        pv += nrm2(w_old);
      } else {
        res_p = p_old + cmul(tod2(a.d), wn);
      }
      res_w = wn;
      pw += nrm2(wn);
    }
    rp_cur = rp_nxt;
    rp_nxt = rp_after;
    T = Tn;
  }
  // The norm partials go through LDS first, then the rows' results: any wait
  // before an LDS access waits for every outstanding store too, and stores
  // still in flight when the wave ends need no wait.
  wait_vmem();  // no copy into this wave's buffers is still in flight
  if (MODE == kLeja) {
    pw = wave_sum(pw);
    pv = wave_sum(pv);
    double* red = reinterpret_cast<double*>(&sh.val[wv][0][0]);  // this wave's own buffer
    if (lane == 0) {
      red[0] = pw;
      red[1] = pv;
    }
    __syncthreads();
    if (tid == 0) {
      double bw = 0.0, bv = 0.0;
      for (int k = 0; k < kSW; ++k) {
        const double* rk = reinterpret_cast<const double*>(&sh.val[k][0][0]);
        bw += rk[0];
        bv += rk[1];
      }
      a.partials[blockIdx.x] = bw;
      if (a.first) a.partials[gridDim.x + blockIdx.x] = bv;
    }
  }
  if (my_valid) {
    a.wout[my_row] = fromd2(res_w);
    a.pacc[my_row] = fromd2(res_p);
  }
}

// ---------------------------------------------------------------------------
// Three-term Leja iteration y = a1 H1 x + a2 H2 x + a3 K x (Method M4 with the
// commutator assembled), streamed the same way: a tile's entry stream is its
// rows' entries of H1, then of H2, then of K; a gather round takes two
// entries of each term per lane (six gathers in flight, as in the two-term
// kernel).  Per lane and term the entries are summed in order and the rows'
// 8 lanes are combined in the fixed shuffle order, the same as the 8-row
// three-term wave-tile kernel, so y is bitwise the same.
constexpr int kNT3 = 3;  // terms
constexpr int kNB3 = 2;  // entries per lane and term in one gather round

__device__ __forceinline__ void lds_read_cols6(const unsigned (&ca)[6], int (&c)[6]) {
  asm volatile(
      "ds_read_b32 %0, %6\n\t"
      "ds_read_b32 %1, %7\n\t"
      "ds_read_b32 %2, %8\n\t"
      "ds_read_b32 %3, %9\n\t"
      "ds_read_b32 %4, %10\n\t"
      "ds_read_b32 %5, %11\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(c[0]), "=&v"(c[1]), "=&v"(c[2]), "=&v"(c[3]), "=&v"(c[4]), "=&v"(c[5])
      : "v"(ca[0]), "v"(ca[1]), "v"(ca[2]), "v"(ca[3]), "v"(ca[4]), "v"(ca[5]));
}

__device__ __forceinline__ void lds_read_vals6(const unsigned (&va)[6], d2 (&h)[6]) {
  asm volatile(
      "ds_read_b128 %0, %6\n\t"
      "ds_read_b128 %1, %7\n\t"
      "ds_read_b128 %2, %8\n\t"
      "ds_read_b128 %3, %9\n\t"
      "ds_read_b128 %4, %10\n\t"
      "ds_read_b128 %5, %11\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(h[0]), "=&v"(h[1]), "=&v"(h[2]), "=&v"(h[3]), "=&v"(h[4]), "=&v"(h[5])
      : "v"(va[0]), "v"(va[1]), "v"(va[2]), "v"(va[3]), "v"(va[4]), "v"(va[5]));
}

struct Tile3 {
  int nr;            // rows of the tile inside the matrix (0: past the end)
  int base[kNT3];    // first entry of each term
  int off[kNT3];     // where each term's entries start in the tile's stream
  int total;         // entries of all terms
};

__global__ __launch_bounds__(kThreads, 4) void csr3_stream_kernel(CsrDev t1, CsrDev t2, CsrDev t3, int dim,
                                                                  IterArgs a_in, double a3_arg, int keep_entries) {
  const IterArgs a = resolve_args(a_in);
  const double a3 = a_in.coef ? a.kap : a3_arg;  // replayed: scale * kappa from the table
  __shared__ StreamLds sh;
  const bool stopped = iteration_stopped(a, reinterpret_cast<double*>(&sh.val[0][0][0]));
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int r = lane % kSR, g = lane / kSR;
  // A lane's term is picked by adding byte offsets between the terms' arrays
  // to term 1's: a three-way select of pointers is compiled into a table of
  // the pointers in scratch memory, indexed per lane.
  const d2* v1 = reinterpret_cast<const d2*>(t1.val);
  const long long dv2 = (long long)((uintptr_t)t2.val - (uintptr_t)t1.val);
  const long long dv3 = (long long)((uintptr_t)t3.val - (uintptr_t)t1.val);
  const long long dc2 = (long long)((uintptr_t)t2.ci - (uintptr_t)t1.ci);
  const long long dc3 = (long long)((uintptr_t)t3.ci - (uintptr_t)t1.ci);
  const long long dr2 = (long long)((uintptr_t)t2.rp - (uintptr_t)t1.rp);
  const long long dr3 = (long long)((uintptr_t)t3.rp - (uintptr_t)t1.rp);
  const d2* x = reinterpret_cast<const d2*>(a.x1);

  auto tile_row0 = [&](int j) { return (L * kSW * kTPW + wv + j * kSW) * kSR; };
  auto tile_rows = [&](int j) { return j < kTPW ? max(0, min(kSR, dim - tile_row0(j))) : 0; };
  // row pointers of tile j: lanes 16 t .. 16 t + nr hold term t's (t < 3); one
  // unconditional load per lane (other lanes and tiles past the end read an
  // entry that exists)
  auto load_rp = [&](int j) {
    const int nr = tile_rows(j);
    const int idx = nr > 0 ? tile_row0(j) + min(lane & 15, nr) : 0;
    const int t = lane >> 4;
    const long long off = t == 0 ? 0 : t == 1 ? dr2 : dr3;
    return *reinterpret_cast<const int*>((uintptr_t)(t1.rp + idx) + off);
  };
  auto tile_of = [&](int j, int v) {
    Tile3 T{tile_rows(j), {0, 0, 0}, {0, 0, 0}, 0};
    if (T.nr > 0) {
      int at = 0;
#pragma unroll
      for (int t = 0; t < kNT3; ++t) {
        T.base[t] = __builtin_amdgcn_readlane(v, 16 * t);
        T.off[t] = at;
        at += __builtin_amdgcn_readlane(v, 16 * t + T.nr) - T.base[t];
      }
      T.total = at;
    }
    return T;
  };
  // copy entries [c0, c0 + 256) of tile T into buffer b (lanes past the end of
  // the chunk re-read its first entry); tiles whose entries start within the
  // first keep_entries of the three terms together are copied with normal
  // loads, the others non-temporal
  auto issue = [&](const Tile3& T, int c0, int b) {
    const int cn = min(kSCap, T.total - c0);
    const bool keep = (long long)T.base[0] + T.base[1] + T.base[2] < keep_entries;  // no int overflow
#pragma unroll 1
    for (int u = 0; u < kSU; ++u) {
      if (u * 64 < cn) {
        const int k = u * 64 + lane;
        const int gk = c0 + (k < cn ? k : 0);
        const bool in1 = gk < T.off[1], in2 = !in1 && gk < T.off[2];
        const int e = in1 ? T.base[0] + gk : in2 ? T.base[1] + (gk - T.off[1]) : T.base[2] + (gk - T.off[2]);
        const d2* vp = reinterpret_cast<const d2*>((uintptr_t)(v1 + e) + (in1 ? 0 : in2 ? dv2 : dv3));
        const int* cp = reinterpret_cast<const int*>((uintptr_t)(t1.ci + e) + (in1 ? 0 : in2 ? dc2 : dc3));
        if (keep) {
          __builtin_amdgcn_global_load_lds(vp, (lds_void*)&sh.val[wv][b][u * 64], 16, 0, 0);
          __builtin_amdgcn_global_load_lds(cp, (lds_void*)&sh.col[wv][b][u * 64], 4, 0, 0);
        } else {
          __builtin_amdgcn_global_load_lds(vp, (lds_void*)&sh.val[wv][b][u * 64], 16, 0, kNonTemporal);
          __builtin_amdgcn_global_load_lds(cp, (lds_void*)&sh.col[wv][b][u * 64], 4, 0, kNonTemporal);
        }
      }
    }
  };

  int rp_cur = load_rp(0);
  int rp_nxt = load_rp(1);
  // own-row operands of row r of tile g (rows past the end read row 0)
  const int my_row = tile_row0(g) + r;
  const bool my_valid = my_row < dim;
  const int my_ld = my_valid ? my_row : 0;
  const d2 w_old = tod2(a.wcur[my_ld]);
  d2 p_old = {0.0, 0.0};
  if (!a.first) p_old = tod2(a.pacc[my_ld]);
  if (stopped) return;  // uniform over the workgroup

  Tile3 T = tile_of(0, rp_cur);
  int buf = 0;
  if (T.total > 0) issue(T, 0, 0);
  double pw = 0.0, pv = 0.0;
  d2 res_w = {0.0, 0.0}, res_p = {0.0, 0.0};

  for (int j = 0; j < kTPW && T.nr > 0; ++j) {
    const Tile3 Tn = tile_of(j + 1, rp_nxt);
    // this lane's entry range of each term in the tile's entry stream
    int s[kNT3] = {0, 0, 0}, e[kNT3] = {0, 0, 0};
#pragma unroll
    for (int t = 0; t < kNT3; ++t) {
      const int q0 = __shfl(rp_cur, 16 * t + r, 64), q1 = __shfl(rp_cur, 16 * t + r + 1, 64);
      if (r < T.nr) {
        s[t] = T.off[t] + q0 - T.base[t];
        e[t] = T.off[t] + q1 - T.base[t];
      }
    }
    int rp_after = 0;
    d2 acc[kNT3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    int c0 = 0;
    do {
      const bool has = c0 < T.total;  // false only for a tile without entries
      const int hi = min(T.total, c0 + kSCap);
      const int nb = has ? buf ^ 1 : buf;  // where the next chunk goes
      wait_vmem();  // this chunk is in LDS; every earlier access has completed
      if (c0 == 0) rp_after = load_rp(j + 2);
      const bool more = has && hi < T.total;
      bool issued = false;
      auto issue_next = [&]() {
        if (more) issue(T, hi, nb);
        else if (Tn.total > 0) issue(Tn, 0, nb);
        issued = true;
      };
      if (has) {
        int lo[kNT3], end[kNT3];
#pragma unroll
        for (int t = 0; t < kNT3; ++t) {
          lo[t] = max(s[t], c0) + g;
          end[t] = min(e[t], hi);
        }
        const unsigned vbase = lds_offset(&sh.val[wv][buf][0]), cbase = lds_offset(&sh.col[wv][buf][0]);
        for (int q = 0;; ++q) {
          int b[kNT3];
#pragma unroll
          for (int t = 0; t < kNT3; ++t) b[t] = lo[t] + q * kNB3 * kSG;
          if (!__any(b[0] < end[0] || b[1] < end[1] || b[2] < end[2])) break;
          // entry positions in the buffer, clamped into it for the lanes
          // whose slots run past their row (those values are not used)
          int k[6];
#pragma unroll
          for (int t = 0; t < kNT3; ++t)
#pragma unroll
            for (int i = 0; i < kNB3; ++i) k[t * kNB3 + i] = min(b[t] + i * kSG - c0, kSCap - 1);
          int c[6];
          {
            unsigned ca[6];
#pragma unroll
            for (int m = 0; m < 6; ++m) ca[m] = cbase + 4u * (unsigned)k[m];
            lds_read_cols6(ca, c);
          }
          d2 gx[6];
#pragma unroll
          for (int t = 0; t < kNT3; ++t)
#pragma unroll
            for (int i = 0; i < kNB3; ++i)
              gx[t * kNB3 + i] = x[b[t] + i * kSG < end[t] ? c[t * kNB3 + i] : 0];
          // the next chunk's copy goes out behind this round's gathers
          if (!issued) issue_next();
          d2 h[6];
          {
            unsigned va[6];
#pragma unroll
            for (int m = 0; m < 6; ++m) va[m] = vbase + 16u * (unsigned)k[m];
            lds_read_vals6(va, h);
          }
#pragma unroll
          for (int t = 0; t < kNT3; ++t)
#pragma unroll
            for (int i = 0; i < kNB3; ++i)
              if (b[t] + i * kSG < end[t]) acc[t] += cmul(h[t * kNB3 + i], gx[t * kNB3 + i]);
        }
        buf = nb;
      }
      if (!issued) issue_next();
      c0 += kSCap;
    } while (c0 < T.total);
#pragma unroll
    for (int off = 32; off >= kSR; off >>= 1)
#pragma unroll
      for (int t = 0; t < kNT3; ++t) {
        acc[t].x += __shfl_xor(acc[t].x, off, 64);
        acc[t].y += __shfl_xor(acc[t].y, off, 64);
      }
    // the lanes of slot j hold this tile's rows: the Leja update
    if (g == j && r < T.nr) {
      const d2 y = rmul(a.a1, acc[0]) + rmul(a.a2, acc[1]) + rmul(a3, acc[2]);
      const d2 wn = y - rmul(a.sigma, w_old);
      if (a.first) {
        res_p = cmul(tod2(a.d0), w_old) + cmul(tod2(a.d), wn);
        pv += nrm2(w_old);
      } else {
        res_p = p_old + cmul(tod2(a.d), wn);
      }
      res_w = wn;
      pw += nrm2(wn);
    }
    rp_cur = rp_nxt;
    rp_nxt = rp_after;
    T = Tn;
  }
  // partials first, then the rows' results (as in the two-term kernel)
  wait_vmem();  // no copy into this wave's buffers is still in flight
  pw = wave_sum(pw);
  pv = wave_sum(pv);
  double* red = reinterpret_cast<double*>(&sh.val[wv][0][0]);  // this wave's own buffer
  if (lane == 0) {
    red[0] = pw;
    red[1] = pv;
  }
  __syncthreads();
  if (tid == 0) {
    double bw = 0.0, bv = 0.0;
    for (int kk = 0; kk < kSW; ++kk) {
      const double* rk = reinterpret_cast<const double*>(&sh.val[kk][0][0]);
      bw += rk[0];
      bv += rk[1];
    }
    a.partials[blockIdx.x] = bw;
    if (a.first) a.partials[gridDim.x + blockIdx.x] = bv;
  }
  if (my_valid) {
    a.wout[my_row] = fromd2(res_w);
    a.pacc[my_row] = fromd2(res_p);
  }
}

}  // namespace

int csr2_stream_grid(int dim) {
  const long long rows = (long long)kSR * kSW * kTPW;
  return (int)std::max<long long>(1, (dim + rows - 1) / rows);
}

hipError_t launch_csr2_stream(int mode, const CsrDev& t1, const CsrDev& t2, int dim, const IterArgs& a,
                              hipStream_t s) {
  // entries (20 bytes each, both terms) kept resident in the MALL
  const long long keep = std::max(0LL, kMallKeepBytes - 80LL * dim) / 20;
  const int keep_entries = (int)std::min<long long>(keep, 1LL << 30);
  if (mode == kLeja) {
    csr2_stream_kernel<kLeja><<<csr2_stream_grid(dim), kThreads, 0, s>>>(t1, t2, dim, a, keep_entries);
  } else if (mode == kSplitComm) {
    if (a.x1 != a.wcur || a.x2 != a.wcur) return hipErrorInvalidValue;  // w is read as its own rows
    csr2_stream_kernel<kSplitComm><<<csr2_stream_grid(dim), kThreads, 0, s>>>(t1, t2, dim, a, keep_entries);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_csr3_stream(const CsrDev& t1, const CsrDev& t2, const CsrDev& t3, int dim, const IterArgs& a,
                              double a3, hipStream_t s) {
  // entries (20 bytes each, the three terms) kept resident in the MALL
  const long long keep = std::max(0LL, kMallKeepBytes - 80LL * dim) / 20;
  const int keep_entries = (int)std::min<long long>(keep, 1LL << 30);
  csr3_stream_kernel<<<csr2_stream_grid(dim), kThreads, 0, s>>>(t1, t2, t3, dim, a, a3, keep_entries);
  return hipGetLastError();
}

}  // namespace magnus
