// Loop-closure correction of the chunk store (Sec. III-G) for gfx950.
//
// "Cross-Chunk Transformation": the chunks each affected keyframe sees (the
// exact visibility test of the chunk selection) are collected once; every
// Gaussian of such a chunk takes the rigid correction (R, t) of the first
// affected keyframe that sees its chunk (the global transformation mask: no
// Gaussian is corrected twice): mean <- R mean + t, quaternion <- q_R (x) q.
// "Chunk Redistribution": a corrected Gaussian goes to the chunk of its new
// mean (Eq. 5); every other Gaussian stays in its chunk.  The chunks that
// lose or receive Gaussians are rebuilt by a stable radix sort on (new
// chunk, old chunk) and a scatter into the page-major store layout.
// "Post-Correction Refinement": the Gaussians of the chunks a junction
// camera sees get their opacity logit capped at logit(0.01), their Adam
// moments and step count cleared, fused into the scatter.
//
// The affected chunks are handled in one batch in device memory: their
// pages are gathered (from the device pool when resident, else from the
// pinned host store), corrected, sorted and scattered into a staging copy
// of the new host block, which one DMA copy writes back.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_set>

#include "internal.h"

namespace dcgs {
namespace {

constexpr int PG = dcgs_pool::PG;
constexpr int kOpacityRow = 10;
constexpr int kCorr = 16;  // per keyframe: R row-major (9), t (3), q_R (w, x, y, z)

__global__ void k_first_owner(const uint16_t *__restrict__ mask, int n, int k0,
                              int32_t *__restrict__ owner) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned m = mask[i];
  if (m != 0 && owner[i] < 0) owner[i] = k0 + __builtin_ctz(m);
}

__global__ void k_or_mask(const uint16_t *__restrict__ mask, int n, uint8_t *__restrict__ hit) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && mask[i] != 0) hit[i] = 1;
}

// One thread per slot of the workspace pages [page0, page0 + gridDim.y).
// seg[page] = {source rank, Gaussians in the page, owner, -}.
__global__ void __launch_bounds__(256)
    k_lc_transform(float *__restrict__ P, int R, const int4 *__restrict__ seg,
                   const uint64_t *__restrict__ page_id, int64_t page0,
                   const double *__restrict__ corr, double s, uint64_t *__restrict__ new_id,
                   unsigned long long *__restrict__ moved, int *__restrict__ flag) {
  const int64_t page = page0 + blockIdx.y;
  const int off = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t slot = page * PG + off;
  const int4 sg = seg[page];
  const uint64_t old = page_id[page];
  bool mv = false;
  if (off >= sg.y) {
    new_id[slot] = ~uint64_t(0);
  } else if (sg.z < 0) {
    new_id[slot] = old;
  } else {
    const double *c = corr + (int64_t)kCorr * sg.z;
    float *g = P + page * R * PG + off;
    const double x = g[0], y = g[PG], z = g[2 * PG];
    float mf[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      // ((R_i0 x + R_i1 y) + R_i2 z) + t_i, each operation rounded (no fma)
      const double a = __dadd_rn(__dmul_rn(c[3 * i], x), __dmul_rn(c[3 * i + 1], y));
      const double b = __dadd_rn(__dadd_rn(a, __dmul_rn(c[3 * i + 2], z)), c[9 + i]);
      mf[i] = (float)b;
      g[i * PG] = mf[i];
    }
    const double aw = c[12], ax = c[13], ay = c[14], az = c[15];
    const double bw = g[6 * PG], bx = g[7 * PG], by = g[8 * PG], bz = g[9 * PG];
    g[6 * PG] = (float)(aw * bw - ax * bx - ay * by - az * bz);
    g[7 * PG] = (float)(aw * bx + ax * bw + ay * bz - az * by);
    g[8 * PG] = (float)(aw * by - ax * bz + ay * bw + az * bx);
    g[9 * PG] = (float)(aw * bz + ax * by - ay * bx + az * bw);
    // Eq. (5) on the corrected float32 mean, Eq. (6) encoding
    const double half = 0.5 * s;
    const int64_t lo = -(int64_t(1) << 20), hi = (int64_t(1) << 20) - 1;
    int64_t cc[3];
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cc[i] = (int64_t)floor(((double)mf[i] + half) / s);
      ok = ok && cc[i] >= lo && cc[i] <= hi;
    }
    uint64_t id = ~uint64_t(0);
    if (ok)
      id = (uint64_t(cc[0] - lo) << 42) | (uint64_t(cc[1] - lo) << 21) | uint64_t(cc[2] - lo);
    else
      *flag = 1;
    new_id[slot] = id;
    mv = id != old;
  }
  const uint64_t b = __ballot(mv);
  if (threadIdx.x % kWave == 0 && b) atomicAdd(moved, (unsigned long long)__popcll(b));
}

// Distinct values of an ascending array (UINT64_MAX entries excluded): the
// first position of each run.
__global__ void k_run_flags(const uint64_t *__restrict__ a, int64_t n, uint32_t *__restrict__ f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  f[i] = (a[i] != ~uint64_t(0) && (i == 0 || a[i] != a[i - 1])) ? 1u : 0u;
}

__global__ void k_run_write(const uint64_t *__restrict__ a, const uint32_t *__restrict__ f,
                            const uint32_t *__restrict__ pos, int64_t n,
                            uint64_t *__restrict__ ids, int64_t *__restrict__ first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !f[i]) return;
  ids[pos[i]] = a[i];
  first[pos[i]] = i;
}

// key = rank of the slot's new chunk among the rebuilt chunks * nS + rank
// of its source chunk; padding slots get pad (sorted last).
__global__ void k_lc_keys(const int4 *__restrict__ seg, const uint64_t *__restrict__ new_id,
                          int64_t n_slots, const uint64_t *__restrict__ out_ids, int n_out,
                          uint32_t nS, uint32_t pad, uint32_t *__restrict__ keys,
                          uint32_t *__restrict__ vals, int *__restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slots) return;
  const int4 sg = seg[i / PG];
  uint32_t key = pad;
  if ((int)(i % PG) < sg.y) {
    const uint64_t id = new_id[i];
    int lo = 0, hi = n_out;  // first out_ids[k] >= id
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (out_ids[mid] < id) lo = mid + 1; else hi = mid;
    }
    if (lo < n_out && out_ids[lo] == id)
      key = (uint32_t)lo * nS + (uint32_t)sg.x;
    else
      *flag = 1;  // a slot whose chunk was not planned: the host plan is wrong
  }
  keys[i] = key;
  vals[i] = (uint32_t)i;
}

struct OutChunk {
  int64_t start;   // first sorted position
  int64_t n;       // Gaussians
  int64_t base;    // float offset of the chunk's params pages in the block
  int64_t pages;
  int32_t reset;
  int32_t pad_;
};

// Sorted position i -> page-major slot of its output chunk.  One thread per
// Gaussian: consecutive threads read consecutive workspace slots and write
// consecutive slots of one chunk for each row.
__global__ void __launch_bounds__(256)
    k_lc_scatter(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                 int64_t n_valid, uint32_t nS, uint32_t nO, const OutChunk *__restrict__ oc,
                 const float *__restrict__ P, const float *__restrict__ M,
                 const float *__restrict__ V, const int32_t *__restrict__ S, int R,
                 float *__restrict__ out, float cap, int *__restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_valid) return;
  const uint32_t k = keys[i] / nS;
  // the host's plan of the rebuilt chunks must agree with the sorted keys;
  // a disagreement is reported and nothing is written out of place
  if (k >= nO) {
    *flag = 1;
    return;
  }
  const OutChunk o = oc[k];
  const int64_t j = i - o.start, src = vals[i];
  if (j < 0 || j >= o.n) {
    *flag = 1;
    return;
  }
  const int64_t sp = src / PG, so = src % PG, pg = j / PG, po = j % PG;
  const int64_t span = o.pages * R * PG;
  float *dP = out + o.base, *dM = dP + span, *dV = dM + span;
  int32_t *dS = reinterpret_cast<int32_t *>(dV + span);
  const bool reset = o.reset != 0;
  for (int r = 0; r < R; ++r) {
    const int64_t a = (sp * R + r) * PG + so, b = (pg * R + r) * PG + po;
    float val = P[a];
    if (reset && r == kOpacityRow) val = fminf(val, cap);
    dP[b] = val;
    dM[b] = reset ? 0.0f : M[a];
    dV[b] = reset ? 0.0f : V[a];
  }
  dS[pg * PG + po] = reset ? 0 : S[sp * PG + so];
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

int64_t pages_of(int64_t n) { return (n + PG - 1) / PG; }

// Unit quaternion (w, x, y, z), w >= 0, of a rotation matrix (row-major),
// by Shepperd's method: the largest of 4w^2, 4x^2, 4y^2, 4z^2 from the
// trace and diagonal, the other components from the off-diagonal sums and
// differences divided by it.
void quat_of(const double *m, double q[4]) {
  const double tr = m[0] + m[4] + m[8];
  const double d[4] = {1 + tr, 1 + 2 * m[0] - tr, 1 + 2 * m[4] - tr, 1 + 2 * m[8] - tr};
  const int k = (int)(std::max_element(d, d + 4) - d);
  const double r = std::sqrt(d[k]), h = 0.5 / r;
  if (k == 0) {
    q[0] = 0.5 * r; q[1] = (m[7] - m[5]) * h; q[2] = (m[2] - m[6]) * h; q[3] = (m[3] - m[1]) * h;
  } else if (k == 1) {
    q[1] = 0.5 * r; q[0] = (m[7] - m[5]) * h; q[2] = (m[1] + m[3]) * h; q[3] = (m[2] + m[6]) * h;
  } else if (k == 2) {
    q[2] = 0.5 * r; q[0] = (m[2] - m[6]) * h; q[1] = (m[1] + m[3]) * h; q[3] = (m[5] + m[7]) * h;
  } else {
    q[3] = 0.5 * r; q[0] = (m[3] - m[1]) * h; q[1] = (m[2] + m[6]) * h; q[2] = (m[5] + m[7]) * h;
  }
  if (q[0] < 0)
    for (int a = 0; a < 4; ++a) q[a] = -q[a];
}

// Copy a chunk's pages (params, m, v, step) to workspace pages [page0, ...).
void gather_chunk(dcgs_pool *p, const HostChunk &h, float *wP, float *wM, float *wV, int32_t *wS,
                  int64_t page0, hipStream_t st) {
  const size_t fpage = (size_t)p->R * PG, spage = PG;
  if (!h.resident) {
    const size_t nf = h.pages * fpage * sizeof(float), ns = h.pages * spage * sizeof(int32_t);
    DCGS_HIP(hipMemcpyAsync(wP + page0 * fpage, h.params, nf, hipMemcpyHostToDevice, st));
    DCGS_HIP(hipMemcpyAsync(wM + page0 * fpage, h.m, nf, hipMemcpyHostToDevice, st));
    DCGS_HIP(hipMemcpyAsync(wV + page0 * fpage, h.v, nf, hipMemcpyHostToDevice, st));
    DCGS_HIP(hipMemcpyAsync(wS + page0 * spage, h.step, ns, hipMemcpyHostToDevice, st));
    return;
  }
  int64_t k = 0;
  while (k < h.pages) {
    int64_t run = 1;
    while (k + run < h.pages && h.dev_pages[k + run] == h.dev_pages[k] + run) ++run;
    const int64_t dp = h.dev_pages[k], wp = page0 + k;
    const size_t nf = run * fpage * sizeof(float), ns = run * spage * sizeof(int32_t);
    DCGS_HIP(hipMemcpyAsync(wP + wp * fpage, p->d_params + dp * fpage, nf, hipMemcpyDeviceToDevice, st));
    DCGS_HIP(hipMemcpyAsync(wM + wp * fpage, p->d_m + dp * fpage, nf, hipMemcpyDeviceToDevice, st));
    DCGS_HIP(hipMemcpyAsync(wV + wp * fpage, p->d_v + dp * fpage, nf, hipMemcpyDeviceToDevice, st));
    DCGS_HIP(hipMemcpyAsync(wS + wp * spage, p->d_step + dp * spage, ns, hipMemcpyDeviceToDevice, st));
    k += run;
  }
}

// Per-chunk OR over groups of up to 16 cameras of the visibility masks.
std::vector<uint8_t> visible(const dcgs_camera *cams, int n, const uint64_t *d_ids, int n_chunks,
                             double s, hipStream_t st) {
  std::vector<uint8_t> hit(n_chunks, 0);
  if (n == 0 || n_chunks == 0) return hit;
  DevBuf<uint16_t> mask;
  DevBuf<uint8_t> d_hit;
  uint16_t *dm = mask.need(n_chunks);
  uint8_t *dh = d_hit.need(n_chunks);
  DCGS_HIP(hipMemsetAsync(dh, 0, n_chunks, st));
  for (int g = 0; g < n; g += kMaxViews) {
    launch_select_mask(cams + g, std::min(kMaxViews, n - g), d_ids, n_chunks, s, dm, st);
    hipLaunchKernelGGL(k_or_mask, dim3(blocks_for(n_chunks)), dim3(256), 0, st, dm, n_chunks, dh);
    DCGS_LAUNCH_CHECK();
  }
  DCGS_HIP(hipMemcpyAsync(hit.data(), dh, n_chunks, hipMemcpyDeviceToHost, st));
  DCGS_HIP(hipStreamSynchronize(st));
  return hit;
}

}  // namespace

void pool_loop_closure(dcgs_pool *p, const dcgs_camera *keyframes, const double *corr_in,
                       int n_kf, const dcgs_camera *junctions, int n_junctions,
                       int64_t *stats, int n_stats, hipStream_t st) {
  DCGS_CHECK(n_kf >= 0 && n_junctions >= 0 && (keyframes && corr_in || n_kf == 0) &&
                 (junctions || n_junctions == 0) && (stats || n_stats <= 0),
             DCGS_E_INVALID, "loop_closure: bad args");
  DCGS_CHECK(!p->chunks.empty(), DCGS_E_INVALID, "loop_closure: the pool holds no scene");
  const double s = p->s;
  const int R = p->R;
  const size_t fpage = (size_t)R * PG;
  int64_t st_out[7] = {0, 0, 0, 0, 0, 0, 0};
  // ingestion is paused: finish every pending kernel and copy first
  DCGS_HIP(hipDeviceSynchronize());
  const int nC = (int)p->chunks.size();
  const uint64_t *d_ids = p->d_ids.p;

  // 1. owner of each chunk: the first affected keyframe that sees it
  std::vector<int32_t> owner(nC, -1);
  DevBuf<double> d_corr;
  if (n_kf > 0) {
    std::vector<double> corr((size_t)n_kf * kCorr);
    for (int k = 0; k < n_kf; ++k) {
      double *c = corr.data() + (size_t)k * kCorr;
      std::memcpy(c, corr_in + (size_t)k * 12, 12 * sizeof(double));
      quat_of(c, c + 12);
    }
    double *dc = d_corr.need(corr.size());
    DCGS_HIP(hipMemcpyAsync(dc, corr.data(), corr.size() * sizeof(double), hipMemcpyHostToDevice,
                            st));
    DevBuf<uint16_t> mask;
    DevBuf<int32_t> d_owner;
    uint16_t *dm = mask.need(nC);
    int32_t *dow = d_owner.need(nC);
    DCGS_HIP(hipMemsetAsync(dow, 0xFF, nC * sizeof(int32_t), st));  // -1
    for (int g = 0; g < n_kf; g += kMaxViews) {
      launch_select_mask(keyframes + g, std::min(kMaxViews, n_kf - g), d_ids, nC, s, dm, st);
      hipLaunchKernelGGL(k_first_owner, dim3(blocks_for(nC)), dim3(256), 0, st, dm, nC, g, dow);
      DCGS_LAUNCH_CHECK();
    }
    DCGS_HIP(hipMemcpyAsync(owner.data(), dow, nC * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    DCGS_HIP(hipStreamSynchronize(st));
  }
  std::vector<int> A;
  int64_t pagesA = 0, nA = 0;
  for (int c = 0; c < nC; ++c)
    if (owner[c] >= 0) {
      A.push_back(c);
      pagesA += p->chunks[c].pages;
      nA += p->chunks[c].n;
    }

  // 2. gather and correct the affected chunks; new chunk of each Gaussian
  DevBuf<float> w1P, w1M, w1V;
  DevBuf<int32_t> w1S;
  DevBuf<int4> d_seg;
  DevBuf<uint64_t> d_pid, d_new, d_tmp;
  DevBuf<unsigned long long> d_moved;
  DevBuf<int> d_flag;
  DevBuf<uint32_t> hist;
  std::vector<uint64_t> tgt_ids;     // distinct new chunks of the corrected Gaussians
  std::vector<int64_t> tgt_count;    // corrected Gaussians going to each
  unsigned long long moved = 0;
  std::vector<int4> seg;
  std::vector<uint64_t> pid;
  if (!A.empty()) {
    float *aP = w1P.need(pagesA * fpage), *aM = w1M.need(pagesA * fpage),
          *aV = w1V.need(pagesA * fpage);
    int32_t *aS = w1S.need(pagesA * PG);
    seg.reserve(pagesA);
    for (int c : A) {
      const HostChunk &h = p->chunks[c];
      gather_chunk(p, h, aP, aM, aV, aS, (int64_t)seg.size(), st);
      for (int64_t k = 0; k < h.pages; ++k) {
        seg.push_back(make_int4(-1, (int)std::min<int64_t>(PG, h.n - k * PG), owner[c], 0));
        pid.push_back(h.id);
      }
    }
    int4 *ds = d_seg.need(pagesA);
    uint64_t *dpid = d_pid.need(pagesA);
    DCGS_HIP(hipMemcpyAsync(ds, seg.data(), pagesA * sizeof(int4), hipMemcpyHostToDevice, st));
    DCGS_HIP(hipMemcpyAsync(dpid, pid.data(), pagesA * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    const int64_t slots = pagesA * PG;
    uint64_t *dn = d_new.need(slots);
    unsigned long long *dmv = d_moved.need(1);
    int *dfl = d_flag.need(1);
    DCGS_HIP(hipMemsetAsync(dmv, 0, sizeof(unsigned long long), st));
    DCGS_HIP(hipMemsetAsync(dfl, 0, sizeof(int), st));
    for (int64_t p0 = 0; p0 < pagesA; p0 += 65535) {
      const int64_t np = std::min<int64_t>(65535, pagesA - p0);
      hipLaunchKernelGGL(k_lc_transform, dim3(PG / 256, (unsigned)np), dim3(256), 0, st, aP, R,
                         ds, dpid, p0, d_corr.p, s, dn, dmv, dfl);
      DCGS_LAUNCH_CHECK();
    }
    // distinct new chunks: sort a copy of the ids, mark run starts
    uint64_t *sorted = d_tmp.need(2 * slots);
    DCGS_HIP(hipMemcpyAsync(sorted, dn, slots * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
    sort_u64_bits(sorted, sorted + slots, slots, 0, 64, hist, st);
    DevBuf<uint32_t> flags, part;
    uint32_t *fl = flags.need(2 * (size_t)slots + 2);
    uint32_t *pos = fl + slots;
    hipLaunchKernelGGL(k_run_flags, dim3(blocks_for(slots)), dim3(256), 0, st, sorted, slots, fl);
    DCGS_LAUNCH_CHECK();
    scan_u32(fl, nullptr, pos, slots, part.need(scan_part_size(slots) + 2), st);
    uint32_t n_t = 0;
    int flag = 0;
    DCGS_HIP(hipMemcpyAsync(&n_t, pos + slots, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    DCGS_HIP(hipMemcpyAsync(&flag, dfl, sizeof(int), hipMemcpyDeviceToHost, st));
    DCGS_HIP(hipMemcpyAsync(&moved, dmv, sizeof(moved), hipMemcpyDeviceToHost, st));
    DCGS_HIP(hipStreamSynchronize(st));
    DCGS_CHECK(flag == 0, DCGS_E_RANGE,
               "loop_closure: a corrected mean leaves the Eq. (6) coordinate range");
    DevBuf<uint64_t> d_tid;
    DevBuf<int64_t> d_first;
    uint64_t *tid = d_tid.need(n_t + 1);
    int64_t *first = d_first.need(n_t + 1);
    hipLaunchKernelGGL(k_run_write, dim3(blocks_for(slots)), dim3(256), 0, st, sorted, fl, pos,
                       slots, tid, first);
    DCGS_LAUNCH_CHECK();
    tgt_ids.resize(n_t);
    std::vector<int64_t> f(n_t);
    DCGS_HIP(hipMemcpyAsync(tgt_ids.data(), tid, n_t * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    DCGS_HIP(hipMemcpyAsync(f.data(), first, n_t * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    DCGS_HIP(hipStreamSynchronize(st));
    tgt_count.resize(n_t);
    for (uint32_t k = 0; k < n_t; ++k) tgt_count[k] = (k + 1 < n_t ? f[k + 1] : nA) - f[k];
  }

  // 3. the store after redistribution, and the junction chunks in it
  std::unordered_set<uint64_t> is_tgt(tgt_ids.begin(), tgt_ids.end());
  std::vector<uint64_t> after;  // ascending
  {
    std::vector<uint64_t> kept;
    for (int c = 0; c < nC; ++c)
      if (owner[c] < 0) kept.push_back(p->chunks[c].id);
    std::set_union(kept.begin(), kept.end(), tgt_ids.begin(), tgt_ids.end(),
                   std::back_inserter(after));
  }
  std::vector<uint8_t> junction;
  if (n_junctions > 0) {
    DevBuf<uint64_t> d_after;
    uint64_t *da = d_after.need(after.size());
    DCGS_HIP(hipMemcpyAsync(da, after.data(), after.size() * sizeof(uint64_t),
                            hipMemcpyHostToDevice, st));
    junction = visible(junctions, n_junctions, da, (int)after.size(), s, st);
  }
  std::unordered_set<uint64_t> is_junction;
  for (size_t k = 0; k < junction.size(); ++k)
    if (junction[k]) is_junction.insert(after[k]);

  // rebuilt chunks: the targets plus untouched junction chunks; sources:
  // affected chunks plus the existing chunks among those
  std::vector<uint64_t> out_ids;
  for (uint64_t id : after)
    if (is_tgt.count(id) || is_junction.count(id)) out_ids.push_back(id);
  std::vector<int> src;  // ascending chunk positions
  for (int c = 0; c < nC; ++c) {
    const uint64_t id = p->chunks[c].id;
    if (owner[c] >= 0 || is_tgt.count(id) || is_junction.count(id)) src.push_back(c);
  }
  if (out_ids.empty() && src.empty()) {
    for (int k = 0; k < std::min(n_stats, 7); ++k) stats[k] = 0;
    return;
  }
  const uint32_t nS = (uint32_t)src.size(), nO = (uint32_t)out_ids.size();
  DCGS_CHECK((uint64_t)nO * nS < 0xFFFFFFFFull, DCGS_E_RANGE,
             "loop_closure: too many chunks in one correction");
  std::unordered_map<uint64_t, int64_t> contrib;
  for (size_t k = 0; k < tgt_ids.size(); ++k) contrib[tgt_ids[k]] = tgt_count[k];

  // 4. full workspace: affected pages first (already corrected), then the
  //    other source chunks
  std::vector<int> rank(nC, -1);
  for (uint32_t r = 0; r < nS; ++r) rank[src[r]] = (int)r;
  for (size_t q = 0, a = 0; a < A.size(); ++a)
    for (int64_t k = 0; k < p->chunks[A[a]].pages; ++k) seg[q++].x = rank[A[a]];
  int64_t pagesS = pagesA;
  std::vector<int> rest;
  for (int c : src)
    if (owner[c] < 0) {
      rest.push_back(c);
      pagesS += p->chunks[c].pages;
    }
  DevBuf<float> wP, wM, wV;
  DevBuf<int32_t> wS;
  float *P = wP.need(pagesS * fpage), *M = wM.need(pagesS * fpage), *V = wV.need(pagesS * fpage);
  int32_t *S = wS.need(pagesS * PG);
  if (pagesA > 0) {
    const size_t nf = pagesA * fpage * sizeof(float);
    DCGS_HIP(hipMemcpyAsync(P, w1P.p, nf, hipMemcpyDeviceToDevice, st));
    DCGS_HIP(hipMemcpyAsync(M, w1M.p, nf, hipMemcpyDeviceToDevice, st));
    DCGS_HIP(hipMemcpyAsync(V, w1V.p, nf, hipMemcpyDeviceToDevice, st));
    DCGS_HIP(hipMemcpyAsync(S, w1S.p, pagesA * PG * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
  }
  for (int c : rest) {
    const HostChunk &h = p->chunks[c];
    gather_chunk(p, h, P, M, V, S, (int64_t)seg.size(), st);
    for (int64_t k = 0; k < h.pages; ++k) {
      seg.push_back(make_int4(rank[c], (int)std::min<int64_t>(PG, h.n - k * PG), -1, 0));
      pid.push_back(h.id);
    }
  }
  const int64_t slots = pagesS * PG;
  DCGS_CHECK(slots < (int64_t(1) << 32), DCGS_E_RANGE,
             "loop_closure: too many Gaussians in one correction");
  int4 *ds = d_seg.need(pagesS);
  // d_seg may have been reallocated: upload the whole table
  DCGS_HIP(hipMemcpyAsync(ds, seg.data(), pagesS * sizeof(int4), hipMemcpyHostToDevice, st));
  uint64_t *dpid = d_pid.need(pagesS);
  DCGS_HIP(hipMemcpyAsync(dpid, pid.data(), pagesS * sizeof(uint64_t), hipMemcpyHostToDevice, st));
  DevBuf<uint64_t> d_new2;
  uint64_t *dn = d_new2.need(slots);
  if (pagesA > 0)
    DCGS_HIP(hipMemcpyAsync(dn, d_new.p, pagesA * PG * sizeof(uint64_t), hipMemcpyDeviceToDevice,
                            st));
  if (pagesS > pagesA) {
    DevBuf<unsigned long long> dmv;
    DevBuf<int> dfl;
    unsigned long long *mv = dmv.need(1);
    int *fl = dfl.need(1);
    DCGS_HIP(hipMemsetAsync(mv, 0, sizeof(unsigned long long), st));
    DCGS_HIP(hipMemsetAsync(fl, 0, sizeof(int), st));
    for (int64_t p0 = pagesA; p0 < pagesS; p0 += 65535) {
      const int64_t np = std::min<int64_t>(65535, pagesS - p0);
      // owner -1 on these pages: ids only, nothing corrected
      hipLaunchKernelGGL(k_lc_transform, dim3(PG / 256, (unsigned)np), dim3(256), 0, st, P, R,
                         ds, dpid, p0, d_corr.p, s, dn, mv, fl);
      DCGS_LAUNCH_CHECK();
    }
  }

  // 5. stable sort by (new chunk, source chunk), then scatter
  std::vector<OutChunk> oc(nO);
  std::vector<int64_t> out_n(nO);
  int64_t n_valid = 0, total_pages = 0;
  for (uint32_t k = 0; k < nO; ++k) {
    const uint64_t id = out_ids[k];
    int64_t n = 0;
    auto it = p->index.find(id);
    if (it != p->index.end() && owner[it->second] < 0) n += p->chunks[it->second].n;
    auto ct = contrib.find(id);
    if (ct != contrib.end()) n += ct->second;
    out_n[k] = n;
    oc[k].start = n_valid;
    oc[k].n = n;
    oc[k].pages = pages_of(n);
    oc[k].base = total_pages * (int64_t)(3 * fpage + PG);
    oc[k].reset = is_junction.count(id) ? 1 : 0;
    n_valid += n;
    total_pages += oc[k].pages;
  }
  const uint32_t pad = nO * nS;
  int bits = 0;
  while (bits < 32 && (uint64_t(1) << bits) <= pad) ++bits;
  DevBuf<uint32_t> d_kv;
  uint32_t *keys = d_kv.need(4 * (size_t)slots);
  uint32_t *vals = keys + slots, *ktmp = vals + slots, *vtmp = ktmp + slots;
  DevBuf<uint64_t> d_out;
  uint64_t *dout = d_out.need(nO);
  DCGS_HIP(hipMemcpyAsync(dout, out_ids.data(), nO * sizeof(uint64_t), hipMemcpyHostToDevice, st));
  DevBuf<int> d_plan;
  int *plan_flag = d_plan.need(1);
  DCGS_HIP(hipMemsetAsync(plan_flag, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_lc_keys, dim3(blocks_for(slots)), dim3(256), 0, st, ds, dn, slots, dout,
                     (int)nO, nS, pad, keys, vals, plan_flag);
  DCGS_LAUNCH_CHECK();
  sort_u32_pairs(keys, vals, ktmp, vtmp, slots, bits, hist, st);
  const size_t block_bytes = (size_t)total_pages * (3 * fpage + PG) * sizeof(float);
  DevBuf<OutChunk> d_oc;
  OutChunk *doc = d_oc.need(nO);
  DCGS_HIP(hipMemcpyAsync(doc, oc.data(), nO * sizeof(OutChunk), hipMemcpyHostToDevice, st));
  DevBuf<float> stage;
  float *dst = stage.need(block_bytes / sizeof(float));
  DCGS_HIP(hipMemsetAsync(dst, 0, block_bytes, st));
  const float cap = (float)std::log(0.01 / 0.99);
  if (n_valid > 0) {
    hipLaunchKernelGGL(k_lc_scatter, dim3(blocks_for(n_valid)), dim3(256), 0, st, keys, vals,
                       n_valid, nS, nO, doc, P, M, V, S, R, dst, cap, plan_flag);
    DCGS_LAUNCH_CHECK();
  }
  char *base = nullptr;
  DCGS_HIP(hipHostMalloc((void **)&base, std::max<size_t>(block_bytes, 1), hipHostMallocDefault));
  struct Guard {
    char *b;
    ~Guard() {
      if (b) (void)hipHostFree(b);
    }
  } guard{base};
  DCGS_HIP(hipMemcpyAsync(base, dst, block_bytes, hipMemcpyDeviceToHost, st));
  int plan_bad = 0;
  DCGS_HIP(hipMemcpyAsync(&plan_bad, plan_flag, sizeof(int), hipMemcpyDeviceToHost, st));
  DCGS_HIP(hipStreamSynchronize(st));
  DCGS_CHECK(plan_bad == 0, DCGS_E_INVALID, "loop_closure: internal chunk plan mismatch");

  // 6. replace the source chunks by the rebuilt ones
  std::vector<HostChunk> fresh(nO);
  const int blk = (int)p->blocks.size();
  for (uint32_t k = 0; k < nO; ++k) {
    HostChunk &h = fresh[k];
    h.id = out_ids[k];
    h.n = out_n[k];
    h.pages = oc[k].pages;
    h.block = blk;
    h.params = reinterpret_cast<float *>(base) + oc[k].base;
    h.m = h.params + h.pages * fpage;
    h.v = h.m + h.pages * fpage;
    h.step = reinterpret_cast<int32_t *>(h.v + h.pages * fpage);
    DCGS_HIP(hipEventCreateWithFlags(&h.ready, hipEventDisableTiming));
  }
  int64_t n_reset = 0;
  for (uint32_t k = 0; k < nO; ++k)
    if (oc[k].reset) n_reset += out_n[k];
  p->blocks.push_back({base, (int64_t)nO});
  guard.b = nullptr;
  std::vector<char> drop(nC, 0);
  for (int c : src) drop[c] = 1;
  std::vector<HostChunk> next;
  next.reserve(nC - src.size() + nO);
  for (int c = 0; c < nC; ++c) {
    if (drop[c])
      pool_release_chunk(p, p->chunks[c]);
    else
      next.push_back(std::move(p->chunks[c]));
  }
  for (auto &h : fresh) next.push_back(std::move(h));
  std::sort(next.begin(), next.end(),
            [](const HostChunk &a, const HostChunk &b) { return a.id < b.id; });
  p->chunks = std::move(next);
  pool_index(p, st);
  st_out[0] = (int64_t)A.size();
  st_out[1] = nA;
  st_out[2] = (int64_t)moved;
  st_out[3] = nS;
  st_out[4] = nO;
  st_out[5] = n_reset;
  st_out[6] = (int64_t)p->chunks.size();
  for (int k = 0; k < std::min(n_stats, 7); ++k) stats[k] = st_out[k];
}

}  // namespace dcgs
