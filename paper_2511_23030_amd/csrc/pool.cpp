// Chunk store and device residency pool (Sec. III-E "Optimization" and "LRU
// Eviction Strategy").
//
// Host store: every chunk's Gaussians (parameters, Adam moments, step
// counts) in pinned blocks, page-major [page][row][4096], so a page moves
// between host and device with one DMA copy.  Ingest writes one block; each
// loop closure writes the chunks it rebuilds into a new one.  Device pool: the same page
// layout, sized for the budget; a resident chunk owns a list of pages,
// allocated lowest-first so a chunk's pages are usually one contiguous run
// (one copy per run).
#include <algorithm>
#include <cstring>
#include <numeric>
#include <thread>

#include "internal.h"

namespace dcgs {

namespace {

constexpr int PG = dcgs_pool::PG;

int64_t pages_of(int64_t n) { return (n + PG - 1) / PG; }

// Allocate `need` pages, preferring the lowest free page numbers.
std::vector<int32_t> alloc_pages(dcgs_pool *p, int64_t need) {
  DCGS_CHECK((int64_t)p->free_pages.size() >= need, DCGS_E_BUDGET,
             "device page pool exhausted");
  std::vector<int32_t> out(need);
  for (int64_t k = 0; k < need; ++k) {
    out[k] = p->free_pages.back();
    p->free_pages.pop_back();
  }
  return out;
}

void release_pages(dcgs_pool *p, const std::vector<int32_t> &pages) {
  p->free_pages.insert(p->free_pages.end(), pages.begin(), pages.end());
  std::sort(p->free_pages.begin(), p->free_pages.end(), std::greater<int32_t>());
}

// Copy a chunk's pages host <-> device on the copy stream, merging runs of
// consecutive device pages into one copy per array.
void move_chunk(dcgs_pool *p, HostChunk &c, bool to_device) {
  const size_t pbytes = (size_t)p->R * PG * sizeof(float);
  const size_t sbytes = (size_t)PG * sizeof(int32_t);
  hipStream_t st = p->copy;
  int64_t k = 0;
  while (k < c.pages) {
    int64_t run = 1;
    while (k + run < c.pages && c.dev_pages[k + run] == c.dev_pages[k] + run) ++run;
    const int64_t dp = c.dev_pages[k];
    float *hp[3] = {c.params + (size_t)k * p->R * PG, c.m + (size_t)k * p->R * PG,
                    c.v + (size_t)k * p->R * PG};
    float *dv[3] = {p->d_params + (size_t)dp * p->R * PG, p->d_m + (size_t)dp * p->R * PG,
                    p->d_v + (size_t)dp * p->R * PG};
    for (int a = 0; a < 3; ++a) {
      if (to_device)
        DCGS_HIP(hipMemcpyAsync(dv[a], hp[a], run * pbytes, hipMemcpyHostToDevice, st));
      else
        DCGS_HIP(hipMemcpyAsync(hp[a], dv[a], run * pbytes, hipMemcpyDeviceToHost, st));
    }
    int32_t *hs = c.step + (size_t)k * PG;
    int32_t *ds = p->d_step + (size_t)dp * PG;
    if (to_device)
      DCGS_HIP(hipMemcpyAsync(ds, hs, run * sbytes, hipMemcpyHostToDevice, st));
    else
      DCGS_HIP(hipMemcpyAsync(hs, ds, run * sbytes, hipMemcpyDeviceToHost, st));
    k += run;
  }
  const int64_t bytes = c.pages * (int64_t)(3 * pbytes + sbytes);
  if (to_device) {
    p->bytes_h2d += bytes;
    ++p->n_loads;
  } else {
    p->bytes_d2h += bytes;
    ++p->n_evictions;
  }
  DCGS_HIP(hipEventRecord(c.ready, st));
}

// The event that follows every compute-stream use of a chunk last used in
// frame u < now: the first frame event recorded after u.
hipEvent_t after_frame(dcgs_pool *p, int64_t u) {
  hipEvent_t best = nullptr;
  int64_t bf = INT64_MAX;
  for (auto &kv : p->frame_event)
    if (kv.first > u && kv.first < bf) {
      bf = kv.first;
      best = kv.second;
    }
  return best;
}

void mark_frame(dcgs_pool *p, int64_t now, hipStream_t st) {
  if (p->frame_event.count(now)) return;
  hipEvent_t e;
  DCGS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  DCGS_HIP(hipEventRecord(e, st));
  p->frame_event[now] = e;
  // forget frames older than every resident chunk's last use
  int64_t oldest = now;
  for (auto &c : p->chunks)
    if (c.resident && c.last_access >= 0) oldest = std::min(oldest, c.last_access);
  for (auto it = p->frame_event.begin(); it != p->frame_event.end();) {
    if (it->first <= oldest && it->first != now && it->first + 1 <= oldest) {
      (void)hipEventDestroy(it->second);
      it = p->frame_event.erase(it);
    } else {
      ++it;
    }
  }
}

// Write an evictable chunk back to the host store and free its pages.  The
// copy waits for the compute-stream work of the chunk's last frame (for a
// chunk already used in frame `now`, for everything enqueued on `st` so far).
void evict_chunk(dcgs_pool *p, HostChunk &h, int64_t now, hipStream_t st) {
  if (h.last_access >= 0 && h.last_access < now) {
    hipEvent_t e = after_frame(p, h.last_access);
    if (e) DCGS_HIP(hipStreamWaitEvent(p->copy, e, 0));
  } else if (h.last_access >= now) {
    DCGS_HIP(hipEventRecord(p->cut, st));
    DCGS_HIP(hipStreamWaitEvent(p->copy, p->cut, 0));
  }
  move_chunk(p, h, false);
  release_pages(p, h.dev_pages);
  h.dev_pages.clear();
  h.resident = false;
  h.staged = false;
  p->resident_g -= h.n;
}

}  // namespace

void pool_create(dcgs_ctx *ctx, int deg, int64_t budget, dcgs_pool **out) {
  DCGS_CHECK(out && deg >= 0 && deg <= 3 && budget > 0, DCGS_E_INVALID, "pool_create: bad args");
  auto *p = new dcgs_pool();
  p->ctx = ctx;
  p->deg = deg;
  p->R = n_rows(deg);
  p->budget = budget;
  DCGS_HIP(hipEventCreateWithFlags(&p->seg_done, hipEventDisableTiming));
  DCGS_HIP(hipEventCreateWithFlags(&p->cut, hipEventDisableTiming));
  DCGS_HIP(hipStreamCreateWithFlags(&p->copy, hipStreamNonBlocking));
  *out = p;
}

void pool_destroy(dcgs_pool *p) {
  if (!p) return;
  if (p->copy) (void)hipStreamSynchronize(p->copy);
  if (p->d_params) (void)hipFree(p->d_params);
  if (p->d_m) (void)hipFree(p->d_m);
  if (p->d_v) (void)hipFree(p->d_v);
  if (p->d_step) (void)hipFree(p->d_step);
  for (auto &b : p->blocks)
    if (b.base) (void)hipHostFree(b.base);
  if (p->h_seg) (void)hipHostFree(p->h_seg);
  if (p->seg_done) (void)hipEventDestroy(p->seg_done);
  if (p->cut) (void)hipEventDestroy(p->cut);
  for (auto &c : p->chunks)
    if (c.ready) (void)hipEventDestroy(c.ready);
  for (auto &kv : p->frame_event) (void)hipEventDestroy(kv.second);
  if (p->copy) (void)hipStreamDestroy(p->copy);
  delete p;
}

void pool_ingest(dcgs_pool *p, const float *params, int64_t n, double s, hipStream_t st) {
  DCGS_CHECK(params && n > 0 && s > 0, DCGS_E_INVALID, "pool_ingest: bad args");
  DCGS_CHECK(p->chunks.empty(), DCGS_E_INVALID, "pool_ingest: pool already holds a scene");
  const int R = p->R;
  p->s = s;
  // 1. chunk id of every Gaussian, computed on the device in batches
  std::vector<uint64_t> ids(n);
  const int64_t B = std::min<int64_t>(n, int64_t(1) << 22);
  float *dmean = nullptr;
  uint64_t *dids = nullptr;
  int *dflag = nullptr;
  DCGS_HIP(hipMalloc(&dmean, 3 * B * sizeof(float)));
  DCGS_HIP(hipMalloc(&dids, B * sizeof(uint64_t)));
  DCGS_HIP(hipMalloc(&dflag, sizeof(int)));
  struct Free {
    void *a, *b, *c;
    ~Free() {
      (void)hipFree(a);
      (void)hipFree(b);
      (void)hipFree(c);
    }
  } fr{dmean, dids, dflag};
  DCGS_HIP(hipMemsetAsync(dflag, 0, sizeof(int), st));
  for (int64_t b0 = 0; b0 < n; b0 += B) {
    const int64_t nb = std::min(B, n - b0);
    DCGS_HIP(hipMemcpy2DAsync(dmean, nb * sizeof(float), params + b0, n * sizeof(float),
                              nb * sizeof(float), 3, hipMemcpyHostToDevice, st));
    launch_chunk_ids(dmean, nb, nb, s, dids, dflag, st);
    DCGS_HIP(hipMemcpyAsync(ids.data() + b0, dids, nb * sizeof(uint64_t),
                            hipMemcpyDeviceToHost, st));
  }
  int flag = 0;
  DCGS_HIP(hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, st));
  DCGS_HIP(hipStreamSynchronize(st));
  DCGS_CHECK(flag == 0, DCGS_E_RANGE, "pool_ingest: chunk coordinate outside Eq. (6) range");
  // 2. group by id, keeping input order inside a chunk
  std::vector<uint32_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0u);
  std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) { return ids[a] < ids[b]; });
  std::vector<std::pair<int64_t, int64_t>> runs;  // [begin, end) into idx
  for (int64_t k = 0; k < n;) {
    int64_t e = k;
    while (e < n && ids[idx[e]] == ids[idx[k]]) ++e;
    runs.push_back({k, e});
    k = e;
  }
  // 3. one pinned block: params, m, v pages + step pages per chunk
  const size_t fpage = (size_t)R * PG * sizeof(float), spage = (size_t)PG * sizeof(int32_t);
  int64_t total_pages = 0;
  for (auto &r : runs) total_pages += pages_of(r.second - r.first);
  const size_t block_bytes = (size_t)total_pages * (3 * fpage + spage);
  char *base = nullptr;
  DCGS_HIP(hipHostMalloc((void **)&base, block_bytes, hipHostMallocDefault));
  p->blocks.push_back({base, (int64_t)runs.size()});
  std::memset(base, 0, block_bytes);
  char *cur = base;
  p->chunks.resize(runs.size());
  for (size_t c = 0; c < runs.size(); ++c) {
    HostChunk &h = p->chunks[c];
    h.block = (int)p->blocks.size() - 1;
    h.id = ids[idx[runs[c].first]];
    h.n = runs[c].second - runs[c].first;
    h.pages = pages_of(h.n);
    h.params = (float *)cur;
    cur += h.pages * fpage;
    h.m = (float *)cur;
    cur += h.pages * fpage;
    h.v = (float *)cur;
    cur += h.pages * fpage;
    h.step = (int32_t *)cur;
    cur += h.pages * spage;
    DCGS_HIP(hipEventCreateWithFlags(&h.ready, hipEventDisableTiming));
  }
  // 4. scatter the input rows into the page-major store (threads over rows)
  auto fill_rows = [&](int r0, int r1) {
    for (int r = r0; r < r1; ++r) {
      const float *src = params + (size_t)r * n;
      for (size_t c = 0; c < runs.size(); ++c) {
        HostChunk &h = p->chunks[c];
        for (int64_t k = 0; k < h.n; ++k) {
          const int64_t pg = k >> dcgs_pool::PG_LOG2, off = k & (PG - 1);
          h.params[((size_t)pg * R + r) * PG + off] = src[idx[runs[c].first + k]];
        }
      }
    }
  };
  const int nt = std::max(1, std::min<int>(R, (int)std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back(fill_rows, R * t / nt, R * (t + 1) / nt);
  for (auto &t : th) t.join();
  // 5. device pool: the budget in pages plus one partial page per chunk
  p->page_cap = std::min<int64_t>(total_pages, pages_of(p->budget) + (int64_t)runs.size());
  DCGS_HIP(hipMalloc(&p->d_params, p->page_cap * fpage));
  DCGS_HIP(hipMalloc(&p->d_m, p->page_cap * fpage));
  DCGS_HIP(hipMalloc(&p->d_v, p->page_cap * fpage));
  DCGS_HIP(hipMalloc(&p->d_step, p->page_cap * spage));
  p->free_pages.resize(p->page_cap);
  for (int64_t k = 0; k < p->page_cap; ++k) p->free_pages[k] = (int32_t)(p->page_cap - 1 - k);
  pool_index(p, st);
}

void pool_index(dcgs_pool *p, hipStream_t st) {
  p->index.clear();
  std::vector<uint64_t> h_ids(p->chunks.size());
  for (size_t c = 0; c < p->chunks.size(); ++c) {
    h_ids[c] = p->chunks[c].id;
    p->index[h_ids[c]] = (int)c;
  }
  if (h_ids.empty()) return;
  uint64_t *d = p->d_ids.need(h_ids.size());
  DCGS_HIP(hipMemcpyAsync(d, h_ids.data(), h_ids.size() * sizeof(uint64_t),
                          hipMemcpyHostToDevice, st));
  DCGS_HIP(hipStreamSynchronize(st));
}

// Drop a chunk from the store (the caller has synchronised the device and
// keeps what it needs of the chunk's data): its device pages go back to the
// pool, and its block is freed once it holds no chunk.
void pool_release_chunk(dcgs_pool *p, HostChunk &h) {
  if (h.resident) {
    release_pages(p, h.dev_pages);
    h.dev_pages.clear();
    h.resident = false;
    p->resident_g -= h.n;
  }
  if (h.ready) (void)hipEventDestroy(h.ready);
  h.ready = nullptr;
  if (h.block >= 0) {
    auto &b = p->blocks[h.block];
    if (--b.live == 0 && b.base) {
      (void)hipHostFree(b.base);
      b.base = nullptr;
    }
  }
  h.block = -1;
}

void pool_require(dcgs_pool *p, const uint64_t *ids, int n, int64_t now, int *loaded,
                  int *evicted, hipStream_t st) {
  DCGS_CHECK(n >= 0 && (ids || n == 0), DCGS_E_INVALID, "pool_require: bad args");
  std::vector<int> need;
  need.reserve(n);
  for (int k = 0; k < n; ++k) {
    auto it = p->index.find(ids[k]);
    DCGS_CHECK(it != p->index.end(), DCGS_E_NOT_RESIDENT, "pool_require: unknown chunk id");
    need.push_back(it->second);
  }
  std::sort(need.begin(), need.end());
  need.erase(std::unique(need.begin(), need.end()), need.end());
  std::vector<char> is_need(p->chunks.size(), 0);
  int64_t total = p->resident_g;
  std::vector<int> load;
  for (int c : need) {
    is_need[c] = 1;
    if (!p->chunks[c].resident) {
      load.push_back(c);
      total += p->chunks[c].n;
    }
  }
  // evictable: resident and not needed, oldest access first, ties by id
  std::vector<int> evictable;
  for (size_t c = 0; c < p->chunks.size(); ++c)
    if (p->chunks[c].resident && !is_need[c]) evictable.push_back((int)c);
  std::sort(evictable.begin(), evictable.end(), [&](int a, int b) {
    const HostChunk &x = p->chunks[a], &y = p->chunks[b];
    return x.last_access != y.last_access ? x.last_access < y.last_access : x.id < y.id;
  });
  std::vector<int> evict;
  for (int c : evictable) {
    if (total <= p->budget) break;
    evict.push_back(c);
    total -= p->chunks[c].n;
  }
  DCGS_CHECK(total <= p->budget, DCGS_E_BUDGET,
             "pool_require: visible chunks exceed the residency budget");
  int64_t free_after = (int64_t)p->free_pages.size();
  for (int c : evict) free_after += p->chunks[c].pages;
  int64_t need_pages = 0;
  for (int c : load) need_pages += p->chunks[c].pages;
  DCGS_CHECK(need_pages <= free_after, DCGS_E_BUDGET, "pool_require: device pages exhausted");
  mark_frame(p, now, st);
  for (int c : evict) evict_chunk(p, p->chunks[c], now, st);
  for (int c : load) {
    HostChunk &h = p->chunks[c];
    h.dev_pages = alloc_pages(p, h.pages);
    move_chunk(p, h, true);
    h.resident = true;
    h.staged = false;
    p->resident_g += h.n;
    ++p->n_misses;
  }
  for (int c : need) {
    HostChunk &h = p->chunks[c];
    if (h.staged) {
      ++p->n_hits;
      h.staged = false;
    }
    // the compute stream waits for the chunk's last copy (no host wait)
    DCGS_HIP(hipStreamWaitEvent(st, h.ready, 0));
    h.last_access = now;
  }
  if (loaded) *loaded = (int)load.size();
  if (evicted) *evicted = (int)evict.size();
}

void pool_prefetch(dcgs_pool *p, const uint64_t *ids, int n, int64_t now, int *staged,
                   hipStream_t st) {
  DCGS_CHECK(n >= 0 && (ids || n == 0), DCGS_E_INVALID, "pool_prefetch: bad args");
  std::vector<int> want;
  want.reserve(n);
  std::vector<char> wanted(p->chunks.size(), 0);
  for (int k = 0; k < n; ++k) {
    auto it = p->index.find(ids[k]);
    DCGS_CHECK(it != p->index.end(), DCGS_E_NOT_RESIDENT, "pool_prefetch: unknown chunk id");
    want.push_back(it->second);
    wanted[it->second] = 1;
  }
  mark_frame(p, now, st);
  int done = 0;
  for (int c : want) {
    HostChunk &h = p->chunks[c];
    if (h.resident) continue;
    // room: evict chunks neither used in this frame nor asked for, oldest
    // first (best effort)
    std::vector<int> evictable;
    for (size_t e = 0; e < p->chunks.size(); ++e) {
      const HostChunk &x = p->chunks[e];
      if (x.resident && x.last_access < now && !wanted[e]) evictable.push_back((int)e);
    }
    std::sort(evictable.begin(), evictable.end(), [&](int a, int b) {
      const HostChunk &x = p->chunks[a], &y = p->chunks[b];
      return x.last_access != y.last_access ? x.last_access < y.last_access : x.id < y.id;
    });
    int64_t total = p->resident_g + h.n, pages_free = (int64_t)p->free_pages.size();
    size_t m = 0;
    while (m < evictable.size() && (total > p->budget || pages_free < h.pages)) {
      total -= p->chunks[evictable[m]].n;
      pages_free += p->chunks[evictable[m]].pages;
      ++m;
    }
    if (total > p->budget || pages_free < h.pages) break;  // budget full: stop staging
    for (size_t q = 0; q < m; ++q) evict_chunk(p, p->chunks[evictable[q]], now, st);
    h.dev_pages = alloc_pages(p, h.pages);
    move_chunk(p, h, true);
    h.resident = true;
    h.staged = true;
    h.last_access = now;
    p->resident_g += h.n;
    ++p->n_prefetched;
    ++done;
  }
  if (staged) *staged = done;
}

void pool_read_chunk(dcgs_pool *p, uint64_t id, float *params, float *m, float *v,
                     int32_t *step) {
  auto it = p->index.find(id);
  DCGS_CHECK(it != p->index.end(), DCGS_E_NOT_RESIDENT, "pool_read_chunk: unknown chunk id");
  HostChunk &h = p->chunks[it->second];
  DCGS_HIP(hipDeviceSynchronize());  // pending copies and kernels touching the chunk
  const int R = p->R;
  const size_t fpage = (size_t)R * PG, n_f = h.pages * fpage;
  std::vector<float> tp, tm, tv;
  std::vector<int32_t> ts;
  const float *sp = h.params, *sm = h.m, *sv = h.v;
  const int32_t *ss = h.step;
  if (h.resident) {
    tp.resize(n_f);
    tm.resize(n_f);
    tv.resize(n_f);
    ts.resize(h.pages * PG);
    for (int64_t k = 0; k < h.pages; ++k) {
      const size_t dp = h.dev_pages[k];
      DCGS_HIP(hipMemcpy(tp.data() + k * fpage, p->d_params + dp * fpage, fpage * 4, hipMemcpyDeviceToHost));
      DCGS_HIP(hipMemcpy(tm.data() + k * fpage, p->d_m + dp * fpage, fpage * 4, hipMemcpyDeviceToHost));
      DCGS_HIP(hipMemcpy(tv.data() + k * fpage, p->d_v + dp * fpage, fpage * 4, hipMemcpyDeviceToHost));
      DCGS_HIP(hipMemcpy(ts.data() + k * PG, p->d_step + dp * PG, PG * 4, hipMemcpyDeviceToHost));
    }
    sp = tp.data();
    sm = tm.data();
    sv = tv.data();
    ss = ts.data();
  }
  for (int64_t k = 0; k < h.n; ++k) {
    const int64_t pg = k >> dcgs_pool::PG_LOG2, off = k & (PG - 1);
    for (int r = 0; r < R; ++r) {
      const size_t src = ((size_t)pg * R + r) * PG + off;
      if (params) params[(size_t)r * h.n + k] = sp[src];
      if (m) m[(size_t)r * h.n + k] = sm[src];
      if (v) v[(size_t)r * h.n + k] = sv[src];
    }
    if (step) step[k] = ss[(size_t)pg * PG + off];
  }
}

void pool_compact(dcgs_pool *p, const uint64_t *ids, const uint16_t *masks, int n_ids,
                  float *out, int64_t out_stride, int32_t *out_src, uint16_t *out_gmask,
                  int64_t capacity, int64_t *n_out, hipStream_t st) {
  DCGS_CHECK(n_ids >= 0 && (ids || n_ids == 0) && n_out, DCGS_E_INVALID, "compact: bad args");
  std::vector<std::pair<int, uint16_t>> act;
  for (int k = 0; k < n_ids; ++k) {
    auto it = p->index.find(ids[k]);
    DCGS_CHECK(it != p->index.end(), DCGS_E_NOT_RESIDENT, "compact: unknown chunk id");
    DCGS_CHECK(p->chunks[it->second].resident, DCGS_E_NOT_RESIDENT, "compact: chunk not resident");
    act.push_back({it->second, masks ? masks[k] : (uint16_t)0xFFFF});
  }
  std::sort(act.begin(), act.end());  // chunks are stored in ascending id order
  int64_t total = 0;
  size_t nseg = 0;
  for (auto &a : act) {
    total += p->chunks[a.first].n;
    nseg += p->chunks[a.first].pages;
  }
  *n_out = total;
  DCGS_CHECK(total <= capacity, DCGS_E_CAPACITY, "compact: output capacity too small");
  DCGS_CHECK(out && out_stride >= total, DCGS_E_INVALID, "compact: bad output");
  if (nseg == 0) return;
  if (nseg > p->h_seg_cap) {
    if (p->h_seg) DCGS_HIP(hipHostFree(p->h_seg));
    p->h_seg_cap = nseg * 2;
    DCGS_HIP(hipHostMalloc((void **)&p->h_seg, p->h_seg_cap * sizeof(int4), hipHostMallocDefault));
  } else {
    DCGS_HIP(hipEventSynchronize(p->seg_done));  // previous upload finished
  }
  int64_t dst = 0;
  size_t s = 0;
  for (auto &a : act) {
    HostChunk &h = p->chunks[a.first];
    for (int64_t k = 0; k < h.pages; ++k) {
      const int cnt = (int)std::min<int64_t>(PG, h.n - k * PG);
      p->h_seg[s++] = make_int4(h.dev_pages[k], cnt, (int)dst, (int)a.second);
      dst += cnt;
    }
  }
  int4 *dseg = p->d_seg.need(nseg);
  DCGS_HIP(hipMemcpyAsync(dseg, p->h_seg, nseg * sizeof(int4), hipMemcpyHostToDevice, st));
  DCGS_HIP(hipEventRecord(p->seg_done, st));
  StageTimer tm(p->ctx, DCGS_STAGE_COMPACT, st);
  launch_compact(p->d_params, p->R, dseg, (int)nseg, nullptr, out, out_stride, out_src,
                 out_gmask, st);
}

}  // namespace dcgs
