// Batches: many boxes of one method and precision advanced together.
//
// A batch keeps a device table of its boxes (BatchBox) and runs each step
// as one kernel over a work list that spans all boxes (LBE: 256-cell runs;
// DUGKS: tile z-chunks of the fused kernel), on one block per work item or
// a persistent grid whose blocks loop over the items, followed by one
// launch that finalises the global sums of every box.  Buffer indices and
// step counters are kept on the device, so a hipGraph holding several
// captured steps is replayed for long runs.  The grid size (and
// for DUGKS the z-chunk length of a work item) are chosen per batch by
// timing candidate settings on the batch itself (uncommitted trial steps,
// which leave every box's state unchanged), for DUGKS together with the
// column-tile width (16 or 32) of the fused kernel; choices are cached per
// process by (method, precision, compute units, grid sizes) and can be
// shared through a file named by the environment variable DHIT_TUNE_CACHE.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "device_common.hpp"
#include "runtime.hpp"

struct dhit_batch {
  std::vector<dhit_box *> boxes;
  int method = 0, precision = 0;
  hipStream_t stream = nullptr;
  dhit::BatchBox *d_boxes = nullptr;
  std::vector<dhit::BatchBox> h_boxes;
  double *d_partials = nullptr;
  double *d_trial = nullptr;
  size_t cap_boxes = 0, cap_partials = 0;  // capacity of d_boxes/d_trial (boxes) and d_partials (doubles)
  int total_items = 0;
  int grid = 0;
  int chunk = 0;  // DUGKS z-chunk of a work item (0 = per-box default)
  int tile = 32;  // DUGKS column-tile width of the batch's kernel (16 or 32)
  int max_n = 0;  // largest box side
  int cells_per_thread = 1;  // LBE: cells a thread updates (the same for every box of the launch)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_steps = 0;
  bool tuned = false;
  // two pinned staging copies of the table: an upload does not wait for the
  // work queued on the stream, and a copy is rewritten only once the upload
  // that read it (two uploads back) has been done
  dhit::BatchBox *stage[2] = {nullptr, nullptr};
  hipEvent_t stage_done[2] = {nullptr, nullptr};
  bool stage_used[2] = {false, false};
  size_t cap_stage = 0;
  int stage_next = 0;
};

namespace {

constexpr int kGraphSteps = 8;

int cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 256;
  return cus > 0 ? cus : 256;
}

// Grid of a batch that was not tuned: for DUGKS, the blocks the device
// holds at once (each block then loops over work items, with no second wave
// of blocks; on mixes of 32^3 to 256^3 boxes 5% faster than one block per
// work item); for LBE, one block per work item (the dispatcher hands the
// blocks to compute units as they free up: a 64-box FP32 ensemble ran 15%
// faster so than with a persistent grid of 32 blocks per compute unit).
int default_grid(const dhit_batch &bt) {
  const int g = bt.method == DHIT_DUGKS ? cu_count() * dhit::fused_resident_blocks_of(bt.precision, bt.tile)
                                        : bt.total_items;
  return std::min(g, std::max(1, bt.total_items));
}

std::mutex g_tune_mu;
struct TuneChoice {
  int grid, chunk, tile;
};
std::map<std::string, TuneChoice> g_tune_cache;  // key -> choice
bool g_tune_file_read = false;

// Cache key: method, precision, the device's compute-unit count (grid sizes
// are multiples of it) and the sorted grid sizes of the boxes.
std::string tune_key(const dhit_batch &bt) {
  std::vector<int> ns;
  for (auto *b : bt.boxes) ns.push_back(b->n);
  std::sort(ns.begin(), ns.end());
  std::string k = std::to_string(bt.method) + "/" + std::to_string(bt.precision) + "/cu" + std::to_string(cu_count()) + "/";
  for (size_t i = 0; i < ns.size(); ++i) k += (i ? "," : "") + std::to_string(ns[i]);
  return k;
}

void read_tune_file() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char *path = std::getenv("DHIT_TUNE_CACHE");
  if (!path) return;
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  char key[4096];
  int grid, chunk, tile;
  while (std::fscanf(f, "%4095s %d %d %d", key, &grid, &chunk, &tile) == 4)
    if (grid > 0 && chunk >= 0 && (tile == 16 || tile == 32)) g_tune_cache[key] = {grid, chunk, tile};
  std::fclose(f);
}

void write_tune_entry(const std::string &key, const TuneChoice &c) {
  const char *path = std::getenv("DHIT_TUNE_CACHE");
  if (!path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d\n", key.c_str(), c.grid, c.chunk, c.tile);
  std::fclose(f);
}

// Builds the host table for a DUGKS chunk length (0 = each box's default).
void build_table(dhit_batch &bt, int chunk) {
  bt.h_boxes.clear();
  int item = 0;
  size_t partial_off = 0;
  std::vector<size_t> offs;
  for (auto *b : bt.boxes) {
    dhit::BatchBox d;
    std::memset(&d, 0, sizeof(d));
    d.f[0] = b->f[0];
    d.f[1] = b->f[1];
    d.sp = b->sp;
    d.ncell = (int)b->ncell;
    d.item_begin = item;
    if (bt.method == DHIT_DUGKS) {
      const int cz = chunk > 0 ? std::min(chunk, b->n) : dhit::fused_default_chunk(b->n);
      d.nz_chunk = cz;
      d.items = dhit::fused_dugks_items(b->n, bt.tile, cz, &d.tiles_x, &d.tiles_y);
    } else {
      d.items = dhit::lbe_items(b->ncell, bt.cells_per_thread);
    }
    d.hist = b->hist;
    d.cur = b->cur;
    d.step = b->steps;
    offs.push_back(partial_off);
    partial_off += (size_t)d.items * dhit::kNumSums;
    item += d.items;
    bt.h_boxes.push_back(d);
  }
  bt.total_items = item;
  // grow-only: re-forming a batch with no more partials frees nothing
  // (hipFree would wait for the whole device)
  if (partial_off > bt.cap_partials) {
    const size_t cap = std::max(partial_off, 2 * bt.cap_partials);
    if (bt.d_partials) {
      DHIT_HIP(hipStreamSynchronize(bt.stream));
      (void)hipFree(bt.d_partials);
    }
    bt.d_partials = nullptr;
    bt.cap_partials = 0;
    if (hipMalloc(&bt.d_partials, cap * sizeof(double)) != hipSuccess)
      throw dhit::Error(DHIT_ENOMEM, "cannot allocate batch partial sums");
    bt.cap_partials = cap;
  }
  for (size_t i = 0; i < bt.h_boxes.size(); ++i) {
    bt.h_boxes[i].partials = bt.d_partials + offs[i];
    bt.h_boxes[i].trial = bt.d_trial + dhit::kNumSums * i;
  }
  bt.chunk = chunk;
}

void free_stage(dhit_batch &bt) {
  for (int k = 0; k < 2; ++k) {
    if (bt.stage_done[k]) {
      (void)hipEventSynchronize(bt.stage_done[k]);
      (void)hipEventDestroy(bt.stage_done[k]);
    }
    if (bt.stage[k]) (void)hipHostFree(bt.stage[k]);
    bt.stage[k] = nullptr;
    bt.stage_done[k] = nullptr;
    bt.stage_used[k] = false;
  }
  bt.cap_stage = 0;
}

// Uploads the table, refreshing buffer indices and step counters from the
// boxes, through the pinned staging copies (asynchronous on the batch's
// stream).
void upload_table(dhit_batch &bt) {
  const size_t nbox = bt.h_boxes.size();
  for (size_t i = 0; i < bt.boxes.size(); ++i) {
    bt.h_boxes[i].cur = bt.boxes[i]->cur;
    bt.h_boxes[i].step = bt.boxes[i]->steps;
  }
  if (nbox > bt.cap_stage) {
    free_stage(bt);
    const size_t cap = std::max(nbox, (size_t)16);
    for (int k = 0; k < 2; ++k) {
      if (hipHostMalloc(reinterpret_cast<void **>(&bt.stage[k]), cap * sizeof(dhit::BatchBox), hipHostMallocDefault) !=
          hipSuccess) {
        free_stage(bt);
        throw dhit::Error(DHIT_ENOMEM, "cannot allocate the batch's pinned table copies");
      }
      DHIT_HIP(hipEventCreateWithFlags(&bt.stage_done[k], hipEventDisableTiming));
    }
    bt.cap_stage = cap;
  }
  const int k = bt.stage_next;
  bt.stage_next ^= 1;
  if (bt.stage_used[k]) DHIT_HIP(hipEventSynchronize(bt.stage_done[k]));
  std::memcpy(bt.stage[k], bt.h_boxes.data(), nbox * sizeof(dhit::BatchBox));
  DHIT_HIP(hipMemcpyAsync(bt.d_boxes, bt.stage[k], nbox * sizeof(dhit::BatchBox), hipMemcpyHostToDevice, bt.stream));
  DHIT_HIP(hipEventRecord(bt.stage_done[k], bt.stream));
  bt.stage_used[k] = true;
}

void enqueue_step(dhit_batch &bt, int commit) {
  const int nbox = (int)bt.boxes.size();
  if (bt.method == DHIT_DUGKS)
    dhit::launch_dugks_batch(bt.stream, bt.precision, bt.tile, bt.max_n, bt.d_boxes, nbox, bt.total_items, bt.grid);
  else
    dhit::launch_lbe_batch(bt.stream, bt.method, bt.precision, bt.cells_per_thread, bt.d_boxes, nbox, bt.total_items,
                           bt.grid);
  dhit::launch_finalize_batch(bt.stream, bt.d_boxes, nbox, commit);
}

void drop_graph(dhit_batch &bt) {
  if (bt.exec) (void)hipGraphExecDestroy(bt.exec);
  if (bt.graph) (void)hipGraphDestroy(bt.graph);
  bt.exec = nullptr;
  bt.graph = nullptr;
  bt.graph_steps = 0;
}

void capture_graph(dhit_batch &bt) {
  drop_graph(bt);
  DHIT_HIP(hipStreamBeginCapture(bt.stream, hipStreamCaptureModeThreadLocal));
  try {
    for (int s = 0; s < kGraphSteps; ++s) enqueue_step(bt, 1);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(bt.stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  DHIT_HIP(hipStreamEndCapture(bt.stream, &bt.graph));
  DHIT_HIP(hipGraphInstantiate(&bt.exec, bt.graph, nullptr, nullptr, 0));
  bt.graph_steps = kGraphSteps;
}

// Times `reps` uncommitted steps with the current settings (ms per step).
float time_trial(dhit_batch &bt, int reps) {
  hipEvent_t e0, e1;
  DHIT_HIP(hipEventCreate(&e0));
  DHIT_HIP(hipEventCreate(&e1));
  float ms = 0.f;
  try {
    upload_table(bt);
    enqueue_step(bt, 0);  // warm-up
    DHIT_HIP(hipEventRecord(e0, bt.stream));
    for (int r = 0; r < reps; ++r) enqueue_step(bt, 0);
    DHIT_HIP(hipEventRecord(e1, bt.stream));
    DHIT_HIP(hipEventSynchronize(e1));
    DHIT_HIP(hipEventElapsedTime(&ms, e0, e1));
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

// Chooses the persistent grid size and, for DUGKS, the column-tile width
// and the z-chunk of a work item, by timing each combination on the batch.
void autotune(dhit_batch &bt) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  read_tune_file();
  const std::string key = tune_key(bt);
  auto it = g_tune_cache.find(key);
  if (it != g_tune_cache.end()) {
    bt.grid = it->second.grid;
    bt.tile = it->second.tile;
    build_table(bt, it->second.chunk);
    bt.tuned = true;
    return;
  }
  const int cus = cu_count();
  // grid sizes: persistent grids of a few blocks per compute unit, and (as
  // INT_MAX, capped at the batch's work items) one block per work item,
  // whose blocks the hardware dispatcher hands out as compute units free up
  std::vector<int> grids, chunks, tiles;
  if (bt.method == DHIT_DUGKS) {
    grids = {cus, 2 * cus, 4 * cus, INT_MAX};  // (the resident grid of each tile width is among them)
    chunks = {0, 8, 16, 32};  // 0: each box's untuned chunk (fused_default_chunk)
    tiles = {32, 16};
  } else {
    grids = {2 * cus, 4 * cus, 8 * cus, 16 * cus, 32 * cus, INT_MAX};
    chunks = {0};
    tiles = {bt.tile};
  }
  float best = 1e30f;
  TuneChoice choice{grids[0], chunks[0], tiles[0]};
  for (int w : tiles) {
    bt.tile = w;
    for (int c : chunks) {
      build_table(bt, c);
      int last = 0;
      for (int g : grids) {
        bt.grid = std::min(g, std::max(1, bt.total_items));
        if (bt.grid == last) continue;  // capped to the same grid as the previous candidate
        last = bt.grid;
        // the better of two trials: one trial of a few steps is noisy
        const float ms = std::min(time_trial(bt, 5), time_trial(bt, 5));
        if (ms < best) {
          best = ms;
          choice = {bt.grid, c, w};
        }
      }
    }
  }
  bt.grid = choice.grid;
  bt.tile = choice.tile;
  build_table(bt, choice.chunk);
  g_tune_cache[key] = choice;
  write_tune_entry(key, choice);
  bt.tuned = true;
}

void destroy(dhit_batch *bt) {
  if (!bt) return;
  if (bt->stream) (void)hipStreamSynchronize(bt->stream);
  drop_graph(*bt);
  free_stage(*bt);
  if (bt->d_boxes) (void)hipFree(bt->d_boxes);
  if (bt->d_partials) (void)hipFree(bt->d_partials);
  if (bt->d_trial) (void)hipFree(bt->d_trial);
  delete bt;
}

void check_boxes(dhit_box **boxes, int32_t nbox) {
  if (!boxes || nbox <= 0) throw dhit::Error(DHIT_EINVAL, "bad batch arguments");
  for (int32_t i = 0; i < nbox; ++i) {
    if (!boxes[i]) throw dhit::Error(DHIT_EINVAL, "null box in batch");
    if (boxes[i]->p.method != boxes[0]->p.method || boxes[i]->p.precision != boxes[0]->p.precision)
      throw dhit::Error(DHIT_EINVAL, "all boxes of a batch must share method and precision");
    if (boxes[i]->p.method == DHIT_DUGKS && boxes[i]->p.variant != DHIT_VARIANT_DEFAULT)
      throw dhit::Error(DHIT_EINVAL, "batched DUGKS uses the fused kernel (variant default)");
    if (boxes[i]->mesh) throw dhit::Error(DHIT_EINVAL, "boxes with a stretched mesh cannot be batched");
    for (int32_t j = 0; j < i; ++j)
      if (boxes[j] == boxes[i]) throw dhit::Error(DHIT_EINVAL, "a box appears twice in a batch");
  }
}

// Later work on the batch's stream waits, on the device, for the work
// already queued on the boxes' own streams (the host does not wait).
void wait_for_boxes(dhit_batch &bt) {
  std::vector<hipStream_t> seen;
  for (auto *b : bt.boxes) {
    if (b->stream == bt.stream || std::find(seen.begin(), seen.end(), b->stream) != seen.end()) continue;
    seen.push_back(b->stream);
    hipEvent_t e;
    DHIT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipError_t r = hipEventRecord(e, b->stream);
    if (r == hipSuccess) r = hipStreamWaitEvent(bt.stream, e, 0);
    (void)hipEventDestroy(e);
    DHIT_HIP(r);
  }
}

// The batch's box set and what depends on it (largest side, LBE cells per
// thread; the device tables grow as needed and never shrink).  The batch's
// stream is ordered after the work queued on the boxes' streams.
void set_boxes(dhit_batch &bt, dhit_box **boxes, int32_t nbox) {
  bt.boxes.assign(boxes, boxes + nbox);
  bt.max_n = 0;
  for (int32_t i = 0; i < nbox; ++i) bt.max_n = std::max(bt.max_n, boxes[i]->n);
  bt.cells_per_thread = dhit::lbe_cells_per_thread(boxes[0]->n, bt.precision);
  for (int32_t i = 1; i < nbox; ++i)
    if (dhit::lbe_cells_per_thread(boxes[i]->n, bt.precision) != bt.cells_per_thread) bt.cells_per_thread = 1;
  if ((size_t)nbox > bt.cap_boxes) {
    if (bt.d_boxes || bt.d_trial) DHIT_HIP(hipStreamSynchronize(bt.stream));
    if (bt.d_boxes) (void)hipFree(bt.d_boxes);
    if (bt.d_trial) (void)hipFree(bt.d_trial);
    bt.d_boxes = nullptr;
    bt.d_trial = nullptr;
    bt.cap_boxes = 0;
    const size_t cap = std::max((size_t)nbox, (size_t)16);
    if (hipMalloc(&bt.d_boxes, cap * sizeof(dhit::BatchBox)) != hipSuccess ||
        hipMalloc(&bt.d_trial, cap * dhit::kNumSums * sizeof(double)) != hipSuccess)
      throw dhit::Error(DHIT_ENOMEM, "cannot allocate batch tables");
    bt.cap_boxes = cap;
  }
  // pending work of every box comes before the batch stream uses it
  wait_for_boxes(bt);
}

dhit_batch *make_batch(dhit_box **boxes, int32_t nbox, int32_t tune) {
  check_boxes(boxes, nbox);
  dhit_batch *bt = new dhit_batch();
  try {
    bt->method = boxes[0]->p.method;
    bt->precision = boxes[0]->p.precision;
    bt->stream = boxes[0]->stream;
    bt->tile = dhit::fused_tile_width_of(bt->precision);
    set_boxes(*bt, boxes, nbox);
    if (tune) {
      autotune(*bt);
    } else {
      build_table(*bt, 0);
      bt->grid = default_grid(*bt);
    }
  } catch (...) {
    destroy(bt);
    throw;
  }
  return bt;
}

// A new box set for an existing batch (same method and precision): the
// tables are rebuilt in the batch's device memory, the tuned tile width
// and z-chunk are kept, and the captured graph is dropped (captured again
// on the next run of eight steps or more).
void update_batch(dhit_batch &bt, dhit_box **boxes, int32_t nbox) {
  check_boxes(boxes, nbox);
  if (boxes[0]->p.method != bt.method || boxes[0]->p.precision != bt.precision)
    throw dhit::Error(DHIT_EINVAL, "batch_update: the boxes must have the batch's method and precision");
  drop_graph(bt);
  set_boxes(bt, boxes, nbox);
  build_table(bt, bt.chunk);
  bt.grid = bt.tuned ? std::min(std::max(bt.grid, 1), std::max(1, bt.total_items))
                     : default_grid(bt);
}

void run_steps(dhit_batch &bt, int32_t nsteps, bool use_graph) {
  if (nsteps < 0) throw dhit::Error(DHIT_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return;
  wait_for_boxes(bt);
  upload_table(bt);
  int32_t left = nsteps;
  if (use_graph && left >= kGraphSteps) {
    if (!bt.exec) capture_graph(bt);
    while (left >= kGraphSteps) {
      DHIT_HIP(hipGraphLaunch(bt.exec, bt.stream));
      left -= kGraphSteps;
    }
  }
  for (; left > 0; --left) enqueue_step(bt, 1);
  for (auto *b : bt.boxes) {
    b->steps += nsteps;
    if (nsteps & 1) b->cur ^= 1;
  }
  // later work queued on another box's own stream must wait for the batch
  hipEvent_t done;
  DHIT_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
  DHIT_HIP(hipEventRecord(done, bt.stream));
  for (auto *b : bt.boxes)
    if (b->stream != bt.stream) DHIT_HIP(hipStreamWaitEvent(b->stream, done, 0));
  (void)hipEventDestroy(done);
}

template <class F>
int32_t guarded_batch(F &&f) {
  try {
    dhit::set_last_error("");
    (void)hipGetLastError();  // clear a pending error of a call outside this library
    return f();
  } catch (const dhit::Error &e) {
    dhit::set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc &) {
    dhit::set_last_error("host allocation failed");
    return DHIT_ENOMEM;
  } catch (const std::exception &e) {
    dhit::set_last_error(e.what());
    return DHIT_EINVAL;
  }
}

}  // namespace

extern "C" {

int32_t create_batch(dhit_box **boxes, int32_t nbox, int32_t autotune_flag, dhit_batch **out) {
  return guarded_batch([&]() -> int32_t {
    if (!out) throw dhit::Error(DHIT_EINVAL, "null output");
    *out = make_batch(boxes, nbox, autotune_flag);
    return DHIT_OK;
  });
}

int32_t batch_update(dhit_batch *bt, dhit_box **boxes, int32_t nbox) {
  return guarded_batch([&]() -> int32_t {
    if (!bt) throw dhit::Error(DHIT_EINVAL, "null batch");
    update_batch(*bt, boxes, nbox);
    return DHIT_OK;
  });
}

int32_t batch_set_stream(dhit_batch *bt, void *stream) {
  return guarded_batch([&]() -> int32_t {
    if (!bt) throw dhit::Error(DHIT_EINVAL, "null batch");
    DHIT_HIP(hipStreamSynchronize(bt->stream));
    bt->stream = static_cast<hipStream_t>(stream);
    return DHIT_OK;
  });
}

int32_t batch_step(dhit_batch *bt, int32_t nsteps) {
  return guarded_batch([&]() -> int32_t {
    if (!bt) throw dhit::Error(DHIT_EINVAL, "null batch");
    for (const dhit_box *b : bt->boxes)  // set_mesh after the batch was built
      if (b->mesh) throw dhit::Error(DHIT_EINVAL, "a box of the batch has a stretched mesh");
    run_steps(*bt, nsteps, true);
    return DHIT_OK;
  });
}

int32_t batch_info(const dhit_batch *bt, int64_t *info) {
  return guarded_batch([&]() -> int32_t {
    if (!bt || !info) throw dhit::Error(DHIT_EINVAL, "null argument");
    info[0] = bt->grid;
    info[1] = bt->chunk;
    info[2] = bt->total_items;
    info[3] = kGraphSteps;
    info[4] = bt->tuned ? 1 : 0;
    info[5] = bt->method == DHIT_DUGKS ? bt->tile : 0;
    return DHIT_OK;
  });
}

int32_t destroy_batch(dhit_batch *bt) {
  destroy(bt);
  return DHIT_OK;
}

int32_t step_batch(dhit_box **boxes, int32_t nbox, int32_t nsteps) {
  return guarded_batch([&]() -> int32_t {
    dhit_batch *bt = make_batch(boxes, nbox, 0);
    try {
      run_steps(*bt, nsteps, false);
    } catch (...) {
      destroy(bt);
      throw;
    }
    destroy(bt);
    return DHIT_OK;
  });
}

}  // extern "C"
