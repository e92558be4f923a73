// C ABI of batched runs over many handles and of the POTRF autotuner
// (declared in include/spi.h).
//
// Energy bands share the pattern of H and differ in W and y (Sect. 2.2.3);
// the paper analyses them one after the other (Sect. 5, Sect. 6).  A batch enqueues
// the whole pipeline of every system (factorisation, right-hand side, solve,
// variances) on each handle's own stream before synchronising once, so
// systems run concurrently and fill the gaps of each other's dependency
// chains (the pivot-block steps between the root sweeps' bulk updates, the
// small fronts of uneven sub-problems).  With graphs, each handle's pipeline is captured into a HIP graph
// on first use and replayed afterwards: one launch per system instead of
// about a thousand.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "spi_internal.h"

using namespace spi;

namespace {

struct Captured {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* key[4] = {nullptr, nullptr, nullptr, nullptr};
  int precision = -1;  // the handle's precision when captured
};

void drop(Captured& c) {
  if (c.exec) (void)hipGraphExecDestroy(c.exec);
  if (c.graph) (void)hipGraphDestroy(c.graph);
  c = Captured{};
}

// The whole pipeline of one system, stream-ordered, no host synchronisation.
int enqueue_system(Handle& h, const double* y, double* b, double* x, double* d) {
  int st = factor_enqueue(h);
  if (st != SPI_OK) return st;
  SPI_CK(launch_rhs(h, y, b), "rhs");
  if ((st = solve_enqueue(h, b, x, h.opts.refine_steps)) != SPI_OK) return st;
  if (d && (st = diag_enqueue(h, d)) != SPI_OK) return st;
  return SPI_OK;
}

}  // namespace

struct spi_batch {
  std::vector<spi_handle*> hs;
  std::vector<Captured> graphs;
  bool use_graphs = false;
};

extern "C" {

int spi_batch_create(spi_batch** out, spi_handle* const* hs, int32_t k,
                     int32_t use_graphs) {
  if (!out || !hs || k < 1) return SPI_E_ARG;
  *out = nullptr;
  for (int32_t i = 0; i < k; ++i) {
    if (!hs[i]) return SPI_E_ARG;
    if (use_graphs && !hs[i]->h.stream) return SPI_E_ARG;  // NULL stream: no capture
    for (int32_t j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return SPI_E_ARG;
  }
  spi_batch* b = new (std::nothrow) spi_batch();
  if (!b) return SPI_E_OOM;
  b->hs.assign(hs, hs + k);
  b->graphs.resize(k);
  b->use_graphs = use_graphs != 0;
  *out = b;
  return SPI_OK;
}

int spi_batch_run(spi_batch* B, const double* const* y, double* const* rhs,
                  double* const* x, double* const* d, int32_t* status) {
  if (!B || !y || !rhs || !x) return SPI_E_ARG;
  const int k = (int)B->hs.size();
  int first_bad = SPI_OK;
  auto note = [&](int i, int st) {
    if (status) status[i] = st;
    if (st != SPI_OK && first_bad == SPI_OK) first_bad = st;
  };
  std::vector<bool> launched(k, false);
  for (int i = 0; i < k; ++i) {
    Handle& h = B->hs[i]->h;
    if (!y[i] || !rhs[i] || !x[i]) {
      note(i, fail(h, SPI_E_ARG, hipSuccess, "null pointer in batch"));
      continue;
    }
    if (!h.have_values) {
      note(i, fail(h, SPI_E_STATE, hipSuccess, "batch run before spi_set_values"));
      continue;
    }
    const int timing = h.opts.timing;
    h.opts.timing = 0;  // no host-side event bookkeeping inside a batch
    int st = SPI_OK;
    hipError_t he = hipSuccess;
    if (!B->use_graphs) {
      st = enqueue_system(h, y[i], rhs[i], x[i], d ? d[i] : nullptr);
    } else {
      Captured& c = B->graphs[i];
      const void* key[4] = {y[i], rhs[i], x[i], d ? d[i] : nullptr};
      if (c.exec && (!std::equal(key, key + 4, c.key) || c.precision != h.opts.precision))
        drop(c);
      if (!c.exec) {
        // everything that allocates or creates must exist before capture
        he = ensure_side_stream(h);
        if (he == hipSuccess)
          he = hipStreamBeginCapture(h.stream, hipStreamCaptureModeThreadLocal);
        if (he == hipSuccess) {
          st = enqueue_system(h, y[i], rhs[i], x[i], d ? d[i] : nullptr);
          hipGraph_t g = nullptr;
          const hipError_t he2 = hipStreamEndCapture(h.stream, &g);
          if (st == SPI_OK) he = he2;
          if (he == hipSuccess && st == SPI_OK) {
            he = hipGraphInstantiate(&c.exec, g, nullptr, nullptr, 0);
            c.graph = g;
            std::copy(key, key + 4, c.key);
            c.precision = h.opts.precision;
          } else if (g) {
            (void)hipGraphDestroy(g);
          }
        }
      }
      if (he == hipSuccess && st == SPI_OK) {
        // state the captured pipeline leaves behind on the handle
        h.have_inv = h.an.n_pad > 0 && h.opts.root_inverse;
        he = hipGraphLaunch(c.exec, h.stream);
      }
    }
    h.opts.timing = timing;
    if (he != hipSuccess) st = fail(h, SPI_E_HIP, he, "batch graph");
    if (st != SPI_OK) {
      note(i, st);
      continue;
    }
    launched[i] = true;
  }
  // one synchronisation per stream; the input and pivot flags, then the
  // sizes of the last two refinement corrections, decide each status
  auto finish = [&](Handle& h) -> int {
    uint64_t f[2] = {0, 0};
    double nv[4] = {0, 0, 0, 0};
    hipError_t he = hipMemcpyAsync(f, h.flag, sizeof(f), hipMemcpyDeviceToHost,
                                   h.stream);
    if (he == hipSuccess)
      he = hipMemcpyAsync(nv, h.vnorm, sizeof(nv), hipMemcpyDeviceToHost, h.stream);
    if (he == hipSuccess) he = hipStreamSynchronize(h.stream);
    if (he != hipSuccess) return fail(h, SPI_E_HIP, he, "batch");
    int st = factor_finish(h, f);
    const int steps = h.opts.refine_steps;
    h.refine_done = steps;
    h.last_norm_pair = steps > 0 ? (steps - 1) & 1 : 0;
    if (st == SPI_OK && h.opts.refine_tol > 0.0) {
      // step s wrote pair s & 1: the last step's pair, then the one before
      auto rel = [&](int s) {
        const double* p = nv + 2 * (s & 1);
        return p[1] > 0.0 ? p[0] / p[1] : 0.0;
      };
      const double cur = steps > 0 ? rel(steps - 1) : 1.0;
      const double prev = steps > 1 ? rel(steps - 2) : 0.0;
      if (!refine_converged(cur, prev, h.opts.refine_tol))
        st = fail(h, SPI_E_NOCONV, hipSuccess,
                  "iterative refinement did not reach refine_tol in the batch");
    }
    return st;
  };
  for (int i = 0; i < k; ++i) {
    if (!launched[i]) continue;
    Handle& h = B->hs[i]->h;
    int st = finish(h);
    if ((st == SPI_E_NOT_SPD || st == SPI_E_NOCONV) && h.opts.fp64_fallback &&
        h.opts.precision == SPI_MIXED) {
      // opts.fp64_fallback: this system alone again, every stage in
      // binary64, outside any graph (its graph is recaptured at the next
      // run); the handle stays in binary64 until new values arrive
      h.opts.precision = SPI_FP64;
      ++h.fp64_fallbacks;
      drop(B->graphs[i]);
      const int timing = h.opts.timing;
      h.opts.timing = 0;
      st = enqueue_system(h, y[i], rhs[i], x[i], d ? d[i] : nullptr);
      h.opts.timing = timing;
      if (st == SPI_OK) st = finish(h);
    }
    note(i, st);
  }
  return first_bad;
}

void spi_batch_destroy(spi_batch* B) {
  if (!B) return;
  for (auto& c : B->graphs) drop(c);
  delete B;
}

int spi_autotune(spi_handle* H, int32_t* chosen) {
  if (!H) return SPI_E_ARG;
  Handle& h = H->h;
  if (!h.have_values)
    return fail(h, SPI_E_STATE, hipSuccess, "spi_autotune before spi_set_values");
  const int cand[4] = {128, 256, 512, 1024};
  // the bulk update's tile: 64 x 64 gives small roots four times the
  // workgroups of 128 x 128 (tried only below order 8192, where that matters)
  const int tiles[2] = {128, 64};
  const int n_tiles_tried = (h.opts.root_inverse && h.an.n_pad <= 8192) ? 2 : 1;
  double best = 1e300;
  int best_b = h.potrf_block, best_t = h.bulk_tile;
  const int timing = h.opts.timing;
  h.opts.timing = 0;
  for (int c : cand)
  for (int ti = 0; ti < n_tiles_tried; ++ti) {
    if ((h.an.n_pad > 0 && c > h.an.n_pad) || c > std::max(512, h.band_nb)) continue;
    // the Cholesky route caps binary32 sums by its outer block
    if (h.opts.precision == SPI_MIXED && !h.opts.root_inverse && c > 256) continue;
    h.potrf_block = c;
    h.bulk_tile = tiles[ti];
    double t_min = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
      SPI_CK(hipStreamSynchronize(h.stream), "autotune");
      const auto t0 = std::chrono::steady_clock::now();
      const int st = spi_factor(H);
      if (st != SPI_OK) {
        h.opts.timing = timing;
        return st;
      }
      const double ms = std::chrono::duration<double, std::milli>(
                            std::chrono::steady_clock::now() - t0).count();
      t_min = std::min(t_min, ms);
    }
    if (t_min < best) {
      best = t_min;
      best_b = c;
      best_t = tiles[ti];
    }
  }
  h.potrf_block = best_b;
  h.bulk_tile = best_t;
  h.opts.timing = timing;
  if (chosen) *chosen = best_b;
  return spi_factor(H);  // leave a factor made with the chosen block
}

int spi_get_potrf_block(const spi_handle* H) { return H ? H->h.potrf_block : -1; }

int spi_get_bulk_tile(const spi_handle* H) { return H ? H->h.bulk_tile : -1; }

int spi_set_bulk_tile(spi_handle* H, int32_t tile) {
  if (!H || (tile != 64 && tile != 128)) return SPI_E_ARG;
  H->h.bulk_tile = tile;
  return SPI_OK;
}

int spi_set_potrf_block(spi_handle* H, int32_t block) {
  if (!H || (block != 128 && block != 256 && block != 512 &&
             !(block == 1024 && H->h.band_nb >= 1024)))
    return SPI_E_ARG;
  H->h.potrf_block = block;
  return SPI_OK;
}

}  // extern "C"
