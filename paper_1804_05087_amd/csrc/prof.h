// Optional per-kernel timing with HIP events on the plan's stream.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

namespace sp {

enum KernelId {
  KID_SYNTH_Y = 0,
  KID_FFT_X_INV,
  KID_Z_PRODUCT,
  KID_FFT_X_FWD,
  KID_ANALYSIS,
  KID_SOLVE,
  KID_AXPBY,
  KID_NORM,
  KID_PACK,
  KID_UNPACK,
  KID_MULTIDOT,
  KID_MULTIAXPY,
  KID_SCALE,
  KID_SOLVE_ADJ,
  KID_ADJ_Z,
  KID_ADJ_X_FWD,
  KID_ADJ_SYNTH,
  KID_ADV,
  KID_COUNT
};

inline const char* kernel_name(int id) {
  static const char* names[KID_COUNT] = {
      "k_synth_y",      "k_fft_x_inv",   "k_z_product", "k_fft_x_fwd", "k_analysis_rhs",
      "k_stokes_solve", "k_axpby",       "k_norm_partial", "k_pack",    "k_unpack",
      "k_multidot",     "k_multiaxpy",   "k_scale",     "k_stokes_solve_adj", "k_adj_z",
      "k_adj_fft_x",    "k_adj_synth_y", "k_adv_apply"};
  return names[id];
}

struct Profiler {
  bool on = false;
  struct Pending {
    int id;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  long long count[KID_COUNT] = {0};
  double ms[KID_COUNT] = {0.0};

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
  }
  void begin(int id, hipStream_t s, hipEvent_t* out) {
    if (!on) return;
    *out = get();
    (void)hipEventRecord(*out, s);
    (void)id;
  }
  void end(int id, hipStream_t s, hipEvent_t a) {
    if (!on) return;
    hipEvent_t b = get();
    (void)hipEventRecord(b, s);
    pending.push_back({id, a, b});
  }
  // Resolves pending pairs (the caller has synchronised the stream).
  void collect() {
    for (auto& pe : pending) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, pe.a, pe.b) == hipSuccess) {
        ms[pe.id] += t;
        count[pe.id] += 1;
      }
      pool.push_back(pe.a);
      pool.push_back(pe.b);
    }
    pending.clear();
  }
  void reset() {
    for (int i = 0; i < KID_COUNT; ++i) {
      ms[i] = 0.0;
      count[i] = 0;
    }
  }
  void release() {
    collect();
    for (auto e : pool) (void)hipEventDestroy(e);
    pool.clear();
  }
};

}  // namespace sp

#define SP_PROF_BEGIN(p, id)   \
  hipEvent_t _prof_ev = nullptr; \
  (p)->prof.begin((id), (p)->stream, &_prof_ev)
#define SP_PROF_END(p, id) (p)->prof.end((id), (p)->stream, _prof_ev)
