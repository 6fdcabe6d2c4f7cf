// tuning.hip -- storage of the configuration table (host code only).
#include "tuning.hpp"

#include <atomic>

namespace desc {
namespace tune {
namespace {

struct Entry {
  const char* name = nullptr;
  int count = 0;
  const char* const* names = nullptr;
  int defaults[kClasses] = {0, 0, 0, 0};
  std::atomic<int> chosen[kClasses];
  Entry() {
    for (auto& c : chosen) c.store(-1);
  }
};

Entry& entry(int op) {
  static Entry table[kNumOps];
  return table[op];
}

}  // namespace

void register_op(int op, const char* name, int count, const char* const* names,
                 const int* defaults) {
  Entry& e = entry(op);
  e.name = name;
  e.count = count;
  e.names = names;
  for (int c = 0; c < kClasses; ++c) e.defaults[c] = defaults[c];
}

int size_class(int op, int64_t size) {
  // element counts: < 2^16, < 2^20, < 2^24, larger;  M*N*K: < 2^24, < 2^30, < 2^36, larger
  const bool gemm = op == kGemmF32 || op == kGemmBf16x3 || op == kGemmFp8 || op == kGemmGrouped ||
                    op == kGemmGroupedBf16x3;
  const int base = gemm ? 24 : 16, step = gemm ? 6 : 4;
  for (int c = 0; c < kClasses - 1; ++c)
    if (size < ((int64_t)1 << (base + step * c))) return c;
  return kClasses - 1;
}

int get(int op, int cls) {
  if (op < 0 || op >= kNumOps || cls < 0 || cls >= kClasses) return 0;
  Entry& e = entry(op);
  const int c = e.chosen[cls].load(std::memory_order_relaxed);
  return c >= 0 && c < e.count ? c : e.defaults[cls];
}

int config_count(int op) { return op >= 0 && op < kNumOps ? entry(op).count : 0; }

const char* config_name(int op, int cfg) {
  if (op < 0 || op >= kNumOps) return nullptr;
  Entry& e = entry(op);
  return cfg >= 0 && cfg < e.count ? e.names[cfg] : nullptr;
}

const char* op_name(int op) { return op >= 0 && op < kNumOps ? entry(op).name : nullptr; }

bool set(int op, int cls, int cfg) {
  if (op < 0 || op >= kNumOps || cls < 0 || cls >= kClasses) return false;
  Entry& e = entry(op);
  if (cfg >= e.count) return false;
  e.chosen[cls].store(cfg < 0 ? -1 : cfg, std::memory_order_relaxed);
  return true;
}

}  // namespace tune
}  // namespace desc
