// tuning.hpp -- the table that picks one compiled configuration per
// operation and problem-size class.
//
// Tile shapes are compile-time parameters of the kernels (the paper's sizes
// are nats in the types); each operation is instantiated for a small set of
// shapes, and this table says which one runs for a given size class.  The
// built-in defaults can be overridden at run time (desc_config_set) or from
// a file written by the offline tuner (desc_config_load).
#pragma once
#include <stdint.h>

namespace desc {
namespace tune {

enum Op : int {
  kReduceI32 = 0,
  kScanI32 = 1,
  kTranspose32 = 2,
  kCopy32 = 3,
  kGemmF32 = 4,
  kGemmBf16x3 = 5,
  kGemmFp8 = 6,
  kSegReduceI32 = 7,
  kSegScanI32 = 8,
  kGemmGrouped = 9,
  kGemmGroupedBf16x3 = 10,
  kNumOps = 11
};
constexpr int kClasses = 4;

// Size class of a problem of `size` work units (elements, or M*N*K for GEMM).
int size_class(int op, int64_t size);
// Configuration index for (op, class); always valid for the op.
int get(int op, int cls);
int config_count(int op);
const char* config_name(int op, int cfg);
const char* op_name(int op);
bool set(int op, int cls, int cfg);     // cfg < 0 restores the default
void register_op(int op, const char* name, int count, const char* const* names,
                 const int* defaults);

}  // namespace tune
}  // namespace desc
