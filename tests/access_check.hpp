// access_check.hpp -- a host-side access checker over enumerated index maps.
//
// The paper's type system rejects a program when two execution resources may
// touch the same memory place without a synchronisation between them, at
// least one of them writing (Sec. 3.3, the access environment of the
// extended borrow checker).  This is the same rule applied to concrete
// indices: a kernel's accesses are replayed on the host through the same
// views the kernel uses, each recorded with the resource that makes it,
// the group that resource synchronises with (its block) and the number of
// barriers that group has passed.  Two accesses to one address conflict when
// they come from different resources, at least one is a write, and no
// barrier orders them -- that is, they are in different groups (blocks never
// synchronise inside a kernel) or in the same group between the same two
// barriers.  Two further orders are known to it: launches on one stream
// (kernel_boundary), and atomic accesses, which the hardware orders among
// themselves.
#pragma once
#include <cstdio>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

namespace access_check {

class Checker {
 public:
  // `group`: the synchronisation group of the resource (its block);
  // `who`: the resource itself (a thread, unique over all groups).
  void read(long group, long who, const void* addr) { add(group, who, addr, false, false); }
  void write(long group, long who, const void* addr) { add(group, who, addr, true, false); }
  // An atomic access (a read-modify-write, or a flag word's store or load):
  // atomics do not conflict with each other, only with plain accesses.
  void atomic(long group, long who, const void* addr, bool write) {
    add(group, who, addr, write, true);
  }
  // Every resource of `group` passes a barrier.
  void sync(long group) { ++epoch_[group]; }
  // The kernel ends: every access so far is ordered before every later one
  // (launches on one stream run in order).
  void kernel_boundary() { ++kernel_; }

  struct Conflict {
    const void* addr;
    long who_a, who_b;
    bool both_write;
  };

  std::vector<Conflict> conflicts(size_t limit = 1u << 20) const {
    std::vector<Conflict> out;
    for (const auto& kv : log_) {
      const auto& v = kv.second;
      for (size_t i = 0; i < v.size() && out.size() < limit; ++i)
        for (size_t j = i + 1; j < v.size() && out.size() < limit; ++j) {
          const Rec &a = v[i], &b = v[j];
          if (a.who == b.who || !(a.write || b.write) || (a.atomic && b.atomic)) continue;
          const bool ordered = a.kernel != b.kernel || (a.group == b.group && a.epoch != b.epoch);
          if (!ordered) out.push_back({kv.first, a.who, b.who, a.write && b.write});
        }
    }
    return out;
  }

  size_t accesses() const { return count_; }

 private:
  struct Rec {
    long group, who;
    int epoch, kernel;
    bool write, atomic;
  };
  void add(long group, long who, const void* addr, bool write, bool atomic) {
    log_[addr].push_back({group, who, epoch_[group], kernel_, write, atomic});
    ++count_;
  }
  std::unordered_map<const void*, std::vector<Rec>> log_;
  std::map<long, int> epoch_;
  int kernel_ = 0;
  size_t count_ = 0;
};

}  // namespace access_check
