// Admission pass of the request server (continuous batching) and the precision
// schedule of a member's rounds: host logic with no device calls, shared by the
// runtime and by the host-only unit tests (built there with the address and
// undefined-behaviour sanitizers).
#pragma once

#include <cstddef>
#include <map>
#include <set>
#include <string>
#include <vector>

namespace icnnm {

// A queued request as the admission pass sees it.
struct AdmitView {
  std::string key;     // group: (V, kernel dims, precision)
  size_t bytes;        // the member's state and its table entries
  size_t group_bytes;  // what a new group adds: V operand copies, slot array
  int* bypassed;       // admissions past this request while it was blocked at the head
};

struct AdmitLimits {
  size_t used;       // budget bytes held now
  size_t limit;      // the budget
  int group_slots;   // members per group
  int max_bypass;    // admissions past one blocked head before strict arrival order
  int bypass_scan;   // queued requests looked at past a blocked head
};

struct AdmitResult {
  std::vector<size_t> admitted;  // queue positions, ascending
  bool head_blocked = false;     // the first queued request could not be admitted
};

// One pass over the queue in arrival order. Bytes are reserved cumulatively within the
// pass; a request that opens a new group also reserves the group's bytes; a group
// takes at most group_slots members (free_slots: free slots of the groups that exist
// now). When a request does not fit, later ones that do may pass it: up to
// bypass_scan of them are looked at, and each admission past it counts in its
// bypassed counter; once that reaches max_bypass the pass stops at it (no starvation).
inline AdmitResult admission_pass(const std::vector<AdmitView>& queue, const std::map<std::string, int>& free_slots,
                                  const AdmitLimits& lim) {
  AdmitResult out;
  size_t reserved = lim.used;
  std::map<std::string, int> slots_left;
  std::set<std::string> opened;
  const AdmitView* blocked = nullptr;
  size_t blocked_at = 0;
  int scanned = 0;
  for (size_t i = 0; i < queue.size(); ++i) {
    if (blocked && (*blocked->bypassed >= lim.max_bypass || scanned >= lim.bypass_scan)) break;
    const AdmitView& r = queue[i];
    const auto fs = free_slots.find(r.key);
    const bool exists = fs != free_slots.end() || opened.count(r.key) != 0;
    auto sl = slots_left.find(r.key);
    if (sl == slots_left.end()) sl = slots_left.emplace(r.key, fs != free_slots.end() ? fs->second : lim.group_slots).first;
    const size_t need = r.bytes + (exists ? 0 : r.group_bytes);
    if (blocked) ++scanned;
    if (sl->second > 0 && need <= lim.limit && reserved <= lim.limit - need) {
      reserved += need;
      sl->second -= 1;
      opened.insert(r.key);
      if (blocked) *blocked->bypassed += 1;
      out.admitted.push_back(i);
      continue;
    }
    if (!blocked) {
      blocked = &r;
      blocked_at = i;
    }
  }
  out.head_blocked = blocked != nullptr && blocked_at == 0;
  return out;
}

// Contraction precision of round r of a member that joined at its round 0 (initial
// forward in FP32; round r >= 1 runs iteration r): FP32 at initialisation, on the
// first iteration, every refresh_every-th and from the last one on (the refresh
// schedule of the column-norm kernel), the member's reduced precision otherwise.
// prec: 0 FP32, otherwise the reduced precision's code.
inline int round_kind(int r, int prec, int max_iter, int refresh_every) {
  if (prec == 0 || r == 0 || refresh_every <= 1 || r >= max_iter) return 0;
  return (r - 1) % refresh_every == 0 ? 0 : prec;
}

}  // namespace icnnm
