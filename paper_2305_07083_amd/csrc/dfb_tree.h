// Per-tile dependency-tree bookkeeping (Sec. 3.1.1; the AlphaBlend tile
// operation of Listing 4 keeps the same three quantities: the generation
// being completed, how many of its tiles are still missing, and the children
// its tiles declared for the next one).  Host code, no GPU.
#pragma once

#include <cstdint>
#include <vector>

namespace dfb {

constexpr int32_t kMaxGeneration = 65535;

class TileTree {
 public:
  enum State : int32_t { kWaiting = 0, kComplete = 1, kError = -1 };

  void reset() {
    gen_ = 0;
    expected_ = 1;  // generation 0 is the single background tile
    state_ = kWaiting;
    got_.assign(1, 0);
    children_.assign(1, 0);
  }

  // One arrival of generation g declaring c children (0 <= g <= kMaxGeneration,
  // c >= 0, checked by the caller).  Returns false when it puts the tree in
  // error; completed is set when this arrival completes the tree.
  bool add(int32_t g, int32_t c, bool& completed) {
    completed = false;
    if (state_ != kWaiting) {  // nothing may follow a complete tree
      state_ = kError;
      return false;
    }
    if (g < gen_) {  // that generation is already done: one tile too many
      state_ = kError;
      return false;
    }
    grow(g);
    got_[g] += 1;
    children_[g] += c;
    if (g > gen_) return true;  // counted until its parents are done
    return advance(completed);
  }

  int32_t state() const { return state_; }
  int32_t generation() const { return gen_; }
  int64_t missing() const {
    if (state_ == kComplete) return 0;
    const int64_t m = expected_ - got_[gen_];
    return m > 0 ? m : 0;
  }
  int32_t count(int32_t g) const { return g < static_cast<int32_t>(got_.size()) ? got_[g] : 0; }

 private:
  void grow(int32_t g) {
    if (g >= static_cast<int32_t>(got_.size())) {
      got_.resize(g + 1, 0);
      children_.resize(g + 1, 0);
    }
  }

  // Move past every generation that now holds exactly what it expects.
  bool advance(bool& completed) {
    for (;;) {
      if (got_[gen_] > expected_) {
        state_ = kError;
        return false;
      }
      if (got_[gen_] < expected_) return true;
      const int64_t next = children_[gen_];
      if (next == 0) {
        // the tree ends here: tiles counted in later generations are extra
        for (size_t h = gen_ + 1; h < got_.size(); ++h)
          if (got_[h] > 0) {
            state_ = kError;
            return false;
          }
        state_ = kComplete;
        completed = true;
        return true;
      }
      gen_ += 1;
      grow(gen_);
      expected_ = next;
    }
  }

  int32_t gen_ = 0;
  int64_t expected_ = 1;
  int32_t state_ = kWaiting;
  std::vector<int32_t> got_{0};
  std::vector<int64_t> children_{0};
};

}  // namespace dfb
