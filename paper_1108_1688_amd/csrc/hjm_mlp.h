// Sizes and parameter layout of the surrogate MLP (internal to libhjm; the C
// ABI is in include/hjm.h).
#pragma once

#include <stdint.h>

namespace hjm_nn {

constexpr int kIn = 8;        // model inputs
constexpr int kInPad = 32;    // inputs padded to one MFMA k-block
constexpr int kHidden = 256;  // width of the four hidden layers
constexpr int kChunk = 256;   // samples per partial weight-gradient block

// flat FP32 parameter vector: W1 (256 x 8), b1, W2 (256 x 256), b2, W3, b3,
// W4, b4, w5 (256), b5 (1); weights row-major (output x input)
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + (int64_t)kHidden * kIn;
constexpr int64_t kOffW2 = kOffB1 + kHidden;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kHidden * kHidden;
constexpr int64_t kOffW3 = kOffB2 + kHidden;
constexpr int64_t kOffB3 = kOffW3 + (int64_t)kHidden * kHidden;
constexpr int64_t kOffW4 = kOffB3 + kHidden;
constexpr int64_t kOffB4 = kOffW4 + (int64_t)kHidden * kHidden;
constexpr int64_t kOffW5 = kOffB4 + kHidden;
constexpr int64_t kOffB5 = kOffW5 + kHidden;
constexpr int64_t kParams = kOffB5 + 1;  // 199,937

}  // namespace hjm_nn

namespace hjm {
// Record msg as the calling thread's last error (read by hjm_last_error) and
// return code.
int32_t report_error(int32_t code, const char* msg);
}  // namespace hjm
