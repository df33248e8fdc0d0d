// Tuning table of the batched kernels, written by tune_batched.py from its
// measurements on the multi-modular workload (4096 matrices, m, n ~ U[16, 512]):
// workgroups per CU of each width class's persistent kernel (n <= 128,
// <= 256, <= 512), and whether the three classes run concurrently.
// Fastest: 6.859 ms per batch.
#pragma once
namespace cup {
constexpr int kTuneWgPerCu[3] = {3, 3, 2};
constexpr int kTuneConcurrent = 1;
}  // namespace cup
