// Sweep block heights (rows of the block triangular sweeps and of the inverted diagonal
// blocks) per precision class of the factors (0: FP64, 1: FP32) and order n, measured on
// AMD Radeon Graphics (gfx950) by `python -m paper_1605_08771_amd.autotune --reps 3`: for each
// order, the fastest converging height of 64, 128, 256 and 512 over whole solves of
// 3 synthetic problems of the batched workload's kind.  Orders past the last row
// use 512.
#pragma once

namespace feast {

struct SweepTuneRow {
  int prec_class;
  int n_max;
  int nbt;
};

static const SweepTuneRow kSweepTune[] = {
    {0, 319, 256}, {0, 895, 128}, {0, 1791, 256}, {0, 6144, 512},
    {1, 319, 256}, {1, 447, 128}, {1, 639, 256}, {1, 2559, 128}, {1, 3583, 64}, {1, 6144, 256},
};

}  // namespace feast
