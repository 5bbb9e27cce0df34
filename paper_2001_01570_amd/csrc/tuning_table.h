// Face tile shapes per direction by grid size, written by the autotuner
// (python -m paper_2001_01570_amd.autotune) from its timings on the GPU;
// the library applies the entry nearest in cell count (log scale) when a 2D
// context is created.  Shapes: 0 = 8x16, 1 = 4x32, 2 = 2x64.
// Sources digest the timings were taken on: 458b7ddb29bfa86f
#pragma once
namespace cgks {
struct TuneEntry { int nx, ny, x, y; };
// Batch: face tile shapes of the two-point FP64 slots and the steps per graph
// replay that gave the serving mix its highest rate.
struct BatchTune { int x, y, steps; };
constexpr BatchTune kBatchTune = {1, 1, 5};
constexpr TuneEntry kTuneTable[] = {
    {64, 64, 2, 0},
    {128, 128, 0, 1},
    {256, 256, 1, 2},
    {512, 512, 1, 1},
    {1024, 1024, 1, 1},
    {2048, 2048, 0, 2},
};
}  // namespace cgks
