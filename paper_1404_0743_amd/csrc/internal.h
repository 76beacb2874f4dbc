// internal.h -- helpers shared by the C ABI implementation files.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/pentago.h"
#include "kernels.h"

namespace pg {

int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *where);
int device_tables(DevTables *out);
// The current device's tables if device_tables() has uploaded them already
// (0), else nonzero; never allocates.
int device_tables_ready(DevTables *out);

bool section_valid(const pentago_section &s);
int section_mover(const pentago_section &s);
int section_stones(const pentago_section &s);
pentago_section child_of(const pentago_section &s, int j);
void section_shape_of(const pentago_section &s, int m[4]);
uint64_t host_block_offset(const int *m, const int *idx);
int make_job(const pentago_section &s, const pentago_superinfo *const child[4],
             pentago_superinfo *out, SweepJob *J, int force_d, int forceG, int force_threads = 0,
             int force_order = -1);
size_t prep_bytes(const SweepJob &J, int j);
int run_job(SweepJob &J, const DevTables &T, hipStream_t st);
// With pentago_set_validate(1): EINVAL unless every child table J reads has
// each entry's win set inside its not-lose set (synchronises st); else 0.
int validate_children(const SweepJob &J, hipStream_t st);
// Tile shape of a section geometry chosen by the autotuner (0 lines: none).
struct TileShape {
    int lines;
    int threads;
    int order;
};
TileShape tuned_tile_shape(const SweepJob &J);
void remember_tile_shape(const SweepJob &J, TileShape t);
pentago_section section_image(const pentago_section &s, int sym);
void section_standardize(const pentago_section &s, pentago_section *rep, int *sym);
void set_child_syms(const pentago_section &s, const pentago_superinfo *const rep[4], SweepJob *J);
int make_sym_job(const pentago_section &s, const pentago_superinfo *table, int sym,
                 pentago_superinfo *out, SymJob *J);
// Keep the device's stream-ordered allocations (hipMallocAsync) pooled.
void keep_pool(int dev);
int board_empties(uint64_t packed);
size_t deep_scratch_bytes(int e, bool half = false);
int eval_deep_enqueue(uint64_t packed, uint4 *out, hipStream_t st, int parity = -1);
int eval_grid(int *grid);
size_t eval_scratch_bytes(size_t n, int grid, bool deep);
int eval_enqueue(const uint64_t *boards, size_t n, uint4 *out, int *status, bool deep, int grid,
                 hipStream_t st);
int eval_enqueue_class(const uint64_t *boards, size_t n, uint4 *out, int cls, bool deep, int grid,
                       hipStream_t st);

}  // namespace pg
