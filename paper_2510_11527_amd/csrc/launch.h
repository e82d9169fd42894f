// launch.h -- kernel launch entry points used by the host runtime.
#pragma once
#include "af_internal.h"

namespace af4 {

struct VariantInfo {
    int tile[3];
    int nt;
    const char *name;
};

int stage_num_variants(int dim);
VariantInfo stage_variant(int dim, int v);

// Properties of a context that specialised stage kernels rely on.
enum : unsigned {
    kCapQF = 1,   // every flux of every instance is c1 u + c2 u^2 (linear or Burgers)
    kCapPP = 2,   // every potential is c1 u + c2 u^2 + c3 u^3 without clamps or signs
    kCapI32 = 4,  // the DoF block of every instance holds fewer than 2^32 bytes
    kCapBQ = 8,   // every flux is c2 u^2 (no linear part)
    kCapOpen = 16,  // some instance has non-periodic ends (only the generic kernel fills ghosts)
    kCapBLF = 32,   // every flux is Buckley-Leverett, with or without gravity
};

// One stage launch over nblocks (instance, tile) work items.
// params points to a StageParams<float> or StageParams<double>.
// Returns hipErrorInvalidValue for a combination that is not built.
hipError_t stage_launch(int dim, int prec, bool lim, bool si, unsigned caps, int variant, int nblocks, const void *params,
                        hipStream_t s);
// true if the (dim, prec, lim, si, variant) kernel is built (LDS fits) and
// applies to a context with the given capabilities
bool stage_supported(int dim, int prec, bool lim, bool si, unsigned caps, int variant);
bool stage_supported_d1(int prec, bool lim, bool si, int variant);
bool stage_supported_d2(int prec, bool lim, bool si, unsigned caps, int variant);
bool stage_supported_d3(int prec, bool lim, bool si, unsigned caps, int variant);
hipError_t stage_launch_d1(int prec, bool lim, bool si, unsigned caps, int variant, int nblocks, const void *params, hipStream_t s);
hipError_t stage_launch_d2(int prec, bool lim, bool si, unsigned caps, int variant, int nblocks, const void *params,
                           hipStream_t s);
hipError_t stage_launch_d3(int prec, bool lim, bool si, unsigned caps, int variant, int nblocks, const void *params, hipStream_t s);

// FP64 max over faces of alpha_l/dx_l + kappa_max/dx_l^2 of the averages of
// U, one slot per chunk (the bits of the chunk's max), plus the divergence
// check.
constexpr int kWaveChunk = 1024;  // cells per wave-speed block (about)
constexpr int kWaveThreads = 256;  // threads per wave-speed block (four waves)
// Cells of wave-speed chunk k of an instance whose rows hold n0 cells
// (nrows rows): whole rows [r0, r1) when a row holds at most kWaveChunk
// cells, else one row r0 split into equal column segments [i0, i1).
struct WaveChunk {
    int r0, r1, i0, i1;
};
__host__ __device__ inline int wave_chunks_per_row(int n0) { return (n0 + kWaveChunk - 1) / kWaveChunk; }
__host__ __device__ inline long long wave_chunk_count(int n0, long long nrows)
{
    if (n0 > kWaveChunk) return nrows * wave_chunks_per_row(n0);
    const long long rpc = (kWaveChunk + n0 - 1) / n0;
    return (nrows + rpc - 1) / rpc;
}
__host__ __device__ inline WaveChunk wave_chunk(int n0, long long nrows, long long k)
{
    WaveChunk c;
    if (n0 > kWaveChunk) {
        const int spr = wave_chunks_per_row(n0), seg = (n0 + spr - 1) / spr, s = (int)(k % spr);
        c.r0 = (int)(k / spr);
        c.r1 = c.r0 + 1;
        c.i0 = s * seg;
        c.i1 = s * seg + seg < n0 ? s * seg + seg : n0;
    } else {
        const long long rpc = (kWaveChunk + n0 - 1) / n0;
        c.r0 = (int)(k * rpc);
        c.r1 = (int)(k * rpc + rpc < nrows ? k * rpc + rpc : nrows);
        c.i0 = 0;
        c.i1 = n0;
    }
    return c;
}
hipError_t wavespeed_launch(int dim, int prec, const InstDev *inst, const int2 *chunks, int nchunks, const void *U,
                            InstState *st, unsigned long long *slots, hipStream_t s);

// dt and t of every instance from the wave speeds (or the prescribed steps);
// wslots != nullptr: from the chunk slots of the wave-speed kernel
// (InstDev::cstart / ccount); mm != nullptr: from the min / max average slots
// written by the previous step's last stage (waves_per_block slot pairs per
// work item) instead (fluxes with convex |f'| only); prec: storage precision
// (the Dirichlet ghost values enter the min / max as stored); max_slots: the
// largest number of slots of one instance on the path taken (sizes the
// reduction).
hipError_t finalize_launch(int n_inst, const InstDev *inst, const StepCtl *ctl, const double *dtp, InstState *st,
                           int dim, int prec, const unsigned long long *mm, const unsigned long long *wslots,
                           int waves_per_block, long long max_slots, hipStream_t s);

// dst = src over n values.
hipError_t copy_launch(int prec, const void *src, void *dst, long long n, hipStream_t s);
// FP64 values to the storage precision (to_storage) or back, over n values
// (round to nearest; a plain copy for FP64 storage).
hipError_t convert_launch(int prec, bool to_storage, const void *src, void *dst, long long n, hipStream_t s);
// dst = src over n16 16-byte elements (the copy-bandwidth reference).
hipError_t copy16_launch(const void *src, void *dst, long long n16, hipStream_t s);

// FP64 norms of one instance: out[0..9] = sum u, sum |u|, sum u^2, max |u|,
// min avg, max avg, min pv, max pv, nonfinite count, (unused).
constexpr int kNormBlocks = 240;
hipError_t norms_launch(int prec, const void *block, long long ncell, long long kstride, int nkinds, double *partials,
                        double *out, hipStream_t s);

// Device address, on the current device, of the library's static scratch
// array of kNoallocScratchDoubles doubles (the partials and results of
// norms_launch), looked up once per device.
constexpr int kNoallocScratchDoubles = 9 * kNormBlocks + 16;
hipError_t noalloc_scratch(double **ptr);

}  // namespace af4
