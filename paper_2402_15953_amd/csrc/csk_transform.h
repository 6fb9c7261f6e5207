// Transform launchers (fp64 FFT and NTT) and the per-prime constants they use.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "csk_internal.h"

namespace csk {

// Geometry of one transform pass: each block transforms 2^log2C interleaved transforms
// of length 2^log2L whose element n of column c sits at
// block_base + c * col_stride + n * elem_stride, block_base = blockIdx.x * block_stride.
struct PassGeom {
    int32_t log2m;
    int32_t log2L;
    int32_t log2C;
    int32_t blocks;
    int64_t elem_stride;
    int64_t col_stride;
    int64_t block_stride;
    int32_t twiddle;   // multiply output n of column c by w_m^(n * (blockIdx.x * C + c))
    int32_t scale;     // multiply by m^-1 (inverse NTT, last pass)
};

// Constants of one NTT prime, as the device reads them.
struct PrimeDev {
    uint32_t p;
    uint32_t pinv_neg;   // -p^-1 mod 2^32
    uint32_t r2;         // 2^64 mod p
    uint32_t r3;         // 2^96 mod p
    uint32_t neg2_64;    // Montgomery form of -2^64 mod p
    uint32_t one;        // Montgomery form of 1 (2^32 mod p)
    uint32_t minv[kMaxLog2N + 1];  // Montgomery form of 2^-L mod p
};

// Row length 2^S of the two-pass transforms (lengths above 4096), which is also their
// tile.  Default: the smallest S >= 10 that leaves the column pass at least 8
// interleaved columns (128 contiguous bytes of fp64 complex per row read): 1024 for
// 2^13..2^17, 2048 for 2^18..2^19, 4096 for 2^20..2^21.  The autotuner may pick another
// S with split_ok(); every transform of one estimate uses the same S for one length.
__host__ __device__ inline int default_split_bits(int log2m) { return (log2m + 4) / 2 > 10 ? (log2m + 4) / 2 : 10; }
// The split an estimate uses for length 2^log2m on `device` (tuned, else the default).
int split_for(int device, int log2m);

// Position of frequency f in the output of the forward transform of length 2^log2m
// with row length 2^S.
__host__ __device__ inline uint32_t freq_pos(uint32_t f, int log2m, int S)
{
    if (log2m <= 12) return f;
    const uint32_t n1 = 1u << (log2m - S);
    return ((f & (n1 - 1)) << S) | (f >> (log2m - S));
}
// Frequency held at position pos of the forward transform's output.
__host__ __device__ inline uint32_t pos_freq(uint32_t pos, int log2m, int S)
{
    if (log2m <= 12) return pos;
    return (pos >> S) | ((pos & ((1u << S) - 1)) << (log2m - S));
}

// Forward fp64 FFTs of n_vec complex vectors re[v] + i im[v] (device pointer tables of
// int64 sketches; im[v] may be null) into buf [n_vec][m].
cs_status fft_f64_forward(const int64_t *const *re, const int64_t *const *im, int n_vec, double2 *buf, int log2m,
                          int S, const double2 *tw, int log2T, hipStream_t s);

// ptrs != null: vector (prime i, j) is loaded from sketch ptrs[j] (device pointer table);
// ptrs == null: transform buf in place.  rep_of / kp (both device, may be null): vector j
// serves repetition rep_of[j], which needs kp[rep_of[j]] primes; the blocks of primes
// beyond that return without touching buf.
cs_status ntt_forward(const int64_t *const *ptrs, int vec_per_prime, int n_primes, uint32_t *buf, int log2m, int S,
                      const PrimeDev *primes, const uint32_t *roots, int log2T, hipStream_t s,
                      const int32_t *rep_of = nullptr, const int32_t *kp = nullptr);
cs_status ntt_inverse(int vec_per_prime, int n_primes, uint32_t *buf, int log2m, int S, const PrimeDev *primes,
                      const uint32_t *roots, int log2T, hipStream_t s);

}  // namespace csk
