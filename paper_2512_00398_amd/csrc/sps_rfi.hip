// sps_rfi.hip - RFI excision (Heimdall++, Section II-B, "RFI Mitigation").
// Narrowband: channels whose lower MAD over the chunk exceeds the median of
// the channels' MADs by k MADs of those MADs are replaced by their median
// (exact byte order statistics from 256-bin histograms).
// Broadband (zero-DM): interference present in every channel at once is
// undispersed; each time sample's level across the band,
// z_t = floor((2 * sum_f I[f][t] + nchan) / (2 * nchan)) (the channel mean
// rounded half up), is subtracted from every channel and the caller's offset
// added, clamped to [0, 255]. Exact integer arithmetic.
//
// Design (gfx950, wave64). Zero-DM has two kernels. The read-once kernel
// (k_zero_dm_reg, below) keeps each wave's channel words in registers from
// the sums to the rewrite, so the filterbank is read once and written once;
// it serves up to 1024 channels with input and output at one alignment mod
// 4. The two-pass kernel (k_zero_dm) serves the rest: a workgroup covers
// 256 consecutive samples; lane l of every wave owns samples 4l .. 4l+3 of
// that range (256 contiguous bytes per wave and channel), and the 16 waves
// split the channels (wave w takes f = w, w+16, ...), so many rows' loads
// are in flight at once. Rows of an odd length start anywhere in a 4-byte
// word, so every access is made on aligned words: a lane's 4 bytes are one
// or two aligned loads and a v_alignbyte, and the rewrite stores whole
// aligned words, byte stores only for the one or two words at the ends of a
// row's stretch. Partial sums meet in LDS, one wave forms the levels, then
// each wave re-reads and rewrites its own channels.
#include <hip/hip_runtime.h>

#include "sps_internal.h"

namespace sps {
namespace {

constexpr int kZdWaves = 16;
constexpr int kZdSpan = 256;  // samples per workgroup: 4 per lane

__device__ __forceinline__ uint32_t clamp8(int v) { return (uint32_t)min(255, max(0, v)); }

// n (1..4) bytes from p, in the low bytes (higher bytes undefined), read as
// the aligned 4-byte words that hold them: rows of an odd length start
// anywhere in a word. The second word is read only when one of the n bytes
// lies in it, so every word read holds a wanted byte (same page: no read
// leaves mapped memory).
__device__ __forceinline__ uint32_t load4(const uint8_t* p, int n) {
  const uintptr_t ap = reinterpret_cast<uintptr_t>(p);
  const uint32_t il = (uint32_t)(ap & 3u);
  const uint32_t* w = reinterpret_cast<const uint32_t*>(ap - il);
  const uint32_t lo = w[0];
  if (il == 0u) return lo;
  const uint32_t hi = (int)il + n > 4 ? w[1] : 0u;
  return __builtin_amdgcn_alignbyte(hi, lo, il);
}

__global__ __launch_bounds__(64 * kZdWaves) void k_zero_dm(ZeroDmArgs a) {
  __shared__ uint32_t part[kZdWaves][64][4];
  __shared__ int zs[kZdSpan];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t t0 = (int64_t)blockIdx.x * kZdSpan;
  const int tv = (int)min<int64_t>(kZdSpan, a.nsamp - t0);  // samples of this tile
  const int tl = 4 * lane;                                  // this lane's first sample in the tile
  const int n = max(0, min(4, tv - tl));
  const uint32_t keep = n >= 4 ? 0xFFFFFFFFu : ((1u << (8 * n)) - 1u);
  uint32_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll 4
  for (int f = wave; f < a.nchan; f += kZdWaves) {
    if (n > 0) {
      const uint32_t w = load4(a.in + (int64_t)f * a.nsamp + t0 + tl, n) & keep;
      s0 += w & 0xFFu;
      s1 += (w >> 8) & 0xFFu;
      s2 += (w >> 16) & 0xFFu;
      s3 += w >> 24;
    }
  }
  part[wave][lane][0] = s0;
  part[wave][lane][1] = s1;
  part[wave][lane][2] = s2;
  part[wave][lane][3] = s3;
  __syncthreads();
  // sums < 255 * 65536 < 2^24: the level fits 32-bit arithmetic
  if (wave == 0) {
    const uint32_t c = (uint32_t)a.nchan;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t sum = 0;
#pragma unroll
      for (int w = 0; w < kZdWaves; ++w) sum += part[w][lane][q];
      zs[tl + q] = (int)((2u * sum + c) / (2u * c)) - a.offset;
    }
  }
  __syncthreads();
  // Rewrite, one row at a time: the aligned output words over the tile's
  // bytes. Word k holds tile bytes 4k - lead .. 4k - lead + 3; words wholly
  // inside the tile are read (aligned, realigned) and stored whole, the one
  // or two at its ends byte by byte, only the tile's own bytes.
  for (int f = wave; f < a.nchan; f += kZdWaves) {
    const int64_t row = (int64_t)f * a.nsamp + t0;
    const int lead = (int)((reinterpret_cast<uintptr_t>(a.out + row)) & 3u);
    for (int k = lane; k <= kZdSpan / 4; k += 64) {
      const int j0 = 4 * k - lead;
      if (j0 >= tv || j0 + 4 <= 0) continue;
      if (j0 >= 0 && j0 + 4 <= tv) {
        const uint32_t v = load4(a.in + row + j0, 4);
        const uint32_t o = clamp8((int)(v & 0xFFu) - zs[j0]) | (clamp8((int)((v >> 8) & 0xFFu) - zs[j0 + 1]) << 8) |
                           (clamp8((int)((v >> 16) & 0xFFu) - zs[j0 + 2]) << 16) |
                           (clamp8((int)(v >> 24) - zs[j0 + 3]) << 24);
        *reinterpret_cast<uint32_t*>(a.out + row + j0) = o;
      } else {
        for (int q = 0; q < 4; ++q) {
          const int j = j0 + q;
          if (j >= 0 && j < tv) a.out[row + j] = (uint8_t)clamp8((int)a.in[row + j] - zs[j]);
        }
      }
    }
  }
}

// Read-once form (up to 1024 channels, input and output at the same
// alignment mod 4, under 4 GiB): a workgroup covers 252 samples and each wave
// keeps the words of its channels (f = wave, wave + 16, ...) in registers
// from the sums to the rewrite, so the filterbank is read once and written
// once, and every load of a wave is issued before the first is needed. Lane l
// of a wave owns word l of the tile, tile bytes 4l - lead .. 4l - lead + 3,
// where lead puts the word on a 4-byte boundary of the row (the same one in
// input and output); 64 words always cover the 252 samples. lead is the same
// for all of a wave's channels: their rows start 16 * nsamp bytes apart and
// the tile start is a multiple of 4. Addresses are one scalar base per wave
// plus 32-bit offsets. Bytes outside the tile are kept out of the sums and
// never written; the aligned word that holds a wanted byte lies in the same
// page, so every read stays in mapped memory.
constexpr int kZrSpan = 252;  // samples per workgroup (a multiple of 4)

template <int CPW>
__global__ __launch_bounds__(64 * kZdWaves) void k_zero_dm_reg(ZeroDmArgs a, int per_xcd) {
  __shared__ uint32_t part[kZdWaves][kZrSpan + 8];  // tile sample j at index j + 4
  __shared__ int zs[kZrSpan + 8];
  // XCD-aware order: workgroup b runs on XCD b % 8, which takes a contiguous
  // range of tiles, so neighbouring tiles (sharing a cache line in every
  // row) run together under one L2
  const int64_t tile = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (tile * kZrSpan >= a.nsamp) return;  // whole workgroup, before any barrier
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t t0 = tile * kZrSpan;
  const int tv = (int)min<int64_t>(kZrSpan, a.nsamp - t0);  // samples of this tile, >= 1
  const uint32_t S = (uint32_t)(kZdWaves * a.nsamp);        // bytes between a wave's channels
  // the wave's first channel (channel 0 for a wave with none: it only reads it)
  const int wrow = wave < a.nchan ? wave : 0;
  const uint8_t* in0 = a.in + (int64_t)wrow * a.nsamp + t0 - 4;  // 4 bytes before the tile
  uint8_t* out0 = a.out + (int64_t)wrow * a.nsamp + t0 - 4;
  const int lead = (int)(reinterpret_cast<uintptr_t>(out0 + 4) & 3u);
  const int j0 = 4 * lane - lead;                        // the word: tile bytes j0 .. j0 + 3
  const int blo = max(0, -j0), bhi = min(4, tv - j0);  // the tile's bytes of the word: [blo, bhi)
  const bool any = bhi > blo;
  const uint32_t keep = !any ? 0u
                             : ((bhi >= 4 ? 0xFFFFFFFFu : ((1u << (8 * bhi)) - 1u)) & ~((1u << (8 * blo)) - 1u));
  const uint32_t vo = (uint32_t)(4 + j0);  // >= 1
  // a lane with no byte of the tile reads the word of tile byte 0 and keeps nothing
  const uint32_t vl = any ? vo : (uint32_t)(4 - lead);
  // Raw buffers over the wave's rows (descriptor word 3 as for every gfx9
  // raw buffer: 32-bit data format; no range limit below 2^32): the lane
  // offset in a VGPR, the channel's offset i * S in a scalar register.
  const __amdgpu_buffer_rsrc_t rin = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(in0), 0, -1, 0x00020000);
  const __amdgpu_buffer_rsrc_t rout = __builtin_amdgcn_make_buffer_rsrc(out0, 0, -1, 0x00020000);
  const int nv = min(CPW, (a.nchan - wave + kZdWaves - 1) / kZdWaves);  // the wave's channels, >= 0
  uint32_t v[CPW];
  uint32_t slo = 0, shi = 0;  // samples 0 and 2, 1 and 3 of the word as 16-bit sums (CPW * 255 < 2^16)
  // A channel past nchan reads the wave's first one again (no branch or mask
  // between the loads); its copies are taken out of the sums after the loop.
#pragma unroll
  for (int i = 0; i < CPW; ++i) {
    const int so = i < nv ? (int)((uint32_t)i * S) : 0;
    v[i] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rin, (int)vl, so, 0) & keep;
    slo += __builtin_amdgcn_perm(0u, v[i], 0x0c020c00u);
    shi += __builtin_amdgcn_perm(0u, v[i], 0x0c030c01u);
  }
  if (nv < CPW) {  // each 16-bit lane holds those copies, so no borrow crosses lanes
    slo -= (uint32_t)(CPW - nv) * __builtin_amdgcn_perm(0u, v[0], 0x0c020c00u);
    shi -= (uint32_t)(CPW - nv) * __builtin_amdgcn_perm(0u, v[0], 0x0c030c01u);
  }
  uint32_t* pw = &part[wave][4 + j0];  // j0 + 4 >= 1
  pw[0] = slo & 0xFFFFu;
  pw[1] = shi & 0xFFFFu;
  pw[2] = slo >> 16;
  pw[3] = shi >> 16;
  __syncthreads();
  // sums <= 255 * 1024: 2 * sum + nchan fits 32 bits
  if ((int)threadIdx.x < tv) {
    uint32_t sum = 0;
#pragma unroll
    for (int w = 0; w < kZdWaves; ++w) sum += part[w][4 + threadIdx.x];
    const uint32_t c = (uint32_t)a.nchan;
    zs[4 + threadIdx.x] = (int)((2u * sum + c) / (2u * c)) - a.offset;
  }
  __syncthreads();
  // levels of the word's four samples as two 16-bit pairs (bytes 0/2, 1/3);
  // in - level lies in [-255, 510], which 16-bit lanes hold
  typedef short short2_t __attribute__((ext_vector_type(2)));
  int z[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) z[q] = (q >= blo && q < bhi) ? zs[4 + j0 + q] : 0;
  const short2_t zl = {(short)z[0], (short)z[2]}, zh = {(short)z[1], (short)z[3]};
  const short2_t lo0 = {0, 0}, hi255 = {255, 255};
  const bool whole = blo == 0 && bhi == 4;
  // the channel stride and count, opaque here: otherwise the compiler keeps
  // the loads' 64 channel offsets and conditions alive for the stores and
  // spills them
  int Sr = (int)S, nvr = nv;
  asm volatile("" : "+s"(Sr), "+s"(nvr));
#pragma unroll
  for (int i = 0; i < CPW; ++i) {
    // the word opaque too: the byte pairs formed for the sums are not kept
    // alive until here (that would be two registers per channel)
    uint32_t x = v[i];
    asm volatile("" : "+v"(x));
    short2_t l = __builtin_bit_cast(short2_t, __builtin_amdgcn_perm(0u, x, 0x0c020c00u)) - zl;
    short2_t h = __builtin_bit_cast(short2_t, __builtin_amdgcn_perm(0u, x, 0x0c030c01u)) - zh;
    l = __builtin_elementwise_min(__builtin_elementwise_max(l, lo0), hi255);
    h = __builtin_elementwise_min(__builtin_elementwise_max(h, lo0), hi255);
    // bytes 0 and 2 of l and of h, interleaved back into sample order
    const uint32_t o = __builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, h), __builtin_bit_cast(uint32_t, l),
                                             0x06020400u);
    if (i < nvr) {
      if (whole) {
        __builtin_amdgcn_raw_buffer_store_b32(o, rout, (int)vo, (int)((uint32_t)i * (uint32_t)Sr), 0);
      } else if (any) {  // a word at the tile's ends: only the tile's own bytes
        uint8_t* ob = out0 + (vo + (uint32_t)i * (uint32_t)Sr);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q >= blo && q < bhi) ob[q] = (uint8_t)(o >> (8 * q));
      }
    }
  }
}

// ---- narrowband: per-channel statistics, flags, replacement -----------------
// Exact order statistics of bytes from a 256-bin histogram H with n values:
// the lower median (rank (n-1)/2) and the lower MAD about it, found by
// widening [mu - D, mu + D] until it holds more than the rank.
__device__ void hist_median_mad(const uint32_t* H, uint32_t n, int& mu, int& mad) {
  const uint32_t r = (n - 1) / 2;
  uint32_t acc = 0;
  int m = 0;
  for (; m < 256; ++m) {
    acc += H[m];
    if (acc > r) break;
  }
  uint32_t cnt = H[m];
  int d = 0;
  while (cnt <= r) {
    ++d;
    if (m - d >= 0) cnt += H[m - d];
    if (m + d <= 255) cnt += H[m + d];
  }
  mu = m;
  mad = d;
}

// One workgroup per channel: byte histogram of the row, then its median and
// MAD. Noise bytes crowd into a few bins, and LDS atomics of one instruction
// on one address are serialised: each wave keeps 16 sub-histograms (lane
// l counts into copy l % 16, so at most 4 lanes share an address), 257 words
// apart so that the copies of a bin fall in different banks. 64 x 257 words
// (66 KB): two workgroups per CU.
constexpr int kCsCopies = 16;
constexpr int kCsStride = 257;

__global__ __launch_bounds__(256) void k_chan_stats(ChanMaskArgs a) {
  __shared__ uint32_t h[4 * kCsCopies * kCsStride];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int f = blockIdx.x;
  for (int b = tid; b < 4 * kCsCopies * kCsStride; b += 256) h[b] = 0;
  __syncthreads();
  uint32_t* mine = h + (wave * kCsCopies + (lane & (kCsCopies - 1))) * kCsStride;
  // The row read as the aligned 16-byte chunks that cover it, whatever its
  // alignment (rows of an odd length start anywhere), four chunks in flight
  // per thread (enough bytes in flight to cover the memory latency); bytes
  // of a chunk outside the row are skipped. A chunk holding one byte of the
  // row lies in the same page as that byte, so the reads stay in mapped
  // memory.
  const uintptr_t start = reinterpret_cast<uintptr_t>(a.in + (int64_t)f * a.nsamp);
  const int lead = (int)(start & 15u);
  const uint4* chunks = reinterpret_cast<const uint4*>(start - (uintptr_t)lead);
  const int64_t last = lead + a.nsamp;  // one past the row's last byte, in chunk-byte units
  auto count4 = [&](uint32_t w) {
    atomicAdd(&mine[w & 0xFFu], 1u);
    atomicAdd(&mine[(w >> 8) & 0xFFu], 1u);
    atomicAdd(&mine[(w >> 16) & 0xFFu], 1u);
    atomicAdd(&mine[w >> 24], 1u);
  };
  auto count16 = [&](const uint4& c) {
    count4(c.x);
    count4(c.y);
    count4(c.z);
    count4(c.w);
  };
  // chunks wholly inside the row: k = kf .. kl, in steps of four chunks per
  // thread; the next step's chunks are loaded while this step's are counted
  // (a thread without a next step loads its current chunks again: every
  // load is issued, none under a lane condition)
  const int64_t kf = lead > 0 ? 1 : 0, kl = (last >> 4) - 1;
  int64_t k = kf + tid;
  if (k + 768 <= kl) {
    uint4 c0 = chunks[k], c1 = chunks[k + 256], c2 = chunks[k + 512], c3 = chunks[k + 768];
    while (true) {
      const int64_t kn = k + 1024;
      const bool more = kn + 768 <= kl;
      const int64_t kq = more ? kn : k;
      const uint4 n0 = chunks[kq], n1 = chunks[kq + 256], n2 = chunks[kq + 512], n3 = chunks[kq + 768];
      count16(c0);
      count16(c1);
      count16(c2);
      count16(c3);
      k = kn;
      if (!more) break;
      c0 = n0;
      c1 = n1;
      c2 = n2;
      c3 = n3;
    }
  }
  for (; k <= kl; k += 256) {
    const uint4 c = chunks[k];  // loaded whole before the atomics
    count16(c);
  }
  // the chunks at the row's ends, byte by byte: only the row's bytes
  if (tid < 2) {
    const int64_t ke = tid == 0 ? 0 : (last >> 4);
    // (the last chunk is thread 1's unless it is chunk 0 and thread 0's already)
    const bool edge = tid == 0 ? lead > 0 : ((last & 15) != 0 && (ke != 0 || lead == 0));
    if (edge) {
      const uint4 c = chunks[ke];
      const uint32_t w4[4] = {c.x, c.y, c.z, c.w};
      for (int q = 0; q < 16; ++q) {
        const int64_t b = 16 * ke + q;
        if (b >= lead && b < last) atomicAdd(&mine[(w4[q >> 2] >> (8 * (q & 3))) & 0xFFu], 1u);
      }
    }
  }
  __syncthreads();
  uint32_t t = 0;
  for (int c = 0; c < 4 * kCsCopies; ++c) t += h[c * kCsStride + tid];
  __syncthreads();
  h[tid] = t;
  __syncthreads();
  if (tid == 0) {
    int mu, mad;
    hist_median_mad(h, (uint32_t)a.nsamp, mu, mad);
    a.stats[3 * (int64_t)f] = (uint8_t)mu;
    a.stats[3 * (int64_t)f + 1] = (uint8_t)mad;
  }
}

// One workgroup: median M and MAD S of the channels' MADs (bytes again),
// then the flags sigma_f > M + k * S.
__global__ __launch_bounds__(256) void k_chan_flags(ChanMaskArgs a) {
  __shared__ uint32_t h[256];
  __shared__ int ms[2];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  for (int f = tid; f < a.nchan; f += 256) atomicAdd(&h[a.stats[3 * (int64_t)f + 1]], 1u);
  __syncthreads();
  if (tid == 0) hist_median_mad(h, (uint32_t)a.nchan, ms[0], ms[1]);
  __syncthreads();
  const int64_t lim = (int64_t)ms[0] + (int64_t)a.k * ms[1];
  for (int f = tid; f < a.nchan; f += 256) a.stats[3 * (int64_t)f + 2] = (int64_t)a.stats[3 * (int64_t)f + 1] > lim;
}

// Flagged channels take their median; the others are copied (nothing to do
// in place). A workgroup writes 1024 aligned output words of a row, four per
// thread 256 words apart (the row read as aligned words too, realigned; all
// four loads issued before the stores: a thread's words are its own, in
// place as well); the one or two words at the row's ends are written byte by
// byte, only the row's own bytes.
constexpr int kApplyWords = 4;

__global__ __launch_bounds__(256) void k_chan_apply(ChanMaskArgs a) {
  for (int f = blockIdx.y; f < a.nchan; f += gridDim.y) {
    const bool flag = a.stats[3 * (int64_t)f + 2] != 0;
    if (!flag && a.in == a.out) continue;
    const int64_t row = (int64_t)f * a.nsamp;
    const int lead = (int)((reinterpret_cast<uintptr_t>(a.out + row)) & 3u);
    const uint8_t mu = a.stats[3 * (int64_t)f];
    // input row at the output row's alignment (the usual case): its words
    // are aligned too, one load each
    const bool al = (int)((reinterpret_cast<uintptr_t>(a.in + row)) & 3u) == lead;
    uint32_t v[kApplyWords];
    int64_t j[kApplyWords];
#pragma unroll
    for (int u = 0; u < kApplyWords; ++u) {
      j[u] = 4 * ((int64_t)blockIdx.x * (256 * kApplyWords) + u * 256 + threadIdx.x) - lead;
      v[u] = 0x01010101u * mu;
    }
    // whole words of the row: j = jf, jf + 4, ..., jl
    const int64_t jf = (4 - lead) & 3, jl = jf + 4 * ((a.nsamp - 4 - jf) >> 2);
    if (!flag) {
      if (al && jl >= jf) {
        // every lane loads (a whole word of the row, clamped) and keeps what
        // it needs: loads under a lane condition make the compiler wait for
        // each before the next
#pragma unroll
        for (int u = 0; u < kApplyWords; ++u) {
          const uint32_t w = *reinterpret_cast<const uint32_t*>(a.in + row + min(max(j[u], jf), jl));
          v[u] = (j[u] >= 0 && j[u] + 4 <= a.nsamp) ? w : v[u];
        }
      } else {
#pragma unroll
        for (int u = 0; u < kApplyWords; ++u)
          if (j[u] >= 0 && j[u] + 4 <= a.nsamp) v[u] = load4(a.in + row + j[u], 4);
      }
    }
#pragma unroll
    for (int u = 0; u < kApplyWords; ++u) {
      const int64_t j0 = j[u];
      if (j0 >= a.nsamp || j0 + 4 <= 0) continue;
      if (j0 >= 0 && j0 + 4 <= a.nsamp) {
        *reinterpret_cast<uint32_t*>(a.out + row + j0) = v[u];
      } else {
        for (int q = 0; q < 4; ++q) {
          const int64_t jj = j0 + q;
          if (jj >= 0 && jj < a.nsamp) a.out[row + jj] = flag ? mu : a.in[row + jj];
        }
      }
    }
  }
}

// The same with 16-byte chunks, for input and output at one alignment mod
// 16 (in place, or same-aligned buffers): chunk k of a row covers its bytes
// 16 k - lead .. 16 k - lead + 15, aligned in both; four chunks per thread,
// 256 apart, all loads before the stores (a lane's chunks are its own).
// Whole chunks move as one load and one store; the one or two at the row's
// ends byte by byte.
__global__ __launch_bounds__(256) void k_chan_apply16(ChanMaskArgs a) {
  for (int f = blockIdx.y; f < a.nchan; f += gridDim.y) {
    const bool flag = a.stats[3 * (int64_t)f + 2] != 0;
    if (!flag && a.in == a.out) continue;
    const int64_t row = (int64_t)f * a.nsamp;
    const int lead = (int)((reinterpret_cast<uintptr_t>(a.out + row)) & 15u);
    const uint8_t mu = a.stats[3 * (int64_t)f];
    const uint32_t fill = 0x01010101u * mu;
    // whole chunks of the row: j = jf, jf + 16, ..., jl
    const int64_t jf = (16 - lead) & 15, jl = jf + 16 * ((a.nsamp - 16 - jf) >> 4);
    const uint4 fv = make_uint4(fill, fill, fill, fill);
    const bool copy = !flag && jl >= jf;  // the row has whole chunks to copy
    uint4 v[kApplyWords];
    int64_t j[kApplyWords];
#pragma unroll
    for (int u = 0; u < kApplyWords; ++u)
      j[u] = 16 * ((int64_t)blockIdx.x * (256 * kApplyWords) + u * 256 + threadIdx.x) - lead;
    // every lane of a copied row loads (a whole chunk of the row, clamped;
    // the others are not stored); a branch on the row's flag, the same for
    // the whole workgroup
    if (copy) {
#pragma unroll
      for (int u = 0; u < kApplyWords; ++u)
        v[u] = *reinterpret_cast<const uint4*>(a.in + row + min(max(j[u], jf), jl));
    } else {
#pragma unroll
      for (int u = 0; u < kApplyWords; ++u) v[u] = fv;
    }
#pragma unroll
    for (int u = 0; u < kApplyWords; ++u)
      if (j[u] >= 0 && j[u] + 16 <= a.nsamp) *reinterpret_cast<uint4*>(a.out + row + j[u]) = v[u];
    // the chunks at the row's ends (no chunk value is needed here)
#pragma unroll
    for (int u = 0; u < kApplyWords; ++u) {
      const int64_t j0 = j[u];
      if (j0 < a.nsamp && j0 + 16 > 0 && !(j0 >= 0 && j0 + 16 <= a.nsamp)) {
        for (int q = 0; q < 16; ++q) {
          const int64_t jj = j0 + q;
          if (jj >= 0 && jj < a.nsamp) a.out[row + jj] = flag ? mu : a.in[row + jj];
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_chan_mask(const ChanMaskArgs& a, hipStream_t s) {
  if (a.nsamp <= 0 || a.nchan <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_chan_stats, dim3((unsigned)a.nchan), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_chan_flags, dim3(1), dim3(256), 0, s, a);
  const unsigned gy = (unsigned)min(a.nchan, 65535);
  if (((reinterpret_cast<uintptr_t>(a.in) ^ reinterpret_cast<uintptr_t>(a.out)) & 15u) == 0) {
    // aligned 16-byte output chunks of a row: at most nsamp / 16 + 2
    const unsigned gx = (unsigned)((a.nsamp / 16 + 2 + 256 * kApplyWords - 1) / (256 * kApplyWords));
    hipLaunchKernelGGL(k_chan_apply16, dim3(gx, gy), dim3(256), 0, s, a);
  } else {
    // aligned output words of a row: at most nsamp / 4 + 2
    const unsigned gx = (unsigned)((a.nsamp / 4 + 2 + 256 * kApplyWords - 1) / (256 * kApplyWords));
    hipLaunchKernelGGL(k_chan_apply, dim3(gx, gy), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_zero_dm(const ZeroDmArgs& a, hipStream_t s) {
  if (a.nsamp <= 0 || a.nchan <= 0) return hipSuccess;
  const dim3 t(64 * kZdWaves);
  // the read-once kernel: same alignment mod 4 in and out, 32-bit offsets
  // (every offset below nchan * nsamp + 4), at most 64 channels per wave
  const bool same4 = ((reinterpret_cast<uintptr_t>(a.in) ^ reinterpret_cast<uintptr_t>(a.out)) & 3u) == 0;
  const bool small = (int64_t)a.nchan * a.nsamp + 8 < ((int64_t)1 << 32);
  const int per_xcd = (int)(((a.nsamp + kZrSpan - 1) / kZrSpan + 7) / 8);
  const dim3 gr(8u * (unsigned)per_xcd);
  if (same4 && small && a.nchan <= 4 * kZdWaves) hipLaunchKernelGGL(k_zero_dm_reg<4>, gr, t, 0, s, a, per_xcd);
  else if (same4 && small && a.nchan <= 16 * kZdWaves) hipLaunchKernelGGL(k_zero_dm_reg<16>, gr, t, 0, s, a, per_xcd);
  else if (same4 && small && a.nchan <= 64 * kZdWaves) hipLaunchKernelGGL(k_zero_dm_reg<64>, gr, t, 0, s, a, per_xcd);
  else hipLaunchKernelGGL(k_zero_dm, dim3((unsigned)((a.nsamp + kZdSpan - 1) / kZdSpan)), t, 0, s, a);
  return hipGetLastError();
}

}  // namespace sps
