// Packed 16-bit pair-scan building blocks shared by the plain and the batched
// scan kernels: two nodes per lane (16-bit halves), Johnson-order records as
// scalar loads, per-(job, lane) masks in LDS read with M0-based addressing.
#pragma once

#include "ws16.h"
#include "bound_common.h"

namespace fspbb {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as16(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t as32(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }

__device__ __forceinline__ void scan_step(u16x2 &s, const unsigned char *lds_lane, uint32_t joff, uint32_t ce)
{
    const uint32_t msk = *reinterpret_cast<const uint32_t *>(lds_lane + joff);
    const unsigned short e = (unsigned short)(ce >> 16), c = (unsigned short)ce;
    const u16x2 E = {e, e};
    const u16x2 C = {c, c};
    const u16x2 t = __builtin_elementwise_max(s, E) + C;
    s = as16((msk & as32(t)) | (~msk & as32(s)));
}

// Mask rows of UNR slots through the LDS "add thread id" read: for each slot
// M0 = row offset, and every lane reads the dword at M0 + 4 * lane, so no
// vector instruction is spent on addresses.  M0 is saved and restored; the
// block waits for its own reads (scalar loads are then complete as well).
// A write of M0 by a scalar instruction needs one wait state before the read.
// The scalar adds write SCC, which the block declares clobbered.
template <int UNR>
__device__ __forceinline__ void gather_rows_addtid(uint32_t (&x)[UNR], const uint32_t (&joff)[UNR], uint32_t base);

#define FSP_ADDTID_1(i) "s_add_u32 m0, %[j" #i "], %[base]\n\ts_nop 0\n\tds_read_addtid_b32 %[x" #i "]\n\t"

template <>
__device__ __forceinline__ void gather_rows_addtid<8>(uint32_t (&x)[8], const uint32_t (&joff)[8], uint32_t base)
{
    uint32_t save;
    asm volatile("s_mov_b32 %[sv], m0\n\t"
                 FSP_ADDTID_1(0) FSP_ADDTID_1(1) FSP_ADDTID_1(2) FSP_ADDTID_1(3)
                 FSP_ADDTID_1(4) FSP_ADDTID_1(5) FSP_ADDTID_1(6) FSP_ADDTID_1(7)
                 "s_waitcnt lgkmcnt(0)\n\t"
                 "s_mov_b32 m0, %[sv]"
                 : [x0] "=&v"(x[0]), [x1] "=&v"(x[1]), [x2] "=&v"(x[2]), [x3] "=&v"(x[3]),
                   [x4] "=&v"(x[4]), [x5] "=&v"(x[5]), [x6] "=&v"(x[6]), [x7] "=&v"(x[7]), [sv] "=&s"(save)
                 : [j0] "s"(joff[0]), [j1] "s"(joff[1]), [j2] "s"(joff[2]), [j3] "s"(joff[3]),
                   [j4] "s"(joff[4]), [j5] "s"(joff[5]), [j6] "s"(joff[6]), [j7] "s"(joff[7]),
                   [base] "s"(base)
                 : "scc");
}

template <>
__device__ __forceinline__ void gather_rows_addtid<4>(uint32_t (&x)[4], const uint32_t (&joff)[4], uint32_t base)
{
    uint32_t save;
    asm volatile("s_mov_b32 %[sv], m0\n\t"
                 FSP_ADDTID_1(0) FSP_ADDTID_1(1) FSP_ADDTID_1(2) FSP_ADDTID_1(3)
                 "s_waitcnt lgkmcnt(0)\n\t"
                 "s_mov_b32 m0, %[sv]"
                 : [x0] "=&v"(x[0]), [x1] "=&v"(x[1]), [x2] "=&v"(x[2]), [x3] "=&v"(x[3]), [sv] "=&s"(save)
                 : [j0] "s"(joff[0]), [j1] "s"(joff[1]), [j2] "s"(joff[2]), [j3] "s"(joff[3]),
                   [base] "s"(base)
                 : "scc");
}

template <>
__device__ __forceinline__ void gather_rows_addtid<16>(uint32_t (&x)[16], const uint32_t (&joff)[16], uint32_t base)
{
    uint32_t save;
    asm volatile("s_mov_b32 %[sv], m0\n\t"
                 FSP_ADDTID_1(0) FSP_ADDTID_1(1) FSP_ADDTID_1(2) FSP_ADDTID_1(3)
                 FSP_ADDTID_1(4) FSP_ADDTID_1(5) FSP_ADDTID_1(6) FSP_ADDTID_1(7)
                 FSP_ADDTID_1(8) FSP_ADDTID_1(9) FSP_ADDTID_1(10) FSP_ADDTID_1(11)
                 FSP_ADDTID_1(12) FSP_ADDTID_1(13) FSP_ADDTID_1(14) FSP_ADDTID_1(15)
                 "s_waitcnt lgkmcnt(0)\n\t"
                 "s_mov_b32 m0, %[sv]"
                 : [x0] "=&v"(x[0]), [x1] "=&v"(x[1]), [x2] "=&v"(x[2]), [x3] "=&v"(x[3]),
                   [x4] "=&v"(x[4]), [x5] "=&v"(x[5]), [x6] "=&v"(x[6]), [x7] "=&v"(x[7]),
                   [x8] "=&v"(x[8]), [x9] "=&v"(x[9]), [x10] "=&v"(x[10]), [x11] "=&v"(x[11]),
                   [x12] "=&v"(x[12]), [x13] "=&v"(x[13]), [x14] "=&v"(x[14]), [x15] "=&v"(x[15]),
                   [sv] "=&s"(save)
                 : [j0] "s"(joff[0]), [j1] "s"(joff[1]), [j2] "s"(joff[2]), [j3] "s"(joff[3]),
                   [j4] "s"(joff[4]), [j5] "s"(joff[5]), [j6] "s"(joff[6]), [j7] "s"(joff[7]),
                   [j8] "s"(joff[8]), [j9] "s"(joff[9]), [j10] "s"(joff[10]), [j11] "s"(joff[11]),
                   [j12] "s"(joff[12]), [j13] "s"(joff[13]), [j14] "s"(joff[14]), [j15] "s"(joff[15]),
                   [base] "s"(base)
                 : "scc");
}

template <>
__device__ __forceinline__ void gather_rows_addtid<32>(uint32_t (&x)[32], const uint32_t (&joff)[32], uint32_t base)
{
    uint32_t lo[16], hi[16], jl[16], jh[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) { jl[c] = joff[c]; jh[c] = joff[16 + c]; }
    gather_rows_addtid<16>(lo, jl, base);
    gather_rows_addtid<16>(hi, jh, base);
#pragma unroll
    for (int c = 0; c < 16; ++c) { x[c] = lo[c]; x[16 + c] = hi[c]; }
}
#undef FSP_ADDTID_1

__device__ __forceinline__ void scan_update(u16x2 &s, uint32_t msk, uint32_t ce)
{
    const unsigned short e = (unsigned short)(ce >> 16), c = (unsigned short)ce;
    const u16x2 E = {e, e};
    const u16x2 C = {c, c};
    const u16x2 t = __builtin_elementwise_max(s, E) + C;
    s = as16((msk & as32(t)) | (~msk & as32(s)));
}

// Scans NCH machine pairs in lockstep over their Johnson-order slots.  The
// chains are independent, so their dependent packed operations interleave.
template <int UNR, int NCH, bool ADDTID>
__device__ __forceinline__ void scan_pairs(const DevTables &T, const int (&prs)[NCH], u16x2 (&s)[NCH],
                                           const unsigned char *lds_lane, uint32_t lds_base)
{
    const int npad = T.npad;  // multiple of 4; padding slots read the zero row
    cptr<uint32_t> rec[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
        rec[ch] = as_const(reinterpret_cast<const uint32_t *>(T.rec16 + (size_t)prs[ch] * npad));
    int i = 0;
    for (; i + UNR <= npad; i += UNR) {
        uint32_t r[NCH][2 * UNR];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int c = 0; c < 2 * UNR; ++c) r[ch][c] = rec[ch][2 * i + c];
        if constexpr (ADDTID) {
            uint32_t jo[NCH * UNR], x[NCH * UNR];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
                for (int c = 0; c < UNR; ++c) jo[ch * UNR + c] = r[ch][2 * c];
            gather_rows_addtid<NCH * UNR>(x, jo, lds_base);
#pragma unroll
            for (int c = 0; c < UNR; ++c)
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) scan_update(s[ch], x[ch * UNR + c], r[ch][2 * c + 1]);
        } else {
#pragma unroll
            for (int c = 0; c < UNR; ++c)
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) scan_step(s[ch], lds_lane, r[ch][2 * c], r[ch][2 * c + 1]);
        }
    }
    for (; i < npad; i += 4) {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            uint32_t r[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) r[c] = rec[ch][2 * i + c];
#pragma unroll
            for (int c = 0; c < 8; c += 2) scan_step(s[ch], lds_lane, r[c], r[c + 1]);
        }
    }
}

}  // namespace fspbb
