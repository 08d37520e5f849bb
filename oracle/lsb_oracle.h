/*
 * lsb_oracle.h -- CPU oracle for k-bit LSB embedding and extraction.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load or call this library.
 * It shares no code, header, table or constant with the GPU library.
 *
 * What it computes (Patel, Pradhan, Ambegaokar, "A Novel Approach for
 * Implementing Steganography ...", arXiv:0912.0947):
 *   - embedding, Section VI step 7: clear the low bits of a cover byte and
 *     OR in a piece of a data byte (the paper fixes 2 bits; here k = 1..8);
 *   - extraction, Section VII step 6: mask the low bits of a stego byte,
 *     shift them into place and OR them into the zero-initialised data byte.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - the bit stream is S = BE32(len) || msg, read most-significant bit first;
 *   - cover byte t (flat HWC raster order, every channel byte) carries stream
 *     bits k*t .. k*t+k-1, the first of them in the highest bit of the field;
 *   - the last field may carry nb < k bits: only its top nb field bits change;
 *   - cover bytes past the stream are left unchanged.
 *
 * All functions are synchronous, operate on host memory and never allocate
 * memory visible to the caller.  Return codes are ORACLE_* below.
 */
#ifndef LSB_ORACLE_H
#define LSB_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORACLE_OK = 0,
    ORACLE_E_ARG = -1,       /* bad k, null pointer, misaligned raw slice   */
    ORACLE_E_CAPACITY = -2,  /* message does not fit the cover              */
    ORACLE_E_HEADER = -3,    /* decoded length does not fit the stego cover */
    ORACLE_E_BUFFER = -4,    /* decoded length exceeds the output buffer    */
    ORACLE_E_NOMEM = -6
};

/* Message capacity in bytes of an n-byte cover at k bits per byte:
 * floor(n*k/8) - 4 (four bytes go to the length header), capped at 2^32-1.
 * ORACLE_E_ARG if k is outside 1..8, ORACLE_E_CAPACITY if floor(n*k/8) < 4. */
int64_t oracle_capacity(uint64_t n, int k);

/* Header-mode embed: stego[0..n) <- cover with S = BE32(len)||msg written
 * into the low k bits.  stego may equal cover (in place).  On any error the
 * output is left untouched. */
int oracle_embed(const uint8_t *cover, uint8_t *stego, uint64_t n,
                 const uint8_t *msg, uint32_t len, int k);

/* Header-mode extract: decode len from the first 32 stream bits, then the
 * message.  *len_out receives the decoded length whenever the 32 header bits
 * fit the cover (also on ORACLE_E_HEADER / ORACLE_E_BUFFER), else 0.  msg_out
 * is written only on ORACLE_OK. */
int oracle_extract(const uint8_t *stego, uint64_t n, int k,
                   uint8_t *msg_out, uint64_t out_cap, uint32_t *len_out);

/* Raw slice embed.  The buffer holds cover bytes [t0, t0+n) of a logical
 * cover; `stream` is byte 0 of the logical stream of `stream_bits` bits.
 * Byte t of the buffer carries stream bits k*(t0+t) .. k*(t0+t)+k-1. */
int oracle_embed_raw(const uint8_t *cover, uint8_t *stego, uint64_t n,
                     uint64_t t0, const uint8_t *stream, uint64_t stream_bits,
                     int k);

/* Raw slice extract: writes stream bits [k*t0, e), e = min(k*(t0+n),
 * stream_bits), into stream_out (byte 0 = logical stream byte 0), bytes
 * k*t0/8 .. ceil(e/8)-1.  Bits at or past stream_bits in the last byte are
 * written as zero.  Requires k*t0 % 8 == 0, and e % 8 == 0 unless
 * e == stream_bits (ORACLE_E_ARG otherwise), so that no output byte is
 * shared with a neighbouring slice. */
int oracle_extract_raw(const uint8_t *stego, uint64_t n, uint64_t t0,
                       uint8_t *stream_out, uint64_t stream_bits, int k);

/* ---------------------------------------------------------------------
 * The paper's own layout (Section VI steps 2-7, Section VII steps 2-6):
 * 2 bits per byte, one colour plane `plane` of an h x w x c (HWC) image,
 * the data split greedily over the rows in order (each row takes
 * L = min(remaining, w/4) bytes, so that 4L <= w), and inside a row bit pair
 * i (bits 2i+1..2i) of data byte j goes to pixel L*i + j of the plane.  No
 * header: the caller passes the data length, as the paper's extract call
 * does.  Capacity: h * floor(w/4) bytes (ORACLE_E_CAPACITY beyond it). */
uint64_t oracle_paper_capacity(uint32_t h, uint32_t w);
int oracle_paper_embed(const uint8_t *cover, uint8_t *stego, uint32_t h,
                       uint32_t w, uint32_t c, uint32_t plane,
                       const uint8_t *data, uint64_t len);
int oracle_paper_extract(const uint8_t *stego, uint32_t h, uint32_t w,
                         uint32_t c, uint32_t plane, uint8_t *data,
                         uint64_t len);

/* ---------------------------------------------------------------------
 * One colour plane (Section VI step 2, Section VII step 2) with the general
 * method: the fields are the bytes of plane `plane` of an image of
 * `pixels` pixels x c channels (HWC), in raster order; everything else as
 * oracle_embed / oracle_extract.  Bytes of the other planes are copied. */
int oracle_embed_plane(const uint8_t *cover, uint8_t *stego, uint64_t pixels,
                       uint32_t c, uint32_t plane, const uint8_t *msg,
                       uint32_t len, int k);
int oracle_extract_plane(const uint8_t *stego, uint64_t pixels, uint32_t c,
                         uint32_t plane, int k, uint8_t *msg_out,
                         uint64_t out_cap, uint32_t *len_out);

/* Sum of squared differences of two byte strings (Section VIII reports the
 * peak signal-to-noise ratio 10*log10(255^2 / MSE), MSE = SSE / count). */
uint64_t oracle_sse(const uint8_t *a, const uint8_t *b, uint64_t n);
double oracle_psnr(uint64_t sse, uint64_t count);

#ifdef __cplusplus
}
#endif
#endif
