// Layout of the late-fusion actor-critic's parameters: the float32 block
// of the C ABI and the bf16 weight copies the kernels read.
#pragma once

// bf16 weight block per network (elements): ego W1 [64][12] (11 inputs,
// zero-padded), ego W2 [64][64], road W1 [96][8] (5, padded), road W2
// [96][96], vehicle W1 [96][8] (7, padded), vehicle W2 [96][96], trunk W1
// [128][256], trunk W2 [64][128]; the heads and every bias come from the
// float32 parameter block (the heads rounded to bf16 on the way).
#define ACB_EW1 0
#define ACB_EW2 (ACB_EW1 + 64 * 12)
#define ACB_RW1 (ACB_EW2 + 64 * 64)
#define ACB_RW2 (ACB_RW1 + 96 * 8)
#define ACB_VW1 (ACB_RW2 + 96 * 96)
#define ACB_VW2 (ACB_VW1 + 96 * 8)
#define ACB_TW1 (ACB_VW2 + 96 * 96)
#define ACB_TW2 (ACB_TW1 + 128 * 256)
#define ACB_NET (ACB_TW2 + 64 * 128)
// float32 parameter block offsets within one network (the order of the
// C ABI's parameter block)
#define ACF_EW1 0
#define ACF_EB1 (ACF_EW1 + 64 * 11)
#define ACF_EW2 (ACF_EB1 + 64)
#define ACF_EB2 (ACF_EW2 + 64 * 64)
#define ACF_RW1 (ACF_EB2 + 64)
#define ACF_RB1 (ACF_RW1 + 96 * 5)
#define ACF_RW2 (ACF_RB1 + 96)
#define ACF_RB2 (ACF_RW2 + 96 * 96)
#define ACF_VW1 (ACF_RB2 + 96)
#define ACF_VB1 (ACF_VW1 + 96 * 7)
#define ACF_VW2 (ACF_VB1 + 96)
#define ACF_VB2 (ACF_VW2 + 96 * 96)
#define ACF_TW1 (ACF_VB2 + 96)
#define ACF_TB1 (ACF_TW1 + 128 * 256)
#define ACF_TW2 (ACF_TB1 + 128)
#define ACF_TB2 (ACF_TW2 + 64 * 128)
#define ACF_HEAD (ACF_TB2 + 64)          // == SF_AC_BODY
// one network's float32 block, its head included: actor W[3][64] b[3]
// log_sigma[3]; critic W[1][64] b[1]
#define ACF_NET0 (SF_AC_BODY + 3 * 64 + 3 + 3)
#define ACF_LOGSTD (SF_AC_BODY + 3 * 64 + 3)
