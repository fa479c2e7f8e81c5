/* swmi_calib.h -- VALU calibration of the DP cell (libswmi_calib.so), a measurement aid
 * beside the search library, not part of the search path.
 *
 * swcal_cellmix times a register-only copy of the Smith-Waterman cell with affine gaps
 * (Section 2, Eqs. 1-3) on the current HIP device: every compute unit runs
 * `waves_per_cu` one-wave workgroups, each lane runs two independent chains of 16 rows
 * over `ncols` columns, and no memory is touched until one word per lane is stored at
 * the end.  The cell is computed at one of three integer widths:
 *   kind 0  packed int16, two alignments per 32-bit lane (saturating add and subtract,
 *           maxima, and one byte permute to pack the two profile values);
 *   kind 1  int32, one alignment per lane;
 *   kind 2  SWAR int8, four alignments per lane, byte arithmetic from 32-bit logic.
 * Outputs: *ms, the duration of the second of two launches (HIP events, null stream);
 * *cells, the number of cells that launch computed (cells / ms / 1e6 = GCUPS-equivalent).
 * The library allocates and frees a small output buffer itself.
 * Returns 0, -1 for a bad argument (kind outside 0..2, waves_per_cu outside 1..32, ncols
 * outside 1..2^20, NULL output), -2 if the buffer cannot be allocated, -3 on a HIP error.
 */
#ifndef SWMI_CALIB_H
#define SWMI_CALIB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int swcal_cellmix(int32_t kind, int32_t waves_per_cu, int32_t ncols, double *ms,
                  double *cells);

#ifdef __cplusplus
}
#endif

#endif /* SWMI_CALIB_H */
