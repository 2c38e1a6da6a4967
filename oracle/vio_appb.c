/* vio_appb.c -- CPU oracle of the textured-patch experiment of App. B
 * (test infrastructure only; see vio.h).
 *
 * Paper anchor (Newson et al., "Video Inpainting of Complex Scenes"),
 * App. B, the table of probabilities that a random patch is closer to a
 * random reference patch than the constant patch of the same mean, and
 * the analysis of the l2 patch distance after it: for a reference patch W
 * and every patch V of a volume, V counts when SSD(W, V) < SSD(W, Z),
 * where Z is the constant patch of value mu.  The distance is the plain
 * sum of squared differences of Sec. 2 on one grey channel.
 *
 * This is the definition written out: every candidate, every voxel, both
 * sums taken directly (no expansion of the square), strict comparison.
 */
#include "vio.h"

int vio_closer_than_constant(const uint8_t* ref, int32_t n_ref, const uint8_t* vol, int32_t W,
                             int32_t H, int32_t T, int32_t pw, int32_t ph, int32_t pt,
                             int32_t mu, uint64_t* counts) {
  if (n_ref < 0 || W < 1 || H < 1 || T < 1 || pw < 1 || ph < 1 || pt < 1 || mu < 0 || mu > 255)
    return VIO_E_INVAL;
  if (n_ref > 0 && (!ref || !vol || !counts)) return VIO_E_INVAL;
  const int64_t N = (int64_t)pw * ph * pt;
  const int64_t Wc = (int64_t)W - pw + 1, Hc = (int64_t)H - ph + 1, Tc = (int64_t)T - pt + 1;
  for (int32_t r = 0; r < n_ref; ++r) {
    const uint8_t* w = ref + (int64_t)r * N;
    /* SSD(W, Z) */
    int64_t dz = 0;
    for (int64_t k = 0; k < N; ++k) dz += ((int64_t)w[k] - mu) * ((int64_t)w[k] - mu);
    uint64_t cnt = 0;
    if (Wc > 0 && Hc > 0 && Tc > 0) {
      /* every patch of the volume whose voxels all lie inside it; its
         voxels in the order dt, dy, dx as the reference's */
#pragma omp parallel for collapse(2) reduction(+ : cnt) schedule(static)
      for (int64_t t = 0; t < Tc; ++t)
        for (int64_t y = 0; y < Hc; ++y)
          for (int64_t x = 0; x < Wc; ++x) {
            int64_t d = 0, k = 0;
            for (int64_t dt = 0; dt < pt; ++dt)
              for (int64_t dy = 0; dy < ph; ++dy)
                for (int64_t dx = 0; dx < pw; ++dx, ++k) {
                  const int64_t v = vol[((t + dt) * H + (y + dy)) * W + (x + dx)];
                  d += ((int64_t)w[k] - v) * ((int64_t)w[k] - v);
                }
            if (d < dz) ++cnt;
          }
    }
    counts[r] = cnt;
  }
  return VIO_OK;
}
