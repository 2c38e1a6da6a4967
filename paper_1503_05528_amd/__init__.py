"""MI355X-native (gfx950, HIP) hot path of Newson et al.'s global
patch-based video inpainting: spatio-temporal PatchMatch NNF search and
weighted patch-vote reconstruction behind a small C ABI (libvi.so)."""
