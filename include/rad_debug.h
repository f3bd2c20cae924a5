/*
 * rad_debug.h - diagnostic entry points of the radiation library (not needed to compute
 * spectra).  Same conventions as rad.h.
 */
#ifndef RAD_DEBUG_H
#define RAD_DEBUG_H

#ifdef __cplusplus
extern "C" {
#endif

/* For each of n revolutions r = in_dev[i] (DEVICE, floats), write to out_dev[4i..4i+3]
 * (DEVICE) the sine and cosine of 2*pi*r from the hardware transcendental unit used to
 * seed the frequency walk, then from the library sincospi used for the per-particle
 * rotation factor.  Lets a test measure both against FP64 references.  Stream-ordered. */
int rad_debug_trig_probe(const float* in_dev, float* out_dev, int n, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RAD_DEBUG_H */
