"""MI355X-native Barnes-Hut tree gravity (the hot path of REBOUND's method,
Rein & Liu 2012): Morton-key octree build, bottom-up moments, per-particle
and grouped tree walks with ghost boxes, and the drift-kick-drift step.

The compute path is the HIP library ``librb.so`` built from ``csrc/``;
``rb`` holds its Python binding.  ``inputs`` draws seeded initial conditions.
"""
