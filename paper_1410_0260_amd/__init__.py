"""MI355X (gfx950) implementation of ASKIT kernel summation.

`askit` is the thin binding of the HIP library (C ABI in include/askit.h);
`synth` holds the seeded synthetic-input generators.  Neither is imported
here, so the generators stay usable where the library is not built.
"""
