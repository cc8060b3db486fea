"""Plain FP64 CPU oracle of the electrofreezing phase-field LBM (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
package.  It shares no code with the GPU library.
"""
