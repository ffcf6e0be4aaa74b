"""FP64 CPU oracle for the D3(BJ) path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import, call, link or execute anything in
this package.  The product path (the HIP library and its Python binding)
never routes through it and shares no code with it.
"""
