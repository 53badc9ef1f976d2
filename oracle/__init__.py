"""Oracle package (test infrastructure only).

Plain serial C (``mgref.c``) plus a ctypes wrapper. Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the GPU library never
does, and this package never imports the GPU library.
"""
