"""FP64 CPU oracle (test infrastructure only).

``oracle.oracle`` is the numpy reference; ``oracle.cpu`` loads the plain C
build of the same definitions for sizes numpy cannot reach in seconds. Only
the tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the GPU path never imports it.
"""
