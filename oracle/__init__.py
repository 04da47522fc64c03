"""FP64 CPU oracle of the FastAlign hot path (test infrastructure only).

Only the test suite, the graft entry point's smoke check and the benchmark's
CPU-baseline leg may import this package.  It never imports the product
package and the product never imports it.
"""
