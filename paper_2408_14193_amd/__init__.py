"""spaLU (recursive sparse LU with nested dissection and low-rank
sparsification) on one MI355X: the C-ABI library libspalu.so and its
ctypes binding.  Import ``paper_2408_14193_amd.spalu`` for the API."""
