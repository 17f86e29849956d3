"""MI355X-native swept-volume collision checking (neural implicit swept volumes).

The compute path is libsv.so (hand-written HIP for gfx950) behind the C ABI in
include/sv.h; ``_binding`` wraps it with torch device tensors.  Importing the
package does not load the library; ``from paper_2402_15281_amd import _binding``
does, and raises if libsv.so has not been built.
"""
