"""CPU oracle for the multilevel compression method (test infrastructure only).

This package is the plain, slow reference that the HIP path is checked
against.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the library itself never does, and the two share no
code.  Everything is written from the method's definition in the paper:

* recursive multilevel decomposition into multilevel coefficients and its
  inverse (Sec. 2, "Software design": decomposition on a multigrid hierarchy,
  the recomposition runs the inverse procedure);
* level-wise linear quantization by a bin width with an L-infinity guarantee
  (Sec. 2, quantization stage; Sec. 2.3, mathematically guaranteed loss);
* lossless encoding of the integers into a self-describing buffer (Sec. 2,
  final stage; Sec. 2.1, self-describing format).

The paper gives no formulas for these steps.  The readings taken here (P1
finite-element L2 projection on tensor grids, plain uniform bin allocation,
canonical Huffman with fixed tie rules, wire format) are listed with each
function and collected in the design notes.

Modules
-------
grid       hierarchy and FP64 per-dimension operator constants
transform  decompose / recompose in a chosen working precision
alloc      operator infinity norms and the plain bin-width allocation
quant      quantization, symbols and stream order
huffman    histogram, codebook, canonical codes, chunked bit packing
codec      end-to-end compress / decompress to the wire format
dense      brute-force dense projections used only to pin the above
mlp        reference MLP (forward, backward, Adam) for the learned allocation
snorm      L2 / s-norm error control
refactor   bitplane precision segments, greedy retrieval, reconstruction
lossless   second-stage zero-suppression coder (two-level bitmaps)
chunked    out-of-core slab container
"""
from . import grid, transform, alloc, quant, huffman, codec, dense, mlp  # noqa: F401
