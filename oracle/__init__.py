"""FP64 CPU oracle for the TSDF-Sampling hot path.

TEST INFRASTRUCTURE ONLY: a plain, slow, obviously correct implementation
written from the paper, used to check the GPU library.  Only ``tests/``, the
smoke check and the CPU-baseline leg of the benchmark may import it; the GPU
library never does, and this package imports nothing from the GPU library.

Modules
  _native   builds/loads the plain-C traversal oracle (tsdf_oracle.c)
  tsdf      integration (supp. Alg. "TSDF integration"), finalize, voxel
            flags, boundary detection (Alg. 1), sample placement (Sec. 3.4)
  field     neural SDF + colour MLP, analytic gradient (supp. normal eq.)
  render    NeuS opacity, volume rendering Eq. 1/2 and normal, the
            hierarchical-sampling baseline
  train     loss and weight gradients for a training step on bounded samples
"""
