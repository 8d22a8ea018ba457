"""Plain FP64 CPU oracle for block stochastic gradient descent (BSGD) tomography.

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import or call anything in this package. It is a slow,
obviously-correct restatement of the method (Gao, Biguri, Blumensath, "Block
stochastic gradient descent for large-scale tomographic reconstruction in a
parallel network"), written from the paper and sharing no code with the GPU path:

* ``geometry``  rays, row/column partitions and sub-detectors (Sec. II, Eq. (e1), Fig. 2-3)
* ``siddon``    exact ray/voxel intersection lengths, the system matrix entries (Sec. I, Eq. (yax))
* ``system``    explicit sparse A for small grids
* ``rng``       counter-based SplitMix64 selection streams
* ``bsgd``      Algorithms 1 (BSGD), 2 (BSGD-IM), 4 (BSGD-TV), Eq. 1, metrics
* ``tv``        the TV proximal step of Algorithm 4 (fast gradient projection)
* ``cfast``     a plain C FP64 matrix-free Siddon projector (timed CPU baseline)

Parity status per function is stated in each module header.
"""
