"""GF(2) products for the tests: (bits @ H^T) mod 2 through a sparse product,
so that syndrome checks on the large models (up to 18816 x 64288) stay cheap."""
import numpy as np
import scipy.sparse as sp


def gf2_product(bits, H) -> np.ndarray:
    """bits: (shots, N) 0/1; H: (M, N) 0/1 -> (shots, M) uint8."""
    Hs = sp.csr_matrix(np.asarray(H, dtype=np.int32))
    prod = Hs @ np.asarray(bits, dtype=np.int32).T
    return (np.asarray(prod).T % 2).astype(np.uint8)
