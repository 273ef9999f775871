"""Parameter sets of the synthetic workloads (shapes only, no arithmetic).

C1 single op     N=2^12, two ~40-bit ciphertext primes + one ~50-bit special
                 prime, scale 2^30, dnum 2.
C2 batched       N=2^14, 8 ciphertext primes (60-bit first, then 40-bit), 2
                 special 60-bit primes, dnum 4, scale 2^40.
C3 large ring    N=2^16, 24 ciphertext primes (60-bit first, then 50-bit), 6
                 special 60-bit primes, dnum 4, scale 2^50.
C4 bag of words  N=2^15, 16 ciphertext primes (60-bit first, then 40-bit), 4
                 special 60-bit primes, dnum 4, scale 2^40.

The prime sizes follow the paper's parameter guidance (Sec. 6.4: the scale
2^rho with rho in 20..60, |q_L| ~ L*rho) and its requirement that the last
prime of the chain is the smallest (Sec. 5.1, the paragraph before Eq. (1)).
"""

from dataclasses import dataclass


@dataclass(frozen=True)
class WorkloadConfig:
    name: str
    log_n: int
    n_q: int        # L, ciphertext primes
    q0_bits: int    # bit length of q_0
    q_bits: int     # bit length of q_1..q_{L-1}
    n_p: int        # K, special primes
    p_bits: int
    dnum: int
    log_scale: int

    @property
    def n(self) -> int:
        return 1 << self.log_n

    @property
    def scale(self) -> float:
        return float(2 ** self.log_scale)


CONFIGS = {
    "C1": WorkloadConfig("C1", 12, 2, 40, 40, 1, 50, 2, 30),
    "C2": WorkloadConfig("C2", 14, 8, 60, 40, 2, 60, 4, 40),
    "C3": WorkloadConfig("C3", 16, 24, 60, 50, 6, 60, 4, 50),
    "C4": WorkloadConfig("C4", 15, 16, 60, 40, 4, 60, 4, 40),
}
