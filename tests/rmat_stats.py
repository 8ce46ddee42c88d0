"""Closed-form expectations for R-MAT (Kronecker) degree classes.

For the plain R-MAT generator with initiator (A, B, C, D), 2**s vertices and
M independent edges, a vertex whose label has k one-bits is the source of an
edge with probability q_k = (A+B)**(s-k) * (C+D)**k, the destination with the
same probability (B = C), and both (a self-loop) with o_k = A**(s-k) * D**k.
An edge therefore touches it as a non-loop edge with p_k = 2 q_k - 2 o_k, and
the number of such edges is Binomial(M, p_k). So

    E[#degree-0] = sum_k C(s,k) (1 - p_k)**M
    E[#exactly one non-loop edge] = sum_k C(s,k) M p_k (1 - p_k)**(M-1)

The second is the degree-1 count up to vertices whose several edges all go to
one neighbour (rare). Standard deviations use independent Bernoulli terms.
"""
from math import comb


def degree01_expectation(scale, edgefactor=16, A=0.57, B=0.19, C=0.19, D=0.05):
    n = 1 << scale
    m = edgefactor * n
    ez = el = vz = vl = 0.0
    for k in range(scale + 1):
        q = (A + B) ** (scale - k) * (C + D) ** k
        o = A ** (scale - k) * D ** k
        p = 2 * q - 2 * o
        p0 = (1 - p) ** m
        p1 = m * p * (1 - p) ** (m - 1)
        c = comb(scale, k)
        ez += c * p0
        el += c * p1
        vz += c * p0 * (1 - p0)
        vl += c * p1 * (1 - p1)
    return ez, el, vz ** 0.5, vl ** 0.5
