"""Named parameter sets (oracle's own copy; test infrastructure only).

``paper``: the defaults stated in Sec. 3.1 (tolerance 1e-3, m <= 6 with the
order capped, split while r~ < 1.3, at most 15 splits, 4x4 Duffy rule,
4 parts x 3 Gauss points per edge) and in Eq. (FMMTruncation) / Eq.
(Farfieldcond) (factor 1.8, minimum expansion length 8, admissibility
2/sqrt(3)).

``tight``: the same rules with a 1e-8 order tolerance, splitting instead of
capping the order (the higher-accuracy variant of Sec. 5.1.2), finer
singular and edge rules, and a wider admissibility with an accuracy-driven
expansion length so that the FMM agrees with the dense operator to ~1e-7.

``mixed``: the quadrature and tree of ``tight``; it differs only in number
format on the GPU, so the oracle treats it like ``tight``.

Coupling: ``paper`` keeps the paper's gamma = i/k (Sec. 2.5);
``tight``/``mixed``/``reference`` use gamma = -i/k, the other sign of the
imaginary coupling, with which the spectrum of the discrete operator lies in
the right half-plane (gamma = gamma_re + i gamma_im_k / k).

``reference``: oracle-only, used to measure each preset's own quadrature
error.
"""

import math

PRESETS = {
    "paper": dict(quad_eps=1e-3, m_max=6, split_on_cap=False, subdiv_ratio=1.3,
                  max_subdiv=15, self_n=4, edge_parts=4, edge_gauss=3,
                  admissibility=2.0 / math.sqrt(3.0), l_factor=1.8, l_min=8,
                  l_mode=0, fmm_eps=1e-3, fmm_eps_mixed=1e-3, t_order=4,
                  gamma_re=0.0, gamma_im_k=1.0),
    "tight": dict(quad_eps=1e-8, m_max=6, split_on_cap=True, subdiv_ratio=1.3,
                  max_subdiv=15, self_n=12, edge_parts=8, edge_gauss=6,
                  admissibility=3.0, l_factor=1.8, l_min=8,
                  l_mode=1, fmm_eps=1e-7, fmm_eps_mixed=1e-4, t_order=6,
                  gamma_re=0.0, gamma_im_k=-1.0),
    "mixed": dict(quad_eps=1e-8, m_max=6, split_on_cap=True, subdiv_ratio=1.3,
                  max_subdiv=15, self_n=12, edge_parts=8, edge_gauss=6,
                  admissibility=3.0, l_factor=1.8, l_min=8,
                  l_mode=1, fmm_eps=1e-7, fmm_eps_mixed=1e-4, t_order=6,
                  gamma_re=0.0, gamma_im_k=-1.0),
    "reference": dict(quad_eps=1e-12, m_max=6, split_on_cap=True, subdiv_ratio=1.3,
                      max_subdiv=15, self_n=20, edge_parts=16, edge_gauss=10,
                      admissibility=3.0, l_factor=1.8, l_min=8,
                      l_mode=1, fmm_eps=1e-10, fmm_eps_mixed=1e-4, t_order=8,
                      gamma_re=0.0, gamma_im_k=-1.0),
}


def preset(name, **overrides):
    p = dict(PRESETS[name])
    p.update(overrides)
    return p
