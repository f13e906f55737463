"""The Python binding refuses tensors the library would misread, before any launch.

The kernels take raw pointers and trust the sizes the mesh implies, so a float32 tensor read
as float64 or a short tensor would be read past its end. These checks run on the CPU: the mesh
below is a bare object with the sizes of a mesh (no library handle), and every call must raise
ValueError before it reaches the C ABI (a call that got that far would fail on the null
handle with MPMError instead)."""
import pytest
import torch

from paper_2606_09275_amd.autograd import MPMForce
from paper_2606_09275_amd.mesh import Mesh, check_state

N_POINT, N_DOF, NNZ = 5, 12, 144


def bare_mesh():
    m = Mesh.__new__(Mesh)
    m.h = None
    m.info = dict(n_point=N_POINT, n_dof=N_DOF, nnz=NNZ)
    return m


def good_state(n=N_POINT, dtype=torch.float64):
    f = lambda c: torch.ones((c, n) if c > 1 else (n,), dtype=dtype)  # noqa: E731
    return dict(x=f(3), l=f(3), vol=f(1), mass=f(1), Jn=f(1), bn=f(6), E=f(1), nu=f(1), sy=f(1))


def test_state_dtype_and_length():
    s = good_state()
    s["E"] = s["E"].to(torch.float32)
    with pytest.raises(ValueError, match="E.*dtype"):
        check_state(s, N_POINT)
    s = good_state()
    s["bn"] = torch.ones((6, N_POINT - 1), dtype=torch.float64)
    with pytest.raises(ValueError, match="bn.*elements"):
        check_state(s, N_POINT)
    s = good_state()
    s["Fn"] = torch.ones((3, 3, N_POINT), dtype=torch.float64).transpose(0, 2)
    with pytest.raises(ValueError, match="contiguous"):
        check_state(s, N_POINT)
    with pytest.raises(ValueError, match="device"):
        check_state(good_state(), N_POINT)  # right dtype and size, but host tensors


@pytest.mark.parametrize("what", ["u_dtype", "u_len", "f_ext", "dirichlet", "K_out"])
def test_assemble_refuses_before_launch(what):
    m = bare_mesh()
    s = good_state()
    u = torch.zeros(N_DOF, dtype=torch.float64)
    kw = {}
    if what == "u_dtype":
        u = u.to(torch.float32)
        pat = "u: expected dtype"
    elif what == "u_len":
        u = torch.zeros(N_DOF - 3, dtype=torch.float64)
        pat = "u: expected 12 elements"
    elif what == "f_ext":
        kw["f_ext"] = torch.zeros(N_DOF, dtype=torch.float32)
        pat = "f_ext: expected dtype"
    elif what == "dirichlet":
        kw["dirichlet"] = torch.zeros(N_DOF, dtype=torch.int32)
        pat = "dirichlet: expected dtype"
    else:
        kw["out"] = {"K": torch.zeros(NNZ, dtype=torch.float32)}
        pat = "K: expected dtype torch.float64"
    with pytest.raises(ValueError, match=pat):
        m.assemble(s, u, "f64", **kw)


def test_fp32k_output_must_be_float32():
    m = bare_mesh()
    with pytest.raises(ValueError, match="K: expected dtype torch.float32"):
        m.assemble(good_state(), torch.zeros(N_DOF, dtype=torch.float64), "f32k",
                   out={"K": torch.zeros(NNZ, dtype=torch.float64), "f_int": torch.zeros(N_DOF, dtype=torch.float64)})


def test_adjoint_and_solver_refuse_before_launch():
    m = bare_mesh()
    u = torch.zeros(N_DOF, dtype=torch.float64)
    with pytest.raises(ValueError, match="lambda: expected dtype"):
        m.adjoint(good_state(), u, torch.zeros(N_DOF, dtype=torch.float32))
    with pytest.raises(ValueError, match="K: expected 144 elements"):
        m.spmv(torch.zeros(NNZ - 1, dtype=torch.float64), u)
    with pytest.raises(ValueError, match="b: expected 12 elements"):
        m.solve_cg(torch.zeros(NNZ, dtype=torch.float64), torch.zeros(N_DOF + 1, dtype=torch.float64))


def test_autograd_casts_float32_parameters():
    """MPMForce converts float32 parameter leaves to float64 before the state check; the
    state check then sees float64 values (here it stops at the host-device check)."""
    m = bare_mesh()
    s = good_state()
    state = {k: s[k] for k in ("x", "l", "mass", "Jn", "bn")}
    E = torch.ones(N_POINT, dtype=torch.float32, requires_grad=True)
    nu, sy, vol = (torch.ones(N_POINT, dtype=torch.float32, requires_grad=True) for _ in range(3))
    u = torch.zeros(N_DOF, dtype=torch.float32)
    with pytest.raises(ValueError, match="device tensor"):
        MPMForce.apply(m, state, u, E, nu, sy, vol, "f64")
    with pytest.raises(ValueError, match="E: expected 5 elements|state\\['E'\\]: expected 5 elements"):
        MPMForce.apply(m, state, u, torch.ones(N_POINT + 1, requires_grad=True), nu, sy, vol, "f64")
