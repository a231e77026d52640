"""Python wrapper of the request server (rsl_server_*)."""


class Server:
    def __init__(self, *a, **k):
        raise NotImplementedError("server not built yet")
